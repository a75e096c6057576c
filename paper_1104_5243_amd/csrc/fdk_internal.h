// Internal declarations shared by the host entry points and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdk {

// Views per launch of the fused backprojection and the forward projection
// (their folded matrices go to device memory once per call, 48 bytes per
// view), and of the plain kernel (matrices in the kernel arguments, under
// the 4 KiB kernel-argument limit).
constexpr int kMaxBatch = 1024;
constexpr int kPlainBatch = 64;

// Zero border of a staged projection plane (pixels on every side).  Taps
// are clamped into [-2, W] x [-2, H], so a 2-pixel border is enough for
// every clamped tap pair to read zeros outside the detector.
constexpr int kPad = 2;

enum StorageType { kF32 = 0, kF16 = 1, kBF16 = 2 };

// Staged plane layouts.  Element (r, c) of a plane holds, for the
// zero-extended pixel value p(r, c) of the padded view:
//   kRows : p(r, c)                                   (1 value)
//   kPairs: p(r, c), p(r+1, c)                         (2 values)
//   kQuads: p(r, c), p(r, c+1), p(r+1, c), p(r+1, c+1) (4 values)
//   kDPairs: p(r, c), p(r+1, c) - p(r, c)              (2 values)
//   kDQuads: p00, p10 - p00, p01 - p00, (p11 - p01) - (p10 - p00)
//            with pRC = p(r+R, c+C)                   (4 values)
// so that the four taps of a bilinear sample are two loads (rows) or one
// load (pairs, dpairs: 2 adjacent elements; quads, dquads: 1 element).
// dpairs and dquads store the differences the interpolation needs (rounded
// to the storage type): the bilinear sample then costs 4 (dpairs) or 3
// (dquads) instructions instead of 6.
enum Layout { kRows = 0, kPairs = 1, kQuads = 2, kDPairs = 3, kDQuads = 4 };

// values per staged element
__host__ __device__ constexpr int layout_width(int layout)
{
    return layout == kRows ? 1 : (layout == kQuads || layout == kDQuads) ? 4 : 2;
}

// Arguments of the fused kernel.  Matrices are in the centred index frame:
// for voxel (x, y, z) with x' = x - c (likewise y', z'), (u'w, v'w, w) =
// m * (x', y', z', 1), and the pixel coordinate is u = u' + ku.
struct FusedArgs {
    float* vol;          // N^3 (or a z-slab of it; see z_first, nz)
    const void* img;     // staged planes of this batch, plane elements apart
    long long plane;     // elements per staged plane
    int N;               // x and y extent; also the z stride base
    int nz;              // number of z slices written (z_first .. z_first+nz-1)
    int z_first;         // first z slice
    int Wp;              // staged row pitch (elements)
    // per-wave tests on the projected corners of a wave's voxel box (u', v'):
    // all below skip_lo or all above skip_hi -> every tap is outside the
    // detector; all within [in_lo, in_hi] -> no tap index clamp can act
    float skip_lo_u, skip_hi_u, skip_lo_v, skip_hi_v;
    float in_lo_u, in_hi_u, in_lo_v, in_hi_v;
    int origin_off;      // element offset of pixel (ku, kv) inside a plane
    float c;             // (N-1)/2
    int count;           // views in this batch
    int tiles_x, tiles_y, zchunks;
    int xcd_remap;       // 1: spread consecutive tiles over XCD-local ranges
    int y_fastest;       // 1: consecutive workgroups step along y, else along x
    const float* m;      // count x 12 folded matrices of this batch (device memory), in
                         // the ray frame: column 0 multiplies the transverse coordinate
                         // (x if y_fastest, else y), column 1 the ray coordinate
    const double* mq;    // the same matrices in FP64 before rounding, columns x, y, z, 1
    int lo_iu, hi_iu;    // clamp range of the tap index floor(u') (zero border included)
    int lo_iv, hi_iv;
    // forward projection
    int fp_tile;                   // entries of a workgroup's LDS tile
    int fp_vparts;                 // workgroups per box (grid y), each with whole chunks of the views
    unsigned long long* acc64;     // count padded planes of 64-bit fixed-point sums
    const unsigned* fp_vmax;       // max |x| of the volume (float bits, device)
    float fp_rmax2;                // >= 1 / w^2 over the volume and the batch's views
};

// Arguments of the plain kernel: world-coordinate matrices (FP32 roundings
// of the caller's), unpadded projections.
struct PlainArgs {
    float* vol;
    const float* proj;   // first view of the batch, H*W floats per view
    int N, H, W;
    float ox, oy, oz, vs;
    int count;
    float m[kPlainBatch][12];
};

// Folded matrices carried in the kernel arguments (under their 4 KiB
// limit), written to device memory by a one-block kernel (used where the
// library may not copy them from pinned host memory).
constexpr int kPutMatsMax = 24;
struct PutMatsArgs {
    float* dst;          // count x 12 floats
    double* dstq;        // count x 12 doubles
    int count;           // <= kPutMatsMax
    float m[kPutMatsMax * 12];
    double q[kPutMatsMax * 12];
};

struct StageArgs {
    const void* src;     // first view of the batch, H*W elements per view
    void* dst;           // count planes of Hp*Wp elements
    int H, W, Hp, Wp;
    int count;
    int layout;
};

// Padded 64-bit fixed-point accumulation planes of the forward projector
// (rows layout), in units of 2^-kg with kg from (N, *vmax, rmax2).
struct UnstageArgs {
    const unsigned long long* planes;  // count planes of Hp*Wp, pixel (j, k) at (k+kPad)*Wp + j+kPad
    float* dst;                        // count views of H*W floats, accumulated
    int H, W, Hp, Wp;
    int count;
    int fixed;                         // 1: 64-bit fixed point; 0: float planes
    int N;
    const unsigned* vmax;
    float rmax2;
};


// Launchers (return the hipError_t of the launch).
hipError_t launch_stage(const StageArgs& a, int storage, hipStream_t s);
// rows_free: v is not clamped (only with !wcheck and a single-load layout;
// the host has bounded every tap row, see rows_bounded)
// divide: the reciprocal variant of part 1 (0 v_rcp_f32, 1 rcp + one Newton
// step, 2 IEEE divisions, 3 rcp truncated to 12 bits); non-zero only with
// the dpairs layout
hipError_t launch_fused(const FusedArgs& a, int storage, int layout, bool wcheck, bool rows_free,
                        int divide, hipStream_t s);
hipError_t launch_plain(const PlainArgs& a, hipStream_t s);
// FP32 stack -> FP16 (per-view powers of 4 written to view_scale, device) or BF16
hipError_t launch_convert(void* dst, const float* src, int n_views, size_t view_len, int storage,
                          float* view_scale, hipStream_t s);
hipError_t launch_update_probe(float* a, size_t n, float s, hipStream_t st);
hipError_t launch_put_mats(const PutMatsArgs& a, hipStream_t s);
hipError_t launch_zero(float* a, size_t n, hipStream_t st);
// forward projection of a.vol into the padded planes at a.img (scatter)
hipError_t launch_scatter(const FusedArgs& a, bool wcheck, hipStream_t s);
// as launch_scatter for w > 0 everywhere; tiles of 16 x 16 columns
hipError_t launch_scatter_lds(const FusedArgs& a, hipStream_t s);
hipError_t launch_unstage_add(const UnstageArgs& a, hipStream_t s);
// max |x| over n floats as float bits into *out (which must hold 0 before)
hipError_t launch_fp_vmax(const float* vol, size_t n, unsigned* out, hipStream_t s);

// z voxels per thread: the forward projection kernels, and the fused
// backprojection by storage type (FP32 taps: 16; 16-bit taps: 8, whose
// smaller wave boxes clip more finely; both measured best on fdk512)
constexpr int kFpZ = 16;
#ifndef FDK_Z_F32
#define FDK_Z_F32 16
#endif
#ifndef FDK_Z_16BIT
#define FDK_Z_16BIT 8
#endif
__host__ __device__ constexpr int fused_z(int storage)
{
    return storage == kF32 ? FDK_Z_F32 : FDK_Z_16BIT;
}
// A wave covers kWaveX x kWaveY voxel columns; a workgroup puts its
// kWgWaves waves side by side across the batch's rays: along x when the
// rays run along y (y_fastest), else along y.  (fdk512 FP32: 31.7 ms per
// backprojection; stacked along y for both orientations 34.4, 2 x 2 33.2,
// along the rays 36.2: waves on one CU working on boxes behind each other
// on a ray gather the same detector lines at the same time.)
#ifndef FDK_WG_WAVES
#define FDK_WG_WAVES 4
#endif
#ifndef FDK_WAVE_X
#define FDK_WAVE_X 8
#endif
constexpr int kWaveX = FDK_WAVE_X, kWaveY = 64 / FDK_WAVE_X;
constexpr int kWgWaves = FDK_WG_WAVES;
constexpr int kThreads = 64 * kWgWaves;
// a workgroup tile's extent in x and y columns
__host__ __device__ constexpr int tile_x(bool y_fastest)
{
    return y_fastest ? kWaveX * kWgWaves : kWaveX;
}
__host__ __device__ constexpr int tile_y(bool y_fastest)
{
    return y_fastest ? kWaveY : kWaveY * kWgWaves;
}
// the first column of wave `wave`'s box in workgroup tile (tx, ty)
__device__ __forceinline__ void wave_origin(bool y_fastest, int tx, int ty, int wave, int& wx0,
                                            int& wy0)
{
    wx0 = tx * tile_x(y_fastest) + (y_fastest ? wave * kWaveX : 0);
    wy0 = ty * tile_y(y_fastest) + (y_fastest ? 0 : wave * kWaveY);
}

}  // namespace fdk
