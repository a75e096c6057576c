// Backprojection kernels for gfx950 (CDNA4).
//
// fused: the optimised kernel.  One thread owns an (x, y) voxel column and
//   fused_z consecutive z voxels; the views of a batch are fused in one
//   pass with the fused_z voxel sums held in registers, so the volume is
//   read and written once per batch (the image-loop blocking of the paper's
//   Section 6.2, with registers in place of the L1-resident voxel line).
//   Per (voxel, view) the work is the paper's three parts (Section 3.2):
//     part 1: (u'w, v'w, w) by three FMAs from a per-column base, one
//             reciprocal r = 1/w, u' = u'w r, v' = v'w r;
//     part 2: floor / fraction, clamp into the staged plane's zero border,
//             one 16-byte load of two adjacent staged elements (the
//             horizontally adjacent tap pairs the paper loads pairwise,
//             Section 4.1, each element holding a vertical tap pair);
//     part 3: bilinear interpolation and acc += r^2 * fx; with the default
//             staged layout the elements hold (p, p_below - p), so the
//             interpolation takes 4 instructions instead of 6.
//   The projections are read from zero-padded staged planes (Section 3.3),
//   so no tap needs a bounds test: out-of-detector taps are clamped onto
//   the zero border.
// plain: one thread per voxel with the listing's arithmetic in world
//   coordinates (two IEEE divisions, bounds-tested taps), for comparison.
// stage: copies a batch of views into zero-padded planes.
// update probe: a[i] = s * a[i], the paper's bandwidth benchmark.
#include "fdk_internal.h"
#include "gfx950_util.h"

namespace fdk {

// ---------------------------------------------------------------------------
// storage types
// ---------------------------------------------------------------------------
struct TF32 { using elem = float; static constexpr int id = kF32; };
struct TF16 { using elem = uint16_t; static constexpr int id = kF16; };
struct TBF16 { using elem = uint16_t; static constexpr int id = kBF16; };

// ---------------------------------------------------------------------------
// stage
// ---------------------------------------------------------------------------
template <typename E>
__device__ __forceinline__ E staged_pixel(const StageArgs& a, const E* src, int row, int col)
{
    const int j = col - kPad, k = row - kPad;
    return (j >= 0 && j < a.W && k >= 0 && k < a.H) ? src[(size_t)k * a.W + j] : E(0);
}

// storage element <-> float; float -> storage rounds to nearest even
__device__ __forceinline__ float to_f(TF32, float x) { return x; }
__device__ __forceinline__ float to_f(TF16, uint16_t x) { return (float)__builtin_bit_cast(_Float16, x); }
__device__ __forceinline__ float to_f(TBF16, uint16_t x)
{
    return __builtin_bit_cast(float, (uint32_t)x << 16);
}
__device__ __forceinline__ float from_f(TF32, float d) { return d; }
__device__ __forceinline__ uint16_t from_f(TF16, float d)
{
    return __builtin_bit_cast(uint16_t, (_Float16)d);
}
__device__ __forceinline__ uint16_t from_f(TBF16, float d)
{
    const uint32_t u = __builtin_bit_cast(uint32_t, d);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
// b - a, and (d - c) - (b - a), rounded to the storage type
template <typename TT, typename E>
__device__ __forceinline__ E diff_elem(TT t, E b, E a)
{
    return from_f(t, to_f(t, b) - to_f(t, a));
}
template <typename TT, typename E>
__device__ __forceinline__ E diff2_elem(TT t, E d, E c, E b, E a)
{
    return from_f(t, (to_f(t, d) - to_f(t, c)) - (to_f(t, b) - to_f(t, a)));
}

// One thread per column and kStageRows consecutive rows of a staged plane:
// the padded pixels of row r + 1 (and column c + 1 for the quad layouts)
// carry over to the next row, so every input pixel is read once per layout
// element column, and the blocks are few enough to stream.
constexpr int kStageRows = 8;

template <typename TT, int LAYOUT>
__global__ __launch_bounds__(256) void stage_kernel(StageArgs a)
{
    using E = typename TT::elem;
    const int col = blockIdx.x * 256 + threadIdx.x;
    const int row0 = blockIdx.y * kStageRows;
    const int view = blockIdx.z;
    if (col >= a.Wp) return;
    const E* src = (const E*)a.src + (size_t)view * a.H * a.W;
    E* dst = (E*)a.dst;
    const int rows = min(kStageRows, a.Hp - row0);
    // pixels (row, col) and (row, col + 1) of the current row
    E p0 = staged_pixel(a, src, row0, col);
    E q0 = (LAYOUT == kQuads || LAYOUT == kDQuads) ? staged_pixel(a, src, row0, col + 1) : E(0);
    for (int k = 0; k < rows; ++k) {
        const int row = row0 + k;
        const size_t e = ((size_t)view * a.Hp + row) * a.Wp + col;
        if (LAYOUT == kRows) {
            dst[e] = p0;
            if (k + 1 < rows) p0 = staged_pixel(a, src, row + 1, col);
            continue;
        }
        const E p1 = staged_pixel(a, src, row + 1, col);
        if (LAYOUT == kPairs) {
            E v[2] = {p0, p1};
            __builtin_memcpy(dst + 2 * e, v, sizeof(v));
        } else if (LAYOUT == kDPairs) {
            E v[2] = {p0, diff_elem(TT{}, p1, p0)};
            __builtin_memcpy(dst + 2 * e, v, sizeof(v));
        } else {
            const E q1 = staged_pixel(a, src, row + 1, col + 1);
            if (LAYOUT == kDQuads) {
                E v[4] = {p0, diff_elem(TT{}, p1, p0), diff_elem(TT{}, q0, p0),
                          diff2_elem(TT{}, q1, q0, p1, p0)};
                __builtin_memcpy(dst + 4 * e, v, sizeof(v));
            } else {
                E v[4] = {p0, q0, p1, q1};
                __builtin_memcpy(dst + 4 * e, v, sizeof(v));
            }
            q0 = q1;
        }
        p0 = p1;
    }
}

template <typename TT>
static void launch_stage_t(const StageArgs& a, dim3 grid, hipStream_t s)
{
    if (a.layout == kRows)
        hipLaunchKernelGGL((stage_kernel<TT, kRows>), grid, dim3(256), 0, s, a);
    else if (a.layout == kPairs)
        hipLaunchKernelGGL((stage_kernel<TT, kPairs>), grid, dim3(256), 0, s, a);
    else if (a.layout == kDPairs)
        hipLaunchKernelGGL((stage_kernel<TT, kDPairs>), grid, dim3(256), 0, s, a);
    else if (a.layout == kDQuads)
        hipLaunchKernelGGL((stage_kernel<TT, kDQuads>), grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((stage_kernel<TT, kQuads>), grid, dim3(256), 0, s, a);
}

hipError_t launch_stage(const StageArgs& a, int storage, hipStream_t s)
{
    dim3 grid((a.Wp + 255) / 256, (a.Hp + kStageRows - 1) / kStageRows, a.count);
    if (storage == kF32)
        launch_stage_t<TF32>(a, grid, s);
    else if (storage == kF16)
        launch_stage_t<TF16>(a, grid, s);
    else
        launch_stage_t<TBF16>(a, grid, s);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// fused
// ---------------------------------------------------------------------------
// The four taps (tl, tr, bl, br) of element (iv, iu): `off` is the byte
// offset of that element, `row` the byte stride of a plane row.  (The
// buffer-load builtins' vector results are reinterpreted whole; extracting
// their elements one by one is miscompiled by this compiler into a single
// dword load.)
template <int LAYOUT>
__device__ __forceinline__ void load_taps(TF32, __amdgpu_buffer_rsrc_t r, uint32_t off,
                                          uint32_t row, float& tl, float& tr, float& bl,
                                          float& br)
{
    if (LAYOUT == kRows) {
        const float2 t = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
        const float2 b = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, off, row, 0));
        tl = t.x; tr = t.y; bl = b.x; br = b.y;
    } else if (LAYOUT == kPairs || LAYOUT == kDPairs) {  // (tl, bl, tr, br); dpairs: bl, br
        // hold the differences bl - tl, br - tr
        const float4 q = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
        tl = q.x; bl = q.y; tr = q.z; br = q.w;
    } else {  // quads: (tl, tr, bl, br); dquads: (p00, dv, dh, dd) in that order
        const float4 q = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
        tl = q.x; tr = q.y; bl = q.z; br = q.w;
    }
}

// 16-bit storage: the two dwords holding the four taps, as loaded.
//   rows : w0 = (tl, tr), w1 = (bl, br)   [low half first]
//   pairs: w0 = (tl, bl), w1 = (tr, br)
//   dpairs: w0 = (tl, bl - tl), w1 = (tr, br - tr)
//   quads: w0 = (tl, tr), w1 = (bl, br)
//   dquads: w0 = (p00, dv), w1 = (dh, dd)
template <int LAYOUT>
__device__ __forceinline__ uint2 load_taps16(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t row)
{
    if (LAYOUT == kRows) {
        uint2 q;
        q.x = __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
        q.y = __builtin_amdgcn_raw_buffer_load_b32(r, off, row, 0);
        return q;
    }
    return __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}

__device__ __forceinline__ float h_lo(uint32_t w)
{
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(w & 0xffffu));
}
__device__ __forceinline__ float h_hi(uint32_t w)
{
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(w >> 16));
}
__device__ __forceinline__ float b_lo(uint32_t w) { return __builtin_bit_cast(float, w << 16); }
__device__ __forceinline__ float b_hi(uint32_t w)
{
    return __builtin_bit_cast(float, w & 0xffff0000u);
}

// bilinear value from FP16 taps: each row is left + au * (right - left)
// evaluated as fma(au, right, fma(-au, left, left)), so that the FP16
// operands feed mixed-precision FMAs directly (no conversions).
__device__ __forceinline__ float lerp16(float a, float left, float right)
{
    return fmaf(a, right, fmaf(-a, left, left));
}

template <int LAYOUT>
__device__ __forceinline__ float bilerp16(TF16, uint2 q, float au, float av)
{
    if (LAYOUT == kDPairs) {
        // columns first: left/right = t + av * d with FP16 operands
        const float left = fmaf(av, h_hi(q.x), h_lo(q.x));
        const float right = fmaf(av, h_hi(q.y), h_lo(q.y));
        return fmaf(au, right - left, left);
    }
    if (LAYOUT == kDQuads)
        return fmaf(au, fmaf(av, h_hi(q.y), h_lo(q.y)), fmaf(av, h_hi(q.x), h_lo(q.x)));
    float top, bot;
    if (LAYOUT == kPairs) {
        top = lerp16(au, h_lo(q.x), h_lo(q.y));
        bot = lerp16(au, h_hi(q.x), h_hi(q.y));
    } else {
        top = lerp16(au, h_lo(q.x), h_hi(q.x));
        bot = lerp16(au, h_lo(q.y), h_hi(q.y));
    }
    return fmaf(av, bot - top, top);
}

template <int LAYOUT>
__device__ __forceinline__ float bilerp16(TBF16, uint2 q, float au, float av)
{
    if (LAYOUT == kDPairs) {
        const float left = fmaf(av, b_hi(q.x), b_lo(q.x));
        const float right = fmaf(av, b_hi(q.y), b_lo(q.y));
        return fmaf(au, right - left, left);
    }
    if (LAYOUT == kDQuads)
        return fmaf(au, fmaf(av, b_hi(q.y), b_lo(q.y)), fmaf(av, b_hi(q.x), b_lo(q.x)));
    float tl, tr, bl, br;
    if (LAYOUT == kPairs) {
        tl = b_lo(q.x); bl = b_hi(q.x); tr = b_lo(q.y); br = b_hi(q.y);
    } else {
        tl = b_lo(q.x); tr = b_hi(q.x); bl = b_lo(q.y); br = b_hi(q.y);
    }
    const float top = fmaf(au, tr - tl, tl);
    const float bot = fmaf(au, br - bl, bl);
    return fmaf(av, bot - top, top);
}

// z voxels whose loads are issued together before their interpolation.
#ifndef FDK_GROUP
#define FDK_GROUP 4
#endif
constexpr int kGroup = FDK_GROUP;
static_assert(kWaveX * kWaveY == 64, "a wave covers 64 columns");

// One view's contribution to the fused_z voxels of this thread.  CLAMP
// selects the clamped tap addressing (needed when some voxel of the wave
// may project outside the zero border of the staged plane); with VCLAMP
// false only u is clamped, and a tap row outside the plane gives a byte
// offset outside the buffer's range, which reads as zero (the host has
// bounded the rows so that the offset cannot wrap into the plane).
//
// The matrices are in the batch's ray frame (column 0 transverse, column 1
// along the rays).  The column base (u'w, v'w, w at z = 0) adds the
// transverse term first and the ray term second (pt, pr: the thread's
// coordinates on those axes), then each voxel its z term: the forward
// projector, which walks the ray axis, rounds every pair's coordinates in
// this same order.
template <typename TT, int LAYOUT, bool WCHECK, bool CLAMP, bool VCLAMP>
__device__ __forceinline__ void accumulate_view(const FusedArgs& A, const const_float* m, float pt,
                                                float pr, float zp0,
                                                __amdgpu_buffer_rsrc_t rsrc,
                                                float (&acc)[fused_z(TT::id)])
{
    constexpr int kFusedZ = fused_z(TT::id);
    using E = typename TT::elem;
    constexpr bool kIsF32 = sizeof(E) == 4;
    constexpr uint32_t kElem = sizeof(E) * layout_width(LAYOUT);
    const int Wp = A.Wp;
    const uint32_t row_bytes = (uint32_t)Wp * kElem;
    const uint32_t centre_bytes = (uint32_t)A.origin_off * kElem;
    const float bu = fmaf(m[1], pr, fmaf(m[0], pt, m[3]));
    const float bv = fmaf(m[5], pr, fmaf(m[4], pt, m[7]));
    const float bw = fmaf(m[9], pr, fmaf(m[8], pt, m[11]));
#pragma unroll
    for (int g = 0; g < kFusedZ; g += kGroup) {
        float au[kGroup], av[kGroup], r2[kGroup];
        float tl[kGroup], tr[kGroup], bl[kGroup], br[kGroup];  // FP32 storage
        uint2 raw[kGroup];                                      // 16-bit storage
#pragma unroll
        for (int q = 0; q < kGroup; ++q) {
            const float zp = zp0 + (float)(g + q);
            // part 1
            const float uw = fmaf(zp, m[2], bu);
            const float vw = fmaf(zp, m[6], bv);
            const float w = fmaf(zp, m[10], bw);
            float r = __builtin_amdgcn_rcpf(w);
            if (WCHECK) r = (w > 0.0f) ? r : 0.0f;
            const float u = uw * r;
            const float v = vw * r;
            r2[q] = r * r;
            // part 2
            au[q] = __builtin_amdgcn_fractf(u);
            av[q] = __builtin_amdgcn_fractf(v);
            const int iu = cvt_floor(CLAMP ? __builtin_amdgcn_fmed3f(u, A.lo_u, A.hi_u) : u);
            const int iv =
                cvt_floor(CLAMP && VCLAMP ? __builtin_amdgcn_fmed3f(v, A.lo_v, A.hi_v) : v);
            const uint32_t off = (uint32_t)mad_i24(iv, Wp, iu) * kElem + centre_bytes;
            if constexpr (kIsF32)
                load_taps<LAYOUT>(TT{}, rsrc, off, row_bytes, tl[q], tr[q], bl[q], br[q]);
            else
                raw[q] = load_taps16<LAYOUT>(rsrc, off, row_bytes);
        }
#pragma unroll
        for (int q = 0; q < kGroup; ++q) {
            // part 3
            float fx;
            if constexpr (kIsF32 && LAYOUT == kDQuads) {
                // (tl, tr, bl, br) hold (p00, dv, dh, dd)
                fx = fmaf(au[q], fmaf(av[q], br[q], bl[q]), fmaf(av[q], tr[q], tl[q]));
            } else if constexpr (kIsF32 && LAYOUT == kDPairs) {
                // bl, br hold the vertical differences
                const float left = fmaf(av[q], bl[q], tl[q]);
                const float right = fmaf(av[q], br[q], tr[q]);
                fx = fmaf(au[q], right - left, left);
            } else if constexpr (kIsF32) {
                const float top = fmaf(au[q], tr[q] - tl[q], tl[q]);
                const float bot = fmaf(au[q], br[q] - bl[q], bl[q]);
                fx = fmaf(av[q], bot - top, top);
            } else {
                fx = bilerp16<LAYOUT>(TT{}, raw[q], au[q], av[q]);
            }
            acc[g + q] = fmaf(r2[q], fx, acc[g + q]);
        }
    }
}

// waves per SIMD the register budget is fitted to (512 VGPRs / 8 = 64)
#ifndef FDK_MIN_WAVES
#define FDK_MIN_WAVES 8
#endif
template <typename TT, int LAYOUT, bool WCHECK, bool VCLAMP>
__global__ __launch_bounds__(kThreads, WCHECK ? 7 : FDK_MIN_WAVES) void bp_fused_kernel(const FusedArgs A)
{
    using E = typename TT::elem;
    constexpr uint32_t kElem = sizeof(E) * layout_width(LAYOUT);
    constexpr int kFusedZ = fused_z(TT::id);
    int bid = blockIdx.x;
    if (A.xcd_remap) {
        const int per = gridDim.x >> 3;
        bid = (bid & 7) * per + (bid >> 3);
    }
    // Workgroup order: the tile axis closest to the batch's rays fastest,
    // then the z chunks, then the transverse axis.  With the XCD remap an
    // XCD gets a contiguous range of this order: a slab a few tiles thick
    // across the rays, spanning the whole ray extent and all z, whose
    // projection is a narrow band of detector columns, and the workgroups
    // resident on it at one time form a compact box along the rays.
    // (Measured on fdk512 FP32: 40.8 ms per backprojection with the z chunks
    // slowest, 34.6 ms in this order.)
    const int t0 = bid % (A.y_fastest ? A.tiles_y : A.tiles_x);
    const int rest = bid / (A.y_fastest ? A.tiles_y : A.tiles_x);
    const int zc = rest % A.zchunks;
    const int t1 = rest / A.zchunks;
    const int tx = A.y_fastest ? t1 : t0;
    const int ty = A.y_fastest ? t0 : t1;

    // each 64-lane wave covers a kWaveX x kWaveY patch of columns
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wx0 = tx * kTileX;
    const int wy0 = ty * kTileY + wave * kWaveY;
    const int x = wx0 + (lane % kWaveX);
    const int y = wy0 + (lane / kWaveX);
    const int zl0 = zc * kFusedZ;  // first z of this thread, relative to z_first
    const float xp = (float)x - A.c;
    const float yp = (float)y - A.c;
    const float zp0 = (float)(A.z_first + zl0) - A.c;
    const float pt = A.y_fastest ? xp : yp;  // transverse and ray coordinates
    const float pr = A.y_fastest ? yp : xp;

    // Lanes 0..7 hold the corners of the wave's kWaveX x kWaveY x kFusedZ
    // voxel box.  With w > 0 on the box, every voxel projects inside the
    // hull of the corner projections, which decides per view whether the
    // whole wave misses the detector (its taps are all zero: skip the view,
    // the paper's clipping of Section 3.3) or stays inside the zero border
    // (no clamping needed).  A 0.5 pixel margin absorbs rounding.
    const float cxp = (float)(wx0 + ((lane & 1) ? kWaveX - 1 : 0)) - A.c;
    const float cyp = (float)(wy0 + ((lane & 2) ? kWaveY - 1 : 0)) - A.c;
    const float czp = zp0 + ((lane & 4) ? (float)(kFusedZ - 1) : 0.0f);
    const float ctp = A.y_fastest ? cxp : cyp, crp = A.y_fastest ? cyp : cxp;
    const bool corner_lane = lane < 8;

    float acc[kFusedZ];
#pragma unroll
    for (int i = 0; i < kFusedZ; ++i) acc[i] = 0.0f;

    const uint32_t plane_bytes = (uint32_t)(A.plane * (long long)kElem);
    const char* plane = (const char*)A.img;
    const const_float* mats = as_constant(A.m);
    for (int j = 0; j < A.count; ++j, plane += plane_bytes) {
        const const_float* m = mats + 12 * j;
        const __amdgpu_buffer_rsrc_t rsrc = make_rsrc(plane, plane_bytes);
        if constexpr (WCHECK) {
            accumulate_view<TT, LAYOUT, WCHECK, true, true>(A, m, pt, pr, zp0, rsrc, acc);
        } else {
            const float cu = fmaf(czp, m[2], fmaf(m[1], crp, fmaf(m[0], ctp, m[3])));
            const float cv = fmaf(czp, m[6], fmaf(m[5], crp, fmaf(m[4], ctp, m[7])));
            const float cw = fmaf(czp, m[10], fmaf(m[9], crp, fmaf(m[8], ctp, m[11])));
            const float cr = __builtin_amdgcn_rcpf(cw);
            const float u = cu * cr, v = cv * cr;
            if (__all(!corner_lane || u < A.skip_lo_u) || __all(!corner_lane || u > A.skip_hi_u) ||
                __all(!corner_lane || v < A.skip_lo_v) || __all(!corner_lane || v > A.skip_hi_v))
                continue;
            accumulate_view<TT, LAYOUT, false, true, VCLAMP>(A, m, pt, pr, zp0, rsrc, acc);
        }
    }

    if (x < A.N && y < A.N) {
        const size_t slice = (size_t)A.N * A.N;
        float* out = A.vol + (size_t)(A.z_first + zl0) * slice + (size_t)y * A.N + x;
        if (zl0 + kFusedZ <= A.nz) {
            // all the column's loads in flight together (a test per voxel
            // would make the compiler wait for each before the next)
            float old[kFusedZ];
#pragma unroll
            for (int i = 0; i < kFusedZ; ++i) old[i] = out[(size_t)i * slice];
#pragma unroll
            for (int i = 0; i < kFusedZ; ++i) out[(size_t)i * slice] = old[i] + acc[i];
        } else {
#pragma unroll
            for (int i = 0; i < kFusedZ; ++i)
                if (zl0 + i < A.nz) out[(size_t)i * slice] += acc[i];
        }
    }
}

template <typename TT, int LAYOUT>
static void launch_fused_t(const FusedArgs& a, bool wcheck, bool rows_free, hipStream_t s)
{
    dim3 grid(a.tiles_x * a.tiles_y * a.zchunks);
    if (wcheck)
        hipLaunchKernelGGL((bp_fused_kernel<TT, LAYOUT, true, true>), grid, dim3(kThreads), 0, s,
                           a);
    else if constexpr (sizeof(typename TT::elem) == 2 && LAYOUT != kRows) {
        if (rows_free)
            hipLaunchKernelGGL((bp_fused_kernel<TT, LAYOUT, false, false>), grid, dim3(kThreads),
                               0, s, a);
        else
            hipLaunchKernelGGL((bp_fused_kernel<TT, LAYOUT, false, true>), grid, dim3(kThreads),
                               0, s, a);
    } else
        hipLaunchKernelGGL((bp_fused_kernel<TT, LAYOUT, false, true>), grid, dim3(kThreads), 0, s,
                           a);
}

template <typename TT>
static void launch_fused_l(const FusedArgs& a, int layout, bool wcheck, bool rows_free,
                           hipStream_t s)
{
    if (layout == kRows)
        launch_fused_t<TT, kRows>(a, wcheck, false, s);
    else if (layout == kPairs)
        launch_fused_t<TT, kPairs>(a, wcheck, rows_free, s);
    else if (layout == kDPairs)
        launch_fused_t<TT, kDPairs>(a, wcheck, rows_free, s);
    else if (layout == kDQuads)
        launch_fused_t<TT, kDQuads>(a, wcheck, rows_free, s);
    else
        launch_fused_t<TT, kQuads>(a, wcheck, rows_free, s);
}

hipError_t launch_fused(const FusedArgs& a, int storage, int layout, bool wcheck, bool rows_free,
                        hipStream_t s)
{
    if (storage == kF32)
        launch_fused_l<TF32>(a, layout, wcheck, rows_free, s);
    else if (storage == kF16)
        launch_fused_l<TF16>(a, layout, wcheck, rows_free, s);
    else
        launch_fused_l<TBF16>(a, layout, wcheck, rows_free, s);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// plain
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void bp_plain_kernel(const PlainArgs A)
{
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= A.N || y >= A.N) return;
    const float wx = A.ox + (float)x * A.vs;
    const float wy = A.oy + (float)y * A.vs;
    const float wz = A.oz + (float)z * A.vs;
    const int H = A.H, W = A.W;
    float sum = 0.0f;
    const float* I = A.proj;
    for (int j = 0; j < A.count; ++j, I += (size_t)H * W) {
        const float* m = A.m[j];
        const float uw = m[0] * wx + m[1] * wy + m[2] * wz + m[3];
        const float vw = m[4] * wx + m[5] * wy + m[6] * wz + m[7];
        const float w = m[8] * wx + m[9] * wy + m[10] * wz + m[11];
        if (!(w > 0.0f)) continue;
        const float u = uw / w;
        const float v = vw / w;
        if (!(u > -2.0f && u < (float)W + 1.0f && v > -2.0f && v < (float)H + 1.0f)) continue;
        const float fu = floorf(u), fv = floorf(v);
        const int iu = (int)fu, iv = (int)fv;
        const float scalx = u - fu, scaly = v - fv;
        float valtl = 0.0f, valtr = 0.0f, valbl = 0.0f, valbr = 0.0f;
        if (iv >= 0 && iv < H) {
            if (iu >= 0 && iu < W) valtl = I[iv * W + iu];
            if (iu >= -1 && iu < W - 1) valtr = I[iv * W + iu + 1];
        }
        if (iv >= -1 && iv < H - 1) {
            if (iu >= 0 && iu < W) valbl = I[(iv + 1) * W + iu];
            if (iu >= -1 && iu < W - 1) valbr = I[(iv + 1) * W + iu + 1];
        }
        const float vall = scaly * valbl + (1.0f - scaly) * valtl;
        const float valr = scaly * valbr + (1.0f - scaly) * valtr;
        const float fx = scalx * valr + (1.0f - scalx) * vall;
        sum += 1.0f / (w * w) * fx;
    }
    A.vol[((size_t)z * A.N + y) * A.N + x] += sum;
}

hipError_t launch_plain(const PlainArgs& a, hipStream_t s)
{
    dim3 grid((a.N + 63) / 64, (a.N + 3) / 4, a.N);
    hipLaunchKernelGGL(bp_plain_kernel, grid, dim3(64, 4), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// matrices from the kernel arguments to device memory
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void put_mats_kernel(const PutMatsArgs a)
{
    for (int i = threadIdx.x; i < 12 * a.count; i += 256) a.dst[i] = a.m[i];
}

hipError_t launch_put_mats(const PutMatsArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(put_mats_kernel, dim3(1), dim3(256), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// update probe
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void update_probe_kernel(float* a, size_t n, float s)
{
    const size_t n4 = n / 4;
    float4* a4 = (float4*)a;
    const size_t stride = (size_t)gridDim.x * 256;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += stride) {
        float4 v = a4[i];
        v.x *= s; v.y *= s; v.z *= s; v.w *= s;
        a4[i] = v;
    }
    for (size_t i = n4 * 4 + (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride)
        a[i] *= s;
}

hipError_t launch_update_probe(float* a, size_t n, float s, hipStream_t st)
{
    size_t blocks = (n / 4 + 255) / 256;
    if (blocks > 256 * 64) blocks = 256 * 64;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(update_probe_kernel, dim3((unsigned)blocks), dim3(256), 0, st, a, n, s);
    return hipGetLastError();
}

}  // namespace fdk
