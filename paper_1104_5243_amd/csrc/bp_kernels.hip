// Backprojection kernels for gfx950 (CDNA4).
//
// fused: the optimised kernel.  One thread owns an (x, y) voxel column and
//   kFusedZ consecutive z voxels; the views of a batch are fused in one
//   pass with the kFusedZ voxel sums held in registers, so the volume is
//   read and written once per batch (the image-loop blocking of the paper's
//   Section 6.3, with registers in place of the L1-resident voxel line).
//   Per (voxel, view) the work is the paper's three parts (Section 3.2):
//     part 1: (u'w, v'w, w) by three FMAs from a per-column base, one
//             reciprocal r = 1/w, u' = u'w r, v' = v'w r;
//     part 2: floor / fraction, clamp into the staged plane's zero border,
//             two 2-element loads (the horizontally adjacent tap pairs the
//             paper loads pairwise, Section 4.1);
//     part 3: bilinear interpolation and acc += r^2 * fx.
//   The projections are read from zero-padded staged planes (Section 3.3),
//   so no tap needs a bounds test: out-of-detector taps are clamped onto
//   the zero border.
// plain: one thread per voxel with the listing's arithmetic in world
//   coordinates (two IEEE divisions, bounds-tested taps), for comparison.
// stage: copies a batch of views into zero-padded planes.
// update probe: a[i] = s * a[i], the paper's bandwidth benchmark.
#include "fdk_internal.h"

namespace fdk {

// ---------------------------------------------------------------------------
// storage types
// ---------------------------------------------------------------------------
struct TF32 { using elem = float; };
struct TF16 { using elem = uint16_t; };
struct TBF16 { using elem = uint16_t; };

__device__ __forceinline__ void load_pair(TF32, const float* p, float& a, float& b)
{
    float2 t;
    __builtin_memcpy(&t, p, sizeof(t));  // 4-byte aligned 8-byte load
    a = t.x;
    b = t.y;
}

__device__ __forceinline__ void load_pair(TF16, const uint16_t* p, float& a, float& b)
{
    uint32_t t;
    __builtin_memcpy(&t, p, sizeof(t));
    a = (float)__builtin_bit_cast(_Float16, (uint16_t)(t & 0xffffu));
    b = (float)__builtin_bit_cast(_Float16, (uint16_t)(t >> 16));
}

__device__ __forceinline__ void load_pair(TBF16, const uint16_t* p, float& a, float& b)
{
    uint32_t t;
    __builtin_memcpy(&t, p, sizeof(t));
    a = __builtin_bit_cast(float, t << 16);
    b = __builtin_bit_cast(float, t & 0xffff0000u);
}

// floor(x) as an integer in one instruction (x is finite and clamped).
__device__ __forceinline__ int cvt_floor(float x)
{
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// a * b + c on 24-bit signed a, b (|a|, |b| < 2^23) in one instruction.
__device__ __forceinline__ int mad_i24(int a, int b, int c)
{
    int r;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// ---------------------------------------------------------------------------
// stage
// ---------------------------------------------------------------------------
template <typename E>
__global__ __launch_bounds__(256) void stage_kernel(StageArgs a)
{
    const int col = blockIdx.x * 256 + threadIdx.x;
    const int row = blockIdx.y;
    const int view = blockIdx.z;
    if (col >= a.Wp) return;
    const int j = col - kPad, k = row - kPad;
    const E* src = (const E*)a.src + (size_t)view * a.H * a.W;
    E v = E(0);
    if (j >= 0 && j < a.W && k >= 0 && k < a.H) v = src[(size_t)k * a.W + j];
    ((E*)a.dst)[((size_t)view * a.Hp + row) * a.Wp + col] = v;
}

hipError_t launch_stage(const StageArgs& a, int storage, hipStream_t s)
{
    dim3 grid((a.Wp + 255) / 256, a.Hp, a.count);
    if (storage == kF32)
        hipLaunchKernelGGL(stage_kernel<float>, grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(stage_kernel<uint16_t>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// fused
// ---------------------------------------------------------------------------
// Raw buffer loads: a 32-bit byte offset per lane, the plane base in a
// buffer descriptor, and the second tap row reached through the scalar
// offset.  An offset outside the descriptor's range would read 0 instead of
// faulting; the clamps keep every offset inside the staged plane.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                             0x00020000);
}

__device__ __forceinline__ void load_pair_buf(TF32, __amdgpu_buffer_rsrc_t r, uint32_t off,
                                              uint32_t soff, float& a, float& b)
{
    auto t = __builtin_amdgcn_raw_buffer_load_b64(r, off, soff, 0);
    float2 f = __builtin_bit_cast(float2, t);
    a = f.x;
    b = f.y;
}

__device__ __forceinline__ void load_pair_buf(TF16, __amdgpu_buffer_rsrc_t r, uint32_t off,
                                              uint32_t soff, float& a, float& b)
{
    uint32_t t = __builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0);
    a = (float)__builtin_bit_cast(_Float16, (uint16_t)(t & 0xffffu));
    b = (float)__builtin_bit_cast(_Float16, (uint16_t)(t >> 16));
}

__device__ __forceinline__ void load_pair_buf(TBF16, __amdgpu_buffer_rsrc_t r, uint32_t off,
                                              uint32_t soff, float& a, float& b)
{
    uint32_t t = __builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0);
    a = __builtin_bit_cast(float, t << 16);
    b = __builtin_bit_cast(float, t & 0xffff0000u);
}

// z voxels whose loads are issued together before their interpolation.
constexpr int kGroup = 4;

template <typename TT, bool WCHECK>
__global__ __launch_bounds__(256) void bp_fused_kernel(const FusedArgs A)
{
    using E = typename TT::elem;
    int bid = blockIdx.x;
    if (A.xcd_remap) {
        const int per = gridDim.x >> 3;
        bid = (bid & 7) * per + (bid >> 3);
    }
    const int tx = bid % A.tiles_x;
    const int rest = bid / A.tiles_x;
    const int ty = rest % A.tiles_y;
    const int zc = rest / A.tiles_y;

    const int x = tx * kFusedTile + (threadIdx.x & (kFusedTile - 1));
    const int y = ty * kFusedTile + (threadIdx.x / kFusedTile);
    const int zl0 = zc * kFusedZ;  // first z of this thread, relative to z_first
    const float xp = (float)x - A.c;
    const float yp = (float)y - A.c;
    const float zp0 = (float)(A.z_first + zl0) - A.c;

    float acc[kFusedZ];
#pragma unroll
    for (int i = 0; i < kFusedZ; ++i) acc[i] = 0.0f;

    const int Wp = A.Wp;
    const uint32_t row_bytes = (uint32_t)Wp * sizeof(E);
    const uint32_t plane_bytes = (uint32_t)(A.plane * (long long)sizeof(E));
    const uint32_t centre_bytes = (uint32_t)A.origin_off * sizeof(E);
    const E* plane = (const E*)A.img;
    for (int j = 0; j < A.count; ++j, plane += A.plane) {
        const __amdgpu_buffer_rsrc_t rsrc = make_rsrc(plane, plane_bytes);
        const float* m = A.m[j];
        const float bu = fmaf(m[1], yp, fmaf(m[0], xp, m[3]));
        const float bv = fmaf(m[5], yp, fmaf(m[4], xp, m[7]));
        const float bw = fmaf(m[9], yp, fmaf(m[8], xp, m[11]));
#pragma unroll
        for (int g = 0; g < kFusedZ; g += kGroup) {
            float au[kGroup], av[kGroup], r2[kGroup];
            float tl[kGroup], tr[kGroup], bl[kGroup], br[kGroup];
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
                const int iu = cvt_floor(__builtin_amdgcn_fmed3f(u, A.lo_u, A.hi_u));
                const int iv = cvt_floor(__builtin_amdgcn_fmed3f(v, A.lo_v, A.hi_v));
                const uint32_t off =
                    (uint32_t)mad_i24(iv, Wp, iu) * (uint32_t)sizeof(E) + centre_bytes;
                load_pair_buf(TT{}, rsrc, off, 0, tl[q], tr[q]);
                load_pair_buf(TT{}, rsrc, off, row_bytes, bl[q], br[q]);
            }
#pragma unroll
            for (int q = 0; q < kGroup; ++q) {
                // part 3
                const float top = fmaf(au[q], tr[q] - tl[q], tl[q]);
                const float bot = fmaf(au[q], br[q] - bl[q], bl[q]);
                const float fx = fmaf(av[q], bot - top, top);
                acc[g + q] = fmaf(r2[q], fx, acc[g + q]);
            }
        }
    }

    if (x < A.N && y < A.N) {
        const size_t slice = (size_t)A.N * A.N;
        float* out = A.vol + (size_t)(A.z_first + zl0) * slice + (size_t)y * A.N + x;
#pragma unroll
        for (int i = 0; i < kFusedZ; ++i)
            if (zl0 + i < A.nz) out[(size_t)i * slice] += acc[i];
    }
}

hipError_t launch_fused(const FusedArgs& a, int storage, bool wcheck, hipStream_t s)
{
    dim3 grid(a.tiles_x * a.tiles_y * a.zchunks);
#define FDK_LAUNCH(TT)                                                              \
    do {                                                                            \
        if (wcheck)                                                                 \
            hipLaunchKernelGGL((bp_fused_kernel<TT, true>), grid, dim3(256), 0, s, a);  \
        else                                                                        \
            hipLaunchKernelGGL((bp_fused_kernel<TT, false>), grid, dim3(256), 0, s, a); \
    } while (0)
    if (storage == kF32)
        FDK_LAUNCH(TF32);
    else if (storage == kF16)
        FDK_LAUNCH(TF16);
    else
        FDK_LAUNCH(TBF16);
#undef FDK_LAUNCH
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
