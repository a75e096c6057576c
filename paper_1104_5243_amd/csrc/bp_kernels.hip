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
#include "anchor.h"
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
// storage conversion (FP32 stack -> FP16 with per-view powers of 4, or BF16)
// ---------------------------------------------------------------------------
// One workgroup per view: the largest |value| of the view, then k, the
// largest integer with 4^k amax <= 2^14, clipped to [-60, 60] (k = 0 for an
// all-zero view), and view_scale = 4^-k.  k is found from the exponent and
// significand of amax exactly (no logarithms): with amax = m 2^e, m in
// [1, 2) and t = 14 - e, 4^k amax <= 2^14 holds iff 2k <= t when m = 1 and
// 2k <= t - 1 otherwise.
__global__ __launch_bounds__(1024) void view_scale_kernel(const float* src, size_t view_len,
                                                          float* view_scale)
{
    __shared__ float part[16];
    const float* v = src + (size_t)blockIdx.x * view_len;
    float amax = 0.0f;
    // 16-byte loads where the view starts 16-byte aligned, the rest one by one
    const size_t lead = ((16 - ((uintptr_t)v & 15)) & 15) / 4;
    const size_t head = lead < view_len ? lead : view_len;
    const size_t n4 = (view_len - head) / 4;
    const float4* v4 = (const float4*)(v + head);
    for (size_t i = threadIdx.x; i < n4; i += 1024) {
        const float4 q = v4[i];
        amax = fmaxf(amax, fmaxf(fmaxf(fabsf(q.x), fabsf(q.y)), fmaxf(fabsf(q.z), fabsf(q.w))));
    }
    for (size_t i = threadIdx.x; i < head; i += 1024) amax = fmaxf(amax, fabsf(v[i]));
    for (size_t i = head + 4 * n4 + threadIdx.x; i < view_len; i += 1024)
        amax = fmaxf(amax, fabsf(v[i]));
    for (int d = 32; d >= 1; d >>= 1) amax = fmaxf(amax, __shfl_xor(amax, d));
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = amax;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 16; ++w) amax = fmaxf(amax, part[w]);
        int k = 0;
        if (amax > 0.0f) {
            int e;
            const float m = 2.0f * frexpf(amax, &e);  // amax = m 2^(e-1), m in [1, 2)
            const int t = 14 - (e - 1) - (m > 1.0f ? 1 : 0);
            k = t >= 0 ? t / 2 : -((1 - t) / 2);  // floor(t / 2)
            k = min(max(k, -60), 60);
        }
        view_scale[blockIdx.x] = __builtin_ldexpf(1.0f, -2 * k);
    }
}

// dst = round-to-nearest-even(src / view_scale[view]) in FP16, or
// round-to-nearest-even(src) in BF16 (view_scale unused).  blockIdx.y is
// the view.  The FP16 scaling is an exponent shift (ldexp by 2k with
// view_scale = 4^-k): exact, sign of zero kept, subnormals rounded once.
template <typename TT>
__global__ __launch_bounds__(256) void convert_kernel(uint16_t* dst, const float* src,
                                                      size_t view_len, const float* view_scale)
{
    const size_t off = (size_t)blockIdx.y * view_len;
    int shift = 0;
    if constexpr (TT::id == kF16) {
        int e;
        frexpf(view_scale[blockIdx.y], &e);  // view_scale = 2^(e-1) = 4^-k
        shift = 1 - e;                       // 2k
    }
    const size_t stride = (size_t)gridDim.x * 256;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < view_len; i += stride) {
        float x = src[off + i];
        if constexpr (TT::id == kF16) x = __builtin_ldexpf(x, shift);
        dst[off + i] = from_f(TT{}, x);
    }
}

hipError_t launch_convert(void* dst, const float* src, int n_views, size_t view_len, int storage,
                          float* view_scale, hipStream_t s)
{
    if (storage == kF16)
        hipLaunchKernelGGL(view_scale_kernel, dim3(n_views), dim3(1024), 0, s, src, view_len,
                           view_scale);
    size_t bx = (view_len + 255) / 256;
    if (bx > 64) bx = 64;
    const dim3 grid((unsigned)bx, (unsigned)n_views);
    if (storage == kF16)
        hipLaunchKernelGGL(convert_kernel<TF16>, grid, dim3(256), 0, s, (uint16_t*)dst, src,
                           view_len, (const float*)view_scale);
    else
        hipLaunchKernelGGL(convert_kernel<TBF16>, grid, dim3(256), 0, s, (uint16_t*)dst, src,
                           view_len, (const float*)view_scale);
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
static_assert(fused_z(kF32) % kGroup == 0 && fused_z(kF16) % kGroup == 0,
              "a thread's z voxels split into whole groups");

// One view's contribution to the fused_z voxels of this thread, from the
// view's anchor (uniform over the wave) and the thread's offsets (d_t, d_r)
// from the box's centre column; voxel i is slice i of the box.  Taps are
// clamped into the staged plane's zero border (integer clamps of the
// anchored indices); with VCLAMP false only u is clamped, and a tap row
// outside the plane gives a byte offset outside the buffer's range, which
// reads as zero (the host has bounded the rows so that the offset cannot
// wrap into the plane).  With CLAMP false nothing is clamped: for a box
// whose projected hull lies a pixel inside the clamp ranges, where every
// clamp of a voxel inside the volume is a no-op (lanes of voxels beyond the
// volume's edge may then read anywhere: their loads stay within the plane's
// range-checked buffer and their sums are never written).
template <typename TT, int LAYOUT, bool WCHECK, bool VCLAMP, int DIV, bool CLAMP = true>
__device__ __forceinline__ void accumulate_view(
    const FusedArgs& A, float uc, float vc, float wc, float su_t, float su_r, float su2,
    float sv_t, float sv_r, float sv2, float sw_t, float sw_r, float sw2, int lo_u, int hi_u,
    int lo_v, int hi_v, int base, float d_t, float d_r, __amdgpu_buffer_rsrc_t rsrc,
    float (&acc)[fused_z(TT::id)])
{
    constexpr int kFusedZ = fused_z(TT::id);
    using E = typename TT::elem;
    constexpr bool kIsF32 = sizeof(E) == 4;
    constexpr uint32_t kElem = sizeof(E) * layout_width(LAYOUT);
    const int Wp = A.Wp;
    const uint32_t row_bytes = (uint32_t)Wp * kElem;
    float bu, bv, bw;
    column_base(uc, vc, wc, su_t, su_r, sv_t, sv_r, sw_t, sw_r, d_t, d_r, bu, bv, bw);
#pragma unroll
    for (int g = 0; g < kFusedZ; g += kGroup) {
        float au[kGroup], av[kGroup], r2[kGroup];
        float tl[kGroup], tr[kGroup], bl[kGroup], br[kGroup];  // FP32 storage
        uint2 raw[kGroup];                                      // 16-bit storage
#pragma unroll
        for (int q = 0; q < kGroup; ++q) {
            // part 1
            float u, v, r;
            voxel_coords<DIV, WCHECK>(bu, bv, bw, su2, sv2, sw2, (float)(g + q), u, v, r);
            r2[q] = r * r;
            // part 2
            au[q] = __builtin_amdgcn_fractf(u);
            av[q] = __builtin_amdgcn_fractf(v);
            const int ju = CLAMP ? med3_i32(cvt_floor(u), lo_u, hi_u) : cvt_floor(u);
            const int jv = (CLAMP && VCLAMP) ? med3_i32(cvt_floor(v), lo_v, hi_v) : cvt_floor(v);
            const uint32_t off = (uint32_t)(mad_i24_ub(jv, Wp, ju) + base) * kElem;
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

// waves per SIMD the register budget is fitted to (512 VGPRs / 7 = 72: with
// the clamp-free copy of the voxel loop, 8 waves' 64 VGPRs spill inside it)
#ifndef FDK_MIN_WAVES
#define FDK_MIN_WAVES 7
#endif
template <typename TT, int LAYOUT, bool WCHECK, bool VCLAMP, int DIV>
__global__ __launch_bounds__(kThreads, WCHECK ? 7 : FDK_MIN_WAVES) void bp_fused_kernel(const FusedArgs A)
{
    using E = typename TT::elem;
    constexpr uint32_t kElem = sizeof(E) * layout_width(LAYOUT);
    constexpr int kFusedZ = fused_z(TT::id);
    // The launch's workgroups go to the 8 XCDs in turn (workgroup i to XCD
    // i mod 8); each XCD takes whole transverse tiles of the workgroup order
    // below (slabs one tile thick across the rays), so that the views'
    // footprints of a slab share its L2.  The slabs at the volume's edges
    // across the rays execute fewer (box, view) pairs (more of their boxes
    // miss the detector), so XCD x takes tiles x, x + 8, x + 16, ..., spread
    // from the edges to the centre, rather than one contiguous eighth of the
    // order (fdk512 FP32: 2014.6 -> 2062.3 GUP/s, fdk1024: 211 -> 205 ms per
    // backprojection; bit-identical).
    int bid = blockIdx.x;
    if (A.xcd_remap) {
        const int xcd = bid & 7, k = bid >> 3;
        const int across = A.y_fastest ? A.tiles_x : A.tiles_y;
        if (across % 8 == 0) {
            const int slab = gridDim.x / across;  // workgroups of one transverse tile
            bid = (xcd + 8 * (k / slab)) * slab + k % slab;
        } else {
            bid = xcd * (gridDim.x >> 3) + k;
        }
    }
    // Workgroup order: the tile axis closest to the batch's rays fastest,
    // then the z chunks, then the transverse axis.  With the XCD remap an
    // XCD gets contiguous ranges of this order: slabs a tile thick across
    // the rays, spanning the whole ray extent and all z, whose
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

    // each 64-lane wave covers a kWaveX x kWaveY patch of columns (the wave
    // index is uniform: read it into a scalar register).  Lanes are laid out
    // in the batch's ray frame: consecutive lanes step across the rays, and
    // lanes 8 apart along them.  Columns along a ray project onto nearly the
    // same pixel, so every gather's eight pixels are each read by eight
    // lanes 8 apart; with the lanes in x/y order, batches whose rays run
    // along x had those eight lanes consecutive instead, and their launches
    // took ~15 % longer (fdk512 FP32: 32.0 -> 29.9 ms per backprojection,
    // FP16 28.2 -> 25.6 ms; bit-identical).
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int wx0, wy0;
    wave_origin(A.y_fastest != 0, tx, ty, wave, wx0, wy0);
    static_assert(kWaveX == kWaveY, "a square wave patch (either axis may run across the rays)");
    const int lx = A.y_fastest ? (lane % kWaveX) : (lane / kWaveX);
    const int ly = A.y_fastest ? (lane / kWaveX) : (lane % kWaveX);
    const int zl0 = zc * kFusedZ;  // first z of this thread, relative to z_first
    // the part of this wave's box inside the volume (kept in scalar
    // registers) and this thread's offsets from its centre column
    BoxFrame bf = box_frame(A, wx0, wy0, A.z_first + zl0, kWaveX, kWaveY, kFusedZ);
    bf.cx = uniform_f(bf.cx);
    bf.cy = uniform_f(bf.cy);
    bf.z0 = uniform_f(bf.z0);
    bf.hx = uniform_f(bf.hx);
    bf.hy = uniform_f(bf.hy);
    bf.hz = uniform_f(bf.hz);
    // the box's centre in FP64 for the anchors, in scalar registers (held in
    // vector registers, these copies and the clamp-free bounds were spilled
    // to scratch: fdk512 FP32 28.6 -> 28.0 ms per backprojection, fdk1024
    // 195.0 -> 191.5 ms; bit-identical)
    const BoxCentre bc = uniform_box_centre(bf);
    const float dx = (float)lx - bf.hx;
    const float dy = (float)ly - bf.hy;
    const float d_t = A.y_fastest ? dx : dy;  // transverse and ray offsets
    const float d_r = A.y_fastest ? dy : dx;

    float acc[kFusedZ];
#pragma unroll
    for (int i = 0; i < kFusedZ; ++i) acc[i] = 0.0f;

    // The anchors of up to 64 views, one row of 16 words per view, in this
    // wave's part of LDS: computed one view per lane, then read back per
    // view at a wave-uniform address (a broadcast), so that they occupy
    // vector registers only while their view is processed.  Row: uc, vc,
    // wc, the u and v slopes (transverse, ray, z), the element offset of
    // pixel (a_u + ku, a_v + kv) in a plane, the tap index clamp ranges
    // shifted by the anchor, the w row's z slope and the clamp-free flag.
    // (The w row's x and y slopes are the folded matrix's, read as scalars.)
    __shared__ float anchors[kWgWaves][64][16];
    float(*an_rows)[16] = anchors[wave];
    const uint32_t plane_bytes = (uint32_t)(A.plane * (long long)kElem);
    const char* plane = (const char*)A.img;
    const const_float* mats = as_constant(A.m);
    for (int j0 = 0; j0 < A.count; j0 += 64) {
        // lane L: the anchor of view j0 + L; WCHECK batches (some voxel may
        // have w <= 0) keep a_u = a_v = 0 and skip nothing
        uint64_t skip;
        {
            const Anchor an = make_anchor<!WCHECK>(A, j0 + lane, bf, bc);
            skip = __ballot(an.skip);
            // the box's hull a pixel inside the tap clamp ranges: the view
            // takes the clamp-free voxel loop
            const bool inside = !WCHECK && an.wmin > 0.0f && an.umin >= A.in_lo_u &&
                                an.umax <= A.in_hi_u && an.vmin >= A.in_lo_v &&
                                an.vmax <= A.in_hi_v;
            const int base = an.av * A.Wp + an.au + A.origin_off;
            float* row = an_rows[lane];
            *(float4*)row = make_float4(an.uc, an.vc, an.wc, an.su_t);
            *(float4*)(row + 4) = make_float4(an.su_r, an.su2, an.sv_t, an.sv_r);
            *(float4*)(row + 8) = make_float4(an.sv2, __builtin_bit_cast(float, base),
                                              __builtin_bit_cast(float, A.lo_iu - an.au),
                                              __builtin_bit_cast(float, A.hi_iu - an.au));
            *(float4*)(row + 12) =
                make_float4(__builtin_bit_cast(float, A.lo_iv - an.av),
                            __builtin_bit_cast(float, A.hi_iv - an.av), an.sw2,
                            __builtin_bit_cast(float, inside ? 1 : 0));
        }
        __syncthreads();
        const int jn = min(64, A.count - j0);
        for (int jj = 0; jj < jn; ++jj, plane += plane_bytes) {
            if ((skip >> jj) & 1) continue;
            // the w row (the same for every box; in the ray frame, as stored)
            const const_float* m = mats + 12 * (j0 + jj);
            const float4 r0 = *(const float4*)an_rows[jj];
            const float4 r1 = *(const float4*)(an_rows[jj] + 4);
            const int4 r2 = *(const int4*)(an_rows[jj] + 8);
            const float4 r3 = *(const float4*)(an_rows[jj] + 12);
            const __amdgpu_buffer_rsrc_t rsrc = make_rsrc(plane, plane_bytes);
            // (the w row's z slope from LDS, a vector register: the slice
            // FMAs take their slice index as an inline literal)
            // (fdk512 FP32: 29.5 -> 28.75 ms per backprojection with the
            // clamp-free copy; 1024^3: 195.3 -> 196.4 ms)
            if (!WCHECK && __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, r3.w)) != 0)
                accumulate_view<TT, LAYOUT, WCHECK, VCLAMP, DIV, false>(
                    A, r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w,
                    __builtin_bit_cast(float, r2.x), m[8], m[9], r3.z, r2.z, r2.w,
                    __builtin_bit_cast(int, r3.x), __builtin_bit_cast(int, r3.y), r2.y, d_t, d_r,
                    rsrc, acc);
            else
                accumulate_view<TT, LAYOUT, WCHECK, VCLAMP, DIV>(
                    A, r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w,
                    __builtin_bit_cast(float, r2.x), m[8], m[9], r3.z, r2.z, r2.w,
                    __builtin_bit_cast(int, r3.x), __builtin_bit_cast(int, r3.y), r2.y, d_t, d_r,
                    rsrc, acc);
        }
        __syncthreads();  // every wave has read its rows before the next chunk's
    }

    // With the rays along x, lane (a, b) holds column (x0 + b, y0 + a):
    // transpose the wave's 8 x 8 patch through the lane crossbar so that
    // consecutive lanes read and write consecutive x in the volume (fdk512:
    // FP32 29.5 -> 29.2 ms per backprojection, FP16 25.3 -> 25.0 ms).
    // (either way lane L then holds column (x0 + L % 8, y0 + L / 8); the lane
    // index is recomputed here rather than kept across the view loop, where
    // it was spilled: with the corner tests' extents kept in scalar registers,
    // fdk512 FP32 28.1 -> 28.0 ms per backprojection, fdk1024 192.1 -> 191.5)
    const int el = (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
    if (!A.y_fastest) {
        const int src = ((el & 7) << 3) | (el >> 3);  // the lane holding (x0 + el % 8, y0 + el / 8)
#pragma unroll
        for (int i = 0; i < kFusedZ; ++i)
            acc[i] = __builtin_bit_cast(
                float, __builtin_amdgcn_ds_bpermute(src << 2, __builtin_bit_cast(int, acc[i])));
    }
    const int ex = wx0 + (el & 7), ey = wy0 + (el >> 3);
    if (ex < A.N && ey < A.N) {
        const size_t slice = (size_t)A.N * A.N;
        float* out = A.vol + (size_t)(A.z_first + zl0) * slice + (size_t)ey * A.N + ex;
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

template <typename TT, int LAYOUT, int DIV>
static void launch_fused_d(const FusedArgs& a, bool wcheck, bool rows_free, hipStream_t s)
{
    dim3 grid(a.tiles_x * a.tiles_y * a.zchunks);
    if (wcheck)
        hipLaunchKernelGGL((bp_fused_kernel<TT, LAYOUT, true, true, DIV>), grid, dim3(kThreads), 0,
                           s, a);
    else if constexpr (sizeof(typename TT::elem) == 2 && LAYOUT != kRows) {
        if (rows_free)
            hipLaunchKernelGGL((bp_fused_kernel<TT, LAYOUT, false, false, DIV>), grid,
                               dim3(kThreads), 0, s, a);
        else
            hipLaunchKernelGGL((bp_fused_kernel<TT, LAYOUT, false, true, DIV>), grid,
                               dim3(kThreads), 0, s, a);
    } else
        hipLaunchKernelGGL((bp_fused_kernel<TT, LAYOUT, false, true, DIV>), grid, dim3(kThreads),
                           0, s, a);
}

template <typename TT, int LAYOUT>
static void launch_fused_t(const FusedArgs& a, bool wcheck, bool rows_free, int divide,
                           hipStream_t s)
{
    // the divide variants exist for the default layout only (the host
    // rejects others)
    if constexpr (LAYOUT == kDPairs) {
        if (divide == kDivRcpNR) return launch_fused_d<TT, LAYOUT, kDivRcpNR>(a, wcheck, rows_free, s);
        if (divide == kDivIEEE) return launch_fused_d<TT, LAYOUT, kDivIEEE>(a, wcheck, rows_free, s);
        if (divide == kDivRcp12) return launch_fused_d<TT, LAYOUT, kDivRcp12>(a, wcheck, rows_free, s);
    }
    launch_fused_d<TT, LAYOUT, kDivRcp>(a, wcheck, rows_free, s);
}

template <typename TT>
static void launch_fused_l(const FusedArgs& a, int layout, bool wcheck, bool rows_free,
                           int divide, hipStream_t s)
{
    if (layout == kRows)
        launch_fused_t<TT, kRows>(a, wcheck, false, divide, s);
    else if (layout == kPairs)
        launch_fused_t<TT, kPairs>(a, wcheck, rows_free, divide, s);
    else if (layout == kDPairs)
        launch_fused_t<TT, kDPairs>(a, wcheck, rows_free, divide, s);
    else if (layout == kDQuads)
        launch_fused_t<TT, kDQuads>(a, wcheck, rows_free, divide, s);
    else
        launch_fused_t<TT, kQuads>(a, wcheck, rows_free, divide, s);
}

hipError_t launch_fused(const FusedArgs& a, int storage, int layout, bool wcheck, bool rows_free,
                        int divide, hipStream_t s)
{
    if (storage == kF32)
        launch_fused_l<TF32>(a, layout, wcheck, rows_free, divide, s);
    else if (storage == kF16)
        launch_fused_l<TF16>(a, layout, wcheck, rows_free, divide, s);
    else
        launch_fused_l<TBF16>(a, layout, wcheck, rows_free, divide, s);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// plain
// ---------------------------------------------------------------------------
// Pixel (column j, row k) of an unpadded H x W view, zero outside it (the
// zero extension of Section 3.3, here by a bounds test per tap).
__device__ __forceinline__ float zero_extended(const float* view, int W, int H, int j, int k)
{
    return ((unsigned)j < (unsigned)W && (unsigned)k < (unsigned)H) ? view[(size_t)k * W + j]
                                                                     : 0.0f;
}

__global__ __launch_bounds__(256) void bp_plain_kernel(const PlainArgs A)
{
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= A.N || y >= A.N) return;
    // world coordinates of the voxel centre (mm)
    const float X = A.ox + (float)x * A.vs;
    const float Y = A.oy + (float)y * A.vs;
    const float Z = A.oz + (float)z * A.vs;
    const int H = A.H, W = A.W;
    float sum = 0.0f;
    const float* view = A.proj;
    for (int j = 0; j < A.count; ++j, view += (size_t)H * W) {
        const float* m = A.m[j];
        // part 1: homogeneous detector coordinates and two IEEE divisions
        const float uw = m[0] * X + m[1] * Y + m[2] * Z + m[3];
        const float vw = m[4] * X + m[5] * Y + m[6] * Z + m[7];
        const float w = m[8] * X + m[9] * Y + m[10] * Z + m[11];
        if (!(w > 0.0f)) continue;
        const float u = uw / w;
        const float v = vw / w;
        // a sample left of column -1 or right of column W - 1 (likewise
        // rows) has all four taps outside the view: nothing to add
        if (!(u >= -1.0f && u < (float)W && v >= -1.0f && v < (float)H)) continue;
        // part 2: the four zero-extended neighbours of (u, v)
        const float fu = floorf(u), fv = floorf(v);
        const int c0 = (int)fu, r0 = (int)fv;
        const float p00 = zero_extended(view, W, H, c0, r0);
        const float p10 = zero_extended(view, W, H, c0 + 1, r0);
        const float p01 = zero_extended(view, W, H, c0, r0 + 1);
        const float p11 = zero_extended(view, W, H, c0 + 1, r0 + 1);
        // part 3: two horizontal lerps, one vertical, weight 1/w^2
        const float a = u - fu, b = v - fv;
        const float upper = fmaf(a, p10 - p00, p00);
        const float lower = fmaf(a, p11 - p01, p01);
        sum = fmaf(fmaf(b, lower - upper, upper), 1.0f / (w * w), sum);
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
    for (int i = threadIdx.x; i < 12 * a.count; i += 256) {
        a.dst[i] = a.m[i];
        a.dstq[i] = a.q[i];
    }
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
