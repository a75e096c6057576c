// Forward projection kernels for gfx950: the exact transpose of the fused
// backprojection, used as its adjoint (gradients through the backprojection)
// and as a matched projector.
#include "fdk_internal.h"
#include "gfx950_util.h"

namespace fdk {

// ---------------------------------------------------------------------------
// forward projection: the exact transpose of the backprojection
// ---------------------------------------------------------------------------
// Every voxel value times r^2 = 1/w^2 is spread onto the four taps the
// backprojection reads, with the same bilinear weights (1-au)(1-av), au(1-av),
// (1-au)av, au av.  The targets are padded FP32 planes (rows layout): taps
// outside the detector land in the 2-pixel border and are dropped when the
// interior is added to the caller's stack.  Float atomics make the order of
// the sums, and so their last bits, vary between runs.
template <bool WCHECK>
__global__ __launch_bounds__(kThreads) void fp_scatter_kernel(const FusedArgs A)
{
    int bid = blockIdx.x;
    if (A.xcd_remap) {
        const int per = gridDim.x >> 3;
        bid = (bid & 7) * per + (bid >> 3);
    }
    const int t0 = bid % (A.y_fastest ? A.tiles_y : A.tiles_x);
    const int rest = bid / (A.y_fastest ? A.tiles_y : A.tiles_x);
    const int t1 = rest % (A.y_fastest ? A.tiles_x : A.tiles_y);
    const int zc = rest / (A.y_fastest ? A.tiles_x : A.tiles_y);
    const int tx = A.y_fastest ? t1 : t0;
    const int ty = A.y_fastest ? t0 : t1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wx0 = tx * kTileX;
    const int wy0 = ty * kTileY + wave * kWaveY;
    const int x = wx0 + (lane % kWaveX);
    const int y = wy0 + (lane / kWaveX);
    const int zl0 = zc * kFpZ;
    const float xp = (float)x - A.c;
    const float yp = (float)y - A.c;
    const float zp0 = (float)(A.z_first + zl0) - A.c;
    const float cxp = (float)(wx0 + ((lane & 1) ? kWaveX - 1 : 0)) - A.c;
    const float cyp = (float)(wy0 + ((lane & 2) ? kWaveY - 1 : 0)) - A.c;
    const float czp = zp0 + ((lane & 4) ? (float)(kFpZ - 1) : 0.0f);
    // transverse and ray coordinates (the matrices are in the ray frame)
    const float ctp = A.y_fastest ? cxp : cyp, crp = A.y_fastest ? cyp : cxp;
    const float pt = A.y_fastest ? xp : yp, pr = A.y_fastest ? yp : xp;
    const bool corner_lane = lane < 8;

    // the thread's voxel values (0 outside the volume)
    float val[kFpZ];
    const bool inside = x < A.N && y < A.N;
    const size_t slice = (size_t)A.N * A.N;
    const float* src = A.vol + (size_t)(A.z_first + zl0) * slice + (size_t)y * A.N + x;
#pragma unroll
    for (int i = 0; i < kFpZ; ++i)
        val[i] = (inside && zl0 + i < A.nz) ? src[(size_t)i * slice] : 0.0f;

    const int Wp = A.Wp;
    const uint32_t row_bytes = (uint32_t)Wp * 4u;
    const uint32_t plane_bytes = (uint32_t)(A.plane * 4ll);
    const uint32_t centre_bytes = (uint32_t)A.origin_off * 4u;
    const char* plane = (const char*)A.img;
    const const_float* mats = as_constant(A.m);
    for (int j = 0; j < A.count; ++j, plane += plane_bytes) {
        const const_float* m = mats + 12 * j;
        const __amdgpu_buffer_rsrc_t rsrc = make_rsrc(plane, plane_bytes);
        if constexpr (!WCHECK) {
            const float cu = fmaf(czp, m[2], fmaf(m[1], crp, fmaf(m[0], ctp, m[3])));
            const float cv = fmaf(czp, m[6], fmaf(m[5], crp, fmaf(m[4], ctp, m[7])));
            const float cw = fmaf(czp, m[10], fmaf(m[9], crp, fmaf(m[8], ctp, m[11])));
            const float cr = __builtin_amdgcn_rcpf(cw);
            const float u = cu * cr, v = cv * cr;
            if (__all(!corner_lane || u < A.skip_lo_u) || __all(!corner_lane || u > A.skip_hi_u) ||
                __all(!corner_lane || v < A.skip_lo_v) || __all(!corner_lane || v > A.skip_hi_v))
                continue;
        }
        // the column base in the backprojection's order: the transverse
        // term first, then the ray term
        const float bu = fmaf(m[1], pr, fmaf(m[0], pt, m[3]));
        const float bv = fmaf(m[5], pr, fmaf(m[4], pt, m[7]));
        const float bw = fmaf(m[9], pr, fmaf(m[8], pt, m[11]));
#pragma unroll
        for (int i = 0; i < kFpZ; ++i) {
            const float zp = zp0 + (float)i;
            const float uw = fmaf(zp, m[2], bu);
            const float vw = fmaf(zp, m[6], bv);
            const float w = fmaf(zp, m[10], bw);
            float r = __builtin_amdgcn_rcpf(w);
            if (WCHECK) r = (w > 0.0f) ? r : 0.0f;
            const float u = uw * r;
            const float v = vw * r;
            const float au = __builtin_amdgcn_fractf(u);
            const float av = __builtin_amdgcn_fractf(v);
            const int iu = cvt_floor(__builtin_amdgcn_fmed3f(u, A.lo_u, A.hi_u));
            const int iv = cvt_floor(__builtin_amdgcn_fmed3f(v, A.lo_v, A.hi_v));
            const uint32_t off = (uint32_t)mad_i24(iv, Wp, iu) * 4u + centre_bytes;
            const float s = val[i] * (r * r);
            const float b = s * av;       // bottom row weight
            const float a = s - b;        // top row weight
            const float tr = a * au, br = b * au;
            __builtin_amdgcn_raw_ptr_buffer_atomic_fadd_f32(a - tr, rsrc, off, 0, 0);
            __builtin_amdgcn_raw_ptr_buffer_atomic_fadd_f32(tr, rsrc, off + 4u, 0, 0);
            __builtin_amdgcn_raw_ptr_buffer_atomic_fadd_f32(b - br, rsrc, off, row_bytes, 0);
            __builtin_amdgcn_raw_ptr_buffer_atomic_fadd_f32(br, rsrc, off + 4u, row_bytes, 0);
        }
    }
}

hipError_t launch_scatter(const FusedArgs& a, bool wcheck, hipStream_t s)
{
    dim3 grid(a.tiles_x * a.tiles_y * a.zchunks);
    if (wcheck)
        hipLaunchKernelGGL((fp_scatter_kernel<true>), grid, dim3(kThreads), 0, s, a);
    else
        hipLaunchKernelGGL((fp_scatter_kernel<false>), grid, dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

// LDS variant of the forward projection.  A workgroup owns a 16 x 16 x 16
// voxel box.  Per view the 8 projected box corners bound the box's
// footprint on the detector (the projection of the box lies in the hull of
// the corners); the workgroup accumulates its scatter into an LDS tile
// covering that footprint (plus a 1-pixel margin against rounding) and then
// adds the tile's non-zero pixels to the padded plane with one global
// atomic each: about one global atomic per footprint pixel instead of four
// per voxel.  A footprint larger than the tile falls back to direct global
// atomics for that view.
//
// The tile accumulates in 32-bit fixed point with integer LDS atomics
// (float LDS atomics measured ~40x slower than integer ones on this GPU).
// Per view the scale is a power of two S with 4096 * max|x| * max r^2 * S
// below 2^31, where max|x| is the largest voxel value of the box and max r^2
// = 1 / min w^2 over the box corners: a pixel receives at most one tap of
// each of the box's 4096 voxels and each tap is at most |x| r^2, so no tile
// sum can overflow.  Each tap is rounded to the nearest multiple of 1/S
// (error <= 2^-32 * 4096 * max|x| * max r^2 per tap); the tile sums are then
// exact, independent of the order of the atomics.
constexpr int kFpTile = 16;

// x rounded to the nearest integer, ties towards +infinity (one instruction)
__device__ __forceinline__ int cvt_nearest(float x)
{
    int r;
    asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// waves per SIMD the registers are fitted to (up to 128 VGPRs).  Five 32 KiB
// tiles would fit the 160 KiB of LDS of a CU, but fitting the kernel to 5
// waves (96 VGPRs) spills: 256^3 x 248 views took 3.46 ms against 2.85 ms.
#ifndef FDK_FP_WAVES
#define FDK_FP_WAVES 4
#endif
template <bool ALONG_Y>
__global__ __launch_bounds__(256, FDK_FP_WAVES) void fp_lds_kernel(const FusedArgs A)
{
    // A.fp_tile tile entries at LDS address 0; the first 4 hold the wave
    // maxima of the box's values before the first view
    extern __shared__ int tile[];
    float* wave_max = (float*)tile;
    int bid = blockIdx.x;
    if (A.xcd_remap) {
        const int per = gridDim.x >> 3;
        bid = (bid & 7) * per + (bid >> 3);
    }
    // the backprojection's workgroup order: ray axis, then z, then across
    const int t0 = bid % (A.y_fastest ? A.tiles_y : A.tiles_x);
    const int rest = bid / (A.y_fastest ? A.tiles_y : A.tiles_x);
    const int zc = rest % A.zchunks;
    const int t1 = rest / A.zchunks;
    const int tx = A.y_fastest ? t1 : t0;
    const int ty = A.y_fastest ? t0 : t1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int bx0 = tx * kFpTile, by0 = ty * kFpTile;
    const int zl0 = zc * kFpZ;
    // A thread owns the 16 voxels of the box along the axis closest to the
    // batch's rays (y if y_fastest, else x); the lanes of a wave span the
    // other horizontal axis (16) and 4 z.  Voxels along a ray project onto
    // the same pixels: this way they fall to one thread, one after the
    // other, and the 64 lanes of an atomic instruction hit 64 distinct
    // places (transverse neighbours ~2 px apart, z neighbours ~2 rows).
    const int tt = threadIdx.x & 15, zz = threadIdx.x >> 4;
    constexpr bool along_y = ALONG_Y;  // == (A.y_fastest != 0)
    const int x = along_y ? bx0 + tt : bx0;  // first voxel of the thread's line
    const int y = along_y ? by0 : by0 + tt;
    const int z = A.z_first + zl0 + zz;
    const float xp = (float)x - A.c;
    const float yp = (float)y - A.c;
    const float zp = (float)z - A.c;
    // lanes 0..7 of every wave hold the corners of the workgroup's box
    const float cxp = (float)(bx0 + ((lane & 1) ? kFpTile - 1 : 0)) - A.c;
    const float cyp = (float)(by0 + ((lane & 2) ? kFpTile - 1 : 0)) - A.c;
    const float czp = (float)(A.z_first + zl0) - A.c + ((lane & 4) ? (float)(kFpZ - 1) : 0.0f);
    // transverse and ray coordinates (the matrices are in the ray frame)
    const float ctp = along_y ? cxp : cyp, crp = along_y ? cyp : cxp;
    const float pt = along_y ? xp : yp, pr0 = along_y ? yp : xp;
    const bool corner_lane = lane < 8;

    float val[kFpTile];
    const size_t slice = (size_t)A.N * A.N;
    const bool zin = zl0 + zz < A.nz;
    // every lane reads an existing voxel (indices clamped into the volume)
    // and keeps it only if it is its own: no test per load, so that the
    // loads are in flight together
    const float* src = A.vol + (size_t)min(z, A.z_first + A.nz - 1) * slice;
    float vmax = 0.0f;
#pragma unroll
    for (int i = 0; i < kFpTile; ++i) {
        const int xi = along_y ? x : x + i, yi = along_y ? y + i : y;
        const float v = src[(size_t)min(yi, A.N - 1) * A.N + min(xi, A.N - 1)];
        val[i] = (zin && xi < A.N && yi < A.N) ? v : 0.0f;
        vmax = fmaxf(vmax, fabsf(val[i]));
    }
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) vmax = fmaxf(vmax, __shfl_xor(vmax, d));
    if (lane == 0) wave_max[wave] = vmax;
    __syncthreads();
    vmax = fmaxf(fmaxf(wave_max[0], wave_max[1]), fmaxf(wave_max[2], wave_max[3]));
    if (vmax == 0.0f) return;  // nothing to project (uniform over the block)
    __syncthreads();           // every wave has read wave_max before the tile is zeroed

    const int Wp = A.Wp;
    const uint32_t row_bytes = (uint32_t)Wp * 4u;
    const uint32_t plane_bytes = (uint32_t)(A.plane * 4ll);
    const uint32_t centre_bytes = (uint32_t)A.origin_off * 4u;
    const int lo_u = (int)A.lo_u, hi_u = (int)(A.hi_u - 0.5f);
    const int lo_v = (int)A.lo_v, hi_v = (int)(A.hi_v - 0.5f);
    const char* plane = (const char*)A.img;
    const const_float* mats = as_constant(A.m);
    for (int j = 0; j < A.count; ++j, plane += plane_bytes) {
        const const_float* m = mats + 12 * j;
        const __amdgpu_buffer_rsrc_t rsrc = make_rsrc(plane, plane_bytes);
        const float cu = fmaf(czp, m[2], fmaf(m[1], crp, fmaf(m[0], ctp, m[3])));
        const float cv = fmaf(czp, m[6], fmaf(m[5], crp, fmaf(m[4], ctp, m[7])));
        const float cw = fmaf(czp, m[10], fmaf(m[9], crp, fmaf(m[8], ctp, m[11])));
        const float cr = __builtin_amdgcn_rcpf(cw);
        float umin = corner_lane ? cu * cr : INFINITY, umax = corner_lane ? cu * cr : -INFINITY;
        float vmin = corner_lane ? cv * cr : INFINITY, vmx = corner_lane ? cv * cr : -INFINITY;
        float wmin = corner_lane ? cw : INFINITY;
#pragma unroll
        for (int d = 1; d < 8; d <<= 1) {
            umin = fminf(umin, __shfl_xor(umin, d));
            umax = fmaxf(umax, __shfl_xor(umax, d));
            vmin = fminf(vmin, __shfl_xor(vmin, d));
            vmx = fmaxf(vmx, __shfl_xor(vmx, d));
            wmin = fminf(wmin, __shfl_xor(wmin, d));
        }
        umin = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(umin)));
        umax = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(umax)));
        vmin = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(vmin)));
        vmx = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(vmx)));
        wmin = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(wmin)));
        // every wave computed the same corners: the decisions below agree
        if (umax < A.skip_lo_u || umin > A.skip_hi_u || vmx < A.skip_lo_v || vmin > A.skip_hi_v)
            continue;
        const int U0 = max((int)floorf(umin) - 1, lo_u);
        const int U1 = min((int)floorf(umax) + 2, hi_u + 1);
        const int V0 = max((int)floorf(vmin) - 1, lo_v);
        const int V1 = min((int)floorf(vmx) + 2, hi_v + 1);
        const int TW = U1 - U0 + 1, TH = V1 - V0 + 1;
        // fixed-point scale: 4096 * vmax * rmax^2 * S < 2^31 (see above);
        // one binade of margin against the rounding of the bound.  Bounds
        // outside [1e-20, 1e30] (or not finite) take the float path.
        const float rmax = 1.0f / wmin;
        const float bound = 4096.0f * vmax * rmax * rmax;
        const bool use_lds = TW * TH <= A.fp_tile && bound >= 1e-20f && bound <= 1e30f;
        const int k = min(max((int)floorf(__builtin_log2f(2147483648.0f / bound)) - 1, -100), 100);
        const float S = __builtin_ldexpf(1.0f, k), invS = __builtin_ldexpf(1.0f, -k);
        if (use_lds) {
            for (int e = threadIdx.x; e < TW * TH; e += 256) tile[e] = 0;
            __syncthreads();
        }
        // (u'w, v'w, w) of voxel i of the line, rounded exactly as the fused
        // backprojection rounds them (the transverse axis's term, then the
        // ray axis's, then z), so that both operators see the same
        // coordinates for every pair; the transverse term is the line's
        // constant.  Then the fractions, the tap indices of the coordinates
        // clamped to [lo, hi], and the weighted value r^2 x.
        const float tu = fmaf(m[0], pt, m[3]);
        const float tv = fmaf(m[4], pt, m[7]);
        const float tw = fmaf(m[8], pt, m[11]);
        auto voxel = [&](int i, float lo_u, float hi_u, float lo_v, float hi_v, float& au,
                         float& av, int& iu, int& iv, float& s) {
            const float pr = pr0 + (float)i;
            const float uw = fmaf(zp, m[2], fmaf(m[1], pr, tu));
            const float vw = fmaf(zp, m[6], fmaf(m[5], pr, tv));
            const float w = fmaf(zp, m[10], fmaf(m[9], pr, tw));
            const float r = __builtin_amdgcn_rcpf(w);
            const float u = uw * r;
            const float v = vw * r;
            au = __builtin_amdgcn_fractf(u);
            av = __builtin_amdgcn_fractf(v);
            iu = cvt_floor(__builtin_amdgcn_fmed3f(u, lo_u, hi_u));
            iv = cvt_floor(__builtin_amdgcn_fmed3f(v, lo_v, hi_v));
            s = val[i] * (r * r);
        };
        if (use_lds) {
            // Tap (iu, iv) at tile index (iv - V0) TW + (iu - U0).  Clamping u
            // to [U0, U1 - 0.5] and v to [V0, V1 - 0.5] keeps all four taps
            // inside the tile; it changes no tap: the box projects inside
            // [umin, umax] x [vmin, vmax], one pixel inside the tile, except
            // where U0 = lo_u or U1 = hi_u + 1 (likewise v), and there it is
            // the clamp to the padded plane's border that every path applies.
            const int base = -(V0 * TW + U0);
            const float cu0 = (float)U0, cu1 = (float)U1 - 0.5f;
            const float cv0 = (float)V0, cv1 = (float)V1 - 0.5f;
#pragma unroll
            for (int i = 0; i < kFpTile; ++i) {
                float au, av, s;
                int iu, iv;
                voxel(i, cu0, cu1, cv0, cv1, au, av, iu, iv, s);
                // in units of 1/S (exact: S is a power of two), rounded to the
                // nearest integer, ties up (the same error bound as any
                // round-to-nearest)
                s *= S;
                const float b = s * av;
                const float a = s - b;
                const float tr = a * au, br = b * au;
                int* t0 = tile + (mad_i24(iv, TW, iu) + base);
                int* t1 = t0 + TW;
                atomicAdd(t0, cvt_nearest(a - tr));
                atomicAdd(t0 + 1, cvt_nearest(tr));
                atomicAdd(t1, cvt_nearest(b - br));
                atomicAdd(t1 + 1, cvt_nearest(br));
            }
        } else {
#pragma unroll
            for (int i = 0; i < kFpTile; ++i) {
                float au, av, s;
                int iu, iv;
                voxel(i, A.lo_u, A.hi_u, A.lo_v, A.hi_v, au, av, iu, iv, s);
                const float b = s * av;
                const float a = s - b;
                const float tr = a * au, br = b * au;
                const uint32_t off = (uint32_t)mad_i24(iv, Wp, iu) * 4u + centre_bytes;
                __builtin_amdgcn_raw_ptr_buffer_atomic_fadd_f32(a - tr, rsrc, off, 0, 0);
                __builtin_amdgcn_raw_ptr_buffer_atomic_fadd_f32(tr, rsrc, off + 4u, 0, 0);
                __builtin_amdgcn_raw_ptr_buffer_atomic_fadd_f32(b - br, rsrc, off, row_bytes, 0);
                __builtin_amdgcn_raw_ptr_buffer_atomic_fadd_f32(br, rsrc, off + 4u, row_bytes, 0);
            }
        }
        if (use_lds) {
            __syncthreads();
            for (int rr = wave; rr < TH; rr += 4) {
                const uint32_t row_off =
                    (uint32_t)mad_i24(V0 + rr, Wp, U0) * 4u + centre_bytes;
                for (int cc = lane; cc < TW; cc += 64) {
                    const float t = (float)tile[rr * TW + cc] * invS;
                    if (t != 0.0f)
                        __builtin_amdgcn_raw_ptr_buffer_atomic_fadd_f32(t, rsrc, row_off + 4u * cc,
                                                                        0, 0);
                }
            }
            __syncthreads();
        }
    }
}

hipError_t launch_scatter_lds(const FusedArgs& a, hipStream_t s)
{
    dim3 grid(a.tiles_x * a.tiles_y * a.zchunks);
    const size_t lds = (size_t)a.fp_tile * sizeof(int);
    if (a.y_fastest)
        hipLaunchKernelGGL(fp_lds_kernel<true>, grid, dim3(256), lds, s, a);
    else
        hipLaunchKernelGGL(fp_lds_kernel<false>, grid, dim3(256), lds, s, a);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void unstage_add_kernel(UnstageArgs a)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    const int k = blockIdx.y;
    const int view = blockIdx.z;
    if (j >= a.W) return;
    const float v = a.planes[((size_t)view * a.Hp + k + kPad) * a.Wp + j + kPad];
    a.dst[((size_t)view * a.H + k) * a.W + j] += v;
}

hipError_t launch_unstage_add(const UnstageArgs& a, hipStream_t s)
{
    dim3 grid((a.W + 255) / 256, a.H, a.count);
    hipLaunchKernelGGL(unstage_add_kernel, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void zero_kernel(float4* a, size_t n4)
{
    const size_t stride = (size_t)gridDim.x * 256;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += stride)
        a[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

// n must be a multiple of 4 and a 16-byte aligned
hipError_t launch_zero(float* a, size_t n, hipStream_t st)
{
    size_t blocks = (n / 4 + 255) / 256;
    if (blocks > 256 * 64) blocks = 256 * 64;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, st, (float4*)a, n / 4);
    return hipGetLastError();
}

}  // namespace fdk
