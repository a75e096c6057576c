// Forward projection kernels for gfx950: the exact transpose of the fused
// backprojection (FP32 storage, default reciprocal), used as its adjoint
// (gradients through the backprojection) and as a matched projector.
//
// Every voxel value times r^2 = 1/w^2 is spread onto the four taps the
// backprojection reads for that (voxel, view) pair, with the same bilinear
// weights (1-au)(1-av), au(1-av), (1-au)av, au av: both kernels take the
// pair's coordinates from the same anchored geometry (anchor.h), with the
// same boxes and the same operations in the same order, so they agree bit
// for bit.  Taps outside the detector land in the 2-pixel border of padded
// planes and are dropped when the interior is added to the caller's stack.
//
// The planes hold 64-bit fixed-point sums: integer additions do not depend
// on their order, so the result is the same on every run.  One scale 2^kg
// per launch, from a bound on any plane sum: the bilinear weights of a
// voxel sum to 1, so a pixel receives at most B = sum |x| r^2 <= N^3 max|x|
// max r^2, and kg keeps B 2^kg below 2^60 (fp_global_exponent).  Each
// contribution is rounded to a multiple of 2^-kg (far below FP32's
// resolution of the sums).
#include "anchor.h"
#include "fdk_internal.h"
#include "gfx950_util.h"

namespace fdk {

static_assert(kFpZ == fused_z(kF32), "forward projection boxes are the FP32 backprojection's");

// kg for a launch: N^3 * vmax * rmax2 * 2^kg < 2^60 (a factor 2 of margin
// over the float rounding of the bound); 0 if there is nothing to project.
__device__ __forceinline__ int fp_global_exponent(int N, float vmax, float rmax2)
{
    const float bound = (float)N * (float)N * (float)N * vmax * rmax2;
    if (!(bound > 0.0f) || !(bound < 1.0e38f)) return 0;
    int e;
    frexpf(bound, &e);  // bound < 2^e
    return min(max(60 - e, -120), 120);
}

// x rounded to the nearest integer, ties towards +infinity (one instruction)
__device__ __forceinline__ int cvt_nearest(float x)
{
    int r;
    asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// A tap value already scaled by 2^kg (|x| < 2^60) as a 64-bit integer,
// rounded to nearest.
__device__ __forceinline__ unsigned long long to_fixed64(float x)
{
    return (unsigned long long)__float2ll_rn(x);
}

__device__ __forceinline__ void add64(unsigned long long* p, unsigned long long v)
{
    if (v) atomicAdd(p, v);
}

// The four taps of one voxel, scaled by 2^kg, added to a padded plane at
// element `off` (top-left tap) with row pitch Wp.
__device__ __forceinline__ void scatter_taps64(unsigned long long* plane, uint32_t off, int Wp,
                                               float s, float au, float av)
{
    const float b = s * av;  // bottom row weight
    const float a = s - b;   // top row weight
    const float tr = a * au, br = b * au;
    add64(plane + off, to_fixed64(a - tr));
    add64(plane + off + 1, to_fixed64(tr));
    add64(plane + off + Wp, to_fixed64(b - br));
    add64(plane + off + Wp + 1, to_fixed64(br));
}

// Largest |x| of the volume as the bits of a non-negative float (whose
// integer order is the float order), merged into *out (zeroed before).
// One atomic per block: the blocks' maxima all go to one address, where
// atomics take turns (one per wave and 4096 blocks: 0.19 ms for 256^3).
__global__ __launch_bounds__(256) void fp_vmax_kernel(const float* vol, size_t n, unsigned* out)
{
    __shared__ float wm[4];
    float m0 = 0.0f, m1 = 0.0f, m2 = 0.0f, m3 = 0.0f;
    const size_t stride = (size_t)gridDim.x * 256;
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    // four loads in flight per thread
    for (; i + 3 * stride < n; i += 4 * stride) {
        m0 = fmaxf(m0, fabsf(vol[i]));
        m1 = fmaxf(m1, fabsf(vol[i + stride]));
        m2 = fmaxf(m2, fabsf(vol[i + 2 * stride]));
        m3 = fmaxf(m3, fabsf(vol[i + 3 * stride]));
    }
    for (; i < n; i += stride) m0 = fmaxf(m0, fabsf(vol[i]));
    float m = fmaxf(fmaxf(m0, m1), fmaxf(m2, m3));
    for (int d = 32; d >= 1; d >>= 1) m = fmaxf(m, __shfl_xor(m, d));
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0)
        atomicMax(out, __float_as_uint(fmaxf(fmaxf(wm[0], wm[1]), fmaxf(wm[2], wm[3]))));
}

hipError_t launch_fp_vmax(const float* vol, size_t n, unsigned* out, hipStream_t s)
{
    size_t blocks = (n + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(fp_vmax_kernel, dim3((unsigned)blocks), dim3(256), 0, s, vol, n, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// scatter: the backprojection's workgroups, waves and boxes, 64-bit atomics
// ---------------------------------------------------------------------------
// One thread per column and kFpZ slices of a wave's 8 x 8 x kFpZ box, as the
// backprojection; each voxel's four taps go straight to the plane.  Used for
// batches where some voxel may have w <= 0 (no anchor, as the
// backprojection there; float planes, since 1/w^2 has no bound) and when the
// LDS kernel is switched off (64-bit planes).
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
    const int zc = rest % A.zchunks;
    const int t1 = rest / A.zchunks;
    const int tx = A.y_fastest ? t1 : t0;
    const int ty = A.y_fastest ? t0 : t1;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int wx0, wy0;
    wave_origin(A.y_fastest != 0, tx, ty, wave, wx0, wy0);
    const int x = wx0 + (lane % kWaveX);
    const int y = wy0 + (lane / kWaveX);
    const int zl0 = zc * kFpZ;
    BoxFrame bf = box_frame(A, wx0, wy0, A.z_first + zl0, kWaveX, kWaveY, kFpZ);
    const float dx = (float)(lane % kWaveX) - bf.hx;
    const float dy = (float)(lane / kWaveX) - bf.hy;
    const float d_t = A.y_fastest ? dx : dy;
    const float d_r = A.y_fastest ? dy : dx;

    // the thread's voxel values (0 outside the volume)
    float val[kFpZ];
    const bool inside = x < A.N && y < A.N;
    const size_t slice = (size_t)A.N * A.N;
    const float* src = A.vol + (size_t)(A.z_first + zl0) * slice + (size_t)y * A.N + x;
#pragma unroll
    for (int i = 0; i < kFpZ; ++i)
        val[i] = (inside && zl0 + i < A.nz) ? src[(size_t)i * slice] : 0.0f;

    const int kg = fp_global_exponent(A.N, __uint_as_float(*A.fp_vmax), A.fp_rmax2);
    const float Sg = __builtin_ldexpf(1.0f, kg);
    const int Wp = A.Wp;
    __shared__ float anchors[kWgWaves][64][16];
    float(*an_rows)[16] = anchors[wave];
    unsigned long long* plane = A.acc64;
    const const_float* mats = as_constant(A.m);
    for (int j0 = 0; j0 < A.count; j0 += 64) {
        uint64_t skip;
        {
            const Anchor an = make_anchor<!WCHECK>(A, j0 + lane, bf);
            skip = __ballot(an.skip);
            float* row = an_rows[lane];
            *(float4*)row = make_float4(an.uc, an.vc, an.wc, an.su_t);
            *(float4*)(row + 4) = make_float4(an.su_r, an.su2, an.sv_t, an.sv_r);
            *(float4*)(row + 8) =
                make_float4(an.sv2, __builtin_bit_cast(float, an.av * Wp + an.au + A.origin_off),
                            __builtin_bit_cast(float, A.lo_iu - an.au),
                            __builtin_bit_cast(float, A.hi_iu - an.au));
            *(float4*)(row + 12) =
                make_float4(__builtin_bit_cast(float, A.lo_iv - an.av),
                            __builtin_bit_cast(float, A.hi_iv - an.av), an.sw2, 0.0f);
        }
        __syncthreads();
        const int jn = min(64, A.count - j0);
        for (int jj = 0; jj < jn; ++jj, plane += A.plane) {
            if ((skip >> jj) & 1) continue;
            const const_float* m = mats + 12 * (j0 + jj);
            const float4 r0 = *(const float4*)an_rows[jj];
            const float4 r1 = *(const float4*)(an_rows[jj] + 4);
            const int4 r2 = *(const int4*)(an_rows[jj] + 8);
            const float4 r3f = *(const float4*)(an_rows[jj] + 12);
            const int2 r3 = make_int2(__builtin_bit_cast(int, r3f.x), __builtin_bit_cast(int, r3f.y));
            float bu, bv, bw;
            column_base(r0.x, r0.y, r0.z, r0.w, r1.x, r1.z, r1.w, m[8], m[9], d_t, d_r, bu, bv,
                        bw);
            const float su2 = r1.y, sv2 = __builtin_bit_cast(float, r2.x), sw2 = r3f.z;
#pragma unroll
            for (int i = 0; i < kFpZ; ++i) {
                float u, v, r;
                voxel_coords<kDivRcp, WCHECK>(bu, bv, bw, su2, sv2, sw2, (float)i, u, v, r);
                const float au = __builtin_amdgcn_fractf(u);
                const float av = __builtin_amdgcn_fractf(v);
                const int ju = med3_i32(cvt_floor(u), r2.z, r2.w);
                const int jv = med3_i32(cvt_floor(v), r3.x, r3.y);
                const uint32_t off = (uint32_t)(mad_i24_ub(jv, Wp, ju) + r2.y);
                if constexpr (WCHECK) {
                    // w may come arbitrarily close to 0 (no fixed-point bound):
                    // float sums, whose last bits depend on the atomics' order
                    float* fp = (float*)plane;
                    const float s = val[i] * (r * r);
                    const float b = s * av, a = s - b, tr = a * au, br = b * au;
                    atomicAdd(fp + off, a - tr);
                    atomicAdd(fp + off + 1, tr);
                    atomicAdd(fp + off + Wp, b - br);
                    atomicAdd(fp + off + Wp + 1, br);
                } else {
                    scatter_taps64(plane, off, Wp, val[i] * (r * r) * Sg, au, av);
                }
            }
        }
        __syncthreads();
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

// ---------------------------------------------------------------------------
// LDS tiles
// ---------------------------------------------------------------------------
// A workgroup owns a box of 16 voxels across the rays, 32 along them and 16
// in z: 2 x 4 of the backprojection's 8 x 8 x 16 boxes.  Per view the
// boxes' projected intervals bound the
// workgroup's footprint on the detector; the workgroup accumulates its
// scatter into an LDS tile covering that footprint (plus a 1-pixel margin)
// and then adds the tile's non-zero pixels to the padded plane with one
// 64-bit atomic each: about one global atomic per footprint pixel instead of
// four per voxel.  A footprint larger than the tile takes the 64-bit
// atomics per tap for that view.
//
// The tile accumulates in 32-bit fixed point with integer LDS atomics
// (float LDS atomics measured ~40x slower than integer ones on this GPU).
// Per view the tile's scale is a power of two St with 8192 * max|x| * max r^2
// * St below 2^31, where max|x| is the largest voxel value of the workgroup's
// box and max r^2 = 1 / (min w)^2 over it: a pixel receives at most one tap
// of each of the box's 8192 voxels and each tap is at most |x| r^2, so no
// tile sum can overflow.  Each tap is rounded to the nearest multiple of
// 1/St; a tile sum is then exact, and its conversion to the plane's scale
// (a shift) is exact or rounds once.
constexpr int kFpTile = 16;                // voxels across the rays and in z
constexpr int kFpRayBoxes = 4;             // backprojection boxes along the ray
constexpr int kFpRay = 8 * kFpRayBoxes;    // voxels per thread along the ray
constexpr int kFpBoxes = 2 * kFpRayBoxes;  // backprojection boxes per workgroup
constexpr int kFpChunk = 64 / kFpBoxes;    // views whose anchors are computed together

// waves per SIMD the registers are fitted to (up to 128 VGPRs)
#ifndef FDK_FP_WAVES
#define FDK_FP_WAVES 4
#endif

// A tile sum t in units of 2^-kt, in units of 2^-kg (rounded to nearest,
// ties up, where kg < kt).
__device__ __forceinline__ unsigned long long rescale_fixed(int t, int kt, int kg)
{
    const int sh = kg - kt;
    const long long v = t;
    if (sh >= 0) return (unsigned long long)(v << sh);
    if (sh < -32) return 0ull;  // |t| < 2^31: below half a unit
    return (unsigned long long)((v + (1ll << (-sh - 1))) >> (-sh));
}

template <bool ALONG_Y>
__global__ __launch_bounds__(256, FDK_FP_WAVES) void fp_lds_kernel(const FusedArgs A)
{
    extern __shared__ int tile[];  // A.fp_tile entries
    // anchors (16 words) and projected bounds (8 words) of the 8 boxes for a
    // chunk of views, and the waves' largest |x|
    __shared__ float rows[kFpBoxes][kFpChunk][16];
    __shared__ float bnds[kFpBoxes][kFpChunk][8];
    __shared__ float wave_max[4];
    // The backprojection's workgroup order (ray axis, then z, then across),
    // dealt to the XCDs one ray line of G boxes at a time: the launch's
    // workgroups go to the 8 XCDs in turn, and XCD x takes lines x, x + 8,
    // x + 16, ...  Boxes along a ray project onto the same pixels, so a line
    // keeps its plane traffic in one L2, while lines spread over the whole
    // volume even out the XCDs' work: only the boxes that hold some of the
    // volume's mass work, and contiguous slabs per XCD (the backprojection's
    // mapping) gave them 0 to 240 of fdk256x8's 949 working boxes.
    // (fdk256x8: 2.75 against 3.07 ms of kernel time per projection.)
    int bid = blockIdx.x;
    const int G = A.y_fastest ? A.tiles_y : A.tiles_x;
    if (A.xcd_remap && gridDim.x % (8 * G) == 0) {  // (whole groups of 8 lines)
        const int k = bid >> 3, xcd = bid & 7;
        bid = ((k / G) * 8 + xcd) * G + k % G;
    }
    const int t0 = bid % (A.y_fastest ? A.tiles_y : A.tiles_x);
    const int rest = bid / (A.y_fastest ? A.tiles_y : A.tiles_x);
    const int zc = rest % A.zchunks;
    const int t1 = rest / A.zchunks;
    const int tx = A.y_fastest ? t1 : t0;
    const int ty = A.y_fastest ? t0 : t1;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int bx0 = tx * (ALONG_Y ? kFpTile : kFpRay), by0 = ty * (ALONG_Y ? kFpRay : kFpTile);
    const int zl0 = zc * kFpZ, zs0 = A.z_first + zl0;
    // A thread owns the 32 voxels of the box along the axis closest to the
    // batch's rays (y if ALONG_Y, else x); the lanes of a wave span the
    // other horizontal axis (16) and 4 slices.  Voxels along a ray project
    // onto the same pixels: this way they fall to one thread, one after the
    // other, and the 64 lanes of an atomic instruction hit 64 distinct
    // places (transverse neighbours ~2 px apart, z neighbours ~2 rows).
    // The same reason makes the box long along the rays: a 16 x 32 x 16 box
    // covers ~1.5 times the pixels of a 16 x 16 x 16 one, so a flushed
    // pixel carries more voxels' taps (fdk256x8: 7.15 against 10.0 ms per
    // projection of a dense volume, 2.23 against 2.77 ms of the phantom).
    const int tt = threadIdx.x & 15, zz = threadIdx.x >> 4;
    const int x = ALONG_Y ? bx0 + tt : bx0;  // first voxel of the thread's line
    const int y = ALONG_Y ? by0 : by0 + tt;
    const int z = zs0 + zz;

    float val[kFpRay];
    const size_t slice = (size_t)A.N * A.N;
    const bool zin = zl0 + zz < A.nz;
    // every lane reads an existing voxel (indices clamped into the volume)
    // and keeps it only if it is its own: no test per load, so that the
    // loads are in flight together
    const float* src = A.vol + (size_t)min(z, A.z_first + A.nz - 1) * slice;
    float vmax = 0.0f;
#pragma unroll
    for (int i = 0; i < kFpRay; ++i) {
        const int xi = ALONG_Y ? x : x + i, yi = ALONG_Y ? y + i : y;
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
    for (int e = threadIdx.x; e < A.fp_tile; e += 256) tile[e] = 0;

    // the thread's boxes along its line (box b = bt + 2 br: bt across the
    // rays, br along them) and its offsets
    const int tb = tt >> 3;
    float d_t[kFpRayBoxes], h_r[kFpRayBoxes];
#pragma unroll
    for (int h = 0; h < kFpRayBoxes; ++h) {
        const int ox = ALONG_Y ? 8 * tb : 8 * h, oy = ALONG_Y ? 8 * h : 8 * tb;
        const BoxFrame f = box_frame(A, bx0 + ox, by0 + oy, zs0, kWaveX, kWaveY, kFpZ);
        d_t[h] = (float)(tt & 7) - (ALONG_Y ? f.hx : f.hy);
        h_r[h] = ALONG_Y ? f.hy : f.hx;
    }

    const int kg = fp_global_exponent(A.N, __uint_as_float(*A.fp_vmax), A.fp_rmax2);
    const float Sg = __builtin_ldexpf(1.0f, kg);
    const int Wp = A.Wp;
    const const_float* mats = as_constant(A.m);
    // this workgroup's views: part blockIdx.y of the batch, whole chunks
    const int per = ((A.count + A.fp_vparts - 1) / A.fp_vparts + kFpChunk - 1) / kFpChunk * kFpChunk;
    const int jbeg = blockIdx.y * per, jend = min(A.count, jbeg + per);
    unsigned long long* plane = A.acc64 + (size_t)jbeg * A.plane;
    for (int j0 = jbeg; j0 < jend; j0 += kFpChunk, plane += kFpChunk * A.plane) {
        if (threadIdx.x < kFpBoxes * kFpChunk) {
            // thread (b, view): the anchor of box b for view j0 + view
            const int b = threadIdx.x / kFpChunk, jv = threadIdx.x % kFpChunk;
            const int ox = ALONG_Y ? 8 * (b & 1) : 8 * (b >> 1);
            const int oy = ALONG_Y ? 8 * (b >> 1) : 8 * (b & 1);
            const BoxFrame f = box_frame(A, bx0 + ox, by0 + oy, zs0, kWaveX, kWaveY, kFpZ);
            const Anchor an = make_anchor<true>(A, j0 + jv, f);
            float* row = rows[b][jv];
            *(float4*)row = make_float4(an.uc, an.vc, an.wc, an.su_t);
            *(float4*)(row + 4) = make_float4(an.su_r, an.su2, an.sv_t, an.sv_r);
            *(float4*)(row + 8) = make_float4(an.sv2, __builtin_bit_cast(float, an.au),
                                              __builtin_bit_cast(float, an.av), an.sw2);
            // a skipped box takes no part in the footprint
            const bool part = !an.skip;
            *(float4*)bnds[b][jv] = make_float4(part ? an.umin : INFINITY,
                                                part ? an.umax : -INFINITY,
                                                part ? an.vmin : INFINITY,
                                                part ? an.vmax : -INFINITY);
            *(float4*)(bnds[b][jv] + 4) = make_float4(part ? an.wmin : INFINITY,
                                                      part ? 1.0f : 0.0f, 0.0f, 0.0f);
        }
        __syncthreads();
        const int jn = min(kFpChunk, jend - j0);
        for (int jj = 0; jj < jn; ++jj) {
            unsigned long long* pl = plane + (size_t)jj * A.plane;
            // footprint of the boxes that reach the detector
            float umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmx = -INFINITY;
            float wmin = INFINITY, parts = 0.0f;
#pragma unroll
            for (int b = 0; b < kFpBoxes; ++b) {
                const float4 q0 = *(const float4*)bnds[b][jj];
                const float4 q1 = *(const float4*)(bnds[b][jj] + 4);
                umin = fminf(umin, q0.x);
                umax = fmaxf(umax, q0.y);
                vmin = fminf(vmin, q0.z);
                vmx = fmaxf(vmx, q0.w);
                wmin = fminf(wmin, q1.x);
                parts += q1.y;
            }
            if (uniform_f(parts) == 0.0f) continue;  // every box misses the detector
            // the tile's extent (tap indices, clamped to the padded plane)
            // and scale; bounds that are not finite take the 64-bit path
            const bool finite = uniform_f(umax - umin) < 65536.0f &&
                                uniform_f(vmx - vmin) < 65536.0f && uniform_f(wmin) > 0.0f;
            const int U0 = finite ? max((int)floorf(uniform_f(umin)) - 1, A.lo_iu) : 0;
            const int U1 = finite ? min((int)floorf(uniform_f(umax)) + 2, A.hi_iu + 1) : 0;
            const int V0 = finite ? max((int)floorf(uniform_f(vmin)) - 1, A.lo_iv) : 0;
            const int V1 = finite ? min((int)floorf(uniform_f(vmx)) + 2, A.hi_iv + 1) : 0;
            const int TW = U1 - U0 + 1, TH = V1 - V0 + 1;
            const float rmax = 1.0f / uniform_f(wmin);
            const float bound = (float)(256 * kFpRay) * vmax * rmax * rmax;
            const bool use_lds = finite && TW * TH <= A.fp_tile && bound >= 1e-20f &&
                                 bound <= 1e30f;
            const int kt =
                min(max((int)floorf(__builtin_log2f(2147483648.0f / bound)) - 1, -100), 100);
            const float St = __builtin_ldexpf(1.0f, kt);
            const const_float* m = mats + 12 * (j0 + jj);
#pragma unroll
            for (int h = 0; h < kFpRayBoxes; ++h) {
                // a box whose every tap is off the detector scatters nothing
                // (the backprojection skips it: its taps read zeros)
                const int bh = tb + 2 * h;
                if (bnds[bh][jj][5] == 0.0f) continue;
                const float* row = rows[bh][jj];
                const float4 r0 = *(const float4*)row;
                const float4 r1 = *(const float4*)(row + 4);
                const float4 r2 = *(const float4*)(row + 8);
                const int au = __builtin_bit_cast(int, r2.y), av = __builtin_bit_cast(int, r2.z);
                const float su2 = r1.y, sv2 = r2.x, sw2 = r2.w;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    // (u' - a_u, v' - a_v, r) of voxel 8h + k of the line, as
                    // the backprojection computes them
                    float bu, bv, bw, u, v, r;
                    column_base(r0.x, r0.y, r0.z, r0.w, r1.x, r1.z, r1.w, m[8], m[9], d_t[h],
                                (float)k - h_r[h], bu, bv, bw);
                    voxel_coords<kDivRcp, false>(bu, bv, bw, su2, sv2, sw2, (float)zz, u, v, r);
                    const float fu = __builtin_amdgcn_fractf(u);
                    const float fv = __builtin_amdgcn_fractf(v);
                    const float s = val[8 * h + k] * (r * r);
                    if (use_lds) {
                        // tap (iu, iv) at tile index (iv - V0) TW + (iu - U0).
                        // Clamping iu to [U0, U1 - 1] and iv to [V0, V1 - 1]
                        // keeps all four taps inside the tile; it changes no
                        // tap: the boxes project inside [umin, umax] x [vmin,
                        // vmax], one pixel inside the tile, except where U0 =
                        // lo_iu or U1 = hi_iu + 1 (likewise v), and there it is
                        // the clamp to the padded plane's border that the
                        // backprojection applies.
                        const int ju = med3_i32(cvt_floor(u), U0 - au, U1 - 1 - au);
                        const int jv = med3_i32(cvt_floor(v), V0 - av, V1 - 1 - av);
                        int* t0p = tile + (mad_i24_ub(jv, TW, ju) + (av - V0) * TW + (au - U0));
                        int* t1p = t0p + TW;
                        // in units of 1/St (exact: St is a power of two),
                        // rounded to the nearest integer, ties up
                        const float sS = s * St;
                        const float b = sS * fv;
                        const float a = sS - b;
                        const float tr = a * fu, br = b * fu;
                        atomicAdd(t0p, cvt_nearest(a - tr));
                        atomicAdd(t0p + 1, cvt_nearest(tr));
                        atomicAdd(t1p, cvt_nearest(b - br));
                        atomicAdd(t1p + 1, cvt_nearest(br));
                    } else {
                        const int ju = med3_i32(cvt_floor(u), A.lo_iu - au, A.hi_iu - au);
                        const int jv = med3_i32(cvt_floor(v), A.lo_iv - av, A.hi_iv - av);
                        const uint32_t off =
                            (uint32_t)(mad_i24_ub(jv, Wp, ju) + av * Wp + au + A.origin_off);
                        scatter_taps64(pl, off, Wp, s * Sg, fu, fv);
                    }
                }
            }
            if (use_lds) {
                __syncthreads();
                // each entry read and cleared: the tile is all zero again
                // for the next view (it is zeroed once, before the first)
                for (int rr = wave; rr < TH; rr += 4) {
                    unsigned long long* prow = pl + (V0 + rr) * Wp + U0 + A.origin_off;
                    for (int cc = lane; cc < TW; cc += 64) {
                        const int t = tile[rr * TW + cc];
                        tile[rr * TW + cc] = 0;
                        if (t != 0) atomicAdd(prow + cc, rescale_fixed(t, kt, kg));
                    }
                }
                __syncthreads();
            }
        }
        __syncthreads();  // every thread has read the chunk's rows
    }
}

hipError_t launch_scatter_lds(const FusedArgs& a, hipStream_t s)
{
    dim3 grid(a.tiles_x * a.tiles_y * a.zchunks, a.fp_vparts);
    const size_t lds = (size_t)a.fp_tile * sizeof(int);
    if (a.y_fastest)
        hipLaunchKernelGGL(fp_lds_kernel<true>, grid, dim3(256), lds, s, a);
    else
        hipLaunchKernelGGL(fp_lds_kernel<false>, grid, dim3(256), lds, s, a);
    return hipGetLastError();
}

// The interior of the planes (64-bit fixed point in units of 2^-kg, or
// float) added to the caller's FP32 views.
__global__ __launch_bounds__(256) void unstage_add_kernel(UnstageArgs a)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    const int k = blockIdx.y;
    const int view = blockIdx.z;
    if (j >= a.W) return;
    // a plane holds Hp*Wp 64-bit sums, or Hp*Wp floats at its start
    const unsigned long long* pl = a.planes + (size_t)view * a.Hp * a.Wp;
    const size_t e = (size_t)(k + kPad) * a.Wp + j + kPad;
    float v;
    if (a.fixed) {
        const int kg = fp_global_exponent(a.N, __uint_as_float(*a.vmax), a.rmax2);
        v = __builtin_ldexpf((float)(long long)pl[e], -kg);
    } else {
        v = ((const float*)pl)[e];
    }
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
