// FP64 FFT row convolution for gfx950: the Feldkamp pre-filter's ramp and
// the learned filter's long ramp convolution.
//
// A linear convolution of a W-sample row with taps h[n], -(W-1) <= n <= W-1,
// equals, on outputs 0 .. W-1, the circular convolution of length L >= 2W-1
// with the taps placed at n mod L.  One workgroup convolves two rows at once:
// it loads them as the real and imaginary parts of one complex row (zero
// padded to L) into LDS, transforms it, multiplies by the taps' spectrum and
// transforms back; since the taps are real, the real part of the result is
// the first row's convolution and the imaginary part the second's.
//
// The forward transform is an in-place decimation-in-frequency FFT (radix 4,
// plus one radix-2 stage when log2 L is odd; a radix-10 pass first at L =
// 2560) whose output is in digit-reversed order; the inverse is the mirrored
// decimation-in-time FFT, which takes that order and returns natural order.
// The taps' spectrum comes from the same forward transform, so it sits in
// the same order and the product is taken position by position: no
// reordering pass.  Twiddles come from a table of exp(-2 pi i k / kFftMax),
// k < kFftMax (and one of exp(-2 pi i k / 2560) at L = 2560).  All
// arithmetic is FP64 (the ramp removes each row's mean: its output is a
// small difference of large terms), rounded once to FP32 on output.
//
// Three kernels run the convolution: a general one for power-of-two L (its
// passes go through LDS, pairs of radix-4 stages at a time), and two that
// keep each pass in registers and fuse the loads, the spectrum product and
// the stores into the passes: L = 2560 (mixed radix 10 x 16 x 16) for rows
// of 513 to 1280 samples (the Feldkamp pre-filter's 1248, the learned
// filter's 624), L = 4096 for rows of 1281 to 2048.
#include "learn_internal.h"

namespace fdk {

// General lengths (and the taps' spectrum): 256 threads, one radix-16 group
// per thread and pass at L = 4096 (1024 threads with one radix-4 butterfly
// each measured the same, 13.4 ms for fdk512's pre-filter; with radix-16
// passes, 512 and 1024 threads leave threads idle: 17.7 and 30 ms).
constexpr int kFftThreads = 256;

// LDS position of element p: one pad element after every 8, so that the
// power-of-two strides of the butterflies spread over the banks.
__device__ __forceinline__ int px(int p) { return p + (p >> 3); }
constexpr int kFftLds = kFftMax + kFftMax / 8;  // double2 elements (72 KiB)

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return {fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x)};
}
// a * conj(b)
__device__ __forceinline__ double2 cmulc(double2 a, double2 b)
{
    return {fma(a.x, b.x, a.y * b.y), fma(a.y, b.x, -a.x * b.y)};
}

// One forward (DIF) stage on sub-transforms of length Ns (radix R = 2 or 4):
// the R inputs j, j + s, ... (s = Ns / R) of each block go through an R-point
// DFT and output q is multiplied by w_Ns^(q j).
template <int R>
__device__ __forceinline__ void dif_stage(double2* x, int L, int Ns, const double2* tw)
{
    const int s = Ns / R;
    const int ts = kFftMax / Ns;
    for (int b = threadIdx.x; b < L / R; b += kFftThreads) {
        const int j = b & (s - 1);
        const int base = (b - j) * R + j;
        if (R == 2) {
            const double2 a0 = x[px(base)], a1 = x[px(base + s)];
            x[px(base)] = cadd(a0, a1);
            x[px(base + s)] = cmul(csub(a0, a1), tw[j * ts]);
        } else {
            const double2 a0 = x[px(base)], a1 = x[px(base + s)], a2 = x[px(base + 2 * s)],
                          a3 = x[px(base + 3 * s)];
            const double2 t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3),
                          t3 = csub(a1, a3);
            // (-i) t3 = (t3.y, -t3.x)
            const double2 y1 = {t1.x + t3.y, t1.y - t3.x};
            const double2 y3 = {t1.x - t3.y, t1.y + t3.x};
            x[px(base)] = cadd(t0, t2);
            x[px(base + s)] = cmul(y1, tw[j * ts]);
            x[px(base + 2 * s)] = cmul(csub(t0, t2), tw[2 * j * ts]);
            x[px(base + 3 * s)] = cmul(y3, tw[3 * j * ts]);
        }
    }
}

// The inverse of dif_stage times R: conjugate twiddles first, then the
// conjugate R-point DFT.
template <int R>
__device__ __forceinline__ void dit_stage(double2* x, int L, int Ns, const double2* tw)
{
    const int s = Ns / R;
    const int ts = kFftMax / Ns;
    for (int b = threadIdx.x; b < L / R; b += kFftThreads) {
        const int j = b & (s - 1);
        const int base = (b - j) * R + j;
        if (R == 2) {
            const double2 a0 = x[px(base)], a1 = cmulc(x[px(base + s)], tw[j * ts]);
            x[px(base)] = cadd(a0, a1);
            x[px(base + s)] = csub(a0, a1);
        } else {
            const double2 a0 = x[px(base)];
            const double2 a1 = cmulc(x[px(base + s)], tw[j * ts]);
            const double2 a2 = cmulc(x[px(base + 2 * s)], tw[2 * j * ts]);
            const double2 a3 = cmulc(x[px(base + 3 * s)], tw[3 * j * ts]);
            const double2 t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3),
                          t3 = csub(a1, a3);
            // (+i) t3 = (-t3.y, t3.x)
            x[px(base)] = cadd(t0, t2);
            x[px(base + s)] = {t1.x - t3.y, t1.y + t3.x};
            x[px(base + 2 * s)] = csub(t0, t2);
            x[px(base + 3 * s)] = {t1.x + t3.y, t1.y - t3.x};
        }
    }
}

// Radix-4 butterflies on registers: forward (the DIF stage's) with output
// twiddles w1..w3, inverse (the DIT stage's) with conjugate input twiddles.
__device__ __forceinline__ void bfly4_fwd(double2& a0, double2& a1, double2& a2, double2& a3,
                                          double2 w1, double2 w2, double2 w3)
{
    const double2 t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = csub(a1, a3);
    a0 = cadd(t0, t2);
    a1 = cmul({t1.x + t3.y, t1.y - t3.x}, w1);  // t1 + (-i) t3
    a2 = cmul(csub(t0, t2), w2);
    a3 = cmul({t1.x - t3.y, t1.y + t3.x}, w3);  // t1 - (-i) t3
}
__device__ __forceinline__ void bfly4_inv(double2& a0, double2& a1, double2& a2, double2& a3,
                                          double2 w1, double2 w2, double2 w3)
{
    const double2 b1 = cmulc(a1, w1), b2 = cmulc(a2, w2), b3 = cmulc(a3, w3);
    const double2 t0 = cadd(a0, b2), t1 = csub(a0, b2), t2 = cadd(b1, b3), t3 = csub(b1, b3);
    a0 = cadd(t0, t2);
    a1 = {t1.x - t3.y, t1.y + t3.x};  // t1 + i t3
    a2 = csub(t0, t2);
    a3 = {t1.x + t3.y, t1.y - t3.x};  // t1 - i t3
}

// Two consecutive radix-4 stages (sub-lengths Ns and Ns / 4) in one pass:
// the 16 elements base + a s + b s/4 (s = Ns / 4, a, b < 4) are closed under
// both, so a thread loads them once, applies both stages in registers and
// stores them once.  Forward: the Ns stage, then the Ns / 4 stage (DIF);
// inverse: the mirrored order (DIT).
template <bool FWD>
__device__ __forceinline__ void pass16(double2* x, int L, int Ns, const double2* tw)
{
    const int s = Ns >> 2, s4 = s >> 2;
    const int tsA = kFftMax / Ns, tsB = kFftMax / s;
    for (int g = threadIdx.x; g < L / 16; g += kFftThreads) {
        const int jj = g & (s4 - 1);
        const int base = (g - jj) * 16 + jj;
        double2 v[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) v[a][b] = x[px(base + a * s + b * s4)];
        const double2 wb1 = tw[jj * tsB], wb2 = tw[2 * jj * tsB], wb3 = tw[3 * jj * tsB];
        if (FWD) {
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int j = jj + b * s4;
                bfly4_fwd(v[0][b], v[1][b], v[2][b], v[3][b], tw[j * tsA], tw[2 * j * tsA],
                          tw[3 * j * tsA]);
            }
#pragma unroll
            for (int a = 0; a < 4; ++a) bfly4_fwd(v[a][0], v[a][1], v[a][2], v[a][3], wb1, wb2, wb3);
        } else {
#pragma unroll
            for (int a = 0; a < 4; ++a) bfly4_inv(v[a][0], v[a][1], v[a][2], v[a][3], wb1, wb2, wb3);
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int j = jj + b * s4;
                bfly4_inv(v[0][b], v[1][b], v[2][b], v[3][b], tw[j * tsA], tw[2 * j * tsA],
                          tw[3 * j * tsA]);
            }
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) x[px(base + a * s + b * s4)] = v[a][b];
    }
}

// Forward: a radix-2 stage on the whole row when log2 L is odd, then pairs
// of radix-4 stages as radix-16 passes, then a last radix-4 stage if one is
// left.  The inverse undoes them in the opposite order.
__device__ void fft_forward(double2* x, int L, int log2L, const double2* tw)
{
    int Ns = L;
    if (log2L & 1) {
        dif_stage<2>(x, L, Ns, tw);
        __syncthreads();
        Ns >>= 1;
    }
    for (; Ns >= 16; Ns >>= 4) {
        pass16<true>(x, L, Ns, tw);
        __syncthreads();
    }
    if (Ns == 4) {
        dif_stage<4>(x, L, 4, tw);
        __syncthreads();
    }
}

__device__ void fft_inverse(double2* x, int L, int log2L, const double2* tw)
{
    const int Ns0 = (log2L & 1) ? L >> 1 : L;  // length of the first radix-4 stage
    int r4 = 0;                                  // number of radix-4 stages
    for (int n = Ns0; n >= 4; n >>= 2) ++r4;
    if (r4 & 1) {  // the forward transform's last, unpaired radix-4 stage
        dit_stage<4>(x, L, 4, tw);
        __syncthreads();
    }
    for (int n = (r4 & 1) ? 64 : 16; n <= Ns0; n <<= 4) {
        pass16<false>(x, L, n, tw);
        __syncthreads();
    }
    if (log2L & 1) {
        dit_stage<2>(x, L, L, tw);
        __syncthreads();
    }
}

// exp(-2 pi i k / kFftMax) for k < kFftMax into tw and, if tw2560 is not
// null, exp(-2 pi i k / 2560) for k < 2560 into tw2560
__global__ __launch_bounds__(256) void fft_twiddle_kernel(double2* tw, double2* tw2560)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= kFftMax) return;
    double s, c;
    sincospi(2.0 * (double)k / (double)kFftMax, &s, &c);
    tw[k] = {c, -s};
    if (tw2560 && k < kL2560) {
        sincospi(2.0 * (double)k / (double)kL2560, &s, &c);
        tw2560[k] = {c, -s};
    }
}

__device__ __forceinline__ double ramlak_tap(int n, double tau)
{
    const double kPi = 3.14159265358979323846;
    if (n == 0) return 1.0 / (4.0 * tau * tau);
    if (n & 1) return -1.0 / (((double)n * kPi * tau) * ((double)n * kPi * tau));
    return 0.0;
}

// Tap h[n] of the call, -(W-1) <= n <= W-1: the Ram-Lak kernel (taps ==
// nullptr) or h[n] = taps[pad - n] (transpose: taps[K - 1 - (pad - n)]).
__device__ __forceinline__ double conv_tap(const FftConvArgs& a, int n)
{
    if (!a.taps) return ramlak_tap(n < 0 ? -n : n, a.tau);
    const int t = a.pad - n;
    return (t >= 0 && t < a.K) ? (double)a.taps[a.transpose ? a.K - 1 - t : t] : 0.0;
}

// Spectrum of the taps, in the forward transform's order, times scale / L
// (power-of-two L).
__global__ __launch_bounds__(kFftThreads) void fft_spectrum_kernel(FftConvArgs a)
{
    __shared__ double2 x[kFftLds];
    for (int p = threadIdx.x; p < a.L; p += kFftThreads) x[px(p)] = {0.0, 0.0};
    __syncthreads();
    for (int n = -(a.W - 1) + (int)threadIdx.x; n <= a.W - 1; n += kFftThreads)
        x[px(n < 0 ? n + a.L : n)] = {conv_tap(a, n), 0.0};
    __syncthreads();
    fft_forward(x, a.L, a.log2L, a.tw);
    const double f = a.scale / (double)a.L;
    // The Ram-Lak taps are even in n, so their spectrum is real: for the
    // fused kernel only the real parts are stored (the imaginary parts of
    // the computed transform are rounding noise), as doubles.
    const bool real = a.L == kFftMax && !a.taps;
    for (int p = threadIdx.x; p < a.L; p += kFftThreads) {
        // the fused L = kFftMax kernel reads element p = 16 t + k as thread
        // t's k-th register: store it at k * (L / 16) + t, lane-contiguous
        const int q = a.L == kFftMax ? (p & 15) * (kFftMax / 16) + (p >> 4) : p;
        if (real)
            ((double*)a.spectrum)[q] = x[px(p)].x * f;
        else
            a.spectrum[q] = {x[px(p)].x * f, x[px(p)].y * f};
    }
}

__device__ __forceinline__ double parker_weight(double beta, double gamma, double delta)
{
    const double kPi = 3.14159265358979323846;
    if (delta < 0.0) return 0.5;  // full circle: every ray seen twice
    if (beta < 0.0) return 0.0;
    if (beta < 2.0 * (delta - gamma)) {
        const double s = sin(0.25 * kPi * beta / (delta - gamma));
        return s * s;
    }
    if (beta < kPi - 2.0 * gamma) return 1.0;
    if (beta <= kPi + 2.0 * delta) {
        const double s = sin(0.25 * kPi * (kPi + 2.0 * delta - beta) / (delta + gamma));
        return s * s;
    }
    return 0.0;
}

// Feldkamp weight tables of a call: Parker's weight of (view, column) and
// the cosine weight of (detector row, column), in FP64.
__global__ __launch_bounds__(256) void fft_weights_kernel(FftConvArgs a)
{
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    const long long np = (long long)a.views * a.W;
    if (i < np) {
        const int view = (int)(i / a.W), j = (int)(i - (long long)view * a.W);
        const double aj = ((double)j - 0.5 * (a.W - 1)) * a.pixel;
        a.parker[i] = parker_weight(a.beta0 + a.dbeta * view, -atan(aj / a.sdd), a.delta);
    } else if (i < np + (long long)a.H * a.W) {
        const long long c = i - np;
        const int k = (int)(c / a.W), j = (int)(c - (long long)k * a.W);
        const double aj = ((double)j - 0.5 * (a.W - 1)) * a.pixel;
        const double b = ((double)k - 0.5 * (a.H - 1)) * a.pixel;
        a.cosw[c] = a.sdd / sqrt(a.sdd * a.sdd + aj * aj + b * b);
    }
}

// Input sample j of row r, in FP64; with the Feldkamp weights when
// a.weighted.
__device__ __forceinline__ double row_sample(const FftConvArgs& a, int r, int j)
{
    const double v = (double)a.in[(size_t)r * a.W + j];
    if (!a.weighted) return v;
    const int view = r / a.H;
    const int k = r - view * a.H;
    return v * a.cosw[(size_t)k * a.W + j] * a.parker[(size_t)view * a.W + j];
}

__device__ __forceinline__ void store_sample(const FftConvArgs& a, int r, int j, double y)
{
    float v = (float)y;
    float* o = a.out + (size_t)r * a.W + j;
    if (a.bias) v += a.bias[0];
    if (a.accumulate) v += *o;
    if (a.relu) v = fmaxf(v, 0.0f);
    if (a.mask) v = *o > 0.0f ? v : 0.0f;
    *o = v;
}

// Rows 2b and 2b + 1 (if any) of the call.
__global__ __launch_bounds__(kFftThreads) void fft_conv_kernel(FftConvArgs a)
{
    __shared__ double2 x[kFftLds];
    const int r0 = 2 * blockIdx.x, r1 = r0 + 1;
    const bool two = r1 < a.rows;
    for (int p = threadIdx.x; p < a.L; p += kFftThreads) {
        double re = 0.0, im = 0.0;
        if (p < a.W) {
            re = row_sample(a, r0, p);
            if (two) im = row_sample(a, r1, p);
        }
        x[px(p)] = {re, im};
    }
    __syncthreads();
    fft_forward(x, a.L, a.log2L, a.tw);
    for (int p = threadIdx.x; p < a.L; p += kFftThreads) x[px(p)] = cmul(x[px(p)], a.spectrum[p]);
    __syncthreads();
    fft_inverse(x, a.L, a.log2L, a.tw);
    for (int j = threadIdx.x; j < a.W; j += kFftThreads) {
        store_sample(a, r0, j, x[px(j)].x);
        if (two) store_sample(a, r1, j, x[px(j)].y);
    }
}

// ---------------------------------------------------------------------------
// L = 4096 = 16^3 with the rows' data in registers.
//
// The forward transform is three radix-16 passes, each one pass16 above (same
// positions and twiddles, so the same output order and the same spectrum).  A
// thread holds its 16 elements of a pass in registers; LDS only carries the
// exchanges between passes.  The first forward pass reads the two rows from
// global memory: only positions below W are non-zero, and W <= L / 2, so the
// inputs at a >= 2 are zero and the first radix-4 stage has two inputs.  The
// third forward pass, the product with the spectrum and the inverse's first
// pass (which works on the same 16 contiguous elements) run on the same
// registers, and the inverse's last pass writes the rows (positions below W
// only, again a < 2) to global memory: four LDS exchanges per transform pair.
//
// Thread t's elements, v[a][b] for a, b < 4:
//   pass 1 (Ns = 4096): t + 1024 a + 256 b
//   pass 2 (Ns = 256):  256 (t >> 4) + (t & 15) + 64 a + 16 b
//   pass 3 (Ns = 16):   16 t + 4 a + b
// Twiddle indices (into the kFftMax table): stage 1 of a pass q (J + 256 b),
// stage 2 4 q J, with J = t, 16 (t & 15) and 0.

constexpr int kF16Threads = kFftMax / 16;
// one pad element after every 16: pass 3's stride-16 lanes then fall into
// distinct banks, and passes 1 and 2 read 16-element runs that hold no pad
__device__ __forceinline__ int qx(int p) { return p + (p >> 4); }
constexpr int kF16Lds = kFftMax + kFftMax / 16;  // one double per position (34 KiB)

__device__ __forceinline__ void dft4_fwd(double2& a0, double2& a1, double2& a2, double2& a3)
{
    const double2 t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = csub(a1, a3);
    a0 = cadd(t0, t2);
    a1 = {t1.x + t3.y, t1.y - t3.x};
    a2 = csub(t0, t2);
    a3 = {t1.x - t3.y, t1.y + t3.x};
}
__device__ __forceinline__ void dft4_inv(double2& a0, double2& a1, double2& a2, double2& a3)
{
    const double2 t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = csub(a1, a3);
    a0 = cadd(t0, t2);
    a1 = {t1.x - t3.y, t1.y + t3.x};
    a2 = csub(t0, t2);
    a3 = {t1.x + t3.y, t1.y - t3.x};
}

// Twiddles of a pass with base exponent J, w = exp(-2 pi i / 4096): stage 1
// takes w^(q (J + 256 b)) = w^(q J) c^(q b) with c = w^256 (a 16th root of
// unity), stage 2 w^(4 q J).  Only w^J is read from the table per pass; the
// powers and the products with c^k (read once, at wave-uniform addresses)
// are formed in FP64, a few units in its last place from the table's values.
struct Roots16 {
    double2 c1, c2, c3, c4, c6, c9;  // c^k
};
__device__ __forceinline__ Roots16 roots16(const double2* __restrict__ tw)
{
    return {tw[256], tw[512], tw[768], tw[1024], tw[1536], tw[2304]};
}
__device__ __forceinline__ double2 root(const Roots16& c, int k)
{
    switch (k) {
    case 1: return c.c1;
    case 2: return c.c2;
    case 3: return c.c3;
    case 4: return c.c4;
    case 6: return c.c6;
    default: return c.c9;
    }
}

struct PassTw {
    double2 u1, u2, u3;  // w^J, w^2J, w^3J
};
__device__ __forceinline__ PassTw pass_tw(int J, const double2* __restrict__ tw)
{
    PassTw p;
    p.u1 = tw[J];
    p.u2 = cmul(p.u1, p.u1);
    p.u3 = cmul(p.u1, p.u2);
    return p;
}

// One forward radix-16 pass on registers (stage 1 over a, stage 2 over b).
// FIRST: v[2][*] and v[3][*] are zero; UNIT: J = 0, so stage 1's twiddles are
// c^(q b) and stage 2's are 1.
template <bool FIRST, bool UNIT>
__device__ __forceinline__ void r16_fwd(double2 (&v)[4][4], int J, const Roots16& c,
                                        const double2* __restrict__ tw)
{
    PassTw u;
    if (!UNIT) u = pass_tw(J, tw);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        double2 w1, w2, w3;
        if (UNIT) {
            if (b == 0) {
                dft4_fwd(v[0][b], v[1][b], v[2][b], v[3][b]);
                continue;
            }
            w1 = root(c, b);
            w2 = root(c, 2 * b);
            w3 = root(c, 3 * b);
        } else if (b == 0) {
            w1 = u.u1;
            w2 = u.u2;
            w3 = u.u3;
        } else {
            w1 = cmul(u.u1, root(c, b));
            w2 = cmul(u.u2, root(c, 2 * b));
            w3 = cmul(u.u3, root(c, 3 * b));
        }
        if (FIRST) {
            const double2 a0 = v[0][b], a1 = v[1][b];
            v[0][b] = cadd(a0, a1);
            v[1][b] = cmul({a0.x + a1.y, a0.y - a1.x}, w1);
            v[2][b] = cmul(csub(a0, a1), w2);
            v[3][b] = cmul({a0.x - a1.y, a0.y + a1.x}, w3);
        } else {
            bfly4_fwd(v[0][b], v[1][b], v[2][b], v[3][b], w1, w2, w3);
        }
    }
    if (UNIT) {
#pragma unroll
        for (int a = 0; a < 4; ++a) dft4_fwd(v[a][0], v[a][1], v[a][2], v[a][3]);
    } else {
        const double2 u4 = cmul(u.u2, u.u2), u8 = cmul(u4, u4), u12 = cmul(u4, u8);
#pragma unroll
        for (int a = 0; a < 4; ++a) bfly4_fwd(v[a][0], v[a][1], v[a][2], v[a][3], u4, u8, u12);
    }
}

// The inverse of r16_fwd (times 16).  LAST: only outputs a < 2 are needed.
template <bool LAST, bool UNIT>
__device__ __forceinline__ void r16_inv(double2 (&v)[4][4], int J, const Roots16& c,
                                        const double2* __restrict__ tw)
{
    PassTw u;
    if (UNIT) {
#pragma unroll
        for (int a = 0; a < 4; ++a) dft4_inv(v[a][0], v[a][1], v[a][2], v[a][3]);
    } else {
        u = pass_tw(J, tw);
        const double2 u4 = cmul(u.u2, u.u2), u8 = cmul(u4, u4), u12 = cmul(u4, u8);
#pragma unroll
        for (int a = 0; a < 4; ++a) bfly4_inv(v[a][0], v[a][1], v[a][2], v[a][3], u4, u8, u12);
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        double2 w1, w2, w3;
        if (UNIT) {
            if (b == 0) {
                dft4_inv(v[0][b], v[1][b], v[2][b], v[3][b]);
                continue;
            }
            w1 = root(c, b);
            w2 = root(c, 2 * b);
            w3 = root(c, 3 * b);
        } else if (b == 0) {
            w1 = u.u1;
            w2 = u.u2;
            w3 = u.u3;
        } else {
            w1 = cmul(u.u1, root(c, b));
            w2 = cmul(u.u2, root(c, 2 * b));
            w3 = cmul(u.u3, root(c, 3 * b));
        }
        if (LAST) {
            const double2 b1 = cmulc(v[1][b], w1), b2 = cmulc(v[2][b], w2),
                          b3 = cmulc(v[3][b], w3);
            const double2 t0 = cadd(v[0][b], b2), t1 = csub(v[0][b], b2), t2 = cadd(b1, b3),
                          t3 = csub(b1, b3);
            v[0][b] = cadd(t0, t2);
            v[1][b] = {t1.x - t3.y, t1.y + t3.x};
        } else {
            bfly4_inv(v[0][b], v[1][b], v[2][b], v[3][b], w1, w2, w3);
        }
    }
}

__device__ __forceinline__ int pos1(int t, int a, int b) { return t + 1024 * a + 256 * b; }
__device__ __forceinline__ int pos2(int t, int a, int b)
{
    return 256 * (t >> 4) + (t & 15) + 64 * a + 16 * b;
}
__device__ __forceinline__ int pos3(int t, int a, int b) { return 16 * t + 4 * a + b; }
template <int P>
__device__ __forceinline__ int posn(int t, int a, int b)
{
    return P == 1 ? pos1(t, a, b) : P == 2 ? pos2(t, a, b) : pos3(t, a, b);
}

// Rows r0 and r0 + 1 (if two) of the call, with the Feldkamp weights when
// a.weighted: y[k] = element t + 256 k of the complex row r0 + i r1 (zero
// from W on), k < NK.  Branch-free, with every lane's address clamped into
// the row and the weighting test outside the element loop, so that all the
// loads are in flight together: guarded per element, the compiler waited for
// each element's loads before issuing the next ones (fdk512's pre-filter at
// L = 4096: 5.87 ms against 4.32 ms).
template <int NK>
__device__ __forceinline__ void load_rows(const FftConvArgs& a, int r0, bool two, int t,
                                          double2* y)
{
    const int r1 = two ? r0 + 1 : r0;
    const int view0 = r0 / a.H, k0 = r0 - view0 * a.H;
    const int view1 = r1 / a.H, k1 = r1 - view1 * a.H;
    const float* in0 = a.in + (size_t)r0 * a.W;
    const float* in1 = a.in + (size_t)r1 * a.W;
    if (a.weighted) {
        const double* c0 = a.cosw + (size_t)k0 * a.W;
        const double* c1 = a.cosw + (size_t)k1 * a.W;
        const double* p0 = a.parker + (size_t)view0 * a.W;
        const double* p1 = a.parker + (size_t)view1 * a.W;
        if (view1 == view0) {
            // (rows of one view, the usual case: one Parker load per sample)
#pragma unroll
            for (int k = 0; k < NK; ++k) {
                const int p = t + 256 * k;
                const int pc = min(p, a.W - 1);
                const double pw = p0[pc];
                const double x0 = (double)in0[pc] * c0[pc] * pw;
                const double x1 = (double)in1[pc] * c1[pc] * pw;
                y[k] = p < a.W ? double2{x0, two ? x1 : 0.0} : double2{0.0, 0.0};
            }
        } else {
#pragma unroll
            for (int k = 0; k < NK; ++k) {
                const int p = t + 256 * k;
                const int pc = min(p, a.W - 1);
                const double x0 = (double)in0[pc] * c0[pc] * p0[pc];
                const double x1 = (double)in1[pc] * c1[pc] * p1[pc];
                y[k] = p < a.W ? double2{x0, two ? x1 : 0.0} : double2{0.0, 0.0};
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            const int p = t + 256 * k;
            const int pc = min(p, a.W - 1);
            const double x0 = (double)in0[pc], x1 = (double)in1[pc];
            y[k] = p < a.W ? double2{x0, two ? x1 : 0.0} : double2{0.0, 0.0};
        }
    }
}

// The first forward pass's registers at L = 4096: v[q][b] = element
// pos1(t, q, b) = t + 256 (4 q + b) for q < 2.
__device__ __forceinline__ void load_rows4096(const FftConvArgs& a, int r0, bool two, int t,
                                              double2 (&v)[4][4])
{
    load_rows<8>(a, r0, two, t, &v[0][0]);
}

// Moves the thread's 16 elements from pattern PW to pattern PR through LDS:
// real parts, then imaginary parts, through a buffer of one double per
// position (34 KiB, so that three workgroups share a CU; one double2 per
// position, 68 KiB and two workgroups, measured 7.3 vs 6.1 ms for fdk512's
// pre-filter).  Each thread writes (and later rewrites) only positions it
// has read itself, so the barriers inside are all that is needed.
template <int PW, int PR>
__device__ __forceinline__ void exchange(double* x, double2 (&v)[4][4], int t)
{
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int b = 0; b < 4; ++b) x[qx(posn<PW>(t, q, b))] = v[q][b].x;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int b = 0; b < 4; ++b) v[q][b].x = x[qx(posn<PR>(t, q, b))];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int b = 0; b < 4; ++b) x[qx(posn<PW>(t, q, b))] = v[q][b].y;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int b = 0; b < 4; ++b) v[q][b].y = x[qx(posn<PR>(t, q, b))];
}

// Forward transform (L = 4096) of the complex row whose element p < W is
// load(p) (zero from W on; W <= 2048) into v, thread t ending with the
// elements 16 t + 4 q + b of the transform's output.  Starts with a barrier:
// the buffer's previous reads may follow any pattern.
template <typename Load>
__device__ __forceinline__ void forward4096(double2 (&v)[4][4], double* x, const Roots16& c,
                                            const double2* __restrict__ tw, int t, int W,
                                            Load load)
{
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            // branch-free, so that the loads are in flight together:
            // load(p, in) reads element p < W, in telling whether it is
            // the real one (the ramp's tap gradient at 128^3: 0.66 against
            // 0.58 ms with a test per element)
            const int p = pos1(t, q, b);
            const bool in = p < W;
            const double2 val = load(min(p, W - 1), in);
            v[q][b] = in ? val : double2{0.0, 0.0};
        }
    r16_fwd<true, false>(v, t, c, tw);
    __syncthreads();
    exchange<1, 2>(x, v, t);
    r16_fwd<false, false>(v, 16 * (t & 15), c, tw);
    exchange<2, 3>(x, v, t);
    r16_fwd<false, true>(v, 0, c, tw);
}

// Rows 2b and 2b + 1 (if any) of the call; a.L == 4096.  Three waves per
// SIMD (168 VGPRs, a few spilled): 6.1 ms for fdk512's pre-filter, against
// 7.6 ms at two waves and 7.9 ms at four (128 VGPRs, 42 spilled).
__global__ __launch_bounds__(kF16Threads, 3) void fft_conv4096_kernel(FftConvArgs a)
{
    __shared__ double x[kF16Lds];
    const int t = threadIdx.x;
    const int r0 = 2 * blockIdx.x, r1 = r0 + 1;
    const bool two = r1 < a.rows;
    const double2* __restrict__ tw = a.tw;
    const Roots16 c = roots16(tw);
    double2 v[4][4];
    load_rows4096(a, r0, two, t, v);
    r16_fwd<true, false>(v, t, c, tw);
    exchange<1, 2>(x, v, t);
    r16_fwd<false, false>(v, 16 * (t & 15), c, tw);
    exchange<2, 3>(x, v, t);
    r16_fwd<false, true>(v, 0, c, tw);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int b = 0; b < 4; ++b)
            v[q][b] = cmul(v[q][b], a.spectrum[(4 * q + b) * kF16Threads + t]);
    r16_inv<false, true>(v, 0, c, tw);
    exchange<3, 2>(x, v, t);
    r16_inv<false, false>(v, 16 * (t & 15), c, tw);
    exchange<2, 1>(x, v, t);
    r16_inv<true, false>(v, t, c, tw);
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int p = pos1(t, q, b);
            if (p < a.W) {
                store_sample(a, r0, p, v[q][b].x);
                if (two) store_sample(a, r1, p, v[q][b].y);
            }
        }
}

// As fft_conv4096_kernel for the Ram-Lak taps (a.taps null), whose spectrum
// is real and stored as doubles: 8-byte loads and two products per element
// (on fdk512's pre-filter 5.85 against 6.20 ms with the complex product).
// (A single template for both kernels spilled registers in the complex one.)
__global__ __launch_bounds__(kF16Threads, 3) void fft_conv4096_real_kernel(FftConvArgs a)
{
    __shared__ double x[kF16Lds];
    const int t = threadIdx.x;
    const int r0 = 2 * blockIdx.x, r1 = r0 + 1;
    const bool two = r1 < a.rows;
    const double2* __restrict__ tw = a.tw;
    const Roots16 c = roots16(tw);
    double2 v[4][4];
    load_rows4096(a, r0, two, t, v);
    r16_fwd<true, false>(v, t, c, tw);
    exchange<1, 2>(x, v, t);
    r16_fwd<false, false>(v, 16 * (t & 15), c, tw);
    exchange<2, 3>(x, v, t);
    r16_fwd<false, true>(v, 0, c, tw);
    const double* hs = (const double*)a.spectrum;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const double h = hs[(4 * q + b) * kF16Threads + t];
            v[q][b] = {v[q][b].x * h, v[q][b].y * h};
        }
    r16_inv<false, true>(v, 0, c, tw);
    exchange<3, 2>(x, v, t);
    r16_inv<false, false>(v, 16 * (t & 15), c, tw);
    exchange<2, 1>(x, v, t);
    r16_inv<true, false>(v, t, c, tw);
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int p = pos1(t, q, b);
            if (p < a.W) {
                store_sample(a, r0, p, v[q][b].x);
                if (two) store_sample(a, r1, p, v[q][b].y);
            }
        }
}

// ---------------------------------------------------------------------------
// L = 2560 = 10 x 16 x 16, for rows of 513 to 1280 samples (2W - 1 <= 2560).
//
// With n = n1 + 256 n2 and k = 10 k1 + k2 (n1, k1 < 256; n2, k2 < 10) and
// w = exp(-2 pi i / 2560), w^(n k) = w256^(n1 k1) w^(n1 k2) w10^(n2 k2): the
// forward transform is a first pass of 10-point DFTs over n2 (group n1 holds
// the elements n1 + 256 n2), output k2 times w^(n1 k2) and left at position
// n1 + 256 k2, followed by a 256-point transform over n1 in each block of
// 256 positions.  Those are the second and third radix-16 passes of the
// L = 4096 kernel (the same pass16 stages at Ns = 256 and 16, on the kFftMax
// table: w256^j = w4096^(16 j)), so bin k ends at position 256 k2 + r(k1),
// r reversing the base-4 digits of k1.  The spectrum kernel runs the same
// passes, and the product is again position by position.  The inverse
// mirrors the forward transform.
//
// Samples sit at n < W <= 1280, i.e. n2 < 5: the first pass's DFTs have five
// non-zero inputs, and the last pass only forms its outputs n2 < 5.  A
// 10-point DFT is two 5-point ones: with inputs x[0..4] only, Y[2m] =
// DFT5(x)[m] and Y[2m+1] = DFT5(x[n] w10^n)[m]; in general, with A and B the
// DFTs of the even and odd inputs, Y[k] = A[k] + w10^k B[k] and Y[k+5] =
// A[k] - w10^k B[k].  Per row pair this is ~0.6 of the L = 4096 kernel's
// arithmetic.
//
// One workgroup of 256 threads per row pair: thread t runs group t of the
// 10-point passes, threads t < 160 the radix-16 passes (thread 16 h + j:
// group j of block h, the positions of pos2 and pos3 above).  Block h is
// touched in those passes by threads 16 h .. 16 h + 15 only, which lie in
// one wave, and the LDS operations of a wave take effect in order, so the
// exchanges between the two radix-16 passes need no workgroup barrier.  The
// exchanges to and from the 10-point passes cross waves: one barrier each,
// with a double2 per position.
constexpr int kT2560 = kL2560 / 16;  // threads of the radix-16 passes

// LDS slot of position p: the low four bits of p XORed with bits 4..7, a
// permutation inside each run of 16 positions (so each block of 256 keeps
// its slots) under which the three access patterns (t + 256 k, pos2, pos3)
// hit distinct banks, with no padding: 40 KiB, four workgroups per CU
// (padded like qx, 42.5 KiB and three: 3.26 against 3.00 ms for fdk512's
// pre-filter).
__device__ __forceinline__ int sx(int p) { return p ^ ((p >> 4) & 15); }

// Orders the wave's LDS accesses before the barrier against those after it
// (LDS operations of one wave take effect in issue order; this keeps the
// compiler from moving them across).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct Roots10 {
    double2 w1, w2, w3, w4;  // w10^k = w^(256 k); w5 = w10^2
};
__device__ __forceinline__ Roots10 roots10(const double2* __restrict__ tw)
{
    return {tw[256], tw[512], tw[768], tw[1024]};
}

// In-place 5-point DFT, forward (w5 = exp(-2 pi i / 5)) or inverse
// (conjugate roots, unscaled): the pairs x1 +- x4 and x2 +- x3 share the
// cosines cos(2 pi / 5), cos(4 pi / 5) and the sines.
template <bool INV>
__device__ __forceinline__ void dft5(double2& x0, double2& x1, double2& x2, double2& x3,
                                     double2& x4, const Roots10& r)
{
    const double c1 = r.w2.x, s1 = -r.w2.y, c2 = r.w4.x, s2 = -r.w4.y;
    const double2 t1 = cadd(x1, x4), t2 = cadd(x2, x3), t3 = csub(x1, x4), t4 = csub(x2, x3);
    const double2 a1 = {fma(c2, t2.x, fma(c1, t1.x, x0.x)), fma(c2, t2.y, fma(c1, t1.y, x0.y))};
    const double2 a2 = {fma(c1, t2.x, fma(c2, t1.x, x0.x)), fma(c1, t2.y, fma(c2, t1.y, x0.y))};
    const double2 b1 = {fma(s2, t4.x, s1 * t3.x), fma(s2, t4.y, s1 * t3.y)};
    const double2 b2 = {fma(-s1, t4.x, s2 * t3.x), fma(-s1, t4.y, s2 * t3.y)};
    x0 = cadd(x0, cadd(t1, t2));
    const double2 m1 = {b1.y, -b1.x}, m2 = {b2.y, -b2.x};  // -i b
    if (!INV) {
        x1 = cadd(a1, m1);
        x4 = csub(a1, m1);
        x2 = cadd(a2, m2);
        x3 = csub(a2, m2);
    } else {
        x1 = csub(a1, m1);
        x4 = cadd(a1, m1);
        x2 = csub(a2, m2);
        x3 = cadd(a2, m2);
    }
}

// y[k] *= w^(g k) (CONJ: its conjugate), k = 1..9, the powers formed from
// w^g in FP64 (a few units in its last place)
template <bool CONJ>
__device__ __forceinline__ void twiddle10(double2 (&y)[10], int g,
                                          const double2* __restrict__ tw2560)
{
    const double2 u1 = tw2560[g];
    const double2 u2 = cmul(u1, u1), u3 = cmul(u2, u1), u4 = cmul(u2, u2);
    const double2 u5 = cmul(u4, u1), u6 = cmul(u3, u3), u8 = cmul(u4, u4);
    const double2 u7 = cmul(u6, u1), u9 = cmul(u8, u1);
    const double2 u[9] = {u1, u2, u3, u4, u5, u6, u7, u8, u9};
#pragma unroll
    for (int k = 1; k < 10; ++k) y[k] = CONJ ? cmulc(y[k], u[k - 1]) : cmul(y[k], u[k - 1]);
}

// The first forward pass for group g: y[k] = element g + 256 k on entry
// (PRUNED: y[5..9] are zero), DFT10 output k times w^(g k) on exit.
template <bool PRUNED>
__device__ __forceinline__ void r10_fwd(double2 (&y)[10], int g, const Roots10& r,
                                        const double2* __restrict__ tw2560)
{
    if (PRUNED) {
        double2 o0 = y[0], o1 = cmul(y[1], r.w1), o2 = cmul(y[2], r.w2), o3 = cmul(y[3], r.w3),
                o4 = cmul(y[4], r.w4);
        double2 e0 = y[0], e1 = y[1], e2 = y[2], e3 = y[3], e4 = y[4];
        dft5<false>(e0, e1, e2, e3, e4, r);
        dft5<false>(o0, o1, o2, o3, o4, r);
        y[0] = e0, y[1] = o0, y[2] = e1, y[3] = o1, y[4] = e2;
        y[5] = o2, y[6] = e3, y[7] = o3, y[8] = e4, y[9] = o4;
    } else {
        double2 a0 = y[0], a1 = y[2], a2 = y[4], a3 = y[6], a4 = y[8];
        double2 b0 = y[1], b1 = y[3], b2 = y[5], b3 = y[7], b4 = y[9];
        dft5<false>(a0, a1, a2, a3, a4, r);
        dft5<false>(b0, b1, b2, b3, b4, r);
        b1 = cmul(b1, r.w1);
        b2 = cmul(b2, r.w2);
        b3 = cmul(b3, r.w3);
        b4 = cmul(b4, r.w4);
        y[0] = cadd(a0, b0), y[5] = csub(a0, b0);
        y[1] = cadd(a1, b1), y[6] = csub(a1, b1);
        y[2] = cadd(a2, b2), y[7] = csub(a2, b2);
        y[3] = cadd(a3, b3), y[8] = csub(a3, b3);
        y[4] = cadd(a4, b4), y[9] = csub(a4, b4);
    }
    twiddle10<false>(y, g, tw2560);
}

// The inverse of r10_fwd (times 10) for outputs n2 < 5: y[k] = the
// transform at g + 256 k on entry, y[n] = element g + 256 n (n < 5) on exit.
__device__ __forceinline__ void r10_inv(double2 (&y)[10], int g, const Roots10& r,
                                        const double2* __restrict__ tw2560)
{
    twiddle10<true>(y, g, tw2560);
    double2 a0 = y[0], a1 = y[2], a2 = y[4], a3 = y[6], a4 = y[8];
    double2 b0 = y[1], b1 = y[3], b2 = y[5], b3 = y[7], b4 = y[9];
    dft5<true>(a0, a1, a2, a3, a4, r);
    dft5<true>(b0, b1, b2, b3, b4, r);
    y[0] = cadd(a0, b0);
    y[1] = cadd(a1, cmulc(b1, r.w1));
    y[2] = cadd(a2, cmulc(b2, r.w2));
    y[3] = cadd(a3, cmulc(b3, r.w3));
    y[4] = cadd(a4, cmulc(b4, r.w4));
}

// The radix-16 passes of thread t < kT2560 between the two cross-wave
// exchanges: forward passes 2 and 3 from the pos2 positions, the product
// with the spectrum (REAL: real values stored as doubles), the inverse
// passes 3 and 2, back to the pos2 positions.
template <bool REAL>
__device__ __forceinline__ void middle2560(double2* x, const FftConvArgs& a, int t)
{
    const double2* __restrict__ tw = a.tw;
    const Roots16 c = roots16(tw);
    double2 v[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int b = 0; b < 4; ++b) v[q][b] = x[sx(pos2(t, q, b))];
    r16_fwd<false, false>(v, 16 * (t & 15), c, tw);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int b = 0; b < 4; ++b) x[sx(pos2(t, q, b))] = v[q][b];
    wave_lds_sync();
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int b = 0; b < 4; ++b) v[q][b] = x[sx(pos3(t, q, b))];
    r16_fwd<false, true>(v, 0, c, tw);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = (4 * q + b) * kT2560 + t;
            if (REAL) {
                const double h = ((const double*)a.spectrum)[i];
                v[q][b] = {v[q][b].x * h, v[q][b].y * h};
            } else {
                v[q][b] = cmul(v[q][b], a.spectrum[i]);
            }
        }
    r16_inv<false, true>(v, 0, c, tw);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int b = 0; b < 4; ++b) x[sx(pos3(t, q, b))] = v[q][b];
    wave_lds_sync();
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int b = 0; b < 4; ++b) v[q][b] = x[sx(pos2(t, q, b))];
    r16_inv<false, false>(v, 16 * (t & 15), c, tw);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int b = 0; b < 4; ++b) x[sx(pos2(t, q, b))] = v[q][b];
}

// Rows 2b and 2b + 1 (if any) of the call; a.L == kL2560 (W <= 1280).
// (Four waves per SIMD; the complex-spectrum kernel fitted to four spills
// a few registers and takes three.)
template <bool REAL>
__global__ __launch_bounds__(256, REAL ? 4 : 3) void fft_conv2560_kernel(FftConvArgs a)
{
    __shared__ double2 x[kL2560];
    const int t = threadIdx.x;
    const int r0 = 2 * blockIdx.x, r1 = r0 + 1;
    const bool two = r1 < a.rows;
    const double2* __restrict__ tw2560 = a.tw2560;
    const Roots10 r = roots10(tw2560);
    // (each loop runs once, g = t: written as loops, the kernel fits four
    // waves per SIMD without spilling; straight-line, it spilled 76 bytes)
    for (int g = t; g < 256; g += 256) {
        double2 y[10];
        load_rows<5>(a, r0, two, g, y);
#pragma unroll
        for (int k = 5; k < 10; ++k) y[k] = {0.0, 0.0};
        r10_fwd<true>(y, g, r, tw2560);
#pragma unroll
        for (int k = 0; k < 10; ++k) x[sx(g + 256 * k)] = y[k];
    }
    __syncthreads();
    if (t < kT2560) middle2560<REAL>(x, a, t);
    __syncthreads();
    for (int g = t; g < 256; g += 256) {
        double2 y[10];
#pragma unroll
        for (int k = 0; k < 10; ++k) y[k] = x[sx(g + 256 * k)];
        r10_inv(y, g, r, tw2560);
#pragma unroll
        for (int n = 0; n < 5; ++n) {
            const int p = g + 256 * n;
            if (p < a.W) {
                store_sample(a, r0, p, y[n].x);
                if (two) store_sample(a, r1, p, y[n].y);
            }
        }
    }
}

// The taps' spectrum at L = kL2560 through the same passes, times scale / L,
// stored where thread t's register (q, b) of the radix-16 passes reads it:
// (4 q + b) kT2560 + t (REAL: the real parts as doubles; the Ram-Lak taps
// are even, so their spectrum is real).
template <bool REAL>
__global__ __launch_bounds__(256) void fft_spectrum2560_kernel(FftConvArgs a)
{
    __shared__ double2 x[kL2560];
    const int t = threadIdx.x;
    const double2* __restrict__ tw2560 = a.tw2560;
    const Roots10 r = roots10(tw2560);
    double2 y[10];
    // the taps at n mod L: positions [0, W) and (L - W, L)
#pragma unroll
    for (int k = 0; k < 10; ++k) {
        const int p = t + 256 * k;
        const int n = p < a.W ? p : p - kL2560;
        y[k] = {(p < a.W || p > kL2560 - a.W) ? conv_tap(a, n) : 0.0, 0.0};
    }
    r10_fwd<false>(y, t, r, tw2560);
#pragma unroll
    for (int k = 0; k < 10; ++k) x[sx(t + 256 * k)] = y[k];
    __syncthreads();
    if (t >= kT2560) return;
    const double2* __restrict__ tw = a.tw;
    const Roots16 c = roots16(tw);
    double2 v[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int b = 0; b < 4; ++b) v[q][b] = x[sx(pos2(t, q, b))];
    r16_fwd<false, false>(v, 16 * (t & 15), c, tw);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int b = 0; b < 4; ++b) x[sx(pos2(t, q, b))] = v[q][b];
    wave_lds_sync();
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int b = 0; b < 4; ++b) v[q][b] = x[sx(pos3(t, q, b))];
    r16_fwd<false, true>(v, 0, c, tw);
    const double f = a.scale / (double)kL2560;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = (4 * q + b) * kT2560 + t;
            if (REAL)
                ((double*)a.spectrum)[i] = v[q][b].x * f;
            else
                a.spectrum[i] = {v[q][b].x * f, v[q][b].y * f};
        }
}

// ---------------------------------------------------------------------------
// Weight gradient of the full-row ramp.
//
// dweight[t] = sum_r sum_j dout[r][j] in[r][j + t - pad] = sum_r c_r[t - pad],
// with c_r[s] = sum_j dy_r[j] x_r[j + s] the cross-correlation of row r's
// output gradient with its input, whose spectrum is conj(DY_r) X_r (both
// rows real, zero padded to L >= 2W - 1, so the circular correlation is the
// linear one on |s| <= W - 1).  Two rows a, b are packed as z_x = x_a + i x_b
// and z_d = dy_a + i dy_b; then conj(Z_d) Z_x = conj(DY_a) X_a + conj(DY_b) X_b
// + i (conj(DY_a) X_b - conj(DY_b) X_a), whose first part transforms back to
// the real signal c_a + c_b and the second to an imaginary one: the real part
// of the inverse transform of the summed conj(Z_d) Z_x is sum_r c_r.  The
// forward transforms leave the spectra in the same (digit-reversed) order,
// so the products and sums are taken position by position, and the inverse
// transform returns natural order.

// Block b sums conj(Z_d) Z_x over row pairs b, b + blocks, ... into its slice
// part[b] (each thread owns the positions p = threadIdx.x + 256 m), and the
// output gradients' plain sum (the bias gradient) into bpart[b].
__global__ __launch_bounds__(kFftThreads) void fft_xcorr_partial_kernel(FftXcorrArgs a)
{
    extern __shared__ double2 sm[];
    const int span = a.L + a.L / 8;  // px(L - 1) < span
    double2* zx = sm;
    double2* zd = sm + span;
    __shared__ double red[kFftThreads];
    double2* S = a.part + (size_t)blockIdx.x * a.L;
    for (int p = threadIdx.x; p < a.L; p += kFftThreads) S[p] = {0.0, 0.0};
    double accb = 0.0;
    const int pairs = (a.rows + 1) / 2;
    for (int q = blockIdx.x; q < pairs; q += gridDim.x) {
        const int r0 = 2 * q, r1 = r0 + 1;
        const bool two = r1 < a.rows;
        for (int p = threadIdx.x; p < a.L; p += kFftThreads) {
            double2 vx = {0.0, 0.0}, vd = {0.0, 0.0};
            if (p < a.W) {
                vx.x = a.in[(size_t)r0 * a.W + p];
                vd.x = a.dout[(size_t)r0 * a.W + p];
                if (two) {
                    vx.y = a.in[(size_t)r1 * a.W + p];
                    vd.y = a.dout[(size_t)r1 * a.W + p];
                }
                accb += vd.x + vd.y;
            }
            zx[px(p)] = vx;
            zd[px(p)] = vd;
        }
        __syncthreads();
        fft_forward(zx, a.L, a.log2L, a.tw);
        fft_forward(zd, a.L, a.log2L, a.tw);
        for (int p = threadIdx.x; p < a.L; p += kFftThreads)
            S[p] = cadd(S[p], cmulc(zx[px(p)], zd[px(p)]));
        __syncthreads();  // the next pair overwrites zx and zd
    }
    red[threadIdx.x] = accb;
    __syncthreads();
    if (threadIdx.x == 0) {
        double sb = 0.0;
        for (int t = 0; t < kFftThreads; ++t) sb += red[t];
        a.bpart[blockIdx.x] = sb;
    }
}

// L = 4096: the forward transforms run on registers as in the convolution
// above (Z_x held while Z_d is formed: two waves per SIMD), and the block's
// sums sit in part[b] in the order the registers hold them (element
// 16 t + k of the transform at k * 256 + t, lane-contiguous).
__global__ __launch_bounds__(kF16Threads, 2) void fft_xcorr4096_partial_kernel(FftXcorrArgs a)
{
    __shared__ double x[kF16Lds];
    __shared__ double red[kF16Threads];
    const int t = threadIdx.x;
    const double2* __restrict__ tw = a.tw;
    const Roots16 c = roots16(tw);
    double2* S = a.part + (size_t)blockIdx.x * kFftMax;
#pragma unroll
    for (int k = 0; k < 16; ++k) S[k * kF16Threads + t] = {0.0, 0.0};
    double accb = 0.0;
    const int pairs = (a.rows + 1) / 2;
    for (int q = blockIdx.x; q < pairs; q += gridDim.x) {
        const int r0 = 2 * q, r1 = r0 + 1;
        const bool two = r1 < a.rows;
        const float* x0 = a.in + (size_t)r0 * a.W;
        const float* d0 = a.dout + (size_t)r0 * a.W;
        double2 zx[4][4], zd[4][4];
        const float* x1 = two ? x0 + a.W : x0;  // a row that exists
        const float* d1 = two ? d0 + a.W : d0;
        forward4096(zx, x, c, tw, t, a.W, [&](int p, bool) {
            const double u0 = (double)x0[p], u1 = (double)x1[p];
            return double2{u0, two ? u1 : 0.0};
        });
        forward4096(zd, x, c, tw, t, a.W, [&](int p, bool in) {
            const double u0 = (double)d0[p], u1 = (double)d1[p];
            const double2 d = {u0, two ? u1 : 0.0};
            accb += in ? d.x + d.y : 0.0;
            return d;
        });
#pragma unroll
        for (int qq = 0; qq < 4; ++qq)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                double2* s = S + (4 * qq + b) * kF16Threads + t;
                *s = cadd(*s, cmulc(zx[qq][b], zd[qq][b]));
            }
    }
    red[t] = accb;
    __syncthreads();
    if (t == 0) {
        double sb = 0.0;
        for (int k = 0; k < kF16Threads; ++k) sb += red[k];
        a.bpart[blockIdx.x] = sb;
    }
}

// total[p] = sum over the blocks (in block order) of part[b][p]
__global__ __launch_bounds__(256) void fft_xcorr_sum_kernel(FftXcorrArgs a)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= a.L) return;
    // the L = 4096 partial sums are in register order
    const int src = a.L == kFftMax ? (p & 15) * kF16Threads + (p >> 4) : p;
    double2 s = {0.0, 0.0};
    for (int b = 0; b < a.blocks; ++b) s = cadd(s, a.part[(size_t)b * a.L + src]);
    a.total[p] = s;
}

// One block: the inverse transform of the total, taps t <- lag t - pad.
__global__ __launch_bounds__(kFftThreads) void fft_xcorr_final_kernel(FftXcorrArgs a)
{
    __shared__ double2 x[kFftLds];
    for (int p = threadIdx.x; p < a.L; p += kFftThreads) x[px(p)] = a.total[p];
    __syncthreads();
    fft_inverse(x, a.L, a.log2L, a.tw);
    const double f = 1.0 / (double)a.L;
    for (int t = threadIdx.x; t < a.K; t += kFftThreads) {
        int s = t - a.pad;
        if (s < 0) s += a.L;
        a.dweight[t] = (float)(x[px(s)].x * f);
    }
    if (threadIdx.x == 0 && a.dbias) {
        double sb = 0.0;
        for (int b = 0; b < a.blocks; ++b) sb += a.bpart[b];
        a.dbias[0] = (float)sb;
    }
}

int xcorr_length(int K)
{
    int L = 4;
    while (L < K) L <<= 1;
    // rows of 513..1024 samples take the register-resident L = 4096 kernel
    return L == kFftMax / 2 ? kFftMax : L;
}

size_t fft_xcorr_workspace(int K)
{
    if (K < 1 || !(K & 1) || K > kFftMax - 1) return 0;
    const int L = xcorr_length(K);
    return ((size_t)kFftMax + L + (size_t)kXcorrBlocks * L) * sizeof(double2) +
           (size_t)kXcorrBlocks * sizeof(double);
}

hipError_t launch_fft_xcorr(const FftXcorrArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(fft_twiddle_kernel, dim3(kFftMax / 256), dim3(256), 0, s, a.tw,
                       (double2*)nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.L == kFftMax) {
        hipLaunchKernelGGL(fft_xcorr4096_partial_kernel, dim3(a.blocks), dim3(kF16Threads), 0, s,
                           a);
    } else {
        const size_t lds = (size_t)2 * (a.L + a.L / 8) * sizeof(double2);
        hipLaunchKernelGGL(fft_xcorr_partial_kernel, dim3(a.blocks), dim3(kFftThreads), lds, s,
                           a);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fft_xcorr_sum_kernel, dim3((a.L + 255) / 256), dim3(256), 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fft_xcorr_final_kernel, dim3(1), dim3(kFftThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fft_conv(const FftConvArgs& a, hipStream_t s)
{
    const bool mixed = a.L == kL2560;
    hipLaunchKernelGGL(fft_twiddle_kernel, dim3(kFftMax / 256), dim3(256), 0, s, a.tw,
                       mixed ? a.tw2560 : nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.weighted) {
        const long long n = ((long long)a.views + a.H) * a.W;
        hipLaunchKernelGGL(fft_weights_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                           a);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (mixed && !a.taps)
        hipLaunchKernelGGL(fft_spectrum2560_kernel<true>, dim3(1), dim3(256), 0, s, a);
    else if (mixed)
        hipLaunchKernelGGL(fft_spectrum2560_kernel<false>, dim3(1), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(fft_spectrum_kernel, dim3(1), dim3(kFftThreads), 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (mixed && !a.taps)
        hipLaunchKernelGGL(fft_conv2560_kernel<true>, dim3((a.rows + 1) / 2),
                           dim3(256), 0, s, a);
    else if (mixed)
        hipLaunchKernelGGL(fft_conv2560_kernel<false>, dim3((a.rows + 1) / 2),
                           dim3(256), 0, s, a);
    else if (a.L == kFftMax && !a.taps)
        hipLaunchKernelGGL(fft_conv4096_real_kernel, dim3((a.rows + 1) / 2), dim3(kF16Threads), 0,
                           s, a);
    else if (a.L == kFftMax)
        hipLaunchKernelGGL(fft_conv4096_kernel, dim3((a.rows + 1) / 2), dim3(kF16Threads), 0, s, a);
    else
        hipLaunchKernelGGL(fft_conv_kernel, dim3((a.rows + 1) / 2), dim3(kFftThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace fdk
