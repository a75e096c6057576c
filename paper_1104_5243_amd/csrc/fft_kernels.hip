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
// plus one radix-2 stage when log2 L is odd) whose output is in digit-
// reversed order; the inverse is the mirrored decimation-in-time FFT, which
// takes that order and returns natural order.  The taps' spectrum comes from
// the same forward transform, so it sits in the same order and the product
// is taken position by position: no reordering pass.  Twiddles come from a
// table of exp(-2 pi i k / kFftMax), k < kFftMax.  All arithmetic is FP64
// (the ramp removes each row's mean: its output is a small difference of
// large terms), rounded once to FP32 on output.
#include "fdk_internal.h"

namespace fdk {

// 16 waves per workgroup: a stage is one radix-4 butterfly per thread at L =
// 4096, and the waves hide each other's LDS latency (256 threads: 16.8 ms,
// 512: 14.6 ms, 1024: 13.4 ms for fdk512's pre-filter)
constexpr int kFftThreads = 1024;

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

// log2 L odd: a radix-2 stage on the whole row first, then radix 4.
__device__ void fft_forward(double2* x, int L, int log2L, const double2* tw)
{
    int Ns = L;
    if (log2L & 1) {
        dif_stage<2>(x, L, Ns, tw);
        __syncthreads();
        Ns >>= 1;
    }
    for (; Ns >= 4; Ns >>= 2) {
        dif_stage<4>(x, L, Ns, tw);
        __syncthreads();
    }
}

__device__ void fft_inverse(double2* x, int L, int log2L, const double2* tw)
{
    const int Ns0 = (log2L & 1) ? L >> 1 : L;  // length of the first radix-4 stage
    for (int Ns = 4; Ns <= Ns0; Ns <<= 2) {
        dit_stage<4>(x, L, Ns, tw);
        __syncthreads();
    }
    if (log2L & 1) {
        dit_stage<2>(x, L, L, tw);
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void fft_twiddle_kernel(double2* tw)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= kFftMax) return;
    double s, c;
    sincospi(2.0 * (double)k / (double)kFftMax, &s, &c);
    tw[k] = {c, -s};
}

__device__ __forceinline__ double ramlak_tap(int n, double tau)
{
    const double kPi = 3.14159265358979323846;
    if (n == 0) return 1.0 / (4.0 * tau * tau);
    if (n & 1) return -1.0 / (((double)n * kPi * tau) * ((double)n * kPi * tau));
    return 0.0;
}

// Spectrum of the taps, in the forward transform's order, times scale / L.
// Taps h[n] for -(W-1) <= n <= W-1: the Ram-Lak kernel (taps == nullptr)
// or h[n] = taps[pad - n] (transpose: taps[K - 1 - (pad - n)]).
__global__ __launch_bounds__(kFftThreads) void fft_spectrum_kernel(FftConvArgs a)
{
    __shared__ double2 x[kFftLds];
    for (int p = threadIdx.x; p < a.L; p += kFftThreads) x[px(p)] = {0.0, 0.0};
    __syncthreads();
    for (int n = -(a.W - 1) + (int)threadIdx.x; n <= a.W - 1; n += kFftThreads) {
        double h;
        if (!a.taps) {
            h = ramlak_tap(n < 0 ? -n : n, a.tau);
        } else {
            const int t = a.pad - n;
            h = (t >= 0 && t < a.K) ? (double)a.taps[a.transpose ? a.K - 1 - t : t] : 0.0;
        }
        x[px(n < 0 ? n + a.L : n)] = {h, 0.0};
    }
    __syncthreads();
    fft_forward(x, a.L, a.log2L, a.tw);
    const double f = a.scale / (double)a.L;
    for (int p = threadIdx.x; p < a.L; p += kFftThreads)
        a.spectrum[p] = {x[px(p)].x * f, x[px(p)].y * f};
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

hipError_t launch_fft_conv(const FftConvArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(fft_twiddle_kernel, dim3(kFftMax / 256), dim3(256), 0, s, a.tw);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.weighted) {
        const long long n = ((long long)a.views + a.H) * a.W;
        hipLaunchKernelGGL(fft_weights_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                           a);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(fft_spectrum_kernel, dim3(1), dim3(kFftThreads), 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fft_conv_kernel, dim3((a.rows + 1) / 2), dim3(kFftThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace fdk
