// Row filtering on gfx950: the Feldkamp pre-processing of line integrals
// (cosine weight, Parker short-scan weight, Ram-Lak ramp filter).
//
// One workgroup filters one detector row: the weighted row goes to LDS (the
// weights are computed in place from the geometry), the ramp kernel's taps
// to LDS, and the threads form the outputs j as a direct linear convolution
//   out[j] = h[0] x[j] + sum over odd n of h[n] (x[j-n] + x[j+n])
// (the Ram-Lak kernel is even and vanishes at even n != 0).  The ramp
// filter removes the row's mean, so its output is a small difference of
// large terms: the row and the taps are held in FP64 and the sum is
// accumulated in FP64 (full-rate FMAs on this GPU), rounded once to FP32.
#include "fdk_internal.h"

namespace fdk {

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

// Each thread forms kOut = 8 consecutive outputs j0 .. j0+7 and takes the odd
// taps four at a time (n, n+2, n+4, n+6 with n = 1 + 8m): one load of the
// windows x[j0-n-6 .. j0-n+7] and x[j0+n .. j0+n+13] into registers serves
// all four, so a tap costs 3.5 LDS reads for eight outputs.  The row sits in
// LDS between zero borders (L >= W + 6 samples on the left, R >= W + 13 on
// the right) and is split into its eight phases i mod 8, each stored
// contiguously: the lanes of a wave then read consecutive doubles in one
// phase, free of bank conflicts (with plain storage lane t would read at a
// stride of 64 bytes).  The taps h[n] are zero-padded up to W + 8.
constexpr int kOut = 8;

struct PrefilterLds {
    int L, S, PL;  // left border, padded row length, phase length
    __host__ __device__ explicit PrefilterLds(int W)
    {
        L = (W + 8 + 7) & ~7;
        S = L + W + W + 16;
        PL = (S + 7) >> 3;
    }
    __host__ __device__ size_t doubles(int W) const { return (size_t)8 * PL + W + 8; }
};

__global__ __launch_bounds__(256) void prefilter_kernel(PrefilterArgs a)
{
    extern __shared__ double lds[];
    const int W = a.W;
    const PrefilterLds g(W);
    const int PL = g.PL;
    double* xs = lds;                 // phase p holds x[8q + p - L] at xs[p * PL + q]
    double* h = lds + 8 * PL;         // taps h[n], n = 0 .. W+7 (the kernel is even)
    const int row = blockIdx.x;       // view * H + k
    const int view = row / a.H;
    const int k = row - view * a.H;
    const double beta = a.beta0 + a.dbeta * view;
    const double cu = 0.5 * (W - 1), cv = 0.5 * (a.H - 1);
    const double b = ((double)k - cv) * a.pixel;
    const float* in = a.in + (size_t)row * W;
    const double kPi = 3.14159265358979323846;
    for (int ip = threadIdx.x; ip < 8 * PL; ip += blockDim.x) {
        const int j = ip - g.L;
        double v = 0.0;
        if (j >= 0 && j < W) {
            // the weights in FP64: the high-pass filter that follows
            // magnifies their relative rounding errors
            const double aj = ((double)j - cu) * a.pixel;
            const double gamma = -atan(aj / a.sdd);
            const double cosw = a.sdd / sqrt(a.sdd * a.sdd + aj * aj + b * b);
            v = (double)in[j] * cosw * parker_weight(beta, gamma, a.delta);
        }
        xs[(ip & 7) * PL + (ip >> 3)] = v;
    }
    for (int j = threadIdx.x; j < W + 8; j += blockDim.x) {
        double hv = 0.0;
        if (j == 0)
            hv = 1.0 / (4.0 * a.tau * a.tau);
        else if ((j & 1) && j < W)
            hv = -1.0 / (((double)j * kPi * a.tau) * ((double)j * kPi * a.tau));
        h[j] = hv * a.scale;
    }
    __syncthreads();
    float* out = a.out + (size_t)row * W;
    for (int j0 = threadIdx.x * kOut; j0 < W; j0 += blockDim.x * kOut) {
        const int base = (j0 + g.L) >> 3;  // j0 + L is a multiple of 8
        double acc[kOut];
#pragma unroll
        for (int o = 0; o < kOut; ++o) acc[o] = h[0] * xs[o * PL + base];
        for (int m = 0; 8 * m + 1 < W; ++m) {
            // padded index of x[j0 - n - 6 + e] is 8 (base - m) + e - 7,
            // of x[j0 + n + e] is 8 (base + m) + e + 1
            double l[kOut + 6], r[kOut + 6];
#pragma unroll
            for (int e = 0; e < kOut + 6; ++e) {
                const int ph = (e + 1) & 7;
                l[e] = xs[ph * PL + base - m + ((e - 7) >> 3)];
                r[e] = xs[ph * PL + base + m + ((e + 1) >> 3)];
            }
            const int n = 8 * m + 1;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double hn = h[n + 2 * q];
#pragma unroll
                for (int o = 0; o < kOut; ++o)
                    acc[o] = fma(hn, l[o + 6 - 2 * q] + r[o + 2 * q], acc[o]);
            }
        }
#pragma unroll
        for (int o = 0; o < kOut; ++o)
            if (j0 + o < W) out[j0 + o] = (float)acc[o];
    }
}

hipError_t launch_prefilter(const PrefilterArgs& a, hipStream_t s)
{
    const PrefilterLds g(a.W);
    const size_t lds = g.doubles(a.W) * sizeof(double);
    int threads = ((a.W + kOut - 1) / kOut + 63) / 64 * 64;
    if (threads > 256) threads = 256;
    hipLaunchKernelGGL(prefilter_kernel, dim3(a.rows), dim3(threads), lds, s, a);
    return hipGetLastError();
}

}  // namespace fdk
