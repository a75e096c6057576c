// Row filtering on gfx950: the Feldkamp pre-processing of line integrals
// (cosine weight, Parker short-scan weight, Ram-Lak ramp filter).
//
// One workgroup filters one detector row: the weighted row goes to LDS (the
// weights are computed in place from the geometry), the ramp kernel's taps
// to LDS, and each thread forms outputs j as a direct linear convolution
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

__global__ __launch_bounds__(256) void prefilter_kernel(PrefilterArgs a)
{
    extern __shared__ double lds[];
    double* x = lds;          // W weighted samples
    double* h = lds + a.W;    // taps h[n] for n = 0 .. W-1 (kernel is even)
    const int row = blockIdx.x;  // view * H + k
    const int view = row / a.H;
    const int k = row - view * a.H;
    const double beta = a.beta0 + a.dbeta * view;
    const double cu = 0.5 * (a.W - 1), cv = 0.5 * (a.H - 1);
    const double b = ((double)k - cv) * a.pixel;
    const float* in = a.in + (size_t)row * a.W;
    const double kPi = 3.14159265358979323846;
    for (int j = threadIdx.x; j < a.W; j += 256) {
        // the weights in FP64: the high-pass filter that follows magnifies
        // their relative rounding errors
        const double aj = ((double)j - cu) * a.pixel;
        const double gamma = -atan(aj / a.sdd);
        const double cosw = a.sdd / sqrt(a.sdd * a.sdd + aj * aj + b * b);
        x[j] = (double)in[j] * cosw * parker_weight(beta, gamma, a.delta);
        double hv;
        if (j == 0)
            hv = 1.0 / (4.0 * a.tau * a.tau);
        else if (j & 1)
            hv = -1.0 / (((double)j * kPi * a.tau) * ((double)j * kPi * a.tau));
        else
            hv = 0.0;
        h[j] = hv * a.scale;
    }
    __syncthreads();
    float* out = a.out + (size_t)row * a.W;
    for (int j = threadIdx.x; j < a.W; j += 256) {
        double acc = h[0] * x[j];
        // odd n with 0 <= j - n or j + n < W
        for (int n = 1; n < a.W; n += 2) {
            const double l = (j - n >= 0) ? x[j - n] : 0.0;
            const double r = (j + n < a.W) ? x[j + n] : 0.0;
            acc = fma(h[n], l + r, acc);
        }
        out[j] = (float)acc;
    }
}

hipError_t launch_prefilter(const PrefilterArgs& a, hipStream_t s)
{
    const size_t lds = (size_t)2 * a.W * sizeof(double);
    hipLaunchKernelGGL(prefilter_kernel, dim3(a.rows), dim3(256), lds, s, a);
    return hipGetLastError();
}

}  // namespace fdk
