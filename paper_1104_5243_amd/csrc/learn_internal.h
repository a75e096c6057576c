// Internal declarations of the row-convolution kernels: the Feldkamp
// pre-filter's and the learned filter's FFT convolution, the learned
// filter's short convolutions, their gradients and the elementwise helpers.
#pragma once

#include "fdk_internal.h"

#include <cstddef>

namespace fdk {

// FFT row convolution (fft_kernels.hip).
constexpr int kFftMax = 4096;  // largest transform: rows of up to 2048 samples
constexpr int kL2560 = 2560;   // mixed-radix transform (10 x 16 x 16): rows of 513..1280
struct FftConvArgs {
    float* out;
    const float* in;
    int rows, W, H;       // H: detector rows per view (weighted input only)
    // transform length >= max(4, 2W - 1): a power of 2 (log2L its log), or
    // kL2560 (log2L unused)
    int L, log2L;
    double2* spectrum;    // L entries, written by the spectrum kernel
    double2* tw;          // kFftMax twiddles, written by the twiddle kernel
    double2* tw2560;      // kL2560 twiddles (L == kL2560 only)
    // taps h[n], -(W-1) <= n <= W-1: Ram-Lak at spacing tau if taps is null,
    // else h[n] = taps[pad - n] (reversed if transpose); all scaled by scale
    const float* taps;
    int K, pad, transpose;
    double tau, scale;
    // Feldkamp weights of the input (weighted = 1): cosine and Parker, with
    // their tables (views x W and H x W, written by the weights kernel)
    int weighted, views;
    double beta0, dbeta, delta, sdd, pixel;
    double* parker;
    double* cosw;
    // output: + bias[0] (if not null), + out (accumulate), ReLU, and kept
    // only where out > 0 on entry (mask)
    const float* bias;
    int accumulate, relu, mask;
};
hipError_t launch_fft_conv(const FftConvArgs& a, hipStream_t s);

// Weight (and bias) gradient of the full-row ramp (one channel, K = 2W - 1
// taps, pad = W - 1) through the FFT: per-block FP64 sums of the row pairs'
// cross-spectra, a fixed-order sum over the blocks, one inverse transform.
struct FftXcorrArgs {
    float* dweight;       // K taps
    float* dbias;         // 1 value, may be null
    const float* dout;    // rows x W
    const float* in;      // rows x W
    int rows, W, K, pad;  // K = 2W - 1, pad = W - 1
    int L, log2L;         // transform length, a power of 2 >= max(4, K)
    int blocks;           // partial-sum blocks
    // workspace slices
    double2* tw;          // kFftMax twiddles
    double2* total;       // L: the summed cross-spectrum
    double* bpart;        // blocks: bias partial sums
    double2* part;        // blocks x L: the blocks' cross-spectrum sums
};
constexpr int kXcorrBlocks = 512;
// transform length of the FFT path for K taps, and its workspace bytes (0 if
// K is not odd or too long)
int xcorr_length(int K);
size_t fft_xcorr_workspace(int K);
hipError_t launch_fft_xcorr(const FftXcorrArgs& a, hipStream_t s);

struct LearnConvArgs {
    float* out;
    const float* in;
    const float* weight;
    const float* bias;   // may be null
    int rows, W, cin, cout, K, pad;
    int relu, accumulate, transpose;
    int mask;            // keep the result where out > 0 on entry, else 0
};

struct LearnGradArgs {
    float* dweight;
    float* dbias;        // may be null
    const float* dout;
    const float* in;
    double* part;        // workspace: blocks x (cout*cin*K + cout)
    int rows, W, cin, cout, K, pad;
};

// Launchers (return the hipError_t of the launch).
hipError_t launch_conv(const LearnConvArgs& a, hipStream_t s);
hipError_t launch_wgrad(const LearnGradArgs& a, int nblocks, hipStream_t s);
hipError_t launch_wgrad_long(const LearnGradArgs& a, int nblocks, hipStream_t s);
hipError_t launch_scale_groups(float* y, const float* x, const float* scale, size_t len,
                               int groups, int accumulate, hipStream_t s);
hipError_t launch_group_dot(float* out, const float* a, const float* b, size_t len, int groups,
                            hipStream_t s);
hipError_t launch_relu_backward(float* dx, const float* dy, const float* y, size_t n, hipStream_t s);
hipError_t launch_matvec(float* y, const float* A, const float* x, int rows, int cols,
                         int transpose, hipStream_t s);
hipError_t launch_adam(float* p, float* m, float* v, const float* g, int n, float lr, float b1,
                       float b2, float eps, int step, hipStream_t s);
hipError_t launch_mse(float* grad, float* loss, double* part, int nparts, const float* a,
                      const float* b, size_t n, hipStream_t s);
constexpr int kGradBlocks = 1024;  // partial-sum blocks of the weight gradients
constexpr int kMseParts = 1024;

}  // namespace fdk
