// Host side of the C-ABI entry points of the row-convolution kernels
// declared in include/fdk.h: the Feldkamp pre-filter, the learned filter's
// convolutions and their gradients, and the elementwise helpers.
#include "../../include/fdk.h"
#include "api_internal.h"
#include "learn_internal.h"

#include <algorithm>

using namespace fdk;
using namespace fdk::host;

namespace {

// FFT row convolution: transform length, tables in the staging buffer
// (ordered after its previous user), the three launches, timed as one.
int run_fft_conv(FftConvArgs A, hipStream_t stream)
{
    int L = 4, log2L = 2;
    while (L < 2 * A.W - 1) {
        L <<= 1;
        ++log2L;
    }
    // rows of 513..1280 samples take the mixed-radix L = 2560 kernel (more
    // zero padding than 2W - 1 leaves the linear convolution unchanged):
    // registers hold each pass, and the transform is 0.6 of L = 4096's;
    // against the general kernel at L = 2048, the register-resident kernels
    // convolve a row pair in about a third of the time (learned filter at
    // 128^3: 1.0 -> 0.4 ms at L = 4096); longer rows take L = 4096
    if (A.W > 512 && 2 * A.W - 1 <= kL2560) {
        L = kL2560;
        log2L = 0;
    }
    A.L = L;
    A.log2L = log2L;
    std::lock_guard<std::mutex> lock(g_stage_mu);
    Staging* st = nullptr;
    const size_t tables = A.weighted ? ((size_t)A.views + A.H) * A.W * sizeof(double) : 0;
    int rc = acquire_staging((size_t)(kFftMax + kL2560 + L) * 16 + tables, stream, &st);
    if (rc != FDK_OK) return rc;
    A.tw = (double2*)st->ptr;
    A.tw2560 = A.tw + kFftMax;
    A.spectrum = A.tw2560 + kL2560;
    A.parker = (double*)(A.spectrum + L);
    A.cosw = A.parker + (size_t)A.views * A.W;
    hipEvent_t t0;
    if ((rc = timed_begin(stream, &t0)) != FDK_OK) return rc;
    hipError_t e = launch_fft_conv(A, stream);
    if (e != hipSuccess) return hip_fail(e, "FFT convolution launch");
    if ((rc = timed_end(stream, t0)) != FDK_OK) return rc;
    e = hipEventRecord(st->last_use, stream);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    return FDK_OK;
}

}  // namespace

extern "C" {

int fdk_prefilter(float* out, const float* in, int n_views, int H, int W, double beta0,
                  double dbeta, double delta, double sid, double sdd, double pixel,
                  void* stream)
{
    g_err.clear();
    if (n_views < 0) return fail(FDK_ERR_INVALID_ARG, "n_views=%d < 0", n_views);
    if (H < 1 || W < 1 || W > kFftMax / 2 || H > 32768)
        return fail(FDK_ERR_INVALID_ARG, "detector %dx%d outside [1, %d] x [1, 32768]", W, H,
                    kFftMax / 2);
    if (n_views == 0) return FDK_OK;
    if (!out || !in) return fail(FDK_ERR_INVALID_ARG, "out or in is NULL");
    if (out == in) return fail(FDK_ERR_INVALID_ARG, "out and in must be distinct buffers");
    if (!(std::isfinite(beta0) && std::isfinite(dbeta) && std::isfinite(delta)))
        return fail(FDK_ERR_INVALID_ARG, "angles must be finite");
    if (!(sid > 0.0 && sdd > 0.0 && pixel > 0.0 && std::isfinite(sid) && std::isfinite(sdd) &&
          std::isfinite(pixel)))
        return fail(FDK_ERR_INVALID_ARG, "sid, sdd and pixel must be finite and > 0");
    if ((long long)n_views * H > 0x7fffffffLL)
        return fail(FDK_ERR_INVALID_ARG, "too many rows");
    FftConvArgs A = {};
    A.out = out;
    A.in = in;
    A.rows = n_views * H;
    A.W = W;
    A.H = H;
    A.tau = pixel * sid / sdd;
    A.scale = A.tau * dbeta;
    A.weighted = 1;
    A.views = n_views;
    A.beta0 = beta0;
    A.dbeta = dbeta;
    A.delta = delta;
    A.sdd = sdd;
    A.pixel = pixel;
    return run_fft_conv(A, (hipStream_t)stream);
}

int fdk_conv_rows(float* out, const float* in, const float* weight, const float* bias, int rows,
                  int W, int cin, int cout, int K, int pad, int flags, void* stream)
{
    g_err.clear();
    if (rows < 0 || W < 1 || cin < 1 || cout < 1 || K < 1)
        return fail(FDK_ERR_INVALID_ARG, "bad sizes rows=%d W=%d cin=%d cout=%d K=%d", rows, W,
                    cin, cout, K);
    if (pad < 0 || pad >= K + W) return fail(FDK_ERR_INVALID_ARG, "pad=%d out of range", pad);
    if (flags & ~(FDK_CONV_RELU | FDK_CONV_ACCUMULATE | FDK_CONV_TRANSPOSE | FDK_CONV_RELU_MASK))
        return fail(FDK_ERR_INVALID_ARG, "unknown flags %d", flags);
    if ((flags & FDK_CONV_RELU_MASK) && (flags & (FDK_CONV_RELU | FDK_CONV_ACCUMULATE)))
        return fail(FDK_ERR_INVALID_ARG, "FDK_CONV_RELU_MASK excludes RELU and ACCUMULATE");
    const bool shortk = K <= 32 && cout <= 64 && cin <= 64;
    const bool longk = cin == 1 && cout == 1 && K <= 8191;
    if (!shortk && !longk)
        return fail(FDK_ERR_UNSUPPORTED, "need K <= 32 and channels <= 64, or cin = cout = 1");
    if (rows == 0) return FDK_OK;
    if (!out || !in || !weight) return fail(FDK_ERR_INVALID_ARG, "out, in or weight is NULL");
    if (out == in) return fail(FDK_ERR_INVALID_ARG, "out and in must be distinct");
    if (rows > 65535) return fail(FDK_ERR_UNSUPPORTED, "rows=%d > 65535 per call", rows);
    if (cin == 1 && cout == 1 && K > 32 && K == 2 * W - 1 && pad == W - 1 && W <= kFftMax / 2) {
        // a full-row ramp: FFT convolution in FP64
        FftConvArgs F = {};
        F.out = out;
        F.in = in;
        F.rows = rows;
        F.W = W;
        F.H = 1;
        F.taps = weight;
        F.K = K;
        F.pad = pad;
        F.transpose = (flags & FDK_CONV_TRANSPOSE) ? 1 : 0;
        F.scale = 1.0;
        F.bias = bias;
        F.relu = (flags & FDK_CONV_RELU) ? 1 : 0;
        F.accumulate = (flags & FDK_CONV_ACCUMULATE) ? 1 : 0;
        F.mask = (flags & FDK_CONV_RELU_MASK) ? 1 : 0;
        return run_fft_conv(F, (hipStream_t)stream);
    }
    LearnConvArgs A = {};
    A.out = out;
    A.in = in;
    A.weight = weight;
    A.bias = bias;
    A.rows = rows;
    A.W = W;
    A.cin = cin;
    A.cout = cout;
    A.K = K;
    A.pad = pad;
    A.relu = (flags & FDK_CONV_RELU) ? 1 : 0;
    A.accumulate = (flags & FDK_CONV_ACCUMULATE) ? 1 : 0;
    A.transpose = (flags & FDK_CONV_TRANSPOSE) ? 1 : 0;
    A.mask = (flags & FDK_CONV_RELU_MASK) ? 1 : 0;
    hipEvent_t t0;
    int rc = timed_begin((hipStream_t)stream, &t0);
    if (rc != FDK_OK) return rc;
    hipError_t e = launch_conv(A, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "conv launch");
    return timed_end((hipStream_t)stream, t0);
}

size_t fdk_conv_rows_wgrad_workspace(int cin, int cout, int K)
{
    if (cin < 1 || cout < 1 || K < 1) return 0;
    const size_t direct = (size_t)kGradBlocks * ((size_t)cin * cout * K + cout) * sizeof(double);
    // a single-channel ramp of K = 2W - 1 taps may take the FFT path
    const size_t fft = cin == 1 && cout == 1 && K > 32 ? fft_xcorr_workspace(K) : 0;
    return std::max(direct, fft);
}

int fdk_conv_rows_wgrad(float* dweight, float* dbias, const float* dout, const float* in, int rows,
                        int W, int cin, int cout, int K, int pad, void* workspace,
                        size_t workspace_bytes, void* stream)
{
    g_err.clear();
    if (rows < 0 || W < 1 || cin < 1 || cout < 1 || K < 1)
        return fail(FDK_ERR_INVALID_ARG, "bad sizes");
    if (pad < 0 || pad >= K + W) return fail(FDK_ERR_INVALID_ARG, "pad=%d out of range", pad);
    const bool longk = cin == 1 && cout == 1 && K > 32;
    if (!longk && (long long)cin * cout * K > 10240)
        return fail(FDK_ERR_UNSUPPORTED, "cin*cout*K > 10240");
    if (longk && K > 8192) return fail(FDK_ERR_UNSUPPORTED, "K > 8192");
    if (!dweight || !dout || !in || !workspace)
        return fail(FDK_ERR_INVALID_ARG, "dweight, dout, in or workspace is NULL");
    if (workspace_bytes < fdk_conv_rows_wgrad_workspace(cin, cout, K))
        return fail(FDK_ERR_INVALID_ARG, "workspace of %zu bytes is too small", workspace_bytes);
    if (longk && (size_t)(2 * W + K) * sizeof(float) > 65536)
        return fail(FDK_ERR_UNSUPPORTED, "row too long for the LDS");
    if (!longk && (size_t)(cout * 128 + cin * (128 + K - 1)) * sizeof(float) > 65536)
        return fail(FDK_ERR_UNSUPPORTED, "channels too many for the LDS");
    if (longk && K == 2 * W - 1 && pad == W - 1 && W <= kFftMax / 2) {
        // the full-row ramp: cross-spectra through the FFT (FP64)
        FftXcorrArgs X;
        X.dweight = dweight;
        X.dbias = dbias;
        X.dout = dout;
        X.in = in;
        X.rows = rows;
        X.W = W;
        X.K = K;
        X.pad = pad;
        X.L = xcorr_length(K);
        X.log2L = 0;
        while ((1 << X.log2L) < X.L) ++X.log2L;
        X.blocks = std::max(1, std::min(kXcorrBlocks, (rows + 1) / 2));
        X.tw = (double2*)workspace;
        X.total = X.tw + kFftMax;
        X.part = X.total + X.L;
        X.bpart = (double*)(X.part + (size_t)kXcorrBlocks * X.L);
        const hipError_t e = launch_fft_xcorr(X, (hipStream_t)stream);
        return e == hipSuccess ? FDK_OK : hip_fail(e, "wgrad launch");
    }
    LearnGradArgs A;
    A.dweight = dweight;
    A.dbias = dbias;
    A.dout = dout;
    A.in = in;
    A.part = (double*)workspace;
    A.rows = rows;
    A.W = W;
    A.cin = cin;
    A.cout = cout;
    A.K = K;
    A.pad = pad;
    hipError_t e = longk ? launch_wgrad_long(A, kGradBlocks, (hipStream_t)stream)
                         : launch_wgrad(A, kGradBlocks, (hipStream_t)stream);
    return e == hipSuccess ? FDK_OK : hip_fail(e, "wgrad launch");
}

int fdk_scale_groups(float* y, const float* x, const float* scale, size_t group_len, int groups,
                     int accumulate, void* stream)
{
    g_err.clear();
    if (groups < 0) return fail(FDK_ERR_INVALID_ARG, "groups < 0");
    if (groups == 0 || group_len == 0) return FDK_OK;
    if (!y || !x || !scale) return fail(FDK_ERR_INVALID_ARG, "NULL pointer");
    hipError_t e = launch_scale_groups(y, x, scale, group_len, groups, accumulate,
                                       (hipStream_t)stream);
    return e == hipSuccess ? FDK_OK : hip_fail(e, "scale launch");
}

int fdk_group_dot(float* out, const float* a, const float* b, size_t group_len, int groups,
                  void* stream)
{
    g_err.clear();
    if (groups < 0 || groups > 0x7fffffff) return fail(FDK_ERR_INVALID_ARG, "bad groups");
    if (groups == 0) return FDK_OK;
    if (!out || !a || !b) return fail(FDK_ERR_INVALID_ARG, "NULL pointer");
    hipError_t e = launch_group_dot(out, a, b, group_len, groups, (hipStream_t)stream);
    return e == hipSuccess ? FDK_OK : hip_fail(e, "group_dot launch");
}

int fdk_relu_backward(float* dx, const float* dy, const float* y, size_t n, void* stream)
{
    g_err.clear();
    if (n == 0) return FDK_OK;
    if (!dx || !dy || !y) return fail(FDK_ERR_INVALID_ARG, "NULL pointer");
    hipError_t e = launch_relu_backward(dx, dy, y, n, (hipStream_t)stream);
    return e == hipSuccess ? FDK_OK : hip_fail(e, "relu_backward launch");
}

int fdk_matvec(float* y, const float* A, const float* x, int rows, int cols, int transpose,
               void* stream)
{
    g_err.clear();
    if (rows < 1 || cols < 1) return fail(FDK_ERR_INVALID_ARG, "bad sizes");
    if (!y || !A || !x) return fail(FDK_ERR_INVALID_ARG, "NULL pointer");
    hipError_t e = launch_matvec(y, A, x, rows, cols, transpose, (hipStream_t)stream);
    return e == hipSuccess ? FDK_OK : hip_fail(e, "matvec launch");
}

int fdk_adam(float* param, float* m, float* v, const float* grad, int n, float lr, float beta1,
             float beta2, float eps, int step, void* stream)
{
    g_err.clear();
    if (n < 0 || step < 1) return fail(FDK_ERR_INVALID_ARG, "n < 0 or step < 1");
    if (n == 0) return FDK_OK;
    if (!param || !m || !v || !grad) return fail(FDK_ERR_INVALID_ARG, "NULL pointer");
    hipError_t e = launch_adam(param, m, v, grad, n, lr, beta1, beta2, eps, step,
                               (hipStream_t)stream);
    return e == hipSuccess ? FDK_OK : hip_fail(e, "adam launch");
}

int fdk_mse(float* grad, float* loss, const float* a, const float* b, size_t n, void* workspace,
            size_t workspace_bytes, void* stream)
{
    g_err.clear();
    if (n == 0) return fail(FDK_ERR_INVALID_ARG, "n == 0");
    if (!loss || !a || !b || !workspace) return fail(FDK_ERR_INVALID_ARG, "NULL pointer");
    if (workspace_bytes < kMseParts * sizeof(double))
        return fail(FDK_ERR_INVALID_ARG, "workspace too small");
    hipError_t e = launch_mse(grad, loss, (double*)workspace, kMseParts, a, b, n,
                              (hipStream_t)stream);
    return e == hipSuccess ? FDK_OK : hip_fail(e, "mse launch");
}

}  // extern "C"
