/*
 * fdk.h - C ABI of the MI355X (gfx950) cone-beam backprojection library.
 *
 * The library computes the voxel-driven backprojection step of the Feldkamp
 * (FDK) reconstruction: for every voxel and every projection i, the 3x4
 * matrix P_i maps the voxel centre to (u w, v w, w); the filtered projection
 * is sampled bilinearly at (u, v) and fx / w^2 is added to the voxel
 * (paper, Section 3.1, Listing 1, and the three parts of Section 3.2).
 *
 * Conventions shared by every entry point:
 *   volume     device float, N*N*N, voxel (x, y, z) at volume[(z*N + y)*N + x];
 *              its centre is origin + voxel_size * (x, y, z) in mm.
 *   proj_stack device, n_views*H*W, pixel (j, k) of view i at
 *              [(i*H + k)*W + j]; the pixel's centre is at u = j, v = k.
 *   P_mats     host double, n_views*12, row-major 3x4 per view mapping
 *              homogeneous world mm (x, y, z, 1) to (u w, v w, w).
 *              Read during the call only (folded into the volume's centred
 *              index frame in FP64 on the host and copied to the device; the
 *              library keeps no pointer to it).
 *   origin     host float[3].
 *   stream     a hipStream_t passed as void*; NULL is the null stream.
 * Semantics:
 *   - The backprojection ACCUMULATES into the volume (+=); zero it first for
 *     a fresh reconstruction.  Views may be streamed over several calls.
 *   - Taps outside the detector read 0; the cast of u, v to a pixel index is
 *     floor; a voxel with w <= 0 receives nothing from that view.
 *   - Calls are asynchronous: they return once the work is enqueued on
 *     `stream`.  The caller keeps every device buffer alive and unmodified
 *     until the stream has passed the call.  Two calls that write the same
 *     output must be ordered on one stream (or by events) by the caller.
 *   - The library never frees or retains caller memory.  It owns one
 *     staging buffer per device (zero-padded copies of a batch of views;
 *     two batches when a call of the fused kernel with FP16 or BF16 views
 *     has several, so that the next batch is staged on a second stream of
 *     the library's while the current one is backprojected), grown on
 *     demand and released by fdk_release().  The second stream starts after
 *     the caller's earlier work on `stream`, and the call's last kernel, on
 *     `stream`, follows all of its work, so the call is ordered on `stream`
 *     as a whole.  Calls on different streams that share the buffer are
 *     ordered by the library with events.  (FDK_STAGE_OVERLAP=0 or 1 in the
 *     environment at load time stages on `stream` itself, or on the second
 *     stream, for every storage type.)
 * Errors: every entry point returns FDK_OK (0) or a negative code, and
 * fdk_last_error() describes the last failure of the calling thread.
 * Arguments are validated before anything is enqueued; a rejected call has
 * no effect.  Non-finite data values propagate unchecked.
 */
#ifndef FDK_H
#define FDK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FDK_OK 0
#define FDK_ERR_INVALID_ARG (-1) /* null pointer, bad size, non-finite geometry */
#define FDK_ERR_HIP (-2)         /* a HIP runtime call or kernel launch failed */
#define FDK_ERR_UNSUPPORTED (-3) /* valid request the library cannot serve */

/* Projection storage types for fdk_backproject_ex. */
#define FDK_DTYPE_F32 0
#define FDK_DTYPE_F16 1
#define FDK_DTYPE_BF16 2

/* Kernel variants for fdk_backproject_ex (flags). */
#define FDK_KERNEL_FUSED 0 /* several views fused per pass, z-line per thread */
#define FDK_KERNEL_PLAIN 1 /* one thread per voxel, the listing's arithmetic */

/*
 * fdk_backproject - FP32 backprojection of n_views projections.
 * Paper Section 3.1 (Listing 1), with the zero-padded projection buffers of
 * Section 3.3 and the image-loop blocking of Section 6.2: views are taken in
 * batches, each batch staged into zero-padded buffers and backprojected in
 * one pass that keeps the voxel sums in registers.
 *   volume      device float[N^3], accumulated (+=)
 *   N           voxels per axis, 1 <= N <= 4096
 *   voxel_size  mm, finite and > 0
 *   origin      host float[3], centre of voxel (0,0,0) in mm
 *   proj_stack  device float[n_views*H*W]
 *   n_views     >= 0 (0 is a no-op returning FDK_OK)
 *   H, W        detector rows and columns, 1..32768
 *   P_mats      host double[n_views*12], finite
 *   stream      hipStream_t as void*
 */
int fdk_backproject(float* volume, int N, float voxel_size, const float origin[3],
                    const float* proj_stack, int n_views, int H, int W, const double* P_mats,
                    void* stream);

/*
 * fdk_backproject_ex - as fdk_backproject, with a choice of projection
 * storage type and kernel.
 *   proj_stack  device, n_views*H*W elements of proj_dtype (FDK_DTYPE_*):
 *               FP16 and BF16 are IEEE binary16 / bfloat16 bit patterns.
 *   view_scale  host float[n_views] or NULL: view i's pixel values are
 *               multiplied by view_scale[i] > 0.  Applied by folding
 *               1/sqrt(view_scale[i]) into the matrix in FP64 before its one
 *               rounding to FP32, so a power of 4 is applied exactly.  Lets
 *               FP16 stacks be stored pre-scaled into range.
 *   flags       FDK_KERNEL_FUSED or FDK_KERNEL_PLAIN (the plain kernel
 *               accepts FP32 only and no view_scale).
 * All arithmetic and the accumulation are FP32 whatever the storage type.
 */
int fdk_backproject_ex(float* volume, int N, float voxel_size, const float origin[3],
                       const void* proj_stack, int proj_dtype, int n_views, int H, int W,
                       const double* P_mats, const float* view_scale, int flags, void* stream);

/*
 * fdk_convert_storage - an FP32 stack in reduced-precision storage for
 * fdk_backproject_ex (FP16 or BF16 taps halve the gather bytes; the
 * arithmetic stays FP32).
 *   dst         device, n_views*H*W 16-bit elements (IEEE binary16 or bfloat16
 *               bit patterns), overwritten
 *   src         device float[n_views*H*W]
 *   dtype       FDK_DTYPE_F16: view i is multiplied by 4^k_i, k_i the largest
 *               integer with 4^k_i max|view i| <= 2^14 (clipped to [-60, 60];
 *               0 for an all-zero view), then rounded to nearest even;
 *               view_scale[i] = 4^-k_i is written (device float[n_views],
 *               required) and undoes the scaling exactly when passed to
 *               fdk_backproject_ex.  (Filtered projections are ~1e-4, where
 *               FP16 would be subnormal.)
 *               FDK_DTYPE_BF16: each value rounded to nearest even (FP32's
 *               range); view_scale is not used and may be NULL.
 * Asynchronous on `stream`; the caller copies view_scale to the host.
 */
int fdk_convert_storage(void* dst, const float* src, int n_views, int H, int W, int dtype,
                        float* view_scale, void* stream);

/*
 * fdk_backproject_noalloc - fdk_backproject_ex's fused path for callers that
 * cannot allocate device memory (code under HIP graph capture, serving loops
 * that forbid allocation).  It calls no hipMalloc, hipFree or allocating
 * library routine and records no events: each pass's staged planes and
 * folded matrices go to a fixed scratch array of FDK_NOALLOC_SCRATCH_BYTES
 * that the library holds on every device it runs on until the process ends,
 * and the matrices reach it through a kernel's arguments.
 *   Arguments as fdk_backproject_ex (flags fixed to FDK_KERNEL_FUSED).
 *   Views per pass: at most the fdk_set_batch value, at most 64, and as many
 *   staged views as fit the scratch array (27 FP32 or 54 FP16/BF16 views of
 *   1248x960 in the default layout); results equal fdk_backproject_ex's run
 *   with that batch.  A single staged view larger than the array is rejected
 *   with FDK_ERR_UNSUPPORTED before anything is enqueued.
 *   Every call on a device shares that device's scratch array and leaves its
 *   contents behind: two calls that may overlap on one device (different
 *   streams, or host threads) race and must be ordered by the caller.
 */
#define FDK_NOALLOC_SCRATCH_BYTES ((size_t)256 * 1024 * 1024)
int fdk_backproject_noalloc(float* volume, int N, float voxel_size, const float origin[3],
                            const void* proj_stack, int proj_dtype, int n_views, int H, int W,
                            const double* P_mats, const float* view_scale, void* stream);

/*
 * fdk_backproject_plain - the plain FP32 path: one thread per voxel, the
 * listing's arithmetic (world coordinates, one IEEE division per
 * coordinate, bounds-checked taps), all views of a batch accumulated in a
 * register.  For comparison with fdk_backproject on the same GPU.
 * Arguments as fdk_backproject.
 */
int fdk_backproject_plain(float* volume, int N, float voxel_size, const float origin[3],
                          const float* proj_stack, int n_views, int H, int W,
                          const double* P_mats, void* stream);

/*
 * fdk_forward_project - the matched cone-beam forward projector, the exact
 * transpose of fdk_backproject (FP32 storage, FDK_DIVIDE_RCP): every
 * voxel's value times 1/w^2 is spread onto the four pixels the
 * backprojection reads, with the same bilinear weights, computed by the same
 * operations; pixels outside the detector are dropped.  ACCUMULATES into
 * proj_stack (+=).  Each view's sums are formed in 64-bit fixed point
 * (integer atomics, whose order does not change the result), so the output
 * is the same on every run; the one exception is a batch of views in which
 * some voxel lies on or behind a source plane (w <= 0), whose sums are
 * formed with float atomics and may differ between runs in the last bits.
 *   proj_stack  device float[n_views*H*W], accumulated
 *   volume      device float[N^3]
 *   other arguments as fdk_backproject.
 */
int fdk_forward_project(float* proj_stack, int n_views, int H, int W, const double* P_mats,
                        const float* volume, int N, float voxel_size, const float origin[3],
                        void* stream);

/*
 * fdk_prefilter - the Feldkamp 2D pre-processing of line integrals on the
 * GPU (the step before the backprojection, named in the paper's Section 1.1):
 * for view i (source angle beta_i = beta0 + i*dbeta) and pixel (j, k) with
 * detector offsets a = (j - (W-1)/2) pixel, b = (k - (H-1)/2) pixel (mm),
 *   q = p * sdd / sqrt(sdd^2 + a^2 + b^2) * parker(beta_i, gamma_j)
 * with gamma_j = -atan(a / sdd) and the Parker short-scan weight over
 * pi + 2*delta (parker = 1/2 everywhere when delta < 0: full circle), then
 * each row is convolved (linear convolution, zero outside the row) with the
 * discrete Ram-Lak kernel h[0] = 1/(4 tau^2), h[odd n] = -1/(n pi tau)^2,
 * h[even n] = 0 at the isocentre spacing tau = pixel * sid / sdd, and scaled
 * by tau * dbeta (the angular step of the backprojection sum).
 *   out, in     device float[n_views*H*W] (out is overwritten; distinct buffers)
 *   all lengths in mm, angles in radians.
 */
int fdk_prefilter(float* out, const float* in, int n_views, int H, int W, double beta0,
                  double dbeta, double delta, double sid, double sdd, double pixel,
                  void* stream);

/*
 * Kernels of the learned filter (training and inference).  The learned
 * Feldkamp filter acts along detector rows: a long learned ramp, a per-view
 * weight, and a small 1D CNN; these entry points are its building blocks.
 * All tensors are device float32, rows of W samples, channel-major within a
 * row: x[r][c][j] at ((r*channels + c)*W + j).  Outputs are overwritten unless
 * stated.  Asynchronous on `stream`.
 */
#define FDK_CONV_RELU 1       /* max(0, .) on the result */
#define FDK_CONV_ACCUMULATE 2 /* add the existing output before the ReLU */
#define FDK_CONV_TRANSPOSE 4  /* the adjoint convolution (data gradient) */
/* keep the result where out > 0 on entry and store 0 elsewhere: with out
 * holding a ReLU's output, this applies that ReLU's backward step to the
 * result (which overwrites it); excludes FDK_CONV_RELU and _ACCUMULATE */
#define FDK_CONV_RELU_MASK 8

/*
 * fdk_conv_rows - batched 1D convolution along rows with zero extension:
 *   out[r][co][j] = bias[co] + sum_{ci < cin, t < K} w(co, ci, t) in[r][ci][j + t - pad]
 * with w(co, ci, t) = weight[(co*cin + ci)*K + t], or with FDK_CONV_TRANSPOSE
 * w(co, ci, t) = weight[(ci*cout + co)*K + K-1-t]: the adjoint of the
 * convolution from `cout` to `cin` channels whose weight is `weight`, when
 * called with pad = K-1-(that convolution's pad).  bias may be NULL.
 * Limits: K <= 32 and cout <= 64, or cin = cout = 1 and K <= 8191.
 */
int fdk_conv_rows(float* out, const float* in, const float* weight, const float* bias, int rows,
                  int W, int cin, int cout, int K, int pad, int flags, void* stream);

/* Bytes of workspace fdk_conv_rows_wgrad needs for these sizes. */
size_t fdk_conv_rows_wgrad_workspace(int cin, int cout, int K);

/*
 * fdk_conv_rows_wgrad - gradients of fdk_conv_rows (forward, no ReLU) with
 * respect to its weight and bias, given dout = dL/dout:
 *   dweight[(co*cin + ci)*K + t] = sum_r sum_j dout[r][co][j] in[r][ci][j + t - pad]
 *   dbias[co] = sum_r sum_j dout[r][co][j]                 (dbias may be NULL)
 * Accumulated in FP64 in a fixed order (deterministic), stored FP32.
 * workspace: device memory of at least fdk_conv_rows_wgrad_workspace() bytes.
 */
int fdk_conv_rows_wgrad(float* dweight, float* dbias, const float* dout, const float* in, int rows,
                        int W, int cin, int cout, int K, int pad, void* workspace,
                        size_t workspace_bytes, void* stream);

/* y[g][i] = x[g][i] * scale[g] (+ y[g][i] with accumulate != 0), i < group_len;
   scale is device float[groups].  y may equal x. */
int fdk_scale_groups(float* y, const float* x, const float* scale, size_t group_len, int groups,
                     int accumulate, void* stream);

/* out[g] = sum_i a[g][i] * b[g][i] (FP64 accumulation), device float[groups]. */
int fdk_group_dot(float* out, const float* a, const float* b, size_t group_len, int groups,
                  void* stream);

/* dx = dy where y > 0 else 0 (ReLU backward; y is the ReLU's output). */
int fdk_relu_backward(float* dx, const float* dy, const float* y, size_t n, void* stream);

/* y = A x, or y = A^T x with transpose != 0; A device float[rows][cols]. */
int fdk_matvec(float* y, const float* A, const float* x, int rows, int cols, int transpose,
               void* stream);

/* One Adam step (Kingma and Ba, 2015, with bias correction; step >= 1):
   m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2; p -= lr m^ / (sqrt(v^) + eps). */
int fdk_adam(float* param, float* m, float* v, const float* grad, int n, float lr, float beta1,
             float beta2, float eps, int step, void* stream);

/* Mean squared error: loss[0] = mean((a - b)^2) (device float), and, if grad
   is not NULL, grad = 2 (a - b) / n.  workspace: >= 8192 bytes of device memory. */
int fdk_mse(float* grad, float* loss, const float* a, const float* b, size_t n, void* workspace,
            size_t workspace_bytes, void* stream);

/*
 * fdk_update_probe - the paper's update benchmark a[i] = s * a[i]
 * (Section 2) over n floats of device memory, used to measure the
 * achievable HBM bandwidth and to scale memory counters.
 */
int fdk_update_probe(float* a, size_t n, float s, void* stream);

/*
 * Timing of the library's main kernels themselves.  After
 * fdk_profile_begin(), every launch of the backprojection, forward
 * projection, pre-filter and row-convolution kernels is bracketed by HIP
 * events on its stream; fdk_profile_end() waits for them and returns the
 * summed kernel milliseconds and the launch count, then stops timing.
 * Process-wide: launches from every host thread between the two calls
 * count (a training framework may run the backward pass on a thread of its
 * own).  Launches enqueued while fdk_profile_begin or fdk_profile_end runs
 * on another thread may or may not be counted.
 */
int fdk_profile_begin(void);
int fdk_profile_end(double* kernel_ms, int* launches);

/* Views per launch of the fused backprojection and the forward projection
   (1..1024, default 64; the staging buffer holds that many views, or twice
   as many when a call stages on the second stream, up to 8 GiB per batch);
   0 reads it back.  The plain kernel takes at most 64 per launch. */
int fdk_set_batch(int views_per_pass);

/*
 * Staged-plane layout of the fused backprojection (a tuning knob; every
 * layout computes the same interpolation, Section 3.2 part 3, and results
 * differ only by rounding).  Element (r, c) of a zero-padded staged plane
 * holds, with p(r, c) the padded view's pixel:
 *   FDK_LAYOUT_ROWS   p(r, c)                                (two loads per sample)
 *   FDK_LAYOUT_PAIRS  p(r, c), p(r+1, c)                     (one load)
 *   FDK_LAYOUT_QUADS  p(r, c), p(r, c+1), p(r+1, c), p(r+1, c+1)
 *   FDK_LAYOUT_DPAIRS p(r, c), p(r+1, c) - p(r, c)
 *   FDK_LAYOUT_DQUADS p00, p10 - p00, p01 - p00, (p11 - p01) - (p10 - p00)
 * (differences rounded to the storage type).  Applies to calls made after
 * it (default FDK_LAYOUT_DPAIRS); -1 reads the current layout back.  Returns the layout or a negative
 * error code (FDK_ERR_INVALID_ARG for an unknown layout).  The environment
 * variable FDK_LAYOUT=rows|pairs|quads|dpairs|dquads sets the initial value.
 */
#define FDK_LAYOUT_ROWS 0
#define FDK_LAYOUT_PAIRS 1
#define FDK_LAYOUT_QUADS 2
#define FDK_LAYOUT_DPAIRS 3
#define FDK_LAYOUT_DQUADS 4
int fdk_set_layout(int layout);

/*
 * Reciprocal of the fused backprojection's part 1 (the divide variants of
 * the paper's accuracy study, Section 7.2).  Per voxel and view, u and v
 * are the anchored numerators divided by w, and the weight is 1/w^2:
 *   FDK_DIVIDE_RCP     r = v_rcp_f32(w) (about 1 ulp), u = num_u r, v = num_v r,
 *                      weight r^2 (the default)
 *   FDK_DIVIDE_RCP_NR  as RCP, r refined by one Newton-Raphson step
 *                      r += r (1 - w r)
 *   FDK_DIVIDE_IEEE    u = num_u / w, v = num_v / w, r = 1 / w, correctly
 *                      rounded divisions (the paper's divps variant)
 *   FDK_DIVIDE_RCP12   r truncated to 12 significant bits, a stand-in for the
 *                      paper's approximate rcpps (relative error < 2^-11)
 * Non-default variants are built for the default layout (FDK_LAYOUT_DPAIRS)
 * only; a fused call in another layout then fails with FDK_ERR_UNSUPPORTED.
 * Applies to calls made after it; -1 reads the setting back.  Returns the
 * setting or FDK_ERR_INVALID_ARG.
 */
#define FDK_DIVIDE_RCP 0
#define FDK_DIVIDE_RCP_NR 1
#define FDK_DIVIDE_IEEE 2
#define FDK_DIVIDE_RCP12 3
int fdk_set_divide(int mode);

/*
 * Row clamping of the fused backprojection's taps (a tuning knob; results
 * are bit-identical either way).  A voxel's tap row outside the staged
 * plane contributes zero (the zero-padded projections of Section 3.3).
 * With 1 every tap row is clamped into the plane's zero border.  With 0
 * (the default) a launch of FP16 or BF16 storage in a single-load layout
 * (not FDK_LAYOUT_ROWS) whose voxels all have w > 0 and tap rows within a
 * bound the host derives from the plane's pitch (so that a 32-bit byte
 * offset cannot wrap) leaves such rows unclamped: their offsets fall
 * outside the plane's buffer range and the loads return zero without
 * touching memory; other launches, and FP32 storage (faster clamped),
 * clamp.  -1 reads the setting back.  Returns the setting or
 * FDK_ERR_INVALID_ARG.  The environment variable FDK_ROWS_FREE=0 sets the
 * initial value to 1.
 */
int fdk_set_row_clamp(int mode);

/* Frees the library's staging buffers (waits for their last users). */
int fdk_release(void);

/* Message for the last failed call on this thread ("" if none). */
const char* fdk_last_error(void);

/* ABI version: (major << 16) | minor. */
int fdk_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FDK_H */
