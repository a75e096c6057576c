// Host side of the C ABI declared in include/fdk.h: argument validation,
// the FP64 matrix fold, the per-device staging buffer, kernel launches,
// timing hooks and error reporting.
#include "../../include/fdk.h"
#include "api_internal.h"
#include "fdk_internal.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <atomic>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

using namespace fdk;

namespace fdk {
namespace host {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    return fail(FDK_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

// ---- staging buffer (one per device; Staging is declared in api_internal.h) ----
std::mutex g_stage_mu;
std::unordered_map<int, Staging> g_stage;
// ---- kernel timing (process-wide: launches from every thread count, e.g.
// a framework's backward pass running on a worker thread) ----------------
struct Timing {
    std::atomic<bool> on{false};
    std::mutex mu;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
};
Timing g_timing;

int timed_begin(hipStream_t s, hipEvent_t* e0)
{
    *e0 = nullptr;
    if (!g_timing.on) return FDK_OK;
    hipError_t e = hipEventCreate(e0);
    if (e == hipSuccess) e = hipEventRecord(*e0, s);
    return e == hipSuccess ? FDK_OK : hip_fail(e, "timing event");
}

int timed_end(hipStream_t s, hipEvent_t e0)
{
    if (!e0) return FDK_OK;
    hipEvent_t e1;
    hipError_t e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(e, "timing event");
    }
    std::lock_guard<std::mutex> lock(g_timing.mu);
    g_timing.ev.emplace_back(e0, e1);
    return FDK_OK;
}


// Acquire the calling device's staging buffer with at least `bytes`, and
// order `stream` after the previous call that used it.  Caller holds the
// staging mutex.
int acquire_staging(size_t bytes, hipStream_t stream, Staging** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    Staging& st = g_stage[dev];
    if (!st.last_use) {
        e = hipEventCreateWithFlags(&st.last_use, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
        e = hipEventRecord(st.last_use, stream);
        if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    }
    if (st.bytes < bytes) {
        e = hipEventSynchronize(st.last_use);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        if (st.ptr) {
            e = hipFree(st.ptr);
            st.ptr = nullptr;
            st.bytes = 0;
            if (e != hipSuccess) return hip_fail(e, "hipFree(staging)");
        }
        e = hipMalloc(&st.ptr, bytes);
        if (e != hipSuccess) {
            st.ptr = nullptr;
            return hip_fail(e, "hipMalloc(staging)");
        }
        st.bytes = bytes;
    }
    e = hipStreamWaitEvent(stream, st.last_use, 0);
    if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
    *out = &st;
    return FDK_OK;
}

}  // namespace host
}  // namespace fdk

using namespace fdk::host;

namespace {

// views per pass of the fused paths (fdk_set_batch); 64 measured best on fdk512
constexpr int kDefaultBatch = 64;
std::atomic<int> g_batch{kDefaultBatch};

// Staged layout of the fused path (tuning knob; FDK_LAYOUT=rows|pairs|quads|
// dpairs|dquads in the environment overrides the default at load time).
int initial_layout()
{
    const char* e = std::getenv("FDK_LAYOUT");
    if (e && !std::strcmp(e, "rows")) return kRows;
    if (e && !std::strcmp(e, "pairs")) return kPairs;
    if (e && !std::strcmp(e, "quads")) return kQuads;
    if (e && !std::strcmp(e, "dpairs")) return kDPairs;
    if (e && !std::strcmp(e, "dquads")) return kDQuads;
    return kDPairs;
}
std::atomic<int> g_layout{initial_layout()};

// forward projection through LDS tiles (FDK_FP_LDS=0 in the environment
// selects direct global atomics)
int g_fp_lds = []() {
    const char* e = std::getenv("FDK_FP_LDS");
    return (e && !std::strcmp(e, "0")) ? 0 : 1;
}();
// backprojection taps of rows outside the staged plane left to the buffer's
// range check where the geometry allows it (FDK_ROWS_FREE=0 in the
// environment always clamps v)
std::atomic<int> g_rows_free = []() {
    const char* e = std::getenv("FDK_ROWS_FREE");
    return (e && !std::strcmp(e, "0")) ? 0 : 1;
}();
constexpr size_t kMaxStagingBytes = size_t(8) << 30;
// the next pass's views staged on a second stream while the current pass
// runs: by default for 16-bit storage only (fdk512, in A/B runs of one box:
// FP16 28.10 -> 27.36 ms per backprojection; FP32 32.2 ms either way, its
// passes slowed by what the staging took from them).  FDK_STAGE_OVERLAP=0
// or 1 in the environment turns it off or on for every storage type.
int g_stage_overlap = []() {
    const char* e = std::getenv("FDK_STAGE_OVERLAP");
    if (e && !std::strcmp(e, "0")) return 0;
    if (e && !std::strcmp(e, "1")) return 1;
    return -1;
}();

// The staging buffer's second stream and its events (created once per device).
int ensure_side(Staging* st)
{
    hipError_t e = hipSuccess;
    if (!st->side) e = hipStreamCreateWithFlags(&st->side, hipStreamNonBlocking);
    if (e != hipSuccess) {
        st->side = nullptr;
        return hip_fail(e, "hipStreamCreateWithFlags");
    }
    hipEvent_t* evs[5] = {&st->fork, &st->staged[0], &st->staged[1], &st->freed[0], &st->freed[1]};
    for (hipEvent_t* ev : evs) {
        if (*ev) continue;
        e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            *ev = nullptr;
            return hip_fail(e, "hipEventCreate");
        }
    }
    return FDK_OK;
}
// reciprocal variant of the fused backprojection (fdk_set_divide)
std::atomic<int> g_divide{FDK_DIVIDE_RCP};

// ---- validation -----------------------------------------------------------
int validate_common(const void* volume, int N, float voxel_size, const float* origin,
                    const void* proj, int n_views, int H, int W, const double* P)
{
    if (!volume) return fail(FDK_ERR_INVALID_ARG, "volume is NULL");
    if (N < 1 || N > 4096) return fail(FDK_ERR_INVALID_ARG, "N=%d outside [1, 4096]", N);
    if (!(std::isfinite(voxel_size) && voxel_size > 0.0f))
        return fail(FDK_ERR_INVALID_ARG, "voxel_size must be finite and > 0");
    if (!origin) return fail(FDK_ERR_INVALID_ARG, "origin is NULL");
    for (int c = 0; c < 3; ++c)
        if (!std::isfinite(origin[c])) return fail(FDK_ERR_INVALID_ARG, "origin not finite");
    if (n_views < 0) return fail(FDK_ERR_INVALID_ARG, "n_views=%d < 0", n_views);
    if (H < 1 || H > 32768 || W < 1 || W > 32768)
        return fail(FDK_ERR_INVALID_ARG, "detector %dx%d outside [1, 32768]^2", W, H);
    if (n_views == 0) return FDK_OK;
    if (!proj) return fail(FDK_ERR_INVALID_ARG, "proj_stack is NULL");
    if (!P) return fail(FDK_ERR_INVALID_ARG, "P_mats is NULL");
    for (long long i = 0; i < 12LL * n_views; ++i)
        if (!std::isfinite(P[i])) return fail(FDK_ERR_INVALID_ARG, "P_mats[%lld] not finite", i);
    return FDK_OK;
}

// ---- geometry fold (FP64, rounded once to FP32) ---------------------------
// Centred index frame: voxel index x = x' + c with c = (N-1)/2, world
// X = origin + voxel_size * x.  The integer principal point (ku, kv) is
// subtracted from the u and v rows so that u' = u - ku stays small, and
// the view's scale s folds in as 1/sqrt(s) (exact for powers of 4).
void fold_matrix(const double* P, int N, double vs, const float* origin, int ku, int kv,
                 double lambda, double Q[12])
{
    const double c = 0.5 * (N - 1);
    for (int r = 0; r < 3; ++r) {
        double t = P[4 * r + 3];
        for (int k = 0; k < 3; ++k) {
            Q[4 * r + k] = vs * P[4 * r + k] * lambda;
            t += P[4 * r + k] * ((double)origin[k] + vs * c);
        }
        Q[4 * r + 3] = t * lambda;
    }
    for (int k = 0; k < 4; ++k) {
        Q[k] -= ku * Q[8 + k];
        Q[4 + k] -= kv * Q[8 + k];
    }
}

// True if some voxel of the centred box [-c, c]^3 may have w <= 0 (or so
// close to 0 that its FP32 value could be) for this folded matrix.
bool needs_wcheck(const double Q[12], double c)
{
    double wmin = INFINITY, wmax = 0.0;
    for (int corner = 0; corner < 8; ++corner) {
        double x = (corner & 1) ? c : -c, y = (corner & 2) ? c : -c, z = (corner & 4) ? c : -c;
        double w = Q[8] * x + Q[9] * y + Q[10] * z + Q[11];
        wmin = std::fmin(wmin, w);
        wmax = std::fmax(wmax, std::fabs(w));
    }
    return !(wmin > 1e-4 * wmax);
}

// True if every voxel of the centred box [-c, c]^3 has w > 0 and |v'| <=
// vlim.  Then the tap row of each voxel, left unclamped, lies within vlim
// (plus the centring) rows of the staged plane, so its 32-bit byte offset
// cannot wrap around into the plane, and a row outside the plane reads as
// zero through the buffer's range check: the kernel may skip the clamp of v.
// (v' is a linear-fractional function of the voxel position; with w > 0 on
// the box its extremes are at the box's corners.)
bool rows_bounded(const double Q[12], double c, double vlim)
{
    double wmin = INFINITY, wmax = 0.0, vmax = 0.0;
    for (int corner = 0; corner < 8; ++corner) {
        double x = (corner & 1) ? c : -c, y = (corner & 2) ? c : -c, z = (corner & 4) ? c : -c;
        double w = Q[8] * x + Q[9] * y + Q[10] * z + Q[11];
        double vw = Q[4] * x + Q[5] * y + Q[6] * z + Q[7];
        wmin = std::fmin(wmin, w);
        wmax = std::fmax(wmax, std::fabs(w));
        vmax = std::fmax(vmax, std::fabs(vw / w));
    }
    return wmin > 1e-4 * wmax && vmax <= vlim;
}

// Unit direction from the volume centre (index frame) towards the source:
// the source is the null vector of the 3x4 matrix, the intersection of the
// planes of its three rows.
void source_direction(const double Q[12], double d[3])
{
    const double* a = Q;
    const double* b = Q + 4;
    const double* c = Q + 8;
    // homogeneous null vector by cofactors: s_k = (-1)^k det(Q without column k)
    auto det3 = [](double a0, double a1, double a2, double b0, double b1, double b2, double c0,
                   double c1, double c2) {
        return a0 * (b1 * c2 - b2 * c1) - a1 * (b0 * c2 - b2 * c0) + a2 * (b0 * c1 - b1 * c0);
    };
    const double s0 = det3(a[1], a[2], a[3], b[1], b[2], b[3], c[1], c[2], c[3]);
    const double s1 = -det3(a[0], a[2], a[3], b[0], b[2], b[3], c[0], c[2], c[3]);
    const double s2 = det3(a[0], a[1], a[3], b[0], b[1], b[3], c[0], c[1], c[3]);
    const double s3 = -det3(a[0], a[1], a[2], b[0], b[1], b[2], c[0], c[1], c[2]);
    // finite source: direction s/s3 from the centre (the origin of the frame)
    double v[3] = {s0, s1, s2};
    if (s3 != 0.0)
        for (int k = 0; k < 3; ++k) v[k] /= s3;
    const double n = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    for (int k = 0; k < 3; ++k) d[k] = n > 0.0 ? v[k] / n : 0.0;
}

int storage_size(int dtype)
{
    return dtype == FDK_DTYPE_F32 ? 4 : 2;
}

// The workgroup tiles of the batch's ray axis (A.y_fastest), the grid they
// make with A.zchunks, and whether that grid takes the XCD remap.
void set_tiles(FusedArgs& A, int N)
{
    const bool yf = A.y_fastest != 0;
    A.tiles_x = (N + tile_x(yf) - 1) / tile_x(yf);
    A.tiles_y = (N + tile_y(yf) - 1) / tile_y(yf);
    const long long blocks = (long long)A.tiles_x * A.tiles_y * A.zchunks;
    A.xcd_remap = (blocks % 8 == 0) ? 1 : 0;
}

// Launch geometry shared by the backprojection and the forward projection:
// everything in FusedArgs except the staged planes and the matrices.
void setup_args(FusedArgs& A, float* volume, int N, int H, int W, int Wp, long long plane, int zdepth)
{
    const int ku = (W - 1) / 2, kv = (H - 1) / 2;
    A.vol = volume;
    A.plane = plane;
    A.N = N;
    A.nz = N;
    A.z_first = 0;
    A.Wp = Wp;
    // u = u' + ku.  Zero contribution iff u <= -1 or u >= W (likewise v);
    // floor(u) stays in [-2, W] iff u in [-2, W + 1).  Margins of 0.5 pixel.
    A.skip_lo_u = (float)(-1 - ku) - 0.5f;
    A.skip_hi_u = (float)(W - ku) + 0.5f;
    A.skip_lo_v = (float)(-1 - kv) - 0.5f;
    A.skip_hi_v = (float)(H - kv) + 0.5f;
    A.lo_iu = -ku - kPad;
    A.hi_iu = W - ku;
    A.lo_iv = -kv - kPad;
    A.hi_iv = H - kv;
    // a pixel inside the index clamp ranges: floor(u') in [lo_iu, hi_iu]
    A.in_lo_u = (float)(A.lo_iu + 1);
    A.in_hi_u = (float)(A.hi_iu - 1);
    A.in_lo_v = (float)(A.lo_iv + 1);
    A.in_hi_v = (float)(A.hi_iv - 1);
    A.origin_off = (kv + kPad) * Wp + (ku + kPad);
    A.c = 0.5f * (float)(N - 1);
    A.zchunks = (N + zdepth - 1) / zdepth;
    set_tiles(A, N);
}

// Fold the matrices of views [v0, v0+cnt) into out (cnt x 12 floats, in
// the batch's ray frame) and outq (cnt x 12 doubles, unrounded, columns x,
// y, z, 1); returns whether some voxel may have w <= 0, sets *rows_free to
// whether every view passes rows_bounded(vlim) (vlim <= 0: never), and sets
// the workgroup order from the batch's mean ray direction.
bool fold_batch(FusedArgs& A, float* out, double* outq, const double* P, const float* view_scale,
                int v0, int cnt, int N, float voxel_size, const float* origin, int H, int W,
                double vlim, bool* rows_free)
{
    const int ku = (W - 1) / 2, kv = (H - 1) / 2;
    const double c = 0.5 * (N - 1);
    bool wcheck = false;
    *rows_free = vlim > 0.0;
    double ray[3] = {0.0, 0.0, 0.0};
    A.count = cnt;
    for (int j = 0; j < cnt; ++j) {
        double lambda = 1.0;
        if (view_scale) lambda = 1.0 / std::sqrt((double)view_scale[v0 + j]);
        double Q[12];
        fold_matrix(P + 12 * (size_t)(v0 + j), N, voxel_size, origin, ku, kv, lambda, Q);
        wcheck |= needs_wcheck(Q, c);
        if (*rows_free) *rows_free = rows_bounded(Q, c, vlim);
        for (int k = 0; k < 12; ++k) {
            out[12 * (size_t)j + k] = (float)Q[k];
            outq[12 * (size_t)j + k] = Q[k];
        }
        double d[3];
        source_direction(Q, d);
        for (int k = 0; k < 3; ++k) ray[k] += std::fabs(d[k]);
    }
    A.y_fastest = ray[1] > ray[0] ? 1 : 0;
    set_tiles(A, N);
    // The kernels take the matrices in the batch's ray frame: column 0
    // multiplies the transverse coordinate, column 1 the one along the
    // rays (the workgroup order's fastest axis).  With rays along x, swap.
    if (!A.y_fastest)
        for (int j = 0; j < cnt; ++j)
            for (int r = 0; r < 3; ++r)
                std::swap(out[12 * (size_t)j + 4 * r], out[12 * (size_t)j + 4 * r + 1]);
    return wcheck;
}

// Per-batch launch parameters of a call, with every view's folded matrix
// copied to the device (at `dev`, inside the staging buffer, so the
// staging buffer's ordering protects it).
struct Batches {
    std::vector<int> v0, count, wcheck, rows_free, y_fastest;
};

// Device (and pinned host) matrix region of a call: n_views x 12 floats,
// then n_views x 12 doubles.
constexpr size_t kMatBytesPerView = 12 * sizeof(float) + 12 * sizeof(double);

int fold_and_upload(Staging* st, float* dev, const double* P, const float* view_scale,
                    int n_views, int batch, int N, float voxel_size, const float* origin, int H,
                    int W, double vlim, hipStream_t stream, Batches* B)
{
    hipError_t e;
    const size_t floats = kMatBytesPerView / sizeof(float) * (size_t)n_views;
    if (!st->mats_copied) {
        e = hipEventCreateWithFlags(&st->mats_copied, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    } else {
        // the previous call's copy must have read the pinned buffer
        e = hipEventSynchronize(st->mats_copied);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    }
    if (st->host_floats < floats) {
        if (st->host_mats) {
            e = hipHostFree(st->host_mats);
            st->host_mats = nullptr;
            st->host_floats = 0;
            if (e != hipSuccess) return hip_fail(e, "hipHostFree");
        }
        e = hipHostMalloc((void**)&st->host_mats, floats * sizeof(float), hipHostMallocDefault);
        if (e != hipSuccess) {
            st->host_mats = nullptr;
            return hip_fail(e, "hipHostMalloc");
        }
        st->host_floats = floats;
    }
    FusedArgs A = {};
    for (int v0 = 0; v0 < n_views; v0 += batch) {
        const int cnt = std::min(batch, n_views - v0);
        bool rows_free = false;
        double* hq = (double*)(st->host_mats + 12 * (size_t)n_views);
        const bool wcheck = fold_batch(A, st->host_mats + 12 * (size_t)v0, hq + 12 * (size_t)v0, P,
                                       view_scale, v0, cnt, N, voxel_size, origin, H, W, vlim,
                                       &rows_free);
        B->v0.push_back(v0);
        B->count.push_back(cnt);
        B->wcheck.push_back(wcheck ? 1 : 0);
        B->rows_free.push_back(rows_free && !wcheck ? 1 : 0);
        B->y_fastest.push_back(A.y_fastest);
    }
    e = hipMemcpyAsync(dev, st->host_mats, floats * sizeof(float), hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return hip_fail(e, "matrix copy");
    e = hipEventRecord(st->mats_copied, stream);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    return FDK_OK;
}

// bytes of `n` views' planes rounded up for the matrices that follow them
size_t planes_region(size_t n, size_t plane_bytes)
{
    return (n * plane_bytes + 255) & ~size_t(255);
}

// Staged-plane geometry of a fused backprojection call.
struct FusedPlan {
    int Hp, Wp, layout, divide;
    size_t esz, elem, plane_bytes;
    double vlim;  // bound on |v'| for unclamped rows (0: always clamp)
};

int plan_fused(int dtype, int H, int W, FusedPlan* F)
{
    F->Hp = H + 2 * kPad;
    F->Wp = ((W + 2 * kPad + 63) / 64) * 64;
    F->esz = storage_size(dtype);
    F->layout = g_layout;
    F->elem = F->esz * layout_width(F->layout);
    F->plane_bytes = (size_t)F->Hp * F->Wp * F->elem;
    if (F->plane_bytes >= (size_t(1) << 31))
        return fail(FDK_ERR_UNSUPPORTED, "staged view of %zu bytes exceeds 2 GiB",
                    F->plane_bytes);
    // Rows outside the staged plane may be left to the buffer's range check
    // (no clamp of v) when a tap row R satisfies |R| * Wp * elem < 2^31, so
    // that its byte offset lands outside [0, plane_bytes) without wrapping:
    // bound |v'| by a quarter of that, less the centring.  Only 16-bit
    // storage, with one load per tap pair (not the rows layout, whose second
    // load adds an offset): on fdk512 the unclamped FP16 kernel took 30.9
    // against 31.5 ms, while the FP32 one, whatever the load schedule, was
    // 2-15 % slower than with the clamp.
    F->divide = g_divide;
    if (F->divide != FDK_DIVIDE_RCP && F->layout != kDPairs)
        return fail(FDK_ERR_UNSUPPORTED,
                    "divide variant %d is built for the dpairs layout only (layout %d)",
                    F->divide, F->layout);
    F->vlim = (F->layout == kRows || dtype == FDK_DTYPE_F32)
                  ? 0.0
                  : 0.25 * 2147483648.0 / ((double)F->Wp * (double)F->elem) -
                        (double)((H - 1) / 2 + kPad + 2);
    return FDK_OK;
}

int run_fused_batches(FusedArgs& A, const FusedPlan& F, Staging* st, hipStream_t stage_stream,
                      hipStream_t stream, bool overlap, size_t planes, float* mats,
                      const double* matsq, const double* P, const float* view_scale,
                      const void* proj, int dtype, int n_views, int batch, int N,
                      float voxel_size, const float* origin, int H, int W);

int run_fused(float* volume, int N, float voxel_size, const float* origin, const void* proj,
              int dtype, int n_views, int H, int W, const double* P, const float* view_scale,
              hipStream_t stream)
{
    FusedPlan F;
    int rc = plan_fused(dtype, H, W, &F);
    if (rc != FDK_OK) return rc;
    const int Hp = F.Hp, Wp = F.Wp;
    const size_t esz = F.esz, plane_bytes = F.plane_bytes;
    int batch = g_batch;
    if ((size_t)batch * plane_bytes > kMaxStagingBytes)
        batch = (int)std::max<size_t>(1, kMaxStagingBytes / plane_bytes);
    batch = std::min(batch, n_views);

    FusedArgs A = {};
    setup_args(A, volume, N, H, W, Wp, (long long)Hp * Wp, fused_z(dtype));

    // With more than one pass the buffer holds two halves of `batch` planes:
    // pass b reads half b % 2 while the side stream stages pass b + 1 into
    // the other half, once pass b - 1 (its previous reader) has finished.
    // The staging is HBM-bound and the passes are ALU-bound, so the two can
    // share the chip.  Every kernel of the call stays ordered after the
    // caller's earlier work on `stream` (the side stream waits for `fork`),
    // and the call's last kernel, on `stream`, follows every staging.
    const bool overlap =
        n_views > batch && (g_stage_overlap == 1 || (g_stage_overlap == -1 && esz == 2));
    std::lock_guard<std::mutex> lock(g_stage_mu);
    Staging* st = nullptr;
    const size_t planes = planes_region(batch, plane_bytes);
    const size_t halves = overlap ? 2 * planes : planes;
    rc = acquire_staging(halves + kMatBytesPerView * (size_t)n_views, stream, &st);
    if (rc != FDK_OK) return rc;
    float* mats = (float*)((char*)st->ptr + halves);
    const double* matsq = (const double*)(mats + 12 * (size_t)n_views);
    hipStream_t stage_stream = stream;
    if (overlap) {
        if ((rc = ensure_side(st)) != FDK_OK) return rc;
        hipError_t e = hipEventRecord(st->fork, stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(st->side, st->fork, 0);
        if (e != hipSuccess) return hip_fail(e, "stream fork");
        stage_stream = st->side;
    }
    rc = run_fused_batches(A, F, st, stage_stream, stream, overlap, planes, mats, matsq, P,
                           view_scale, proj, dtype, n_views, batch, N, voxel_size, origin, H, W);
    hipError_t e = hipSuccess;
    if (overlap) {
        // join the side stream back, also after a failure part-way, so that
        // later users of the buffer on `stream` follow every staging
        e = hipEventRecord(st->staged[0], stage_stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(stream, st->staged[0], 0);
        if (e != hipSuccess && rc == FDK_OK) rc = hip_fail(e, "stream join");
    }
    e = hipEventRecord(st->last_use, stream);
    if (e != hipSuccess && rc == FDK_OK) rc = hip_fail(e, "hipEventRecord");
    return rc;
}

// The passes of run_fused: fold and upload the matrices, then per pass
// stage its views (on `stage_stream`) and launch the backprojection.
int run_fused_batches(FusedArgs& A, const FusedPlan& F, Staging* st, hipStream_t stage_stream,
                      hipStream_t stream, bool overlap, size_t planes, float* mats,
                      const double* matsq, const double* P, const float* view_scale,
                      const void* proj, int dtype, int n_views, int batch, int N,
                      float voxel_size, const float* origin, int H, int W)
{
    const int Hp = F.Hp, Wp = F.Wp, layout = F.layout;
    const size_t esz = F.esz;
    Batches B;
    int rc = fold_and_upload(st, mats, P, view_scale, n_views, batch, N, voxel_size, origin, H,
                             W, F.vlim, stream, &B);
    if (rc != FDK_OK) return rc;

    for (size_t b = 0; b < B.v0.size(); ++b) {
        const int v0 = B.v0[b], cnt = B.count[b];
        const int half = overlap ? (int)(b & 1) : 0;
        char* img = (char*)st->ptr + (size_t)half * planes;
        hipError_t e = hipSuccess;
        if (overlap && b >= 2) e = hipStreamWaitEvent(stage_stream, st->freed[half], 0);
        if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
        StageArgs S;
        S.src = (const char*)proj + (size_t)v0 * H * W * esz;
        S.dst = img;
        S.H = H;
        S.W = W;
        S.Hp = Hp;
        S.Wp = Wp;
        S.count = cnt;
        S.layout = layout;
        e = launch_stage(S, dtype, stage_stream);
        if (e != hipSuccess) return hip_fail(e, "stage launch");
        if (overlap) {
            e = hipEventRecord(st->staged[half], stage_stream);
            if (e == hipSuccess) e = hipStreamWaitEvent(stream, st->staged[half], 0);
            if (e != hipSuccess) return hip_fail(e, "stream join");
        }
        A.img = img;
        A.count = cnt;
        A.m = mats + 12 * (size_t)v0;
        A.mq = matsq + 12 * (size_t)v0;
        A.y_fastest = B.y_fastest[b];
        set_tiles(A, N);
        hipEvent_t t0;
        if ((rc = timed_begin(stream, &t0)) != FDK_OK) return rc;
        e = launch_fused(A, dtype, layout, B.wcheck[b] != 0, g_rows_free && B.rows_free[b] != 0,
                         F.divide, stream);
        if (e != hipSuccess) return hip_fail(e, "backprojection launch");
        if ((rc = timed_end(stream, t0)) != FDK_OK) return rc;
        if (overlap) {
            e = hipEventRecord(st->freed[half], stream);
            if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
        }
    }
    return FDK_OK;
}

// ---- allocation-free backprojection: one fixed scratch array per device ----
// Holds a pass's staged planes followed by its folded matrices.  Every call
// of fdk_backproject_noalloc on a device shares that device's copy.
constexpr int kMaxDevices = 64;
constexpr int kNoallocMaxBatch = 64;  // views per pass (host-side matrix arrays below)
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

}  // namespace

static __device__ __align__(256) unsigned char scratch[FDK_NOALLOC_SCRATCH_BYTES];

namespace {

// The calling device's copy of `scratch`: its address is looked up once per
// device (with that device current) and kept; host code uses that address,
// never the array's name, which on the host is only a stand-in.
int scratch_address(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return fail(FDK_ERR_UNSUPPORTED, "device %d beyond the %d the scratch table holds", dev,
                    kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(FDK_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return FDK_OK;
}

// The fused backprojection with the staged planes and matrices of each
// pass in the device's scratch array: no allocation, no pinned copy (the
// matrices travel in a kernel's arguments), no library events.
int run_fused_noalloc(float* volume, int N, float voxel_size, const float* origin,
                      const void* proj, int dtype, int n_views, int H, int W, const double* P,
                      const float* view_scale, hipStream_t stream)
{
    FusedPlan F;
    int rc = plan_fused(dtype, H, W, &F);
    if (rc != FDK_OK) return rc;
    const size_t bytes = FDK_NOALLOC_SCRATCH_BYTES;
    // views per pass: as many planes as fit with their matrices, at most
    // the configured batch and what one matrix upload carries
    int batch = std::min(std::min((int)g_batch, kNoallocMaxBatch), n_views);
    while (batch > 0 &&
           planes_region(batch, F.plane_bytes) + kMatBytesPerView * (size_t)batch > bytes)
        --batch;
    if (batch < 1)
        return fail(FDK_ERR_UNSUPPORTED,
                    "a staged view of %zu bytes does not fit the %zu-byte scratch array",
                    F.plane_bytes, bytes);
    void* base = nullptr;
    rc = scratch_address(&base);
    if (rc != FDK_OK) return rc;

    FusedArgs A = {};
    setup_args(A, volume, N, H, W, F.Wp, (long long)F.Hp * F.Wp, fused_z(dtype));
    A.img = base;
    float* mats = (float*)((char*)base + planes_region(batch, F.plane_bytes));
    double* matsq = (double*)(mats + 12 * (size_t)batch);
    float hm[kNoallocMaxBatch * 12];
    double hq[kNoallocMaxBatch * 12];
    PutMatsArgs M;
    for (int v0 = 0; v0 < n_views; v0 += batch) {
        const int cnt = std::min(batch, n_views - v0);
        bool rows_free = false;
        const bool wcheck = fold_batch(A, hm, hq, P, view_scale, v0, cnt, N, voxel_size, origin,
                                       H, W, F.vlim, &rows_free);
        hipError_t e;
        for (int k0 = 0; k0 < cnt; k0 += kPutMatsMax) {
            M.count = std::min(kPutMatsMax, cnt - k0);
            M.dst = mats + 12 * (size_t)k0;
            M.dstq = matsq + 12 * (size_t)k0;
            std::memcpy(M.m, hm + 12 * k0, sizeof(float) * 12 * M.count);
            std::memcpy(M.q, hq + 12 * k0, sizeof(double) * 12 * M.count);
            e = launch_put_mats(M, stream);
            if (e != hipSuccess) return hip_fail(e, "matrix upload launch");
        }
        StageArgs S;
        S.src = (const char*)proj + (size_t)v0 * H * W * F.esz;
        S.dst = base;
        S.H = H;
        S.W = W;
        S.Hp = F.Hp;
        S.Wp = F.Wp;
        S.count = cnt;
        S.layout = F.layout;
        e = launch_stage(S, dtype, stream);
        if (e != hipSuccess) return hip_fail(e, "stage launch");
        A.count = cnt;
        A.m = mats;
        A.mq = matsq;
        e = launch_fused(A, dtype, F.layout, wcheck, g_rows_free && rows_free && !wcheck,
                         F.divide, stream);
        if (e != hipSuccess) return hip_fail(e, "backprojection launch");
    }
    return FDK_OK;
}

// LDS tile of the forward projection: the largest detector footprint (with
// the kernel's margins) of a workgroup box (16 voxels across the rays, 32
// along them, 16 in z; `mats` are in the batch's ray frame) at the volume's
// corners or centre over the batch's views, rounded up to a multiple of 512
// in [8192, 32768] entries (32-128 KiB).  Boxes with a larger footprint
// fall back to global atomics in the kernel.  (Sized to the footprint
// rather than to a power of two: fdk256x8's 8547 entries fit 36 KiB, and
// three workgroups a CU, instead of 64 KiB and two.)
int fp_tile_entries(const float* mats, int cnt, int N)
{
    const double c = 0.5 * (N - 1);
    const double e = std::min(15.0, (double)(N - 1));   // across the rays and in z
    const double er = std::min(31.0, (double)(N - 1));  // along the rays
    double worst = 0.0;
    for (int j = 0; j < cnt; ++j) {
        const float* q = mats + 12 * (size_t)j;
        for (int b = 0; b < 9; ++b) {
            // box origin: a volume corner (b < 8) or the centre
            const double bx = b == 8 ? -0.5 * e : ((b & 1) ? c - e : -c);
            const double by = b == 8 ? -0.5 * er : ((b & 2) ? c - er : -c);
            const double bz = b == 8 ? -0.5 * e : ((b & 4) ? c - e : -c);
            double umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
            bool ok = true;
            for (int k = 0; k < 8; ++k) {
                const double x = bx + ((k & 1) ? e : 0), y = by + ((k & 2) ? er : 0),
                             z = bz + ((k & 4) ? e : 0);
                const double w = q[8] * x + q[9] * y + q[10] * z + q[11];
                if (!(w > 0.0)) ok = false;
                const double u = (q[0] * x + q[1] * y + q[2] * z + q[3]) / w;
                const double v = (q[4] * x + q[5] * y + q[6] * z + q[7]) / w;
                umin = std::min(umin, u);
                umax = std::max(umax, u);
                vmin = std::min(vmin, v);
                vmax = std::max(vmax, v);
            }
            if (!ok) continue;
            const double area = (std::floor(umax) - std::floor(umin) + 4.0) *
                                (std::floor(vmax) - std::floor(vmin) + 4.0);
            worst = std::max(worst, area);
        }
    }
    return (int)std::min(32768.0, std::max(8192.0, std::ceil(worst / 512.0) * 512.0));
}

// The largest 1/w^2 over the centred box [-c, c]^3 (w is affine: its
// minimum is at a corner) for the folded FP64 matrices of `cnt` views, with
// a small margin; 0 if w may be <= 0 somewhere.
float batch_rmax2(const double* Q, int cnt, int N)
{
    const double c = 0.5 * (N - 1);
    double wmin = INFINITY;
    for (int j = 0; j < cnt; ++j)
        for (int corner = 0; corner < 8; ++corner) {
            const double x = (corner & 1) ? c : -c, y = (corner & 2) ? c : -c,
                         z = (corner & 4) ? c : -c;
            const double* q = Q + 12 * (size_t)j;
            wmin = std::fmin(wmin, q[8] * x + q[9] * y + q[10] * z + q[11]);
        }
    if (!(wmin > 0.0)) return 0.0f;
    return (float)(1.0 / (wmin * wmin) * (1.0 + 1e-5));
}

int run_forward(float* proj, int n_views, int H, int W, const double* P, const float* volume,
                int N, float voxel_size, const float* origin, hipStream_t stream)
{
    const int Hp = H + 2 * kPad;
    const int Wp = ((W + 2 * kPad + 63) / 64) * 64;
    // 64-bit fixed-point sums (float in batches that need the w check)
    const size_t plane_bytes = (size_t)Hp * Wp * 8;
    if (plane_bytes >= (size_t(1) << 31))
        return fail(FDK_ERR_UNSUPPORTED, "padded view of %zu bytes exceeds 2 GiB", plane_bytes);
    int batch = g_batch;
    if ((size_t)batch * plane_bytes > kMaxStagingBytes)
        batch = (int)std::max<size_t>(1, kMaxStagingBytes / plane_bytes);
    batch = std::min(batch, n_views);

    FusedArgs A = {};
    setup_args(A, const_cast<float*>(volume), N, H, W, Wp, (long long)Hp * Wp, kFpZ);

    std::lock_guard<std::mutex> lock(g_stage_mu);
    Staging* st = nullptr;
    // planes, then 256 bytes for the volume's largest |x|, then the matrices
    const size_t planes = planes_region(batch, plane_bytes);
    int rc = acquire_staging(planes + 256 + kMatBytesPerView * (size_t)n_views, stream, &st);
    if (rc != FDK_OK) return rc;
    A.acc64 = (unsigned long long*)st->ptr;
    unsigned* vmax = (unsigned*)((char*)st->ptr + planes);
    float* mats = (float*)((char*)st->ptr + planes + 256);
    const double* matsq = (const double*)(mats + 12 * (size_t)n_views);
    Batches B;
    rc = fold_and_upload(st, mats, P, nullptr, n_views, batch, N, voxel_size, origin, H, W, 0.0,
                         stream, &B);
    if (rc != FDK_OK) return rc;
    const double* host_q = (const double*)(st->host_mats + 12 * (size_t)n_views);
    hipError_t e = launch_zero((float*)vmax, 4, stream);
    if (e == hipSuccess) e = launch_fp_vmax(volume, (size_t)N * N * N, vmax, stream);
    if (e != hipSuccess) return hip_fail(e, "volume maximum launch");
    A.fp_vmax = vmax;

    for (size_t b = 0; b < B.v0.size(); ++b) {
        const int v0 = B.v0[b], cnt = B.count[b];
        e = launch_zero((float*)st->ptr, (size_t)cnt * Hp * Wp * 2, stream);
        if (e != hipSuccess) return hip_fail(e, "zero launch");
        A.count = cnt;
        A.m = mats + 12 * (size_t)v0;
        A.mq = matsq + 12 * (size_t)v0;
        A.y_fastest = B.y_fastest[b];
        set_tiles(A, N);
        const bool wcheck = B.wcheck[b] != 0;
        A.fp_rmax2 = wcheck ? 0.0f : batch_rmax2(host_q + 12 * (size_t)v0, cnt, N);
        hipEvent_t t0;
        if ((rc = timed_begin(stream, &t0)) != FDK_OK) return rc;
        if (wcheck || !g_fp_lds) {
            e = launch_scatter(A, wcheck, stream);
        } else {
            FusedArgs C = A;  // column tiles of 16 across the rays x 32 along them
            C.fp_tile = fp_tile_entries(st->host_mats + 12 * (size_t)v0, cnt, N);
            C.tiles_x = C.y_fastest ? (N + 15) / 16 : (N + 31) / 32;
            C.tiles_y = C.y_fastest ? (N + 31) / 32 : (N + 15) / 16;
            const long long blocks = (long long)C.tiles_x * C.tiles_y * C.zchunks;
            C.xcd_remap = (blocks % 8 == 0) ? 1 : 0;
            // each box's views split over up to 4 workgroups of >= 16 views:
            // more workgroups in flight where only the phantom's boxes work
            // (fdk256x8: 949 of 4096 boxes; 1 part 3.21, 2 parts 3.10, 4
            // parts 3.08, 8 parts 3.28 ms per projection)
            C.fp_vparts = std::max(1, std::min(4, (cnt + 15) / 16));
            e = launch_scatter_lds(C, stream);
        }
        if (e != hipSuccess) return hip_fail(e, "forward projection launch");
        if ((rc = timed_end(stream, t0)) != FDK_OK) return rc;
        UnstageArgs U;
        U.planes = (const unsigned long long*)st->ptr;
        U.dst = proj + (size_t)v0 * H * W;
        U.H = H;
        U.W = W;
        U.Hp = Hp;
        U.Wp = Wp;
        U.count = cnt;
        U.fixed = wcheck ? 0 : 1;
        U.N = N;
        U.vmax = vmax;
        U.rmax2 = A.fp_rmax2;
        e = launch_unstage_add(U, stream);
        if (e != hipSuccess) return hip_fail(e, "unstage launch");
    }
    e = hipEventRecord(st->last_use, stream);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    return FDK_OK;
}

int run_plain(float* volume, int N, float voxel_size, const float* origin, const float* proj,
              int n_views, int H, int W, const double* P, hipStream_t stream)
{
    PlainArgs A = {};
    A.vol = volume;
    A.N = N;
    A.H = H;
    A.W = W;
    A.ox = origin[0];
    A.oy = origin[1];
    A.oz = origin[2];
    A.vs = voxel_size;
    const int batch = std::min(std::min(g_batch.load(), kPlainBatch), n_views);
    for (int v0 = 0; v0 < n_views; v0 += batch) {
        const int cnt = std::min(batch, n_views - v0);
        A.proj = proj + (size_t)v0 * H * W;
        A.count = cnt;
        for (int j = 0; j < cnt; ++j)
            for (int k = 0; k < 12; ++k) A.m[j][k] = (float)P[12 * (size_t)(v0 + j) + k];
        hipEvent_t t0;
        int rc;
        if ((rc = timed_begin(stream, &t0)) != FDK_OK) return rc;
        hipError_t e = launch_plain(A, stream);
        if (e != hipSuccess) return hip_fail(e, "plain backprojection launch");
        if ((rc = timed_end(stream, t0)) != FDK_OK) return rc;
    }
    return FDK_OK;
}

}  // namespace

// ===========================================================================
extern "C" {

int fdk_backproject_ex(float* volume, int N, float voxel_size, const float origin[3],
                       const void* proj_stack, int proj_dtype, int n_views, int H, int W,
                       const double* P_mats, const float* view_scale, int flags, void* stream)
{
    g_err.clear();
    int rc = validate_common(volume, N, voxel_size, origin, proj_stack, n_views, H, W, P_mats);
    if (rc != FDK_OK || n_views == 0) return rc;
    if (proj_dtype != FDK_DTYPE_F32 && proj_dtype != FDK_DTYPE_F16 && proj_dtype != FDK_DTYPE_BF16)
        return fail(FDK_ERR_INVALID_ARG, "unknown proj_dtype %d", proj_dtype);
    if (view_scale)
        for (int i = 0; i < n_views; ++i)
            if (!(std::isfinite(view_scale[i]) && view_scale[i] > 0.0f))
                return fail(FDK_ERR_INVALID_ARG, "view_scale[%d] must be finite and > 0", i);
    hipStream_t s = (hipStream_t)stream;
    if (flags == FDK_KERNEL_PLAIN) {
        if (proj_dtype != FDK_DTYPE_F32 || view_scale)
            return fail(FDK_ERR_UNSUPPORTED, "the plain kernel takes FP32 and no view_scale");
        return run_plain(volume, N, voxel_size, origin, (const float*)proj_stack, n_views, H, W,
                         P_mats, s);
    }
    if (flags != FDK_KERNEL_FUSED) return fail(FDK_ERR_INVALID_ARG, "unknown flags %d", flags);
    return run_fused(volume, N, voxel_size, origin, proj_stack, proj_dtype, n_views, H, W, P_mats,
                     view_scale, s);
}

int fdk_backproject(float* volume, int N, float voxel_size, const float origin[3],
                    const float* proj_stack, int n_views, int H, int W, const double* P_mats,
                    void* stream)
{
    return fdk_backproject_ex(volume, N, voxel_size, origin, proj_stack, FDK_DTYPE_F32, n_views,
                              H, W, P_mats, nullptr, FDK_KERNEL_FUSED, stream);
}

int fdk_backproject_noalloc(float* volume, int N, float voxel_size, const float origin[3],
                            const void* proj_stack, int proj_dtype, int n_views, int H, int W,
                            const double* P_mats, const float* view_scale, void* stream)
{
    g_err.clear();
    int rc = validate_common(volume, N, voxel_size, origin, proj_stack, n_views, H, W, P_mats);
    if (rc != FDK_OK || n_views == 0) return rc;
    if (proj_dtype != FDK_DTYPE_F32 && proj_dtype != FDK_DTYPE_F16 && proj_dtype != FDK_DTYPE_BF16)
        return fail(FDK_ERR_INVALID_ARG, "unknown proj_dtype %d", proj_dtype);
    if (view_scale)
        for (int i = 0; i < n_views; ++i)
            if (!(std::isfinite(view_scale[i]) && view_scale[i] > 0.0f))
                return fail(FDK_ERR_INVALID_ARG, "view_scale[%d] must be finite and > 0", i);
    return run_fused_noalloc(volume, N, voxel_size, origin, proj_stack, proj_dtype, n_views, H,
                             W, P_mats, view_scale, (hipStream_t)stream);
}

int fdk_backproject_plain(float* volume, int N, float voxel_size, const float origin[3],
                          const float* proj_stack, int n_views, int H, int W,
                          const double* P_mats, void* stream)
{
    return fdk_backproject_ex(volume, N, voxel_size, origin, proj_stack, FDK_DTYPE_F32, n_views,
                              H, W, P_mats, nullptr, FDK_KERNEL_PLAIN, stream);
}

int fdk_forward_project(float* proj_stack, int n_views, int H, int W, const double* P_mats,
                        const float* volume, int N, float voxel_size, const float origin[3],
                        void* stream)
{
    g_err.clear();
    if (!proj_stack && n_views > 0) return fail(FDK_ERR_INVALID_ARG, "proj_stack is NULL");
    int rc = validate_common(volume, N, voxel_size, origin, proj_stack, n_views, H, W, P_mats);
    if (rc != FDK_OK || n_views == 0) return rc;
    return run_forward(proj_stack, n_views, H, W, P_mats, volume, N, voxel_size, origin,
                       (hipStream_t)stream);
}

int fdk_convert_storage(void* dst, const float* src, int n_views, int H, int W, int dtype,
                        float* view_scale, void* stream)
{
    g_err.clear();
    if (n_views < 0) return fail(FDK_ERR_INVALID_ARG, "n_views=%d < 0", n_views);
    if (H < 1 || H > 32768 || W < 1 || W > 32768)
        return fail(FDK_ERR_INVALID_ARG, "detector %dx%d outside [1, 32768]^2", W, H);
    if (dtype != FDK_DTYPE_F16 && dtype != FDK_DTYPE_BF16)
        return fail(FDK_ERR_INVALID_ARG, "dtype %d is not FDK_DTYPE_F16 or FDK_DTYPE_BF16", dtype);
    if (n_views == 0) return FDK_OK;
    if (!dst || !src) return fail(FDK_ERR_INVALID_ARG, "dst or src is NULL");
    if (dtype == FDK_DTYPE_F16 && !view_scale)
        return fail(FDK_ERR_INVALID_ARG, "FP16 storage needs view_scale");
    hipError_t e = launch_convert(dst, src, n_views, (size_t)H * W,
                                  dtype == FDK_DTYPE_F16 ? kF16 : kBF16, view_scale,
                                  (hipStream_t)stream);
    return e == hipSuccess ? FDK_OK : hip_fail(e, "conversion launch");
}

int fdk_update_probe(float* a, size_t n, float s, void* stream)
{
    g_err.clear();
    if (!a && n) return fail(FDK_ERR_INVALID_ARG, "a is NULL");
    if (n == 0) return FDK_OK;
    hipError_t e = launch_update_probe(a, n, s, (hipStream_t)stream);
    return e == hipSuccess ? FDK_OK : hip_fail(e, "update probe launch");
}

int fdk_profile_begin(void)
{
    g_err.clear();
    std::lock_guard<std::mutex> lock(g_timing.mu);
    for (auto& p : g_timing.ev) {
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    g_timing.ev.clear();
    g_timing.on = true;
    return FDK_OK;
}

int fdk_profile_end(double* kernel_ms, int* launches)
{
    g_err.clear();
    double total = 0.0;
    int rc = FDK_OK;
    std::lock_guard<std::mutex> lock(g_timing.mu);
    for (auto& p : g_timing.ev) {
        float ms = 0.0f;
        hipError_t e = hipEventSynchronize(p.second);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.first, p.second);
        if (e != hipSuccess && rc == FDK_OK) rc = hip_fail(e, "timing readback");
        total += ms;
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    if (kernel_ms) *kernel_ms = total;
    if (launches) *launches = (int)g_timing.ev.size();
    g_timing.ev.clear();
    g_timing.on = false;
    return rc;
}

int fdk_set_batch(int views_per_pass)
{
    g_err.clear();
    if (views_per_pass == 0) return g_batch;
    if (views_per_pass < 1 || views_per_pass > kMaxBatch)
        return fail(FDK_ERR_INVALID_ARG, "views_per_pass=%d outside [1, %d]", views_per_pass,
                    kMaxBatch);
    g_batch = views_per_pass;
    return g_batch;
}

int fdk_set_layout(int layout)
{
    g_err.clear();
    if (layout == -1) return g_layout;
    if (layout < kRows || layout > kDQuads)
        return fail(FDK_ERR_INVALID_ARG, "layout=%d is not one of 0..4", layout);
    g_layout = layout;
    return g_layout;
}

int fdk_set_divide(int mode)
{
    g_err.clear();
    if (mode == -1) return g_divide;
    if (mode < FDK_DIVIDE_RCP || mode > FDK_DIVIDE_RCP12)
        return fail(FDK_ERR_INVALID_ARG, "divide mode %d is not one of 0..3", mode);
    g_divide = mode;
    return mode;
}

int fdk_set_row_clamp(int mode)
{
    g_err.clear();
    if (mode == -1) return g_rows_free ? 0 : 1;
    if (mode != 0 && mode != 1) return fail(FDK_ERR_INVALID_ARG, "mode=%d is not 0 or 1", mode);
    g_rows_free = mode == 0 ? 1 : 0;
    return mode;
}

int fdk_release(void)
{
    g_err.clear();
    std::lock_guard<std::mutex> lock(g_stage_mu);
    int rc = FDK_OK;
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto& kv : g_stage) {
        Staging& st = kv.second;
        (void)hipSetDevice(kv.first);
        if (st.last_use) {
            hipError_t e = hipEventSynchronize(st.last_use);
            if (e != hipSuccess && rc == FDK_OK) rc = hip_fail(e, "hipEventSynchronize");
            (void)hipEventDestroy(st.last_use);
        }
        if (st.ptr) {
            hipError_t e = hipFree(st.ptr);
            if (e != hipSuccess && rc == FDK_OK) rc = hip_fail(e, "hipFree(staging)");
        }
        if (st.mats_copied) {
            hipError_t e = hipEventSynchronize(st.mats_copied);
            if (e != hipSuccess && rc == FDK_OK) rc = hip_fail(e, "hipEventSynchronize");
            (void)hipEventDestroy(st.mats_copied);
        }
        if (st.host_mats) {
            hipError_t e = hipHostFree(st.host_mats);
            if (e != hipSuccess && rc == FDK_OK) rc = hip_fail(e, "hipHostFree");
        }
        if (st.side) {
            hipError_t e = hipStreamSynchronize(st.side);
            if (e != hipSuccess && rc == FDK_OK) rc = hip_fail(e, "hipStreamSynchronize");
        }
        for (hipEvent_t ev : {st.fork, st.staged[0], st.staged[1], st.freed[0], st.freed[1]})
            if (ev) (void)hipEventDestroy(ev);
        if (st.side) (void)hipStreamDestroy(st.side);
    }
    g_stage.clear();
    (void)hipSetDevice(cur);
    return rc;
}

const char* fdk_last_error(void)
{
    return g_err.c_str();
}

int fdk_version(void)
{
    return (1 << 16) | 0;
}

}  // extern "C"
