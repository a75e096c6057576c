/*
 * FP64 CPU oracle for voxel-driven cone-beam backprojection and its exact
 * transpose.  TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may call it; the library's product
 * path never does.  It shares no code with the GPU path.
 *
 * What it computes (paper, Section 3.1, Listing 1 and its three parts as
 * described in Section 3.2, with the zero-padded projection buffers of
 * Section 3.3):
 *
 *   For every voxel with world centre X = origin + voxel_size * (x, y, z)
 *   and every projection i, in ascending order of i:
 *     (uw, vw, w) = P_i (X, 1)                    [part 1: geometry]
 *     skip the view if w <= 0 (voxel not in front of the source)
 *     u = uw / w,  v = vw / w                     (exact division)
 *     iu = floor(u), iv = floor(v), scalx = u - iu, scaly = v - iv
 *     the four neighbours valtl = T(iu, iv), valtr = T(iu+1, iv),
 *       valbl = T(iu, iv+1), valbr = T(iu+1, iv+1), where T(j, k) is the
 *       projection pixel I_i[k][j] inside the detector and 0 outside it
 *                                                 [part 2: load]
 *     vall = scaly valbl + (1 - scaly) valtl
 *     valr = scaly valbr + (1 - scaly) valtr
 *     fx   = scalx valr  + (1 - scalx) vall       [part 3: interpolate]
 *     VOL[z][y][x] += fx / w^2
 *
 * Readings of the paper taken here (it does not state them):
 *   - taps outside the detector read 0 (the padded buffers of Section 3.3);
 *   - the integer cast is floor, not truncation (the listing's guards on
 *     iu >= -1 only make sense with floor);
 *   - pixel (j, k) has its centre at u = j, v = k; u runs along a row (W),
 *     v across rows (H);
 *   - P_i is row-major 3x4 (the listing's A is its column-major image);
 *   - the volume is accumulated into (+=), never overwritten.
 *
 * All arithmetic is IEEE double; the projections are promoted exactly from
 * FP32.  Parallelism: OpenMP over z slices with a static,1 schedule (the
 * paper's choice in Section 6), which does not change any result.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <omp.h>

/* Zero-extended pixel read T(j, k). */
static inline double tap(const float* I, int H, int W, long long j, long long k)
{
    if (j < 0 || j >= W || k < 0 || k >= H) return 0.0;
    return (double)I[(size_t)k * W + j];
}

/* Contribution of projection I (with matrix P) to the voxel at world X. */
static inline double voxel_update(const double* P, const float* I, int H, int W,
                                  double wx, double wy, double wz)
{
    /* part 1 */
    double uw = P[0] * wx + P[1] * wy + P[2] * wz + P[3];
    double vw = P[4] * wx + P[5] * wy + P[6] * wz + P[7];
    double w = P[8] * wx + P[9] * wy + P[10] * wz + P[11];
    if (!(w > 0.0)) return 0.0;
    double u = uw / w, v = vw / w;
    /* every tap is outside the detector: the zero-extended value is 0
       (this also keeps the integer conversion below in range) */
    if (!(u > -2.0 && u < W + 1.0 && v > -2.0 && v < H + 1.0)) return 0.0;
    double fu = floor(u), fv = floor(v);
    long long iu = (long long)fu, iv = (long long)fv;
    double scalx = u - fu, scaly = v - fv;
    /* part 2 */
    double valtl = tap(I, H, W, iu, iv);
    double valtr = tap(I, H, W, iu + 1, iv);
    double valbl = tap(I, H, W, iu, iv + 1);
    double valbr = tap(I, H, W, iu + 1, iv + 1);
    /* part 3 */
    double vall = scaly * valbl + (1.0 - scaly) * valtl;
    double valr = scaly * valbr + (1.0 - scaly) * valtr;
    double fx = scalx * valr + (1.0 - scalx) * vall;
    return fx / (w * w);
}

/*
 * Backprojection of n_views projections into the box
 * [x0, x0+nx) x [y0, y0+ny) x [z0, z0+nz) of the N^3 grid.
 *   R      : nz*ny*nx doubles, R[((z-z0)*ny + (y-y0))*nx + (x-x0)], accumulated
 *   origin : world centre of voxel (0,0,0), mm
 *   proj   : n_views*H*W floats, I_i[k][j] = proj[(i*H + k)*W + j]
 *   P      : n_views*12 doubles, row-major 3x4 per view
 * Returns 0, or -1 on invalid arguments.
 */
int oracle_backproject_box(double* R, int N, double voxel_size, const double* origin,
                           const float* proj, int n_views, int H, int W, const double* P,
                           int x0, int nx, int y0, int ny, int z0, int nz)
{
    if (!R || !origin || !P || !proj || N < 1 || n_views < 0 || H < 1 || W < 1) return -1;
    if (x0 < 0 || y0 < 0 || z0 < 0 || nx < 0 || ny < 0 || nz < 0 || x0 + nx > N ||
        y0 + ny > N || z0 + nz > N)
        return -1;
    const size_t img = (size_t)H * W;
#pragma omp parallel for schedule(static, 1)
    for (int z = z0; z < z0 + nz; ++z) {
        double wz = origin[2] + voxel_size * z;
        for (int y = y0; y < y0 + ny; ++y) {
            double wy = origin[1] + voxel_size * y;
            for (int x = x0; x < x0 + nx; ++x) {
                double wx = origin[0] + voxel_size * x;
                double sum = 0.0;
                for (int i = 0; i < n_views; ++i)
                    sum += voxel_update(P + 12 * (size_t)i, proj + i * img, H, W, wx, wy, wz);
                R[((size_t)(z - z0) * ny + (y - y0)) * nx + (x - x0)] += sum;
            }
        }
    }
    return 0;
}

/*
 * Backprojection at a list of voxels: R[p] += sum over views for the voxel
 * (xyz[3p], xyz[3p+1], xyz[3p+2]).  Same conventions as above.
 */
int oracle_backproject_points(double* R, const int* xyz, long long n_points, int N,
                              double voxel_size, const double* origin, const float* proj,
                              int n_views, int H, int W, const double* P)
{
    if (!R || !xyz || !origin || !P || !proj || N < 1 || n_views < 0 || H < 1 || W < 1 ||
        n_points < 0)
        return -1;
    for (long long p = 0; p < n_points; ++p)
        for (int c = 0; c < 3; ++c)
            if (xyz[3 * p + c] < 0 || xyz[3 * p + c] >= N) return -1;
    const size_t img = (size_t)H * W;
#pragma omp parallel for schedule(static, 1)
    for (long long p = 0; p < n_points; ++p) {
        double wx = origin[0] + voxel_size * xyz[3 * p];
        double wy = origin[1] + voxel_size * xyz[3 * p + 1];
        double wz = origin[2] + voxel_size * xyz[3 * p + 2];
        double sum = 0.0;
        for (int i = 0; i < n_views; ++i)
            sum += voxel_update(P + 12 * (size_t)i, proj + i * img, H, W, wx, wy, wz);
        R[p] += sum;
    }
    return 0;
}

/*
 * The exact transpose of the backprojection above (the matched cone-beam
 * forward projector): for every view i and voxel, the voxel value times
 * 1/w^2 is spread onto the four pixels the backprojection reads, with the
 * same bilinear weights, dropping pixels outside the detector.
 *   F   : n_views*H*W doubles, accumulated
 *   vol : N^3 doubles, vol[(z*N + y)*N + x]
 * Parallel over views (each view's image is written by one thread).
 */
int oracle_forward_project(double* F, int n_views, int H, int W, const double* P,
                           const double* vol, int N, double voxel_size, const double* origin)
{
    if (!F || !P || !vol || !origin || N < 1 || n_views < 0 || H < 1 || W < 1) return -1;
    const size_t img = (size_t)H * W;
#pragma omp parallel for schedule(static, 1)
    for (int i = 0; i < n_views; ++i) {
        const double* A = P + 12 * (size_t)i;
        double* Fi = F + i * img;
        for (int z = 0; z < N; ++z) {
            double wz = origin[2] + voxel_size * z;
            for (int y = 0; y < N; ++y) {
                double wy = origin[1] + voxel_size * y;
                for (int x = 0; x < N; ++x) {
                    double val = vol[((size_t)z * N + y) * N + x];
                    if (val == 0.0) continue;
                    double wx = origin[0] + voxel_size * x;
                    double uw = A[0] * wx + A[1] * wy + A[2] * wz + A[3];
                    double vw = A[4] * wx + A[5] * wy + A[6] * wz + A[7];
                    double w = A[8] * wx + A[9] * wy + A[10] * wz + A[11];
                    if (!(w > 0.0)) continue;
                    double u = uw / w, v = vw / w;
                    if (!(u > -2.0 && u < W + 1.0 && v > -2.0 && v < H + 1.0)) continue;
                    double fu = floor(u), fv = floor(v);
                    long long iu = (long long)fu, iv = (long long)fv;
                    double scalx = u - fu, scaly = v - fv;
                    double s = val / (w * w);
                    double wt[4] = {(1.0 - scalx) * (1.0 - scaly), scalx * (1.0 - scaly),
                                    (1.0 - scalx) * scaly, scalx * scaly};
                    long long jj[4] = {iu, iu + 1, iu, iu + 1};
                    long long kk[4] = {iv, iv, iv + 1, iv + 1};
                    for (int t = 0; t < 4; ++t)
                        if (jj[t] >= 0 && jj[t] < W && kk[t] >= 0 && kk[t] < H)
                            Fi[(size_t)kk[t] * W + jj[t]] += s * wt[t];
                }
            }
        }
    }
    return 0;
}

/* Number of OpenMP threads the oracle's parallel loops use. */
int oracle_threads(void)
{
    int n = 1;
#pragma omp parallel
    {
#pragma omp single
        n = omp_get_num_threads();
    }
    return n;
}
