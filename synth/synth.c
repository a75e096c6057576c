/*
 * Seeded synthetic inputs for the cone-beam backprojection workloads.
 *
 * This file holds no step of the backprojection itself.  It makes the data a
 * C-arm scanner would hand to the reconstruction:
 *   - analytic line integrals of an ellipsoid phantom through a flat-panel
 *     cone-beam geometry (the stand-in for the measured rabbit projections
 *     of the paper's benchmark, which are not available);
 *   - the Feldkamp 2D pre-processing of those integrals (cosine weight,
 *     Parker short-scan weight, row-wise Ram-Lak filter), so that the
 *     backprojection input has the shape and value distribution of real
 *     filtered projections (signed, heavy-tailed at object edges);
 *   - a point-sampled voxelisation of the same phantom (ground truth for
 *     image-quality comparisons).
 *
 * Everything is computed in double precision and is independent of the
 * number of OpenMP threads (each output element is produced by exactly one
 * thread with a fixed operation order).
 *
 * Ellipsoid record (17 doubles): centre[3], semi-axes[3], R[9] (row-major,
 * the columns are the ellipsoid axes in world coordinates, so a world point
 * is c + R (a .* q) for q on the unit sphere), density, unused.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ELL_STRIDE 17

static double ray_ellipsoid_sum(const double s[3], const double d[3], double dlen,
                                const double* ell, int n_ell)
{
    double total = 0.0;
    for (int e = 0; e < n_ell; ++e) {
        const double* E = ell + (size_t)e * ELL_STRIDE;
        const double* c = E;
        const double* a = E + 3;
        const double* R = E + 6;
        double rho = E[15];
        double sc[3] = {s[0] - c[0], s[1] - c[1], s[2] - c[2]};
        double sp[3], dp[3];
        for (int k = 0; k < 3; ++k) {
            /* (R^T v)_k = sum_j R[j][k] v_j */
            double ts = R[0 * 3 + k] * sc[0] + R[1 * 3 + k] * sc[1] + R[2 * 3 + k] * sc[2];
            double td = R[0 * 3 + k] * d[0] + R[1 * 3 + k] * d[1] + R[2 * 3 + k] * d[2];
            sp[k] = ts / a[k];
            dp[k] = td / a[k];
        }
        double A = dp[0] * dp[0] + dp[1] * dp[1] + dp[2] * dp[2];
        double B = sp[0] * dp[0] + sp[1] * dp[1] + sp[2] * dp[2];
        double C = sp[0] * sp[0] + sp[1] * sp[1] + sp[2] * sp[2] - 1.0;
        double disc = B * B - A * C;
        if (disc > 0.0) total += rho * 2.0 * sqrt(disc) / A * dlen;
    }
    return total;
}

/* Line integrals p[v][k][j] of the phantom along the ray from the source of
 * view v to the centre of detector pixel (j,k).  Pixel (j,k) sits at
 * det + (j - cu) * pixel * eu + (k - cv) * pixel * ev, cu = (W-1)/2,
 * cv = (H-1)/2. */
int synth_line_integrals(float* out, int V, int H, int W, const double* src,
                         const double* det, const double* eu, const double* ev, double pixel,
                         const double* ell, int n_ell)
{
    if (!out || V < 0 || H < 1 || W < 1 || !src || !det || !eu || !ev || !ell) return -1;
    const double cu = 0.5 * (W - 1), cv = 0.5 * (H - 1);
    const long long rows = (long long)V * H;
#pragma omp parallel for schedule(dynamic, 4)
    for (long long r = 0; r < rows; ++r) {
        int v = (int)(r / H), k = (int)(r % H);
        const double* s = src + 3 * (size_t)v;
        const double* d0 = det + 3 * (size_t)v;
        const double* U = eu + 3 * (size_t)v;
        const double* Vv = ev + 3 * (size_t)v;
        double b = (k - cv) * pixel;
        float* row = out + (size_t)r * W;
        for (int j = 0; j < W; ++j) {
            double a = (j - cu) * pixel;
            double dir[3];
            for (int q = 0; q < 3; ++q) dir[q] = d0[q] + a * U[q] + b * Vv[q] - s[q];
            double dl = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
            row[j] = (float)ray_ellipsoid_sum(s, dir, dl, ell, n_ell);
        }
    }
    return 0;
}

/* In-place iterative radix-2 complex FFT (sign = -1 forward, +1 inverse,
 * no scaling).  n must be a power of two; tw holds exp(-2 pi i k / n) for
 * k < n/2 as (cos, sin) pairs. */
static void fft_inplace(double* re, double* im, int n, const double* tw, int sign)
{
    for (int i = 1, j = 0; i < n; ++i) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) {
            double t = re[i]; re[i] = re[j]; re[j] = t;
            t = im[i]; im[i] = im[j]; im[j] = t;
        }
    }
    for (int len = 2; len <= n; len <<= 1) {
        int half = len >> 1, step = n / len;
        for (int i = 0; i < n; i += len) {
            for (int k = 0; k < half; ++k) {
                double wr = tw[2 * (k * step)], wi = sign * tw[2 * (k * step) + 1];
                int p = i + k, q = p + half;
                double xr = re[q] * wr - im[q] * wi;
                double xi = re[q] * wi + im[q] * wr;
                re[q] = re[p] - xr; im[q] = im[p] - xi;
                re[p] += xr; im[p] += xi;
            }
        }
    }
}

/* Parker short-scan redundancy weight for source angle beta and fan angle
 * gamma over a scan of pi + 2*delta (delta >= max |gamma|). */
static double parker_weight(double beta, double gamma, double delta)
{
    const double PI = 3.14159265358979323846;
    if (beta < 0.0) return 0.0;
    if (beta < 2.0 * (delta - gamma)) {
        double s = sin(0.25 * PI * beta / (delta - gamma));
        return s * s;
    }
    if (beta < PI - 2.0 * gamma) return 1.0;
    if (beta <= PI + 2.0 * delta) {
        double s = sin(0.25 * PI * (PI + 2.0 * delta - beta) / (delta + gamma));
        return s * s;
    }
    return 0.0;
}

/* Feldkamp 2D pre-processing, in place: for every view v and pixel (j,k)
 *   p~ = p * SDD / sqrt(SDD^2 + a^2 + b^2) * parker(beta_v, gamma_j)
 * with a = (j - cu) pixel, b = (k - cv) pixel, gamma_j = -atan(a / SDD)
 * (the sign makes the conjugate ray of (beta, gamma) sit at beta + pi +
 * 2 gamma for this geometry), then each row is convolved with the discrete
 * Ram-Lak kernel h[0] = 1/(4 tau^2), h[odd n] = -1/(n pi tau)^2, h[even] = 0
 * sampled at the isocentre spacing tau = pixel * SID / SDD, as a linear
 * convolution (zero-padded FFT of length fft_len >= 2W - 1), and scaled by
 * tau * dbeta.  parker != 0 selects the Parker weight (short scan);
 * otherwise the weight is 1/2 (full-circle scan). */
int synth_fdk_prefilter(float* proj, int V, int H, int W, const double* betas, double delta,
                        double dbeta, double sid, double sdd, double pixel, int fft_len,
                        int parker)
{
    if (!proj || V < 0 || H < 1 || W < 1 || !betas) return -1;
    if (fft_len < 2 * W - 1 || (fft_len & (fft_len - 1))) return -2;
    const double PI = 3.14159265358979323846;
    const int L = fft_len;
    const double tau = pixel * sid / sdd;
    const double cu = 0.5 * (W - 1), cv = 0.5 * (H - 1);
    double* tw = (double*)malloc(sizeof(double) * L);
    double* Hk = (double*)malloc(sizeof(double) * L);
    double* hre = (double*)calloc((size_t)L, sizeof(double));
    double* him = (double*)calloc((size_t)L, sizeof(double));
    if (!tw || !Hk || !hre || !him) { free(tw); free(Hk); free(hre); free(him); return -3; }
    for (int k = 0; k < L / 2; ++k) {
        tw[2 * k] = cos(2.0 * PI * k / L);
        tw[2 * k + 1] = -sin(2.0 * PI * k / L);
    }
    /* kernel at circular positions n mod L for |n| <= W-1 */
    hre[0] = 1.0 / (4.0 * tau * tau);
    for (int n = 1; n <= W - 1; ++n) {
        double hv = (n & 1) ? -1.0 / ((double)n * n * PI * PI * tau * tau) : 0.0;
        hre[n] = hv;
        hre[L - n] = hv;
    }
    fft_inplace(hre, him, L, tw, -1);
    const double scale = tau * dbeta / L; /* 1/L undoes the unscaled inverse FFT */
    for (int k = 0; k < L; ++k) Hk[k] = hre[k] * scale;
    free(hre); free(him);

    const long long pairs = (long long)V * ((H + 1) / 2);
#pragma omp parallel
    {
        double* re = (double*)malloc(sizeof(double) * L);
        double* im = (double*)malloc(sizeof(double) * L);
        double* wcol = (double*)malloc(sizeof(double) * W);
#pragma omp for schedule(dynamic, 8)
        for (long long pr = 0; pr < pairs; ++pr) {
            int v = (int)(pr / ((H + 1) / 2));
            int k0 = 2 * (int)(pr % ((H + 1) / 2));
            int k1 = k0 + 1;
            for (int j = 0; j < W; ++j) {
                double a = (j - cu) * pixel;
                double gamma = -atan(a / sdd);
                wcol[j] = parker ? parker_weight(betas[v], gamma, delta) : 0.5;
            }
            memset(re, 0, sizeof(double) * L);
            memset(im, 0, sizeof(double) * L);
            float* r0 = proj + ((size_t)v * H + k0) * W;
            float* r1 = (k1 < H) ? r0 + W : NULL;
            double b0 = (k0 - cv) * pixel, b1 = (k1 - cv) * pixel;
            for (int j = 0; j < W; ++j) {
                double a = (j - cu) * pixel;
                re[j] = r0[j] * wcol[j] * sdd / sqrt(sdd * sdd + a * a + b0 * b0);
                if (r1) im[j] = r1[j] * wcol[j] * sdd / sqrt(sdd * sdd + a * a + b1 * b1);
            }
            fft_inplace(re, im, L, tw, -1);
            for (int k = 0; k < L; ++k) { re[k] *= Hk[k]; im[k] *= Hk[k]; }
            fft_inplace(re, im, L, tw, +1);
            for (int j = 0; j < W; ++j) {
                r0[j] = (float)re[j];
                if (r1) r1[j] = (float)im[j];
            }
        }
        free(re); free(im); free(wcol);
    }
    free(tw); free(Hk);
    return 0;
}

/* Phantom density at the centre of every voxel of an nx*ny*nz grid with
 * voxel (x,y,z) centred at origin + voxel_size * (x,y,z); sub > 1 averages
 * sub^3 regularly spaced samples inside each voxel. */
int synth_voxelize(float* vol, int nx, int ny, int nz, double voxel_size, const double* origin,
                   const double* ell, int n_ell, int sub)
{
    if (!vol || nx < 1 || ny < 1 || nz < 1 || !origin || !ell || sub < 1) return -1;
#pragma omp parallel for schedule(static, 1)
    for (int z = 0; z < nz; ++z) {
        for (int y = 0; y < ny; ++y) {
            for (int x = 0; x < nx; ++x) {
                double acc = 0.0;
                for (int sz = 0; sz < sub; ++sz)
                for (int sy = 0; sy < sub; ++sy)
                for (int sx = 0; sx < sub; ++sx) {
                    double p[3] = {
                        origin[0] + voxel_size * (x + (sx + 0.5) / sub - 0.5),
                        origin[1] + voxel_size * (y + (sy + 0.5) / sub - 0.5),
                        origin[2] + voxel_size * (z + (sz + 0.5) / sub - 0.5)};
                    for (int e = 0; e < n_ell; ++e) {
                        const double* E = ell + (size_t)e * ELL_STRIDE;
                        const double* R = E + 6;
                        double d[3] = {p[0] - E[0], p[1] - E[1], p[2] - E[2]};
                        double q = 0.0;
                        for (int k = 0; k < 3; ++k) {
                            double t = (R[0 * 3 + k] * d[0] + R[1 * 3 + k] * d[1] +
                                        R[2 * 3 + k] * d[2]) / E[3 + k];
                            q += t * t;
                        }
                        if (q <= 1.0) acc += E[15];
                    }
                }
                vol[((size_t)z * ny + y) * nx + x] = (float)(acc / ((double)sub * sub * sub));
            }
        }
    }
    return 0;
}
