/*
 * Host-code sanitizer driver: the FP64 oracle (oracle/oracle.c) and the
 * input generator (synth/synth.c) built with -fsanitize=address,undefined
 * and exercised on small cases, including sub-boxes at the volume's edges,
 * voxels whose taps straddle the detector border, views that miss the
 * volume and invalid arguments.  Besides memory and undefined-behaviour
 * errors (reported by the sanitizers, which abort), it checks two exact
 * properties: box and point evaluations agree bit for bit with the full
 * volume, and the adjoint identity <B p, x> = <p, F x> holds to 1e-10.
 * Exit status 0 when every check passes.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_backproject_box(double* R, int N, double voxel_size, const double* origin,
                           const float* proj, int n_views, int H, int W, const double* P,
                           int x0, int nx, int y0, int ny, int z0, int nz);
int oracle_backproject_points(double* R, const int* xyz, long long n_points, int N,
                              double voxel_size, const double* origin, const float* proj,
                              int n_views, int H, int W, const double* P);
int oracle_forward_project(double* F, int n_views, int H, int W, const double* P,
                           const double* vol, int N, double voxel_size, const double* origin);
int synth_line_integrals(float* out, int V, int H, int W, const double* src, const double* det,
                         const double* eu, const double* ev, double pixel, const double* ell,
                         int n_ell);
int synth_fdk_prefilter(float* proj, int V, int H, int W, const double* betas, double delta,
                        double dbeta, double sid, double sdd, double pixel, int fft_len,
                        int parker);
int synth_voxelize(float* vol, int nx, int ny, int nz, double voxel_size, const double* origin,
                   const double* ell, int n_ell, int sub);

static int failures = 0;
#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++failures;                                                 \
        }                                                               \
    } while (0)

static double dot3(const double* a, const double* b)
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* circular scan about z: source at distance sid, flat detector at sdd,
 * w = depth along the detector normal / sid */
static void geometry(int V, int H, int W, double sid, double sdd, double pixel, double* P,
                     double* src, double* det, double* eu, double* ev, double* betas)
{
    const double cu = 0.5 * (W - 1), cv = 0.5 * (H - 1);
    for (int i = 0; i < V; ++i) {
        const double b = i * 3.5 / (V > 1 ? V - 1 : 1);
        double* s = src + 3 * i;
        double* d = det + 3 * i;
        double* e1 = eu + 3 * i;
        double* e2 = ev + 3 * i;
        const double n[3] = {-cos(b), -sin(b), 0.0};
        s[0] = sid * cos(b);
        s[1] = sid * sin(b);
        s[2] = 0.3 * i;
        for (int k = 0; k < 3; ++k) d[k] = s[k] + sdd * n[k];
        e1[0] = -sin(b);
        e1[1] = cos(b);
        e1[2] = 0.0;
        e2[0] = e2[1] = 0.0;
        e2[2] = 1.0;
        betas[i] = b;
        double dsn[3] = {d[0] - s[0], d[1] - s[1], d[2] - s[2]};
        const double D = dot3(dsn, n);
        const double rho[4] = {n[0], n[1], n[2], -dot3(n, s)};
        double* M = P + 12 * i;
        for (int c = 0; c < 4; ++c) M[8 + c] = rho[c] / sid;
        for (int r = 0; r < 2; ++r) {
            const double* e = r == 0 ? e1 : e2;
            const double cc = r == 0 ? cu : cv;
            const double ee[4] = {e[0], e[1], e[2], -dot3(e, s)};
            double sd[3] = {s[0] - d[0], s[1] - d[1], s[2] - d[2]};
            const double f = dot3(sd, e);
            for (int c = 0; c < 4; ++c)
                M[4 * r + c] = (D * ee[c] + f * rho[c]) / (pixel * sid) + cc * M[8 + c];
        }
    }
}

int main(void)
{
    const int V = 5, H = 11, W = 13, N = 9, L = 32;
    const double sid = 60.0, sdd = 100.0, pixel = 2.5, vs = 3.0;
    const double origin[3] = {-12.0, -12.5, -11.0};
    double *P = malloc(sizeof(double) * 12 * V), *src = malloc(sizeof(double) * 3 * V),
           *det = malloc(sizeof(double) * 3 * V), *eu = malloc(sizeof(double) * 3 * V),
           *ev = malloc(sizeof(double) * 3 * V), *betas = malloc(sizeof(double) * V);
    geometry(V, H, W, sid, sdd, pixel, P, src, det, eu, ev, betas);
    /* one view shifted far off the detector: it must contribute nothing */
    for (int c = 0; c < 4; ++c) P[12 * 4 + c] += 1e4 * P[12 * 4 + 8 + c];

    /* two ellipsoids (centre, semi-axes, rotation, density, unused) */
    double ell[34] = {0};
    const double e0[17] = {0.5, -0.5, 0.0, 9.0, 7.0, 8.0, 1, 0, 0, 0, 1, 0, 0, 0, 1, 0.02, 0};
    const double e1[17] = {3.0, 2.0, -1.0, 3.0, 2.0, 4.0, 0, 1, 0, -1, 0, 0, 0, 0, 1, -0.01, 0};
    memcpy(ell, e0, sizeof(e0));
    memcpy(ell + 17, e1, sizeof(e1));

    float* proj = calloc((size_t)V * H * W, sizeof(float));
    CHECK(synth_line_integrals(proj, V, H, W, src, det, eu, ev, pixel, ell, 2) == 0);
    CHECK(synth_fdk_prefilter(proj, V, H, W, betas, 0.2, 0.8, sid, sdd, pixel, L, 1) == 0);
    CHECK(synth_fdk_prefilter(proj, V, H, W, betas, -1.0, 0.8, sid, sdd, pixel, L, 0) == 0);
    float* vox = malloc(sizeof(float) * N * N * N);
    CHECK(synth_voxelize(vox, N, N, N, vs, origin, ell, 2, 2) == 0);

    /* the full volume, every sub-box touching an edge, and points */
    const size_t n3 = (size_t)N * N * N;
    double* R = calloc(n3, sizeof(double));
    CHECK(oracle_backproject_box(R, N, vs, origin, proj, V, H, W, P, 0, N, 0, N, 0, N) == 0);
    const int boxes[4][6] = {{0, 1, 0, 1, 0, 1}, {N - 1, 1, N - 2, 2, 0, N},
                             {2, 5, N - 3, 3, N - 4, 4}, {0, N, 4, 1, 8, 1}};
    for (int b = 0; b < 4; ++b) {
        const int* q = boxes[b];
        double* Rb = calloc((size_t)q[1] * q[3] * q[5], sizeof(double));
        CHECK(oracle_backproject_box(Rb, N, vs, origin, proj, V, H, W, P, q[0], q[1], q[2], q[3],
                                     q[4], q[5]) == 0);
        for (int z = 0; z < q[5]; ++z)
            for (int y = 0; y < q[3]; ++y)
                for (int x = 0; x < q[1]; ++x)
                    CHECK(Rb[((size_t)z * q[3] + y) * q[1] + x] ==
                          R[((size_t)(z + q[4]) * N + y + q[2]) * N + x + q[0]]);
        free(Rb);
    }
    int pts[6 * 3] = {0, 0, 0, N - 1, N - 1, N - 1, 4, 4, 4, 0, N - 1, 3, N - 1, 0, 5, 2, 7, 1};
    double Rp[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  /* accumulated into: start at zero */
    CHECK(oracle_backproject_points(Rp, pts, 6, N, vs, origin, proj, V, H, W, P) == 0);
    for (int i = 0; i < 6; ++i)
        CHECK(Rp[i] == R[((size_t)pts[3 * i + 2] * N + pts[3 * i + 1]) * N + pts[3 * i]]);

    /* the shifted view alone contributes nothing */
    double* R4 = calloc(n3, sizeof(double));
    CHECK(oracle_backproject_box(R4, N, vs, origin, proj + (size_t)4 * H * W, 1, H, W, P + 48, 0,
                                 N, 0, N, 0, N) == 0);
    for (size_t i = 0; i < n3; ++i) CHECK(R4[i] == 0.0);

    /* adjoint identity with the voxelised phantom as x */
    double* x = malloc(sizeof(double) * n3);
    for (size_t i = 0; i < n3; ++i) x[i] = vox[i] + 0.001 * (double)(i % 7);
    double* F = calloc((size_t)V * H * W, sizeof(double));
    CHECK(oracle_forward_project(F, V, H, W, P, x, N, vs, origin) == 0);
    double lhs = 0.0, rhs = 0.0, scale = 0.0;
    for (size_t i = 0; i < n3; ++i) {
        lhs += R[i] * x[i];
        scale += fabs(R[i] * x[i]);
    }
    for (size_t i = 0; i < (size_t)V * H * W; ++i) rhs += (double)proj[i] * F[i];
    CHECK(fabs(lhs - rhs) <= 1e-10 * scale);

    /* invalid arguments are refused */
    CHECK(oracle_backproject_box(NULL, N, vs, origin, proj, V, H, W, P, 0, 1, 0, 1, 0, 1) == -1);
    CHECK(oracle_backproject_box(R, 0, vs, origin, proj, V, H, W, P, 0, 1, 0, 1, 0, 1) == -1);
    CHECK(oracle_forward_project(F, V, 0, W, P, x, N, vs, origin) == -1);
    CHECK(synth_line_integrals(proj, V, H, 0, src, det, eu, ev, pixel, ell, 2) == -1);
    CHECK(synth_voxelize(vox, N, N, N, vs, origin, ell, 2, 0) == -1);

    free(P); free(src); free(det); free(eu); free(ev); free(betas); free(proj); free(vox);
    free(R); free(R4); free(x); free(F);
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("sanitized oracle and generator: all checks passed (<Bp,x> = %.12g, <p,Fx> = %.12g)\n",
           lhs, rhs);
    return 0;
}
