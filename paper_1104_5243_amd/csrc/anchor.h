// Anchored voxel geometry shared by the fused backprojection and the
// forward projection, so that both compute bit-identical coordinates,
// weights and taps for every (voxel, view) pair (the forward projection is
// then the exact transpose of the backprojection).
//
// The volume is cut into boxes of kWaveX x kWaveY columns x kBoxZ slices
// (kBoxZ = the backprojection's z voxels per thread).  For a box and a view,
// in FP64, from the view's folded matrix Q (centred index frame, columns x,
// y, z, 1):
//   C = the centre of the box's voxels inside the volume,
//   (Uc, Vc, Wc) = Q (C, 1),  a_u = round(Uc / Wc),  a_v = round(Vc / Wc),
//   S_u = Q_u - a_u Q_w,  S_v = Q_v - a_v Q_w   (rows with a_u, a_v times the
//                                                w row subtracted),
// and the anchored numerators at the centre of the box's first slice z0,
//   uc0 = S_u (Cx, Cy, z0, 1),  vc0 = S_v (...),  wc0 = Q_w (...).
// These and the slopes are rounded once to FP32.  For a voxel at offsets
// (dx, dy) from the centre column and slice index i from z0,
//   num_u = fma(i, S_u.z, fma(S_u.y, dy, fma(S_u.x, dx, uc0)))
// (likewise v and w), and u' - a_u = num_u / w.  Inside the box every FP32
// quantity stays within ~20 pixels of 0 instead of ~600 (u' itself), so
// their rounding errors shrink by that factor; the tap index adds a_u, a_v
// back as integers.  (The paper's Section 3.3 hoists invariants out of the
// voxel loop; this hoists the large part of the coordinates, exactly.)
#pragma once

#include "fdk_internal.h"
#include "gfx950_util.h"

namespace fdk {

// Reciprocal / division variants of part 1 (fdk_set_divide).
enum Divide { kDivRcp = 0, kDivRcpNR = 1, kDivIEEE = 2, kDivRcp12 = 3 };

// A wave-uniform float read into a scalar register.
__device__ __forceinline__ float uniform_f(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x)));
}

// A wave-uniform double held in scalar registers (its two halves read from
// the first lane).
__device__ __forceinline__ double uniform_d(double x)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)b);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// The part of a box inside the volume, in the centred index frame (all
// values are multiples of 1/2, exact in FP32).  x0, y0: the box's first
// column; zs0: its first slice (absolute); the box spans kx x ky columns
// and kz slices of which those inside [0, N) x [0, N) x [z_first,
// z_first + nz) count.
struct BoxFrame {
    float cx, cy;   // centre column
    float z0;       // first slice
    float hx, hy;   // half extents (centre to the outermost voxel)
    float hz;
};

__device__ __forceinline__ BoxFrame box_frame(const FusedArgs& A, int x0, int y0, int zs0, int kx,
                                              int ky, int kz)
{
    const int x1 = max(min(x0 + kx, A.N) - 1, x0);
    const int y1 = max(min(y0 + ky, A.N) - 1, y0);
    const int z1 = max(min(zs0 + kz, A.z_first + A.nz) - 1, zs0);
    BoxFrame f;
    f.cx = 0.5f * (float)(x0 + x1) - A.c;
    f.cy = 0.5f * (float)(y0 + y1) - A.c;
    f.z0 = (float)zs0 - A.c;
    f.hx = 0.5f * (float)(x1 - x0);
    f.hy = 0.5f * (float)(y1 - y0);
    f.hz = 0.5f * (float)(z1 - zs0);
    return f;
}

// Slopes are kept in the batch's ray frame: t = the transverse axis (x if
// y_fastest, else y), r = the axis along the batch's rays.  Every kernel
// adds the transverse term first, then the ray term, then z: the forward
// projection, whose threads walk the ray axis, then rounds every pair
// exactly as the backprojection does.
struct Anchor {
    float uc, vc, wc;        // anchored numerators and w at the first slice's centre
    float su_t, su_r, su2;   // S_u (transverse, ray, z columns)
    float sv_t, sv_r, sv2;   // S_v
    float sw_t, sw_r, sw2;   // the w row
    int au, av;
    bool skip;               // every voxel of the box misses the detector
    // the hull of the box's projection (u', v' including the anchor) and the
    // smallest w over the box; valid when wmin > 0
    float umin, umax, vmin, vmax, wmin;
};

// The anchor of view `view` of the batch (view >= A.count: a skipped dummy)
// for the box `f`.  ANCHOR false (batches where some voxel may have w <= 0)
// keeps a_u = a_v = 0 and skips nothing.  `bc`: box_centre(f), or where `f`
// is the same on every lane of the wave, uniform_box_centre(f).
// The box's centre column, first slice and centre slice in FP64.
struct BoxCentre {
    double cx, cy, cz, z0;
};
__device__ __forceinline__ BoxCentre box_centre(const BoxFrame& f)
{
    return BoxCentre{f.cx, f.cy, (double)f.z0 + (double)f.hz, f.z0};
}
// ... the same, wave-uniform, held in scalar registers
__device__ __forceinline__ BoxCentre uniform_box_centre(const BoxFrame& f)
{
    const BoxCentre c = box_centre(f);
    return BoxCentre{uniform_d(c.cx), uniform_d(c.cy), uniform_d(c.cz), uniform_d(c.z0)};
}

template <bool ANCHOR>
__device__ __forceinline__ Anchor make_anchor(const FusedArgs& A, int view, const BoxFrame& f,
                                              const BoxCentre& bc)
{
    Anchor a;
    const bool valid = view < A.count;
    const double* q = A.mq + 12 * (size_t)(valid ? view : A.count - 1);
    double Q[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) Q[k] = q[k];
    const double cx = bc.cx, cy = bc.cy, cz = bc.cz, z0 = bc.z0;
    int au = 0, av = 0;
    if (ANCHOR) {
        // nearest integers to u', v' at the centre (any integer near them
        // would do: the anchor only has to keep the numerators small)
        const double Uc = fma(Q[2], cz, fma(Q[1], cy, fma(Q[0], cx, Q[3])));
        const double Vc = fma(Q[6], cz, fma(Q[5], cy, fma(Q[4], cx, Q[7])));
        const double Wc = fma(Q[10], cz, fma(Q[9], cy, fma(Q[8], cx, Q[11])));
        const float rw = __builtin_amdgcn_rcpf((float)Wc);
        au = (int)rintf(fminf(fmaxf((float)Uc * rw, -1048576.0f), 1048576.0f));
        av = (int)rintf(fminf(fmaxf((float)Vc * rw, -1048576.0f), 1048576.0f));
    }
    // the anchored rows, in place: S_u = Q_u - a_u Q_w, S_v = Q_v - a_v Q_w
    const double du = (double)au, dv = (double)av;
    double* S = Q;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        S[k] = fma(-du, Q[8 + k], Q[k]);
        S[4 + k] = fma(-dv, Q[8 + k], Q[4 + k]);
    }
    a.au = au;
    a.av = av;
    a.uc = (float)fma(S[2], z0, fma(S[1], cy, fma(S[0], cx, S[3])));
    a.vc = (float)fma(S[6], z0, fma(S[5], cy, fma(S[4], cx, S[7])));
    a.wc = (float)fma(S[10], z0, fma(S[9], cy, fma(S[8], cx, S[11])));
    const float su0 = (float)S[0], su1 = (float)S[1], sv0 = (float)S[4], sv1 = (float)S[5];
    const float sw0 = (float)S[8], sw1 = (float)S[9];
    const bool yf = A.y_fastest != 0;
    a.su_t = yf ? su0 : su1;
    a.su_r = yf ? su1 : su0;
    a.su2 = (float)S[2];
    a.sv_t = yf ? sv0 : sv1;
    a.sv_r = yf ? sv1 : sv0;
    a.sv2 = (float)S[6];
    a.sw_t = yf ? sw0 : sw1;
    a.sw_r = yf ? sw1 : sw0;
    a.sw2 = (float)S[10];
    // Clipping (Section 3.3).  With w > 0 on the box (w is affine: its
    // minimum is at a corner), the box projects inside the convex hull of
    // its 8 corners' projections; if that hull falls off the detector (0.5
    // pixel margins), every tap of every voxel of the box is zero and the
    // box skips the view.  Corners from the anchored FP32 values (their
    // rounding is far below the margins).
    bool skip = !valid;
    a.umin = a.vmin = -INFINITY;
    a.umax = a.vmax = INFINITY;
    a.wmin = 0.0f;
    if (ANCHOR && valid) {
        float umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
        float wmin = INFINITY;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            // (the corner's -h x s as h x -s, exactly: the box's extents stay
            // in scalar registers)
            const bool px = k & 1, py = k & 2;
            const float ez = (k & 4) ? 2.0f * f.hz : 0.0f;
            const float nu = fmaf(ez, (float)S[2], fmaf(f.hy, py ? su1 : -su1,
                                                        fmaf(f.hx, px ? su0 : -su0, a.uc)));
            const float nv = fmaf(ez, (float)S[6], fmaf(f.hy, py ? sv1 : -sv1,
                                                        fmaf(f.hx, px ? sv0 : -sv0, a.vc)));
            const float nw = fmaf(ez, (float)S[10], fmaf(f.hy, py ? sw1 : -sw1,
                                                         fmaf(f.hx, px ? sw0 : -sw0, a.wc)));
            const float r = __builtin_amdgcn_rcpf(nw);  // (~1 ulp: far inside the margins)
            umin = fminf(umin, nu * r);
            umax = fmaxf(umax, nu * r);
            vmin = fminf(vmin, nv * r);
            vmax = fmaxf(vmax, nv * r);
            wmin = fminf(wmin, nw);
        }
        if (wmin > 0.0f) {
            a.umin = umin + (float)au;
            a.umax = umax + (float)au;
            a.vmin = vmin + (float)av;
            a.vmax = vmax + (float)av;
            a.wmin = wmin;
            skip = a.umax < A.skip_lo_u || a.umin > A.skip_hi_u || a.vmax < A.skip_lo_v ||
                   a.vmin > A.skip_hi_v;
        }
    }
    a.skip = skip;
    return a;
}
template <bool ANCHOR>
__device__ __forceinline__ Anchor make_anchor(const FusedArgs& A, int view, const BoxFrame& f)
{
    return make_anchor<ANCHOR>(A, view, f, box_centre(f));
}

// Part 1 of a voxel from its column base (num_u, num_v, w at the box's
// first slice, from column_base) and its slice index i in the box:
// (u' - a_u, v' - a_v) and r ~ 1/w by the reciprocal variant DIV; with
// WCHECK, a voxel with w <= 0 gets u = v = r = 0.
// (d_t, d_r: the voxel's offsets from the box's centre column along the
// transverse and the ray axis.)
__device__ __forceinline__ void column_base(float uc, float vc, float wc, float su_t, float su_r,
                                            float sv_t, float sv_r, float sw_t, float sw_r,
                                            float d_t, float d_r, float& bu, float& bv, float& bw)
{
    bu = fmaf(su_r, d_r, fmaf(su_t, d_t, uc));
    bv = fmaf(sv_r, d_r, fmaf(sv_t, d_t, vc));
    bw = fmaf(sw_r, d_r, fmaf(sw_t, d_t, wc));
}

template <int DIV, bool WCHECK>
__device__ __forceinline__ void voxel_coords(float bu, float bv, float bw, float su2, float sv2,
                                             float sw2, float zi, float& u, float& v, float& r)
{
    const float uw = fmaf(zi, su2, bu);
    const float vw = fmaf(zi, sv2, bv);
    const float w = fmaf(zi, sw2, bw);
    if constexpr (DIV == kDivIEEE) {
        r = 1.0f / w;
        u = uw / w;
        v = vw / w;
    } else {
        r = __builtin_amdgcn_rcpf(w);
        if constexpr (DIV == kDivRcpNR) r = fmaf(fmaf(-w, r, 1.0f), r, r);
        if constexpr (DIV == kDivRcp12)
            r = __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, r) & 0xfffff000u);
        u = uw * r;
        v = vw * r;
    }
    if (WCHECK) {
        r = (w > 0.0f) ? r : 0.0f;
        u = (w > 0.0f) ? u : 0.0f;
        v = (w > 0.0f) ? v : 0.0f;
    }
}

}  // namespace fdk
