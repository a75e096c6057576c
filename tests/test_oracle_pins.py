"""Pins for the FP64 oracle against facts the paper and the mathematics fix.

Each test computes its expectation without the oracle's formula:
geometry comes from explicit ray/plane intersection (synth.ray_plane_project),
interpolation from the tent-function form of bilinear interpolation
(sum over pixels of I[k][j] * hat(u - j) * hat(v - k), hat(t) = max(0, 1-|t|)),
which needs neither a floor nor a special case at the detector edge.

What the pins cover (a plausible mistake and the test that catches it):
  - transposed or column-major matrix, wrong w scale, wrong pixel centre:
    affine image, single pixel, hand-computed isocentre;
  - dropped 1/w^2 or 1/w instead: constant and affine images;
  - truncation instead of floor, missing zero extension, clamping instead
    of zeros: single pixel at the detector edge, explicit transpose;
  - swapped u/v, swapped bilinear weights: single pixel, affine image;
  - overwrite instead of accumulate: accumulate test.
"""
import numpy as np
import pytest

import oracle
import synth


def hat(t):
    return np.maximum(0.0, 1.0 - np.abs(t))


def tent_backproject_points(proj, geom, views, X):
    """Backprojection at world points X (n,3) by the tent form, with
    (u, v, w) from ray/plane intersection."""
    out = np.zeros(len(X))
    V, H, W = proj.shape
    jj = np.arange(W)
    kk = np.arange(H)
    for n, i in enumerate(views):
        u, v, w = synth.ray_plane_project(geom, i, X)
        for p in range(len(X)):
            if w[p] <= 0:
                continue
            wu = hat(u[p] - jj)
            wv = hat(v[p] - kk)
            out[p] += (wv @ proj[n].astype(np.float64) @ wu) / w[p] ** 2
    return out


def tent_forward_bruteforce(vol, P, H, W, vs, origin):
    """Per-pixel ("ray-driven") enumeration: F[i][k][j] = sum over voxels of
    vol * hat(u - j) * hat(v - k) / w^2.  O(pixels x voxels): tiny grids."""
    N = vol.shape[0]
    z, y, x = np.indices((N, N, N)).reshape(3, -1)
    X = np.stack([origin[0] + vs * x, origin[1] + vs * y, origin[2] + vs * z, np.ones(x.size)])
    f = vol.reshape(-1)
    F = np.zeros((len(P), H, W))
    for i, A in enumerate(np.asarray(P).reshape(-1, 3, 4)):
        uw, vw, w = A @ X
        ok = w > 0
        u = np.where(ok, uw / np.where(ok, w, 1), 0)
        v = np.where(ok, vw / np.where(ok, w, 1), 0)
        g = np.where(ok, f / np.where(ok, w, 1) ** 2, 0)
        for k in range(H):
            for j in range(W):
                F[i, k, j] = np.sum(g * hat(u - j) * hat(v - k))
    return F


def world(idx, vs, origin):
    idx = np.asarray(idx, dtype=np.float64)
    return np.asarray(origin) + vs * idx


# ---------------------------------------------------------------------------
def test_isocentre_voxel_lands_on_centre_pixel():
    """Odd detector (9x7) and odd grid: the isocentre voxel projects onto
    pixel (4, 3) with w = 1 in every unjittered view, so the result is the
    plain sum of that pixel over the views."""
    g = synth.cone_beam_geometry(n_views=11, H=7, W=9, pixel=20.0, jitter_mm=0.0)
    rng = np.random.default_rng(1)
    proj = np.zeros((11, 7, 9), np.float32)
    proj[:, 3, 4] = rng.uniform(-1, 1, 11).astype(np.float32)
    R = oracle.backproject(proj, g.P, 5, 2.0, (-4.0, -4.0, -4.0), box=((2, 1), (2, 1), (2, 1)))
    assert R[0, 0, 0] == pytest.approx(proj[:, 3, 4].astype(np.float64).sum(), rel=1e-12)


def test_constant_image_closed_form():
    """I = kappa everywhere -> R = kappa * sum_i 1/w_i^2 for voxels whose
    four taps are inside the detector; kappa * V at the isocentre."""
    g = synth.cone_beam_geometry(n_views=24)
    kappa = 0.75
    proj = np.full((24, g.H, g.W), kappa, np.float32)
    N, vs = 16, 16.0
    o = (-120.0,) * 3
    rng = np.random.default_rng(2)
    idx = rng.integers(0, N, size=(40, 3))
    X = world(idx, vs, o)
    R = oracle.backproject_points(proj, g.P, N, vs, o, idx)
    for p in range(len(idx)):
        want, interior = 0.0, True
        for i in range(24):
            u, v, w = synth.ray_plane_project(g, i, X[p:p + 1])
            interior &= bool(0 <= u[0] <= g.W - 1 and 0 <= v[0] <= g.H - 1)
            want += kappa / w[0] ** 2
        if interior:
            assert R[p] == pytest.approx(want, rel=1e-12)
    g0 = synth.cone_beam_geometry(n_views=24, jitter_mm=0.0)
    r0 = oracle.backproject_points(proj, g0.P, 3, 1.0, (-1.0, -1.0, -1.0), [[1, 1, 1]])
    assert r0[0] == pytest.approx(kappa * 24, rel=1e-12)


def test_affine_image_closed_form():
    """Bilinear interpolation reproduces an affine image exactly, so
    I(j, k) = a + b j + c k gives R = sum_i (a + b u_i + c v_i) / w_i^2 with
    (u_i, v_i, w_i) from ray/plane geometry (pins matrix order, pixel
    centres and the w scale)."""
    g = synth.cone_beam_geometry(n_views=16)
    a, b, c = 0.25, 1.5e-3, -2.5e-3
    jj, kk = np.meshgrid(np.arange(g.W), np.arange(g.H))
    img = (a + b * jj + c * kk).astype(np.float32)
    proj = np.broadcast_to(img, (16, g.H, g.W)).copy()
    N, vs, o = 32, 4.0, (-62.0, -62.0, -62.0)
    rng = np.random.default_rng(3)
    idx = rng.integers(0, N, size=(25, 3))
    X = world(idx, vs, o)
    R = oracle.backproject_points(proj, g.P, N, vs, o, idx)
    want = np.zeros(len(X))
    for i in range(16):
        u, v, w = synth.ray_plane_project(g, i, X)
        assert np.all((u > 0) & (u < g.W - 1) & (v > 0) & (v < g.H - 1))
        want += (a + b * u + c * v) / w ** 2
    np.testing.assert_allclose(R, want, rtol=2e-6)  # FP32 rounding of the image values
    # exact up to FP64 rounding against the tent form of the FP32-rounded image
    np.testing.assert_allclose(R, tent_backproject_points(proj, g, range(16), X), rtol=1e-11)


def test_single_pixel_hat_and_floor_at_detector_edge():
    """A one-pixel image at column 0 lights voxels whose u is in (-1, 1):
    for u in (-1, 0) floor gives iu = -1 and weight u + 1 on column 0, while
    truncation would give iu = 0 and weight 1 - u (an extrapolation).  Also checks the top
    edge row and the hat shape in v."""
    g = synth.cone_beam_geometry(n_views=1, H=7, W=9, pixel=1.0, jitter_mm=0.0)
    proj = np.zeros((1, 7, 9), np.float32)
    proj[0, 0, 0] = 1.0
    # beta = 0: u = 4 + y * 1.6, v = 3 + z * 1.6 at x = 0
    ys = np.array([-3.0, -2.9, -2.75, -2.6, -2.5, -2.2, -2.0, -1.9])
    zs = np.array([-2.1, -1.9, -1.75, -1.6])
    X = np.array([[0.0, y, z] for y in ys for z in zs])
    got = np.array([oracle.backproject_points(proj, g.P, 1, 1.0, tuple(x), [[0, 0, 0]])[0]
                    for x in X])
    u, v, w = synth.ray_plane_project(g, 0, X)
    want = hat(u - 0) * hat(v - 0) / w ** 2
    assert np.any((u > -1) & (u < 0) & (want > 0))
    np.testing.assert_allclose(got, want, atol=1e-13)
    trunc = np.where((u > -1) & (u < 0), 1 - u, hat(u)) * hat(v) / w ** 2
    assert not np.allclose(got, trunc, atol=1e-6)


def test_explicit_transpose_against_bruteforce():
    """Assemble the backprojection operator column by column (one pixel
    basis image at a time) and compare it element by element with the
    brute-force per-pixel forward projector in tent form: B = F^T."""
    g = synth.cone_beam_geometry(n_views=3, H=5, W=7, pixel=12.0)
    N, vs, o = 4, 9.0, (-13.5, -13.5, -13.5)
    V, H, W = 3, 5, 7
    rng = np.random.default_rng(4)
    vol = rng.uniform(-1, 1, (N, N, N))
    F = tent_forward_bruteforce(vol, g.P, H, W, vs, o)
    B = np.zeros((V * H * W, N ** 3))
    for q in range(V * H * W):
        e = np.zeros(V * H * W, np.float32)
        e[q] = 1.0
        B[q] = oracle.backproject(e.reshape(V, H, W), g.P, N, vs, o).reshape(-1)
    np.testing.assert_allclose(B @ vol.reshape(-1), F.reshape(-1), rtol=1e-12, atol=1e-13)
    # and the oracle's own transpose equals the brute force element-wise
    Fo = oracle.forward_project(vol, g.P, H, W, vs, o)
    np.testing.assert_allclose(Fo, F, rtol=1e-12, atol=1e-13)
    assert np.count_nonzero(F) > 20 and np.count_nonzero(F == 0) > 0  # edge pixels exercised


def test_adjoint_dot_product_identity():
    """<B p, x> = <p, F x> with F the brute-force per-pixel projector."""
    g = synth.cone_beam_geometry(n_views=4, H=6, W=8, pixel=9.0)
    N, vs, o = 5, 7.0, (-14.0, -14.0, -14.0)
    rng = np.random.default_rng(5)
    p = rng.uniform(-1, 1, (4, 6, 8)).astype(np.float32)
    x = rng.uniform(-1, 1, (N, N, N))
    Bp = oracle.backproject(p, g.P, N, vs, o)
    Fx = tent_forward_bruteforce(x, g.P, 6, 8, vs, o)
    lhs = float(np.sum(Bp * x))
    rhs = float(np.sum(p.astype(np.float64) * Fx))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_random_voxels_match_tent_form_on_real_geometry():
    g = synth.cone_beam_geometry(n_views=6)
    rng = np.random.default_rng(6)
    proj = rng.standard_normal((6, g.H, g.W)).astype(np.float32)
    N = 64
    vs, o = synth.volume_frame(N)
    idx = rng.integers(0, N, size=(12, 3))
    idx[0] = (0, 0, 0)
    idx[1] = (N - 1, N - 1, N - 1)  # corners: partly off the detector
    got = oracle.backproject_points(proj, g.P, N, vs, o, idx)
    want = tent_backproject_points(proj, g, range(6), world(idx, vs, o))
    np.testing.assert_allclose(got, want, rtol=1e-10, atol=1e-12)


def test_nonpositive_w_contributes_nothing():
    """A matrix whose third row is w = z (mm): voxels with z <= 0 are not
    in front of the source and must receive nothing."""
    P = np.array([[[1.0, 0.0, 0.0, 2.0], [0.0, 1.0, 0.0, 2.0], [0.0, 0.0, 1.0, 0.0]]])
    proj = np.ones((1, 5, 5), np.float32)
    R = oracle.backproject(proj, P, 4, 1.0, (0.0, 0.0, -1.5))
    assert np.all(R[:2] == 0.0)  # z = -1.5, -0.5
    assert np.all(R[2:].sum(axis=(1, 2)) > 0)


def test_accumulates_and_box_matches_full_volume():
    g = synth.cone_beam_geometry(n_views=5)
    rng = np.random.default_rng(8)
    proj = rng.standard_normal((5, g.H, g.W)).astype(np.float32)
    N = 24
    vs, o = synth.volume_frame(N)
    full = oracle.backproject(proj, g.P, N, vs, o)
    box = oracle.backproject(proj, g.P, N, vs, o, box=((3, 7), (10, 5), (17, 7)))
    np.testing.assert_array_equal(box, full[17:24, 10:15, 3:10])
    pts = np.array([[3, 10, 17], [23, 0, 5], [12, 12, 12]])
    np.testing.assert_array_equal(oracle.backproject_points(proj, g.P, N, vs, o, pts),
                                  full[pts[:, 2], pts[:, 1], pts[:, 0]])
    twice = oracle.backproject(proj, g.P, N, vs, o, out=full.copy())
    np.testing.assert_allclose(twice, 2 * full, rtol=1e-15)
    split = oracle.backproject(proj[:2], g.P[:2], N, vs, o)
    split = oracle.backproject(proj[2:], g.P[2:], N, vs, o, out=split)
    np.testing.assert_allclose(split, full, rtol=1e-12, atol=1e-15)


def test_oracle_rejects_bad_arguments():
    g = synth.cone_beam_geometry(n_views=2, H=4, W=4, pixel=50.0)
    proj = np.zeros((2, 4, 4), np.float32)
    with pytest.raises(ValueError):
        oracle.backproject(proj, g.P, 4, 1.0, (0, 0, 0), box=((0, 5), (0, 4), (0, 4)))
    with pytest.raises(ValueError):
        oracle.backproject(proj, g.P[:1], 4, 1.0, (0, 0, 0))
    with pytest.raises(ValueError):
        oracle.backproject_points(proj, g.P, 4, 1.0, (0, 0, 0), [[0, 0, 4]])


def test_metrics():
    R = np.array([0.0, 1.0, 2.0, 3.0])
    assert oracle.rel_rmse(R, R) == 0.0
    assert oracle.rel_rmse(R * 1.01, R) == pytest.approx(0.01)
    # PSNR with range M = 3 and MSE 0.01: 10 log10(9 / 0.01)
    assert oracle.psnr(R + np.array([0.1, -0.1, 0.1, -0.1]), R) == pytest.approx(
        10 * np.log10(900.0))
