"""Pins for the seeded input generator (geometry, phantom, FDK pre-filter).

The generator is not the method, but every GPU and oracle result is taken
on its output, so its geometry is pinned to hand-computed projections and
an explicit ray/plane intersection, and its phantom and filter to closed
forms.
"""
import math
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "geometry_points.txt")


def _golden_rows():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append([float(t) for t in line.split()])
    return rows


def test_geometry_hand_computed_points():
    # 21 views over 200 degrees: beta = 0, 10, ..., 200 degrees
    g = synth.cone_beam_geometry(n_views=21, jitter_mm=0.0)
    for beta, x, y, z, u, v, w in _golden_rows():
        i = int(round(beta / 10.0))
        assert abs(math.degrees(g.betas[i]) - beta) < 1e-12
        h = g.P[i] @ np.array([x, y, z, 1.0])
        assert h[2] == pytest.approx(w, rel=1e-13, abs=1e-13)
        assert h[0] / h[2] == pytest.approx(u, abs=1e-9)
        assert h[1] / h[2] == pytest.approx(v, abs=1e-9)


def test_matrix_matches_ray_plane_intersection():
    g = synth.cone_beam_geometry(n_views=40)  # jittered
    rng = np.random.default_rng(7)
    X = rng.uniform(-128.0, 128.0, size=(200, 3))
    Xh = np.c_[X, np.ones(len(X))]
    for i in range(g.n_views):
        u, v, w = synth.ray_plane_project(g, i, X)
        h = Xh @ g.P[i].T
        np.testing.assert_allclose(h[:, 2], w, rtol=1e-13, atol=1e-13)
        np.testing.assert_allclose(h[:, 0] / h[:, 2], u, rtol=0, atol=1e-9)
        np.testing.assert_allclose(h[:, 1] / h[:, 2], v, rtol=0, atol=1e-9)


def test_jitter_is_bounded_and_seeded():
    g0 = synth.cone_beam_geometry(n_views=50, jitter_mm=0.0)
    g1 = synth.cone_beam_geometry(n_views=50)
    g2 = synth.cone_beam_geometry(n_views=50)
    d_src = g1.src - g0.src
    d_det = g1.det - g0.det
    assert np.all(np.abs(d_src) <= 0.5) and np.all(np.abs(d_det) <= 0.5)
    assert np.abs(d_src).max() > 0.3
    np.testing.assert_array_equal(g1.P, g2.P)


def test_splitmix64_reference_values():
    # first outputs for seed 0 of the published splitmix64 generator
    r = synth.SplitMix64(0)
    assert r.next_u64() == 0xE220A8397B1DCDAF
    assert r.next_u64() == 0x6E789E6AA1B965F4
    assert r.next_u64() == 0x06C45D188009454F


def test_sphere_chord_closed_form():
    g = synth.cone_beam_geometry(n_views=3, H=31, W=41, pixel=2.0, jitter_mm=0.0)
    r0 = 50.0
    c = np.array([5.0, -3.0, 2.0])
    p = synth.line_integrals(g, synth.sphere_phantom(r0, 1.0, c))
    for i in range(g.n_views):
        s = g.src[i]
        for k in range(0, g.H, 5):
            for j in range(0, g.W, 4):
                pt = (g.det[i] + (j - 20) * 2.0 * g.eu[i] + (k - 15) * 2.0 * g.ev[i])
                d = (pt - s) / np.linalg.norm(pt - s)
                dist = np.linalg.norm(np.cross(c - s, d))
                want = 2.0 * math.sqrt(r0 * r0 - dist * dist) if dist < r0 else 0.0
                assert p[i, k, j] == pytest.approx(want, rel=1e-6, abs=1e-4)


def test_voxelize_sphere_volume():
    vs, o = synth.volume_frame(64)
    vol = synth.voxelize(synth.sphere_phantom(60.0, 1.0), 64, vs, o, sub=2)
    # 64^3 voxels of 4 mm: sum * voxel volume approximates 4/3 pi r^3
    got = vol.sum() * vs ** 3
    assert got == pytest.approx(4.0 / 3.0 * math.pi * 60.0 ** 3, rel=0.01)


def test_fdk_prefilter_reconstructs_uniform_sphere():
    """Textbook special case: FDK of a centred uniform sphere returns its
    density in the central plane (pins the filter's scale, the cosine and
    Parker weights, and the short-scan normalisation)."""
    g = synth.cone_beam_geometry(n_views=180, H=480, W=624, pixel=0.616, jitter_mm=0.0)
    mu = 0.02
    p = synth.filtered_projections(g, synth.sphere_phantom(60.0, mu))
    xs = np.arange(10, 119, 6)
    mid = np.full_like(xs, 64)
    for pts in (np.stack([xs, mid, mid], 1), np.stack([mid, xs, mid], 1)):
        r = oracle.backproject_points(p, g.P, 129, 1.0, (-64.0, -64.0, -64.0), pts)
        np.testing.assert_allclose(r / mu, 1.0, atol=2e-3)
    # along the rotation axis the cone-beam approximation loses < 1% inside
    r = oracle.backproject_points(p, g.P, 129, 1.0, (-64.0, -64.0, -64.0),
                                  np.stack([mid, mid, xs], 1))
    np.testing.assert_allclose(r / mu, 1.0, atol=1e-2)
