"""Pins for the FP64 oracle of the Feldkamp pre-processing (CPU only)."""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import prefilter as opf


def test_direct_convolution_matches_fft_generator():
    """Two independent algorithms for the same filter: the oracle's direct
    linear convolution and the input generator's zero-padded FFT (computed in
    FP64, stored FP32)."""
    g = synth.cone_beam_geometry(n_views=10, H=30, W=80, pixel=3.0)
    li = synth.line_integrals(g, synth.ellipsoid_phantom())
    ref = opf.fdk_prefilter(li, g.betas, 0.5 * (g.arc - math.pi), g.dbeta, g.sid, g.sdd, g.pixel)
    got = synth.fdk_prefilter(li.copy(), g)
    assert np.abs(got - ref).max() <= 2.0 ** -22 * np.abs(ref).max()


def test_parker_weights_sum_to_one_over_conjugate_rays():
    """Ray (beta, gamma) and its conjugate (beta + pi + 2 gamma, -gamma)
    measure the same line; their weights sum to 1 (Parker's condition)."""
    delta = math.radians(10.0)
    gam = np.linspace(-math.radians(9.0), math.radians(9.0), 37)
    for beta in np.linspace(0.0, math.pi + 2 * delta, 101):
        w = opf.parker(beta, gam, delta)
        bc = beta + math.pi + 2 * gam
        inside = bc <= math.pi + 2 * delta
        wc = np.array([opf.parker(b, np.array([-g_]), delta)[0] for b, g_ in zip(bc, gam)])
        np.testing.assert_allclose((w + wc)[inside], 1.0, atol=1e-12)


def test_ramlak_kernel_has_vanishing_dc():
    """sum_n h[n] -> 0: h[0] = 1/(4 tau^2) cancels 2 sum_{odd n} 1/(n pi tau)^2
    = 2/(pi tau)^2 * pi^2/8 (the ramp filter removes the mean)."""
    tau = 0.3
    h = opf.ramlak(20001, tau)
    assert abs(h.sum()) * tau * tau < 1e-4
    assert h[20000] == pytest.approx(1 / (4 * tau * tau))


def test_oracle_fbp_of_uniform_sphere():
    g = synth.cone_beam_geometry(n_views=120, H=240, W=312, pixel=1.232, jitter_mm=0.0)
    mu = 0.02
    li = synth.line_integrals(g, synth.sphere_phantom(60.0, mu))
    q = opf.fdk_prefilter(li, g.betas, 0.5 * (g.arc - math.pi), g.dbeta, g.sid, g.sdd, g.pixel)
    xs = np.arange(20, 109, 8)
    mid = np.full_like(xs, 64)
    r = oracle.backproject_points(q.astype(np.float32), g.P, 129, 1.0, (-64.0,) * 3,
                                  np.stack([xs, mid, mid], 1))
    np.testing.assert_allclose(r / mu, 1.0, atol=5e-3)
