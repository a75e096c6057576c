"""Pins for the FP64 oracle of the learned filter (CPU only).

The hand-written backward pass is checked against central finite
differences of the forward pass for every parameter group, and the ramp
parametrisation against the Ram-Lak taps it must reproduce at
initialisation (then the model is plain FBP)."""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import learned as L
from oracle import prefilter as opf


def tiny_case(seed=0):
    g = synth.cone_beam_geometry(n_views=3, H=5, W=9, pixel=30.0)
    rng = np.random.default_rng(seed)
    V, H, W = 3, 5, 9
    p = rng.uniform(0.0, 2.0, (V, H, W))
    T = L.weights(g.betas, H, W, g.sid, g.sdd, g.pixel, g.arc)
    tau = g.pixel * g.sid / g.sdd
    M = L.ramp_map(W, tau, g.dbeta)
    params = dict(theta=L.ramlak_theta(W, tau) * (1 + 0.1 * rng.standard_normal(1025)),
                  lam=1 + 0.1 * rng.standard_normal(V),
                  W1=rng.standard_normal((32, 1, 9)) * 0.4, b1=rng.standard_normal(32) * 0.1,
                  W2=rng.standard_normal((32, 32, 9)) * 0.08, b2=rng.standard_normal(32) * 0.1,
                  W3=rng.standard_normal((1, 32, 9)) * 0.08, b3=rng.standard_normal(1) * 0.1)
    N = 6
    vs, o = 20.0, (-50.0, -50.0, -50.0)
    gt = rng.uniform(0.0, 1e-3, (N, N, N))
    mask = (rng.uniform(size=(N, N, N)) > 0.2).astype(np.float64)
    return g, p, T, M, params, N, vs, o, gt, mask


def test_ramp_parametrisation_reproduces_ramlak():
    W, tau, dbeta = 40, 0.2, 0.01
    M = L.ramp_map(W, tau, dbeta)
    h = M @ L.ramlak_theta(W, tau)
    ref = opf.ramlak(W, tau) * tau * dbeta
    np.testing.assert_allclose(h, ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())


def test_conv_adjoint_and_wgrad_definitions():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((4, 3, 11))
    w = rng.standard_normal((2, 3, 5))
    dy = rng.standard_normal((4, 2, 11))
    # <conv(x), dy> = <x, conv_adjoint(dy)>
    lhs = np.sum(L.conv(x, w, None, 2) * dy)
    rhs = np.sum(x * L.conv_adjoint(dy, w, 2))
    assert lhs == pytest.approx(rhs, rel=1e-12)
    # d<conv(x; w, b), dy>/dw = wgrad, checked by finite differences
    dW, db = L.conv_wgrad(dy, x, 5, 2)
    e = np.zeros_like(w)
    e[1, 2, 3] = 1e-6
    fd = (np.sum(L.conv(x, w + e, None, 2) * dy) - np.sum(L.conv(x, w - e, None, 2) * dy)) / 2e-6
    assert fd == pytest.approx(dW[1, 2, 3], rel=1e-6)
    b = rng.standard_normal(2)
    fdb = (np.sum(L.conv(x, w, b + [1e-6, 0], 2) * dy) - np.sum(L.conv(x, w, b - [1e-6, 0], 2) * dy)) / 2e-6
    assert fdb == pytest.approx(db[0], rel=1e-6)
    # the conv definition against numpy's correlate for one channel
    y = L.conv(x[:1, :1], w[:1, :1], None, 2)[0, 0]
    ref = np.correlate(np.pad(x[0, 0], (2, 2)), w[0, 0], mode="valid")
    np.testing.assert_allclose(y, ref, rtol=1e-12)


GROUPS = ["theta", "lam", "W1", "b1", "W2", "b2", "W3", "b3"]


@pytest.mark.parametrize("group", GROUPS)
def test_model_gradient_finite_differences(group):
    g, p, T, M, params, N, vs, o, gt, mask = tiny_case()
    sigma = 1e-3
    loss, grads = L.loss_and_grads(params, p, T, M, g.P, N, vs, o, sigma, gt, mask)
    # a fixed direction per parameter group (the same in every process)
    rng = np.random.default_rng(101 + GROUPS.index(group))
    d = rng.standard_normal(params[group].shape)
    if group == "theta":
        d[L.N_BINS:] = 0.0
    # small steps: the ReLUs make the loss piecewise smooth, and a step that
    # crosses a kink biases the difference quotient
    scale = np.abs(params[group]).max() if group not in ("b1", "b2", "b3") else 0.1
    eps = 1e-7 * scale

    def f(s):
        q = dict(params)
        q[group] = params[group] + s * eps * d
        vol, _ = L.forward(q, p, T, M, g.P, N, vs, o, sigma)
        dd = (vol - gt) * mask
        return float(np.mean(dd * dd))
    fd = (f(1.0) - f(-1.0)) / (2 * eps)
    an = float(np.sum(grads[group] * d))
    assert abs(an) > 0
    assert fd == pytest.approx(an, rel=1e-4)
