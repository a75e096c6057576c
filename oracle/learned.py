"""FP64 oracle of the learned Feldkamp filter (test infrastructure).

Plain definitions of the model the GPU trains (see the description of the
learned filter in the package): a fixed cosine x Parker weighting, a row
convolution with taps h = M theta (theta: a real frequency response on the
bins of a 2048-point DFT), per-view weights, and a residual 1D CNN of three
9-tap convolutions (1 -> 32 -> 32 -> 1 channels, ReLU between), followed by
the backprojection (the FP64 backprojection oracle).  The loss is the mean
squared error inside a mask.

The backward pass is written out by hand from the chain rule: the adjoint of
a row convolution is the correlation with the same taps, the adjoint of the
backprojection is the oracle's exact transpose.  Tests pin it to central
finite differences of the forward pass.
"""
from __future__ import annotations

import math

import numpy as np

from . import backproject, forward_project
from .prefilter import parker

FFT_LEN = 2048
N_BINS = 1024


def conv(x, w, b, pad):
    """out[r, co, j] = b[co] + sum_{ci, t} w[co, ci, t] x[r, ci, j + t - pad],
    x zero outside [0, W).  x: (R, Cin, W), w: (Cout, Cin, K)."""
    R, Cin, W = x.shape
    Cout, _, K = w.shape
    xp = np.zeros((R, Cin, W + K - 1))
    lo = max(0, pad)
    # xp[:, :, s] = x[:, :, s - pad]
    src0 = max(0, -pad)
    n = min(W - src0, W + K - 1 - lo)
    xp[:, :, lo:lo + n] = x[:, :, src0:src0 + n]
    out = np.zeros((R, Cout, W))
    if b is not None:
        out += np.asarray(b)[None, :, None]
    for t in range(K):
        out += np.einsum("oc,rcj->roj", w[:, :, t], xp[:, :, t:t + W])
    return out


def conv_adjoint(dy, w, pad):
    """Adjoint of conv(., w, None, pad): dx[r, ci, s] = sum_{co, t} w[co, ci, t]
    dy[r, co, s - t + pad]."""
    R, Cout, W = dy.shape
    _, Cin, K = w.shape
    dx = np.zeros((R, Cin, W))
    for t in range(K):
        shift = t - pad  # out[j] reads x[j + shift]
        for j in range(W):
            s = j + shift
            if 0 <= s < W:
                dx[:, :, s] += np.einsum("oc,ro->rc", w[:, :, t], dy[:, :, j])
    return dx


def conv_wgrad(dy, x, K, pad):
    """dW[co, ci, t] = sum_{r, j} dy[r, co, j] x[r, ci, j + t - pad]; db = sum dy."""
    R, Cin, W = x.shape
    Cout = dy.shape[1]
    dW = np.zeros((Cout, Cin, K))
    for t in range(K):
        shift = t - pad
        j0, j1 = max(0, -shift), min(W, W - shift)
        if j1 > j0:
            dW[:, :, t] = np.einsum("roj,rcj->oc", dy[:, :, j0:j1], x[:, :, j0 + shift:j1 + shift])
    return dW, dy.sum(axis=(0, 2))


def weights(betas, H, W, sid, sdd, pixel, arc):
    a = (np.arange(W) - 0.5 * (W - 1)) * pixel
    b = (np.arange(H) - 0.5 * (H - 1)) * pixel
    cosw = sdd / np.sqrt(sdd ** 2 + a[None, :] ** 2 + b[:, None] ** 2)
    gamma = -np.arctan(a / sdd)
    delta = 0.5 * (arc - math.pi)
    return np.stack([cosw * parker(float(bt), gamma, delta)[None, :] for bt in betas])


def ramp_map(W, tau, dbeta):
    """M (2W-1, 1025): h[n] = sum_k M[n, k] theta_k for n = -(W-1) .. W-1,
    the inverse real DFT of a real, even response (theta = response * tau^2),
    times the quadrature factor tau * dbeta."""
    L = FFT_LEN
    n = np.arange(-(W - 1), W)[:, None]
    k = np.arange(L // 2 + 1)[None, :]
    c = np.where((k == 0) | (k == L // 2), 1.0, 2.0)
    return c * np.cos(2 * math.pi * n * k / L) / L * (dbeta / tau)


def ramlak_theta(W, tau):
    """theta of the Ram-Lak taps (zero beyond |n| = W-1), by a direct DFT."""
    L = FFT_LEN
    n = np.arange(-(W - 1), W)
    h = np.where(n == 0, 1.0 / (4 * tau * tau),
                 np.where(n % 2 != 0, -1.0 / (np.maximum(np.abs(n), 1) * math.pi * tau) ** 2, 0.0))
    k = np.arange(L // 2 + 1)
    H = (h[None, :] * np.cos(2 * math.pi * np.outer(k, n) / L)).sum(axis=1)
    return H * tau * tau


def forward(params, p, T, M, P, N, vs, origin, sigma):
    """FP64 forward pass; returns (vol, cache)."""
    V, H, W = p.shape
    K = 2 * W - 1
    x0 = p * T
    h = M @ params["theta"]
    y1 = conv(x0.reshape(V * H, 1, W), h[None, None, :], None, W - 1).reshape(V, H, W)
    y2 = y1 * params["lam"][:, None, None]
    z = (y2 / sigma).reshape(V * H, 1, W)
    a1 = np.maximum(conv(z, params["W1"], params["b1"], 4), 0.0)
    a2 = np.maximum(conv(a1, params["W2"], params["b2"], 4), 0.0)
    c = conv(a2, params["W3"], params["b3"], 4).reshape(V, H, W)
    y3 = y2 + sigma * c
    # the backprojection oracle takes FP32 projections; it is linear, so two
    # calls on the FP32 head and tail of y3 give its FP64 result
    hi = y3.astype(np.float32)
    lo = (y3 - hi).astype(np.float32)
    vol = backproject(hi, P, N, vs, origin) + backproject(lo, P, N, vs, origin)
    return vol, dict(x0=x0, y1=y1, z=z, a1=a1, a2=a2, y3=y3, K=K)


def loss_and_grads(params, p, T, M, P, N, vs, origin, sigma, gt, mask):
    """Masked MSE (mean over all N^3 voxels) and FP64 gradients."""
    V, H, W = p.shape
    vol, c = forward(params, p, T, M, P, N, vs, origin, sigma)
    d = (vol - gt) * mask
    loss = float(np.mean(d * d))
    dvol = 2.0 * d * mask / d.size
    dy3 = forward_project(dvol, P, H, W, vs, origin)
    g = {}
    dc = (sigma * dy3).reshape(V * H, 1, W)
    g["W3"], g["b3"] = conv_wgrad(dc, c["a2"], 9, 4)
    da2 = conv_adjoint(dc, params["W3"], 4) * (c["a2"] > 0)
    g["W2"], g["b2"] = conv_wgrad(da2, c["a1"], 9, 4)
    da1 = conv_adjoint(da2, params["W2"], 4) * (c["a1"] > 0)
    g["W1"], g["b1"] = conv_wgrad(da1, c["z"], 9, 4)
    dz = conv_adjoint(da1, params["W1"], 4).reshape(V, H, W)
    dy2 = dy3 + dz / sigma
    g["lam"] = (dy2 * c["y1"]).sum(axis=(1, 2))
    dy1 = dy2 * params["lam"][:, None, None]
    dh, _ = conv_wgrad(dy1.reshape(V * H, 1, W), c["x0"].reshape(V * H, 1, W), c["K"], W - 1)
    g["theta"] = M.T @ dh[0, 0]
    g["theta"][N_BINS:] = 0.0
    return loss, g
