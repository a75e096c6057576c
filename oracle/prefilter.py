"""FP64 oracle of the Feldkamp 2D pre-processing (test infrastructure).

Plain definitions, in the order the Feldkamp method applies them to a line
integral p(beta, a, b) on a flat detector (a, b: mm from the detector centre):
  1. cosine weight  sdd / sqrt(sdd^2 + a^2 + b^2);
  2. Parker's short-scan redundancy weight w(beta, gamma) over pi + 2*delta,
     gamma = -atan(a / sdd) (1/2 for a full circle);
  3. row-wise linear convolution with the discrete Ram-Lak kernel sampled at
     the isocentre spacing tau = pixel * sid / sdd:
       h[0] = 1 / (4 tau^2),  h[n odd] = -1 / (n pi tau)^2,  h[n even] = 0;
  4. the quadrature factor tau * dbeta.
The convolution is np.convolve over the full row (a library primitive used
as one step); no FFT, no blocking.
"""
from __future__ import annotations

import math

import numpy as np


def parker(beta: float, gamma: np.ndarray, delta: float) -> np.ndarray:
    """Parker weight for one source angle and an array of fan angles."""
    if delta < 0:
        return np.full_like(gamma, 0.5)
    w = np.zeros_like(gamma)
    r1 = beta < 2 * (delta - gamma)
    r2 = (~r1) & (beta < math.pi - 2 * gamma)
    r3 = (~r1) & (~r2) & (beta <= math.pi + 2 * delta)
    if beta >= 0:
        w[r1] = np.sin(0.25 * math.pi * beta / (delta - gamma[r1])) ** 2
    w[r2] = 1.0
    w[r3] = np.sin(0.25 * math.pi * (math.pi + 2 * delta - beta) / (delta + gamma[r3])) ** 2
    return w


def ramlak(W: int, tau: float) -> np.ndarray:
    """Taps h[n] for n = -(W-1) .. W-1."""
    n = np.arange(-(W - 1), W)
    h = np.zeros(n.shape)
    h[n == 0] = 1.0 / (4.0 * tau * tau)
    odd = (n % 2) != 0
    h[odd] = -1.0 / (n[odd] * math.pi * tau) ** 2
    return h


def fdk_prefilter(p, betas, delta: float, dbeta: float, sid: float, sdd: float,
                  pixel: float) -> np.ndarray:
    """FP64 pre-filtered projections of line integrals p (V, H, W)."""
    p = np.asarray(p, dtype=np.float64)
    V, H, W = p.shape
    a = (np.arange(W) - 0.5 * (W - 1)) * pixel
    b = (np.arange(H) - 0.5 * (H - 1)) * pixel
    cosw = sdd / np.sqrt(sdd ** 2 + a[None, :] ** 2 + b[:, None] ** 2)
    gamma = -np.arctan(a / sdd)
    tau = pixel * sid / sdd
    h = ramlak(W, tau)
    out = np.empty_like(p)
    for i in range(V):
        q = p[i] * cosw * parker(float(betas[i]), gamma, delta)[None, :]
        for k in range(H):
            out[i, k] = np.convolve(q[k], h, mode="full")[W - 1:2 * W - 1]
    return out * (tau * dbeta)
