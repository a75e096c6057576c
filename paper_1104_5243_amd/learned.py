"""Learned Feldkamp filter: trainable ramp, per-view weights and a row CNN.

The plain Feldkamp reconstruction filters each view's line integrals p
along detector rows (cosine and Parker weights, Ram-Lak ramp) and
backprojects.  Here the filter gains trainable parts, all acting on rows:

    x0 = p * T                                 T: cosine x Parker weights (fixed)
    y1 = h (*) x0                              row convolution, h = M theta
    y2 = lambda_v * y1                         one weight per view
    z  = y2 / sigma
    a1 = relu(conv9(z;  W1, b1))               1 -> 32 channels
    a2 = relu(conv9(a1; W2, b2))               32 -> 32
    y3 = y2 + sigma * conv9(a2; W3, b3)        32 -> 1, residual
    vol = B(y3)                                the backprojection kernel

theta holds the ramp's frequency response on bins k = 0..1023 of a
2048-point DFT (times tau^2, dimensionless); the Nyquist bin is fixed to the
Ram-Lak value.  h spans the 2W-1 taps a linear convolution of a W-sample row
needs; M maps theta to them (the inverse real DFT).  At initialisation
(theta = Ram-Lak, lambda = 1, W3 = b3 = 0) the model is exactly plain FBP,
the baseline a trained filter is compared with.

Training minimises the mean squared error between vol and the voxelised
phantom inside the field of view.  The gradient of vol is mapped back by the
matched forward projector (the backprojection's exact adjoint), then through
the CNN, the view weights and the ramp, all by the library's kernels; Adam
updates the parameters.  torch only allocates memory.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from . import (CONV_RELU, CONV_RELU_MASK, CONV_TRANSPOSE, adam, backproject, conv_rows,
               conv_rows_wgrad, conv_rows_wgrad_workspace, forward_project, group_dot, matvec, mse,
               scale_groups)

FFT_LEN = 2048
N_BINS = 1024
CH = 32
KC = 9


@dataclass
class Geometry:
    """What the filter needs of the scan geometry."""
    P: np.ndarray        # (V, 3, 4) FP64 matrices
    betas: np.ndarray    # (V,) source angles, radians
    H: int
    W: int
    sid: float
    sdd: float
    pixel: float
    arc: float           # scan range, radians

    @property
    def V(self):
        return len(self.betas)

    @property
    def tau(self):
        return self.pixel * self.sid / self.sdd

    @property
    def dbeta(self):
        return self.arc / max(self.V - 1, 1)


def weight_table(g: Geometry) -> np.ndarray:
    """Cosine x Parker weights, (V, H, W), FP64."""
    a = (np.arange(g.W) - 0.5 * (g.W - 1)) * g.pixel
    b = (np.arange(g.H) - 0.5 * (g.H - 1)) * g.pixel
    cosw = g.sdd / np.sqrt(g.sdd ** 2 + a[None, :] ** 2 + b[:, None] ** 2)
    gamma = -np.arctan(a / g.sdd)
    delta = 0.5 * (g.arc - math.pi)
    T = np.empty((g.V, g.H, g.W))
    for i, beta in enumerate(g.betas):
        w = np.zeros(g.W)
        for j, gm in enumerate(gamma):
            if beta < 2 * (delta - gm):
                w[j] = math.sin(0.25 * math.pi * beta / (delta - gm)) ** 2
            elif beta < math.pi - 2 * gm:
                w[j] = 1.0
            elif beta <= math.pi + 2 * delta:
                w[j] = math.sin(0.25 * math.pi * (math.pi + 2 * delta - beta) / (delta + gm)) ** 2
        T[i] = cosw * w[None, :]
    return T


def ramp_basis(g: Geometry):
    """(M, theta0, theta_nyq): taps h = M @ [theta, theta_nyq] for offsets
    n = -(W-1) .. W-1, and the Ram-Lak initialisation of theta."""
    L = FFT_LEN
    W = g.W
    if 2 * W - 1 > L:
        # the 2W-1 taps would wrap around the L-periodic grid and alias
        raise ValueError(f"learned filter: detector rows of {W} pixels need more than "
                         f"{L} DFT bins (at most {(L + 1) // 2} pixels)")
    tau = g.tau
    n = np.arange(-(W - 1), W)
    # Ram-Lak taps on |n| <= W-1, zero elsewhere on the L-periodic grid
    h = np.zeros(L)
    idx = np.arange(-(W - 1), W)
    vals = np.where(idx == 0, 1.0 / (4 * tau * tau),
                    np.where(idx % 2 != 0, -1.0 / (np.maximum(np.abs(idx), 1) * math.pi * tau) ** 2,
                             0.0))
    h[idx % L] = vals
    H = np.fft.rfft(h).real                    # real: h is even
    k = np.arange(L // 2 + 1)
    c = np.where((k == 0) | (k == L // 2), 1.0, 2.0)
    # h[n] = (1/L) sum_k c_k H_k cos(2 pi k n / L), times tau * dbeta, with
    # theta = H tau^2
    M = (c[None, :] * np.cos(2 * math.pi * np.outer(n, k) / L) / L) * (g.dbeta / tau)
    theta = H * tau * tau
    return M, theta[:N_BINS], theta[N_BINS:]


class LearnedFilter:
    """Parameters, forward pass and gradients on one GPU."""

    def __init__(self, g: Geometry, device, seed: int = 0, sigma: float = None):
        self.g = g
        self.dev = device
        self.K = 2 * g.W - 1
        M, theta0, nyq = ramp_basis(g)
        self.M = torch.from_numpy(M.astype(np.float32)).to(device).contiguous()   # K x 1025
        self.theta = torch.zeros(N_BINS + 1, device=device)
        self.theta.copy_(torch.from_numpy(np.concatenate([theta0, nyq]).astype(np.float32)))
        self.T = torch.from_numpy(weight_table(g).astype(np.float32)).to(device).contiguous()
        self.lam = torch.ones(g.V, device=device)
        gen = torch.Generator().manual_seed(seed)
        self.W1 = (torch.randn(CH, 1, KC, generator=gen) * math.sqrt(2.0 / KC)).to(device)
        self.b1 = torch.zeros(CH, device=device)
        self.W2 = (torch.randn(CH, CH, KC, generator=gen) * math.sqrt(2.0 / (CH * KC))).to(device)
        self.b2 = torch.zeros(CH, device=device)
        self.W3 = torch.zeros(1, CH, KC, device=device)
        self.b3 = torch.zeros(1, device=device)
        self.sigma = float(sigma) if sigma else 1.0
        self.sigma_t = torch.tensor([1.0 / self.sigma], device=device)
        self.sigma_f = torch.tensor([self.sigma], device=device)
        self.params = ["theta", "lam", "W1", "b1", "W2", "b2", "W3", "b3"]
        self.adam_state = {n: (torch.zeros_like(getattr(self, n)), torch.zeros_like(getattr(self, n)))
                           for n in self.params}
        self.step_count = 0
        self.ws = torch.empty(max(conv_rows_wgrad_workspace(CH, CH, KC),
                                  conv_rows_wgrad_workspace(1, 1, self.K)) // 4 + 1,
                              dtype=torch.float32, device=device)
        self.ws_mse = torch.empty(2048 + 16, dtype=torch.float32, device=device)

    # -- pieces ------------------------------------------------------------
    def taps(self):
        h = torch.empty(self.K, device=self.dev)
        matvec(h, self.M, self.theta, self.K, N_BINS + 1)
        return h

    def filter(self, p, keep=False):
        """Filtered projections y3 (V, H, W) of line integrals p; with
        keep=True also the intermediates the backward pass needs."""
        g = self.g
        V, H, W = g.V, g.H, g.W
        R = V * H
        n = V * H * W
        x0 = torch.empty(V, H, W, device=self.dev)
        scale_groups(x0, p, self.T, 1, n)
        h = self.taps()
        y1 = torch.empty_like(x0)
        conv_rows(y1, x0, h, None, R, W, 1, 1, self.K, W - 1)
        y2 = torch.empty_like(x0)
        scale_groups(y2, y1, self.lam, H * W, V)
        z = torch.empty_like(x0)
        scale_groups(z, y2, self.sigma_t, n, 1)
        a1 = torch.empty(R, CH, W, device=self.dev)
        conv_rows(a1, z, self.W1, self.b1, R, W, 1, CH, KC, KC // 2, CONV_RELU)
        a2 = torch.empty(R, CH, W, device=self.dev)
        conv_rows(a2, a1, self.W2, self.b2, R, W, CH, CH, KC, KC // 2, CONV_RELU)
        c = torch.empty(V, H, W, device=self.dev)
        conv_rows(c, a2, self.W3, self.b3, R, W, CH, 1, KC, KC // 2)
        y3 = y2.clone()
        scale_groups(y3, c, self.sigma_f, n, 1, accumulate=True)
        if keep:
            return y3, dict(x0=x0, y1=y1, z=z, a1=a1, a2=a2)
        return y3

    def reconstruct(self, p, N, voxel_size, origin):
        y3 = self.filter(p)
        vol = torch.zeros(N, N, N, device=self.dev)
        backproject(vol, y3, self.g.P, voxel_size, origin)
        return vol

    # -- gradients -----------------------------------------------------------
    def loss_and_grads(self, p, gt_masked, mask, N, voxel_size, origin):
        """Masked MSE of the reconstruction and the gradient of every
        parameter (dict of tensors)."""
        g = self.g
        V, H, W = g.V, g.H, g.W
        R = V * H
        n = V * H * W
        y3, c = self.filter(p, keep=True)
        vol = torch.zeros(N, N, N, device=self.dev)
        backproject(vol, y3, g.P, voxel_size, origin)
        nv = N * N * N
        volm = torch.empty_like(vol)
        scale_groups(volm, vol, mask, 1, nv)
        dvol = torch.empty_like(vol)
        loss = torch.empty(1, device=self.dev)
        mse(dvol, loss, volm, gt_masked, self.ws_mse)
        scale_groups(dvol, dvol, mask, 1, nv)
        # back through the backprojection: its adjoint
        dy3 = torch.zeros(V, H, W, device=self.dev)
        forward_project(dy3, dvol, g.P, voxel_size, origin)
        grads = {}
        # CNN branch: y3 = y2 + sigma * conv3(a2)
        dc = torch.empty_like(dy3)
        scale_groups(dc, dy3, self.sigma_f, n, 1)
        grads["W3"] = torch.empty_like(self.W3)
        grads["b3"] = torch.empty_like(self.b3)
        conv_rows_wgrad(grads["W3"], grads["b3"], dc, c["a2"], R, W, CH, 1, KC, KC // 2, self.ws)
        # the ReLU's backward step rides on the data-gradient convolution,
        # which overwrites the activation it masks by (no longer needed)
        da2 = c.pop("a2")
        conv_rows(da2, dc, self.W3, None, R, W, 1, CH, KC, KC - 1 - KC // 2,
                  CONV_TRANSPOSE | CONV_RELU_MASK)
        grads["W2"] = torch.empty_like(self.W2)
        grads["b2"] = torch.empty_like(self.b2)
        conv_rows_wgrad(grads["W2"], grads["b2"], da2, c["a1"], R, W, CH, CH, KC, KC // 2, self.ws)
        da1 = c.pop("a1")
        conv_rows(da1, da2, self.W2, None, R, W, CH, CH, KC, KC - 1 - KC // 2,
                  CONV_TRANSPOSE | CONV_RELU_MASK)
        del da2
        grads["W1"] = torch.empty_like(self.W1)
        grads["b1"] = torch.empty_like(self.b1)
        conv_rows_wgrad(grads["W1"], grads["b1"], da1, c["z"], R, W, 1, CH, KC, KC // 2, self.ws)
        dz = torch.empty(V, H, W, device=self.dev)
        conv_rows(dz, da1, self.W1, None, R, W, CH, 1, KC, KC - 1 - KC // 2, CONV_TRANSPOSE)
        del da1
        # y2 feeds y3 directly and z = y2 / sigma
        dy2 = dy3
        scale_groups(dy2, dz, self.sigma_t, n, 1, accumulate=True)
        # view weights
        grads["lam"] = torch.empty(V, device=self.dev)
        group_dot(grads["lam"], dy2, c["y1"], H * W, V)
        dy1 = torch.empty_like(dy2)
        scale_groups(dy1, dy2, self.lam, H * W, V)
        # ramp taps, then the bins
        dh = torch.empty(self.K, device=self.dev)
        conv_rows_wgrad(dh, None, dy1, c["x0"], R, W, 1, 1, self.K, W - 1, self.ws)
        grads["theta"] = torch.empty(N_BINS + 1, device=self.dev)
        matvec(grads["theta"], self.M, dh, self.K, N_BINS + 1, transpose=True)
        grads["theta"][N_BINS] = 0.0  # the Nyquist bin is fixed
        return loss, grads

    def apply_grads(self, grads, lr):
        self.step_count += 1
        for name in self.params:
            m, v = self.adam_state[name]
            adam(getattr(self, name), m, v, grads[name].contiguous(), lr, self.step_count)


def fov_mask(N: int, voxel_size: float, origin, radius_mm: float, half_height_mm: float):
    """1 inside the cylinder r <= radius, |z| <= half_height (mm), else 0."""
    c = np.asarray(origin, dtype=np.float64) + voxel_size * np.arange(N)[:, None]
    x = c[:, 0][None, None, :]
    y = c[:, 1][None, :, None]
    z = c[:, 2][:, None, None]
    m = ((x * x + y * y) <= radius_mm ** 2) & (np.abs(z) <= half_height_mm)
    return m.astype(np.float32)


# --------------------------------------------------------------------------
# data, training and evaluation
# --------------------------------------------------------------------------
def geometry_from(g) -> Geometry:
    """Geometry of a synth.Geometry."""
    return Geometry(P=g.P, betas=g.betas, H=g.H, W=g.W, sid=g.sid, sdd=g.sdd, pixel=g.pixel,
                    arc=g.arc)


def phantom_case(seed: int, geo: Geometry, N: int, voxel_size: float, origin, device,
                 projector: str = "analytic", sync=None):
    """(ground-truth volume, line integrals) of the seeded ellipsoid phantom.

    The volume averages 2^3 samples per voxel.  projector="analytic": exact
    line integrals of the ellipsoids (resolution-free, like a scanner's);
    "matched": the forward projection of the volume by the library's matched
    projector (its projections carry that voxel grid's sampling)."""
    import synth
    ell = synth.ellipsoid_phantom(seed)
    gt = synth.voxelize_torch(ell, N, voxel_size, origin, device, sub=2)
    if projector == "matched":
        p = torch.zeros(geo.V, geo.H, geo.W, device=device)
        forward_project(p, gt, geo.P, voxel_size, origin)
        return gt, p
    g = synth.cone_beam_geometry(n_views=geo.V, H=geo.H, W=geo.W, pixel=geo.pixel,
                                 sid=geo.sid, sdd=geo.sdd, arc_deg=math.degrees(geo.arc))
    if not np.array_equal(g.P, geo.P):
        raise ValueError("analytic projections need the synthetic scan geometry")
    p = torch.from_numpy(synth.line_integrals(g, ell)).to(device)
    return gt, p


def masked_rmse(vol, gt, mask) -> float:
    d = (vol - gt) * mask
    return float(torch.sqrt((d.double() ** 2).sum() / mask.double().sum()))


def train(model: LearnedFilter, seeds, N, voxel_size, origin, mask, epochs=1, lr=1e-3,
          log=print, projector="analytic"):
    """Adam over the phantoms of `seeds`, one phantom per step."""
    import time
    gm = None
    step = 0
    seeds = list(seeds)
    for ep in range(epochs):
        t0 = time.time()
        tot = 0.0
        for s in seeds:
            gt, p = phantom_case(s, model.g, N, voxel_size, origin, model.dev, projector)
            gm = gt * mask
            loss, grads = model.loss_and_grads(p, gm, mask, N, voxel_size, origin)
            model.apply_grads(grads, lr)
            tot += float(loss)
            step += 1
            if step % 32 == 0:
                log(f"  step {step}: mean loss so far this epoch {tot / (step - ep * len(seeds)):.4e}"
                    f" ({time.time() - t0:.1f} s)")
        log(f"epoch {ep}: mean loss {tot / len(seeds):.4e} ({time.time() - t0:.1f} s, "
            f"{len(seeds)} steps)")
    return model


def evaluate(model: LearnedFilter, seeds, N, voxel_size, origin, mask, projector="analytic"):
    """Masked RMSE of plain FBP and of the learned filter on `seeds`
    (plain FBP: the library's pre-filter kernel and the backprojection)."""
    out = []
    g = model.g
    for s in seeds:
        gt, p = phantom_case(s, g, N, voxel_size, origin, model.dev, projector)
        vol_l = model.reconstruct(p, N, voxel_size, origin)
        q = torch.empty_like(p)
        from . import prefilter
        prefilter(q, p, float(g.betas[0]), g.dbeta, 0.5 * (g.arc - math.pi), g.sid, g.sdd,
                  g.pixel)
        vol_p = torch.zeros(N, N, N, device=model.dev)
        backproject(vol_p, q, g.P, voxel_size, origin)
        out.append((masked_rmse(vol_p, gt, mask), masked_rmse(vol_l, gt, mask)))
    return out


def default_sigma(model: LearnedFilter, seed: int, N, voxel_size, origin,
                  projector="analytic") -> float:
    """RMS of the plain-filtered projections of one phantom (CNN input scale)."""
    gt, p = phantom_case(seed, model.g, N, voxel_size, origin, model.dev, projector)
    y = model.filter(p)
    return float(torch.sqrt((y.double() ** 2).mean()))


def main(argv=None):
    import argparse
    import time

    import synth
    ap = argparse.ArgumentParser(description="train the learned Feldkamp filter on one GPU")
    ap.add_argument("--phantoms", type=int, default=512)
    ap.add_argument("--epochs", type=int, default=2)
    ap.add_argument("--N", type=int, default=128)
    ap.add_argument("--eval-N", type=int, default=512)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--held-out", type=int, nargs="+", default=[9999])
    ap.add_argument("--projector", choices=("analytic", "matched"), default="analytic")
    ap.add_argument("--save", default=None, help="write the trained parameters (.npz)")
    args = ap.parse_args(argv)
    dev = torch.device("cuda:0")
    g = synth.cone_beam_geometry(n_views=62, H=480, W=624, pixel=0.616)
    geo = geometry_from(g)
    vs, o = synth.volume_frame(args.N)
    mask = torch.from_numpy(fov_mask(args.N, vs, o, 110.0, 80.0)).to(dev)
    model = LearnedFilter(geo, dev)
    model.sigma = default_sigma(model, 1, args.N, vs, o, args.projector)
    model.sigma_t.fill_(1.0 / model.sigma)
    model.sigma_f.fill_(model.sigma)
    print(f"sigma {model.sigma:.3e}", flush=True)
    before = evaluate(model, args.held_out, args.N, vs, o, mask, args.projector)
    t0 = time.time()
    train(model, range(1, args.phantoms + 1), args.N, vs, o, mask, args.epochs, args.lr,
          log=lambda m: print(m, flush=True), projector=args.projector)
    print(f"training {time.time() - t0:.1f} s", flush=True)
    for N in sorted({args.N, args.eval_N}):
        vsn, on = synth.volume_frame(N)
        mk = torch.from_numpy(fov_mask(N, vsn, on, 110.0, 80.0)).to(dev)
        res = evaluate(model, args.held_out, N, vsn, on, mk, args.projector)
        for s, (rp, rl) in zip(args.held_out, res):
            print(f"held-out phantom {s} at {N}^3: RMSE plain FBP {rp:.4e}, learned {rl:.4e} "
                  f"({100 * (1 - rl / rp):+.1f}%)", flush=True)
    print("before training (plain == learned):", before, flush=True)
    if args.save:
        np.savez(args.save, sigma=model.sigma,
                 **{n: getattr(model, n).cpu().numpy() for n in model.params})


if __name__ == "__main__":
    main()
