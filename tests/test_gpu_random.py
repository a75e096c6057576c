"""Seeded random cases of the fused backprojection against the FP64 oracle.

Each case draws a scan (source and detector distances, pixel size, arc,
jitter), a detector size, a view count, a volume size and placement (partly
off the field of view at times, so the per-wave clipping and the clamped
taps at the detector's edges are exercised), the views per pass, the staged
layout and FP32 or FP16 storage.  The projections are smooth random images
(sums of a few random plane waves), so that the FP32 rounding of the
coordinates stays well inside the tolerance.  FP32 storage is held to
1e-5 sqrt(496 / V), FP16 storage to 1e-3 (its rounding counts as error).
"""
import math

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_1104_5243_amd as fdk
    fdk.lib()
    return torch, fdk, torch.device("cuda:0")


def _case(seed, layouts):
    rng = np.random.default_rng(20_000 + seed)
    V = int(rng.integers(1, 90))
    H = int(rng.integers(3, 48))
    W = int(rng.integers(3, 64))
    sid = float(rng.uniform(300.0, 900.0))
    sdd = sid * float(rng.uniform(1.2, 2.0))
    pixel = float(rng.uniform(0.3, 1.2))
    g = synth.cone_beam_geometry(n_views=V, H=H, W=W, sid=sid, sdd=sdd, pixel=pixel,
                                 arc_deg=float(rng.uniform(30.0, 360.0)),
                                 jitter_mm=float(rng.uniform(0.0, 2.0)),
                                 seed=int(rng.integers(1, 1 << 30)))
    N = int(rng.integers(1, 28))
    fov = W * pixel * sid / sdd  # detector width at the isocentre, mm
    vs = fov / N * float(rng.uniform(0.5, 1.3))
    origin = tuple(-0.5 * vs * (N - 1) + float(rng.uniform(-0.2, 0.2)) * fov for _ in range(3))
    j = np.arange(W)[None, None, :]
    k = np.arange(H)[None, :, None]
    proj = np.zeros((V, H, W))
    for _ in range(4):
        fu, fv = rng.uniform(0.0, 0.3, 2)
        proj += rng.normal() * np.cos(fu * j + fv * k + rng.uniform(0.0, 2 * math.pi))
    return dict(geom=g, N=N, vs=vs, origin=origin, proj=proj.astype(np.float32),
                layout=str(rng.choice(layouts)), storage=str(rng.choice(["f32", "f32", "f16"])),
                batch=int(rng.integers(1, 80)))


@pytest.mark.parametrize("seed", range(16))
def test_random_case(env, seed):
    torch, fdk, dev = env
    c = _case(seed, list(fdk.LAYOUTS))
    g, N, V = c["geom"], c["N"], c["geom"].n_views
    print(f"case {seed}: N={N} V={V} {g.W}x{g.H} layout={c['layout']} {c['storage']} "
          f"batch={c['batch']}", flush=True)
    proj_d = torch.from_numpy(c["proj"]).to(dev)
    vol = torch.zeros(N, N, N, device=dev)
    old_layout = fdk.set_layout(None)
    old_batch = fdk.lib().fdk_set_batch(0)
    try:
        fdk.set_layout(c["layout"])
        assert fdk.lib().fdk_set_batch(c["batch"]) == c["batch"]
        if c["storage"] == "f32":
            fdk.backproject(vol, proj_d, g.P, c["vs"], c["origin"])
        else:
            st, scale = fdk.to_storage(proj_d, torch.float16)
            fdk.backproject(vol, st, g.P, c["vs"], c["origin"], view_scale=scale)
        torch.cuda.synchronize()
    finally:
        fdk.set_layout(old_layout)
        fdk.lib().fdk_set_batch(old_batch)
    ref = oracle.backproject(c["proj"], g.P, N, c["vs"], c["origin"])
    if not np.any(ref):
        # the volume misses every view: nothing may be added
        assert not torch.any(vol).item()
        return
    err = oracle.rel_rmse(vol.cpu().numpy(), ref)
    tol = 1e-5 * max(1.0, math.sqrt(496.0 / V)) if c["storage"] == "f32" else 1e-3
    print(f"  relRMSE {err:.3e} (tolerance {tol:.1e})", flush=True)
    assert err <= tol


@pytest.mark.parametrize("seed", range(12))
def test_random_forward_case(env, seed):
    """The forward projector on the same random scans, of a smooth random
    volume: against the oracle's transpose (2e-5, the tolerance of smooth
    inputs), and the adjoint identity <B p, x> = <p, F x> between the two
    GPU operators."""
    torch, fdk, dev = env
    c = _case(seed, ["dpairs"])
    g, N, V = c["geom"], c["N"], c["geom"].n_views
    rng = np.random.default_rng(30_000 + seed)
    grid = np.arange(N, dtype=np.float64)
    x3 = np.zeros((N, N, N))
    for _ in range(3):
        f = rng.uniform(0.0, 0.4, 3)
        x3 += rng.normal() * np.cos(f[0] * grid[None, None, :] + f[1] * grid[None, :, None]
                                    + f[2] * grid[:, None, None] + rng.uniform(0, 2 * math.pi))
    x3 = x3.astype(np.float32)
    print(f"case {seed}: N={N} V={V} {g.W}x{g.H}", flush=True)
    vol_d = torch.from_numpy(x3).to(dev)
    fp = torch.zeros(V, g.H, g.W, device=dev)
    fdk.forward_project(fp, vol_d, g.P, c["vs"], c["origin"])
    proj_d = torch.from_numpy(c["proj"]).to(dev)
    bp = torch.zeros(N, N, N, device=dev)
    fdk.backproject(bp, proj_d, g.P, c["vs"], c["origin"])
    torch.cuda.synchronize()
    ref = oracle.forward_project(x3, g.P, g.H, g.W, c["vs"], c["origin"])
    got = fp.cpu().numpy()
    if not np.any(ref):
        assert not np.any(got)
        return
    err = oracle.rel_rmse(got, ref)
    lhs = float(np.dot(bp.cpu().numpy().ravel().astype(np.float64), x3.ravel()))
    rhs = float(np.dot(c["proj"].ravel().astype(np.float64), got.ravel()))
    scale = float(np.linalg.norm(bp.cpu().numpy()) * np.linalg.norm(x3))
    print(f"  relRMSE {err:.3e}; adjoint |lhs - rhs| / scale {abs(lhs - rhs) / scale:.2e}",
          flush=True)
    assert err <= 2e-5
    assert abs(lhs - rhs) <= 1e-5 * scale
