"""The matched forward projector (exact transpose of the backprojection) and
the autograd pair built on it.

Parity: the GPU forward projector against the oracle's transpose, FP32 with
float atomics.  The error comes from the FP32 pixel coordinate u' (|u'| up
to ~624, a few half-ulps of 2^-24 * 1024 = 6e-5 pixel each), and a bilinear
weight's error equals the coordinate's.  The backprojection sums band-limited
filtered projections, which damp that error by the image gradient; a
forward projection of a voxelised phantom (piecewise constant, sharp edges)
passes it on at the edges, and of white noise everywhere.  Tolerances:
2e-5 relative RMSE on the phantom, 1e-4 on white noise.  The adjoint
identity <B p, x> =
<p, F x> with both GPU operators at the differentiable-pair workload (256^3,
248 views of 624x480); finite differences at 16^3 (the operators are linear,
so a central difference equals the directional derivative up to rounding).
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_1104_5243_amd as fdk
    from paper_1104_5243_amd import autograd as ag
    fdk.lib()
    geom, ell, vs, o, N = synth.workload("fdk256x8")
    return torch, fdk, ag, torch.device("cuda:0"), geom


WHITE_TOL = 1e-4


def test_forward_projector_phantom_parity(env):
    torch, fdk, ag, dev, geom = env
    N = 64
    vs, o = synth.volume_frame(N)
    vol = synth.voxelize(synth.ellipsoid_phantom(), N, vs, o)
    out = torch.zeros(geom.n_views, geom.H, geom.W, device=dev)
    fdk.forward_project(out, torch.from_numpy(vol).to(dev), geom.P, vs, o)
    torch.cuda.synchronize()
    ref = oracle.forward_project(vol.astype(np.float64), geom.P, geom.H, geom.W, vs, o)
    err = oracle.rel_rmse(out.cpu().numpy(), ref)
    print(f"forward projector phantom {N}^3 x {geom.n_views} views: relRMSE {err:.3e}",
          flush=True)
    assert err <= 2e-5


def test_forward_projector_lds_tiles_at_256(env):
    """1 mm voxels: each workgroup's footprint fits the LDS tile, so the
    scatter goes through LDS; compared with the oracle on 8 views."""
    torch, fdk, ag, dev, geom = env
    N = 256
    vs, o = synth.volume_frame(N)
    vol = synth.voxelize(synth.ellipsoid_phantom(), N, vs, o)
    idx = np.arange(0, geom.n_views, 31)[:8]
    P = geom.P[idx]
    out = torch.zeros(len(idx), geom.H, geom.W, device=dev)
    fdk.forward_project(out, torch.from_numpy(vol).to(dev), P, vs, o)
    torch.cuda.synchronize()
    ref = oracle.forward_project(vol.astype(np.float64), P, geom.H, geom.W, vs, o)
    err = oracle.rel_rmse(out.cpu().numpy(), ref)
    print(f"forward projector (LDS tiles) phantom 256^3 x 8 views: relRMSE {err:.3e}", flush=True)
    assert err <= 2e-5


def test_forward_projector_behind_source_uses_guarded_path(env):
    """w <= 0 for part of the grid: the guarded scatter (global atomics)."""
    torch, fdk, ag, dev, geom = env
    P = np.array([[[1.0, 0.0, 0.0, 2.0], [0.0, 1.0, 0.0, 2.0], [0.0, 0.0, 1.0, 0.0]]])
    N, vs, o = 6, 1.0, (-2.5, -2.5, -2.5)
    rng = np.random.default_rng(4)
    vol = rng.uniform(-1, 1, (N, N, N)).astype(np.float32)
    out = torch.zeros(1, 5, 5, device=dev)
    fdk.forward_project(out, torch.from_numpy(vol).to(dev), P, vs, o)
    torch.cuda.synchronize()
    ref = oracle.forward_project(vol.astype(np.float64), P, 5, 5, vs, o)
    assert oracle.rel_rmse(out.cpu().numpy(), ref) <= WHITE_TOL


def test_forward_projector_matches_oracle_transpose(env):
    torch, fdk, ag, dev, geom = env
    N = 40
    vs, o = synth.volume_frame(N)
    rng = np.random.default_rng(11)
    vol = rng.uniform(-1.0, 1.0, (N, N, N)).astype(np.float32)
    V = 30
    P = geom.P[:V]
    out = torch.zeros(V, geom.H, geom.W, device=dev)
    fdk.forward_project(out, torch.from_numpy(vol).to(dev), P, vs, o)
    torch.cuda.synchronize()
    ref = oracle.forward_project(vol.astype(np.float64), P, geom.H, geom.W, vs, o)
    err = oracle.rel_rmse(out.cpu().numpy(), ref)
    print(f"forward projector white noise {N}^3 x {V} views: relRMSE {err:.3e}", flush=True)
    assert err <= WHITE_TOL


def test_forward_projector_accumulates_and_handles_ragged_grids(env):
    """Volumes smaller than one workgroup box, and 70^3: two whole boxes of
    32 voxels along the rays and a ragged third (6), ragged in z and across
    the rays too."""
    torch, fdk, ag, dev, geom = env
    for N in (1, 7, 19, 70):
        vs = 150.0 / N
        o = (-75.0 + vs / 2 + 1.0, -75.0 + vs / 2, -75.0 + vs / 2 - 2.0)
        rng = np.random.default_rng(N)
        vol = rng.uniform(-1, 1, (N, N, N)).astype(np.float32)
        init = rng.uniform(-1, 1, (9, geom.H, geom.W)).astype(np.float32)
        out = torch.from_numpy(init).to(dev)
        fdk.forward_project(out, torch.from_numpy(vol).to(dev), geom.P[:9], vs, o)
        torch.cuda.synchronize()
        ref = init.astype(np.float64) + oracle.forward_project(vol.astype(np.float64), geom.P[:9],
                                                               geom.H, geom.W, vs, o)
        assert oracle.rel_rmse(out.cpu().numpy(), ref) <= WHITE_TOL


def test_adjoint_identity_at_256(env):
    """<B p, x> = <p, F x> with the GPU operators at 256^3 x 248 views."""
    torch, fdk, ag, dev, geom = env
    N = 256
    vs, o = synth.volume_frame(N)
    g = torch.Generator(device=dev).manual_seed(5)
    p = torch.rand(geom.n_views, geom.H, geom.W, device=dev, generator=g) - 0.5
    x = torch.rand(N, N, N, device=dev, generator=g) - 0.5
    Bp = torch.zeros(N, N, N, device=dev)
    fdk.backproject(Bp, p, geom.P, vs, o)
    Fx = torch.zeros_like(p)
    fdk.forward_project(Fx, x, geom.P, vs, o)
    torch.cuda.synchronize()
    lhs = float((Bp.double() * x.double()).sum())
    rhs = float((p.double() * Fx.double()).sum())
    scale = float(Bp.double().abs().mul(x.double().abs()).sum())
    print(f"adjoint 256^3 x 248: <Bp,x> {lhs:.6e} <p,Fx> {rhs:.6e} rel {(lhs - rhs) / scale:.2e}",
          flush=True)
    assert abs(lhs - rhs) <= 1e-6 * scale


def test_autograd_finite_differences_16(env):
    torch, fdk, ag, dev, geom = env
    N = 16
    vs, o = 9.0, (-67.5, -67.5, -67.5)
    V = 12
    P = geom.P[::20][:V]
    g = torch.Generator(device=dev).manual_seed(7)
    p = (torch.rand(V, geom.H, geom.W, device=dev, generator=g) - 0.5).requires_grad_(True)
    wvol = torch.rand(N, N, N, device=dev, generator=g) - 0.5
    # backprojection: dL/dp for L = <w, B p>
    L = (ag.backproject_op(p, P, N, vs, o) * wvol).sum()
    L.backward()
    d = torch.rand(V, geom.H, geom.W, device=dev, generator=g) - 0.5
    eps = 1.0
    with torch.no_grad():
        Lp = (ag.backproject_op(p + eps * d, P, N, vs, o) * wvol).double().sum()
        Lm = (ag.backproject_op(p - eps * d, P, N, vs, o) * wvol).double().sum()
    fd = float((Lp - Lm) / (2 * eps))
    an = float((p.grad.double() * d.double()).sum())
    print(f"BackProject FD {fd:.6e} autograd {an:.6e}", flush=True)
    assert abs(fd - an) <= 1e-4 * abs(an)
    # and the gradient equals the oracle transpose applied to w
    ref = oracle.forward_project(wvol.cpu().double().numpy(), P, geom.H, geom.W, vs, o)
    assert oracle.rel_rmse(p.grad.cpu().numpy(), ref) <= WHITE_TOL
    # forward projection: dL/dx for L = <q, F x>
    x = (torch.rand(N, N, N, device=dev, generator=g) - 0.5).requires_grad_(True)
    q = torch.rand(V, geom.H, geom.W, device=dev, generator=g) - 0.5
    L2 = (ag.forward_project_op(x, P, geom.H, geom.W, vs, o) * q).sum()
    L2.backward()
    dx = torch.rand(N, N, N, device=dev, generator=g) - 0.5
    with torch.no_grad():
        Lp = (ag.forward_project_op(x + eps * dx, P, geom.H, geom.W, vs, o) * q).double().sum()
        Lm = (ag.forward_project_op(x - eps * dx, P, geom.H, geom.W, vs, o) * q).double().sum()
    fd = float((Lp - Lm) / (2 * eps))
    an = float((x.grad.double() * dx.double()).sum())
    print(f"ForwardProject FD {fd:.6e} autograd {an:.6e}", flush=True)
    assert abs(fd - an) <= 1e-4 * abs(an)
    ref = oracle.backproject(q.cpu().numpy(), P, N, vs, o)
    assert oracle.rel_rmse(x.grad.cpu().numpy(), ref) <= WHITE_TOL


def test_autograd_batch_of_8(env):
    """Batch of 8 volumes: forward = backprojection of 8 stacks, backward =
    forward projection, each item equal to its own single call."""
    torch, fdk, ag, dev, geom = env
    N = 32
    vs, o = synth.volume_frame(N)
    V = 24
    P = geom.P[::10][:V]
    g = torch.Generator(device=dev).manual_seed(9)
    p = (torch.rand(8, V, geom.H, geom.W, device=dev, generator=g) - 0.5).requires_grad_(True)
    vol = ag.backproject_op(p, P, N, vs, o)
    assert vol.shape == (8, N, N, N)
    wv = torch.rand(8, N, N, N, device=dev, generator=g)
    (vol * wv).sum().backward()
    for b in (0, 5):
        one = torch.zeros(N, N, N, device=dev)
        fdk.backproject(one, p[b].detach().contiguous(), P, vs, o)
        gp = torch.zeros(V, geom.H, geom.W, device=dev)
        fdk.forward_project(gp, wv[b].contiguous(), P, vs, o)
        torch.cuda.synchronize()
        assert torch.equal(one, vol[b].detach())
        assert oracle.rel_rmse(p.grad[b].cpu().numpy(), gp.cpu().numpy()) <= 1e-6


def test_autograd_batch_of_8_at_256(env):
    """The differentiable pair at its stated size: a batch of 8 volumes of
    256^3 from 248 views of 624x480.  Item 3's forward result on two 32^3
    blocks and its gradient on three views against the oracle."""
    torch, fdk, ag, dev, geom = env
    N = 256
    vs, o = synth.volume_frame(N)
    V, H, W = geom.n_views, geom.H, geom.W
    g = torch.Generator(device=dev).manual_seed(11)
    p = (torch.rand(8, V, H, W, device=dev, generator=g) - 0.5).requires_grad_(True)
    print(f"\n  batch 8 x {N}^3, {V} views {W}x{H}", flush=True)
    vol = ag.backproject_op(p, geom.P, N, vs, o)
    assert vol.shape == (8, N, N, N)
    wv = torch.rand(8, N, N, N, device=dev, generator=g)
    (vol * wv).sum().backward()
    torch.cuda.synchronize()
    b = 3
    pr = p.detach()[b].cpu().numpy()
    for box in (((112, 32), (112, 32), (112, 32)), ((8, 32), (200, 32), (40, 32))):
        (x0, nx), (y0, ny), (z0, nz) = box
        ref = oracle.backproject(pr, geom.P, N, vs, o, box=box)
        got = vol[b, z0:z0 + nz, y0:y0 + ny, x0:x0 + nx].detach().double().cpu().numpy()
        e = oracle.rel_rmse(got, ref)
        print(f"  forward block {box}: relRMSE {e:.3e}", flush=True)
        assert e <= WHITE_TOL
    views = [0, 101, 247]
    refg = oracle.forward_project(wv[b].double().cpu().numpy(), geom.P[views], H, W, vs, o)
    e = oracle.rel_rmse(p.grad[b, views].double().cpu().numpy(), refg)
    print(f"  gradient views {views}: relRMSE {e:.3e}", flush=True)
    assert e <= WHITE_TOL


def test_forward_projector_is_deterministic(env):
    """The forward projection sums in 64-bit fixed point: two runs on the
    same volume give the same bits (the LDS-tile path at 256^3 and the
    per-tap path of footprints larger than a tile at 48^3 with wide
    voxels)."""
    torch, fdk, ag, dev, geom = env
    for N, vs_mm in ((256, None), (48, 6.0)):
        if vs_mm is None:
            vs, o = synth.volume_frame(N)
        else:
            vs, o = vs_mm, (-0.5 * vs_mm * (N - 1),) * 3
        P = geom.P[::8]
        g = torch.Generator(device=dev).manual_seed(N)
        vol = torch.rand(N, N, N, device=dev, generator=g) - 0.25
        outs = []
        for _ in range(2):
            p = torch.zeros(P.shape[0], geom.H, geom.W, device=dev)
            fdk.forward_project(p, vol, P, vs, o)
            torch.cuda.synchronize()
            outs.append(p)
        print(f"  {N}^3 x {P.shape[0]} views: max |run1 - run2| "
              f"{float((outs[0] - outs[1]).abs().max()):.3e}", flush=True)
        assert torch.equal(outs[0], outs[1])
