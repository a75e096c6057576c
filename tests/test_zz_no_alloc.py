"""The allocation-free backprojection entry point (fdk_backproject_noalloc).

It stages each pass into the library's fixed per-device scratch array.  Its
output must equal fdk_backproject_ex's (the fused path with the same views
per pass) bit for bit, and both stay within the FP32 tolerance of the FP64
oracle.  Two calls in a row, the second smaller (fewer views, a smaller
volume and detector, another storage type), show that what the first call
leaves in the scratch array does not leak into the second.
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
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    fdk.lib()
    return torch, fdk, torch.device("cuda:0")


def _pair(torch, fdk, dev, proj_d, P, N, vs, o, batch, view_scale=None):
    """(no-alloc result, fused result with `batch` views per pass)."""
    old = fdk.set_batch(0)
    try:
        fdk.set_batch(batch)
        a = torch.zeros(N, N, N, device=dev)
        print(f"  noalloc: N={N} views={proj_d.shape[0]} {tuple(proj_d.shape[1:])} "
              f"{proj_d.dtype}", flush=True)
        fdk.backproject_noalloc(a, proj_d, P, vs, o, view_scale=view_scale)
        torch.cuda.synchronize()
        b = torch.zeros(N, N, N, device=dev)
        fdk.backproject(b, proj_d, P, vs, o, view_scale=view_scale)
        torch.cuda.synchronize()
    finally:
        fdk.set_batch(old)
    return a, b


def test_noalloc_matches_fused_two_calls(env):
    torch, fdk, dev = env
    # call 1: 1248x960 FP32, 80 views; 27 staged views fit the scratch array
    g1 = synth.cone_beam_geometry(n_views=80)
    p1 = synth.filtered_projections(g1, synth.ellipsoid_phantom())
    N1 = 72
    vs1, o1 = synth.volume_frame(N1)
    a1, b1 = _pair(torch, fdk, dev, torch.from_numpy(p1).to(dev), g1.P, N1, vs1, o1, 27)
    assert torch.equal(a1, b1)
    ref1 = oracle.backproject(p1, g1.P, N1, vs1, o1)
    e1 = oracle.rel_rmse(a1.cpu().numpy(), ref1)
    print(f"  call 1 relRMSE vs oracle {e1:.3e}", flush=True)
    assert e1 <= 1e-5 * math.sqrt(496 / 80)

    # call 2, smaller: 624x480 FP16 with per-view scales, 21 views, 40^3
    g2 = synth.cone_beam_geometry(n_views=21, H=480, W=624, pixel=0.616, seed=7)
    p2 = synth.filtered_projections(g2, synth.ellipsoid_phantom(seed=11))
    N2 = 40
    vs2, o2 = synth.volume_frame(N2)
    st, sc = fdk.to_storage(torch.from_numpy(p2).to(dev), torch.float16)
    a2, b2 = _pair(torch, fdk, dev, st, g2.P, N2, vs2, o2, 64, view_scale=sc)
    assert torch.equal(a2, b2)
    ref2 = oracle.backproject(p2, g2.P, N2, vs2, o2)
    e2 = oracle.rel_rmse(a2.cpu().numpy(), ref2)
    print(f"  call 2 relRMSE vs oracle {e2:.3e}", flush=True)
    assert e2 <= 1e-3


def test_noalloc_accumulates_and_ragged_last_pass(env):
    """Accumulation into an existing volume and a last pass of 1 view."""
    torch, fdk, dev = env
    g = synth.cone_beam_geometry(n_views=28, H=96, W=128, pixel=3.0, seed=3)
    p = synth.filtered_projections(g, synth.ellipsoid_phantom(seed=4))
    N = 33
    vs, o = synth.volume_frame(N)
    pd = torch.from_numpy(p).to(dev)
    ref = oracle.backproject(p, g.P, N, vs, o)
    # an initial volume of the result's own size, so that the error of the
    # added part is not hidden under the rounding of a larger one
    rms = float(np.sqrt(np.mean(ref ** 2)))
    init = rms * torch.randn(N, N, N, device=dev, generator=torch.Generator(dev).manual_seed(5))
    old = fdk.set_batch(0)
    try:
        fdk.set_batch(9)  # passes of 9, 9, 9, 1 views
        a = init.clone()
        fdk.backproject_noalloc(a, pd, g.P, vs, o)
        b = init.clone()
        fdk.backproject(b, pd, g.P, vs, o)
        torch.cuda.synchronize()
    finally:
        fdk.set_batch(old)
    assert torch.equal(a, b)
    err = oracle.rel_rmse(a.double().cpu().numpy() - init.double().cpu().numpy(), ref)
    assert err <= 1e-5 * math.sqrt(496 / 28)
