"""GPU Feldkamp pre-filter (cosine, Parker, Ram-Lak; FP64 FFT convolution)
against the FP64 oracle (direct convolution), and plain FBP on the GPU
(pre-filter + backprojection) of a uniform sphere.  Tolerance: relative
RMSE <= 1e-5; the GPU path is FP64 inside, so the FP32 output rounding
(~3e-8) is what remains."""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import prefilter as opf

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_1104_5243_amd as fdk
    fdk.lib()
    return torch, fdk, torch.device("cuda:0")


def _gpu_prefilter(fdk, torch, dev, li, g, full_scan=False):
    x = torch.from_numpy(li).to(dev)
    out = torch.empty_like(x)
    delta = -1.0 if full_scan else 0.5 * (g.arc - math.pi)
    fdk.prefilter(out, x, float(g.betas[0]), g.dbeta, delta, g.sid, g.sdd, g.pixel)
    torch.cuda.synchronize()
    return out


# W = 513..1280 take the L = 2560 kernel (1248, 624, 513, 1025, 1280 and an
# odd row count), 1281..2048 the L = 4096 one, shorter rows the general one
@pytest.mark.parametrize("shape", [(6, 960, 1248), (5, 480, 624), (3, 7, 9), (3, 5, 2048),
                                   (3, 4, 1), (4, 3, 2), (3, 9, 513),
                                   (3, 3, 1025), (3, 5, 1280), (3, 3, 1281)])
def test_prefilter_parity(env, shape):
    torch, fdk, dev = env
    V, H, W = shape
    g = synth.cone_beam_geometry(n_views=V, H=H, W=W, pixel=0.308 * 1248 / max(W, 9))
    li = synth.line_integrals(g, synth.ellipsoid_phantom())
    got = _gpu_prefilter(fdk, torch, dev, li, g).cpu().numpy()
    ref = opf.fdk_prefilter(li, g.betas, 0.5 * (g.arc - math.pi), g.dbeta, g.sid, g.sdd, g.pixel)
    assert np.abs(ref).max() > 0  # a short scan's first and last views weigh 0
    err = oracle.rel_rmse(got, ref)
    print(f"prefilter {shape}: relRMSE {err:.3e}", flush=True)
    assert err <= 1e-5


def test_prefilter_full_circle_weights(env):
    """delta < 0 selects the full-circle weighting (1/2 for every ray)."""
    torch, fdk, dev = env
    g = synth.cone_beam_geometry(n_views=4, H=33, W=100, pixel=0.308 * 1248 / 100)
    li = synth.line_integrals(g, synth.ellipsoid_phantom())
    got = _gpu_prefilter(fdk, torch, dev, li, g, full_scan=True).cpu().numpy()
    ref = opf.fdk_prefilter(li, g.betas, -1.0, g.dbeta, g.sid, g.sdd, g.pixel)
    assert oracle.rel_rmse(got, ref) <= 1e-5


def test_gpu_fbp_of_uniform_sphere(env):
    """Plain FBP on the GPU: line integrals -> fdk_prefilter -> fdk_backproject
    returns the sphere's density in the central plane."""
    torch, fdk, dev = env
    g = synth.cone_beam_geometry(n_views=248, H=480, W=624, pixel=0.616, jitter_mm=0.0)
    mu = 0.02
    li = synth.line_integrals(g, synth.sphere_phantom(60.0, mu))
    q = _gpu_prefilter(fdk, torch, dev, li, g)
    N = 128
    vs, o = synth.volume_frame(N)
    vol = torch.zeros(N, N, N, device=dev)
    fdk.backproject(vol, q, g.P, vs, o)
    torch.cuda.synchronize()
    v = vol.cpu().numpy()
    centre = v[N // 2, N // 2 - 20:N // 2 + 20, N // 2 - 20:N // 2 + 20]
    print(f"GPU FBP sphere: mean {centre.mean() / mu:.5f} x density", flush=True)
    np.testing.assert_allclose(centre / mu, 1.0, atol=5e-3)
