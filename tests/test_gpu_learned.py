"""GPU kernels of the learned filter against the FP64 oracle, the whole
model's gradients against the oracle's hand-derived (and FD-pinned)
gradients, and training: the learned filter must beat plain FBP on held-out
phantoms.  Tolerances: FP32 kernels with FP64 accumulation where sums are
long: 1e-5 relative for single kernels; 1e-3 for whole-model gradients (FP32
forward projector with atomics, and FP32 ReLU decisions near zero)."""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import learned as OL

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_1104_5243_amd as fdk
    from paper_1104_5243_amd import learned as GL
    fdk.lib()
    return torch, fdk, GL, torch.device("cuda:0")


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("cin,cout,W,rows,relu", [(1, 32, 37, 5, True), (32, 32, 64, 3, True),
                                                  (32, 1, 70, 4, False), (3, 5, 1, 2, False),
                                                  (1, 32, 300, 3, True), (32, 1, 513, 2, False),
                                                  (4, 8, 130, 3, True), (32, 1, 1028, 2, False)])
def test_conv_short_forward_adjoint_wgrad(env, cin, cout, W, rows, relu):
    torch, fdk, GL, dev = env
    rng = np.random.default_rng(cin * 100 + cout)
    K, pad = 9, 4
    x = rng.standard_normal((rows, cin, W)).astype(np.float32)
    w = rng.standard_normal((cout, cin, K)).astype(np.float32)
    b = rng.standard_normal(cout).astype(np.float32)
    dy = rng.standard_normal((rows, cout, W)).astype(np.float32)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    out = torch.empty(rows, cout, W, device=dev)
    fdk.conv_rows(out, T(x), T(w), T(b), rows, W, cin, cout, K, pad,
                  fdk.CONV_RELU if relu else 0)
    ref = OL.conv(x.astype(np.float64), w.astype(np.float64), b, pad)
    if relu:
        ref = np.maximum(ref, 0)
    assert rel(out.cpu().numpy(), ref) <= 1e-5
    dx = torch.empty(rows, cin, W, device=dev)
    fdk.conv_rows(dx, T(dy), T(w), None, rows, W, cout, cin, K, K - 1 - pad, fdk.CONV_TRANSPOSE)
    rdx = OL.conv_adjoint(dy.astype(np.float64), w.astype(np.float64), pad)
    assert rel(dx.cpu().numpy(), rdx) <= 1e-5
    # ReLU-masked data gradient: out holds the activation on entry
    act = rng.standard_normal((rows, cin, W)).astype(np.float32)
    dxm = T(act)
    fdk.conv_rows(dxm, T(dy), T(w), None, rows, W, cout, cin, K, K - 1 - pad,
                  fdk.CONV_TRANSPOSE | fdk.CONV_RELU_MASK)
    assert rel(dxm.cpu().numpy(), np.where(act > 0, rdx, 0.0)) <= 1e-5
    dw = torch.empty(cout, cin, K, device=dev)
    db = torch.empty(cout, device=dev)
    ws = torch.empty(fdk.conv_rows_wgrad_workspace(cin, cout, K) // 4, device=dev)
    fdk.conv_rows_wgrad(dw, db, T(dy), T(x), rows, W, cin, cout, K, pad, ws)
    rdw, rdb = OL.conv_wgrad(dy.astype(np.float64), x.astype(np.float64), K, pad)
    torch.cuda.synchronize()
    assert rel(dw.cpu().numpy(), rdw) <= 1e-5
    assert rel(db.cpu().numpy(), rdb) <= 1e-5
    # accumulate flag
    out2 = out.clone()
    fdk.conv_rows(out2, T(x), T(w), T(b), rows, W, cin, cout, K, pad, fdk.CONV_ACCUMULATE)
    base = OL.conv(x.astype(np.float64), w.astype(np.float64), b, pad)
    assert rel(out2.cpu().numpy(), out.cpu().numpy() + base) <= 1e-5


@pytest.mark.parametrize("W,rows,pad", [(300, 5, 0), (257, 3, 8), (70, 4, 12), (513, 2, 4)])
def test_wgrad_one_output_channel(env, W, rows, pad):
    """32 -> 1 weight gradients: pad <= 8 takes the kernel with the input
    channels as MFMA rows (chunks of 256 positions, ragged last chunk),
    larger pads the general one; both against the oracle."""
    torch, fdk, GL, dev = env
    rng = np.random.default_rng(W * 10 + pad)
    K = 9
    x = rng.standard_normal((rows, 32, W)).astype(np.float32)
    dy = rng.standard_normal((rows, 1, W)).astype(np.float32)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    dw = torch.empty(1, 32, K, device=dev)
    db = torch.empty(1, device=dev)
    ws = torch.empty(fdk.conv_rows_wgrad_workspace(32, 1, K) // 4, device=dev)
    fdk.conv_rows_wgrad(dw, db, T(dy), T(x), rows, W, 32, 1, K, pad, ws)
    rdw, rdb = OL.conv_wgrad(dy.astype(np.float64), x.astype(np.float64), K, pad)
    torch.cuda.synchronize()
    assert rel(dw.cpu().numpy(), rdw) <= 1e-5
    assert rel(db.cpu().numpy(), rdb) <= 1e-5


@pytest.mark.parametrize("W,rows,pad", [(624, 220, 4), (129, 6, 2), (1, 5, 4), (200, 300, 4)])
def test_conv_mfma_path_shapes(env, W, rows, pad):
    """The 32 -> 32 channel, 9-tap layers run on matrix cores: forward,
    transposed and weight gradient against the oracle, with ragged tails
    (W not a multiple of the 128- and 64-position chunks) and more chunks
    than blocks (each block walks several)."""
    torch, fdk, GL, dev = env
    rng = np.random.default_rng(W * 1000 + rows)
    cin = cout = 32
    K = 9
    x = rng.standard_normal((rows, cin, W)).astype(np.float32)
    w = (rng.standard_normal((cout, cin, K)) * 0.1).astype(np.float32)
    b = rng.standard_normal(cout).astype(np.float32)
    dy = rng.standard_normal((rows, cout, W)).astype(np.float32)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    out = torch.empty(rows, cout, W, device=dev)
    fdk.conv_rows(out, T(x), T(w), T(b), rows, W, cin, cout, K, pad, fdk.CONV_RELU)
    ref = np.maximum(OL.conv(x.astype(np.float64), w.astype(np.float64), b, pad), 0)
    e_fwd = rel(out.cpu().numpy(), ref)
    dx = torch.empty(rows, cin, W, device=dev)
    fdk.conv_rows(dx, T(dy), T(w), None, rows, W, cout, cin, K, K - 1 - pad, fdk.CONV_TRANSPOSE)
    e_adj = rel(dx.cpu().numpy(), OL.conv_adjoint(dy.astype(np.float64), w.astype(np.float64),
                                                  pad))
    dw = torch.empty(cout, cin, K, device=dev)
    db = torch.empty(cout, device=dev)
    ws = torch.empty(fdk.conv_rows_wgrad_workspace(cin, cout, K) // 4, device=dev)
    fdk.conv_rows_wgrad(dw, db, T(dy), T(x), rows, W, cin, cout, K, pad, ws)
    rdw, rdb = OL.conv_wgrad(dy.astype(np.float64), x.astype(np.float64), K, pad)
    torch.cuda.synchronize()
    e_dw, e_db = rel(dw.cpu().numpy(), rdw), rel(db.cpu().numpy(), rdb)
    print(f"mfma conv W={W} rows={rows} pad={pad}: fwd {e_fwd:.2e} adj {e_adj:.2e} "
          f"dW {e_dw:.2e} db {e_db:.2e}", flush=True)
    assert max(e_fwd, e_adj, e_dw, e_db) <= 1e-5
    # the weight gradient is reduced in a fixed order: two calls agree bit for bit
    dw2 = torch.empty_like(dw)
    fdk.conv_rows_wgrad(dw2, None, T(dy), T(x), rows, W, cin, cout, K, pad, ws)
    torch.cuda.synchronize()
    assert torch.equal(dw, dw2)


@pytest.mark.parametrize("W,rows", [(100, 7), (624, 3)])
def test_conv_long_forward_wgrad(env, W, rows):
    torch, fdk, GL, dev = env
    rng = np.random.default_rng(W)
    K, pad = 2 * W - 1, W - 1
    x = rng.standard_normal((rows, 1, W)).astype(np.float32)
    h = rng.standard_normal((1, 1, K)).astype(np.float32)
    dy = rng.standard_normal((rows, 1, W)).astype(np.float32)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    out = torch.empty(rows, 1, W, device=dev)
    fdk.conv_rows(out, T(x), T(h), None, rows, W, 1, 1, K, pad)
    assert rel(out.cpu().numpy(), OL.conv(x.astype(np.float64), h.astype(np.float64), None,
                                          pad)) <= 1e-6
    dh = torch.empty(K, device=dev)
    db = torch.empty(1, device=dev)
    ws = torch.empty(fdk.conv_rows_wgrad_workspace(1, 1, K) // 4, device=dev)
    fdk.conv_rows_wgrad(dh, db, T(dy), T(x), rows, W, 1, 1, K, pad, ws)
    rdh, rdb = OL.conv_wgrad(dy.astype(np.float64), x.astype(np.float64), K, pad)
    torch.cuda.synchronize()
    assert rel(dh.cpu().numpy(), rdh[0, 0]) <= 1e-6
    assert rel(db.cpu().numpy(), rdb) <= 1e-6
    # a pad other than W - 1 takes the direct kernel
    fdk.conv_rows_wgrad(dh, None, T(dy), T(x), rows, W, 1, 1, K, pad - 3, ws)
    rdh3, _ = OL.conv_wgrad(dy.astype(np.float64), x.astype(np.float64), K, pad - 3)
    torch.cuda.synchronize()
    assert rel(dh.cpu().numpy(), rdh3[0, 0]) <= 1e-6


@pytest.mark.parametrize("W,rows", [(1280, 3), (1300, 5), (2048, 2)])
def test_conv_long_register_fft(env, W, rows):
    """Rows of 513..1280 samples take the L = 2560 FFT kernel, rows of
    1281..2048 the L = 4096 one, both keeping their passes in registers
    (complex spectrum of learned taps): forward with bias and accumulation, and the
    transposed call.  The adjoint of the correlation with taps w at offset
    pad is the correlation with the reversed taps at offset K - 1 - pad."""
    torch, fdk, GL, dev = env
    rng = np.random.default_rng(W + 7)
    K, pad = 2 * W - 1, W - 1
    x = rng.standard_normal((rows, 1, W))
    h = rng.standard_normal((1, 1, K))
    b = rng.standard_normal(1)
    base = rng.standard_normal((rows, 1, W))
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
    F = lambda a: a.astype(np.float32).astype(np.float64)
    out = T(base)
    fdk.conv_rows(out, T(x), T(h), T(b), rows, W, 1, 1, K, pad, fdk.CONV_ACCUMULATE)
    ref = OL.conv(F(x), F(h), F(b), pad) + F(base)
    assert rel(out.cpu().numpy(), ref) <= 1e-6
    dx = torch.empty(rows, 1, W, device=dev)
    fdk.conv_rows(dx, T(x), T(h), None, rows, W, 1, 1, K, K - 1 - pad, fdk.CONV_TRANSPOSE)
    ref_t = OL.conv(F(x), F(h)[:, :, ::-1], None, K - 1 - pad)
    torch.cuda.synchronize()
    assert rel(dx.cpu().numpy(), ref_t) <= 1e-6
    dxm = T(base)
    fdk.conv_rows(dxm, T(x), T(h), None, rows, W, 1, 1, K, K - 1 - pad,
                  fdk.CONV_TRANSPOSE | fdk.CONV_RELU_MASK)
    torch.cuda.synchronize()
    assert rel(dxm.cpu().numpy(), np.where(F(base) > 0, ref_t, 0.0)) <= 1e-6
    # the taps' gradient (FFT cross-spectra at L = 4096)
    dh = torch.empty(K, device=dev)
    ws = torch.empty(fdk.conv_rows_wgrad_workspace(1, 1, K) // 4, device=dev)
    fdk.conv_rows_wgrad(dh, None, T(base), T(x), rows, W, 1, 1, K, pad, ws)
    rdh, _ = OL.conv_wgrad(F(base), F(x), K, pad)
    torch.cuda.synchronize()
    assert rel(dh.cpu().numpy(), rdh[0, 0]) <= 1e-6


@pytest.mark.parametrize("rows,cols", [(7, 11), (1247, 1025), (5, 300), (300, 5)])
def test_matvec_shapes(env, rows, cols):
    """A x (a wave per row: four partial sums over columns, tails) and A^T x
    (a block per 64 outputs: rows split over four waves, tails)."""
    torch, fdk, GL, dev = env
    rng = np.random.default_rng(rows * 7 + cols)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
    A = rng.standard_normal((rows, cols)).astype(np.float32)
    v = rng.standard_normal(cols).astype(np.float32)
    u = rng.standard_normal(rows).astype(np.float32)
    r1 = torch.empty(rows, device=dev)
    fdk.matvec(r1, T(A), T(v), rows, cols)
    r2 = torch.empty(cols, device=dev)
    fdk.matvec(r2, T(A), T(u), rows, cols, transpose=True)
    torch.cuda.synchronize()
    assert rel(r1.cpu().numpy(), A.astype(np.float64) @ v) <= 1e-6
    assert rel(r2.cpu().numpy(), A.astype(np.float64).T @ u) <= 1e-6


@pytest.mark.parametrize("groups,len_", [(3, 20000), (2, 8 * 1024), (4, 8 * 1024 + 5)])
def test_group_dot_long_groups(env, groups, len_):
    """Groups longer than one pass of 1024 threads x 8 partial sums."""
    torch, fdk, GL, dev = env
    rng = np.random.default_rng(len_)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
    a = rng.standard_normal((groups, len_)).astype(np.float32)
    b = rng.standard_normal((groups, len_)).astype(np.float32)
    out = torch.empty(groups, device=dev)
    fdk.group_dot(out, T(a), T(b), len_, groups)
    torch.cuda.synchronize()
    np.testing.assert_allclose(out.cpu().numpy(), (a.astype(np.float64) * b).sum(1), rtol=1e-5)


def test_elementwise_kernels(env):
    torch, fdk, GL, dev = env
    rng = np.random.default_rng(2)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
    x = rng.standard_normal((5, 13)).astype(np.float32)
    s = rng.standard_normal(5).astype(np.float32)
    y = T(rng.standard_normal((5, 13)))
    y0 = y.clone()
    fdk.scale_groups(y, T(x), T(s), 13, 5, accumulate=True)
    np.testing.assert_allclose(y.cpu().numpy(), y0.cpu().numpy() + x * s[:, None], rtol=1e-6)
    out = torch.empty(5, device=dev)
    a = rng.standard_normal((5, 1000)).astype(np.float32)
    b = rng.standard_normal((5, 1000)).astype(np.float32)
    fdk.group_dot(out, T(a), T(b), 1000, 5)
    np.testing.assert_allclose(out.cpu().numpy(), (a.astype(np.float64) * b).sum(1), rtol=1e-5)
    dy = rng.standard_normal(100).astype(np.float32)
    yy = rng.standard_normal(100).astype(np.float32)
    dx = torch.empty(100, device=dev)
    fdk.relu_backward(dx, T(dy), T(yy))
    np.testing.assert_array_equal(dx.cpu().numpy(), np.where(yy > 0, dy, 0))
    A = rng.standard_normal((7, 11)).astype(np.float32)
    v = rng.standard_normal(11).astype(np.float32)
    u = rng.standard_normal(7).astype(np.float32)
    r1 = torch.empty(7, device=dev)
    fdk.matvec(r1, T(A), T(v), 7, 11)
    r2 = torch.empty(11, device=dev)
    fdk.matvec(r2, T(A), T(u), 7, 11, transpose=True)
    np.testing.assert_allclose(r1.cpu().numpy(), A.astype(np.float64) @ v, rtol=1e-5)
    np.testing.assert_allclose(r2.cpu().numpy(), A.astype(np.float64).T @ u, rtol=1e-5)
    # Adam against its published update
    p = rng.standard_normal(50).astype(np.float32)
    m = np.zeros(50, np.float32)
    vv = np.zeros(50, np.float32)
    pd, md, vd = T(p), T(m), T(vv)
    pr = p.astype(np.float64)
    mr = np.zeros(50)
    vr = np.zeros(50)
    for step in (1, 2, 3):
        gr = rng.standard_normal(50)
        fdk.adam(pd, md, vd, T(gr), 1e-2, step)
        mr = 0.9 * mr + 0.1 * gr
        vr = 0.999 * vr + 0.001 * gr * gr
        pr = pr - 1e-2 * (mr / (1 - 0.9 ** step)) / (np.sqrt(vr / (1 - 0.999 ** step)) + 1e-8)
    np.testing.assert_allclose(pd.cpu().numpy(), pr, rtol=1e-5, atol=1e-6)
    # mse
    aa = rng.standard_normal(3000).astype(np.float32)
    bb = rng.standard_normal(3000).astype(np.float32)
    g = torch.empty(3000, device=dev)
    loss = torch.empty(1, device=dev)
    ws = torch.empty(4096, device=dev)
    fdk.mse(g, loss, T(aa), T(bb), ws)
    d = aa.astype(np.float64) - bb
    assert float(loss.cpu()) == pytest.approx(np.mean(d * d), rel=1e-6)
    np.testing.assert_allclose(g.cpu().numpy(), 2 * d / 3000, rtol=1e-6)


def _tiny(env, seed=0):
    torch, fdk, GL, dev = env
    g = synth.cone_beam_geometry(n_views=3, H=5, W=9, pixel=30.0)
    geo = GL.Geometry(P=g.P, betas=g.betas, H=g.H, W=g.W, sid=g.sid, sdd=g.sdd, pixel=g.pixel,
                      arc=g.arc)
    return g, geo


def test_model_gradients_match_oracle(env):
    torch, fdk, GL, dev = env
    import sys
    sys.path.insert(0, __file__.rsplit("/", 1)[0])
    from test_learned_oracle import tiny_case
    g, p, T, M, params, N, vs, o, gt, mask = tiny_case()
    sigma = 1e-3
    loss_r, grads_r = OL.loss_and_grads(params, p, T, M, g.P, N, vs, o, sigma, gt, mask)
    geo = GL.Geometry(P=g.P, betas=g.betas, H=g.H, W=g.W, sid=g.sid, sdd=g.sdd, pixel=g.pixel,
                      arc=g.arc)
    model = GL.LearnedFilter(geo, dev, sigma=sigma)
    # the model's own fixed parts against the oracle's (built independently)
    assert rel(model.T.cpu().numpy(), T) <= 1e-6
    assert rel(model.M.cpu().numpy(), M) <= 1e-6
    for name, val in params.items():
        getattr(model, name).copy_(torch.from_numpy(np.asarray(val, dtype=np.float32)).reshape(
            getattr(model, name).shape))
    Tt = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
    loss, grads = model.loss_and_grads(Tt(p), Tt(gt * mask), Tt(mask), N, vs, o)
    torch.cuda.synchronize()
    # the GPU loss is the mean over all voxels of the masked difference, like the oracle's
    assert float(loss.cpu()) == pytest.approx(loss_r, rel=1e-4)
    for name in grads_r:
        e = rel(grads[name].cpu().numpy().reshape(np.shape(grads_r[name])), grads_r[name])
        print(f"  grad {name}: rel err {e:.2e}", flush=True)
        assert e <= 1e-3, name


def test_model_initialisation_is_plain_fbp(env):
    """At initialisation the learned pipeline equals the GPU plain FBP
    (fdk_prefilter + fdk_backproject) up to FP32 rounding."""
    torch, fdk, GL, dev = env
    g = synth.cone_beam_geometry(n_views=62, H=480, W=624, pixel=0.616)
    geo = GL.Geometry(P=g.P, betas=g.betas, H=g.H, W=g.W, sid=g.sid, sdd=g.sdd, pixel=g.pixel,
                      arc=g.arc)
    model = GL.LearnedFilter(geo, dev, sigma=1e-3)
    li = torch.from_numpy(synth.line_integrals(g, synth.ellipsoid_phantom())).to(dev)
    y3 = model.filter(li)
    q = torch.empty_like(li)
    fdk.prefilter(q, li, float(g.betas[0]), g.dbeta, 0.5 * (g.arc - math.pi), g.sid, g.sdd, g.pixel)
    torch.cuda.synchronize()
    e = rel(y3.cpu().numpy(), q.cpu().numpy())
    print(f"learned filter at init vs plain pre-filter: rel {e:.2e}", flush=True)
    assert e <= 1e-4


def test_learned_filter_beats_plain_fbp_on_held_out_phantoms(env):
    """Train on 32 seeded phantoms (two passes, 62 views of 624x480, 128^3,
    exact line integrals), then reconstruct two held-out phantoms: the
    learned filter's masked RMSE must be at least 2 % below plain FBP's."""
    torch, fdk, GL, dev = env
    g = synth.cone_beam_geometry(n_views=62, H=480, W=624, pixel=0.616)
    geo = GL.geometry_from(g)
    N = 128
    vs, o = synth.volume_frame(N)
    mask = torch.from_numpy(GL.fov_mask(N, vs, o, 110.0, 80.0)).to(dev)
    model = GL.LearnedFilter(geo, dev)
    model.sigma = GL.default_sigma(model, 1, N, vs, o)
    model.sigma_t.fill_(1.0 / model.sigma)
    model.sigma_f.fill_(model.sigma)
    before = GL.evaluate(model, [9999, 9998], N, vs, o, mask)
    for rp, rl in before:  # untrained: the learned path is plain FBP
        assert rl == pytest.approx(rp, rel=1e-4)
    GL.train(model, range(1, 33), N, vs, o, mask, epochs=2, lr=1e-3,
             log=lambda m: print(m, flush=True))
    after = GL.evaluate(model, [9999, 9998], N, vs, o, mask)
    for rp, rl in after:
        print(f"held-out RMSE: plain {rp:.4e} learned {rl:.4e}", flush=True)
        assert rl < 0.98 * rp
