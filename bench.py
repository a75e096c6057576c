"""GUP/s benchmark of the MI355X cone-beam backprojection.

One step = one full backprojection of the 512^3 workload: zero the volume,
then backproject all 496 filtered projections of 1248x960 (FP32) through
the C ABI (fdk_backproject).  Inputs are synthetic (seeded C-arm geometry
and ellipsoid phantom) and resident in HBM before the timed region.

Prints one JSON line with the throughput, the roofline position of the
backprojection kernel (timed with HIP events on its own stream), the
plain-path comparison on the same GPU, the error against the FP64 oracle on
a sampled slab, and the oracle's own throughput on the host cores.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import re
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GUP/s (voxel updates/s) at 512^3 x 496 views; RMSE vs FP64 oracle"
# algorithmic work per voxel update: 31 flop once invariants are hoisted and
# the three divides become one reciprocal (paper, Section 3.3)
FLOP_PER_UPDATE = 31
# FP32 vector peak without packed-FP32 instructions (disabled in this build):
# 256 CUs x 64 lanes x 2 flop (FMA) x 2.4 GHz
PEAK_FP32_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12
PEAK_HBM_GBS = 8000.0
# dense FP32 matrix-core (MFMA) peak of MI355X
PEAK_FP32_MFMA_TFLOPS = 157.3
# paper, Section 7.2: 3.79 GUP/s with IEEE divides, 512^3 x 496 views of
# 1248x960, 2-socket Xeon X5670 (Westmere EP), all optimisations
PAPER_GUPS = 3.79
# the sources the fused kernel's launches depend on (kernel, argument
# structs, device helpers, host set-up with its default layout)
KERNEL_SRC = [os.path.join(ROOT, "paper_1104_5243_amd", "csrc", f)
              for f in ("bp_kernels.hip", "anchor.h", "gfx950_util.h", "fdk_internal.h",
                        "api_internal.h", "api.hip")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "bp_fused_fdk512_traffic.txt")


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash() -> str:
    """Hash of the kernel sources' code (comments and blank lines removed),
    so that the recorded counter traffic stays tied to the code measured."""
    text = "".join(open(f).read() for f in KERNEL_SRC)
    text = re.sub(r"//[^\n]*", "", text)
    code = "\n".join(l.rstrip() for l in text.splitlines() if l.strip())
    return hashlib.sha256(code.encode()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the fused FP32 kernel from the committed
    rocprofv3 counter summary, or None if the kernel source changed since."""
    rec = {}
    try:
        for line in open(TRAFFIC_FILE):
            line = line.strip()
            if line and not line.startswith("#") and "=" in line:
                k, v = line.split("=", 1)
                rec[k.strip()] = v.strip()
    except OSError:
        return None
    if rec.get("kernel_sha") != kernel_hash() or "hbm_bytes_per_launch" not in rec:
        return None
    return int(float(rec["hbm_bytes_per_launch"]))


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def clipped_fraction(geom, N, vs, origin, stride=8):
    """Fraction of (voxel, view) pairs with every tap off the detector
    (u <= -1, u >= W, v <= -1 or v >= H, or w <= 0), over a sub-grid of
    voxels (every `stride`-th per axis) and all views, in FP64."""
    import numpy as np
    idx = np.arange(0, N, stride, dtype=np.float64)
    X = origin[0] + vs * idx
    Y = origin[1] + vs * idx
    Z = origin[2] + vs * idx
    xx, yy = np.meshgrid(X, Y, indexing="ij")
    off = 0
    total = 0
    for P in geom.P:
        for z in Z:
            uw = P[0, 0] * xx + P[0, 1] * yy + P[0, 2] * z + P[0, 3]
            vw = P[1, 0] * xx + P[1, 1] * yy + P[1, 2] * z + P[1, 3]
            w = P[2, 0] * xx + P[2, 1] * yy + P[2, 2] * z + P[2, 3]
            u = uw / w
            v = vw / w
            miss = (w <= 0) | (u <= -1) | (u >= geom.W) | (v <= -1) | (v >= geom.H)
            off += int(miss.sum())
            total += miss.size
    return {"exact_fraction": round(off / total, 4),
            "sample": f"every {stride}th voxel per axis x all {geom.n_views} views, FP64"}


def _timed(torch, fdk, fn, warmup, steps):
    """Wall time per step over `steps` calls (after `warmup`), and the mean
    duration of the library's kernels inside, from its HIP events."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    fdk.profile_begin()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    kernel_ms, launches = fdk.profile_end()
    return t, kernel_ms, launches


def _common(args, metric, value, unit, t, dtype, workload, roofline, cpu):
    return {
        "metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(t * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": {"workload": workload}, "roofline": roofline, "cpu_baseline": cpu,
    }


def bench_forward(args, torch, fdk, synth, dev):
    """Matched forward projection of a 256^3 phantom volume onto 248 views of
    624x480 (the exact transpose of the backprojection)."""
    import oracle
    geom, ell, vs, origin, N = synth.workload("fdk256x8")
    V, H, W = geom.n_views, geom.H, geom.W
    vol = synth.voxelize_torch(ell, N, vs, origin, dev, sub=1)
    proj = torch.zeros(V, H, W, device=dev)

    def step():
        proj.zero_()
        fdk.forward_project(proj, vol, geom.P, vs, origin)

    t, kms, launches = _timed(torch, fdk, step, args.warmup, args.steps)
    updates = float(N) ** 3 * V
    ks = kms / 1e3
    # The kernel skips the workgroup boxes (16 voxels across the rays, 32
    # along them, 16 in z) whose voxels are all zero: the roofline counts
    # the pairs of the other boxes only (both ray orientations, averaged).
    busy = []
    for shape in ((16, 32, 16), (32, 16, 16)):  # (x, y, z) extents: rays along y, along x
        bz, by, bx = shape[2], shape[1], shape[0]
        m = vol.abs().reshape(N // bz, bz, N // by, by, N // bx, bx).amax(dim=(1, 3, 5))
        busy.append(float((m > 0).float().mean()))
    work = sum(busy) / len(busy)
    ach = FLOP_PER_UPDATE * updates * work * args.steps / ks / 1e12
    log(f"forward: {t * 1e3:.2f} ms/step, {updates / t / 1e9:.1f} GUP/s; "
        f"{launches} scatter launches, {kms / max(launches, 1):.3f} ms each; "
        f"boxes holding mass {busy[0]:.3f} / {busy[1]:.3f}")
    # the oracle on the same volume and all views (under a second on 16 threads)
    Vs = V
    tc, err = None, None
    if not args.no_extras:
        vol_h = vol.double().cpu().numpy()
        t0 = time.perf_counter()
        ref = oracle.forward_project(vol_h, geom.P[:Vs], H, W, vs, origin)
        tc = time.perf_counter() - t0
        step()
        torch.cuda.synchronize()
        err = oracle.rel_rmse(proj[:Vs].double().cpu().numpy(), ref)
    out = _common(
        args, "forward projection voxel-view pairs/s at 256^3 x 248 views of 624x480",
        round(updates / t / 1e9, 2), "GUP/s", t, "f32",
        f"fdk256x8 forward: {N}^3 FP32 phantom volume, {V} views of {W}x{H}",
        {"bound": "alu", "achieved": round(ach, 3), "peak": round(PEAK_FP32_TFLOPS, 1),
         "unit": "TFLOP/s", "frac": round(ach / PEAK_FP32_TFLOPS, 4), "traffic": None,
         "kernel": "fp_lds_kernel (31 flop per pair of the boxes holding mass)",
         "work_fraction": round(work, 4),
         "launches_per_step": launches // args.steps,
         "kernel_ms_per_step": round(kms / args.steps, 3)},
        None if tc is None else
        {"value": round(float(N) ** 3 * Vs / tc / 1e9, 4), "unit": "GUP/s",
         "cores": oracle.threads(), "kind": "oracle",
         "sample": f"the whole workload: the {N}^3 volume onto all {Vs} views, FP64, "
                   f"{tc:.2f} s"})
    if err is not None:
        out["rel_rmse_vs_oracle"] = float(f"{err:.3e}")
    return out


def bench_autograd(args, torch, fdk, synth, dev):
    """The differentiable pair at its stated size: a batch of 8 volumes of
    256^3, 248 views of 624x480.  One step = BackProject forward (8
    backprojections) and, through autograd, its backward (8 forward
    projections of the volume gradient)."""
    import numpy as np

    import oracle
    from paper_1104_5243_amd import autograd as ag
    geom, ell, vs, origin, N = synth.workload("fdk256x8")
    V, H, W = geom.n_views, geom.H, geom.W
    B = 8
    t0 = time.time()
    stacks = []
    for k in range(B):
        e = synth.ellipsoid_phantom(5243 + k)
        stacks.append(torch.from_numpy(synth.filtered_projections(geom, e)))
    p = torch.stack(stacks).to(dev).requires_grad_(True)
    del stacks
    log(f"autograd: {B} stacks of {V} views {W}x{H} in {time.time() - t0:.1f}s")
    g = torch.Generator(device=dev).manual_seed(4)
    wv = torch.rand(B, N, N, N, device=dev, generator=g)

    def step():
        p.grad = None
        vol = ag.backproject_op(p, geom.P, N, vs, origin)
        vol.backward(wv)

    t, kms, launches = _timed(torch, fdk, step, args.warmup, args.steps)
    pairs = 2.0 * B * float(N) ** 3 * V  # both passes visit every (voxel, view) pair
    ks = kms / 1e3
    ach = FLOP_PER_UPDATE * pairs * args.steps / ks / 1e12
    log(f"autograd: {t * 1e3:.2f} ms/step, {pairs / t / 1e9:.1f} GUP/s; {launches} launches, "
        f"{kms / args.steps:.2f} ms of library kernels per step")
    tc, err_f, err_g = None, None, None
    if not args.no_extras:
        # item 0 against the oracle: two 32^3 blocks of the forward result,
        # and 3 views of the gradient (the forward projection of wv[0])
        vol = ag.backproject_op(p.detach(), geom.P, N, vs, origin)
        step()
        torch.cuda.synchronize()
        pr = p.detach()[0].cpu().numpy()
        num = den = 0.0
        t0 = time.perf_counter()
        for box in (((112, 32), (112, 32), (112, 32)), ((16, 32), (200, 32), (40, 32))):
            (x0, nx), (y0, ny), (z0, nz) = box
            ref = oracle.backproject(pr, geom.P, N, vs, origin, box=box)
            got = vol[0, z0:z0 + nz, y0:y0 + ny, x0:x0 + nx].double().cpu().numpy()
            num += float(((got - ref) ** 2).sum())
            den += float((ref ** 2).sum())
        tc = time.perf_counter() - t0
        err_f = (num / den) ** 0.5
        views = [0, 123, 247]
        refg = oracle.forward_project(wv[0].double().cpu().numpy(), geom.P[views], H, W, vs,
                                      origin)
        err_g = oracle.rel_rmse(p.grad[0, views].double().cpu().numpy(), refg)
        log(f"autograd item 0 vs oracle: forward blocks {err_f:.3e}, gradient views {err_g:.3e}")
    out = _common(
        args, "differentiable pair voxel-view pairs/s, batch 8 x 256^3, 248 views of 624x480",
        round(pairs / t / 1e9, 2), "GUP/s", t, "f32",
        f"fdk256x8 autograd: BackProject forward + ForwardProject backward of {B} x {N}^3 "
        f"FP32 volumes, {V} views of {W}x{H}",
        {"bound": "alu", "achieved": round(ach, 3), "peak": round(PEAK_FP32_TFLOPS, 1),
         "unit": "TFLOP/s", "frac": round(ach / PEAK_FP32_TFLOPS, 4), "traffic": None,
         "kernel": "bp_fused_kernel<f32> + fp_lds_kernel (31 flop per pair and pass)",
         "launches_per_step": launches // args.steps,
         "kernel_ms_per_step": round(kms / args.steps, 3)},
        None if tc is None else
        {"value": round(2 * 32 ** 3 * V / tc / 1e9, 4), "unit": "GUP/s",
         "cores": oracle.threads(), "kind": "oracle",
         "sample": f"two 32^3 blocks of item 0's backprojection x all {V} views, FP64, "
                   f"{tc:.2f} s"})
    out["config"]["batch"] = B
    if err_f is not None:
        out["rel_rmse_vs_oracle"] = {"forward_blocks": float(f"{err_f:.3e}"),
                                     "gradient_views": float(f"{err_g:.3e}")}
    return out


def bench_prefilter(args, torch, fdk, synth, dev):
    """Feldkamp pre-filter (cosine x Parker x Ram-Lak, FP64 inside) of the
    496 line-integral views of 1248x960."""
    import math

    import numpy as np

    from oracle.prefilter import fdk_prefilter
    geom, ell, vs, origin, N = synth.workload("fdk512")
    V, H, W = geom.n_views, geom.H, geom.W
    t0 = time.time()
    li = synth.line_integrals(geom, ell)
    log(f"line integrals {V}x{H}x{W} in {time.time() - t0:.1f}s")
    li_d = torch.from_numpy(li).to(dev)
    out_d = torch.empty_like(li_d)
    delta = 0.5 * (geom.arc - math.pi)

    def step():
        fdk.prefilter(out_d, li_d, float(geom.betas[0]), geom.dbeta, delta, geom.sid, geom.sdd,
                      geom.pixel)

    t, kms, launches = _timed(torch, fdk, step, args.warmup, args.steps)
    rows = V * H
    # FFT convolution of two rows per complex transform of length L, forward
    # and inverse, and the spectrum product (6 flop per point).  The library
    # takes L = 2560 = 10 x 16 x 16 for 513 <= W <= 1280: per 10-point group
    # two 5-point DFTs (48 flop each), 4 twiddle products and 10 complex
    # additions (44) and 9 twiddle products (54), 194 flop; per 16-point
    # group two radix-4 stages, 8 butterflies of 34 flop.  Power-of-two L:
    # radix 4 (34 flop per butterfly) and one radix-2 stage (10 flop) if
    # log2 L is odd.  (Counted without the pruning of zero inputs and unused
    # outputs that the kernels apply.)
    if 512 < W and 2 * W - 1 <= 2560:
        L = 2560
        per_transform = (L // 10) * 194 + 2 * (L // 16) * 8 * 34
    else:
        L, lg = 4, 2
        while L < 2 * W - 1:
            L, lg = 2 * L, lg + 1
        per_transform = (lg // 2) * (L // 4) * 34 + (lg % 2) * (L // 2) * 10
    flop = (rows + 1) // 2 * (2 * per_transform + 6 * L)
    ks = kms / 1e3
    ach = flop * args.steps / ks / 1e12
    log(f"prefilter: {t * 1e3:.2f} ms/step, {ach:.2f} TFLOP/s FP64")
    Vs = 2
    tc, err = None, None
    if not args.no_extras:
        t0 = time.perf_counter()
        ref = fdk_prefilter(li[:Vs], geom.betas[:Vs], delta, geom.dbeta, geom.sid, geom.sdd,
                            geom.pixel)
        tc = time.perf_counter() - t0
        err = float(np.sqrt(((out_d[:Vs].double().cpu().numpy() - ref) ** 2).sum()
                            / (ref ** 2).sum()))
    out = _common(
        args, "pre-filtered detector rows/s, 496 views of 1248x960", round(rows / t / 1e6, 3),
        "Mrow/s", t, "f64",
        f"fdk512 pre-filter: {V} line-integral views of {W}x{H}, FP32 in/out, FP64 inside",
        {"bound": "alu", "achieved": round(ach, 3), "peak": 78.6, "unit": "TFLOP/s",
         "frac": round(ach / 78.6, 4), "traffic": None,
         "kernel": ("fft_conv2560_kernel<true> (FP64 FFT, L=2560 = 10x16x16, passes in "
                    "registers, two rows per transform, real Ram-Lak spectrum)" if L == 2560 else
                    "fft_conv4096_real_kernel (FP64 FFT, L=4096, radix-16 passes in "
                    "registers, two rows per transform, real Ram-Lak spectrum)" if L == 4096 else
                    f"fft_conv_kernel (FP64 FFT, L={L}, two rows per transform)"),
         "flop_per_row_pair": 2 * per_transform + 6 * L,
         "launches_per_step": launches // args.steps,
         "kernel_ms_per_step": round(kms / args.steps, 3)},
        None if tc is None else
        {"value": round(Vs * H / tc / 1e6, 5), "unit": "Mrow/s", "cores": 1, "kind": "oracle",
         "sample": f"the first {Vs} of {V} views ({Vs * H} rows), np.convolve in FP64, "
                   f"{tc:.1f} s"})
    if err is not None:
        out["rel_rmse_vs_oracle"] = float(f"{err:.3e}")
    return out


def bench_learn_step(args, torch, fdk, synth, dev):
    """One training step of the learned filter (forward through the filter
    and the backprojection, masked MSE, backward through the forward
    projector, the CNN, the view weights and the ramp, Adam) at 128^3 x 62
    views of 624x480; the phantom's data are resident before timing."""
    import oracle
    from oracle import learned as OL
    from paper_1104_5243_amd import learned as GL
    g = synth.cone_beam_geometry(n_views=62, H=480, W=624, pixel=0.616)
    geo = GL.geometry_from(g)
    N = 128
    vs, o = synth.volume_frame(N)
    mask = torch.from_numpy(GL.fov_mask(N, vs, o, 110.0, 80.0)).to(dev)
    model = GL.LearnedFilter(geo, dev)
    model.sigma = GL.default_sigma(model, 1, N, vs, o)
    model.sigma_t.fill_(1.0 / model.sigma)
    model.sigma_f.fill_(model.sigma)
    gt, p = GL.phantom_case(1, geo, N, vs, o, dev)
    gm = gt * mask

    def step():
        _, grads = model.loss_and_grads(p, gm, mask, N, vs, o)
        model.apply_grads(grads, 0.0)  # lr 0: every kernel runs, parameters stay

    t, kms, launches = _timed(torch, fdk, step, args.warmup, args.steps)
    # the dominant kernel: the 32 -> 32 channel, 9-tap row convolution
    R, W = geo.V * geo.H, geo.W
    a1 = torch.randn(R, GL.CH, W, device=dev)
    a2 = torch.empty_like(a1)

    def conv():
        fdk.conv_rows(a2, a1, model.W2, model.b2, R, W, GL.CH, GL.CH, GL.KC, GL.KC // 2,
                      fdk.CONV_RELU)

    tcv, cms, cl = _timed(torch, fdk, conv, 1, 5)
    conv_s = cms / cl / 1e3
    conv_flop = 2.0 * R * W * GL.CH * GL.CH * GL.KC
    ach = conv_flop / conv_s / 1e12
    log(f"learn step: {t * 1e3:.1f} ms; conv 32->32: {conv_s * 1e3:.3f} ms, {ach:.1f} TFLOP/s")
    # oracle step on a bounded sample: 2 of the 62 views
    Vs = 2
    tc = None
    if not args.no_extras:
        params = {n: getattr(model, n).double().cpu().numpy() for n in model.params}
        params["lam"] = params["lam"][:Vs]
        T = GL.weight_table(geo)[:Vs]
        M, _, _ = GL.ramp_basis(geo)
        t0 = time.perf_counter()
        OL.loss_and_grads(params, p[:Vs].double().cpu().numpy(), T, M, geo.P[:Vs], N, vs, o,
                          model.sigma, gt.double().cpu().numpy(), mask.double().cpu().numpy())
        tc = time.perf_counter() - t0
    out = _common(
        args, "learned-filter training steps/s at 128^3 x 62 views of 624x480",
        round(1.0 / t, 3), "steps/s", t, "f32",
        "learn128: one Adam step of the learned Feldkamp filter (1025-bin ramp, 62 view "
        "weights, 1->32->32->1 9-tap row CNN) through backprojection and its adjoint",
        {"bound": "mfma", "achieved": round(ach, 3), "peak": PEAK_FP32_MFMA_TFLOPS,
         "unit": "TFLOP/s", "frac": round(ach / PEAK_FP32_MFMA_TFLOPS, 4), "traffic": None,
         "kernel": "conv_mfma_kernel<32,32,9> (FP32 MFMA)",
         "kernel_ms": round(conv_s * 1e3, 3)},
        None if tc is None else
        {"value": round(Vs / geo.V / tc, 5), "unit": "steps/s", "cores": oracle.threads(),
         "kind": "oracle",
         "sample": f"FP64 oracle step on {Vs} of {geo.V} views ({tc:.1f} s), scaled by "
                   f"{Vs}/{geo.V} to a full step"})
    out["library_kernel_ms_per_step"] = round(kms / args.steps, 3)
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--kernel", choices=("fused", "plain"), default="fused")
    ap.add_argument("--storage", choices=("f32", "f16", "bf16"), default="f32",
                    help="projection storage type of the fused path (arithmetic is FP32)")
    ap.add_argument("--workload", choices=("fdk512", "fdk1024"), default="fdk512")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the plain comparison, oracle sample and CPU baseline "
                         "(for profiler runs)")
    ap.add_argument("--cpu-slices", type=int, default=128,
                    help="z slices of the 512^3 volume in the CPU-baseline sample")
    ap.add_argument("--probe-hbm", action="store_true",
                    help="also run the update benchmark a[i] = s*a[i] over 2 GiB")
    ap.add_argument("--path", choices=("backproject", "forward", "prefilter", "learn-step",
                                        "autograd"),
                    default="backproject",
                    help="which part to measure: the backprojection (default), the matched "
                         "forward projector, the Feldkamp pre-filter, one training step "
                         "of the learned filter, or the differentiable pair (batch of 8)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the backprojection's multi-GPU z-slab sharding is a design, not built)",
              file=sys.stderr)
        return 2
    if args.steps < 1 or args.warmup < 0:
        print("need --steps >= 1 and --warmup >= 0", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1104_5243_amd as fdk
    import synth

    fdk.lib()  # fails loudly if the HIP library is not built
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.path != "backproject":
        out = {"forward": bench_forward, "prefilter": bench_prefilter,
               "learn-step": bench_learn_step, "autograd": bench_autograd}[args.path](
            args, torch, fdk, synth, dev)
        print(json.dumps(out), flush=True)
        return 0

    geom, ell, vs, origin, N = synth.workload(args.workload)
    V, H, W = geom.n_views, geom.H, geom.W
    t0 = time.time()
    proj = synth.filtered_projections(geom, ell)
    log(f"synthesised {V} views {W}x{H} in {time.time() - t0:.1f}s")
    proj32_d = torch.from_numpy(proj).to(dev)
    sdt = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[args.storage]
    proj_d, view_scale = fdk.to_storage(proj32_d, sdt)
    if args.storage != "f32":
        del proj32_d
    vol = torch.empty(N, N, N, device=dev)
    torch.cuda.synchronize()
    updates = float(N) ** 3 * V

    def step(kernel):
        vol.zero_()
        if kernel == "fused":
            fdk.backproject(vol, proj_d, geom.P, vs, origin, view_scale=view_scale)
        else:
            fdk.backproject_plain(vol, proj_d, geom.P, vs, origin)

    for _ in range(args.warmup):
        step(args.kernel)
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} done; timing {args.steps} steps")

    fdk.profile_begin()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(args.kernel)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    kernel_ms, launches = fdk.profile_end()
    gups = updates * args.steps / t / 1e9
    log(f"{args.kernel}: {t / args.steps * 1e3:.2f} ms/step, {gups:.1f} GUP/s; "
        f"{launches} kernel launches, {kernel_ms / max(launches, 1):.3f} ms each")

    # roofline of the backprojection kernel: algorithmic flops per launch over
    # its mean duration (HIP events on the launch stream)
    kernel_s = kernel_ms / 1e3
    achieved_tflops = FLOP_PER_UPDATE * updates * args.steps / kernel_s / 1e12
    traffic = (measured_traffic() if args.kernel == "fused" and args.storage == "f32"
               and args.workload == "fdk512" else None)
    roofline = {
        "bound": "alu",
        "achieved": round(achieved_tflops, 3),
        "peak": round(PEAK_FP32_TFLOPS, 1),
        "unit": "TFLOP/s",
        "frac": round(achieved_tflops / PEAK_FP32_TFLOPS, 4),
        "traffic": traffic,
        "kernel": (f"bp_fused_kernel<{args.storage}>" if args.kernel == "fused"
                   else "bp_plain_kernel"),
        "launches_per_step": launches // args.steps,
        "kernel_ms_per_step": round(kernel_ms / args.steps, 3),
        "kernel_gups": round(updates * args.steps / kernel_s / 1e9, 1),
    }
    # the other bounds of the same kernel time: HBM at the algorithmic bytes
    # (each view read once, one volume read-modify-write per launch) and at
    # the measured traffic, if recorded
    esz = {"f32": 4, "f16": 2, "bf16": 2}[args.storage]
    alg_bytes = 8.0 * N ** 3 * (launches // args.steps) + float(V) * H * W * esz
    alg_tbs = alg_bytes * args.steps / kernel_s / 1e12
    roofline["other_bounds"] = {
        "hbm_algorithmic": {"achieved_TBps": round(alg_tbs, 3), "peak_TBps": PEAK_HBM_GBS / 1e3,
                            "frac": round(alg_tbs / (PEAK_HBM_GBS / 1e3), 4)},
        "hbm_measured": None if traffic is None else {
            "achieved_TBps": round(traffic * launches / kernel_s / 1e12, 3),
            "peak_TBps": PEAK_HBM_GBS / 1e3},
    }

    out = {
        "metric": METRIC,
        "value": round(gups, 2),
        "unit": "GUP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": round(gups / PAPER_GUPS, 1),
        "vs_baseline_ref": "3.79 GUP/s: paper Sec. 7.2, 512^3 x 496 views of 1248x960, "
                           "2x Xeon X5670, IEEE divide (another machine; context)",
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {N}^3 FP32 volume (256 mm cube), {V} views "
                               f"of {W}x{H} {args.storage.upper()} filtered projections, "
                               "200-degree C-arm short scan, seeded ellipsoid phantom",
                   "N": N, "n_views": V, "H": H, "W": W, "kernel": args.kernel},
        "roofline": roofline,
    }

    if args.storage != "f32" or args.kernel != "fused":
        out["config"]["storage"] = args.storage
    if not args.no_extras and args.storage == "f32" and args.workload == "fdk512":
        # the plain FP32 path on the same GPU
        other = "plain" if args.kernel == "fused" else "fused"
        step(other)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 2
        for _ in range(reps):
            step(other)
        torch.cuda.synchronize()
        tp = (time.perf_counter() - t0) / reps
        out[f"{other}_gpu"] = {"value": round(updates / tp / 1e9, 2), "unit": "GUP/s",
                               "ms_per_step": round(tp * 1e3, 3)}
        log(f"{other}: {tp * 1e3:.2f} ms/step")

        # accuracy and CPU baseline on a central slab of the same workload
        import oracle
        step(args.kernel)
        torch.cuda.synchronize()
        S = args.cpu_slices
        z0 = N // 2 - S // 2
        got = vol[z0:z0 + S].double().cpu().numpy()
        cores = oracle.threads()
        log(f"oracle on {N}x{N}x{S} slab x {V} views, {cores} threads")
        t0 = time.perf_counter()
        ref = oracle.backproject(proj, geom.P, N, vs, origin, box=((0, N), (0, N), (z0, S)))
        tc = time.perf_counter() - t0
        cpu_updates = float(N) * N * S * V
        out["rel_rmse_vs_oracle"] = float(f"{oracle.rel_rmse(got, ref):.3e}")
        out["psnr_db_vs_oracle"] = round(oracle.psnr(got, ref), 1)
        out["cpu_baseline"] = {
            "value": round(cpu_updates / tc / 1e9, 4), "unit": "GUP/s", "cores": cores,
            "kind": "oracle",
            "sample": f"z-slab [{z0},{z0 + S}) of the 512^3 volume (512x512x{S} voxels) x "
                      f"all {V} views, FP64, {tc:.1f} s",
        }
        log(f"oracle: {tc:.1f}s, relRMSE {out['rel_rmse_vs_oracle']:.3e}")
        out["cpu_baseline"]["cpu_model"] = cpu_model()

        # the divide variants of part 1 (the paper's accuracy study, Section
        # 7.2) on the same stack: throughput and error on the same slab
        divides = {}
        for dv in ("rcp", "rcp_nr", "ieee", "rcp12"):
            fdk.set_divide(dv)
            step("fused")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                step("fused")
            torch.cuda.synchronize()
            td = (time.perf_counter() - t0) / 3
            gd = vol[z0:z0 + S].double().cpu().numpy()
            divides[dv] = {"value": round(updates / td / 1e9, 2), "unit": "GUP/s",
                           "ms_per_step": round(td * 1e3, 3),
                           "rel_rmse_vs_oracle": float(f"{oracle.rel_rmse(gd, ref):.3e}"),
                           "psnr_db_vs_oracle": round(oracle.psnr(gd, ref), 1)}
        fdk.set_divide("rcp")
        out["divide_variants"] = divides
        log(f"divide variants: {divides}")

        # clipping: the exact fraction of (voxel, view) pairs whose four taps
        # all lie off the detector (every 8th voxel per axis, all views)
        out["clipping"] = clipped_fraction(geom, N, vs, origin)
        log(f"clipping: {out['clipping']}")

        # reduced-precision storage of the same stack on the same GPU
        variants = {}
        for name, dt in (("f16", torch.float16), ("bf16", torch.bfloat16)):
            st, sc = fdk.to_storage(proj_d, dt)
            vol.zero_()
            fdk.backproject(vol, st, geom.P, vs, origin, view_scale=sc)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                vol.zero_()
                fdk.backproject(vol, st, geom.P, vs, origin, view_scale=sc)
            torch.cuda.synchronize()
            ts = (time.perf_counter() - t0) / 3
            variants[name] = {"value": round(updates / ts / 1e9, 2), "unit": "GUP/s",
                              "ms_per_step": round(ts * 1e3, 3)}
            del st
        out["storage_variants"] = variants
        log(f"storage variants: {variants}")

        # context, not the metric: the stack copied from pinned host memory
        # (PCIe) and backprojected
        host = torch.empty(proj_d.shape, dtype=proj_d.dtype, pin_memory=True)
        host.copy_(proj_d)
        dst = torch.empty_like(proj_d)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dst.copy_(host, non_blocking=True)
        vol.zero_()
        fdk.backproject(vol, dst, geom.P, vs, origin)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        out["pcie_inclusive_context"] = {
            "value": round(updates / tp / 1e9, 2), "unit": "GUP/s", "ms": round(tp * 1e3, 3),
            "note": f"H2D copy of the {proj_d.numel() * 4 / 1e9:.2f} GB FP32 stack from pinned "
                    "memory + backprojection; not the metric"}
        del host, dst

    if args.probe_hbm:
        a = torch.ones(512 * 1024 * 1024, device=dev)  # 2 GiB
        fdk.update_probe(a)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(5):
            fdk.update_probe(a)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / 5
        out["hbm_update_probe_gbs"] = round(2 * a.numel() * 4 / (ms / 1e3) / 1e9, 1)
        log(f"update probe: {out['hbm_update_probe_gbs']} GB/s")

    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
