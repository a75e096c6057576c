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
# paper, Section 7.2: 3.79 GUP/s with IEEE divides, 512^3 x 496 views of
# 1248x960, 2-socket Xeon X5670 (Westmere EP), all optimisations
PAPER_GUPS = 3.79
KERNEL_SRC = os.path.join(ROOT, "paper_1104_5243_amd", "csrc", "bp_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "bp_fused_fdk512_traffic.txt")


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash() -> str:
    """Hash of the kernel source's code (comments and blank lines removed),
    so that the recorded counter traffic stays tied to the code measured."""
    text = open(KERNEL_SRC).read()
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
