#!/usr/bin/env python
"""Benchmark of the WSKP per-frame path on one MI355X.

Workload: one synthetic 1280x720 frame (1-spp-like noisy radiance + albedo,
normal, depth), a 4-level U-Net (32/64/96/128 channels) predicting 5 weight
maps (k = 3, 5, 7, 9, 11) and 5 fusion logits, then the fused decode +
fusion + remodulation.  A step is one whole frame through wskp_denoise
(input pack, encoder, decoder, head, decode), inputs resident in HBM.

Prints ONE JSON line on stdout.  `value` is frames/s of the BF16-conv path
(the FP32 path is reported beside it), `roofline` is for the kernel that
takes the most time per frame, `decode_roofline` for the decode kernel,
`cpu_baseline` is the FP64 CPU oracle on the same frame.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("1280×720 frames/s + p50/p99 ms; decode HBM GB/s %peak; "
          "BF16 vs FP32 at stated err")
PEAK = {"fp32": 157.3e12, "bf16": 2.5e15, "fp8": 5.0e15}   # dense MFMA FLOP/s
HBM_PEAK = 8.0e12                                          # bytes/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def conv_flops(cfg, H, W):
    """Algorithmic FLOPs of each conv layer (2 * pixels * 9 * Cin * Cout)."""
    from paper_2202_05977_amd import synth
    out = {}
    for name, ci, co in synth.conv_shapes(cfg):
        lvl = 0 if name in ("head",) else int(name[3:])
        px = (H >> lvl) * (W >> lvl)
        out[name] = 2.0 * px * 9 * ci * co
    return out


def decode_bytes(cfg, H, W):
    """Algorithmic HBM bytes of the fused decode: head (2M floats), radiance,
    albedo read once, output written once."""
    return float(H * W * (2 * cfg.M * 4 + 12 + 12 + 12))


def time_precision(cfg, blob, dev, H, W, prec, steps, warmup, lat_frames):
    import torch
    from paper_2202_05977_amd import wskp
    dn = wskp.Denoiser(cfg, blob, prec)
    out = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        dn(dev, out)
    torch.cuda.synchronize()
    # throughput: frames queued back to back on one stream
    t0 = time.perf_counter()
    for _ in range(steps):
        dn(dev, out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / steps
    # latency: one frame at a time, HIP events on the launch stream
    lat = []
    for _ in range(lat_frames):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        dn(dev, out)
        e1.record(stream)
        e1.synchronize()
        lat.append(e0.elapsed_time(e1))
    # per-kernel durations: events recorded by the library around each launch
    kt = max(1, min(steps, 100))
    wskp.wskp_timing_enable(dn.h, kt)
    for _ in range(kt):
        dn(dev, out)
    ms, ncalls = wskp.wskp_timing_read(dn.h)
    wskp.wskp_timing_enable(dn.h, 0)
    per_kernel_us = {k: 1e3 * v / ncalls for k, v in ms.items()}
    torch.cuda.synchronize()
    y = out.cpu().numpy().astype(np.float64)
    dn.close()
    lat = np.array(lat)
    return {
        "ms_per_step": ms_per_step,
        "fps": 1e3 / ms_per_step,
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "per_kernel_us": per_kernel_us,
        "y": y,
    }


def omp_threads() -> int:
    try:
        omp = ctypes.CDLL("libgomp.so.1")
        return int(omp.omp_get_max_threads())
    except OSError:
        return os.cpu_count() or 1


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precisions", default="bf16,fp32",
                    help="first one is the headline value")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle leg (no error or CPU figures)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="only run a plain device copy of MB megabytes 5 times (reference "
                         "kernel for scaling HBM traffic counters) and exit")
    ap.add_argument("--height", type=int, default=720)
    ap.add_argument("--width", type=int, default=1280)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); frames are "
              "independent, so several GPUs would each run this same loop.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2202_05977_amd import synth, wskp  # noqa: F401

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "launches": 5}))
        return

    H, W = args.height, args.width
    cfg = synth.HD
    blob = synth.make_weights(cfg, 0)
    fr = synth.make_frame(1, H, W)
    dev = {k: torch.from_numpy(v).cuda() for k, v in fr.items()}
    torch.cuda.synchronize()
    precs = args.precisions.split(",")
    res = {}
    for p in precs:
        log(f"[bench] timing {p} at {W}x{H}: warmup {args.warmup}, steps {args.steps}")
        res[p] = time_precision(cfg, blob, dev, H, W, p, args.steps, args.warmup,
                                min(args.steps, 300))
        log(f"[bench] {p}: {res[p]['fps']:.1f} frames/s, {res[p]['ms_per_step']:.3f} ms/frame, "
            f"p50 {res[p]['p50_ms']:.3f} p99 {res[p]['p99_ms']:.3f} ms")
        log(f"[bench] {p} per kernel (us): " +
            ", ".join(f"{k} {v:.1f}" for k, v in res[p]["per_kernel_us"].items()))

    head = precs[0]
    flops = conv_flops(cfg, H, W)
    pk = res[head]["per_kernel_us"]
    dom = max(pk, key=pk.get)
    if dom == "decode":
        achieved = decode_bytes(cfg, H, W) / (pk[dom] * 1e-6)
        roof = {"kernel": dom, "bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9,
                "unit": "GB/s", "frac": achieved / HBM_PEAK, "traffic": None}
    else:
        achieved = flops[dom] / (pk[dom] * 1e-6)
        roof = {"kernel": dom, "bound": "mfma", "achieved": achieved / 1e12,
                "peak": PEAK[head] / 1e12, "unit": "TFLOP/s", "frac": achieved / PEAK[head],
                "traffic": None}
    dbytes = decode_bytes(cfg, H, W)
    dec_gbs = dbytes / (pk["decode"] * 1e-6)
    decode_roof = {"kernel": "decode", "bound": "hbm", "achieved": dec_gbs / 1e9,
                   "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": dec_gbs / HBM_PEAK,
                   "bytes_per_launch": dbytes, "traffic": None}
    conv_mfma = {}
    for p in precs:
        tot = sum(flops.values())
        t = sum(v for k, v in res[p]["per_kernel_us"].items() if k != "decode") * 1e-6
        conv_mfma[p] = {"tflops": tot / t / 1e12, "frac_of_peak": tot / t / PEAK[p]}

    cpu = None
    errors = {}
    if not args.no_cpu_baseline:
        import oracle
        threads = omp_threads()
        log(f"[bench] FP64 oracle on the same {W}x{H} frame ({threads} threads)")
        t0 = time.perf_counter()
        yref = oracle.denoise(fr, blob, cfg)
        dt = time.perf_counter() - t0
        cpu = {"value": 1.0 / dt, "unit": "frames/s", "cores": threads, "kind": "oracle",
               "sample": f"one full {W}x{H} frame of the same workload (FP64 U-Net + decode), "
                         f"{dt:.1f} s"}
        for p in precs:
            y = res[p]["y"]
            errors[p] = {
                "rel_l2": float(np.linalg.norm(y - yref) / np.linalg.norm(yref)),
                "max_rel": float(np.abs(y - yref).max() / np.abs(yref).max()),
            }
        log(f"[bench] errors vs FP64 oracle: {errors}")

    line = {
        "metric": METRIC,
        "value": res[head]["fps"],
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res[head]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head,
        "data": "synthetic",
        "config": {"workload": f"{W}x{H} frame, 4-level U-Net 32/64/96/128, "
                               f"M=5 kernels k=3..11, convs {head}, decode fp32",
                   "height": H, "width": W, "conv_precision": head},
        "latency_ms": {"p50": res[head]["p50_ms"], "p99": res[head]["p99_ms"]},
        "per_kernel_us": res[head]["per_kernel_us"],
        "roofline": roof,
        "decode_roofline": decode_roof,
        "conv_mfma": conv_mfma,
        "error_vs_fp64_oracle": errors,
        "precisions": {p: {"frames_per_s": res[p]["fps"], "ms_per_step": res[p]["ms_per_step"],
                           "p50_ms": res[p]["p50_ms"], "p99_ms": res[p]["p99_ms"],
                           "per_kernel_us": res[p]["per_kernel_us"]} for p in precs},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
