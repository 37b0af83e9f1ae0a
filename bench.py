#!/usr/bin/env python
"""Benchmark of the WSKP per-frame path on one MI355X.

Workload: one synthetic 1280x720 frame (1-spp-like noisy radiance + albedo,
normal, depth), a 4-level U-Net (32/64/96/128 channels) predicting 5 weight
maps (k = 3, 5, 7, 9, 11) and 5 fusion logits, then the fused decode +
fusion + remodulation.  A step is one whole frame through wskp_denoise
(input pack, encoder, decoder, head, decode), inputs resident in HBM.

Prints ONE JSON line on stdout.  `value` is frames/s of the BF16-conv path
with consecutive frames in flight on --streams HIP streams (frames/s on one
stream, latency of single frames and the FP32 path are reported beside it),
`roofline` is for the kernel that
takes the most time per frame, `decode_roofline` for the decode kernel,
`serving` compares bf16 continuous batching with the plain per-frame loop
(bf16 and fp32) on one 64-stream request trace of mixed resolutions (not
part of the timed region), `cpu_baseline` is the FP64 CPU oracle on the
same frame.
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


def time_precision(cfg, blob, dev, H, W, prec, steps, warmup, lat_frames, nstreams=3):
    import torch
    from paper_2202_05977_amd import synth, wskp
    scales = None
    if prec == "fp8":
        # activation scales calibrated on a different frame (seed 999) by the fp32 path
        calib = {k: torch.from_numpy(v).cuda() for k, v in synth.make_frame(999, H, W).items()}
        scales = wskp.calibrate_fp8_scales(cfg, blob, calib)
    dn = wskp.Denoiser(cfg, blob, prec, act_scales=scales)
    out = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        dn(dev, out)
    torch.cuda.synchronize()
    # throughput, one stream: frames queued back to back
    t0 = time.perf_counter()
    for _ in range(steps):
        dn(dev, out)
    torch.cuda.synchronize()
    ms_single = (time.perf_counter() - t0) * 1e3 / steps
    # throughput, several streams (the headline): consecutive frames go to
    # the streams in turn, each stream with its own workspace and output, so
    # that one frame's kernels fill the CUs another frame's ramp-down and
    # ramp-up leave idle
    extra = [wskp.Denoiser(cfg, blob, prec, act_scales=scales) for _ in range(nstreams - 1)]
    lanes = [(dn, out)] + [(d, torch.empty_like(out)) for d in extra]
    streams = [torch.cuda.Stream() for _ in range(nstreams)]
    for s_ in streams:
        s_.wait_stream(stream)

    def pipelined(n):
        for k in range(n):
            d_, o_ = lanes[k % nstreams]
            d_(dev, o_, stream=streams[k % nstreams])

    pipelined(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pipelined(steps)
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1e3 / steps
    # every stream's last frame is bitwise the one-stream result of the frame
    ref = dn(dev, torch.empty_like(out))
    torch.cuda.synchronize()
    streams_equal = all(bool(torch.equal(o_, ref)) for _, o_ in lanes)
    for d in extra:
        d.close()
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
    # throughput with the frame's launches captured once in a HIP graph
    g = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    cap.wait_stream(stream)
    with torch.cuda.stream(cap):
        dn(dev, out)                      # warm the capture stream
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=cap):
            dn(dev, out)
    torch.cuda.synchronize()
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    ms_graph = (time.perf_counter() - t0) * 1e3 / steps
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
        "streams": nstreams,
        "single_stream_ms_per_step": ms_single,
        "single_stream_fps": 1e3 / ms_single,
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "graph_fps": 1e3 / ms_graph,
        "streams_equal_single": streams_equal,
        "per_kernel_us": per_kernel_us,
        "y": y,
    }


def decode_cold_warm(cfg, blob, H, W, reps=20):
    """The decode alone (tensor form, wskp_decode) on one H x W frame, timed
    with HIP events: warm (launched back to back, inputs left in the caches by
    the previous launch) and cold (a 1 GiB buffer written between launches
    evicts the L2s and the 256 MB last-level cache first)."""
    import torch
    from paper_2202_05977_amd import wskp
    g = torch.Generator().manual_seed(5)
    M = len(cfg.kernel_sizes)
    head = torch.randn(1, H, W, 2 * M, generator=g).cuda()
    head[..., :M] = torch.nn.functional.softplus(head[..., :M])
    c = torch.rand(1, H, W, 3, generator=g).cuda()
    mod = torch.rand(1, H, W, 3, generator=g).cuda() + 0.1
    out = torch.empty_like(c)
    dn = wskp.Denoiser(cfg, blob, "fp32")
    flush = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream()

    def timed(cold):
        ts = []
        for _ in range(reps):
            if cold:
                flush.fill_(1)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            wskp.wskp_decode(dn.h, head, c, mod, out)
            e1.record(s)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e3)
        return float(np.median(ts))

    timed(False)
    warm, cold = timed(False), timed(True)
    dn.close()
    b = H * W * (8 * M + 36)        # head 2M floats + c + mod read, out written
    return {"workload": f"{W}x{H}, M={M}, tensor form", "bytes": b,
            "warm_us": warm, "cold_us": cold,
            "warm_GBps": b / warm / 1e3, "cold_GBps": b / cold / 1e3}


def gpu_clocks():
    """Shader and memory clock levels the driver reports (the current level
    is marked with *), where the sysfs files are readable."""
    import glob
    out = {}
    for dev in sorted(glob.glob("/sys/class/drm/card*/device")):
        for k in ("pp_dpm_sclk", "pp_dpm_mclk"):
            try:
                with open(os.path.join(dev, k)) as f:
                    cur = [l.strip() for l in f if l.strip().endswith("*")]
                if cur:
                    out.setdefault(os.path.basename(os.path.dirname(dev)), {})[k] = cur[0]
            except OSError:
                pass
    return out or None


def rel_errors(y, yref):
    return {"rel_l2": float(np.linalg.norm(y - yref) / np.linalg.norm(yref)),
            "max_rel": float(np.abs(y - yref).max() / np.abs(yref).max()),
            "max_abs": float(np.abs(y - yref).max())}


def mode_sweep(args):
    """1920x1080 frame: frames/s and error vs the FP64 oracle per precision."""
    import torch
    import oracle
    from paper_2202_05977_amd import synth
    H, W = 1080, 1920
    cfg = synth.HD
    blob = synth.make_weights(cfg, 0)
    fr = synth.make_frame(1, H, W)
    dev = {k: torch.from_numpy(v).cuda() for k, v in fr.items()}
    log("[sweep] FP64 oracle at 1920x1080")
    yref = oracle.denoise(fr, blob, cfg)
    out = {}
    for p in args.precisions.split(","):
        r = time_precision(cfg, blob, dev, H, W, p, args.steps, args.warmup, min(args.steps, 100),
                           args.streams)
        out[p] = {"frames_per_s": r["fps"], "graph_frames_per_s": r["graph_fps"],
                  "p50_ms": r["p50_ms"], "p99_ms": r["p99_ms"],
                  "per_kernel_us": r["per_kernel_us"], **rel_errors(r["y"], yref)}
        log(f"[sweep] {p}: {r['fps']:.1f} frames/s, errors {rel_errors(r['y'], yref)}")
    print(json.dumps({"mode": "precision_sweep", "workload": "1920x1080 frame, hd net",
                      "results": out}), flush=True)


def mode_train(args):
    """8 crops of 256x256: decode forward + L1 cotangent + hand-written adjoint."""
    import torch
    import oracle
    from paper_2202_05977_amd import synth, wskp
    N, H, W = 8, 256, 256
    cfg = synth.HD
    blob = synth.make_weights(cfg, 0)
    fb = synth.make_frame_batch(range(2000, 2000 + N), H, W)
    # head records from the network itself (fp32), one frame at a time
    dn = wskp.Denoiser(cfg, blob, "fp32")
    heads = []
    for n in range(N):
        f = {k: torch.from_numpy(fb[k][n]).cuda() for k in ("radiance", "albedo", "normal", "depth")}
        dn(f)
        heads.append(dn.intermediate([H], [W], 0, 200).clone())
    head = torch.stack(heads).contiguous()
    r = torch.from_numpy(fb["radiance"]).cuda()
    a = torch.from_numpy(fb["albedo"]).cuda()
    t = torch.from_numpy(fb["clean"]).cuda()
    mod = a + cfg.eps_albedo
    c = r / mod
    out = torch.empty_like(c)
    gh = torch.empty_like(head)
    gc = torch.empty_like(c)
    ws = torch.empty(wskp.wskp_backward_workspace_size(dn.h, N, H, W), dtype=torch.uint8,
                     device="cuda")
    def step():
        wskp.wskp_decode(dn.h, head, c, mod, out)
        g = torch.sign(out - t) / out.numel()          # L1 cotangent
        wskp.wskp_backward(dn.h, head, c, mod, g, gh, gc, ws)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    # kernel times with events on the launch stream: 20 calls of each queued
    # back to back between two events (one call between events would also
    # time its own launch from the host), median over 5 such rounds
    s = torch.cuda.current_stream()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    g = torch.sign(out - t) / out.numel()
    fw, bw = [], []
    for _ in range(5):
        wskp.wskp_decode(dn.h, head, c, mod, out)
        e[0].record(s)
        for _ in range(20):
            wskp.wskp_decode(dn.h, head, c, mod, out)
        e[1].record(s)
        for _ in range(20):
            wskp.wskp_backward(dn.h, head, c, mod, g, gh, gc, ws)
        e[2].record(s)
        e[2].synchronize()
        fw.append(e[0].elapsed_time(e[1]) / 20)
        bw.append(e[1].elapsed_time(e[2]) / 20)
    px = N * H * W
    fwd_us, bwd_us = 1e3 * float(np.median(fw)), 1e3 * float(np.median(bw))
    # adjoint against the oracle VJP on crop 0 with the same cotangent
    g0 = g[0].double().cpu().numpy()
    rh, rc = oracle.decode_vjp(head[0].double().cpu().numpy(), c[0].double().cpu().numpy(),
                               mod[0].double().cpu().numpy(), cfg.kernel_sizes, g0)
    err = {"grad_head_rel_l2": float(np.linalg.norm(gh[0].double().cpu().numpy() - rh) /
                                     np.linalg.norm(rh)),
           "grad_c_rel_l2": float(np.linalg.norm(gc[0].double().cpu().numpy() - rc) /
                                  np.linalg.norm(rc))}
    # the whole training step of the network (Eq. 1, SMAPE of Eq. 6, Adam):
    # forward of the 8 crops, loss, every layer's gradients, one Adam update
    frames = []
    for n in range(N):
        f = {k: torch.from_numpy(fb[k][n]).cuda() for k in ("radiance", "albedo", "normal", "depth")}
        f["out"] = torch.empty_like(f["radiance"])
        frames.append(f)
    targets = [t[n] for n in range(N)]
    nw = blob.size
    grad = torch.empty(nw, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    m1 = torch.zeros(nw, dtype=torch.float32, device="cuda")
    v1 = torch.zeros(nw, dtype=torch.float32, device="cuda")
    tws = torch.empty(wskp.wskp_train_workspace_size(dn.h, [H] * N, [W] * N), dtype=torch.uint8,
                      device="cuda")
    losses = []
    for k in range(args.warmup):
        wskp.wskp_train_grads(dn.h, frames, targets, grad, loss, tws)
        wskp.wskp_adam(dn.h, grad, m1, v1, k + 1, lr=1e-3)
    torch.cuda.synchronize()
    steps = max(1, min(args.steps, 50))
    t0 = time.perf_counter()
    for k in range(steps):
        wskp.wskp_train_grads(dn.h, frames, targets, grad, loss, tws)
        wskp.wskp_adam(dn.h, grad, m1, v1, args.warmup + k + 1, lr=1e-3)
        if k in (0, steps - 1):
            losses.append(float(loss.item()))
    torch.cuda.synchronize()
    ms_train = (time.perf_counter() - t0) * 1e3 / steps
    fl = conv_flops(cfg, H, W)
    step_flops = 3.0 * N * sum(fl.values())   # forward + input and weight gradients
    print(json.dumps({
        "mode": "train_step", "workload": "8 crops of 256x256, decode+fusion forward, L1, adjoint",
        "crops_per_s": N * 1e3 / ms, "ms_per_step": ms,
        "decode_fwd_us": fwd_us, "adjoint_us": bwd_us,
        "decode_fwd_GBps": px * 76 / (fwd_us * 1e-6) / 1e9,
        "adjoint_GBps_algorithmic": px * 128 / (bwd_us * 1e-6) / 1e9,
        "adjoint_vs_fp64_oracle": err,
        "network_training_step": {
            "workload": "8 crops of 256x256, hd net fp32, SMAPE loss, all layers' gradients, Adam",
            "ms_per_step": ms_train, "crops_per_s": N * 1e3 / ms_train,
            "conv_flops_per_step": step_flops, "achieved_TFLOPs": step_flops / ms_train / 1e9,
            "loss_first_and_last_timed_step": losses}}), flush=True)
    dn.close()


def serve_setup(args):
    """The C4 workload: 64 streams with resolutions drawn from 360p..1440p,
    Poisson arrivals at 2000 frames/s in total, ``--serve-frames`` frames per
    stream, every stream's input frame resident on the device."""
    import torch
    from paper_2202_05977_amd import serve, synth
    sizes, reqs = serve.poisson_trace(64, args.serve_frames, 2000.0, synth.SERVE_RESOLUTIONS,
                                      seed=7)
    proto = {}
    for (H, W) in set(sizes):
        proto[(H, W)] = {k: torch.from_numpy(v).cuda()
                         for k, v in synth.make_frame(1000 + H, H, W).items() if k != "clean"}
    inputs = {s: {k: v.clone() for k, v in proto[sizes[s]].items()} for s in range(64)}
    return sizes, reqs, proto, inputs


def _warm(serve, ex, sizes, proto):
    for (H, W) in proto:
        tok = ex.launch([serve.Request(-1, sizes.index((H, W)), 0.0, H, W)], 0, 0)
        ex.wait(tok)


def _stats(st, **extra):
    d = {"frames_per_s": st.frames_per_s, "p50_ms": st.p50_ms, "p99_ms": st.p99_ms,
         "frames": st.frames, "errors": st.errors, "mean_batch": st.mean_batch,
         "max_batch": st.max_batch, "wall_s": st.wall_s}
    d.update(extra)
    return d


def serving_comparison(args):
    """bf16 continuous batching against the plain per-frame loop (bf16 and
    fp32) on the SAME request trace, all requests of it, arrivals in real
    time.  Returns the dict the headline line carries under "serving"."""
    import torch
    from paper_2202_05977_amd import serve, synth, wskp
    cfg = synth.HD
    blob = synth.make_weights(cfg, 0)
    sizes, reqs, proto, inputs = serve_setup(args)
    budget = 64 << 30
    out = {"workload": f"64 streams, Poisson 2000 frames/s, {args.serve_frames} frames/stream "
                       f"({len(reqs)} requests), resolutions 360p/720p/1080p/1440p, "
                       "64 GB admission budget, inputs resident on the device",
           "mean_megapixels": float(np.mean([H * W for (H, W) in sizes])) / 1e6}
    dn = wskp.Denoiser(cfg, blob, "bf16")
    ex = serve.GpuExecutor(dn, inputs, budget, slots=args.inflight)
    _warm(serve, ex, sizes, proto)
    st = serve.Server(ex, budget, max_inflight=args.inflight, max_batch=args.max_batch).run(
        [dataclasses_replace(r) for r in reqs])
    out["bf16_continuous_batching"] = _stats(st, batches_in_flight=args.inflight)
    log(f"[serve] bf16 continuous batching: {st}")
    st = serve.Server(ex, budget, max_inflight=args.inflight, max_batch=args.max_batch).run(
        [dataclasses_replace(r) for r in reqs], realtime=False)
    out["bf16_capacity_frames_per_s"] = st.frames / st.wall_s
    log(f"[serve] bf16 capacity (whole trace queued): {st.frames / st.wall_s:.1f} frames/s, "
        f"mean batch {st.mean_batch:.1f}")
    st = serve.fifo_single(ex, [dataclasses_replace(r) for r in reqs])
    out["bf16_per_frame_loop"] = _stats(st)
    log(f"[serve] bf16 per-frame loop: {st}")
    del ex
    dn.close()
    dn = wskp.Denoiser(cfg, blob, "fp32")
    ex = serve.GpuExecutor(dn, inputs, 8 << 30)
    _warm(serve, ex, sizes, proto)
    st = serve.fifo_single(ex, [dataclasses_replace(r) for r in reqs])
    out["fp32_per_frame_loop"] = _stats(st)
    log(f"[serve] fp32 per-frame loop: {st}")
    del ex
    dn.close()
    torch.cuda.synchronize()
    return out


def mode_serve(args):
    """The C4 trace through the bf16 server in more forms than the headline
    line carries: direct launches, graph replay (two passes), capacity."""
    from paper_2202_05977_amd import serve, synth, wskp
    cfg = synth.HD
    blob = synth.make_weights(cfg, 0)
    sizes, reqs, proto, inputs = serve_setup(args)
    budget = 64 << 30
    res = {}
    dn = wskp.Denoiser(cfg, blob, "bf16")
    ex = serve.GpuExecutor(dn, inputs, budget, slots=args.inflight)
    _warm(serve, ex, sizes, proto)
    st = serve.Server(ex, budget, max_inflight=args.inflight, max_batch=args.max_batch).run(
        [dataclasses_replace(r) for r in reqs])
    res["bf16_continuous_batching"] = _stats(st)
    log(f"[serve] bf16 batching: {st}")
    # the same server, every batch a graph replay (one graph per stream and
    # capacity bucket, captured on first use).  The first pass over the trace
    # captures the buckets it meets (each capture stalls the loop); the
    # second pass is the steady state of a long-running server
    exg = serve.GpuExecutor(dn, inputs, budget, slots=args.inflight, graph=True)
    for k in range(2):
        st = serve.Server(exg, budget, max_inflight=args.inflight, max_batch=args.max_batch).run(
            [dataclasses_replace(r) for r in reqs])
        res["bf16_continuous_batching_graph" + ("_first_pass" if k == 0 else "")] = _stats(st)
        log(f"[serve] bf16 batching, graph replay, pass {k + 1}: {st}")
    del exg
    st = serve.Server(ex, budget, max_inflight=args.inflight, max_batch=args.max_batch).run(
        [dataclasses_replace(r) for r in reqs], realtime=False)
    res["bf16_capacity"] = _stats(st)
    log(f"[serve] bf16 batching capacity: {st.frames / st.wall_s:.1f} frames/s "
        f"(mean batch {st.mean_batch:.1f})")
    del ex
    dn.close()
    mean_px = float(np.mean([H * W for (H, W) in sizes]))
    print(json.dumps({"mode": "serve", "workload": "64 streams, Poisson 2000 frames/s, "
                      f"{args.serve_frames} frames/stream, resolutions 360p..1440p, 64 GB budget",
                      "mean_megapixels": mean_px / 1e6, "batches_in_flight": args.inflight,
                      "max_batch": args.max_batch, "results": res}), flush=True)


def mode_kernels(args):
    """Reconstruction time against the number of fused kernel sizes (the time
    halves of the paper's kernel-count figures, Sec. 6 and Sec. 7.1) and the
    explicit kernel-map comparison of Sec. 5.3, at 1280x720: for M = 1..6
    sizes k = 3, 5, ..., 2M+1 (and a single k = 9) with exp weights, the
    decode's time inside the bf16 frame path; then, for the paper's six
    sizes, the weight-sharing decode against a reconstruction that reads
    every pixel's explicit k x k kernels (same inputs, same result)."""
    import dataclasses
    import torch
    from paper_2202_05977_amd import synth, wskp
    H, W = args.height, args.width
    fr = {k: torch.from_numpy(v).cuda() for k, v in synth.make_frame(1, H, W).items()}
    out = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
    sets = [(9,)] + [tuple(range(3, 2 * m + 2, 2)) for m in range(1, 7)]
    sweep = []
    for ks in sets:
        cfg = dataclasses.replace(synth.HD, kernel_sizes=ks, weight_act="exp")
        dn = wskp.Denoiser(cfg, synth.make_weights(cfg, 0), "bf16")
        for _ in range(args.warmup):
            dn(fr, out)
        torch.cuda.synchronize()
        n = max(1, min(args.steps, 100))
        wskp.wskp_timing_enable(dn.h, n)
        for _ in range(n):
            dn(fr, out)
        ms, nc = wskp.wskp_timing_read(dn.h)
        wskp.wskp_timing_enable(dn.h, 0)
        dec = 1e3 * ms["decode"] / nc
        net = 1e3 * sum(v for k, v in ms.items() if k != "decode") / nc
        bytes_ = H * W * (8 * len(ks) + 36)
        sweep.append({"kernel_sizes": list(ks), "M": len(ks), "decode_us": dec, "net_us": net,
                      "decode_GBps": bytes_ / dec / 1e3})
        log(f"[kernels] k={ks}: decode {dec:.1f} us ({bytes_ / dec / 1e3:.0f} GB/s), net {net:.1f} us")
        dn.close()
    # explicit kernel maps vs weight sharing, the paper's six sizes
    ks = (3, 5, 7, 9, 11, 13)
    cfg = dataclasses.replace(synth.HD, kernel_sizes=ks)
    dn = wskp.Denoiser(cfg, synth.make_weights(cfg, 0), "fp32")
    M = len(ks)
    head = torch.from_numpy(synth.make_head(5, 1, H, W, M)).cuda()
    c = torch.rand(1, H, W, 3, generator=torch.Generator().manual_seed(6)).cuda()
    mod = torch.rand(1, H, W, 3, generator=torch.Generator().manual_seed(7)).cuda() + 0.1
    y_ws, y_kp = torch.empty_like(c), torch.empty_like(c)
    nb = wskp.wskp_kp_map_bytes(dn.h, H, W)
    maps = torch.empty(nb // 4, dtype=torch.float32, device="cuda")
    wskp.wskp_kp_expand(dn.h, head, maps)
    s = torch.cuda.current_stream()

    def timed(fn, rounds=5, calls=10):
        """us per call: `calls` calls queued back to back between two events
        (one call between events would also time its launch from the host),
        median over `rounds`."""
        ts = []
        fn()
        for _ in range(rounds):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            for _ in range(calls):
                fn()
            e1.record(s)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e3 / calls)
        return float(np.median(ts))

    t_ws = timed(lambda: wskp.wskp_decode(dn.h, head, c, mod, y_ws))
    t_kp = timed(lambda: wskp.wskp_kp_decode(dn.h, maps, head, c, mod, y_kp))
    torch.cuda.synchronize()
    diff = float((y_ws - y_kp).norm() / y_ws.norm())
    ws_in = H * W * (8 * M + 24)            # head 2M floats + c + mod
    kp_in = nb + H * W * (4 * M + 24)       # maps + logits + c + mod
    comp = {"kernel_sizes": list(ks), "weight_sharing_us": t_ws, "explicit_maps_us": t_kp,
            "speedup": t_kp / t_ws, "weight_sharing_input_bytes": ws_in,
            "explicit_input_bytes": kp_in, "memory_ratio": kp_in / ws_in,
            "rel_l2_between_forms": diff}
    log(f"[kernels] explicit maps {t_kp:.1f} us ({kp_in / 1e9:.2f} GB of input) vs weight sharing "
        f"{t_ws:.1f} us ({ws_in / 1e6:.1f} MB): {t_kp / t_ws:.1f}x; rel-L2 between them {diff:.1e}")
    dn.close()
    # temporal accumulation (Sec. 4.1) of a moving 720p frame against the
    # previous frame's state; algorithmic bytes: current radiance, normal,
    # world position (36 B), motion (8), the previous radiance, length,
    # normal, world position (40) read once, radiance and length (16) written
    seq = synth.make_sequence(3, H, W, 2)
    dv = [{k: torch.from_numpy(v).cuda() for k, v in f.items() if k != "clean"} for f in seq]
    acc = [torch.empty((H, W, 3), device="cuda") for _ in range(2)]
    lng = [torch.empty((H, W), device="cuda") for _ in range(2)]
    dn = wskp.Denoiser(synth.SMALL, synth.make_weights(synth.SMALL, 0), "fp32")
    wskp.wskp_temporal(dn.h, dv[0]["radiance"], dv[0]["normal"], dv[0]["wpos"], dv[0]["motion"], None,
                       acc[0], lng[0])
    prev = {"radiance": acc[0], "length": lng[0], "normal": dv[0]["normal"], "wpos": dv[0]["wpos"]}
    t_tmp = timed(lambda: wskp.wskp_temporal(dn.h, dv[1]["radiance"], dv[1]["normal"], dv[1]["wpos"],
                                             dv[1]["motion"], prev, acc[1], lng[1]))
    tb = H * W * 100
    temporal = {"workload": f"{W}x{H} moving frame, previous state resident", "us": t_tmp,
                "algorithmic_bytes": tb, "GBps": tb / t_tmp / 1e3, "frac_of_hbm_peak": tb / t_tmp / 1e3 / 8000.0,
                "history_kept": float((lng[1] > 1.0).float().mean())}
    log(f"[kernels] temporal accumulation {t_tmp:.1f} us ({tb / t_tmp / 1e3:.0f} GB/s), "
        f"history kept for {temporal['history_kept']:.2f} of the pixels")
    # multi-resolution reconstruction (Eq. 7): three levels, kernels {3, 5} at
    # each (the paper's high-spp network), heads and blend weights given
    ks2 = (3, 5)
    cfg2 = dataclasses.replace(synth.HD, kernel_sizes=ks2)
    dn2 = wskp.Denoiser(cfg2, synth.make_weights(cfg2, 0), "fp32")
    heads = [torch.from_numpy(synth.make_head(20 + l, 1, H >> l, W >> l, 2)).cuda() for l in range(3)]
    g = torch.Generator().manual_seed(8)
    alphas = [torch.rand(H >> l, W >> l, generator=g).cuda() for l in range(2)]
    c0 = c[0].contiguous()
    t_mr = timed(lambda: wskp.mr_reconstruct(dn2.h, heads, c0, alphas, mod[0].contiguous()))
    mr = {"workload": f"{W}x{H}, 3 levels, kernels (3, 5) per level", "us": t_mr,
          "launches": "2 pools + 3 decodes + 2 blends"}
    log(f"[kernels] multi-resolution reconstruction {t_mr:.1f} us")
    dn.close()
    dn2.close()
    print(json.dumps({"mode": "kernels", "workload": f"{W}x{H}, hd net, bf16 convs, exp weights",
                      "sweep": sweep, "explicit_kernel_maps": comp, "temporal": temporal,
                      "multiresolution": mr}), flush=True)


def mode_repvgg(args):
    """The U-Net with RepVGG blocks as encoders and decoders (every conv a
    merged 5x5 conv, Sec. 4.1) at 1280x720: frames/s and per-kernel times in
    bf16 and fp32 beside the 3x3 net, errors against the oracle's
    multi-branch network when the CPU leg runs."""
    import torch
    from paper_2202_05977_amd import synth, wskp
    H, W = args.height, args.width
    fr = synth.make_frame(1, H, W)
    dev = {k: torch.from_numpy(v).cuda() for k, v in fr.items()}
    cfg = synth.REPVGG
    br = synth.make_repvgg_branches(cfg, 0)
    blob = wskp.repvgg_blob(cfg, br)
    out = {}
    for p in args.precisions.split(","):
        r = time_precision(cfg, blob, dev, H, W, p, args.steps, args.warmup, min(args.steps, 100),
                           args.streams)
        flops = {k: v * 25.0 / 9.0 for k, v in conv_flops(cfg, H, W).items()}
        t = sum(v for k, v in r["per_kernel_us"].items() if k != "decode") * 1e-6
        out[p] = {"frames_per_s": r["fps"], "single_stream_frames_per_s": r["single_stream_fps"],
                  "p50_ms": r["p50_ms"], "p99_ms": r["p99_ms"], "per_kernel_us": r["per_kernel_us"],
                  "conv_tflops": sum(flops.values()) / t / 1e12,
                  "conv_frac_of_peak": sum(flops.values()) / t / PEAK[p]}
        log(f"[repvgg] {p}: {r['fps']:.1f} frames/s, per kernel (us): " +
            ", ".join(f"{k} {v:.1f}" for k, v in r["per_kernel_us"].items()))
        if not args.no_cpu_baseline:
            import oracle
            y = oracle.denoise(fr, None, cfg, branches=br)
            out[p]["rel_l2_vs_oracle"] = float(np.linalg.norm(r["y"] - y) / np.linalg.norm(y))
    print(json.dumps({"mode": "repvgg", "workload": f"{W}x{H} frame, 4-level U-Net 32/64/96/128 of "
                      "RepVGG blocks (merged 5x5 convs), M=5 kernels k=3..11", "results": out}),
          flush=True)


def dataclasses_replace(r):
    import dataclasses
    return dataclasses.replace(r)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_720p.json")
TRAFFIC_NOTE = ("not measured in this run: HBM bytes per launch from the committed rocprofv3 "
                "FETCH_SIZE/WRITE_SIZE counters in profiles/traffic_720p.json, scaled by a plain "
                "device copy; null when the kernel's source changed since they were taken")


def source_sha(rel: str) -> str:
    import hashlib
    with open(os.path.join(ROOT, rel), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(kernel: str, prec: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counters
    (FETCH_SIZE and WRITE_SIZE in KiB, scaled by the factors a plain device
    copy of known size gives), or None if there are none for this kernel or
    its source has changed since they were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    e = t.get("kernels", {}).get(f"{kernel}/{prec}")
    if not e or source_sha(e["source"]) != e["source_sha256"]:
        return None
    return (e["fetch_kib"] * t["fetch_factor"] + e["write_kib"] * t["write_factor"]) * 1024.0


def omp_threads() -> int:
    try:
        omp = ctypes.CDLL("libgomp.so.1")
        return int(omp.omp_get_max_threads())
    except OSError:
        return os.cpu_count() or 1


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_stages(oracle, fr, blob, cfg):
    """The oracle's per-frame path in two timed parts: (y, seconds of
    preprocess + U-Net + head activation, seconds of decode + fusion +
    remodulation, the decode's inputs).  The same composition as
    oracle.denoise."""
    t0 = time.perf_counter()
    X, c, mod = oracle.preprocess(fr["radiance"], fr["albedo"], fr["normal"], fr["depth"],
                                  cfg.gamma, cfg.depth_near, cfg.depth_far, cfg.eps_albedo)
    h = oracle.unet(X, blob, cfg.levels, cfg.channels, 2 * len(cfg.kernel_sizes))
    head = oracle.activate(h, len(cfg.kernel_sizes), cfg.weight_act)
    t1 = time.perf_counter()
    y = oracle.decode(head, c, mod, cfg.kernel_sizes, cfg.eps_norm)
    t2 = time.perf_counter()
    return y, t1 - t0, t2 - t1, (head, c, mod)


def cpu_baseline(fr, blob, cfg, H: int, W: int):
    """The FP64 oracle timed on the host: the whole frame on all OpenMP
    threads (the reported value), split into net and decode, plus a
    one-thread figure (the decode on the whole frame, the net on a crop of
    about 1/16 of its pixels, scaled by pixel count).  Returns (cpu_baseline
    object, oracle output)."""
    import oracle
    threads = omp_threads()
    log(f"[bench] FP64 oracle on the same {W}x{H} frame ({threads} threads)")
    yref, t_net, t_dec, dec_in = oracle_stages(oracle, fr, blob, cfg)
    dt = t_net + t_dec
    a = 2 ** (cfg.levels - 1)          # the net needs sides that are multiples of this
    ch = max(a, (H // 4) // a * a)
    cw = max(a, (W // 4) // a * a)
    crop = {k: np.ascontiguousarray(v[:ch, :cw]) for k, v in fr.items()}
    oracle.set_threads(1)
    try:
        _, t1_net, _, _ = oracle_stages(oracle, crop, blob, cfg)
        t1_dec = time.perf_counter()
        oracle.decode(*dec_in, cfg.kernel_sizes, cfg.eps_norm)
        t1_dec = time.perf_counter() - t1_dec
    finally:
        oracle.set_threads(threads)
    t1_net *= (H * W) / (ch * cw)
    log(f"[bench] oracle: net {t_net:.2f} s + decode {t_dec:.2f} s on {threads} threads; "
        f"one thread: net {t1_net:.1f} s (from a {cw}x{ch} crop), decode {t1_dec:.2f} s")
    cpu = {"value": 1.0 / dt, "unit": "frames/s", "cores": threads, "kind": "oracle",
           "sample": f"one full {W}x{H} frame of the same workload (FP64 U-Net + decode), {dt:.1f} s",
           "net_s": t_net, "decode_s": t_dec,
           "one_thread": {"net_s": t1_net, "decode_s": t1_dec,
                          "sample": f"net timed on a {cw}x{ch} crop of the frame and scaled by pixel "
                                    f"count; decode on the whole frame"},
           "cpu_model": cpu_model(), "cpus_visible": len(os.sched_getaffinity(0))}
    return cpu, yref


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precisions", default=None,
                    help="first one is the headline value (default bf16,fp32; sweep: fp32,bf16,fp8)")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle leg (no error or CPU figures)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="only run a plain device copy of MB megabytes 5 times (reference "
                         "kernel for scaling HBM traffic counters) and exit")
    ap.add_argument("--mode", default="headline",
                    choices=["headline", "sweep", "train", "serve", "kernels", "repvgg"],
                    help="headline: the 720p JSON line; sweep: 1080p precisions vs oracle; "
                         "train: decode adjoint on 8x256^2 crops; serve: 64-stream trace; "
                         "kernels: decode time vs number of kernel sizes, explicit kernel maps; "
                         "repvgg: the U-Net of merged RepVGG (5x5) blocks")
    ap.add_argument("--serve-frames", type=int, default=300,
                    help="serving trace: frames per stream (64 streams)")
    ap.add_argument("--no-serve", action="store_true",
                    help="headline: skip the serving comparison")
    ap.add_argument("--max-batch", type=int, default=64,
                    help="serve: most frames one batch may hold")
    ap.add_argument("--streams", type=int, default=3,
                    help="headline throughput: frames in flight on this many HIP streams")
    ap.add_argument("--inflight", type=int, default=3,
                    help="serve: batches in flight at once, one HIP stream each")
    ap.add_argument("--latency-frames", type=int, default=300,
                    help="single frames timed one at a time for p50/p99 (outside the timed "
                         "throughput region, independent of --steps)")
    ap.add_argument("--height", type=int, default=720)
    ap.add_argument("--width", type=int, default=1280)
    args = ap.parse_args()
    if args.precisions is None:
        args.precisions = "fp32,bf16,fp8" if args.mode == "sweep" else "bf16,fp32"
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

    if args.mode != "headline":
        {"sweep": mode_sweep, "train": mode_train, "serve": mode_serve,
         "kernels": mode_kernels, "repvgg": mode_repvgg}[args.mode](args)
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
                                args.latency_frames, args.streams)
        log(f"[bench] {p}: {res[p]['fps']:.1f} frames/s, {res[p]['ms_per_step']:.3f} ms/frame, "
            f"p50 {res[p]['p50_ms']:.3f} p99 {res[p]['p99_ms']:.3f} ms, "
            f"one stream {res[p]['single_stream_fps']:.1f} frames/s, "
            f"graph replay (one stream) {res[p]['graph_fps']:.1f} frames/s, "
            f"{args.streams}-stream outputs == one-stream: {res[p]['streams_equal_single']}")
        log(f"[bench] {p} per kernel (us): " +
            ", ".join(f"{k} {v:.1f}" for k, v in res[p]["per_kernel_us"].items()))

    head = precs[0]
    flops = conv_flops(cfg, H, W)
    pk = res[head]["per_kernel_us"]
    dom = max(pk, key=pk.get)
    if dom == "decode":
        achieved = decode_bytes(cfg, H, W) / (pk[dom] * 1e-6)
        roof = {"kernel": dom, "bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9,
                "unit": "GB/s", "frac": achieved / HBM_PEAK,
                "traffic": measured_traffic(dom, head), "traffic_source": TRAFFIC_NOTE}
    else:
        achieved = flops[dom] / (pk[dom] * 1e-6)
        roof = {"kernel": dom, "bound": "mfma", "achieved": achieved / 1e12,
                "peak": PEAK[head] / 1e12, "unit": "TFLOP/s", "frac": achieved / PEAK[head],
                "traffic": measured_traffic(dom, head), "traffic_source": TRAFFIC_NOTE}
    dbytes = decode_bytes(cfg, H, W)
    dec_gbs = dbytes / (pk["decode"] * 1e-6)
    dcw = decode_cold_warm(cfg, blob, H, W)
    log(f"[bench] decode alone (tensor form): warm {dcw['warm_us']:.1f} us = {dcw['warm_GBps']:.0f} GB/s, "
        f"cold {dcw['cold_us']:.1f} us = {dcw['cold_GBps']:.0f} GB/s")
    decode_roof = {"kernel": "decode", "bound": "hbm", "achieved": dec_gbs / 1e9,
                   "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": dec_gbs / HBM_PEAK,
                   "bytes_per_launch": dbytes, "traffic": measured_traffic("decode", head),
                   "traffic_source": TRAFFIC_NOTE}
    conv_mfma = {}
    for p in precs:
        tot = sum(flops.values())
        t = sum(v for k, v in res[p]["per_kernel_us"].items() if k != "decode") * 1e-6
        conv_mfma[p] = {"tflops": tot / t / 1e12, "frac_of_peak": tot / t / PEAK[p]}

    serving = None
    if not args.no_serve:
        serving = serving_comparison(args)

    cpu = None
    errors = {}
    if not args.no_cpu_baseline:
        cpu, yref = cpu_baseline(fr, blob, cfg, H, W)
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
                   "height": H, "width": W, "conv_precision": head,
                   "streams": args.streams},
        "single_stream": {"frames_per_s": res[head]["single_stream_fps"],
                          "ms_per_step": res[head]["single_stream_ms_per_step"]},
        "streams_bitwise_equal_single_stream": res[head]["streams_equal_single"],
        "latency_ms": {"p50": res[head]["p50_ms"], "p99": res[head]["p99_ms"],
                       "samples": args.latency_frames},
        "per_kernel_us": res[head]["per_kernel_us"],
        "roofline": roof,
        "decode_roofline": decode_roof,
        "decode_tensor_form": dcw,
        "clocks": gpu_clocks(),
        "conv_mfma": conv_mfma,
        "error_vs_fp64_oracle": errors,
        "precisions": {p: {"frames_per_s": res[p]["fps"], "ms_per_step": res[p]["ms_per_step"],
                           "graph_frames_per_s": res[p]["graph_fps"],
                           "single_stream_frames_per_s": res[p]["single_stream_fps"],
                           "p50_ms": res[p]["p50_ms"], "p99_ms": res[p]["p99_ms"],
                           "per_kernel_us": res[p]["per_kernel_us"]} for p in precs},
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
