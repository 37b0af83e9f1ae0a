"""GPU parity of the whole per-frame path (prediction network on MFMA +
fused decode) against the FP64 oracle, layer by layer and end to end."""
import numpy as np
import pytest

import oracle
from paper_2202_05977_amd import synth
from _helpers import rel_l2, max_rel, to_dev, TOL_FP32, TOL_BF16, TOL_BF16_MAX

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _denoiser(cfg, prec):
    from paper_2202_05977_amd import wskp
    return wskp.Denoiser(cfg, synth.make_weights(cfg, 0), prec)


def _run(dn, fr):
    out = dn(to_dev(fr))
    torch.cuda.synchronize()
    return out.cpu().numpy()


_ORACLE_CACHE = {}


def _oracle(cfg_name, seed, H, W):
    key = (cfg_name, seed, H, W)
    if key not in _ORACLE_CACHE:
        cfg = synth.CONFIGS[cfg_name]
        fr = synth.make_frame(seed, H, W)
        y, it = oracle.denoise(fr, synth.make_weights(cfg, 0), cfg, return_all=True)
        _ORACLE_CACHE[key] = (fr, y, it)
    return _ORACLE_CACHE[key]


@pytest.mark.parametrize("shape", [(128, 128), (72, 104)])
def test_small_fp32_layer_by_layer(shape):
    H, W = shape
    cfg = synth.SMALL
    fr, y, it = _oracle("small", 1, H, W)
    layers = oracle.unet_layers(it["X"], synth.make_weights(cfg, 0), cfg)
    dn = _denoiser(cfg, "fp32")
    out = _run(dn, fr)
    L = cfg.levels
    for l in range(L):
        g = dn.intermediate([H], [W], 0, l).float().cpu().numpy()
        assert rel_l2(g, layers[f"e{l}"]) <= TOL_FP32, f"e{l}"
    for l in range(L - 1):
        g = dn.intermediate([H], [W], 0, 100 + l).float().cpu().numpy()
        assert rel_l2(g, layers[f"u{l}"]) <= TOL_FP32, f"u{l}"
    head = dn.intermediate([H], [W], 0, 200).cpu().numpy()
    assert rel_l2(head, it["head"]) <= TOL_FP32
    assert rel_l2(out, y) <= TOL_FP32
    assert max_rel(out, y) <= TOL_FP32


def test_hd_fp32_720p_end_to_end():
    fr, y, _ = _oracle("hd", 1, 720, 1280)
    out = _run(_denoiser(synth.HD, "fp32"), fr)
    assert np.all(np.isfinite(out))
    assert rel_l2(out, y) <= TOL_FP32
    assert max_rel(out, y) <= TOL_FP32


def test_hd_bf16_720p_end_to_end():
    fr, y, _ = _oracle("hd", 1, 720, 1280)
    out = _run(_denoiser(synth.HD, "bf16"), fr)
    err = rel_l2(out, y)
    print(f"bf16 720p rel-L2 vs FP64 oracle: {err:.3e}, max-rel {max_rel(out, y):.3e}")
    assert err <= TOL_BF16
    assert max_rel(out, y) <= TOL_BF16_MAX


@pytest.mark.parametrize("shape", [(8, 16384), (16384, 8), (8, 8)])
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_extreme_frame_shapes(shape, prec):
    """The largest accepted width or height (16384) and the smallest frame the
    hd net accepts (8 x 8: its coarsest level is one pixel), end to end
    against the FP64 oracle."""
    H, W = shape
    fr, y, _ = _oracle("hd", 7, H, W)
    out = _run(_denoiser(synth.HD, prec), fr)
    assert np.all(np.isfinite(out))
    if prec == "fp32":
        assert rel_l2(out, y) <= TOL_FP32
        assert max_rel(out, y) <= TOL_FP32
    else:
        assert rel_l2(out, y) <= TOL_BF16
        assert max_rel(out, y) <= TOL_BF16_MAX


def test_hd_bf16_layers_and_pooled_copies():
    """bf16 HD net layer by layer against the FP64 oracle (bf16 tolerance),
    and the pooled copies p_l that the encoder epilogues pass on: each is
    exactly the 2x2 mean of the stored e_l (summed in fp32 in the order
    (2y,2x), (2y,2x+1), (2y+1,2x), (2y+1,2x+1), rounded to bf16)."""
    H, W = 64, 96
    cfg = synth.HD
    L = cfg.levels
    fr, y, it = _oracle("hd", 2, H, W)
    layers = oracle.unet_layers(it["X"], synth.make_weights(cfg, 0), cfg)
    dn = _denoiser(cfg, "bf16")
    out = _run(dn, fr)
    for l in range(L):
        g = dn.intermediate([H], [W], 0, l).float().cpu().numpy()
        assert rel_l2(g, layers[f"e{l}"]) <= TOL_BF16, f"e{l}"
    for l in range(L - 1):
        g = dn.intermediate([H], [W], 0, 100 + l).float().cpu().numpy()
        assert rel_l2(g, layers[f"u{l}"]) <= TOL_BF16, f"u{l}"
    assert rel_l2(out, y) <= TOL_BF16
    for l in range(L - 1):
        e = dn.intermediate([H], [W], 0, l).float()
        p = dn.intermediate([H], [W], 0, 300 + l)
        m = (((e[0::2, 0::2] + e[0::2, 1::2]) + e[1::2, 0::2]) + e[1::2, 1::2]) * 0.25
        assert torch.equal(p, m.to(torch.bfloat16)), f"p{l}"


def test_small_bf16_ragged():
    fr, y, _ = _oracle("small", 1, 72, 104)
    out = _run(_denoiser(synth.SMALL, "bf16"), fr)
    assert rel_l2(out, y) <= TOL_BF16
    assert max_rel(out, y) <= TOL_BF16_MAX


# five levels: from level 4 on the bf16 direct convs run on 4-row tiles with
# one output block per workgroup (112 x 176: 7 x 11 pixels at level 4)
FIVE_LEVEL = synth.NetConfig(levels=5, channels=(32, 32, 64, 64, 96), kernel_sizes=(3, 5, 7))


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_five_level_net_against_oracle(prec):
    fr = synth.make_frame(7, 112, 176)
    blob = synth.make_weights(FIVE_LEVEL, 0)
    y = oracle.denoise(fr, blob, FIVE_LEVEL)
    out = _run(_denoiser(FIVE_LEVEL, prec), fr)
    assert np.all(np.isfinite(out))
    if prec == "fp32":
        assert rel_l2(out, y) <= TOL_FP32 and max_rel(out, y) <= TOL_FP32
    else:
        assert rel_l2(out, y) <= TOL_BF16 and max_rel(out, y) <= TOL_BF16_MAX


@pytest.mark.parametrize("ks", [(3,), (1, 5), (3, 5, 7, 9), (3, 5, 7, 9, 11, 13, 15), (1, 3, 5, 7, 9, 11, 13, 15)])
def test_frames_decode_every_kernel_count_against_oracle(ks):
    """The decode inside the per-frame path is compiled once per number of
    kernel sizes M (its size loop unrolled, each weight map fetched two sizes
    ahead): M = 1, 2, 4, 7 and 8, with k = 1 and k = 15 among them, through
    the fp32 path on a frame of 2 x 3 decode tiles with ragged tails."""
    import dataclasses
    cfg = dataclasses.replace(synth.SMALL, kernel_sizes=ks)
    fr = synth.make_frame(60 + len(ks), 52, 84)
    blob = synth.make_weights(cfg, 0)
    y = oracle.denoise(fr, blob, cfg)
    out = _run(_denoiser(cfg, "fp32"), fr)
    assert np.all(np.isfinite(out))
    assert rel_l2(out, y) <= TOL_FP32 and max_rel(out, y) <= TOL_FP32


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_three_stream_pipeline_matches_single_stream(prec):
    """The launch configuration of the throughput figure: 720p frames dealt
    in turn to three streams, each stream with its own handle, workspace and
    outputs, so that kernels of different frames run concurrently.  Two
    different frames alternate; every result is bitwise the one-stream
    result of its frame."""
    frames = [to_dev(synth.make_frame(seed, 720, 1280)) for seed in (1, 2)]
    dns = [_denoiser(synth.HD, prec) for _ in range(3)]
    refs = [dns[0](f).clone() for f in frames]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in range(3)]
    for s_ in streams:
        s_.wait_stream(torch.cuda.current_stream())
    outs = []
    for k in range(9):
        o = torch.empty((720, 1280, 3), dtype=torch.float32, device="cuda")
        o.fill_(float("nan"))
        streams[k % 3].wait_stream(torch.cuda.current_stream())
        dns[k % 3](frames[k % 2], o, stream=streams[k % 3])
        outs.append(o)
    torch.cuda.synchronize()
    for k, o in enumerate(outs):
        assert torch.equal(o, refs[k % 2]), f"frame {k} on stream {k % 3} differs"
    assert not torch.equal(refs[0], refs[1])
    for d in dns:
        d.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_graph_replay_matches_eager(prec):
    """One frame's launches captured once in a HIP graph: every replay, with
    eager work (other frames through the same workspace, fills) and
    synchronisations between the replays, equals the eager result bitwise."""
    cfg = synth.HD
    dn = _denoiser(cfg, prec)
    H, W = 96, 160
    f = to_dev(synth.make_frame(3, H, W))
    eager = dn(f).clone()
    out = torch.full_like(eager, float("nan"))
    dn.workspace([H], [W])                      # no allocation inside the capture
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        dn(f, out, stream=s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        dn(f, out, stream=s)
    other = to_dev(synth.make_frame(4, H, W))
    for k in range(4):
        out.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), f"replay {k}"
        dn(other)
        torch.cuda.synchronize()


def _check_oracle(out, cfg, fr, prec, what):
    """One frame's result against the FP64 oracle, at the gates of its
    precision."""
    y = oracle.denoise(fr, synth.make_weights(cfg, 0), cfg)
    o = out.cpu().numpy() if hasattr(out, "cpu") else out
    assert np.all(np.isfinite(o)), what
    if prec == "fp32":
        assert rel_l2(o, y) <= TOL_FP32 and max_rel(o, y) <= TOL_FP32, what
    else:
        assert rel_l2(o, y) <= TOL_BF16 and max_rel(o, y) <= TOL_BF16_MAX, what


def test_batch_mixed_sizes_equals_single_frames():
    """Each frame alone == in a mixed-resolution batch == with tiles walked in
    reverse (bitwise), and every batched frame against the FP64 oracle."""
    from paper_2202_05977_amd import wskp
    cfg = synth.SMALL
    dn = _denoiser(cfg, "fp32")
    sizes = [(64, 64), (128, 96), (32, 160), (72, 104)]
    host = [synth.make_frame(10 + i, H, W) for i, (H, W) in enumerate(sizes)]
    frames = [to_dev(f) for f in host]
    singles = []
    for f in frames:
        singles.append(dn(f).clone())
    for flags in (0, wskp.BATCH_REVERSE_TILES):
        for f in frames:
            f["out"] = torch.full_like(f["radiance"], float("nan"))
        dn.batch(frames, flags=flags)
        torch.cuda.synchronize()
        for f, s in zip(frames, singles):
            assert torch.equal(f["out"], s)
    for i, f in enumerate(frames):
        _check_oracle(f["out"], cfg, host[i], "fp32", f"frame {i} {sizes[i]}")


def test_batch_hd_bf16_with_360p_frame_against_oracle():
    """A mixed bf16 batch of the hd net that holds a 640x360 frame (the
    smallest serving resolution) beside smaller ones: each batched frame
    equals the frame alone bitwise and meets the BF16 gates against the FP64
    oracle."""
    cfg = synth.HD
    dn = _denoiser(cfg, "bf16")
    sizes = [(360, 640), (64, 96), (128, 160), (8, 8)]
    host = [synth.make_frame(20 + i, H, W) for i, (H, W) in enumerate(sizes)]
    frames = [to_dev(f) for f in host]
    singles = [dn(f).clone() for f in frames]
    for f in frames:
        f["out"] = torch.full_like(f["radiance"], float("nan"))
    dn.batch(frames)
    torch.cuda.synchronize()
    for i, (f, s) in enumerate(zip(frames, singles)):
        assert torch.equal(f["out"], s), i
        _check_oracle(f["out"], cfg, host[i], "bf16", f"frame {i} {sizes[i]}")


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_batch_graph_replay_equals_single_frames(prec):
    """Batches run as graph replays: batches of different compositions that
    fall in the same capacity bucket replay one graph (the workgroups beyond
    each batch's tiles exit), on two streams, with eager work in between;
    every frame equals the frame denoised alone, bitwise."""
    from paper_2202_05977_amd import wskp
    cfg = synth.SMALL
    dn = _denoiser(cfg, prec)
    sizes = [(64, 64), (128, 96), (32, 160), (72, 104), (16, 16), (128, 160)]
    host = [synth.make_frame(40 + i, H, W) for i, (H, W) in enumerate(sizes)]
    frames = [to_dev(f) for f in host]
    singles = [dn(f).clone() for f in frames]
    batches = [[0, 1, 2, 3], [3, 2, 1, 0], [0, 1, 2], [5], [4, 5, 0], [0, 1, 2, 3], [4]]
    checked = set()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    wss = [torch.empty(wskp.wskp_workspace_size(dn.h, [H for H, _ in sizes], [W for _, W in sizes]),
                       dtype=torch.uint8, device="cuda") for _ in streams]
    for rep in range(2):
        for j, b in enumerate(batches):
            k = j % 2
            fb = [dict(frames[i]) for i in b]
            for f in fb:
                f["out"] = torch.full_like(f["radiance"], float("nan"))
            torch.cuda.synchronize()
            wskp.wskp_denoise_batch(dn.h, fb, wss[k], wskp.BATCH_GRAPH, streams[k])
            torch.cuda.synchronize()
            for i, f in zip(b, fb):
                assert torch.equal(f["out"], singles[i]), (rep, j, i)
                if i not in checked:
                    _check_oracle(f["out"], cfg, host[i], prec, f"replayed frame {i}")
                    checked.add(i)
            dn(frames[(j + 1) % len(frames)])          # eager work between replays


def test_batch_of_more_than_64_frames():
    """Frame lookup in batches that span several 64-frame groups: 130 small
    frames of five sizes, each equal to the frame denoised alone."""
    cfg = synth.SMALL
    dn = _denoiser(cfg, "bf16")
    sizes = [(4, 4), (8, 12), (16, 8), (12, 36), (28, 20)]
    protos = [to_dev(synth.make_frame(40 + i, H, W)) for i, (H, W) in enumerate(sizes)]
    singles = [dn(f).clone() for f in protos]
    order = [(7 * i + i // 11) % len(sizes) for i in range(130)]
    frames = []
    for j in order:
        f = {k: v for k, v in protos[j].items() if k != "clean"}
        f["out"] = torch.full_like(f["radiance"], float("nan"))
        frames.append(f)
    dn.batch(frames)
    torch.cuda.synchronize()
    for j, f in zip(order, frames):
        assert torch.equal(f["out"], singles[j]), j


def test_shape_errors():
    from paper_2202_05977_amd import wskp
    dn = _denoiser(synth.HD, "fp32")
    fr = to_dev(synth.make_frame(1, 36, 64))     # 36 is not a multiple of 8
    with pytest.raises(wskp.WskpError) as ei:
        dn(fr)
    assert ei.value.status == -2


@pytest.mark.parametrize("graph", [False, True])
def test_served_results_equal_single_frames(graph):
    """Frames pushed through the continuous-batching server (mixed sizes,
    two batches in flight, shared workspace arena; direct launches or graph
    replay).  Every request has its own input (a frame seed per request) and
    its own output slot; each served result equals that input denoised alone
    (bitwise) and meets the BF16 gates against the FP64 oracle."""
    from paper_2202_05977_amd import serve, wskp
    cfg = synth.SMALL
    dn = _denoiser(cfg, "bf16")
    res = [(64, 64), (128, 96), (32, 160), (72, 104)]
    nf = 6
    sizes, reqs = serve.poisson_trace(8, nf, 4000.0, res, seed=5)
    host = {s: [synth.make_frame(300 + 10 * s + k, *sizes[s]) for k in range(nf)]
            for s in range(8)}
    inputs = {s: [to_dev(f) for f in host[s]] for s in range(8)}
    budget = 4 * wskp.wskp_workspace_size(dn.h, [128] * 3, [160] * 3)
    ex = serve.GpuExecutor(dn, inputs, budget, slots=2, ring=nf, graph=graph)
    srv = serve.Server(ex, budget, max_inflight=2, max_batch=5)
    st = srv.run(reqs, realtime=False)
    torch.cuda.synchronize()
    assert st.errors == 0 and st.frames == len(reqs) and st.max_batch > 1
    assert srv.max_stream_inflight <= nf
    for r in reqs:
        alone = dn(inputs[r.stream][r.seq]).clone()
        torch.cuda.synchronize()
        got = ex.output_of(r.stream, r.seq)
        assert torch.equal(got, alone), (r.stream, r.seq)
        _check_oracle(got, cfg, host[r.stream][r.seq], "bf16", f"stream {r.stream} frame {r.seq}")


def test_hd_fp8_720p_reported_error():
    """FP8 (e4m3, per-channel weight scales, calibrated activation scales)
    convs: the error vs the FP64 oracle is reported; the gate only catches a
    wrong encoding or layout (those give errors of order 1)."""
    from paper_2202_05977_amd import wskp
    cfg = synth.HD
    blob = synth.make_weights(cfg, 0)
    scales = wskp.calibrate_fp8_scales(cfg, blob, to_dev(synth.make_frame(999, 720, 1280)))
    assert scales.shape == (len(synth.conv_shapes(cfg)),) and np.all(scales > 0)
    fr, y, _ = _oracle("hd", 1, 720, 1280)
    dn = wskp.Denoiser(cfg, blob, "fp8", act_scales=scales)
    out = _run(dn, fr)
    err = rel_l2(out, y)
    print(f"fp8 720p rel-L2 vs FP64 oracle: {err:.3e}, max-rel {max_rel(out, y):.3e}")
    assert np.all(np.isfinite(out))
    assert err <= 0.1


def test_hd_1080p_every_precision_against_oracle():
    """The 1920x1080 frame in each precision against one FP64 oracle run:
    fp32 to the FP32 gate (relative L2 and relative max norm), bf16 to the
    BF16 gate, fp8 reported with the encoding gate of the 720p test."""
    from paper_2202_05977_amd import wskp
    cfg = synth.HD
    blob = synth.make_weights(cfg, 0)
    fr, y, _ = _oracle("hd", 1, 1080, 1920)
    out = _run(wskp.Denoiser(cfg, blob, "fp32"), fr)
    assert rel_l2(out, y) <= TOL_FP32 and max_rel(out, y) <= TOL_FP32
    out = _run(wskp.Denoiser(cfg, blob, "bf16"), fr)
    assert rel_l2(out, y) <= TOL_BF16
    assert max_rel(out, y) <= TOL_BF16_MAX
    scales = wskp.calibrate_fp8_scales(cfg, blob, to_dev(synth.make_frame(999, 1080, 1920)))
    out = _run(wskp.Denoiser(cfg, blob, "fp8", act_scales=scales), fr)
    err = rel_l2(out, y)
    print(f"fp8 1080p rel-L2 vs FP64 oracle: {err:.3e}, max-rel {max_rel(out, y):.3e}")
    assert np.all(np.isfinite(out)) and err <= 0.1


def test_hd_1440p_bf16_against_oracle():
    """The largest resolution of the serving mix (2560x1440), in the serving
    precision, against the FP64 oracle."""
    fr, y, _ = _oracle("hd", 1, 1440, 2560)
    out = _run(_denoiser(synth.HD, "bf16"), fr)
    assert np.all(np.isfinite(out))
    assert rel_l2(out, y) <= TOL_BF16
    assert max_rel(out, y) <= TOL_BF16_MAX


def test_fp8_needs_scales_and_32_wide_levels():
    from paper_2202_05977_amd import wskp
    with pytest.raises(wskp.WskpError) as ei:
        wskp.Denoiser(synth.HD, synth.make_weights(synth.HD), "fp8")
    assert ei.value.status == -1
    with pytest.raises(wskp.WskpError) as ei:
        wskp.Denoiser(synth.SMALL, synth.make_weights(synth.SMALL), "fp8",
                      act_scales=np.ones(6, np.float32))
    assert ei.value.status == -3


@pytest.mark.parametrize("shift", [0.0, 120.0, -120.0])
def test_exp_weights_end_to_end_against_oracle(shift):
    """The literal Eq. 3 form (W = exp(h)) through the whole path in fp32.
    The head biases of the weight channels are moved by `shift`: at +120 a
    plain fp32 exp of h would overflow (e^120 > 3.4e38); the kernel takes
    exp(h - m) with a per-tile maximum m and scales the floor eps the same
    way, so the result is the oracle's FP64 exp(h) ratio, including at -120
    where every window sum falls below eps and the floor binds."""
    import dataclasses
    from paper_2202_05977_amd import wskp
    cfg = dataclasses.replace(synth.SMALL, weight_act="exp")
    blob = synth.make_weights(cfg, 0).copy()
    M = cfg.M
    blob[len(blob) - 2 * M:len(blob) - M] += np.float32(shift)
    H, W = 72, 104
    fr = synth.make_frame(5, H, W)
    y = oracle.denoise(fr, blob, cfg)
    dn = wskp.Denoiser(cfg, blob, "fp32")
    out = _run(dn, fr)
    assert np.all(np.isfinite(out))
    if shift < 0:
        # eps binds: out = mod * N / eps with N ~ e^-120: zero to within fp32
        assert np.abs(y).max() < 1e-30 and np.abs(out).max() < 1e-30
    else:
        assert rel_l2(out, y) <= TOL_FP32 and max_rel(out, y) <= TOL_FP32
    dn.close()


def test_exp_weights_hd_bf16_against_oracle():
    """exp weights with the hd net in bf16 at 1280x720 (BF16 gates)."""
    import dataclasses
    from paper_2202_05977_amd import wskp
    cfg = dataclasses.replace(synth.HD, weight_act="exp")
    blob = synth.make_weights(cfg, 0)
    fr = synth.make_frame(1, 720, 1280)
    y = oracle.denoise(fr, blob, cfg)
    out = _run(wskp.Denoiser(cfg, blob, "bf16"), fr)
    assert np.all(np.isfinite(out))
    assert rel_l2(out, y) <= TOL_BF16 and max_rel(out, y) <= TOL_BF16_MAX


def test_zero_albedo_epsilon_against_oracle():
    """eps_albedo = 0 with strictly positive albedo (the synthetic albedo
    lies in [0.1, 0.9]): c = r / a exactly; halo pixels outside the image
    must contribute nothing (not 0 * rcp(0))."""
    import dataclasses
    from paper_2202_05977_amd import wskp
    cfg = dataclasses.replace(synth.SMALL, eps_albedo=0.0)
    blob = synth.make_weights(cfg, 0)
    fr = synth.make_frame(6, 72, 104)
    assert fr["albedo"].min() > 0
    y = oracle.denoise(fr, blob, cfg)
    out = _run(wskp.Denoiser(cfg, blob, "fp32"), fr)
    assert np.all(np.isfinite(out))
    assert rel_l2(out, y) <= TOL_FP32 and max_rel(out, y) <= TOL_FP32


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_paper_kernel_set_720p_against_oracle(prec):
    """The paper's configuration of the reconstruction: six kernel sizes
    3, 5, ..., 13 with exp weights (the window softmax of Eq. 3) and six
    fusion logits, end to end at 1280x720 against the FP64 oracle."""
    from paper_2202_05977_amd import wskp
    cfg = synth.PAPER6
    blob = synth.make_weights(cfg, 0)
    fr, y, _ = _oracle("paper6", 1, 720, 1280)
    out = _run(wskp.Denoiser(cfg, blob, prec), fr)
    assert np.all(np.isfinite(out))
    err, mx = rel_l2(out, y), max_rel(out, y)
    print(f"paper kernel set 720p {prec}: rel-L2 {err:.3e}, max-rel {mx:.3e}")
    if prec == "fp32":
        assert err <= TOL_FP32 and mx <= TOL_FP32
    else:
        assert err <= TOL_BF16 and mx <= TOL_BF16_MAX
