"""GPU parity of temporal accumulation (Sec. 4.1, last paragraph) against
the FP64 oracle: the accumulation chain over a moving synthetic sequence,
and the accumulated frame through the whole denoiser."""
import numpy as np
import pytest

import oracle
from paper_2202_05977_amd import synth
from _helpers import rel_l2, max_rel, to_dev, TOL_FP32

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _gpu_chain(h, seq):
    """GPU accumulation over the sequence; returns [(radiance, length)] on the host."""
    from paper_2202_05977_amd import wskp
    outs, prev = [], None
    for f in seq:
        d = to_dev({k: f[k] for k in ("radiance", "normal", "wpos", "motion")})
        H, W = f["radiance"].shape[:2]
        r = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
        ln = torch.empty((H, W), dtype=torch.float32, device="cuda")
        wskp.wskp_temporal(h, d["radiance"], d["normal"], d["wpos"], d["motion"], prev, r, ln)
        prev = {"radiance": r, "length": ln, "normal": d["normal"], "wpos": d["wpos"]}
        outs.append((r, ln))
    torch.cuda.synchronize()
    return [(r.cpu().numpy(), ln.cpu().numpy()) for r, ln in outs]


def _oracle_chain(seq):
    outs, prev = [], None
    for f in seq:
        r, ln = oracle.temporal(f["radiance"], f["normal"], f["wpos"], f["motion"], prev)
        prev = {"radiance": r.astype(np.float32), "length": ln.astype(np.float32),
                "normal": f["normal"], "wpos": f["wpos"]}
        outs.append((r, ln))
    return outs


@pytest.mark.parametrize("shape,T", [((72, 128), 6), ((37, 53), 4), ((720, 1280), 3)])
def test_accumulation_chain_matches_oracle(shape, T):
    from paper_2202_05977_amd import wskp
    H, W = shape
    seq = synth.make_sequence(8, H, W, T)
    h = wskp.wskp_create(synth.SMALL, synth.make_weights(synth.SMALL), "fp32")
    got = _gpu_chain(h, seq)
    want = _oracle_chain(seq)
    for t, ((gr, gl), (wr, wl)) in enumerate(zip(got, want)):
        assert rel_l2(gr, wr) <= TOL_FP32 and max_rel(gr, wr) <= TOL_FP32, t
        # the accept/reject decisions are the same on both sides: history
        # lengths agree, and pixels reset to length 1 coincide exactly
        assert np.array_equal(gl == 1.0, wl == 1.0), t
        assert rel_l2(gl, wl) <= TOL_FP32, t
    # accumulation helps: the last frame is much closer to the clean image
    last = seq[-1]
    assert rel_l2(got[-1][0], last["clean"]) < 0.7 * rel_l2(last["radiance"], last["clean"])
    wskp.wskp_destroy(h)


def test_accumulated_frame_denoised_against_oracle():
    """Accumulate four frames, then denoise the last one (fp32, hd net):
    the composition against the oracle's accumulation and denoiser."""
    from paper_2202_05977_amd import wskp
    H, W = 96, 160
    seq = synth.make_sequence(9, H, W, 4)
    cfg = synth.HD
    blob = synth.make_weights(cfg, 0)
    dn = wskp.Denoiser(cfg, blob, "fp32")
    got = _gpu_chain(dn.h, seq)
    want = _oracle_chain(seq)
    last = dict(seq[-1])
    f_gpu = to_dev({k: last[k] for k in ("albedo", "normal", "depth")})
    f_gpu["radiance"] = torch.from_numpy(got[-1][0]).cuda()
    y = dn(f_gpu)
    torch.cuda.synchronize()
    ref_in = {k: last[k] for k in ("albedo", "normal", "depth")}
    ref_in["radiance"] = want[-1][0].astype(np.float32)
    ref = oracle.denoise(ref_in, blob, cfg)
    out = y.cpu().numpy()
    assert rel_l2(out, ref) <= TOL_FP32 and max_rel(out, ref) <= TOL_FP32
    dn.close()


def test_temporal_rejects_partial_history():
    from paper_2202_05977_amd import wskp
    h = wskp.wskp_create(synth.SMALL, synth.make_weights(synth.SMALL), "fp32")
    f = to_dev({k: v for k, v in synth.make_sequence(1, 16, 16, 1)[0].items()})
    r = torch.empty((16, 16, 3), device="cuda")
    ln = torch.empty((16, 16), device="cuda")
    with pytest.raises(wskp.WskpError) as ei:
        wskp.wskp_temporal(h, f["radiance"], f["normal"], f["wpos"], f["motion"],
                           {"radiance": r, "length": ln, "normal": f["normal"], "wpos": None},
                           torch.empty_like(r), torch.empty_like(ln))
    assert ei.value.status == -1
    wskp.wskp_destroy(h)


def test_served_streams_with_temporal_state():
    """Four streams of moving sequences through the continuous-batching
    server with per-stream accumulation state on the device: every frame's
    result equals the same stream accumulated and denoised frame by frame
    alone (bitwise), and the last frame of each stream meets the fp32 gates
    against the oracle's accumulation and denoiser."""
    from paper_2202_05977_amd import serve, wskp
    cfg = synth.SMALL
    blob = synth.make_weights(cfg, 0)
    dn = wskp.Denoiser(cfg, blob, "fp32")
    res = [(64, 96), (32, 64), (72, 104), (48, 48)]
    nf = 5
    sizes, reqs = serve.poisson_trace(4, nf, 4000.0, res, seed=11)
    seqs = {s: synth.make_sequence(50 + s, *sizes[s], nf) for s in range(4)}
    inputs = {s: [to_dev({k: v for k, v in f.items() if k != "clean"}) for f in seqs[s]]
              for s in range(4)}
    budget = 4 * wskp.wskp_workspace_size(dn.h, [72] * 2, [104] * 2)
    ex = serve.GpuExecutor(dn, inputs, budget, slots=2, ring=nf, temporal=True)
    srv = serve.Server(ex, budget, max_inflight=2, max_batch=4)
    st = srv.run(reqs, realtime=False)
    torch.cuda.synchronize()
    assert st.errors == 0 and st.frames == len(reqs)
    assert srv.max_stream_inflight == 1
    for s in range(4):
        H, W = sizes[s]
        prev = None
        for k in range(nf):
            f = inputs[s][k]
            acc = torch.empty((H, W, 3), device="cuda")
            ln = torch.empty((H, W), device="cuda")
            wskp.wskp_temporal(dn.h, f["radiance"], f["normal"], f["wpos"], f["motion"], prev, acc, ln)
            alone = dn({"radiance": acc, "albedo": f["albedo"], "normal": f["normal"],
                        "depth": f["depth"]}).clone()
            torch.cuda.synchronize()
            assert torch.equal(ex.output_of(s, k), alone), (s, k)
            prev = {"radiance": acc, "length": ln, "normal": f["normal"], "wpos": f["wpos"]}
        want = _oracle_chain(seqs[s])
        ref_in = {k: seqs[s][-1][k] for k in ("albedo", "normal", "depth")}
        ref_in["radiance"] = want[-1][0].astype(np.float32)
        ref = oracle.denoise(ref_in, blob, cfg)
        got = ex.output_of(s, nf - 1).cpu().numpy()
        assert rel_l2(got, ref) <= TOL_FP32 and max_rel(got, ref) <= TOL_FP32, s
    dn.close()
