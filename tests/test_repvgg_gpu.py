"""GPU parity of the U-Net whose every conv is a RepVGG block run as its
merged 5x5 conv (Sec. 4.1, prediction phase) against the FP64 oracle's
training-time network (every block evaluated branch by branch: 1x1, 3x3,
5x5 convs and the identity, summed).  The library merges the branches
(wskp_repvgg_merge) and runs 5x5 implicit-GEMM convs; the oracle shares
neither step."""
import numpy as np
import pytest

import oracle
from paper_2202_05977_amd import synth
from _helpers import rel_l2, max_rel, to_dev, TOL_FP32, TOL_BF16, TOL_BF16_MAX

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# an equal-width net, so that the identity branch is present in enc1, enc2
EQUAL = synth.NetConfig(levels=3, channels=(32, 32, 32), kernel_sizes=(3, 5, 7), conv_size=5)


def _check(out, y, prec, what):
    o = out.cpu().numpy() if hasattr(out, "cpu") else out
    assert np.all(np.isfinite(o)), what
    e, m = rel_l2(o, y), max_rel(o, y)
    print(f"{what}: rel-L2 {e:.2e} max-rel {m:.2e}", flush=True)
    if prec == "fp32":
        assert e <= TOL_FP32 and m <= TOL_FP32, what
    else:
        assert e <= TOL_BF16 and m <= TOL_BF16_MAX, what


@pytest.mark.parametrize("cfg_name,prec,shape", [
    ("repvgg_small", "fp32", (64, 96)),
    ("repvgg_small", "fp32", (72, 104)),
    ("equal", "fp32", (36, 52)),
    ("repvgg_small", "bf16", (72, 104)),
    ("equal", "bf16", (64, 96)),
    ("repvgg", "bf16", (128, 192)),
    ("repvgg", "fp32", (48, 80)),
])
def test_repvgg_net_against_multi_branch_oracle(cfg_name, prec, shape):
    from paper_2202_05977_amd import wskp
    cfg = EQUAL if cfg_name == "equal" else synth.CONFIGS[cfg_name]
    H, W = shape
    br = synth.make_repvgg_branches(cfg, 3)
    dn = wskp.Denoiser(cfg, wskp.repvgg_blob(cfg, br), prec)
    fr = synth.make_frame(31, H, W)
    out = dn(to_dev(fr))
    torch.cuda.synchronize()
    y = oracle.denoise(fr, None, cfg, branches=br)
    _check(out, y, prec, f"{cfg_name} {prec} {shape}")
    dn.close()


def test_repvgg_720p_bf16_against_oracle():
    from paper_2202_05977_amd import wskp
    cfg = synth.REPVGG
    br = synth.make_repvgg_branches(cfg, 4)
    dn = wskp.Denoiser(cfg, wskp.repvgg_blob(cfg, br), "bf16")
    fr = synth.make_frame(32, 720, 1280)
    out = dn(to_dev(fr))
    torch.cuda.synchronize()
    y = oracle.denoise(fr, None, cfg, branches=br)
    _check(out, y, "bf16", "repvgg bf16 720p")
    dn.close()


def test_repvgg_mixed_batch_equals_single_frames_and_oracle():
    """A mixed-size batch of the 5x5 net: each frame equals the frame alone
    bitwise and meets the fp32 gates against the oracle."""
    from paper_2202_05977_amd import wskp
    cfg = synth.REPVGG_SMALL
    br = synth.make_repvgg_branches(cfg, 5)
    dn = wskp.Denoiser(cfg, wskp.repvgg_blob(cfg, br), "fp32")
    sizes = [(64, 64), (40, 56), (8, 12)]
    host = [synth.make_frame(40 + i, H, W) for i, (H, W) in enumerate(sizes)]
    frames = [to_dev(f) for f in host]
    singles = [dn(f).clone() for f in frames]
    for f in frames:
        f["out"] = torch.full_like(f["radiance"], float("nan"))
    dn.batch(frames, flags=wskp.BATCH_REVERSE_TILES)
    torch.cuda.synchronize()
    for i, (f, s) in enumerate(zip(frames, singles)):
        assert torch.equal(f["out"], s), i
        _check(f["out"], oracle.denoise(host[i], None, cfg, branches=br), "fp32", f"batch frame {i}")
    dn.close()


def test_training_rejects_5x5_nets():
    from paper_2202_05977_amd import wskp
    cfg = synth.REPVGG_SMALL
    h = wskp.wskp_create(cfg, synth.make_weights(cfg), "fp32")
    with pytest.raises(wskp.WskpError) as ei:
        wskp.wskp_train_workspace_size(h, [32], [32])
    assert ei.value.status == -3
    wskp.wskp_destroy(h)
