"""GPU training step (Eq. 1 with the SMAPE loss of Eq. 6, Adam as in
Sec. 5.3; fp32) against the FP64 oracle: loss and weight gradient of a batch
of crops, then one Adam step."""
import numpy as np
import pytest

import oracle
from paper_2202_05977_amd import synth
from _helpers import rel_l2, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# fp32 gradient vs FP64: each weight gradient is a sum over every pixel of
# the batch (10^4..10^5 terms of both signs, accumulated in fp32 per pixel
# chunk and across chunks) after a forward pass at ~1e-7 relative error;
# per conv the relative L2 error is gated at 1e-4.
TOL_GRAD = 1e-4


def _batch(cfg, sizes, seed0):
    host = [synth.make_frame(seed0 + i, H, W) for i, (H, W) in enumerate(sizes)]
    frames = []
    for f in host:
        d = to_dev({k: v for k, v in f.items() if k != "clean"})
        d["out"] = torch.empty_like(d["radiance"])
        frames.append(d)
    targets = [torch.from_numpy(f["clean"]).cuda() for f in host]
    return host, frames, targets


def _oracle_batch(host, blob, cfg):
    """Batch loss and gradient: SMAPE's mean runs over all values of the
    batch, so each frame's loss and gradient weigh by its pixel count."""
    P = [f["radiance"].shape[0] * f["radiance"].shape[1] for f in host]
    tot = float(sum(P))
    loss, grad = 0.0, 0.0
    for f, p in zip(host, P):
        l, g = oracle.train_grads(f, f["clean"], blob, cfg)
        loss += l * p / tot
        grad = grad + g * (p / tot)
    return loss, grad


# one- and two-level nets: the bottleneck's gradient is the head's input
# gradient (one level) or comes from the only decoder (two levels).  Frames
# of one size run the backward pass as one group (every kernel over all of
# them), frames of mixed sizes one at a time: both are covered.
ONE_LEVEL = synth.NetConfig(levels=1, channels=(16,), kernel_sizes=(3, 5))
TWO_LEVEL = synth.NetConfig(levels=2, channels=(16, 32), kernel_sizes=(3, 5, 7))


@pytest.mark.parametrize("cfg_name,sizes", [("small", [(64, 96), (64, 96)]),
                                            ("small", [(48, 80), (32, 32), (72, 104)]),
                                            ("hd", [(64, 64)]),
                                            ("hd", [(64, 64)] * 3),
                                            ("one_level", [(40, 56), (24, 32)]),
                                            ("one_level", [(40, 56)] * 2),
                                            ("two_level", [(48, 64), (36, 44)]),
                                            ("two_level", [(48, 64)] * 3),
                                            # 18 frames: the per-crop kernels take 16 frames'
                                            # buffers per launch, so two groups, one partial
                                            ("small", [(16, 24)] * 18),
                                            # 16 frames of 64x64: 256 chunk partials per
                                            # weight of the input layer, summed in two levels
                                            ("small", [(64, 64)] * 16)])
def test_train_grads_match_oracle(cfg_name, sizes):
    from paper_2202_05977_amd import wskp
    cfg = {"one_level": ONE_LEVEL, "two_level": TWO_LEVEL}.get(cfg_name) or synth.CONFIGS[cfg_name]
    blob = synth.make_weights(cfg, 3)
    host, frames, targets = _batch(cfg, sizes, 2000)
    dn = wskp.Denoiser(cfg, blob, "fp32")
    nw = blob.size
    grad = torch.empty(nw, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    ws = torch.empty(wskp.wskp_train_workspace_size(dn.h, [H for H, _ in sizes], [W for _, W in sizes]),
                     dtype=torch.uint8, device="cuda")
    wskp.wskp_train_grads(dn.h, frames, targets, grad, loss, ws)
    torch.cuda.synchronize()
    g = grad.cpu().numpy().astype(np.float64)
    l_ref, g_ref = _oracle_batch(host, blob, cfg)
    assert abs(float(loss.item()) - l_ref) <= 1e-5 * l_ref
    off = 0
    for name, ci, co in synth.conv_shapes(cfg):
        n = ci * co * 9 + co
        err = rel_l2(g[off:off + n], g_ref[off:off + n])
        print(f"{name}: gradient rel-L2 {err:.2e}")
        assert err <= TOL_GRAD, name
        off += n
    # the reconstruction the loss was taken on is the denoiser's
    for f, fh in zip(frames, host):
        ref = dn(f)
        torch.cuda.synchronize()
        assert torch.equal(ref, f["out"])
    # run-to-run identical
    grad2 = torch.empty_like(grad)
    wskp.wskp_train_grads(dn.h, frames, targets, grad2, loss, ws)
    torch.cuda.synchronize()
    assert torch.equal(grad, grad2)
    dn.close()


def test_adam_step_updates_the_denoiser():
    """Two training steps: the handle's weights after each Adam step against
    the oracle's Adam on the oracle's gradient (both steps from the same
    start), and the denoiser's output after the step is that of a fresh
    handle built from the updated blob (the kernels' weight layout was
    refreshed)."""
    from paper_2202_05977_amd import wskp
    cfg = synth.SMALL
    blob = synth.make_weights(cfg, 4)
    host, frames, targets = _batch(cfg, [(48, 64), (48, 64)], 2100)
    dn = wskp.Denoiser(cfg, blob, "fp32")
    nw = blob.size
    grad = torch.empty(nw, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    m = torch.zeros(nw, dtype=torch.float32, device="cuda")
    v = torch.zeros(nw, dtype=torch.float32, device="cuda")
    ws = torch.empty(wskp.wskp_train_workspace_size(dn.h, [48, 48], [64, 64]), dtype=torch.uint8,
                     device="cuda")
    w_ref = blob.astype(np.float64)
    m_ref, v_ref = np.zeros(nw), np.zeros(nw)
    for step in (1, 2):
        wskp.wskp_train_grads(dn.h, frames, targets, grad, loss, ws)
        wskp.wskp_adam(dn.h, grad, m, v, step, lr=1e-3)
        cur = torch.empty(nw, dtype=torch.float32, device="cuda")
        wskp.wskp_get_weights(dn.h, cur)
        torch.cuda.synchronize()
        _, g_ref = _oracle_batch(host, w_ref.astype(np.float32), cfg)
        oracle.adam(w_ref, g_ref, m_ref, v_ref, step, lr=1e-3)
        w_gpu = cur.cpu().numpy().astype(np.float64)
        # Adam moves each weight by about lr: compare the moves where the
        # gradient is well above the fp32 noise of the sum (elsewhere its
        # sign, and so the direction of the move, is not determined)
        dg, dr = w_gpu - blob, w_ref - blob
        off = 0
        for name, ci, co in synth.conv_shapes(cfg):
            n = ci * co * 9 + co
            gl = np.abs(g_ref[off:off + n])
            big = gl > 1e-3 * gl.max()
            assert big.mean() > 0.5, name
            assert rel_l2(dg[off:off + n][big], dr[off:off + n][big]) <= 1e-4, (step, name)
            off += n
        assert np.mean(np.sign(dg) != np.sign(dr)) <= 0.01, step
    fresh = wskp.Denoiser(cfg, cur.cpu().numpy(), "fp32")
    for f in frames:
        a = dn(f).clone()
        b = fresh(f)
        torch.cuda.synchronize()
        assert torch.equal(a, b)
    dn.close()
    fresh.close()


def test_training_rejects_other_precisions():
    from paper_2202_05977_amd import wskp
    dn = wskp.Denoiser(synth.SMALL, synth.make_weights(synth.SMALL), "bf16")
    with pytest.raises(wskp.WskpError) as ei:
        wskp.wskp_train_workspace_size(dn.h, [32], [32])
    assert ei.value.status == -3
    dn.close()
