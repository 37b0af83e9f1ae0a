"""Pins of the oracle's training gradient (Eq. 1 with the SMAPE loss of
Eq. 6, trained with Adam as in Sec. 5.3): SMAPE and its derivative by hand
and by central differences, the conv backward by the adjoint identity, the
whole network gradient by central differences on every layer and by torch
float64 autograd through an independent U-Net composition, and Adam's
first step in closed form."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2202_05977_amd import synth

torch = pytest.importorskip("torch")


def test_smape_by_hand_and_its_gradient():
    y = np.array([1.0, -2.0, 0.5, 3.0])
    t = np.array([0.5, 1.0, 0.5, 0.0])
    eps = 0.01
    want = np.mean(np.abs(y - t) / (np.abs(y) + np.abs(t) + eps))
    v, g = oracle.smape(y, t, eps)
    assert abs(v - want) < 1e-15
    # central differences away from the kinks (y != t, y != 0)
    for i in (0, 1, 3):
        h = 1e-6
        yp, ym = y.copy(), y.copy()
        yp[i] += h
        ym[i] -= h
        fd = (oracle.smape(yp, t, eps)[0] - oracle.smape(ym, t, eps)[0]) / (2 * h)
        assert abs(fd - g[i]) < 1e-8 * max(1.0, abs(g[i]))
    assert g[2] == 0.0        # y == t: sign(0) = 0 and |y - t| = 0


def test_conv_backward_adjoint_identity():
    """<conv(x; w, 0), g> = <x, dx> = <w, dw> (the conv is bilinear)."""
    rng = np.random.default_rng(3)
    x = rng.normal(size=(7, 9, 5))
    w = rng.normal(size=(4, 5, 3, 3))
    g = rng.normal(size=(7, 9, 4))
    y = oracle.conv3x3(x, w, np.zeros(4), relu=False)
    dx, dw, db = oracle.conv3x3_backward(x, w, g)
    lhs = float(np.sum(y * g))
    assert abs(lhs - float(np.sum(x * dx))) < 1e-10 * abs(lhs)
    assert abs(lhs - float(np.sum(w * dw))) < 1e-10 * abs(lhs)
    np.testing.assert_allclose(db, g.sum(axis=(0, 1)), rtol=1e-13)


TINY = dataclasses.replace(synth.SMALL, channels=(4, 6, 8))


def _loss(blob32, fr, g):
    return oracle.train_grads(fr, fr["clean"], blob32, TINY, cotangent=g)[0]


def test_network_gradient_by_central_differences():
    """Linear loss sum(g * y) (smooth apart from ReLU kinks, which a 1e-6
    step does not cross here): the analytic gradient of a sample of weights
    and biases of every layer against central differences; the step is the
    exact difference of the float32-rounded perturbed weights."""
    fr = synth.make_frame(3, 8, 12)
    g = np.random.default_rng(5).normal(size=(8, 12, 3))
    blob = synth.make_weights(TINY, 1)
    _, grad = oracle.train_grads(fr, fr["clean"], blob, TINY, cotangent=g)
    rng = np.random.default_rng(6)
    # a few indices in every conv's weights and bias
    idx, off = [], 0
    for _, ci, co in synth.conv_shapes(TINY):
        nw = ci * co * 9
        idx += list(off + rng.choice(nw, 3, replace=False)) + [off + nw + int(rng.integers(co))]
        off += nw + co
    for i in idx:
        bp, bm = blob.copy(), blob.copy()
        bp[i] = np.float32(blob[i] + np.float32(1e-6) * max(1.0, abs(blob[i])))
        bm[i] = np.float32(blob[i] - np.float32(1e-6) * max(1.0, abs(blob[i])))
        fd = (_loss(bp, fr, g) - _loss(bm, fr, g)) / (float(bp[i]) - float(bm[i]))
        assert abs(fd - grad[i]) <= 1e-5 * max(abs(grad[i]), 1e-3 * np.abs(grad).max()), (i, fd, grad[i])


def _torch_unet_head_grad(X, blob, cfg, dh):
    """Gradient of sum(dh * h) with respect to every conv's (w, b), h the
    U-Net output, by torch float64 autograd through conv2d / avg_pool2d /
    interpolate / cat / relu."""
    import torch.nn.functional as F
    convs = [(torch.tensor(w, requires_grad=True), torch.tensor(b, requires_grad=True))
             for w, b in oracle._convs(blob, cfg)]
    L = cfg.levels
    x = torch.tensor(X).permute(2, 0, 1)[None]
    e = [F.relu(F.conv2d(x, *convs[0], padding=1))]
    for l in range(1, L):
        e.append(F.relu(F.conv2d(F.avg_pool2d(e[-1], 2), *convs[l], padding=1)))
    u = e[-1]
    for j, l in enumerate(range(L - 2, -1, -1)):
        cat = torch.cat([F.interpolate(u, scale_factor=2, mode="nearest"), e[l]], dim=1)
        u = F.relu(F.conv2d(cat, *convs[L + j], padding=1))
    h = F.conv2d(u, *convs[-1], padding=1)
    (h * torch.tensor(dh).permute(2, 0, 1)[None]).sum().backward()
    return np.concatenate([np.concatenate([w.grad.numpy().ravel(), b.grad.numpy()]) for w, b in convs])


def test_network_gradient_against_torch_autograd():
    """SMAPE loss on the small configuration: the oracle's gradient equals
    torch float64 autograd through an independent U-Net composition, given
    the gradient at the U-Net output that the oracle's decode adjoint and
    softplus derivative produce (both pinned elsewhere)."""
    cfg = synth.SMALL
    fr = synth.make_frame(4, 16, 24)
    blob = synth.make_weights(cfg, 2)
    _, grad = oracle.train_grads(fr, fr["clean"], blob, cfg)
    X, c, mod = oracle.preprocess(fr["radiance"], fr["albedo"], fr["normal"], fr["depth"])
    lay = oracle.unet_layers(X, blob, cfg)
    M = cfg.M
    head = oracle.activate(lay["h"], M)
    y = oracle.decode(head, c, mod, cfg.kernel_sizes)
    _, gy = oracle.smape(y, fr["clean"])
    dhead, _ = oracle.decode_vjp(head, c, mod, cfg.kernel_sizes, gy)
    dh = dhead.copy()
    dh[..., :M] *= 1.0 / (1.0 + np.exp(-lay["h"][..., :M]))
    ref = _torch_unet_head_grad(X, blob, cfg, dh)
    np.testing.assert_allclose(grad, ref, rtol=1e-9, atol=1e-12 * np.abs(ref).max())


def test_adam_first_step_closed_form():
    """Step 1: m^ = g, v^ = g^2, so w moves by -lr g / (|g| + eps)."""
    rng = np.random.default_rng(7)
    w0 = rng.normal(size=50)
    g = rng.normal(size=50)
    w, m, v = w0.copy(), np.zeros(50), np.zeros(50)
    oracle.adam(w, g, m, v, 1, lr=1e-3, eps=1e-8)
    np.testing.assert_allclose(w, w0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-13)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-14)
