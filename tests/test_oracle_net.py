"""Pins of the oracle's preprocessing (Sec. 5.1) and prediction network
(Sec. 4.1, Eq. 2).

The network pins compare against an independent composition of library
routines (torch CPU float64 conv2d / avg_pool2d / interpolate / cat), plus
closed forms that fix the conv orientation and the bias path.
"""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

import oracle
from paper_2202_05977_amd import synth


def test_preprocess_closed_forms():
    r = np.array([[[-1.0, 0.0, 0.25], [0.5, 1.0, 7.0]]], dtype=np.float32)       # [1,2,3]
    a = np.array([[[0.5, 0.25, 0.0], [0.9, 0.1, 0.3]]], dtype=np.float32)
    n = np.array([[[-1.0, 0.0, 1.0], [0.6, -0.8, 0.0]]], dtype=np.float32)
    d = np.array([[[0.5], [5.5]]], dtype=np.float32)
    X, c, mod = oracle.preprocess(r, a, n, d, gamma=2.2, near=1.0, far=10.0, eps_albedo=1e-3)
    # gamma tone map of the clamped radiance
    np.testing.assert_allclose(X[0, 0, :3], [0.0, 0.0, 0.25 ** (1 / 2.2)], rtol=1e-15)
    np.testing.assert_allclose(X[0, 1, :3], [0.5 ** (1 / 2.2), 1.0, 1.0], rtol=1e-15)
    np.testing.assert_array_equal(X[..., 3:6], a.astype(np.float64))
    np.testing.assert_allclose(X[0, 0, 6:9], [0.0, 0.5, 1.0], rtol=1e-15)
    # depth (d - 1) / 9, clamped
    assert X[0, 0, 9] == 0.0
    assert X[0, 1, 9] == pytest.approx(0.5, rel=1e-15)
    # demodulation uses a + eps, the same factor as the remodulation
    np.testing.assert_allclose(mod, a.astype(np.float64) + 1e-3, rtol=1e-15)
    np.testing.assert_allclose(c * mod, r.astype(np.float64), rtol=1e-15)


def test_conv_orientation_by_delta_image():
    """A unit impulse at (y0, x0) yields w[co][ci][ky][kx] + b at output
    (y0 - ky + 1, x0 - kx + 1): a cross-correlation, not a flipped conv."""
    rng = np.random.default_rng(0)
    H, W, Cin, Cout = 7, 8, 3, 4
    w = rng.normal(size=(Cout, Cin, 3, 3))
    b = rng.normal(size=Cout)
    x = np.zeros((H, W, Cin))
    y0, x0, ci = 3, 4, 1
    x[y0, x0, ci] = 1.0
    out = oracle.conv3x3(x, w, b, relu=False)
    for ky in range(3):
        for kx in range(3):
            np.testing.assert_allclose(out[y0 - ky + 1, x0 - kx + 1], w[:, ci, ky, kx] + b,
                                       rtol=1e-15)
    np.testing.assert_allclose(out[0, 0], b, rtol=1e-15)


def test_identity_tap_and_relu():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(5, 6, 4))
    w = np.zeros((4, 4, 3, 3))
    for c in range(4):
        w[c, c, 1, 1] = 1.0
    np.testing.assert_array_equal(oracle.conv3x3(x, w, np.zeros(4), relu=False), x)
    np.testing.assert_array_equal(oracle.conv3x3(x, w, np.zeros(4), relu=True), np.maximum(x, 0))


def test_pool_and_upsample_closed_forms():
    x = np.arange(16, dtype=np.float64).reshape(4, 4, 1)
    p = oracle.avgpool2(x)
    np.testing.assert_array_equal(p[..., 0], [[2.5, 4.5], [10.5, 12.5]])
    u = oracle.upsample2(p)
    np.testing.assert_array_equal(u[..., 0], [[2.5, 2.5, 4.5, 4.5], [2.5, 2.5, 4.5, 4.5],
                                              [10.5, 10.5, 12.5, 12.5], [10.5, 10.5, 12.5, 12.5]])


def torch_unet(X, blob, cfg):
    """Independent torch CPU float64 composition of the same U-Net."""
    t = torch.from_numpy(np.ascontiguousarray(X)).permute(2, 0, 1)[None]
    off = 0
    convs = []
    for _, ci, co in synth.conv_shapes(cfg):
        w = torch.from_numpy(blob[off:off + co * ci * 9].astype(np.float64)).reshape(co, ci, 3, 3)
        off += co * ci * 9
        b = torch.from_numpy(blob[off:off + co].astype(np.float64))
        off += co
        convs.append((w, b))
    L = cfg.levels
    e = [F.relu(F.conv2d(t, *convs[0], padding=1))]
    for l in range(1, L):
        e.append(F.relu(F.conv2d(F.avg_pool2d(e[-1], 2), *convs[l], padding=1)))
    u = e[L - 1]
    for j, l in enumerate(range(L - 2, -1, -1)):
        cat = torch.cat([F.interpolate(u, scale_factor=2, mode="nearest"), e[l]], dim=1)
        u = F.relu(F.conv2d(cat, *convs[L + j], padding=1))
    h = F.conv2d(u, *convs[-1], padding=1)
    return h[0].permute(1, 2, 0).numpy()


@pytest.mark.parametrize("name,H,W", [("small", 16, 16), ("small", 24, 40), ("hd", 16, 24)])
def test_unet_vs_torch_composition(name, H, W):
    cfg = synth.CONFIGS[name]
    blob = synth.make_weights(cfg, seed=0)
    fr = synth.make_frame(1, H, W)
    X, _, _ = oracle.preprocess(fr["radiance"], fr["albedo"], fr["normal"], fr["depth"])
    h = oracle.unet(X, blob, cfg.levels, cfg.channels, cfg.out_channels)
    ht = torch_unet(X, blob, cfg)
    assert np.linalg.norm(h - ht) / np.linalg.norm(ht) < 1e-13


def test_unet_rejects_misaligned_size():
    cfg = synth.CONFIGS["hd"]
    blob = synth.make_weights(cfg)
    with pytest.raises(ValueError):
        oracle.unet(np.zeros((12, 20, 10)), blob, cfg.levels, cfg.channels, cfg.out_channels)


def test_activations():
    h = np.linspace(-40, 40, 81 * 4).reshape(9, 9, 4)
    head = oracle.activate(h, 2, "softplus")
    # log(1 + e^x) by the library's logaddexp (torch's softplus switches to
    # the identity above x = 20, which is an approximation)
    ref = np.logaddexp(0.0, h[..., :2])
    np.testing.assert_allclose(head[..., :2], ref, rtol=1e-14)
    np.testing.assert_array_equal(head[..., 2:], h[..., 2:])
    assert np.all(head[..., :2] > 0)
    he = oracle.activate(h, 2, "exp")
    np.testing.assert_allclose(he[..., :2], np.exp(h[..., :2]), rtol=1e-15)


def test_full_path_small_frame_is_finite_and_bounded():
    """End to end on the small configuration: finite, and every pixel's
    filtered irradiance lies in the hull of c over the largest window."""
    cfg = synth.CONFIGS["small"]
    blob = synth.make_weights(cfg)
    fr = synth.make_frame(1, 32, 32)
    y, it = oracle.denoise(fr, blob, cfg, return_all=True)
    assert np.all(np.isfinite(y))
    Fm = y / it["mod"]
    c = it["c"]
    r = max(cfg.kernel_sizes) // 2
    for py in range(0, 32, 5):
        for px in range(0, 32, 5):
            win = c[max(0, py - r):py + r + 1, max(0, px - r):px + r + 1].reshape(-1, 3)
            assert np.all(Fm[py, px] >= win.min(0) - 1e-12)
            assert np.all(Fm[py, px] <= win.max(0) + 1e-12)
