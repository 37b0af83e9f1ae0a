"""Pins of the oracle's decode + fusion + remodulation (Eq. 3, Eq. 4, Eq. 5).

Each check comes from something other than the oracle itself: a
hand-worked example, an explicit kernel map built the way the original
kernel-prediction method stores it (Sec. 4.2, "Kernel Construction"), a
library box filter, or an invariant the paper states or the mathematics
forces.  The arrays are tiny, so these run in well under a second each.
"""
import json
import os

import numpy as np
import pytest
import torch
import torch.nn.functional as F

import oracle
from paper_2202_05977_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rand_case(seed, H, W, M, spread=1.0):
    rng = np.random.default_rng(seed)
    head = synth.make_head(seed, 1, H, W, M, spread)[0].astype(np.float64)
    c = rng.gamma(0.5, 2.0, size=(H, W, 3))
    mod = rng.uniform(0.1, 1.0, size=(H, W, 3))
    return head, c, mod


# ---------------------------------------------------------------- brute force
def brute_kernel_map(Wmap, k):
    """Explicit H x W x k^2 kernel map: unfold the weight map with a k x k
    window (outside-image taps get weight 0) and normalise each pixel's k^2
    weights to sum to one."""
    H, Wd = Wmap.shape
    r = k // 2
    pad = np.zeros((H + 2 * r, Wd + 2 * r))
    pad[r:r + H, r:r + Wd] = Wmap
    K = np.empty((H, Wd, k * k))
    for dy in range(k):
        for dx in range(k):
            K[:, :, dy * k + dx] = pad[dy:dy + H, dx:dx + Wd]
    K /= K.sum(axis=-1, keepdims=True)
    return K


def brute_apply(K, c, k):
    H, Wd, _ = c.shape
    r = k // 2
    pad = np.zeros((H + 2 * r, Wd + 2 * r, 3))
    pad[r:r + H, r:r + Wd] = c
    out = np.zeros((H, Wd, 3))
    for dy in range(k):
        for dx in range(k):
            out += K[:, :, dy * k + dx, None] * pad[dy:dy + H, dx:dx + Wd]
    return out


def brute_decode(head, c, mod, ks):
    M = len(ks)
    outs = [brute_apply(brute_kernel_map(head[..., i], k), c, k) for i, k in enumerate(ks)]
    lg = head[..., M:]
    a = np.exp(lg - lg.max(axis=-1, keepdims=True))
    a /= a.sum(axis=-1, keepdims=True)
    Fm = sum(a[..., i, None] * outs[i] for i in range(M))
    return mod * Fm


def torch_box_decode(head, c, mod, ks):
    """Ratio of two library box means (count_include_pad=False: truncated
    windows), then a library softmax over the logits."""
    M = len(ks)
    h = torch.from_numpy(head).permute(2, 0, 1)[None]        # [1, 2M, H, W]
    cc = torch.from_numpy(c).permute(2, 0, 1)[None]          # [1, 3, H, W]
    alpha = torch.softmax(h[:, M:], dim=1)
    Fm = torch.zeros_like(cc)
    for i, k in enumerate(ks):
        w = h[:, i:i + 1]
        num = F.avg_pool2d(w * cc, k, 1, k // 2, count_include_pad=False)
        den = F.avg_pool2d(w, k, 1, k // 2, count_include_pad=False)
        Fm = Fm + alpha[:, i:i + 1] * num / den
    return (Fm[0].permute(1, 2, 0).numpy()) * mod


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("ks", [(1,), (3,), (3, 5, 7), (3, 5, 7, 9, 11), (11, 13), (1, 3, 15)])
@pytest.mark.parametrize("shape", [(8, 8), (5, 13)])
def test_decode_vs_brute_force(ks, shape):
    """Explicit normalised kernel map (windows larger than the image included)."""
    H, W = shape
    head, c, mod = rand_case(7 + len(ks), H, W, len(ks))
    y = oracle.decode(head, c, mod, ks)
    yb = brute_decode(head, c, mod, ks)
    assert rel(y, yb) < 1e-13


@pytest.mark.parametrize("ks", [(3, 5, 7), (3, 5, 7, 9, 11)])
def test_decode_vs_library_box_filter(ks):
    head, c, mod = rand_case(3, 24, 20, len(ks), spread=2.0)
    y = oracle.decode(head, c, mod, ks)
    yt = torch_box_decode(head, c, mod, ks)
    assert rel(y, yt) < 1e-13


def test_exp_weights_are_the_window_softmax():
    """With W = exp(I) the normalised weight of Eq. 3 is a softmax of the
    importance values over the (truncated) window; build that softmax
    literally and apply it."""
    rng = np.random.default_rng(11)
    H, W, k = 7, 9, 5
    I = rng.normal(0.0, 1.5, size=(H, W))
    c = rng.uniform(0.0, 3.0, size=(H, W, 3))
    r = k // 2
    ref = np.zeros((H, W, 3))
    for py in range(H):
        for px in range(W):
            vals, cols = [], []
            for qy in range(py - r, py + r + 1):
                for qx in range(px - r, px + r + 1):
                    if 0 <= qy < H and 0 <= qx < W:
                        vals.append(I[qy, qx])
                        cols.append(c[qy, qx])
            sm = torch.softmax(torch.tensor(vals, dtype=torch.float64), 0).numpy()
            ref[py, px] = (sm[:, None] * np.array(cols)).sum(0)
    h = np.concatenate([I[..., None], np.zeros((H, W, 1))], axis=-1)
    head = oracle.activate(h, 1, "exp")
    y = oracle.decode(head, c, None, (k,))
    assert rel(y, ref) < 1e-13


def test_handworked_golden():
    g = json.load(open(os.path.join(GOLDEN, "decode_3x3_handworked.json")))
    W1 = np.array(g["W1"], dtype=np.float64)
    W3 = np.array(g["W3"], dtype=np.float64)
    c0 = np.array(g["c0"], dtype=np.float64)
    c = np.stack([c0, np.ones_like(c0), 2 * c0], axis=-1)
    lg = np.broadcast_to(np.array(g["logits"]), (3, 3, 2))
    head = np.concatenate([W1[..., None], W3[..., None], lg], axis=-1)
    mod = np.full((3, 3, 3), g["mod"])
    y, outs, alpha = oracle.decode(head, c, mod, g["kernel_sizes"], diagnostics=True)
    for key, v in g["expected_out3_c0"].items():
        py, px = map(int, key.split(","))
        assert outs[py, px, 1, 0] == pytest.approx(v, rel=1e-15)
    for key, v in g["expected_y"].items():
        py, px = map(int, key.split(","))
        np.testing.assert_allclose(y[py, px], v, rtol=1e-14)
    np.testing.assert_allclose(alpha, np.broadcast_to([0.25, 0.75], (3, 3, 2)), rtol=1e-14)


# ---------------------------------------------------------------- invariants
def test_k1_is_identity():
    """k = 1: each window holds only its centre, so out = c, and with
    mod = a + eps_a (the same factor that demodulated) y = r exactly."""
    rng = np.random.default_rng(0)
    H, W = 6, 10
    r = rng.gamma(0.5, 2.0, size=(H, W, 3)).astype(np.float32)
    a = rng.uniform(0.0, 0.9, size=(H, W, 3)).astype(np.float32)
    n = rng.normal(size=(H, W, 3)).astype(np.float32)
    d = rng.uniform(1, 10, size=(H, W, 1)).astype(np.float32)
    _, c, mod = oracle.preprocess(r, a, n, d)
    head = np.concatenate([rng.uniform(0.1, 5, size=(H, W, 1)), np.zeros((H, W, 1))], -1)
    y = oracle.decode(head, c, mod, (1,))
    np.testing.assert_allclose(y, r.astype(np.float64), rtol=1e-15, atol=0)


@pytest.mark.parametrize("k", [3, 5, 11])
def test_uniform_weights_give_box_filter(k):
    """W constant: the normalised kernel is a box with truncated windows."""
    rng = np.random.default_rng(k)
    H, W = 9, 14
    c = rng.uniform(0, 4, size=(H, W, 3))
    head = np.concatenate([np.full((H, W, 1), 0.37), np.zeros((H, W, 1))], -1)
    y = oracle.decode(head, c, None, (k,))
    r = k // 2
    ref = np.zeros_like(c)
    for py in range(H):
        for px in range(W):
            win = c[max(0, py - r):py + r + 1, max(0, px - r):px + r + 1]
            ref[py, px] = win.reshape(-1, 3).mean(0)
    assert rel(y, ref) < 1e-14
    lib = F.avg_pool2d(torch.from_numpy(c).permute(2, 0, 1)[None], k, 1, r,
                       count_include_pad=False)[0].permute(1, 2, 0).numpy()
    assert rel(y, lib) < 1e-14


def test_constant_image_is_preserved_everywhere():
    """Per-window normalisation conserves energy (Sec. 4.2): a constant c
    stays constant for any positive W, borders included."""
    head, _, _ = rand_case(5, 11, 7, 5, spread=3.0)
    c = np.broadcast_to(np.array([0.3, 1.7, 42.0]), (11, 7, 3)).copy()
    y = oracle.decode(head, c, None, (3, 5, 7, 9, 11))
    np.testing.assert_allclose(y, c, rtol=1e-14)


def test_scale_invariance_of_weights():
    """The importance is only relative within a window (Sec. 3): W -> lam W
    per kernel size leaves the output unchanged."""
    ks = (3, 5, 7)
    head, c, mod = rand_case(9, 12, 12, 3)
    y = oracle.decode(head, c, mod, ks)
    h2 = head.copy()
    h2[..., 0] *= 1e3
    h2[..., 1] *= 1e-4
    h2[..., 2] *= 7.0
    assert rel(oracle.decode(h2, c, mod, ks), y) < 1e-14


def test_exp_shift_invariance():
    """For W = exp(I), I -> I + const is the same as W -> e^const W."""
    rng = np.random.default_rng(4)
    h = rng.normal(size=(10, 10, 4))
    c = rng.uniform(size=(10, 10, 3))
    ks = (3, 5)
    y1 = oracle.decode(oracle.activate(h, 2, "exp"), c, None, ks)
    h2 = h.copy()
    h2[..., :2] += 3.25
    y2 = oracle.decode(oracle.activate(h2, 2, "exp"), c, None, ks)
    assert rel(y2, y1) < 1e-14


def test_linear_in_irradiance():
    ks = (3, 7)
    head, c1, mod = rand_case(12, 10, 9, 2)
    c2 = np.random.default_rng(1).normal(size=c1.shape)
    y = oracle.decode(head, 2.5 * c1 - 0.75 * c2, mod, ks)
    y12 = 2.5 * oracle.decode(head, c1, mod, ks) - 0.75 * oracle.decode(head, c2, mod, ks)
    assert rel(y, y12) < 1e-13


def test_convex_hull_of_window():
    """Each filtered value is a convex combination of c over its window."""
    head, c, _ = rand_case(13, 10, 10, 1, spread=2.0)
    _, outs, _ = oracle.decode(head, c, None, (5,), diagnostics=True)
    for py in range(10):
        for px in range(10):
            win = c[max(0, py - 2):py + 3, max(0, px - 2):px + 3].reshape(-1, 3)
            o = outs[py, px, 0]
            assert np.all(o >= win.min(0) - 1e-12) and np.all(o <= win.max(0) + 1e-12)


def test_fusion_special_cases():
    ks = (3, 5, 7)
    head, c, _ = rand_case(21, 9, 9, 3)
    _, outs, _ = oracle.decode(head, c, None, ks, diagnostics=True)
    # M = 1: fusion returns the single filtered image
    y1 = oracle.decode(np.concatenate([head[..., :1], head[..., 3:4]], -1), c, None, (3,))
    np.testing.assert_allclose(y1, outs[:, :, 0], rtol=1e-15)
    # equal logits: plain mean of the filtered images
    h = head.copy()
    h[..., 3:] = 0.8
    y = oracle.decode(h, c, None, ks)
    np.testing.assert_allclose(y, outs.mean(axis=2), rtol=1e-14)
    # a logit gap of 100 selects that kernel size (e^-100 ~ 4e-44)
    h[..., 3:] = 0.0
    h[..., 4] = 100.0
    y = oracle.decode(h, c, None, ks)
    np.testing.assert_allclose(y, outs[:, :, 1], rtol=1e-14)
    # fusion weights are a probability vector (0 <= alpha <= 1, sum 1; Eq. 5)
    _, _, alpha = oracle.decode(head, c, None, ks, diagnostics=True)
    assert np.all(alpha >= 0) and np.all(alpha <= 1)
    np.testing.assert_allclose(alpha.sum(-1), 1.0, rtol=1e-14)


def test_all_equal_filtered_images():
    """If every kernel size gives the same image, fusion returns it."""
    rng = np.random.default_rng(2)
    H, W = 8, 8
    c = rng.uniform(size=(H, W, 3))
    Wm = rng.uniform(0.5, 2.0, size=(H, W, 1))
    lg = rng.normal(size=(H, W, 3))
    head = np.concatenate([Wm, Wm, Wm, lg], -1)
    y = oracle.decode(head, c, None, (5, 5, 5))
    y1 = oracle.decode(np.concatenate([Wm, lg[..., :1]], -1), c, None, (5,))
    np.testing.assert_allclose(y, y1, rtol=1e-14)


def test_zero_weights_hit_the_floor():
    """All-zero weights: the eps floor makes every filtered value 0."""
    c = np.random.default_rng(3).uniform(size=(6, 6, 3))
    head = np.zeros((6, 6, 4))
    y = oracle.decode(head, c, None, (3, 5))
    assert np.all(y == 0.0)
