"""Pins of the oracle's vector-Jacobian product of decode + fusion.

The paper gives no gradient formulas; it trains end to end through the
construction and fusion operators (Sec. 5.2-5.3).  The VJP is pinned by
central finite differences of <g, y(theta)> in float64, by torch float64
autograd through an independent box-filter composition, and by the
dot-product identity <J v, g> = <v, J^T g>.
"""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

import oracle
from paper_2202_05977_amd import synth

KS = (3, 5, 7, 9, 11)


def case(seed, H, W, M):
    rng = np.random.default_rng(seed)
    head = synth.make_head(seed, 1, H, W, M)[0].astype(np.float64)
    c = rng.gamma(0.5, 2.0, size=(H, W, 3))
    mod = rng.uniform(0.1, 1.0, size=(H, W, 3))
    g = rng.normal(size=(H, W, 3))
    return head, c, mod, g


def test_vjp_vs_central_differences_every_coordinate():
    """16x16 crop, five kernel sizes, every coordinate of the weights, the
    logits and c; step h = 1e-3 (FP64)."""
    H, W, M = 16, 16, len(KS)
    head, c, mod, g = case(0, H, W, M)
    dhead, dc = oracle.decode_vjp(head, c, mod, KS, g)
    f = lambda hd, cc: float(np.sum(g * oracle.decode(hd, cc, mod, KS)))
    h = 1e-3
    fd_head = np.empty_like(head)
    for idx in np.ndindex(head.shape):
        hp = head.copy(); hp[idx] += h
        hm = head.copy(); hm[idx] -= h
        fd_head[idx] = (f(hp, c) - f(hm, c)) / (2 * h)
    fd_c = np.empty_like(c)
    for idx in np.ndindex(c.shape):
        cp = c.copy(); cp[idx] += h
        cm = c.copy(); cm[idx] -= h
        fd_c[idx] = (f(head, cp) - f(head, cm)) / (2 * h)
    assert np.linalg.norm(dhead - fd_head) / np.linalg.norm(fd_head) < 1e-6
    assert np.linalg.norm(dc - fd_c) / np.linalg.norm(fd_c) < 1e-9   # linear in c
    # separately for the weight and the logit halves
    for sl in (slice(0, M), slice(M, 2 * M)):
        a, b = dhead[..., sl], fd_head[..., sl]
        assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-6


def torch_decode(head, c, mod, ks):
    M = len(ks)
    h = head.permute(2, 0, 1)[None]
    cc = c.permute(2, 0, 1)[None]
    alpha = torch.softmax(h[:, M:], dim=1)
    Fm = 0
    for i, k in enumerate(ks):
        w = h[:, i:i + 1]
        Fm = Fm + alpha[:, i:i + 1] * (F.avg_pool2d(w * cc, k, 1, k // 2, count_include_pad=False)
                                       / F.avg_pool2d(w, k, 1, k // 2, count_include_pad=False))
    return Fm[0].permute(1, 2, 0) * mod


@pytest.mark.parametrize("shape", [(32, 32), (20, 45)])
def test_vjp_vs_torch_autograd(shape):
    H, W = shape
    head, c, mod, g = case(1, H, W, len(KS))
    th = torch.from_numpy(head).requires_grad_(True)
    tc = torch.from_numpy(c).requires_grad_(True)
    y = torch_decode(th, tc, torch.from_numpy(mod), KS)
    (y * torch.from_numpy(g)).sum().backward()
    dhead, dc = oracle.decode_vjp(head, c, mod, KS, g)
    rel = lambda a, b: np.linalg.norm(a - b) / np.linalg.norm(b)
    assert rel(dhead, th.grad.numpy()) < 1e-12
    assert rel(dc, tc.grad.numpy()) < 1e-12


def test_dot_product_identity():
    """<J v, g> from a directional difference equals <v, J^T g>."""
    H, W = 24, 24
    head, c, mod, g = case(2, H, W, len(KS))
    rng = np.random.default_rng(5)
    vh = rng.normal(size=head.shape) * head * 0.1      # relative perturbation keeps W > 0
    vc = rng.normal(size=c.shape)
    dhead, dc = oracle.decode_vjp(head, c, mod, KS, g)
    lhs_adj = float(np.sum(vh * dhead) + np.sum(vc * dc))
    t = 1e-4
    yp = oracle.decode(head + t * vh, c + t * vc, mod, KS)
    ym = oracle.decode(head - t * vh, c - t * vc, mod, KS)
    jv_g = float(np.sum(g * (yp - ym) / (2 * t)))
    assert jv_g == pytest.approx(lhs_adj, rel=1e-7)


def test_l1_gradient_convention():
    y = np.array([1.0, 2.0, 3.0, 4.0])
    t = np.array([0.0, 2.0, 5.0, 4.5])
    v, gr = oracle.l1(y, t)
    assert v == pytest.approx((1 + 0 + 2 + 0.5) / 4)
    np.testing.assert_array_equal(gr, [0.25, 0.0, -0.25, -0.25])
