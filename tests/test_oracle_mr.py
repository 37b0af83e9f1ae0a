"""Pins of the oracle's multi-resolution blend (Eq. 7, Sec. 5.2) and of the
multi-resolution reconstruction built on it: special cases of alpha, the
identity D U = 1 (with alpha = 1 the blend's 2x2 means are the coarse
image), a hand-worked 2x2 case, and the one-level reconstruction reducing
to the single-resolution decode."""
import numpy as np

import oracle
from paper_2202_05977_amd import synth


def _rand(shape, seed):
    return np.random.default_rng(seed).uniform(0.0, 2.0, size=shape)


def test_alpha_zero_keeps_the_fine_image():
    f, c = _rand((6, 8, 3), 1), _rand((3, 4, 3), 2)
    out = oracle.mr_blend(f, c, np.zeros((6, 8)))
    assert np.array_equal(out, f)


def test_alpha_one_makes_the_coarse_image_the_low_band():
    """With alpha = 1, o = f - U D f + U c, so D o = D f - D f + c = c
    (D U is the identity): the blend keeps the fine image's detail within
    each 2x2 block and takes its means from the coarse image."""
    f, c = _rand((6, 8, 3), 3), _rand((3, 4, 3), 4)
    out = oracle.mr_blend(f, c, np.ones((6, 8)))
    np.testing.assert_allclose(oracle.avgpool2(out), c, rtol=1e-14, atol=1e-14)
    # the detail within each block is the fine image's
    d_out = out - oracle.upsample2(oracle.avgpool2(out))
    d_f = f - oracle.upsample2(oracle.avgpool2(f))
    np.testing.assert_allclose(d_out, d_f, atol=1e-14)


def test_consistent_levels_are_unchanged():
    """If the coarse image already is D of the fine one, any alpha gives f."""
    f = _rand((4, 6, 3), 5)
    out = oracle.mr_blend(f, oracle.avgpool2(f), _rand((4, 6), 6) / 2.0)
    np.testing.assert_allclose(out, f, rtol=1e-14, atol=1e-14)


def test_hand_worked_block():
    """One 2x2 block, channel 0: f = [[1, 2], [3, 6]] (mean 3), c = 5,
    alpha = [[0, 0.5], [1, 0.25]]: o = f + alpha (5 - 3)."""
    f = np.zeros((2, 2, 3))
    f[..., 0] = [[1, 2], [3, 6]]
    c = np.zeros((1, 1, 3))
    c[0, 0, 0] = 5.0
    a = np.array([[0.0, 0.5], [1.0, 0.25]])
    out = oracle.mr_blend(f, c, a)
    np.testing.assert_allclose(out[..., 0], [[1, 3], [5, 6.5]], rtol=1e-15)
    np.testing.assert_allclose(out[..., 1:], 0.0)


def test_one_level_reconstruction_is_the_decode():
    ks = (3, 5)
    head = synth.make_head(7, 1, 10, 12, 2)[0]
    c = _rand((10, 12, 3), 8)
    mod = _rand((10, 12, 3), 9)
    y = oracle.mr_reconstruct([head], c, [], mod, ks)
    np.testing.assert_allclose(y, oracle.decode(head, c, mod, ks), rtol=1e-15)


def test_constant_irradiance_survives_every_level():
    """Constant c is preserved by each level's normalised filter, by the
    2x2 means and by the blend, for any weights and alphas."""
    ks = (3, 5)
    H, W = 16, 24
    heads = [synth.make_head(10 + l, 1, H >> l, W >> l, 2)[0] for l in range(3)]
    alphas = [_rand((H >> l, W >> l), 20 + l) / 2.0 for l in range(2)]
    c = np.broadcast_to(np.array([0.3, 1.5, 4.0]), (H, W, 3)).copy()
    y = oracle.mr_reconstruct(heads, c, alphas, None, ks)
    np.testing.assert_allclose(y, c, rtol=1e-13)
