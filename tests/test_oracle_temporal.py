"""Pins of the oracle's temporal accumulation (Sec. 4.1, last paragraph)
against closed forms and special cases: first frame, static scene (the
exponential-average blend), integer and half-pixel motion (the sign and
index conventions, bilinear reprojection), rejected geometry, partial
rejection (renormalised taps) and motion out of the image."""
import numpy as np

import oracle


def _geom(H, W, seed=0):
    rng = np.random.default_rng(seed)
    n = rng.normal(size=(H, W, 3))
    n[..., 2] = np.abs(n[..., 2]) + 2.0
    n /= np.linalg.norm(n, axis=-1, keepdims=True)
    wp = rng.uniform(0, 1, size=(H, W, 3))
    return n.astype(np.float32), wp.astype(np.float32)


def _prev(r, ln, n, wp):
    return {"radiance": r.astype(np.float32), "length": ln.astype(np.float32),
            "normal": n, "wpos": wp}


def test_first_frame_is_the_input():
    H, W = 5, 7
    r = np.random.default_rng(1).gamma(0.5, 2.0, size=(H, W, 3)).astype(np.float32)
    n, wp = _geom(H, W)
    out, ln = oracle.temporal(r, n, wp, np.zeros((H, W, 2), np.float32), None)
    assert np.array_equal(out, r.astype(np.float64)) and np.all(ln == 1.0)


def test_static_scene_is_the_exponential_average():
    """Zero motion, same geometry: out = (1 - a) h + a r with
    a = max(1 / (L + 1), alpha_min) and the new length L + 1."""
    H, W = 4, 6
    rng = np.random.default_rng(2)
    r = rng.uniform(0, 2, size=(H, W, 3)).astype(np.float32)
    h = rng.uniform(0, 2, size=(H, W, 3)).astype(np.float32)
    n, wp = _geom(H, W)
    mv = np.zeros((H, W, 2), np.float32)
    amin = float(np.float32(0.2))      # the parameters are float32 values
    for L, a in ((1.0, 0.5), (3.0, 0.25), (9.0, amin), (50.0, amin)):
        out, ln = oracle.temporal(r, n, wp, mv, _prev(h, np.full((H, W), L), n, wp))
        np.testing.assert_allclose(out, (1 - a) * h.astype(np.float64) + a * r.astype(np.float64), rtol=1e-14)
        assert np.all(ln == L + 1)


def test_integer_motion_reads_the_offset_pixel():
    """mv = (+2, -1): the history of pixel (y, x) is the previous frame's
    pixel (y - 1, x + 2); pixels whose offset leaves the image keep r."""
    H, W = 6, 8
    rng = np.random.default_rng(3)
    r = rng.uniform(0, 1, size=(H, W, 3)).astype(np.float32)
    h = rng.uniform(0, 1, size=(H, W, 3)).astype(np.float32)
    n = np.zeros((H, W, 3), np.float32)
    n[..., 2] = 1.0
    wp = np.zeros((H, W, 3), np.float32)
    mv = np.zeros((H, W, 2), np.float32)
    mv[..., 0], mv[..., 1] = 2.0, -1.0
    out, ln = oracle.temporal(r, n, wp, mv, _prev(h, np.ones((H, W)), n, wp))
    for y in range(H):
        for x in range(W):
            if 0 <= x + 2 < W and 0 <= y - 1 < H:
                want = 0.5 * h[y - 1, x + 2].astype(np.float64) + 0.5 * r[y, x]
                assert ln[y, x] == 2.0
            else:
                want = r[y, x].astype(np.float64)
                assert ln[y, x] == 1.0
            np.testing.assert_allclose(out[y, x], want, rtol=1e-14, atol=0)


def test_half_pixel_motion_interpolates_bilinearly():
    """A history that is linear in x and y is reproduced exactly at
    fractional offsets (bilinear reprojection)."""
    H, W = 5, 9
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    h = np.stack([xx, 2 * yy, xx + yy], axis=-1).astype(np.float32)
    r = np.zeros((H, W, 3), np.float32)
    n = np.zeros((H, W, 3), np.float32)
    n[..., 2] = 1.0
    wp = np.zeros((H, W, 3), np.float32)
    mv = np.zeros((H, W, 2), np.float32)
    mv[..., 0], mv[..., 1] = 0.5, 0.25
    L = 9.0   # alpha = alpha_min = float32(0.2)
    a = float(np.float32(0.2))
    out, _ = oracle.temporal(r, n, wp, mv, _prev(h, np.full((H, W), L), n, wp))
    for y in range(H - 1):
        for x in range(W - 1):
            qx, qy = x + 0.5, y + 0.25
            np.testing.assert_allclose(out[y, x], (1 - a) * np.array([qx, 2 * qy, qx + qy]), rtol=1e-12)


def test_rejected_geometry_keeps_the_input():
    H, W = 4, 5
    rng = np.random.default_rng(4)
    r = rng.uniform(0, 1, size=(H, W, 3)).astype(np.float32)
    h = rng.uniform(0, 1, size=(H, W, 3)).astype(np.float32)
    n, wp = _geom(H, W)
    mv = np.zeros((H, W, 2), np.float32)
    # world positions moved by 0.03 > pos_tol = 0.02
    wp2 = (wp + np.float32(0.03) * np.array([1, 0, 0], np.float32)).astype(np.float32)
    out, ln = oracle.temporal(r, n, wp, mv, _prev(h, np.ones((H, W)), n, wp2))
    assert np.array_equal(out, r.astype(np.float64)) and np.all(ln == 1.0)
    # normals turned away (dot < 0.9)
    out, ln = oracle.temporal(r, n, wp, mv, _prev(h, np.ones((H, W)), -n, wp))
    assert np.array_equal(out, r.astype(np.float64)) and np.all(ln == 1.0)
    # a shift of 0.015 < pos_tol passes
    wp3 = (wp + np.float32(0.015) * np.array([1, 0, 0], np.float32)).astype(np.float32)
    out, ln = oracle.temporal(r, n, wp, mv, _prev(h, np.ones((H, W)), n, wp3))
    assert np.all(ln == 2.0)


def test_partial_rejection_renormalises_the_taps():
    """Half-pixel motion in x over two columns of which one is rejected:
    the history is the accepted tap's value alone, with its full weight."""
    H, W = 3, 4
    r = np.zeros((H, W, 3), np.float32)
    h = np.zeros((H, W, 3), np.float32)
    h[:, 1] = 10.0
    h[:, 2] = 20.0
    n = np.zeros((H, W, 3), np.float32)
    n[..., 2] = 1.0
    wp = np.zeros((H, W, 3), np.float32)
    wp_prev = wp.copy()
    wp_prev[:, 2, 0] = 1.0              # column 2 rejected
    mv = np.zeros((H, W, 2), np.float32)
    mv[..., 0] = 0.5
    out, ln = oracle.temporal(r, n, wp, mv, _prev(h, np.ones((H, W)), n, wp_prev))
    # pixel x = 1: taps x = 1 (10, accepted) and x = 2 (rejected), weight 1/2 each
    np.testing.assert_allclose(out[:, 1], 0.5 * 10.0, rtol=1e-14)
    assert np.all(ln[:, 1] == 2.0)
    # pixel x = 2: taps x = 2 (rejected) and x = 3 (0, accepted)
    np.testing.assert_allclose(out[:, 2], 0.0, atol=0)
