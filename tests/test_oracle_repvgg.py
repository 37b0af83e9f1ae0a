"""Pins of the oracle's k x k convolution, its RepVGG block and the block's
merge into one 5x5 conv (Sec. 4.1, prediction phase), and of the U-Net with
5x5 convs: library routines (torch float64 conv2d, pooling, nearest
upsampling), closed forms (1x1 conv = per-pixel matrix product, the unit
centre tap = identity), the paper's statement that the merged conv computes
what the multi-branch block computes, and the reduction of a 5x5 net whose
outer kernel ring is zero to the 3x3 net."""
import numpy as np
import pytest

import oracle
from paper_2202_05977_amd import synth

torch = pytest.importorskip("torch")
F = torch.nn.functional


def _rand(shape, seed, lo=-1.0, hi=1.0):
    return np.random.default_rng(seed).uniform(lo, hi, size=shape)


def _torch_conv(x, w, b, relu=False):
    """torch float64 conv2d, padding (k-1)/2, NHWC in and out."""
    k = w.shape[-1]
    t = F.conv2d(torch.from_numpy(np.ascontiguousarray(x.transpose(2, 0, 1)))[None],
                 torch.from_numpy(w), torch.from_numpy(b), padding=(k - 1) // 2)[0]
    if relu:
        t = torch.relu(t)
    return t.numpy().transpose(1, 2, 0)


@pytest.mark.parametrize("k,shape", [(1, (4, 5, 3, 2)), (3, (6, 7, 2, 3)), (5, (7, 9, 3, 4)),
                                     (5, (3, 2, 2, 2)), (7, (8, 6, 2, 1))])
def test_conv2d_matches_torch_float64(k, shape):
    H, W, Ci, Co = shape
    x = _rand((H, W, Ci), 1)
    w = _rand((Co, Ci, k, k), 2)
    b = _rand((Co,), 3)
    for relu in (False, True):
        np.testing.assert_allclose(oracle.conv2d(x, w, b, relu), _torch_conv(x, w, b, relu),
                                   rtol=1e-13, atol=1e-13)


def test_conv1x1_is_a_per_pixel_matrix_product():
    x = _rand((5, 6, 4), 4)
    w = _rand((3, 4, 1, 1), 5)
    b = _rand((3,), 6)
    np.testing.assert_allclose(oracle.conv2d(x, w, b), x @ w[:, :, 0, 0].T + b, rtol=1e-14)


def test_unit_centre_tap_is_the_identity():
    x = _rand((6, 5, 3), 7)
    w = np.zeros((3, 3, 5, 5))
    for c in range(3):
        w[c, c, 2, 2] = 1.0
    np.testing.assert_array_equal(oracle.conv2d(x, w, np.zeros(3)), x)


def test_conv3x3_is_conv2d_with_k3():
    x = _rand((6, 7, 3), 8)
    w = _rand((4, 3, 3, 3), 9)
    b = _rand((4,), 10)
    np.testing.assert_array_equal(oracle.conv3x3(x, w, b, True), oracle.conv2d(x, w, b, True))


def _branches(ci, co, seed, identity):
    rng = np.random.default_rng(seed)
    br = {}
    for k in (1, 3, 5):
        br[f"w{k}"] = rng.normal(0, 0.3, size=(co, ci, k, k))
        br[f"b{k}"] = rng.uniform(-0.1, 0.1, size=(co,))
    br["identity"] = identity
    return br


@pytest.mark.parametrize("ci,co,identity", [(3, 3, True), (3, 5, False), (4, 4, False)])
def test_merged_conv_computes_the_multi_branch_block(ci, co, identity):
    """The inference-time 5x5 conv gives the training-time block's output
    everywhere, the image border included (each branch's own zero padding
    is the merged kernel's zero ring)."""
    br = _branches(ci, co, 11 + ci + co, identity)
    x = _rand((9, 11, ci), 12)
    w, b = oracle.repvgg_merge(br, ci, co)
    for relu in (False, True):
        np.testing.assert_allclose(oracle.conv2d(x, w, b, relu), oracle.repvgg_block(x, br, relu),
                                   rtol=1e-12, atol=1e-12)


def test_merge_places_each_branch_at_the_centre():
    br = {"w3": _rand((2, 2, 3, 3), 13), "b3": _rand((2,), 14)}
    w, b = oracle.repvgg_merge(br, 2, 2)
    np.testing.assert_array_equal(w[:, :, 1:4, 1:4], br["w3"])
    inner = np.zeros((5, 5), bool)
    inner[1:4, 1:4] = True
    assert np.all(w[:, :, ~inner] == 0.0)
    np.testing.assert_array_equal(b, br["b3"])
    # identity alone: the unit centre tap, so the block is ReLU(x)
    x = _rand((4, 4, 2), 15)
    np.testing.assert_array_equal(oracle.repvgg_block(x, {"identity": True}), np.maximum(x, 0.0))
    wi, bi = oracle.repvgg_merge({"identity": True}, 2, 2)
    np.testing.assert_array_equal(wi[:, :, 2, 2], np.eye(2))
    assert np.all(bi == 0.0)


def _torch_unet(X, convs, L):
    """The U-Net from torch float64 primitives (conv2d, avg_pool2d,
    nearest interpolate, cat), NCHW inside."""
    t = torch.from_numpy(np.ascontiguousarray(X.transpose(2, 0, 1)))[None]

    def conv(x, wb, relu):
        w, b = wb
        k = w.shape[-1]
        y = F.conv2d(x, torch.from_numpy(np.ascontiguousarray(w, dtype=np.float64)),
                     torch.from_numpy(np.ascontiguousarray(b, dtype=np.float64)), padding=(k - 1) // 2)
        return torch.relu(y) if relu else y

    e = [conv(t, convs[0], True)]
    for l in range(1, L):
        e.append(conv(F.avg_pool2d(e[-1], 2), convs[l], True))
    u = e[-1]
    for j, l in enumerate(range(L - 2, -1, -1)):
        u = conv(torch.cat([F.interpolate(u, scale_factor=2, mode="nearest"), e[l]], dim=1),
                 convs[L + j], True)
    return conv(u, convs[-1], False)[0].numpy().transpose(1, 2, 0)


def _split(blob, cfg):
    k = cfg.conv_size
    out, off = [], 0
    for _, ci, co in synth.conv_shapes(cfg):
        w = blob[off:off + co * ci * k * k].reshape(co, ci, k, k).astype(np.float64)
        off += co * ci * k * k
        out.append((w, blob[off:off + co].astype(np.float64)))
        off += co
    return out


def test_unet_with_5x5_convs_matches_torch_composition():
    cfg = synth.NetConfig(levels=3, channels=(16, 16, 32), kernel_sizes=(3, 5), conv_size=5)
    blob = synth.make_weights(cfg, 3)
    X = _rand((16, 12, 10), 16, 0.0, 1.0)
    h = oracle.unet(X, blob, cfg.levels, cfg.channels, cfg.out_channels, 5)
    np.testing.assert_allclose(h, _torch_unet(X, _split(blob, cfg), cfg.levels), rtol=1e-11, atol=1e-12)


def test_5x5_net_with_zero_outer_ring_is_the_3x3_net():
    c3 = synth.NetConfig(levels=3, channels=(16, 32, 32), kernel_sizes=(3, 5, 7))
    c5 = synth.NetConfig(levels=3, channels=(16, 32, 32), kernel_sizes=(3, 5, 7), conv_size=5)
    b3 = synth.make_weights(c3, 4)
    parts = []
    for w, b in _split(b3, c3):
        w5 = np.zeros(w.shape[:2] + (5, 5))
        w5[:, :, 1:4, 1:4] = w
        parts += [w5.astype(np.float32).ravel(), b.astype(np.float32)]
    b5 = np.concatenate(parts)
    assert b5.size == synth.num_weights(c5)
    X = _rand((8, 12, 10), 17, 0.0, 1.0)
    np.testing.assert_array_equal(oracle.unet(X, b5, 3, c5.channels, 6, 5),
                                  oracle.unet(X, b3, 3, c3.channels, 6, 3))


def test_repvgg_unet_equals_the_merged_net():
    """The training-time network (every conv a multi-branch block, identity
    where widths match) and the merged 5x5 network give the same h."""
    cfg = synth.NetConfig(levels=3, channels=(16, 16, 16), kernel_sizes=(3, 5), conv_size=5)
    br = synth.make_repvgg_branches(cfg, 5)
    assert sum(b["identity"] for b in br) == 2      # enc1 and enc2 map 16 -> 16
    parts = []
    for (_, ci, co), b in zip(synth.conv_shapes(cfg), br):
        w, bb = oracle.repvgg_merge(b, ci, co)
        parts += [w.ravel(), bb]
    merged = np.concatenate(parts)                  # float64: no rounding of the merge
    X = _rand((12, 8, 10), 18, 0.0, 1.0)
    # wo_unet reads float32 weights: compare in the merged net's own precision
    want = oracle.repvgg_unet(X, br, cfg)
    got = oracle.unet(X, merged.astype(np.float32), cfg.levels, cfg.channels, cfg.out_channels, 5)
    np.testing.assert_allclose(got, want, rtol=1e-5, atol=1e-6)
    # with the float64 merged weights the two agree up to rounding order
    convs = [oracle.repvgg_merge(b, ci, co) for (_, ci, co), b in zip(synth.conv_shapes(cfg), br)]
    L = cfg.levels
    e = [oracle.conv2d(X, *convs[0], relu=True)]
    for l in range(1, L):
        e.append(oracle.conv2d(oracle.avgpool2(e[-1]), *convs[l], relu=True))
    u = e[-1]
    for j, l in enumerate(range(L - 2, -1, -1)):
        u = oracle.conv2d(np.concatenate([oracle.upsample2(u), e[l]], axis=-1), *convs[L + j], relu=True)
    h = oracle.conv2d(u, *convs[-1])
    np.testing.assert_allclose(h, want, rtol=1e-11, atol=1e-12)
