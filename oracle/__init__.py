"""FP64 CPU oracle of the WSKP per-frame path (test infrastructure only).

Only the tests, the package's smoke check and the benchmark's CPU-baseline
leg may import this package.  The product library never loads it, and it
shares no code with the HIP path: the arithmetic lives in
``wskp_oracle.c`` (plain loops in double precision); this module only
marshals NumPy arrays into it.

Every step is pinned by the tests against something other than itself; the
end-to-end output of ``denoise`` is parity unpinned against the paper (it
prints no numeric example and no trained weights exist).

Functions take and return NumPy arrays in NHWC layout without a batch axis
unless stated.  Inputs may be float32; everything is widened to float64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wskp_oracle.c")
_LIB = os.path.join(_HERE, "libwskp_oracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_ip = ctypes.POINTER(ctypes.c_int)
_L = ctypes.c_long


def build(force: bool = True) -> str:
    """Compile the C oracle into ``libwskp_oracle.so`` next to its source."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", "-std=c99", _SRC,
               "-o", _LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        lib.wo_preprocess.argtypes = [_L, _L, _fp, _fp, _fp, _fp, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      _dp, _dp, _dp]
        lib.wo_conv3x3.argtypes = [_L, _L, _L, _L, _dp, _dp, _dp, ctypes.c_int, _dp]
        lib.wo_conv2d.argtypes = [_L, _L, _L, _L, ctypes.c_int, _dp, _dp, _dp, ctypes.c_int, _dp]
        lib.wo_avgpool2.argtypes = [_L, _L, _L, _dp, _dp]
        lib.wo_upsample2.argtypes = [_L, _L, _L, _dp, _dp]
        lib.wo_unet.argtypes = [_L, _L, ctypes.c_int, _ip, ctypes.c_int, ctypes.c_int,
                                ctypes.c_int, _fp, _dp, _dp]
        lib.wo_unet.restype = ctypes.c_int
        lib.wo_activate.argtypes = [_L, ctypes.c_int, ctypes.c_int, _dp, _dp]
        lib.wo_decode.argtypes = [_L, _L, ctypes.c_int, _ip, _dp, _dp, _dp, ctypes.c_double,
                                  _dp, _dp, _dp]
        lib.wo_decode_vjp.argtypes = [_L, _L, ctypes.c_int, _ip, _dp, _dp, _dp,
                                      ctypes.c_double, _dp, _dp, _dp]
        lib.wo_temporal.argtypes = [_L, _L, _fp, _fp, _fp, _fp, _fp, _fp, _fp, _fp,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp, _dp]
        lib.wo_mr_blend.argtypes = [_L, _L, _dp, _dp, _dp, _dp]
        lib.wo_smape.argtypes = [_L, _dp, _dp, ctypes.c_double, _dp]
        lib.wo_smape.restype = ctypes.c_double
        lib.wo_conv3x3_backward.argtypes = [_L, _L, _L, _L, _dp, _dp, _dp, _dp, _dp, _dp]
        lib.wo_avgpool2_backward.argtypes = [_L, _L, _L, _dp, _dp]
        lib.wo_upsample2_backward.argtypes = [_L, _L, _L, _dp, _dp]
        lib.wo_adam.argtypes = [_L, _dp, _dp, _dp, _dp, _L, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, ctypes.c_double]
        lib.wo_l1.argtypes = [_L, _dp, _dp, _dp]
        lib.wo_l1.restype = ctypes.c_double
        _lib = lib
    return _lib


def _d(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _f(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


def _ptr(a: np.ndarray, t=_dp):
    return a.ctypes.data_as(t)


def _ints(seq: Sequence[int]):
    arr = (ctypes.c_int * len(seq))(*[int(s) for s in seq])
    return arr


def set_threads(n: int) -> None:
    """Set the OpenMP thread count used by the C oracle."""
    lib = _load()
    try:
        omp = ctypes.CDLL("libgomp.so.1")
        omp.omp_set_num_threads(int(n))
    except OSError:  # pragma: no cover - libgomp always present with gcc
        os.environ["OMP_NUM_THREADS"] = str(n)
    del lib


def preprocess(radiance, albedo, normal, depth, gamma=2.2, near=1.0, far=10.0,
               eps_albedo=1e-3) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Network input X [H,W,10], irradiance c [H,W,3] and mod = a + eps [H,W,3]."""
    r, a, n, d = _f(radiance), _f(albedo), _f(normal), _f(depth)
    H, W = r.shape[:2]
    X = np.empty((H, W, 10))
    c = np.empty((H, W, 3))
    mod = np.empty((H, W, 3))
    _load().wo_preprocess(H, W, _ptr(r, _fp), _ptr(a, _fp), _ptr(n, _fp), _ptr(d, _fp),
                          gamma, near, far, eps_albedo, _ptr(X), _ptr(c), _ptr(mod))
    return X, c, mod


def conv3x3(x, w, b, relu: bool) -> np.ndarray:
    """3x3 cross-correlation, zero pad 1, + bias; x [H,W,Cin], w [Cout,Cin,3,3]."""
    x, w, b = _d(x), _d(w), _d(b)
    H, W, Cin = x.shape
    Cout = w.shape[0]
    assert w.shape == (Cout, Cin, 3, 3) and b.shape == (Cout,)
    out = np.empty((H, W, Cout))
    _load().wo_conv3x3(H, W, Cin, Cout, _ptr(x), _ptr(w), _ptr(b), int(relu), _ptr(out))
    return out


def conv2d(x, w, b, relu: bool = False) -> np.ndarray:
    """k x k cross-correlation (k odd, from w's shape), zero pad (k-1)/2, +
    bias; x [H,W,Cin], w [Cout,Cin,k,k]."""
    x, w, b = _d(x), _d(w), _d(b)
    H, W, Cin = x.shape
    Cout, k = w.shape[0], w.shape[-1]
    assert w.shape == (Cout, Cin, k, k) and k % 2 == 1 and b.shape == (Cout,)
    out = np.empty((H, W, Cout))
    _load().wo_conv2d(H, W, Cin, Cout, k, _ptr(x), _ptr(w), _ptr(b), int(relu), _ptr(out))
    return out


def avgpool2(x) -> np.ndarray:
    x = _d(x)
    H, W, C = x.shape
    out = np.empty((H // 2, W // 2, C))
    _load().wo_avgpool2(H, W, C, _ptr(x), _ptr(out))
    return out


def upsample2(x) -> np.ndarray:
    x = _d(x)
    H, W, C = x.shape
    out = np.empty((2 * H, 2 * W, C))
    _load().wo_upsample2(H, W, C, _ptr(x), _ptr(out))
    return out


def unet(X, blob, levels: int, channels: Sequence[int], out_channels: int,
         conv_size: int = 3) -> np.ndarray:
    """Raw network output h [H,W,out_channels] for input X [H,W,Cin]; every
    conv is conv_size x conv_size."""
    X = _d(X)
    blob = _f(blob)
    H, W, Cin = X.shape
    h = np.empty((H, W, out_channels))
    rc = _load().wo_unet(H, W, levels, _ints(channels), Cin, out_channels, int(conv_size),
                         _ptr(blob, _fp), _ptr(X), _ptr(h))
    if rc != 0:
        raise ValueError(f"wo_unet failed ({rc}): H, W must be multiples of 2^(L-1)")
    return h


def activate(h, M: int, act: str = "softplus") -> np.ndarray:
    """Head record: act(h[..., :M]) then raw logits h[..., M:2M]."""
    h = _d(h)
    head = np.empty_like(h)
    P = h.size // (2 * M)
    _load().wo_activate(P, M, 1 if act == "exp" else 0, _ptr(h), _ptr(head))
    return head


def decode(head, c, mod, kernel_sizes: Sequence[int], eps: float = 1e-10,
           diagnostics: bool = False):
    """Decode + fusion + remodulation of one frame: y [H,W,3].

    With ``diagnostics`` also returns the per-size filtered images
    [H,W,M,3] and the fusion weights [H,W,M].
    """
    head, c = _d(head), _d(c)
    H, W, twoM = head.shape
    M = twoM // 2
    assert M == len(kernel_sizes) and c.shape == (H, W, 3)
    modp = None
    if mod is not None:
        mod = _d(mod)
        modp = _ptr(mod)
    y = np.empty((H, W, 3))
    outs = np.empty((H, W, M, 3)) if diagnostics else None
    alpha = np.empty((H, W, M)) if diagnostics else None
    _load().wo_decode(H, W, M, _ints(kernel_sizes), _ptr(head), _ptr(c), modp, eps, _ptr(y),
                      _ptr(outs) if diagnostics else None, _ptr(alpha) if diagnostics else None)
    if diagnostics:
        return y, outs, alpha
    return y


def decode_vjp(head, c, mod, kernel_sizes: Sequence[int], g, eps: float = 1e-10):
    """(dL/dhead [H,W,2M], dL/dc [H,W,3]) for cotangent g = dL/dy [H,W,3]."""
    head, c, g = _d(head), _d(c), _d(g)
    H, W, twoM = head.shape
    M = twoM // 2
    modp = None
    if mod is not None:
        mod = _d(mod)
        modp = _ptr(mod)
    dhead = np.empty((H, W, twoM))
    dc = np.empty((H, W, 3))
    _load().wo_decode_vjp(H, W, M, _ints(kernel_sizes), _ptr(head), _ptr(c), modp, eps,
                          _ptr(g), _ptr(dhead), _ptr(dc))
    return dhead, dc


def temporal(radiance, normal, wpos, motion, prev=None, alpha_min: float = 0.2,
             pos_tol: float = 0.02, normal_tol: float = 0.9):
    """Temporal accumulation of one frame: (radiance [H,W,3], length [H,W]).

    ``prev`` is None (first frame) or a dict with the previous frame's
    accumulated ``radiance`` [H,W,3] and ``length`` [H,W] (float32, as the
    GPU path stores them) and its ``normal`` and ``wpos`` [H,W,3].
    ``motion`` [H,W,2]: offset (x, y) in pixels from a pixel to its surface
    point's position in the previous frame.  The three parameters are
    float32 values (as the library's interface takes them), widened.
    """
    alpha_min, pos_tol, normal_tol = (float(np.float32(v)) for v in (alpha_min, pos_tol, normal_tol))
    r, n, wp, mv = _f(radiance), _f(normal), _f(wpos), _f(motion)
    H, W = r.shape[:2]
    out = np.empty((H, W, 3))
    ln = np.empty((H, W))
    if prev is None:
        pr = pl = pn = pw = None
    else:
        pr, pl = _f(prev["radiance"]), _f(prev["length"])
        pn, pw = _f(prev["normal"]), _f(prev["wpos"])
    fp = lambda a: None if a is None else _ptr(a, _fp)
    _load().wo_temporal(H, W, _ptr(r, _fp), _ptr(n, _fp), _ptr(wp, _fp), _ptr(mv, _fp), fp(pr), fp(pl),
                        fp(pn), fp(pw), alpha_min, pos_tol, normal_tol, _ptr(out), _ptr(ln))
    return out, ln


def mr_blend(fine, coarse, alpha) -> np.ndarray:
    """Eq. 7: o = fine - alpha * U(D(fine)) + alpha * U(coarse); fine
    [H,W,3], coarse [H/2,W/2,3], alpha [H,W] (H, W even)."""
    fine, coarse, alpha = _d(fine), _d(coarse), _d(alpha)
    H, W = fine.shape[:2]
    assert H % 2 == 0 and W % 2 == 0 and coarse.shape == (H // 2, W // 2, 3)
    assert alpha.shape == (H, W)
    out = np.empty((H, W, 3))
    _load().wo_mr_blend(H, W, _ptr(fine), _ptr(coarse), _ptr(alpha), _ptr(out))
    return out


def mr_reconstruct(heads, c, alphas, mod, kernel_sizes: Sequence[int], eps: float = 1e-10):
    """Multi-resolution reconstruction (Sec. 5.2): level l filters the
    irradiance pooled l times, c_l = D^l c, with its own head record
    heads[l] [H>>l, W>>l, 2M] (the weight-sharing decode of Eq. 3-5 without
    remodulation), and the levels are blended from the coarsest with
    Eq. 7 using alphas[l] [H>>l, W>>l] for l < L-1; the result is
    remodulated with mod [H,W,3] (None = 1)."""
    L = len(heads)
    cs = [_d(c)]
    for _ in range(1, L):
        cs.append(avgpool2(cs[-1]))
    i = [decode(heads[l], cs[l], None, kernel_sizes, eps) for l in range(L)]
    o = i[L - 1]
    for l in range(L - 2, -1, -1):
        o = mr_blend(i[l], o, alphas[l])
    return o if mod is None else o * _d(mod)


def l1(y, t):
    """(mean |y - t|, gradient sign(y - t) / n)."""
    y, t = _d(y), _d(t)
    g = np.empty_like(y)
    v = _load().wo_l1(y.size, _ptr(y), _ptr(t), _ptr(g))
    return v, g


def denoise(frame: Dict[str, np.ndarray], blob, cfg, return_all: bool = False,
            branches=None):
    """Whole per-frame path for one frame: y [H,W,3] in float64.

    ``cfg`` carries levels, channels, kernel_sizes, eps_norm, eps_albedo,
    gamma, depth_near, depth_far, weight_act and conv_size (3 if absent).
    With ``branches`` (and ``blob`` None) the network is the training-time
    RepVGG form: every conv is the multi-branch block of ``repvgg_block``.
    With ``return_all`` the intermediates (X, c, mod, h, head) come back in a
    dict as well.
    """
    X, c, mod = preprocess(frame["radiance"], frame["albedo"], frame["normal"], frame["depth"],
                           cfg.gamma, cfg.depth_near, cfg.depth_far, cfg.eps_albedo)
    if branches is not None:
        h = repvgg_unet(X, branches, cfg)
    else:
        h = unet(X, blob, cfg.levels, cfg.channels, 2 * len(cfg.kernel_sizes),
                 getattr(cfg, "conv_size", 3))
    head = activate(h, len(cfg.kernel_sizes), cfg.weight_act)
    y = decode(head, c, mod, cfg.kernel_sizes, cfg.eps_norm)
    if return_all:
        return y, {"X": X, "c": c, "mod": mod, "h": h, "head": head}
    return y


def unet_layers(X, blob, cfg) -> Dict[str, np.ndarray]:
    """Every intermediate map of the U-Net: e0..e_{L-1}, u_{L-2}..u0, h.

    The same steps as ``unet`` composed from the single-op routines, for
    layer-by-layer comparisons.
    """
    blob = _f(blob)
    L, ch = cfg.levels, cfg.channels
    convs = []
    off = 0
    cin = [X.shape[-1]] + [ch[l - 1] for l in range(1, L)] + \
          [ch[l + 1] + ch[l] for l in range(L - 2, -1, -1)] + [ch[0]]
    cout = [ch[l] for l in range(L)] + [ch[l] for l in range(L - 2, -1, -1)] + \
           [2 * len(cfg.kernel_sizes)]
    k = getattr(cfg, "conv_size", 3)
    for ci, co in zip(cin, cout):
        w = blob[off:off + co * ci * k * k].reshape(co, ci, k, k)
        off += co * ci * k * k
        b = blob[off:off + co]
        off += co
        convs.append((w, b))
    out = {}
    e = conv2d(X, *convs[0], relu=True)
    out["e0"] = e
    for l in range(1, L):
        e = conv2d(avgpool2(e), *convs[l], relu=True)
        out[f"e{l}"] = e
    u = out[f"e{L - 1}"]
    for j, l in enumerate(range(L - 2, -1, -1)):
        cat = np.concatenate([upsample2(u), out[f"e{l}"]], axis=-1)
        u = conv2d(cat, *convs[L + j], relu=True)
        out[f"u{l}"] = u
    out["h"] = conv2d(u, *convs[-1], relu=False)
    return out


# ---------------------------------------------------------------- RepVGG
# A RepVGG block (Sec. 4.1, prediction phase) is, while training, the sum of
# a 1x1, a 3x3 and a 5x5 conv branch (each with its bias) and, when it maps
# C channels to C channels, the identity, followed by ReLU; for inference
# the branches are merged into one 5x5 conv that computes the same map.
# A block's parameters are a dict with "w1" [Co,Ci,1,1], "b1", "w3"
# [Co,Ci,3,3], "b3", "w5" [Co,Ci,5,5], "b5" (a missing pair is an absent
# branch) and "identity" (bool, only with Ci == Co).
def repvgg_block(x, br, relu: bool = True) -> np.ndarray:
    """The training-time block: each branch's conv of x, summed, plus x for
    the identity branch, then ReLU (when ``relu``)."""
    x = _d(x)
    y = None
    for k in (1, 3, 5):
        if br.get(f"w{k}") is not None:
            t = conv2d(x, br[f"w{k}"], br[f"b{k}"])
            y = t if y is None else y + t
    if br.get("identity"):
        assert y is None or x.shape[-1] == y.shape[-1], "identity branch needs C_in == C_out"
        y = x.copy() if y is None else y + x
    return np.maximum(y, 0.0) if relu else y


def repvgg_merge(br, cin: int, cout: int) -> Tuple[np.ndarray, np.ndarray]:
    """The inference-time 5x5 conv (w [Co,Ci,5,5], b [Co]) of a block: each
    branch's kernel placed at the centre of a zero 5x5 kernel, the identity
    as a unit tap at the centre of (co, co), all summed; biases summed."""
    w = np.zeros((cout, cin, 5, 5))
    b = np.zeros(cout)
    for k in (1, 3, 5):
        if br.get(f"w{k}") is not None:
            o = (5 - k) // 2
            w[:, :, o:o + k, o:o + k] += _d(br[f"w{k}"])
            b += _d(br[f"b{k}"])
    if br.get("identity"):
        assert cin == cout
        for c in range(cout):
            w[c, c, 2, 2] += 1.0
    return w, b


def repvgg_unet(X, branches, cfg) -> np.ndarray:
    """Raw network output h of the U-Net whose every conv is a training-time
    RepVGG block (branches in blob order; the head block has no ReLU)."""
    L = cfg.levels
    X = _d(X)
    e = [repvgg_block(X, branches[0])]
    for l in range(1, L):
        e.append(repvgg_block(avgpool2(e[-1]), branches[l]))
    u = e[L - 1]
    for j, l in enumerate(range(L - 2, -1, -1)):
        u = repvgg_block(np.concatenate([upsample2(u), e[l]], axis=-1), branches[L + j])
    return repvgg_block(u, branches[-1], relu=False)


# ---------------------------------------------------------------- training
def smape(y, t, eps: float = 0.01):
    """(SMAPE (Eq. 6), its gradient with respect to y)."""
    y, t = _d(y), _d(t)
    g = np.empty_like(y)
    v = _load().wo_smape(y.size, _ptr(y), _ptr(t), eps, _ptr(g))
    return v, g


def conv3x3_backward(x, w, g, need_dx: bool = True):
    """(dx, dw, db) of out = conv3x3(x; w, b) for upstream gradient g."""
    x, w, g = _d(x), _d(w), _d(g)
    H, W, Cin = x.shape
    Cout = w.shape[0]
    dx = np.empty_like(x) if need_dx else None
    dw = np.empty_like(w)
    db = np.empty(Cout)
    _load().wo_conv3x3_backward(H, W, Cin, Cout, _ptr(x), _ptr(w), _ptr(g),
                                _ptr(dx) if need_dx else None, _ptr(dw), _ptr(db))
    return dx, dw, db


def avgpool2_backward(dout) -> np.ndarray:
    dout = _d(dout)
    Ho, Wo, C = dout.shape
    din = np.empty((2 * Ho, 2 * Wo, C))
    _load().wo_avgpool2_backward(2 * Ho, 2 * Wo, C, _ptr(dout), _ptr(din))
    return din


def upsample2_backward(dout) -> np.ndarray:
    dout = _d(dout)
    H2, W2, C = dout.shape
    din = np.empty((H2 // 2, W2 // 2, C))
    _load().wo_upsample2_backward(H2 // 2, W2 // 2, C, _ptr(dout), _ptr(din))
    return din


def adam(w, g, m, v, t: int, lr: float = 1e-3, b1: float = 0.9, b2: float = 0.999,
         eps: float = 1e-8):
    """One Adam step in place on float64 arrays w, m, v (t >= 1)."""
    for a in (w, m, v):
        assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    g = _d(g)
    _load().wo_adam(w.size, _ptr(w), _ptr(g), _ptr(m), _ptr(v), t, lr, b1, b2, eps)


def _convs(blob, cfg, in_ch: int = 10):
    """[(w [Co,Ci,3,3], b [Co])] in blob order, as float64."""
    blob = _d(blob)
    L, ch = cfg.levels, cfg.channels
    cin = [in_ch] + [ch[l - 1] for l in range(1, L)] + \
          [ch[l + 1] + ch[l] for l in range(L - 2, -1, -1)] + [ch[0]]
    cout = [ch[l] for l in range(L)] + [ch[l] for l in range(L - 2, -1, -1)] + \
           [2 * len(cfg.kernel_sizes)]
    out, off = [], 0
    for ci, co in zip(cin, cout):
        w = blob[off:off + co * ci * 9].reshape(co, ci, 3, 3)
        off += co * ci * 9
        b = blob[off:off + co]
        off += co
        out.append((w, b))
    return out


def train_grads(frame: Dict[str, np.ndarray], target, blob, cfg, eps_smape: float = 0.01,
                cotangent=None):
    """(SMAPE loss, gradient of the loss with respect to the weight blob)
    for one frame: the whole per-frame path forward (preprocess, U-Net,
    weight activation, decode, fusion, remodulation), SMAPE against the
    reference ``target`` [H,W,3], and the chain rule back through every step
    (Eq. 1 minimised over the network parameters).  The gradient has the
    blob's layout.  With ``cotangent`` g [H,W,3] the loss is instead the
    linear functional sum(g * y) (a smooth loss, for finite differences)."""
    L, ch, M = cfg.levels, cfg.channels, len(cfg.kernel_sizes)
    X, c, mod = preprocess(frame["radiance"], frame["albedo"], frame["normal"], frame["depth"],
                           cfg.gamma, cfg.depth_near, cfg.depth_far, cfg.eps_albedo)
    lay = unet_layers(X, blob, cfg)
    h = lay["h"]
    head = activate(h, M, cfg.weight_act)
    y = decode(head, c, mod, cfg.kernel_sizes, cfg.eps_norm)
    if cotangent is None:
        loss, gy = smape(y, target, eps_smape)
    else:
        gy = _d(cotangent)
        loss = float(np.sum(gy * y))
    dhead, _ = decode_vjp(head, c, mod, cfg.kernel_sizes, gy, cfg.eps_norm)
    dh = dhead.copy()
    if cfg.weight_act == "exp":
        dh[..., :M] *= head[..., :M]
    else:
        dh[..., :M] *= 1.0 / (1.0 + np.exp(-h[..., :M]))      # softplus' = logistic
    convs = _convs(blob, cfg)
    grads = [None] * len(convs)
    e = [lay[f"e{l}"] for l in range(L)]
    u = [lay[f"u{l}"] for l in range(L - 1)] + [e[L - 1]]
    # head
    du = [np.zeros_like(x) for x in u]
    de = [np.zeros_like(x) for x in e]
    dx, dw, db = conv3x3_backward(u[0], convs[-1][0], dh)
    grads[-1] = (dw, db)
    du[0] += dx
    # decoders, finest first (blob index L + j for level l = L - 2 - j)
    for l in range(0, L - 1):
        j = L - 2 - l
        gpre = du[l] * (u[l] > 0.0)
        cat = np.concatenate([upsample2(u[l + 1]), e[l]], axis=-1)
        dcat, dw, db = conv3x3_backward(cat, convs[L + j][0], gpre)
        grads[L + j] = (dw, db)
        du[l + 1] += upsample2_backward(dcat[..., :ch[l + 1]])
        de[l] += dcat[..., ch[l + 1]:]
    de[L - 1] += du[L - 1] if L > 1 else 0.0
    if L == 1:
        de[0] = du[0]
    # encoders, coarsest first
    for l in range(L - 1, 0, -1):
        gpre = de[l] * (e[l] > 0.0)
        dpool, dw, db = conv3x3_backward(avgpool2(e[l - 1]), convs[l][0], gpre)
        grads[l] = (dw, db)
        de[l - 1] += avgpool2_backward(dpool)
    gpre = de[0] * (e[0] > 0.0)
    _, dw, db = conv3x3_backward(X, convs[0][0], gpre, need_dx=False)
    grads[0] = (dw, db)
    flat = np.concatenate([np.concatenate([dw.ravel(), db]) for dw, db in grads])
    return loss, flat
