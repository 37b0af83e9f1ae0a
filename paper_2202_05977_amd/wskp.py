"""Python binding of libwskp (argument marshalling only).

Every function here has the name of the C entry point it calls (see
include/wskp.h) and does no arithmetic of its own: it checks that tensors
are contiguous float32 CUDA (HIP) tensors, passes their device pointers and
the current stream, and turns a failing status into ``WskpError``.  The
library is loaded after ``import torch`` so that it binds to the HIP runtime
torch already loaded.  There is no fallback: if libwskp.so is missing or
the device is not gfx950, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from .synth import NetConfig

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwskp.so")

PREC = {"fp32": 0, "bf16": 1, "fp8": 2}
ACT = {"softplus": 0, "exp": 1}
BATCH_REVERSE_TILES = 1
BATCH_GRAPH = 2

_lib = None
# number of kernel sizes M of each live handle (by handle value): the C
# entry points that take a head record have no channel argument, so the
# binding checks head tensors against the handle's 2M channels itself
_handle_M: Dict[int, int] = {}


class WskpError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where} failed: status {status} ({detail})")
        self.status = status


class wskp_config_t(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("levels", ctypes.c_int32),
        ("channels", ctypes.c_int32 * 8),
        ("num_kernels", ctypes.c_int32),
        ("kernel_sizes", ctypes.c_int32 * 8),
        ("precision", ctypes.c_int32),
        ("weight_act", ctypes.c_int32),
        ("eps_norm", ctypes.c_float),
        ("eps_albedo", ctypes.c_float),
        ("gamma", ctypes.c_float),
        ("depth_near", ctypes.c_float),
        ("depth_far", ctypes.c_float),
        ("conv_size", ctypes.c_int32),
    ]


class wskp_frame_t(ctypes.Structure):
    _fields_ = [
        ("H", ctypes.c_int32), ("W", ctypes.c_int32),
        ("radiance", ctypes.c_void_p), ("albedo", ctypes.c_void_p),
        ("normal", ctypes.c_void_p), ("depth", ctypes.c_void_p),
        ("out", ctypes.c_void_p),
    ]


def lib():
    """The loaded library (loads it on first use; raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, sz, i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int
        ip = ctypes.POINTER(ctypes.c_int)
        L.wskp_num_weights.argtypes = [ctypes.POINTER(wskp_config_t)]
        L.wskp_num_weights.restype = sz
        L.wskp_create.argtypes = [ctypes.POINTER(wskp_config_t), vp, sz, vp, i32,
                                  ctypes.POINTER(vp)]
        L.wskp_destroy.argtypes = [vp]
        L.wskp_workspace_size.argtypes = [vp, i32, ip, ip, ctypes.POINTER(sz)]
        L.wskp_denoise.argtypes = [vp, vp, i32, i32, vp, vp, vp, vp, vp, vp, sz]
        L.wskp_denoise_static.argtypes = [vp, vp, i32, i32, vp, vp, vp, vp, vp]
        L.wskp_static_scratch_bytes.argtypes = []
        L.wskp_static_scratch_bytes.restype = sz
        L.wskp_denoise_batch.argtypes = [vp, vp, i32, ctypes.POINTER(wskp_frame_t),
                                         ctypes.c_uint32, vp, sz]
        L.wskp_decode.argtypes = [vp, vp, i32, i32, i32, vp, vp, vp, vp]
        L.wskp_backward.argtypes = [vp, vp, i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, sz]
        L.wskp_backward_workspace_size.argtypes = [vp, i32, i32, i32, ctypes.POINTER(sz)]
        L.wskp_train_workspace_size.argtypes = [vp, i32, ip, ip, ctypes.POINTER(sz)]
        L.wskp_train_grads.argtypes = [vp, vp, i32, ctypes.POINTER(wskp_frame_t),
                                       ctypes.POINTER(vp), ctypes.c_float, vp, vp, vp, sz]
        L.wskp_adam.argtypes = [vp, vp, vp, vp, vp, i32, ctypes.c_float, ctypes.c_float,
                                ctypes.c_float, ctypes.c_float]
        L.wskp_get_weights.argtypes = [vp, vp, vp]
        L.wskp_repvgg_merge.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp, i32, vp, vp]
        L.wskp_pool2.argtypes = [vp, vp, i32, i32, vp, vp]
        L.wskp_mr_blend.argtypes = [vp, vp, i32, i32, vp, vp, vp, vp, vp]
        L.wskp_mr_workspace_size.argtypes = [vp, i32, i32, i32, ctypes.POINTER(sz)]
        L.wskp_mr_reconstruct.argtypes = [vp, vp, i32, i32, i32, vp, vp, vp, vp, vp, vp, sz]
        L.wskp_temporal.argtypes = [vp, vp, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp,
                                    ctypes.c_float, ctypes.c_float, ctypes.c_float, vp, vp]
        L.wskp_kp_map_bytes.argtypes = [vp, i32, i32, ctypes.POINTER(sz)]
        L.wskp_kp_expand.argtypes = [vp, vp, i32, i32, vp, vp, sz]
        L.wskp_kp_decode.argtypes = [vp, vp, i32, i32, vp, sz, vp, vp, vp, vp]
        L.wskp_workspace_tensor.argtypes = [vp, i32, ip, ip, i32, i32, ctypes.POINTER(sz),
                                            ip, ip, ip, ip]
        L.wskp_timing_enable.argtypes = [vp, i32]
        L.wskp_timing_read.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_float), ip, ip]
        L.wskp_launch_name.argtypes = [vp, i32]
        L.wskp_launch_name.restype = ctypes.c_char_p
        L.wskp_fp8_e4m3_encode.argtypes = [vp, vp, sz]
        L.wskp_fp8_e4m3_encode.restype = None
        L.wskp_status_string.argtypes = [i32]
        L.wskp_status_string.restype = ctypes.c_char_p
        L.wskp_last_error.argtypes = []
        L.wskp_last_error.restype = ctypes.c_char_p
        for name in ("wskp_create", "wskp_destroy", "wskp_workspace_size", "wskp_denoise",
                     "wskp_denoise_static", "wskp_denoise_batch", "wskp_decode", "wskp_backward",
                     "wskp_backward_workspace_size", "wskp_workspace_tensor",
                     "wskp_kp_map_bytes", "wskp_kp_expand", "wskp_kp_decode", "wskp_temporal",
                     "wskp_pool2", "wskp_mr_blend", "wskp_mr_workspace_size", "wskp_mr_reconstruct",
                     "wskp_train_workspace_size",
                     "wskp_train_grads", "wskp_adam", "wskp_get_weights", "wskp_repvgg_merge",
                     "wskp_timing_enable", "wskp_timing_read"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(status: int, where: str):
    if status != 0:
        L = lib()
        detail = L.wskp_last_error().decode() or L.wskp_status_string(status).decode()
        raise WskpError(status, where, detail)


def _ptr(t: Optional[torch.Tensor], name: str, shape: Optional[Sequence[int]] = None):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous float32")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def make_config(cfg: NetConfig, precision: str = "fp32") -> wskp_config_t:
    c = wskp_config_t()
    c.struct_size = ctypes.sizeof(wskp_config_t)
    c.levels = cfg.levels
    for i, ch in enumerate(cfg.channels[:8]):
        c.channels[i] = ch
    c.num_kernels = cfg.M          # the library rejects M > 8
    for i, k in enumerate(cfg.kernel_sizes[:8]):
        c.kernel_sizes[i] = k
    c.precision = PREC[precision]
    c.weight_act = ACT[cfg.weight_act]
    c.eps_norm = cfg.eps_norm
    c.eps_albedo = cfg.eps_albedo
    c.gamma = cfg.gamma
    c.depth_near = cfg.depth_near
    c.depth_far = cfg.depth_far
    c.conv_size = getattr(cfg, "conv_size", 3)
    return c


# ---------------------------------------------------------------- entry points
def wskp_num_weights(cfg: NetConfig) -> int:
    c = make_config(cfg)
    return int(lib().wskp_num_weights(ctypes.byref(c)))


def wskp_create(cfg: NetConfig, weights: np.ndarray, precision: str = "fp32",
                act_scales: Optional[np.ndarray] = None, device: int = 0) -> ctypes.c_void_p:
    c = make_config(cfg, precision)
    w = np.ascontiguousarray(weights, dtype=np.float32)
    sc = None
    if act_scales is not None:
        sc = np.ascontiguousarray(act_scales, dtype=np.float32)
    h = ctypes.c_void_p()
    _check(lib().wskp_create(ctypes.byref(c), w.ctypes.data, w.size,
                             None if sc is None else sc.ctypes.data, device, ctypes.byref(h)),
           "wskp_create")
    _handle_M[h.value] = cfg.M
    return h


def wskp_repvgg_merge(branch: dict, cin: int, cout: int):
    """The 5x5 conv (w [cout, cin, 5, 5] float32, b [cout]) that a RepVGG
    block computes: ``branch`` holds "w1"/"b1", "w3"/"b3", "w5"/"b5" (a
    missing pair is an absent branch) and "identity"."""
    def arr(key, shape):
        a = branch.get(key)
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=np.float32)
        if a.shape != shape:
            raise ValueError(f"{key} has shape {a.shape}, expected {shape}")
        return a
    parts = []
    for k in (1, 3, 5):
        if (branch.get(f"w{k}") is None) != (branch.get(f"b{k}") is None):
            raise ValueError(f"branch {k}x{k}: give both w{k} and b{k}, or neither")
        parts += [arr(f"w{k}", (cout, cin, k, k)), arr(f"b{k}", (cout,))]
    w = np.empty((cout, cin, 5, 5), np.float32)
    b = np.empty((cout,), np.float32)
    ptr = [None if a is None else a.ctypes.data for a in parts]
    _check(lib().wskp_repvgg_merge(cin, cout, *ptr, int(bool(branch.get("identity"))),
                                   w.ctypes.data, b.ctypes.data), "wskp_repvgg_merge")
    return w, b


def repvgg_blob(cfg: NetConfig, branches) -> np.ndarray:
    """The weight blob of ``cfg`` (conv_size 5) from training-time RepVGG
    parameters, one block per conv in blob order, merged by the library."""
    from .synth import conv_shapes
    parts = []
    for (_, ci, co), br in zip(conv_shapes(cfg), branches):
        w, b = wskp_repvgg_merge(br, ci, co)
        parts += [w.ravel(), b]
    return np.concatenate(parts)


def wskp_destroy(h) -> None:
    _check(lib().wskp_destroy(h), "wskp_destroy")
    _handle_M.pop(getattr(h, "value", h), None)


def _check_head(h, head, name: str = "head") -> None:
    """head must be [N,H,W,2M] for the handle's M (the kernels index it with
    that stride; a narrower tensor would be read or written out of bounds)."""
    M = _handle_M.get(getattr(h, "value", h))
    if M is None:
        raise ValueError("unknown handle (not created by this binding, or destroyed)")
    if head.dim() != 4 or head.shape[-1] != 2 * M:
        raise ValueError(f"{name} has shape {tuple(head.shape)}; expected [N,H,W,{2 * M}] "
                         f"for a handle with M = {M}")


def wskp_workspace_size(h, Hs: Sequence[int], Ws: Sequence[int]) -> int:
    n = len(Hs)
    a = (ctypes.c_int * n)(*Hs)
    b = (ctypes.c_int * n)(*Ws)
    out = ctypes.c_size_t()
    _check(lib().wskp_workspace_size(h, n, a, b, ctypes.byref(out)), "wskp_workspace_size")
    return out.value


def wskp_workspace_tensor(h, Hs, Ws, frame: int, which: int):
    n = len(Hs)
    a = (ctypes.c_int * n)(*Hs)
    b = (ctypes.c_int * n)(*Ws)
    off = ctypes.c_size_t()
    th, tw, tc, eb = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(lib().wskp_workspace_tensor(h, n, a, b, frame, which, ctypes.byref(off),
                                       ctypes.byref(th), ctypes.byref(tw), ctypes.byref(tc),
                                       ctypes.byref(eb)), "wskp_workspace_tensor")
    return off.value, (th.value, tw.value, tc.value), eb.value


def wskp_denoise(h, radiance, albedo, normal, depth, out, ws, stream=None) -> None:
    H, W = radiance.shape[:2]
    _check(lib().wskp_denoise(h, _stream(stream), H, W,
                              _ptr(radiance, "radiance", (H, W, 3)),
                              _ptr(albedo, "albedo", (H, W, 3)),
                              _ptr(normal, "normal", (H, W, 3)),
                              _ptr(depth, "depth", (H, W, 1)),
                              _ptr(out, "out", (H, W, 3)),
                              ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size()),
           "wskp_denoise")


def wskp_denoise_static(h, radiance, albedo, normal, depth, out, stream=None) -> None:
    H, W = radiance.shape[:2]
    _check(lib().wskp_denoise_static(h, _stream(stream), H, W,
                                     _ptr(radiance, "radiance", (H, W, 3)),
                                     _ptr(albedo, "albedo", (H, W, 3)),
                                     _ptr(normal, "normal", (H, W, 3)),
                                     _ptr(depth, "depth", (H, W, 1)),
                                     _ptr(out, "out", (H, W, 3))), "wskp_denoise_static")


def wskp_static_scratch_bytes() -> int:
    return int(lib().wskp_static_scratch_bytes())


def wskp_denoise_batch(h, frames: List[Dict[str, torch.Tensor]], ws, flags: int = 0,
                       stream=None) -> None:
    n = len(frames)
    arr = (wskp_frame_t * n)()
    for i, f in enumerate(frames):
        H, W = f["radiance"].shape[:2]
        arr[i].H, arr[i].W = H, W
        arr[i].radiance = _ptr(f["radiance"], "radiance", (H, W, 3)).value
        arr[i].albedo = _ptr(f["albedo"], "albedo", (H, W, 3)).value
        arr[i].normal = _ptr(f["normal"], "normal", (H, W, 3)).value
        arr[i].depth = _ptr(f["depth"], "depth", (H, W, 1)).value
        arr[i].out = _ptr(f["out"], "out", (H, W, 3)).value
    _check(lib().wskp_denoise_batch(h, _stream(stream), n, arr, flags,
                                    ctypes.c_void_p(ws.data_ptr()),
                                    ws.numel() * ws.element_size()), "wskp_denoise_batch")


def wskp_decode(h, head, c, mod, out, stream=None) -> None:
    _check_head(h, head)
    N, H, W, twoM = head.shape
    _check(lib().wskp_decode(h, _stream(stream), N, H, W, _ptr(head, "head"),
                             _ptr(c, "c", (N, H, W, 3)),
                             _ptr(mod, "mod", (N, H, W, 3)),
                             _ptr(out, "out", (N, H, W, 3))), "wskp_decode")


def wskp_backward_workspace_size(h, N: int, H: int, W: int) -> int:
    out = ctypes.c_size_t()
    _check(lib().wskp_backward_workspace_size(h, N, H, W, ctypes.byref(out)),
           "wskp_backward_workspace_size")
    return out.value


def wskp_backward(h, head, c, mod, grad_out, grad_head, grad_c, ws, stream=None) -> None:
    _check_head(h, head)
    N, H, W, twoM = head.shape
    _check(lib().wskp_backward(h, _stream(stream), N, H, W, _ptr(head, "head"),
                               _ptr(c, "c", (N, H, W, 3)), _ptr(mod, "mod", (N, H, W, 3)),
                               _ptr(grad_out, "grad_out", (N, H, W, 3)),
                               _ptr(grad_head, "grad_head", (N, H, W, twoM)),
                               _ptr(grad_c, "grad_c", (N, H, W, 3)),
                               ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size()),
           "wskp_backward")


def wskp_train_workspace_size(h, Hs, Ws) -> int:
    n = len(Hs)
    a = (ctypes.c_int * n)(*Hs)
    b = (ctypes.c_int * n)(*Ws)
    out = ctypes.c_size_t()
    _check(lib().wskp_train_workspace_size(h, n, a, b, ctypes.byref(out)), "wskp_train_workspace_size")
    return out.value


def wskp_train_grads(h, frames, targets, grad, loss, ws, eps_smape: float = 0.01, stream=None) -> None:
    """frames: dicts as for wskp_denoise_batch (with "out"); targets: [H,W,3]
    device tensors; grad: [wskp_num_weights] float32; loss: [1] float32."""
    n = len(frames)
    arr = (wskp_frame_t * n)()
    for i, f in enumerate(frames):
        H, W = f["radiance"].shape[:2]
        arr[i].H, arr[i].W = H, W
        arr[i].radiance = _ptr(f["radiance"], "radiance", (H, W, 3)).value
        arr[i].albedo = _ptr(f["albedo"], "albedo", (H, W, 3)).value
        arr[i].normal = _ptr(f["normal"], "normal", (H, W, 3)).value
        arr[i].depth = _ptr(f["depth"], "depth", (H, W, 1)).value
        arr[i].out = _ptr(f["out"], "out", (H, W, 3)).value
    tg = (ctypes.c_void_p * n)(*[_ptr(t, "target", tuple(frames[i]["radiance"].shape)).value
                                 for i, t in enumerate(targets)])
    _check(lib().wskp_train_grads(h, _stream(stream), n, arr, tg, eps_smape, _ptr(grad, "grad"),
                                  _ptr(loss, "loss", (1,)), ctypes.c_void_p(ws.data_ptr()),
                                  ws.numel() * ws.element_size()), "wskp_train_grads")


def wskp_adam(h, grad, m, v, step: int, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8, stream=None) -> None:
    _check(lib().wskp_adam(h, _stream(stream), _ptr(grad, "grad"), _ptr(m, "m"), _ptr(v, "v"), step,
                           lr, beta1, beta2, eps), "wskp_adam")


def wskp_get_weights(h, dst, stream=None) -> None:
    _check(lib().wskp_get_weights(h, _stream(stream), _ptr(dst, "dst")), "wskp_get_weights")


def wskp_pool2(h, x, out, stream=None) -> None:
    H, W = x.shape[:2]
    _check(lib().wskp_pool2(h, _stream(stream), H, W, _ptr(x, "in", (H, W, 3)),
                            _ptr(out, "out", (H // 2, W // 2, 3))), "wskp_pool2")


def wskp_mr_blend(h, fine, coarse, alpha, mod, out, stream=None) -> None:
    H, W = fine.shape[:2]
    _check(lib().wskp_mr_blend(h, _stream(stream), H, W, _ptr(fine, "fine", (H, W, 3)),
                               _ptr(coarse, "coarse", (H // 2, W // 2, 3)),
                               _ptr(alpha, "alpha", (H, W)), _ptr(mod, "mod", (H, W, 3)),
                               _ptr(out, "out", (H, W, 3))), "wskp_mr_blend")


def wskp_mr_workspace_size(h, L: int, H: int, W: int) -> int:
    n = ctypes.c_size_t()
    _check(lib().wskp_mr_workspace_size(h, L, H, W, ctypes.byref(n)), "wskp_mr_workspace_size")
    return int(n.value)


def mr_reconstruct(h, heads, c, alphas, mod, stream=None, ws=None):
    """Multi-resolution reconstruction (wskp_mr_reconstruct): heads[l]
    [1, H>>l, W>>l, 2M] activated head records, c [H,W,3] irradiance,
    alphas[l] [H>>l, W>>l] for the L-1 finer levels, mod [H,W,3] or None.
    ``ws``: optional uint8 device workspace of wskp_mr_workspace_size bytes."""
    L = len(heads)
    H, W = c.shape[:2]
    if len(alphas) != L - 1:
        raise ValueError(f"{L} levels need {L - 1} blend weights, got {len(alphas)}")
    hp = (ctypes.c_void_p * L)()
    for l in range(L):
        _check_head(h, heads[l], f"heads[{l}]")
        hp[l] = _ptr(heads[l], f"heads[{l}]", (1, H >> l, W >> l, heads[l].shape[-1]))
    ap = (ctypes.c_void_p * max(1, L - 1))()
    for l in range(L - 1):
        ap[l] = _ptr(alphas[l], f"alphas[{l}]", (H >> l, W >> l))
    need = wskp_mr_workspace_size(h, L, H, W)
    if ws is None:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=c.device)
    elif ws.numel() < need:
        raise ValueError(f"workspace of {ws.numel()} bytes, need {need}")
    out = torch.empty((H, W, 3), dtype=torch.float32, device=c.device)
    _check(lib().wskp_mr_reconstruct(h, _stream(stream), L, H, W, ctypes.cast(hp, ctypes.c_void_p),
                                     _ptr(c, "c", (H, W, 3)), ctypes.cast(ap, ctypes.c_void_p),
                                     _ptr(mod, "mod", (H, W, 3)), _ptr(out, "out", (H, W, 3)),
                                     ctypes.c_void_p(ws.data_ptr()), ws.numel()), "wskp_mr_reconstruct")
    return out


TEMPORAL_DEFAULTS = {"alpha_min": 0.2, "pos_tol": 0.02, "normal_tol": 0.9}


def wskp_temporal(h, radiance, normal, wpos, motion, prev, out_radiance, out_length,
                  alpha_min: float = 0.2, pos_tol: float = 0.02, normal_tol: float = 0.9,
                  stream=None) -> None:
    """prev: None (first frame) or a dict with the previous call's
    ``radiance`` and ``length`` and the previous frame's ``normal`` and
    ``wpos``."""
    H, W = radiance.shape[:2]
    p = prev or {}
    _check(lib().wskp_temporal(
        h, _stream(stream), H, W, _ptr(radiance, "radiance", (H, W, 3)),
        _ptr(normal, "normal", (H, W, 3)), _ptr(wpos, "wpos", (H, W, 3)),
        _ptr(motion, "motion", (H, W, 2)),
        _ptr(p.get("radiance"), "prev radiance", (H, W, 3)),
        _ptr(p.get("length"), "prev length", (H, W)),
        _ptr(p.get("normal"), "prev normal", (H, W, 3)),
        _ptr(p.get("wpos"), "prev wpos", (H, W, 3)),
        alpha_min, pos_tol, normal_tol, _ptr(out_radiance, "out radiance", (H, W, 3)),
        _ptr(out_length, "out length", (H, W))), "wskp_temporal")


def wskp_kp_map_bytes(h, H: int, W: int) -> int:
    out = ctypes.c_size_t()
    _check(lib().wskp_kp_map_bytes(h, H, W, ctypes.byref(out)), "wskp_kp_map_bytes")
    return out.value


def wskp_kp_expand(h, head, maps, stream=None) -> None:
    _check_head(h, head)
    N, H, W, _ = head.shape
    if N != 1:
        raise ValueError("wskp_kp_expand takes one frame")
    _check(lib().wskp_kp_expand(h, _stream(stream), H, W, _ptr(head, "head"), _ptr(maps, "maps"),
                                maps.numel() * 4), "wskp_kp_expand")


def wskp_kp_decode(h, maps, head, c, mod, out, stream=None) -> None:
    _check_head(h, head)
    N, H, W, _ = head.shape
    if N != 1:
        raise ValueError("wskp_kp_decode takes one frame")
    _check(lib().wskp_kp_decode(h, _stream(stream), H, W, _ptr(maps, "maps"), maps.numel() * 4,
                                _ptr(head, "head"), _ptr(c, "c", (1, H, W, 3)),
                                _ptr(mod, "mod", (1, H, W, 3)), _ptr(out, "out", (1, H, W, 3))),
           "wskp_kp_decode")


def wskp_fp8_e4m3_encode(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float32)
    out = np.empty(x.shape, dtype=np.uint8)
    lib().wskp_fp8_e4m3_encode(x.ctypes.data, out.ctypes.data, x.size)
    return out


def wskp_timing_enable(h, max_calls: int) -> None:
    _check(lib().wskp_timing_enable(h, max_calls), "wskp_timing_enable")


def wskp_timing_read(h):
    """{launch name: (ms summed over calls)}, number of calls."""
    ms = (ctypes.c_float * 64)()
    nl, nc = ctypes.c_int(), ctypes.c_int()
    _check(lib().wskp_timing_read(h, 64, ms, ctypes.byref(nl), ctypes.byref(nc)),
           "wskp_timing_read")
    names = [lib().wskp_launch_name(h, i).decode() for i in range(nl.value)]
    return {n: float(ms[i]) for i, n in enumerate(names)}, nc.value


# ---------------------------------------------------------------- conveniences
class Denoiser:
    """Owns a handle and a workspace; ``__call__`` denoises one frame."""

    def __init__(self, cfg: NetConfig, weights: np.ndarray, precision: str = "fp32",
                 device: int = 0, act_scales: Optional[np.ndarray] = None):
        self.cfg = cfg
        self.precision = precision
        self.device = torch.device("cuda", device)
        self.h = wskp_create(cfg, weights, precision, act_scales, device)
        self._ws = None

    def workspace(self, Hs, Ws) -> torch.Tensor:
        need = wskp_workspace_size(self.h, Hs, Ws)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        return self._ws

    def __call__(self, frame: Dict[str, torch.Tensor], out: Optional[torch.Tensor] = None,
                 stream=None) -> torch.Tensor:
        H, W = frame["radiance"].shape[:2]
        if out is None:
            out = torch.empty((H, W, 3), dtype=torch.float32, device=self.device)
        ws = self.workspace([H], [W])
        wskp_denoise(self.h, frame["radiance"], frame["albedo"], frame["normal"], frame["depth"],
                     out, ws, stream)
        return out

    def batch(self, frames: List[Dict[str, torch.Tensor]], flags: int = 0, stream=None):
        Hs = [f["radiance"].shape[0] for f in frames]
        Ws = [f["radiance"].shape[1] for f in frames]
        ws = self.workspace(Hs, Ws)
        wskp_denoise_batch(self.h, frames, ws, flags, stream)

    def intermediate(self, Hs, Ws, frame: int, which: int) -> torch.Tensor:
        """View of an intermediate map in the current workspace (debugging),
        as [H_l, W_l, C]; the planar head record (which = 200) is returned as
        a permuted [H, W, 2M] view."""
        off, (th, tw, tc), eb = wskp_workspace_tensor(self.h, Hs, Ws, frame, which)
        ws = self._ws
        raw = ws[off:off + th * tw * tc * eb]
        if eb == 4:
            t = raw.view(torch.float32).view(th, tw, tc)
            return t.permute(1, 2, 0) if which == 200 else t
        return raw.view(torch.bfloat16).view(th, tw, tc)

    def close(self):
        if self.h is not None:
            wskp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def calibrate_fp8_scales(cfg: NetConfig, weights: np.ndarray, frame: Dict[str, torch.Tensor],
                         margin: float = 2.0) -> np.ndarray:
    """Per-conv input scales for the FP8 form from one pass of the FP32 path.

    Each conv's input activations are stored as e4m3(x / s) with
    s = margin * amax(x) / 448, amax measured on ``frame`` (the network input
    lies in [0, 1]; a decoder conv's input is [up(u_{l+1}), e_l], so its
    amax is the larger of the two).
    """
    dn = Denoiser(cfg, weights, "fp32")
    H, W = frame["radiance"].shape[:2]
    dn(frame)
    torch.cuda.synchronize()
    L = cfg.levels
    amax_e = [float(dn.intermediate([H], [W], 0, l).abs().max()) for l in range(L)]
    amax_u = [float(dn.intermediate([H], [W], 0, 100 + l).abs().max()) for l in range(L - 1)]
    amax_u.append(amax_e[L - 1])
    amax = [1.0] + [amax_e[l - 1] for l in range(1, L)]
    amax += [max(amax_u[l + 1], amax_e[l]) for l in range(L - 2, -1, -1)]
    amax.append(amax_u[0])
    dn.close()
    return (np.maximum(np.array(amax), 1e-6) * margin / 448.0).astype(np.float32)


class WskpDecode(torch.autograd.Function):
    """Decode + fusion + remodulation with the hand-written adjoint.

    forward(head [N,H,W,2M], c [N,H,W,3], mod [N,H,W,3] or None) -> y.
    Gradients flow to head (weights and logits) and c; mod is a constant.
    """

    @staticmethod
    def forward(ctx, handle, head, c, mod):
        head = head.contiguous()
        c = c.contiguous()
        mod = None if mod is None else mod.contiguous()
        out = torch.empty(c.shape, dtype=torch.float32, device=c.device)
        wskp_decode(handle, head, c, mod, out)
        ctx.handle = handle
        ctx.save_for_backward(head, c, mod if mod is not None else torch.empty(0))
        ctx.has_mod = mod is not None
        return out

    @staticmethod
    def backward(ctx, g):
        head, c, mod = ctx.saved_tensors
        mod = mod if ctx.has_mod else None
        N, H, W, _ = head.shape
        g = g.contiguous()
        gh = torch.empty_like(head)
        gc = torch.empty_like(c)
        ws = torch.empty(wskp_backward_workspace_size(ctx.handle, N, H, W), dtype=torch.uint8,
                         device=head.device)
        wskp_backward(ctx.handle, head, c, mod, g, gh, gc, ws)
        return None, gh, gc, None
