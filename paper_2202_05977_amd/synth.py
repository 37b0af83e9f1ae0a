"""Seeded synthetic inputs: frames, network weights and workload configurations.

This module is shared by the HIP path's tests and benchmarks and by the CPU
oracle's tests.  It holds no arithmetic of the denoising method itself: it
only draws numbers.  Everything is NumPy (PCG64 via ``default_rng``) so a seed
gives the same arrays on every machine.

The frames stand in for the 1-spp path-traced buffers of the paper's BMFR
workload (Sec. 5.1): 1280x720 frames carrying noisy radiance plus noise-free
albedo, shading normal and depth (10 network input channels, Sec. 5.1), with
heavy-tailed per-sample noise.  The network weights stand in for a trained
ImportanceNet (Sec. 4.1): no trained weights exist, so convolutions are drawn
He-normal from a seed.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Tuple

import numpy as np

__all__ = [
    "NetConfig", "CONFIGS", "make_frame", "make_weights", "num_weights",
    "conv_shapes", "make_frame_batch",
]


@dataclasses.dataclass(frozen=True)
class NetConfig:
    """Shape of the U-Net encoder and of the kernel set it predicts.

    ``channels[l]`` is the width of U-Net level ``l`` (level 0 is full
    resolution).  The network predicts ``M = len(kernel_sizes)`` weight maps
    and ``M`` fusion logits (Eq. 5 and Sec. 4.2, "Kernel Fusion").
    """
    levels: int
    channels: Tuple[int, ...]
    kernel_sizes: Tuple[int, ...]
    in_channels: int = 10
    eps_norm: float = 1e-10
    eps_albedo: float = 1e-3
    gamma: float = 2.2
    depth_near: float = 1.0
    depth_far: float = 10.0
    weight_act: str = "softplus"   # "softplus" or "exp" (Eq. 3)
    conv_size: int = 3             # 3, or 5: every conv a merged RepVGG block (Sec. 4.1)

    @property
    def M(self) -> int:
        return len(self.kernel_sizes)

    @property
    def out_channels(self) -> int:
        return 2 * self.M

    @property
    def align(self) -> int:
        """Frame sides must be a multiple of this (one 2x2 pool per level)."""
        return 1 << (self.levels - 1)


# The workloads: a small launch-bound parity frame, the 720p headline frame,
# the 1080p precision sweep (same net), the serving mix and the
# differentiation batch.
SMALL = NetConfig(levels=3, channels=(16, 32, 64), kernel_sizes=(3, 5, 7))
HD = NetConfig(levels=4, channels=(32, 64, 96, 128), kernel_sizes=(3, 5, 7, 9, 11))
# The paper's own kernel set (Sec. 5.3: six weight maps and six fusion
# weights; Sec. 4.2 "Kernel Fusion": k_i = k_b + i k_s with k_b = 3, k_s = 2)
# and its literal weight form (Eq. 3: the window softmax, W = exp(h)), on the
# hd U-Net.
PAPER6 = NetConfig(levels=4, channels=(32, 64, 96, 128), kernel_sizes=(3, 5, 7, 9, 11, 13),
                   weight_act="exp")
# RepVGG encoders and decoders (Sec. 4.1, prediction phase): every conv of
# the U-Net is a RepVGG block, run as its merged 5x5 conv.
REPVGG = NetConfig(levels=4, channels=(32, 64, 96, 128), kernel_sizes=(3, 5, 7, 9, 11),
                   conv_size=5)
REPVGG_SMALL = NetConfig(levels=3, channels=(16, 32, 64), kernel_sizes=(3, 5, 7), conv_size=5)
CONFIGS: Dict[str, NetConfig] = {"small": SMALL, "hd": HD, "paper6": PAPER6, "repvgg": REPVGG,
                                 "repvgg_small": REPVGG_SMALL}

SERVE_RESOLUTIONS: Tuple[Tuple[int, int], ...] = ((360, 640), (720, 1280), (1080, 1920), (1440, 2560))


def conv_shapes(cfg: NetConfig) -> List[Tuple[str, int, int]]:
    """(name, C_in, C_out) of every 3x3 conv, in weight-blob order.

    Order: enc0..enc_{L-1}, dec_{L-2}..dec_0, head.  A decoder conv at level
    l reads [up(u_{l+1}), e_l] so C_in = C_{l+1} + C_l.
    """
    L, ch = cfg.levels, cfg.channels
    shapes = [("enc0", cfg.in_channels, ch[0])]
    for l in range(1, L):
        shapes.append((f"enc{l}", ch[l - 1], ch[l]))
    for l in range(L - 2, -1, -1):
        shapes.append((f"dec{l}", ch[l + 1] + ch[l], ch[l]))
    shapes.append(("head", ch[0], cfg.out_channels))
    return shapes


def num_weights(cfg: NetConfig) -> int:
    k2 = cfg.conv_size * cfg.conv_size
    return sum(co * ci * k2 + co for _, ci, co in conv_shapes(cfg))


def make_weights(cfg: NetConfig, seed: int = 0) -> np.ndarray:
    """Flat float32 blob: for each conv, w[C_out][C_in][k][k] then b[C_out]
    (k = cfg.conv_size).

    He-normal weights, N(0, 2 / (k^2 C_in)); biases U(-0.05, 0.05) so the
    bias path is exercised.
    """
    rng = np.random.default_rng(seed)
    k = cfg.conv_size
    parts = []
    for _, ci, co in conv_shapes(cfg):
        w = rng.normal(0.0, np.sqrt(2.0 / (k * k * ci)), size=(co, ci, k, k))
        b = rng.uniform(-0.05, 0.05, size=(co,))
        parts.append(w.astype(np.float32).ravel())
        parts.append(b.astype(np.float32))
    blob = np.concatenate(parts)
    assert blob.size == num_weights(cfg)
    return blob


def make_repvgg_branches(cfg: NetConfig, seed: int = 0) -> List[Dict[str, np.ndarray]]:
    """Training-time RepVGG parameters for every conv of ``cfg`` (blob
    order): 1x1, 3x3 and 5x5 branches, float32, each He-normal with a third
    of the usual variance (the branches add up), biases U(-0.02, 0.02), and
    the identity branch wherever C_in == C_out."""
    rng = np.random.default_rng(seed)
    out = []
    for _, ci, co in conv_shapes(cfg):
        br: Dict[str, np.ndarray] = {}
        for k in (1, 3, 5):
            br[f"w{k}"] = rng.normal(0.0, np.sqrt(2.0 / (3 * k * k * ci)),
                                     size=(co, ci, k, k)).astype(np.float32)
            br[f"b{k}"] = rng.uniform(-0.02, 0.02, size=(co,)).astype(np.float32)
        br["identity"] = ci == co
        out.append(br)
    return out


def make_frame(seed: int, H: int, W: int) -> Dict[str, np.ndarray]:
    """One synthetic 1-spp frame, NHWC float32 without the batch axis.

    Returns ``radiance`` [H,W,3] (noisy), ``albedo`` [H,W,3], ``normal``
    [H,W,3] (unit vectors), ``depth`` [H,W,1] in [1, 10] and ``clean``
    [H,W,3] (the noise-free radiance, used as the training target).
    """
    rng = np.random.default_rng(seed)
    x = (np.arange(W, dtype=np.float64) + 0.5) / W
    y = (np.arange(H, dtype=np.float64) + 0.5) / H
    u, v = np.meshgrid(x, y)                                  # [H, W]

    # irradiance: a sum of 8 random plane waves on a floor of 0.25
    A = rng.uniform(0.02, 0.12, size=8)
    fx = rng.uniform(-12.0, 12.0, size=8)
    fy = rng.uniform(-12.0, 12.0, size=8)
    ph = rng.uniform(0.0, 2 * np.pi, size=8)
    E = np.full((H, W), 0.25)
    for j in range(8):
        E += A[j] * (1.0 + np.sin(2 * np.pi * (fx[j] * u + fy[j] * v) + ph[j]))
    tint = rng.uniform(0.8, 1.2, size=3)

    # albedo: 12 Voronoi cells (pixel-space distance, ties -> lowest index)
    sites = rng.uniform(0.0, 1.0, size=(12, 2))
    colours = rng.uniform(0.1, 0.9, size=(12, 3))
    px = u * W
    py = v * H
    best = np.full((H, W), np.inf)
    label = np.zeros((H, W), dtype=np.int64)
    for s in range(12):
        dist = (px - sites[s, 0] * W) ** 2 + (py - sites[s, 1] * H) ** 2
        closer = dist < best
        best = np.where(closer, dist, best)
        label = np.where(closer, s, label)
    albedo = colours[label]                                  # [H, W, 3]

    clean = albedo * tint[None, None, :] * E[..., None]

    # normals from a height field of 4 waves; slopes w.r.t. normalised coords
    B = rng.uniform(0.005, 0.02, size=4)
    g = rng.uniform(-6.0, 6.0, size=(4, 2))
    psi = rng.uniform(0.0, 2 * np.pi, size=4)
    hx = np.zeros((H, W))
    hy = np.zeros((H, W))
    for j in range(4):
        arg = 2 * np.pi * (g[j, 0] * u + g[j, 1] * v) + psi[j]
        hx += B[j] * np.cos(arg) * 2 * np.pi * g[j, 0]
        hy += B[j] * np.cos(arg) * 2 * np.pi * g[j, 1]
    nrm = np.stack([-hx, -hy, np.ones_like(hx)], axis=-1)
    nrm /= np.linalg.norm(nrm, axis=-1, keepdims=True)

    # depth in [1, 10]
    s1, s2 = rng.uniform(1.0, 4.0, size=2)
    t1, t2 = rng.uniform(0.0, 2 * np.pi, size=2)
    dd = 0.5 + 0.25 * (np.sin(2 * np.pi * u * s1 + t1) + np.sin(2 * np.pi * v * s2 + t2))
    depth = 1.0 + 9.0 * np.clip(dd, 0.0, 1.0)

    # 1-spp-like noise: Gamma(0.5, scale 2) per sample (mean 1, var 2) and
    # 0.1% fireflies that multiply all three channels by 50
    G = rng.gamma(0.5, 2.0, size=(H, W, 3))
    fire = rng.random(size=(H, W)) < 1e-3
    G = G * np.where(fire, 50.0, 1.0)[..., None]
    radiance = clean * G

    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return {
        "radiance": f32(radiance),
        "albedo": f32(albedo),
        "normal": f32(nrm),
        "depth": f32(depth[..., None]),
        "clean": f32(clean),
    }


def make_sequence(seed: int, H: int, W: int, T: int, pan=(1.37, -0.61), obj_vel=(2.3, 1.1)):
    """T consecutive synthetic 1-spp frames of a moving scene, for temporal
    accumulation (Sec. 4.1, last paragraph).

    The camera pans across the procedural scene of ``make_frame`` by
    ``pan`` pixels per frame and a disk (radius 0.12 min(H, W), a flat
    surface at depth 1.2 with its own albedo) moves over it by ``obj_vel``
    pixels per frame.  Each frame has fresh noise and, besides the keys of
    ``make_frame``, ``wpos`` [H,W,3] (world position: scene x and y in units
    of 1000 pixels, depth / 100) and ``motion`` [H,W,2] (offset in pixels from a
    pixel to where its surface point was in the previous frame: ``pan`` on
    the background, ``pan - obj_vel`` on the disk; zero in frame 0).  Where
    the disk uncovers background, the previous frame showed the disk there
    and the world positions disagree.
    """
    rng = np.random.default_rng(seed)
    A = rng.uniform(0.02, 0.12, size=8)
    fx = rng.uniform(-12.0, 12.0, size=8)
    fy = rng.uniform(-12.0, 12.0, size=8)
    ph = rng.uniform(0.0, 2 * np.pi, size=8)
    tint = rng.uniform(0.8, 1.2, size=3)
    sites = rng.uniform(0.0, 1.0, size=(12, 2))
    colours = rng.uniform(0.1, 0.9, size=(12, 3))
    B = rng.uniform(0.005, 0.02, size=4)
    g = rng.uniform(-6.0, 6.0, size=(4, 2))
    psi = rng.uniform(0.0, 2 * np.pi, size=4)
    s1, s2 = rng.uniform(1.0, 4.0, size=2)
    t1, t2 = rng.uniform(0.0, 2 * np.pi, size=2)
    obj_albedo = np.array([0.8, 0.35, 0.2])
    rad = 0.12 * min(H, W)
    c0 = np.array([0.3 * W, 0.4 * H])
    xs, ys = np.meshgrid(np.arange(W, dtype=np.float64) + 0.5, np.arange(H, dtype=np.float64) + 0.5)
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    frames = []
    for t in range(T):
        # background: the scene at pixel coordinates shifted by the pan
        px, py = xs + t * pan[0], ys + t * pan[1]
        u, v = px / W, py / H
        E = np.full((H, W), 0.25)
        for j in range(8):
            E += A[j] * (1.0 + np.sin(2 * np.pi * (fx[j] * u + fy[j] * v) + ph[j]))
        best = np.full((H, W), np.inf)
        label = np.zeros((H, W), dtype=np.int64)
        for k in range(12):
            dist = (px - sites[k, 0] * W) ** 2 + (py - sites[k, 1] * H) ** 2
            closer = dist < best
            best = np.where(closer, dist, best)
            label = np.where(closer, k, label)
        albedo = colours[label]
        hx = np.zeros((H, W))
        hy = np.zeros((H, W))
        for j in range(4):
            arg = 2 * np.pi * (g[j, 0] * u + g[j, 1] * v) + psi[j]
            hx += B[j] * np.cos(arg) * 2 * np.pi * g[j, 0]
            hy += B[j] * np.cos(arg) * 2 * np.pi * g[j, 1]
        nrm = np.stack([-hx, -hy, np.ones_like(hx)], axis=-1)
        nrm /= np.linalg.norm(nrm, axis=-1, keepdims=True)
        dd = 0.5 + 0.25 * (np.sin(2 * np.pi * u * s1 + t1) + np.sin(2 * np.pi * v * s2 + t2))
        depth = 1.0 + 9.0 * np.clip(dd, 0.0, 1.0)
        wpos = np.stack([px / 1000.0, py / 1000.0, depth / 100.0], axis=-1)
        motion = np.broadcast_to(np.array(pan, dtype=np.float64), (H, W, 2)).copy()
        # the moving disk (screen space)
        cx, cy = c0[0] + t * obj_vel[0], c0[1] + t * obj_vel[1]
        inside = (xs - cx) ** 2 + (ys - cy) ** 2 <= rad * rad
        E = np.where(inside, 0.6, E)
        albedo = np.where(inside[..., None], obj_albedo[None, None, :], albedo)
        nrm = np.where(inside[..., None], np.array([0.0, 0.0, 1.0])[None, None, :], nrm)
        depth = np.where(inside, 1.2, depth)
        obj_w = np.stack([(xs - cx + c0[0] + t * obj_vel[0]) / 1000.0,
                          (ys - cy + c0[1] + t * obj_vel[1]) / 1000.0, np.full((H, W), 0.012)], axis=-1)
        wpos = np.where(inside[..., None], obj_w, wpos)
        motion = np.where(inside[..., None], np.array([pan[0] - obj_vel[0], pan[1] - obj_vel[1]]), motion)
        if t == 0:
            motion = np.zeros_like(motion)
        clean = albedo * tint[None, None, :] * E[..., None]
        G = rng.gamma(0.5, 2.0, size=(H, W, 3))
        fire = rng.random(size=(H, W)) < 1e-3
        G = G * np.where(fire, 50.0, 1.0)[..., None]
        frames.append({"radiance": f32(clean * G), "albedo": f32(albedo), "normal": f32(nrm),
                       "depth": f32(depth[..., None]), "clean": f32(clean), "wpos": f32(wpos),
                       "motion": f32(motion)})
    return frames


def make_frame_batch(seeds, H: int, W: int) -> Dict[str, np.ndarray]:
    """Stack frames of one size along a leading batch axis."""
    frames = [make_frame(s, H, W) for s in seeds]
    return {k: np.stack([f[k] for f in frames]) for k in frames[0]}


def make_head(seed: int, N: int, H: int, W: int, M: int, spread: float = 1.0) -> np.ndarray:
    """A random head record [N,H,W,2M] for decode-only tests.

    Channels 0..M-1 are positive weights (log-normal, width ``spread``),
    channels M..2M-1 are fusion logits ~ N(0, 1).
    """
    rng = np.random.default_rng(seed)
    Wm = np.exp(rng.normal(0.0, spread, size=(N, H, W, M)))
    lg = rng.normal(0.0, 1.0, size=(N, H, W, M))
    return np.ascontiguousarray(np.concatenate([Wm, lg], axis=-1), dtype=np.float32)
