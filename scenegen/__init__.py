"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This module only draws random numbers and builds cameras; it holds none of the
rasterizer's arithmetic.  Every array is float32 (or uint16 bfloat16 bits) and
C-contiguous, laid out the way the C-ABI library expects:

  means   [N,3]   world-space centres
  scales  [N,3]   activated (positive) per-axis standard deviations
  quats   [N,4]   unit quaternion (w, x, y, z)
  opacity [N]     activated opacity in (0, 1)
  sh      [N,B,3] real spherical-harmonic coefficients, B = (L+1)^2
  feat    [N,D]   per-Gaussian semantic feature (frozen, never differentiated)

The distributions follow the synthetic workloads of the benchmark suite:
means uniform in a cube, log-scales normal around -3, uniformly random
rotations, opacity = sigmoid of a standard normal, a DC colour that is uniform
in [0, 1] (drawn directly as its SH coefficient, uniform in [-sqrt(pi),
sqrt(pi)]), small normal higher-order SH coefficients and standard-normal
features.  They stand in for the COLMAP-initialised scenes and SAM feature maps
the paper trains on (Section 4), which are not available here.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Camera",
    "Workload",
    "WORKLOADS",
    "make_gaussians",
    "make_cameras",
    "make_view_tensors",
    "make_view_tensors_device",
    "look_at_camera",
    "to_bf16_bits",
    "bf16_bits_to_f32",
]


@dataclasses.dataclass
class Camera:
    """Pinhole camera, OpenCV axes (x right, y down, z forward).

    R is the 3x3 world-to-camera rotation (row-major float32), t the
    translation, so that p_cam = R @ p_world + t.
    """

    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray
    t: np.ndarray

    @property
    def npix(self) -> int:
        return self.width * self.height


@dataclasses.dataclass
class Workload:
    name: str
    n: int                 # Gaussians
    half_extent: float     # means ~ U[-h, h]^3
    sh_degree: int
    d: int                 # feature channels
    feat_dtype: str        # "f32" or "bf16"
    views: str             # camera recipe: "front128", "front800", "front1080", "sphere16", "sphere8_1080"
    fusion: bool           # does the workload include feature fusion
    description: str


WORKLOADS = {
    "c1": Workload("c1", 1_000, 1.0, 0, 16, "f32", "front128", False,
                   "1k Gaussians, SH0, D=16 fp32, one 128x128 view"),
    "c2": Workload("c2", 200_000, 3.0, 3, 64, "f32", "front800", False,
                   "200k Gaussians, SH3, D=64 fp32, one 800x800 view"),
    "c3": Workload("c3", 500_000, 3.0, 3, 256, "bf16", "front1080", True,
                   "500k Gaussians, SH3, D=256 bf16 features, one 1920x1080 view, fwd+bwd+fusion"),
    "c4": Workload("c4", 1_000_000, 3.0, 3, 128, "bf16", "sphere16", True,
                   "1M Gaussians, SH3, D=128 bf16, 16 views 640x480..1600x1200, fwd+bwd+fusion"),
    "c5": Workload("c5", 3_000_000, 3.0, 3, 512, "bf16", "sphere8_1080", True,
                   "3M Gaussians, SH3, D=512 bf16, 8 views 1920x1080, fwd+bwd+fusion"),
}


def to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """Round float32 to bfloat16 (round to nearest, ties to even); returns uint16 bits."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16).astype(np.uint16)
    nan = np.isnan(x)
    if nan.any():
        r[nan] = 0x7FC0
    return r


def bf16_bits_to_f32(b: np.ndarray) -> np.ndarray:
    """Exact widening of bfloat16 bits to float32."""
    b = np.ascontiguousarray(b, dtype=np.uint16)
    return (b.astype(np.uint32) << 16).view(np.float32)


def make_gaussians(n: int, half_extent: float, sh_degree: int, d: int, seed: int = 0,
                   feat_dtype: str = "f32") -> dict:
    """Draw n Gaussians with default_rng(seed), in a fixed draw order."""
    rng = np.random.default_rng(seed)
    nb = (sh_degree + 1) ** 2
    means = rng.uniform(-half_extent, half_extent, size=(n, 3)).astype(np.float32)
    scales = np.exp(rng.normal(-3.0, 0.5, size=(n, 3))).astype(np.float32)
    q = rng.normal(0.0, 1.0, size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    quats = q.astype(np.float32)
    opacity = (1.0 / (1.0 + np.exp(-rng.normal(0.0, 1.0, size=n)))).astype(np.float32)
    sh = np.zeros((n, nb, 3), dtype=np.float32)
    sh[:, 0, :] = rng.uniform(-math.sqrt(math.pi), math.sqrt(math.pi), size=(n, 3))
    if nb > 1:
        sh[:, 1:, :] = rng.normal(0.0, 0.1, size=(n, nb - 1, 3))
    feat = rng.standard_normal(size=(n, d), dtype=np.float32)
    out = dict(means=means, scales=scales, quats=quats, opacity=opacity, sh=sh,
               sh_degree=sh_degree, d=d, feat_dtype=feat_dtype)
    if feat_dtype == "bf16":
        bits = to_bf16_bits(feat)
        out["feat_bits"] = bits
        out["feat"] = bf16_bits_to_f32(bits)
    else:
        out["feat"] = feat
    return out


def look_at_camera(position, width: int, height: int, hfov_deg: float = 60.0) -> Camera:
    """Camera at `position` looking at the world origin, world up +z (fallback +y)."""
    c = np.asarray(position, dtype=np.float64)
    f = -c / np.linalg.norm(c)
    up = np.array([0.0, 0.0, 1.0])
    if abs(float(f @ up)) > 0.99:
        up = np.array([0.0, 1.0, 0.0])
    right = np.cross(f, up)
    right /= np.linalg.norm(right)
    down = np.cross(f, right)
    R = np.stack([right, down, f]).astype(np.float32)
    t = (-(R.astype(np.float64) @ c)).astype(np.float32)
    fx = (width / 2.0) / math.tan(math.radians(hfov_deg) / 2.0)
    return Camera(width=width, height=height, fx=float(np.float32(fx)), fy=float(np.float32(fx)),
                  cx=width / 2.0, cy=height / 2.0, R=R, t=t)


def make_cameras(recipe: str, seed: int = 1) -> list:
    rng = np.random.default_rng(seed)
    if recipe == "front128":
        return [look_at_camera((0.0, -4.0, 0.0), 128, 128)]
    if recipe == "front800":
        return [look_at_camera((0.0, -4.0, 0.0), 800, 800)]
    if recipe == "front1080":
        return [look_at_camera((0.0, -4.0, 0.0), 1920, 1080)]
    if recipe == "sphere16":
        ws = rng.integers(640, 1601, size=16)
        dirs = rng.normal(size=(16, 3))
        dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
        return [look_at_camera(5.0 * dirs[i], int(ws[i]), int(round(3 * int(ws[i]) / 4)))
                for i in range(16)]
    if recipe == "sphere8_1080":
        dirs = rng.normal(size=(8, 3))
        dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
        return [look_at_camera(5.0 * dirs[i], 1920, 1080) for i in range(8)]
    if recipe.startswith("front"):
        # "frontWxH": one camera at distance 4, used for small test scenes
        wh = recipe[len("front"):]
        w, h = (int(s) for s in wh.split("x"))
        return [look_at_camera((0.0, -4.0, 0.0), w, h)]
    raise ValueError(f"unknown camera recipe {recipe!r}")


def make_view_tensors(view_index: int, npix: int, d: int, with_dT: bool = False,
                      target_dtype: str = "f32") -> dict:
    """Upstream gradients and the fusion target map for one view (default_rng(100+v))."""
    rng = np.random.default_rng(100 + view_index)
    dC = rng.standard_normal(size=(npix, 3), dtype=np.float32)
    dF = rng.standard_normal(size=(npix, d), dtype=np.float32)
    dT_draw = rng.standard_normal(size=npix, dtype=np.float32)
    dT = dT_draw if with_dT else np.zeros(npix, dtype=np.float32)
    target = rng.standard_normal(size=(npix, d), dtype=np.float32)
    out = dict(dC=dC, dF=dF, dT=dT, target=target)
    if target_dtype == "bf16":
        bits = to_bf16_bits(target)
        out["target_bits"] = bits
        out["target"] = bf16_bits_to_f32(bits)
    return out


def make_view_tensors_device(view_index: int, npix: int, d: int, device, with_dT: bool = False,
                             target_dtype: str = "f32") -> dict:
    """The per-view maps of make_view_tensors' distributions, drawn on the device
    with torch's seeded generator (seed 100 + v) for workloads whose maps are too
    large to draw on the host.  dC, dF, dT, target ~ N(0, 1) in float32; a BF16
    target is the round-to-nearest-even of the float32 draw.  Consumers that
    need values on the host copy the rows they use."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(100 + view_index)
    f32 = torch.float32
    dC = torch.randn((npix, 3), generator=gen, device=device, dtype=f32)
    dF = torch.randn((npix, d), generator=gen, device=device, dtype=f32)
    dT_draw = torch.randn((npix,), generator=gen, device=device, dtype=f32)
    dT = dT_draw if with_dT else torch.zeros_like(dT_draw)
    target = torch.randn((npix, d), generator=gen, device=device, dtype=f32)
    if target_dtype == "bf16":
        target = target.to(torch.bfloat16)
    return dict(dC=dC, dF=dF, dT=dT, target=target)
