"""Seeded synthetic inputs shaped like the 3DGS training workloads.

This module only draws random inputs and builds cameras; it holds none of the
rasterizer's arithmetic.  Both the CPU oracle (via the tests) and the HIP path
consume exactly the float32 tensors produced here.

Layout (structure of arrays, float32, CPU tensors):
    means           [3, N]   camera-frame x, y ~ U[-1, 1], z ~ U[2, 6]
    log_scales      [3, N]   N(-4, 0.5)
    quats           [4, N]   (w, x, y, z), normalised draws of N(0, I4)
    opacity_logits  [N]      N(0, 1)
    sh_dc           [3, N]   N(0, 0.3), plane c = colour channel
    sh_rest         [45, N]  N(0, 0.05), plane (k-1)*3 + c for SH index k = 1..15

"N(a, b)" means mean a and standard deviation b.  Values are drawn in float64
from a seeded ``torch.Generator`` in the fixed order above and then rounded to
float32.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, Optional, Tuple

import numpy as np
import torch

SH_REST_PLANES = 45
PARAM_NAMES = ("means", "log_scales", "quats", "opacity_logits", "sh_dc", "sh_rest")


@dataclasses.dataclass
class Camera:
    """Pinhole camera: world_to_cam is the 4x4 row-major matrix W of Eq. (1)."""

    world_to_cam: np.ndarray  # float32 [4, 4]
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    near: float = 0.2
    bg: Tuple[float, float, float] = (0.0, 0.0, 0.0)

    def copy(self, **kw) -> "Camera":
        d = dataclasses.asdict(self)
        d["world_to_cam"] = self.world_to_cam.copy()
        d.update(kw)
        return Camera(**d)


@dataclasses.dataclass
class Workload:
    name: str
    n: int
    width: int
    height: int
    focal: float
    description: str


# The workloads the parity tests and the benchmark use (sizes from the paper's
# problem shapes: a small single view, a 720p training step and a 3M-Gaussian
# 1600x1060 training step).
WORKLOADS: Dict[str, Workload] = {
    "c1": Workload("c1", 10_000, 256, 256, 256.0,
                   "plain single-view fwd+bwd, 10k Gaussians, 256x256, fx=fy=256"),
    "c2": Workload("c2", 500_000, 1280, 720, 1000.0,
                   "full training step, 500k Gaussians, 1280x720, fx=fy=1000, L1 + Adam"),
    "c3": Workload("c3", 3_000_000, 1600, 1060, 1200.0,
                   "full training step, 3M Gaussians, 1600x1060, fx=fy=1200, L1 + Adam"),
}

# Adam learning rates per parameter group for the full-step workloads.
ADAM_LR = {
    "means": 1.6e-4,
    "sh_dc": 5e-3,
    "sh_rest": 5e-3,
    "log_scales": 5e-3,
    "quats": 1e-3,
    "opacity_logits": 2.5e-2,
}


def identity_camera(width: int, height: int, focal: float, *, bg=(0.0, 0.0, 0.0),
                    near: float = 0.2, cx: Optional[float] = None,
                    cy: Optional[float] = None) -> Camera:
    return Camera(np.eye(4, dtype=np.float32), float(focal), float(focal),
                  float(width) / 2 if cx is None else float(cx),
                  float(height) / 2 if cy is None else float(cy),
                  int(width), int(height), float(near), tuple(float(b) for b in bg))


def look_at_camera(eye, target, width: int, height: int, focal: float,
                   up=(0.0, 1.0, 0.0), bg=(0.0, 0.0, 0.0)) -> Camera:
    """World-to-camera matrix for a camera at ``eye`` looking at ``target``
    (camera +z forward, +x right, +y down in the image)."""
    eye = np.asarray(eye, np.float64)
    fwd = np.asarray(target, np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    upv = np.asarray(up, np.float64)
    if abs(float(np.dot(fwd, upv))) > 0.999:
        upv = np.array([1.0, 0.0, 0.0])
    right = np.cross(upv, fwd)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    rot = np.stack([right, down, fwd])  # rows: camera axes in world coords
    m = np.eye(4)
    m[:3, :3] = rot
    m[:3, 3] = -rot @ eye
    return Camera(m.astype(np.float32), float(focal), float(focal), width / 2.0,
                  height / 2.0, int(width), int(height), 0.2, tuple(bg))


def make_scene(n: int, seed: int = 0, *, z_range=(2.0, 6.0), xy_range=(-1.0, 1.0),
               log_scale_mean: float = -4.0, log_scale_std: float = 0.5,
               dc_std: float = 0.3, rest_std: float = 0.05) -> Dict[str, torch.Tensor]:
    """Draw ``n`` Gaussians (see the module docstring for the recipe)."""
    g = torch.Generator(device="cpu")
    g.manual_seed(int(seed))
    f64 = torch.float64
    lo, hi = xy_range
    means = torch.empty(3, n, dtype=f64)
    means[0:2] = torch.rand(2, n, generator=g, dtype=f64) * (hi - lo) + lo
    means[2] = torch.rand(n, generator=g, dtype=f64) * (z_range[1] - z_range[0]) + z_range[0]
    log_scales = torch.randn(3, n, generator=g, dtype=f64) * log_scale_std + log_scale_mean
    q = torch.randn(4, n, generator=g, dtype=f64)
    q = q / q.norm(dim=0, keepdim=True).clamp_min(1e-30)
    logits = torch.randn(n, generator=g, dtype=f64)
    sh_dc = torch.randn(3, n, generator=g, dtype=f64) * dc_std
    sh_rest = torch.empty(SH_REST_PLANES, n, dtype=f64)
    for k in range(0, SH_REST_PLANES, 9):  # plane groups bound peak memory at 3M
        sh_rest[k:k + 9] = torch.randn(9, n, generator=g, dtype=f64) * rest_std
    out = {
        "means": means, "log_scales": log_scales, "quats": q,
        "opacity_logits": logits, "sh_dc": sh_dc, "sh_rest": sh_rest,
    }
    return {k: v.to(torch.float32).contiguous() for k, v in out.items()}


def workload_camera(name: str, bg=(0.0, 0.0, 0.0)) -> Camera:
    w = WORKLOADS[name]
    return identity_camera(w.width, w.height, w.focal, bg=bg)


def make_dl_dimage(height: int, width: int, seed: int = 0) -> torch.Tensor:
    """Upstream gradient dL/dC ~ N(0, 1) per pixel and channel, [3, H, W] float32."""
    g = torch.Generator(device="cpu")
    g.manual_seed(int(seed) + 1_000_003)
    return torch.randn(3, height, width, generator=g, dtype=torch.float64).to(torch.float32)


def make_target(height: int, width: int, seed: int = 0) -> torch.Tensor:
    """L1 target image ~ U[0, 1] per pixel and channel, [3, H, W] float32."""
    g = torch.Generator(device="cpu")
    g.manual_seed(int(seed) + 2_000_003)
    return torch.rand(3, height, width, generator=g, dtype=torch.float64).to(torch.float32)


def uniform_sphere_cameras(n_views: int, seed: int, radius: float = 5.0,
                           w_range=(640, 1920), h_range=(480, 1080)):
    """Cameras on a sphere around the origin with seeded uneven resolutions."""
    g = torch.Generator(device="cpu")
    g.manual_seed(int(seed) + 3_000_003)
    cams = []
    for _ in range(n_views):
        v = torch.randn(3, generator=g, dtype=torch.float64)
        v = (v / v.norm()).numpy() * radius
        w = int(torch.randint(w_range[0], w_range[1] + 1, (1,), generator=g))
        h = int(torch.randint(h_range[0], h_range[1] + 1, (1,), generator=g))
        cams.append(look_at_camera(v, (0.0, 0.0, 0.0), w, h, float(w)))
    return cams


def make_motion(n: int, seed: int = 0, v_std: float = 0.1, a_std: float = 0.02) -> Dict[str, torch.Tensor]:
    """Per-Gaussian velocity ~ N(0, v_std) and acceleration ~ N(0, a_std),
    float32 [3, n] each (the dynamic workload's motion model)."""
    g = torch.Generator(device="cpu")
    g.manual_seed(int(seed) + 4_000_003)
    vel = torch.randn(3, n, generator=g, dtype=torch.float64) * v_std
    acc = torch.randn(3, n, generator=g, dtype=torch.float64) * a_std
    return {"velocity": vel.to(torch.float32).contiguous(), "accel": acc.to(torch.float32).contiguous()}


def make_cond4d(scene: Dict[str, torch.Tensor], seed: int = 0, t_range=(0.0, 1.0), log_scale_t_mean: float = -1.0,
                log_scale_t_std: float = 0.3, mix: float = 0.3) -> Dict[str, torch.Tensor]:
    """Extra planes of conditional 4D Gaussians for a scene: time of the mean
    ~ U[t_range], temporal log-scale ~ N(mean, std), and a right quaternion
    equal to the conjugate of the scene's (left) quaternion plus N(0, mix)
    noise per component, so that space and time mix a little (a pure
    conjugate would leave time unmixed).  float32: mean_t [n], log_scale_t
    [n], quats_r [4][n]."""
    n = count(scene)
    g = torch.Generator(device="cpu")
    g.manual_seed(int(seed) + 6_000_003)
    f64 = torch.float64
    lo, hi = t_range
    mean_t = torch.rand(n, generator=g, dtype=f64) * (hi - lo) + lo
    log_st = torch.randn(n, generator=g, dtype=f64) * log_scale_t_std + log_scale_t_mean
    conj = scene["quats"].to(f64) * torch.tensor([1.0, -1.0, -1.0, -1.0], dtype=f64)[:, None]
    quats_r = conj + torch.randn(4, n, generator=g, dtype=f64) * mix
    return {"mean_t": mean_t.to(torch.float32), "log_scale_t": log_st.to(torch.float32),
            "quats_r": quats_r.to(torch.float32).contiguous()}


def timesteps(count: int):
    """t_k = k / (count - 1), k = 0 .. count-1 (times in [0, 1])."""
    return [k / (count - 1) if count > 1 else 0.0 for k in range(count)]


def make_adam_state(shapes: Dict[str, Tuple[int, ...]], scales: Dict[str, float],
                    seed: int = 0) -> Tuple[Dict[str, torch.Tensor], Dict[str, torch.Tensor]]:
    """Seeded Adam moments for a step that does not start from zero: per group
    g, exp_avg ~ N(0, (scales[g] / 2)^2) and exp_avg_sq = scales[g]^2 (1/2 + U[0, 1]),
    float32 tensors of shapes[g]."""
    g = torch.Generator(device="cpu")
    g.manual_seed(int(seed) + 5_000_003)
    m, v = {}, {}
    for k in sorted(shapes):
        sh, sc = tuple(shapes[k]), float(scales[k])
        m[k] = (torch.randn(sh, generator=g, dtype=torch.float64) * (0.5 * sc)).to(torch.float32)
        v[k] = ((torch.rand(sh, generator=g, dtype=torch.float64) + 0.5) * sc * sc).to(torch.float32)
    return m, v


def batch_scene(n: int, seed: int = 0) -> Dict[str, torch.Tensor]:
    """The multi-view workload's scene: the usual draws with means recentred to
    x, y in [-1, 1], z in [-2, 2] around the origin the cameras look at."""
    return make_scene(n, seed, z_range=(-2.0, 2.0))


def subset(scene: Dict[str, torch.Tensor], idx) -> Dict[str, torch.Tensor]:
    """Gaussians ``idx`` of a scene (same SoA layout)."""
    return {k: (v[..., idx] if v.dim() > 1 else v[idx]).contiguous() for k, v in scene.items()}


def count(scene: Dict[str, torch.Tensor]) -> int:
    return int(scene["opacity_logits"].shape[0])


def bytes_per_gaussian() -> int:
    return 4 * (3 + 3 + 4 + 1 + 3 + SH_REST_PLANES)


def scene_checksum(scene: Dict[str, torch.Tensor]) -> float:
    return float(sum(float(v.double().sum()) for v in scene.values()))


__all__ = [
    "Camera", "Workload", "WORKLOADS", "ADAM_LR", "PARAM_NAMES", "identity_camera",
    "look_at_camera", "make_scene", "workload_camera", "make_dl_dimage", "make_target",
    "uniform_sphere_cameras", "subset", "count", "bytes_per_gaussian", "scene_checksum", "make_motion",
    "timesteps", "batch_scene", "make_adam_state", "make_cond4d",
]
