"""Python binding of the C ABI, one function per entry point with the same name.

torch supplies device memory and the current stream; every step of the
rasterizer and the optimizer runs in the HIP kernels of libfastergs.so.
Parameter tensors use the library's structure-of-arrays layout:

    means [3, N], log_scales [3, N], quats [4, N], opacity_logits [N],
    sh_dc [3, N], sh_rest [45, N]   (float32, contiguous, on the GPU)
"""
from __future__ import annotations

import ctypes
from typing import Dict, Iterable, Optional, Sequence, Tuple

import numpy as np
import torch

from . import _lib as L

PARAM_SHAPES = {"means": 3, "log_scales": 3, "quats": 4, "opacity_logits": 0, "sh_dc": 3, "sh_rest": 45}
PARAM_NAMES = tuple(PARAM_SHAPES)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _check_tensor(t: torch.Tensor, name: str, dtype=torch.float32, shape=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


def make_camera(cam) -> L.Camera:
    """ctypes camera from any object with world_to_cam, fx, fy, cx, cy, width, height, near, bg."""
    c = L.Camera()
    w = np.asarray(cam.world_to_cam, dtype=np.float32).reshape(16)
    for k in range(16):
        c.world_to_cam[k] = float(w[k])
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    c.near_z = float(getattr(cam, "near", 0.2))
    bg = getattr(cam, "bg", (0.0, 0.0, 0.0))
    for k in range(3):
        c.bg[k] = float(bg[k])
    return c


def default_settings(**overrides) -> L.Settings:
    s = L.Settings()
    L.check(L.load().fgs_default_settings(ctypes.byref(s)), "fgs_default_settings")
    for k, v in overrides.items():
        setattr(s, k, v)
    return s


def gaussians_struct(params: Dict[str, torch.Tensor], sh_degree: int = 3) -> L.Gaussians:
    n = int(params["opacity_logits"].shape[0])
    for name, rows in PARAM_SHAPES.items():
        _check_tensor(params[name], name, shape=(n,) if rows == 0 else (rows, n))
    g = L.Gaussians()
    g.n = n
    g.means, g.log_scales, g.quats = (_ptr(params[k]) for k in ("means", "log_scales", "quats"))
    g.opacity_logits, g.sh_dc, g.sh_rest = (_ptr(params[k]) for k in ("opacity_logits", "sh_dc", "sh_rest"))
    g.sh_dtype = L.FGS_F32
    g.sh_degree = int(sh_degree)
    return g


def workspace_size(n: int, camera, settings: Optional[L.Settings] = None, instance_capacity: int = 0) -> int:
    st = settings or default_settings()
    out = ctypes.c_size_t()
    L.check(L.load().fgs_workspace_size(int(n), ctypes.byref(make_camera(camera)), ctypes.byref(st),
                                        int(instance_capacity), ctypes.byref(out)), "fgs_workspace_size")
    return int(out.value)


def workspace_layout(n: int, camera, settings: Optional[L.Settings] = None, instance_capacity: int = 0) -> L.Layout:
    st = settings or default_settings()
    out = L.Layout()
    L.check(L.load().fgs_workspace_layout(int(n), ctypes.byref(make_camera(camera)), ctypes.byref(st),
                                          int(instance_capacity), ctypes.byref(out)), "fgs_workspace_layout")
    return out


def rasterize_forward(params: Dict[str, torch.Tensor], camera, settings: Optional[L.Settings],
                      workspace: torch.Tensor, instance_capacity: int, image: torch.Tensor,
                      t_final: Optional[torch.Tensor], last: torch.Tensor, *, sh_degree: int = 3,
                      stream=None, raise_on_capacity: bool = True) -> Dict[str, int]:
    """fgs_rasterize_forward.  Returns the forward statistics; on an instance
    capacity overflow raises (or, with raise_on_capacity=False, returns the
    statistics with "status" = FGS_ERR_CAPACITY)."""
    st = settings or default_settings()
    cam = make_camera(camera)
    g = gaussians_struct(params, sh_degree)
    h, w = cam.height, cam.width
    _check_tensor(image, "image", shape=(3, h, w))
    _check_tensor(last, "last", dtype=torch.int32, shape=(h, w))
    if t_final is not None:
        _check_tensor(t_final, "t_final", shape=(h, w))
    _check_tensor(workspace, "workspace", dtype=torch.uint8)
    stats = L.ForwardStats()
    status = L.load().fgs_rasterize_forward(
        ctypes.byref(g), ctypes.byref(cam), ctypes.byref(st), _ptr(workspace), workspace.numel(),
        int(instance_capacity), _ptr(image), _ptr(t_final), _ptr(last), ctypes.byref(stats),
        _stream_handle(stream))
    out = {"status": int(status), "n_visible": int(stats.n_visible), "n_instances": int(stats.n_instances),
           "tiles_x": int(stats.tiles_x), "tiles_y": int(stats.tiles_y)}
    if status == L.FGS_ERR_CAPACITY and not raise_on_capacity:
        return out
    L.check(status, "fgs_rasterize_forward")
    return out


def rasterize_backward(params: Dict[str, torch.Tensor], camera, settings: Optional[L.Settings],
                       workspace: torch.Tensor, instance_capacity: int, image: torch.Tensor, last: torch.Tensor,
                       dl_dimage: torch.Tensor, grads: Dict[str, torch.Tensor], *, sh_degree: int = 3,
                       stream=None) -> None:
    """fgs_rasterize_backward: fills every tensor of ``grads`` (same shapes as params)."""
    st = settings or default_settings()
    cam = make_camera(camera)
    g = gaussians_struct(params, sh_degree)
    n = g.n
    h, w = cam.height, cam.width
    _check_tensor(image, "image", shape=(3, h, w))
    _check_tensor(dl_dimage, "dl_dimage", shape=(3, h, w))
    _check_tensor(last, "last", dtype=torch.int32, shape=(h, w))
    _check_tensor(workspace, "workspace", dtype=torch.uint8)
    for name, rows in PARAM_SHAPES.items():
        _check_tensor(grads[name], f"grads[{name}]", shape=(n,) if rows == 0 else (rows, n))
    gr = L.GaussianGrads()
    for name in PARAM_NAMES:
        setattr(gr, name, _ptr(grads[name]))
    L.check(L.load().fgs_rasterize_backward(
        ctypes.byref(g), ctypes.byref(cam), ctypes.byref(st), _ptr(workspace), workspace.numel(),
        int(instance_capacity), _ptr(image), _ptr(last), _ptr(dl_dimage), ctypes.byref(gr),
        _stream_handle(stream)), "fgs_rasterize_backward")


def adam_step(groups: Sequence[Tuple[torch.Tensor, torch.Tensor, torch.Tensor, torch.Tensor, float]], step: int,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-15, *, stream=None) -> None:
    """fgs_adam_step over groups of (param, grad, exp_avg, exp_avg_sq, lr), updated in place."""
    arr = (L.AdamGroup * len(groups))()
    for k, (p, g, m, v, lr) in enumerate(groups):
        for t, nm in ((p, "param"), (g, "grad"), (m, "exp_avg"), (v, "exp_avg_sq")):
            _check_tensor(t, nm, shape=p.shape)
        arr[k].param, arr[k].grad, arr[k].exp_avg, arr[k].exp_avg_sq = _ptr(p), _ptr(g), _ptr(m), _ptr(v)
        arr[k].numel = p.numel()
        arr[k].lr = float(lr)
        arr[k].dtype = L.FGS_F32
    L.check(L.load().fgs_adam_step(arr, len(groups), int(step), float(beta1), float(beta2), float(eps),
                                   _stream_handle(stream)), "fgs_adam_step")


def l1_loss_backward(image: torch.Tensor, target: torch.Tensor, dl_dimage: torch.Tensor,
                     loss: Optional[torch.Tensor] = None, *, stream=None) -> None:
    """fgs_l1_loss_backward: dl_dimage = sign(image - target) / numel; loss (float64[1]) = mean |.|."""
    _check_tensor(image, "image")
    _check_tensor(target, "target", shape=image.shape)
    _check_tensor(dl_dimage, "dl_dimage", shape=image.shape)
    if loss is not None:
        _check_tensor(loss, "loss", dtype=torch.float64, shape=(1,))
    L.check(L.load().fgs_l1_loss_backward(_ptr(image), _ptr(target), image.numel(), _ptr(dl_dimage), _ptr(loss),
                                          _stream_handle(stream)), "fgs_l1_loss_backward")


class Rasterizer:
    """Owns a workspace for one camera and grows it when the instance count
    exceeds its capacity.  forward() and backward() call the C ABI."""

    def __init__(self, camera, settings: Optional[L.Settings] = None, sh_degree: int = 3,
                 device: Optional[torch.device] = None, headroom: float = 1.25):
        self.camera = camera
        self.settings = settings or default_settings()
        self.sh_degree = sh_degree
        self.device = device or torch.device("cuda", torch.cuda.current_device())
        self.headroom = headroom
        self.capacity = 0
        self.n = -1
        self.workspace: Optional[torch.Tensor] = None
        self.last_stats: Dict[str, int] = {}

    def _ensure(self, n: int, capacity: int) -> None:
        if self.workspace is not None and n == self.n and capacity <= self.capacity:
            return
        capacity = max(capacity, self.capacity if n == self.n else 0)
        size = workspace_size(n, self.camera, self.settings, capacity)
        self.workspace = torch.empty(size, dtype=torch.uint8, device=self.device)
        self.capacity, self.n = capacity, n

    def layout(self) -> L.Layout:
        return workspace_layout(self.n, self.camera, self.settings, self.capacity)

    def forward(self, params: Dict[str, torch.Tensor], image: Optional[torch.Tensor] = None,
                t_final: Optional[torch.Tensor] = None, last: Optional[torch.Tensor] = None, stream=None):
        n = int(params["opacity_logits"].shape[0])
        h, w = int(self.camera.height), int(self.camera.width)
        if image is None:
            image = torch.empty(3, h, w, dtype=torch.float32, device=self.device)
        if last is None:
            last = torch.empty(h, w, dtype=torch.int32, device=self.device)
        if t_final is None:
            t_final = torch.empty(h, w, dtype=torch.float32, device=self.device)
        self._ensure(n, max(self.capacity, 1024) if n == self.n else max(1024, 16 * n))
        for _ in range(3):
            st = rasterize_forward(params, self.camera, self.settings, self.workspace, self.capacity, image,
                                   t_final, last, sh_degree=self.sh_degree, stream=stream, raise_on_capacity=False)
            if st["status"] == L.FGS_OK:
                self.last_stats = st
                return image, t_final, last
            self._ensure(n, int(st["n_instances"] * self.headroom) + 1024)
        raise RuntimeError("instance capacity could not be satisfied")

    def backward(self, params: Dict[str, torch.Tensor], image: torch.Tensor, last: torch.Tensor,
                 dl_dimage: torch.Tensor, grads: Optional[Dict[str, torch.Tensor]] = None, stream=None):
        if grads is None:
            grads = {k: torch.empty_like(v) for k, v in params.items()}
        rasterize_backward(params, self.camera, self.settings, self.workspace, self.capacity, image, last,
                           dl_dimage.contiguous(), grads, sh_degree=self.sh_degree, stream=stream)
        return grads

    # -- views of the workspace (for inspection and tests)
    def view(self, field: str, count: int, dtype=torch.int32, index: Optional[int] = None) -> torch.Tensor:
        lay = self.layout()
        off = getattr(lay, field)
        if index is not None:
            off = off[index]
        itemsize = torch.empty(0, dtype=dtype).element_size()
        return self.workspace[off:off + count * itemsize].view(dtype)


def exported_symbols() -> Iterable[str]:
    return tuple(L.SIGNATURES)
