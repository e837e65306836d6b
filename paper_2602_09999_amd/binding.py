"""Python binding of the C ABI, one function per entry point with the same name.

torch supplies device memory and the current stream; every step of the
rasterizer and the optimizer runs in the HIP kernels of libfastergs.so.
Parameter tensors use the library's structure-of-arrays layout:

    means [3, N], log_scales [3, N], quats [4, N], opacity_logits [N],
    sh_dc [3, N], sh_rest [45, N]   (contiguous, on the GPU)

All planes are float32, except that sh_dc and sh_rest may both be bfloat16
(the precision form); their gradients then are bfloat16 too.
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


SH_NAMES = ("sh_dc", "sh_rest")


def sh_dtype_of(params: Dict[str, torch.Tensor]) -> torch.dtype:
    """torch.float32 or torch.bfloat16: the element type of both SH tensors."""
    dt = params["sh_dc"].dtype
    if dt not in (torch.float32, torch.bfloat16):
        raise TypeError(f"SH coefficients must be float32 or bfloat16, got {dt}")
    return dt


def param_dtype(name: str, sh_dtype: torch.dtype) -> torch.dtype:
    return sh_dtype if name in SH_NAMES else torch.float32


def gaussians_struct(params: Dict[str, torch.Tensor], sh_degree: int = 3) -> L.Gaussians:
    n = int(params["opacity_logits"].shape[0])
    shd = sh_dtype_of(params)
    for name, rows in PARAM_SHAPES.items():
        _check_tensor(params[name], name, dtype=param_dtype(name, shd), shape=(n,) if rows == 0 else (rows, n))
    g = L.Gaussians()
    g.n = n
    g.means, g.log_scales, g.quats = (_ptr(params[k]) for k in ("means", "log_scales", "quats"))
    g.opacity_logits, g.sh_dc, g.sh_rest = (_ptr(params[k]) for k in ("opacity_logits", "sh_dc", "sh_rest"))
    g.sh_dtype = L.FGS_BF16 if shd == torch.bfloat16 else L.FGS_F32
    g.sh_degree = int(sh_degree)
    if "velocity" in params or "accel" in params:
        for name in ("velocity", "accel"):
            _check_tensor(params[name], name, shape=(3, n))
        g.velocity, g.accel = _ptr(params["velocity"]), _ptr(params["accel"])
    if any(k in params for k in COND4D_NAMES):
        for name in COND4D_NAMES:
            _check_tensor(params[name], name, shape=(4, n) if name == "quats_r" else (n,))
        g.mean_t, g.log_scale_t, g.quats_r = (_ptr(params[k]) for k in COND4D_NAMES)
    return g


DYNAMIC_NAMES = ("velocity", "accel")
# conditional 4D Gaussians (Sec. 3.4): time of the mean, temporal log-scale,
# right-isoclinic quaternion (quats holds the left one)
COND4D_NAMES = ("mean_t", "log_scale_t", "quats_r")
COND4D_SHAPES = {"mean_t": 0, "log_scale_t": 0, "quats_r": 4}


def _camera_array(cameras: Sequence) -> "ctypes.Array":
    arr = (L.Camera * len(cameras))()
    for k, c in enumerate(cameras):
        arr[k] = make_camera(c)
    return arr


def _times_array(times: Optional[Sequence[float]], n_views: int):
    if times is None:
        return None
    if len(times) != n_views:
        raise ValueError(f"{len(times)} times for {n_views} views")
    return (ctypes.c_float * n_views)(*[float(t) for t in times])


def batch_workspace_size(n: int, cameras: Sequence, settings: Optional[L.Settings] = None,
                         instance_capacity: int = 0) -> int:
    st = settings or default_settings()
    out = ctypes.c_size_t()
    L.check(L.load().fgs_batch_workspace_size(int(n), _camera_array(cameras), len(cameras), ctypes.byref(st),
                                              int(instance_capacity), ctypes.byref(out)), "fgs_batch_workspace_size")
    return int(out.value)


def batch_workspace_layout(n: int, cameras: Sequence, settings: Optional[L.Settings] = None,
                           instance_capacity: int = 0) -> L.Layout:
    st = settings or default_settings()
    out = L.Layout()
    L.check(L.load().fgs_batch_workspace_layout(int(n), _camera_array(cameras), len(cameras), ctypes.byref(st),
                                                int(instance_capacity), ctypes.byref(out)),
            "fgs_batch_workspace_layout")
    return out


def view_pixels(cameras: Sequence) -> Tuple[int, ...]:
    return tuple(int(c.width) * int(c.height) for c in cameras)


def rasterize_forward_batch(params: Dict[str, torch.Tensor], cameras: Sequence, times: Optional[Sequence[float]],
                            settings: Optional[L.Settings], workspace: torch.Tensor, instance_capacity: int,
                            images: torch.Tensor, t_finals: Optional[torch.Tensor], lasts: torch.Tensor, *,
                            mode: int = 0, sh_degree: int = 3, stream=None,
                            raise_on_capacity: bool = True) -> Dict[str, int]:
    """fgs_rasterize_forward_batch.  images: float32 [3 * sum(H_v W_v)] (the
    views' [3][H][W] blocks one after another); t_finals float32 and lasts int32
    [sum(H_v W_v)].  mode=FGS_FORWARD_NO_SYNC never synchronises (graph capture)."""
    st = settings or default_settings()
    g = gaussians_struct(params, sh_degree)
    npix = sum(view_pixels(cameras))
    _check_tensor(images, "images", shape=(3 * npix,))
    _check_tensor(lasts, "lasts", dtype=torch.int32, shape=(npix,))
    if t_finals is not None:
        _check_tensor(t_finals, "t_finals", shape=(npix,))
    _check_tensor(workspace, "workspace", dtype=torch.uint8)
    stats = L.ForwardStats()
    status = L.load().fgs_rasterize_forward_batch(
        ctypes.byref(g), _camera_array(cameras), _times_array(times, len(cameras)), len(cameras), ctypes.byref(st),
        _ptr(workspace), workspace.numel(), int(instance_capacity), _ptr(images), _ptr(t_finals), _ptr(lasts),
        int(mode), ctypes.byref(stats), _stream_handle(stream))
    out = {"status": int(status), "n_visible": int(stats.n_visible), "n_instances": int(stats.n_instances),
           "depth_key_bits": int(stats.depth_key_bits)}
    if status == L.FGS_ERR_CAPACITY and not raise_on_capacity:
        return out
    L.check(status, "fgs_rasterize_forward_batch")
    return out


def rasterize_backward_batch(params: Dict[str, torch.Tensor], cameras: Sequence, times: Optional[Sequence[float]],
                             settings: Optional[L.Settings], workspace: torch.Tensor, instance_capacity: int,
                             images: torch.Tensor, lasts: torch.Tensor, dl_dimages: torch.Tensor,
                             grads: Dict[str, torch.Tensor], *, sh_degree: int = 3, stream=None) -> None:
    """fgs_rasterize_backward_batch: gradients summed over the views (plus
    velocity / accel gradients for dynamic Gaussians)."""
    st = settings or default_settings()
    g = gaussians_struct(params, sh_degree)
    n = g.n
    npix = sum(view_pixels(cameras))
    _check_tensor(images, "images", shape=(3 * npix,))
    _check_tensor(dl_dimages, "dl_dimages", shape=(3 * npix,))
    _check_tensor(lasts, "lasts", dtype=torch.int32, shape=(npix,))
    shd = sh_dtype_of(params)
    gr = L.GaussianGrads()
    names = PARAM_NAMES + (DYNAMIC_NAMES if "velocity" in params else ()) + \
        (COND4D_NAMES if "quats_r" in params else ())
    for name in names:
        rows = PARAM_SHAPES.get(name, COND4D_SHAPES.get(name, 3))
        _check_tensor(grads[name], f"grads[{name}]", dtype=param_dtype(name, shd),
                      shape=(n,) if rows == 0 else (rows, n))
        setattr(gr, name, _ptr(grads[name]))
    L.check(L.load().fgs_rasterize_backward_batch(
        ctypes.byref(g), _camera_array(cameras), _times_array(times, len(cameras)), len(cameras), ctypes.byref(st),
        _ptr(workspace), workspace.numel(), int(instance_capacity), _ptr(images), _ptr(lasts), _ptr(dl_dimages),
        ctypes.byref(gr), _stream_handle(stream)), "fgs_rasterize_backward_batch")


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
           "tiles_x": int(stats.tiles_x), "tiles_y": int(stats.tiles_y), "depth_key_bits": int(stats.depth_key_bits)}
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
    shd = sh_dtype_of(params)
    for name, rows in PARAM_SHAPES.items():
        _check_tensor(grads[name], f"grads[{name}]", dtype=param_dtype(name, shd),
                      shape=(n,) if rows == 0 else (rows, n))
    gr = L.GaussianGrads()
    for name in PARAM_NAMES:
        setattr(gr, name, _ptr(grads[name]))
    L.check(L.load().fgs_rasterize_backward(
        ctypes.byref(g), ctypes.byref(cam), ctypes.byref(st), _ptr(workspace), workspace.numel(),
        int(instance_capacity), _ptr(image), _ptr(last), _ptr(dl_dimage), ctypes.byref(gr),
        _stream_handle(stream)), "fgs_rasterize_backward")


def rasterize_backward_adam(params: Dict[str, torch.Tensor], camera, settings: Optional[L.Settings],
                            workspace: torch.Tensor, instance_capacity: int, image: torch.Tensor,
                            last: torch.Tensor, dl_dimage: torch.Tensor, exp_avg: Dict[str, torch.Tensor],
                            exp_avg_sq: Dict[str, torch.Tensor], lrs: Dict[str, float], step: int,
                            beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-15, *, sh_degree: int = 3,
                            stream=None) -> None:
    """fgs_rasterize_backward_adam: backward fused with the Adam step; params
    and the float32 moments are updated in place, no gradient is returned."""
    st = settings or default_settings()
    cam = make_camera(camera)
    g = gaussians_struct(params, sh_degree)
    n = g.n
    h, w = cam.height, cam.width
    _check_tensor(image, "image", shape=(3, h, w))
    _check_tensor(dl_dimage, "dl_dimage", shape=(3, h, w))
    _check_tensor(last, "last", dtype=torch.int32, shape=(h, w))
    _check_tensor(workspace, "workspace", dtype=torch.uint8)
    mo = L.AdamMoments()
    for k, name in enumerate(PARAM_NAMES):
        rows = PARAM_SHAPES[name]
        shape = (n,) if rows == 0 else (rows, n)
        _check_tensor(exp_avg[name], f"exp_avg[{name}]", shape=shape)
        _check_tensor(exp_avg_sq[name], f"exp_avg_sq[{name}]", shape=shape)
        mo.exp_avg[k], mo.exp_avg_sq[k] = _ptr(exp_avg[name]), _ptr(exp_avg_sq[name])
        mo.lr[k] = float(lrs[name])
    L.check(L.load().fgs_rasterize_backward_adam(
        ctypes.byref(g), ctypes.byref(cam), ctypes.byref(st), _ptr(workspace), workspace.numel(),
        int(instance_capacity), _ptr(image), _ptr(last), _ptr(dl_dimage), ctypes.byref(mo), int(step),
        float(beta1), float(beta2), float(eps), _stream_handle(stream)), "fgs_rasterize_backward_adam")


def adam_step(groups: Sequence[Tuple[torch.Tensor, torch.Tensor, torch.Tensor, torch.Tensor, float]], step: int,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-15, *, stream=None) -> None:
    """fgs_adam_step over groups of (param, grad, exp_avg, exp_avg_sq, lr), updated in place.
    param and grad: float32 or bfloat16 (the same); moments: float32."""
    arr = (L.AdamGroup * len(groups))()
    for k, (p, g, m, v, lr) in enumerate(groups):
        if p.dtype not in (torch.float32, torch.bfloat16):
            raise TypeError(f"param must be float32 or bfloat16, got {p.dtype}")
        _check_tensor(p, "param", dtype=p.dtype)
        _check_tensor(g, "grad", dtype=p.dtype, shape=p.shape)
        for t, nm in ((m, "exp_avg"), (v, "exp_avg_sq")):
            _check_tensor(t, nm, shape=p.shape)
        arr[k].param, arr[k].grad, arr[k].exp_avg, arr[k].exp_avg_sq = _ptr(p), _ptr(g), _ptr(m), _ptr(v)
        arr[k].numel = p.numel()
        arr[k].lr = float(lr)
        arr[k].dtype = L.FGS_BF16 if p.dtype == torch.bfloat16 else L.FGS_F32
    L.check(L.load().fgs_adam_step(arr, len(groups), int(step), float(beta1), float(beta2), float(eps),
                                   _stream_handle(stream)), "fgs_adam_step")


def adam_step_device(groups: Sequence[Tuple[torch.Tensor, torch.Tensor, torch.Tensor, torch.Tensor, float]],
                     state: torch.Tensor, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-15, *,
                     stream=None) -> None:
    """fgs_adam_step_device: like adam_step with the step counter kept on the
    device in ``state`` (>= 256 bytes, its first int64 the counter t, zeroed
    before the first step), so a captured graph advances t on every replay."""
    _check_tensor(state, "state", dtype=state.dtype)
    if state.numel() * state.element_size() < 256:
        raise ValueError("state must hold at least 256 bytes")
    arr = (L.AdamGroup * len(groups))()
    for k, (p, g, m, v, lr) in enumerate(groups):
        _check_tensor(p, "param", dtype=p.dtype)
        _check_tensor(g, "grad", dtype=p.dtype, shape=p.shape)
        for t, nm in ((m, "exp_avg"), (v, "exp_avg_sq")):
            _check_tensor(t, nm, shape=p.shape)
        arr[k].param, arr[k].grad, arr[k].exp_avg, arr[k].exp_avg_sq = _ptr(p), _ptr(g), _ptr(m), _ptr(v)
        arr[k].numel = p.numel()
        arr[k].lr = float(lr)
        arr[k].dtype = L.FGS_BF16 if p.dtype == torch.bfloat16 else L.FGS_F32
    L.check(L.load().fgs_adam_step_device(arr, len(groups), _ptr(state), float(beta1), float(beta2), float(eps),
                                          _stream_handle(stream)), "fgs_adam_step_device")


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


def time_next_launch(step: Optional[str], start: Optional[torch.cuda.Event] = None,
                     stop: Optional[torch.cuda.Event] = None) -> None:
    """fgs_time_next_launch: record `start`/`stop` (timing-enabled torch events
    that have been recorded at least once, so that they exist) around the next
    run of `step` on this thread; None disarms."""
    if step is None:
        L.check(L.load().fgs_time_next_launch(None, None, None), "fgs_time_next_launch")
        return
    ha, hb = int(start.cuda_event), int(stop.cuda_event)
    if not ha or not hb:
        raise ValueError("record each event once before passing it (torch creates events lazily)")
    L.check(L.load().fgs_time_next_launch(step.encode(), ha, hb), "fgs_time_next_launch")


def zorder_workspace_size(n: int) -> int:
    out = ctypes.c_size_t()
    L.check(L.load().fgs_zorder_workspace_size(int(n), ctypes.byref(out)), "fgs_zorder_workspace_size")
    return int(out.value)


def zorder_permutation(means: torch.Tensor, *, stream=None) -> torch.Tensor:
    """fgs_zorder_permutation: int32 [n] tensor (uint32 values) with perm[k] =
    index of the Gaussian placed at position k of the Morton order."""
    n = int(means.shape[1]) if means.dim() == 2 else 0
    _check_tensor(means, "means", shape=(3, n))
    perm = torch.empty(n, dtype=torch.int32, device=means.device)
    ws = torch.empty(max(zorder_workspace_size(n), 256), dtype=torch.uint8, device=means.device)
    L.check(L.load().fgs_zorder_permutation(_ptr(means), n, _ptr(ws), ws.numel(), _ptr(perm),
                                            _stream_handle(stream)), "fgs_zorder_permutation")
    return perm


def sort_workspace_size(n: int, key_bytes: int) -> int:
    out = ctypes.c_size_t(0)
    L.check(L.load().fgs_sort_workspace_size(int(n), int(key_bytes), ctypes.byref(out)), "fgs_sort_workspace_size")
    return int(out.value)


def sort_pairs(keys: torch.Tensor, vals: torch.Tensor, key_bits: int, *, stream=None) -> None:
    """fgs_sort_pairs: stable in-place sort of (keys, vals) by key bits
    [0, key_bits); keys int16 or int32 (read as unsigned), vals int32 [n]."""
    if keys.dtype not in (torch.int16, torch.int32):
        raise TypeError(f"keys must be int16 or int32, got {keys.dtype}")
    n = int(keys.numel())
    _check_tensor(keys, "keys", dtype=keys.dtype, shape=(n,))
    _check_tensor(vals, "vals", dtype=torch.int32, shape=(n,))
    kb = keys.element_size()
    ws = torch.empty(max(sort_workspace_size(n, kb), 256), dtype=torch.uint8, device=keys.device)
    L.check(L.load().fgs_sort_pairs(_ptr(keys), _ptr(vals), n, kb, int(key_bits), _ptr(ws), ws.numel(),
                                    _stream_handle(stream)), "fgs_sort_pairs")


def sort_pairs_noalloc(keys: torch.Tensor, vals: torch.Tensor, key_bits: int, *, stream=None) -> None:
    """fgs_sort_pairs_noalloc: fgs_sort_pairs with the library's static scratch
    (no workspace; n <= FGS_SORT_NOALLOC_MAX_PAIRS)."""
    if keys.dtype not in (torch.int16, torch.int32):
        raise TypeError(f"keys must be int16 or int32, got {keys.dtype}")
    n = int(keys.numel())
    _check_tensor(keys, "keys", dtype=keys.dtype, shape=(n,))
    _check_tensor(vals, "vals", dtype=torch.int32, shape=(n,))
    L.check(L.load().fgs_sort_pairs_noalloc(_ptr(keys), _ptr(vals), n, keys.element_size(), int(key_bits),
                                            _stream_handle(stream)), "fgs_sort_pairs_noalloc")


def permute_planes(src: torch.Tensor, perm: torch.Tensor, out: Optional[torch.Tensor] = None, *,
                   stream=None) -> torch.Tensor:
    """fgs_permute_planes: out[..., k] = src[..., perm[k]] for a [P, n] or [n]
    tensor of float32 or bfloat16."""
    if src.dtype not in (torch.float32, torch.bfloat16):
        raise TypeError(f"src must be float32 or bfloat16, got {src.dtype}")
    n = int(src.shape[-1])
    planes = 1 if src.dim() == 1 else int(src.shape[0])
    _check_tensor(src, "src", dtype=src.dtype)
    _check_tensor(perm, "perm", dtype=torch.int32, shape=(n,))
    if out is None:
        out = torch.empty_like(src)
    _check_tensor(out, "out", dtype=src.dtype, shape=src.shape)
    L.check(L.load().fgs_permute_planes(_ptr(src), _ptr(out), n, planes, src.element_size(), _ptr(perm),
                                        _stream_handle(stream)), "fgs_permute_planes")
    return out


def apply_zorder(params: Dict[str, torch.Tensor], optimizer=None, *, stream=None) -> torch.Tensor:
    """Re-lay the Gaussians out in Morton order: every tensor of ``params``
    (and, when given, the optimizer's moments) is replaced in its dict by its
    permuted copy.  Returns the permutation."""
    perm = zorder_permutation(params["means"], stream=stream)
    dicts = [params]
    if optimizer is not None:
        dicts += [optimizer.exp_avg, optimizer.exp_avg_sq]
    for d in dicts:
        for k in list(d):
            d[k] = permute_planes(d[k], perm, stream=stream)
    return perm


def no_sync_mode(sync_stats: Dict[str, int]) -> int:
    """FGS_FORWARD_NO_SYNC with the depth-key bits a synchronised forward
    reported (none when it found at most one visible key value)."""
    bits = int(sync_stats.get("depth_key_bits", 0))
    return L.FGS_FORWARD_NO_SYNC | (L.FGS_FORWARD_DEPTH_BITS(bits) if 1 <= bits <= 31 else 0)


def owned_workspace_settings(settings: Optional[L.Settings], keep_accum_zero: bool) -> L.Settings:
    """A copy of ``settings`` (default: the library's) for a workspace the
    caller owns: with FGS_FLAG_KEEP_ACCUM_ZERO set when ``keep_accum_zero``."""
    st = default_settings() if settings is None else settings
    st = default_settings(**{f: getattr(st, f) for f, _ in st._fields_})
    if keep_accum_zero:
        st.flags |= L.FGS_FLAG_KEEP_ACCUM_ZERO
    return st


def new_workspace(size: int, layout: L.Layout, device) -> torch.Tensor:
    """An uninitialised workspace whose accumulator state reads "not known to
    be zero" (counters[12..13] cleared)."""
    ws = torch.empty(size, dtype=torch.uint8, device=device)
    ws[layout.counters + 48:layout.counters + 56].zero_()
    return ws


class Rasterizer:
    """Owns a workspace for one camera and grows it when the instance count
    exceeds its capacity.  forward() and backward() call the C ABI.  The
    workspace is kept for the library alone, so by default the backward
    leaves its accumulators zero for the next one (FGS_FLAG_KEEP_ACCUM_ZERO)
    instead of clearing them at each call."""

    def __init__(self, camera, settings: Optional[L.Settings] = None, sh_degree: int = 3,
                 device: Optional[torch.device] = None, headroom: float = 1.25, keep_accum_zero: bool = True):
        self.camera = camera
        self.settings = owned_workspace_settings(settings, keep_accum_zero)
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
        self.workspace = new_workspace(size, workspace_layout(n, self.camera, self.settings, capacity), self.device)
        self.capacity, self.n = capacity, n

    def layout(self) -> L.Layout:
        return workspace_layout(self.n, self.camera, self.settings, self.capacity)

    def forward(self, params: Dict[str, torch.Tensor], image: Optional[torch.Tensor] = None,
                t_final: Optional[torch.Tensor] = None, last: Optional[torch.Tensor] = None, stream=None,
                sync: bool = True):
        """sync=False (once a synchronised forward has sized the workspace for
        this Gaussian count): the host never waits for the GPU; launches are
        sized by the capacity and read the counts on the device, and the depth
        sort covers the key bits the synchronised forward found varying.  An
        instance count beyond the capacity, or depth keys varying in more bits,
        then only set a flag, see overflowed()."""
        n = int(params["opacity_logits"].shape[0])
        h, w = int(self.camera.height), int(self.camera.width)
        if image is None:
            image = torch.empty(3, h, w, dtype=torch.float32, device=self.device)
        if last is None:
            last = torch.empty(h, w, dtype=torch.int32, device=self.device)
        if t_final is None:
            t_final = torch.empty(h, w, dtype=torch.float32, device=self.device)
        if not sync and self.workspace is not None and n == self.n:
            rasterize_forward_batch(params, [self.camera], None, self.settings, self.workspace, self.capacity,
                                    image.view(-1), t_final.view(-1), last.view(-1),
                                    mode=no_sync_mode(self.last_stats), sh_degree=self.sh_degree, stream=stream)
            return image, t_final, last
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

    def backward_adam(self, params: Dict[str, torch.Tensor], image: torch.Tensor, last: torch.Tensor,
                      dl_dimage: torch.Tensor, optimizer, stream=None) -> None:
        """Backward fused with optimizer's Adam step (a FusedAdam over params):
        updates params and the moments in place and advances optimizer.t."""
        optimizer.t += 1
        rasterize_backward_adam(params, self.camera, self.settings, self.workspace, self.capacity, image, last,
                                dl_dimage.contiguous(), optimizer.exp_avg, optimizer.exp_avg_sq, optimizer.lrs,
                                optimizer.t, optimizer.betas[0], optimizer.betas[1], optimizer.eps,
                                sh_degree=self.sh_degree, stream=stream)

    def overflowed(self) -> bool:
        """Whether the last forward found more instances than the capacity, or
        depth keys varying above the bits it sorted (its result is then
        incomplete or misordered); reads the device counters, so it waits for
        the GPU."""
        return bool(int(self.view("counters", 8)[7].item()))

    def lookback_slow_count(self) -> int:
        """Workgroups of the last forward's duplication whose look-back wait ran
        out and that summed the earlier counts directly (exact, slower; 0 in
        normal operation); waits for the GPU."""
        return int(self.view("dup_scan", 1)[0].item())

    # -- views of the workspace (for inspection and tests)
    def view(self, field: str, count: int, dtype=torch.int32, index: Optional[int] = None) -> torch.Tensor:
        lay = self.layout()
        off = getattr(lay, field)
        if index is not None:
            off = off[index]
        itemsize = torch.empty(0, dtype=dtype).element_size()
        return self.workspace[off:off + count * itemsize].view(dtype)


class BatchRasterizer:
    """Several views (or timesteps) per call: owns the workspace and the
    concatenated outputs.  forward() returns per-view (image [3,H,W], t_final,
    last) views of those buffers; backward() the gradients summed over views.
    As with Rasterizer, the accumulators are kept zero between backward passes
    by default (FGS_FLAG_KEEP_ACCUM_ZERO)."""

    def __init__(self, cameras: Sequence, settings: Optional[L.Settings] = None,
                 times: Optional[Sequence[float]] = None, sh_degree: int = 3,
                 device: Optional[torch.device] = None, headroom: float = 1.25, keep_accum_zero: bool = True):
        if not 1 <= len(cameras) <= L.FGS_MAX_VIEWS:
            raise ValueError(f"1..{L.FGS_MAX_VIEWS} views")
        self.cameras = list(cameras)
        self.times = None if times is None else [float(t) for t in times]
        self.settings = owned_workspace_settings(settings, keep_accum_zero)
        self.sh_degree = sh_degree
        self.device = device or torch.device("cuda", torch.cuda.current_device())
        self.headroom = headroom
        self.capacity = 0
        self.n = -1
        self.workspace: Optional[torch.Tensor] = None
        self.last_stats: Dict[str, int] = {}
        npix = sum(view_pixels(self.cameras))
        self.images = torch.empty(3 * npix, dtype=torch.float32, device=self.device)
        self.t_finals = torch.empty(npix, dtype=torch.float32, device=self.device)
        self.lasts = torch.empty(npix, dtype=torch.int32, device=self.device)

    def ensure(self, n: int, capacity: int) -> None:
        if self.workspace is not None and n == self.n and capacity <= self.capacity:
            return
        capacity = max(capacity, self.capacity if n == self.n else 0)
        size = batch_workspace_size(n, self.cameras, self.settings, capacity)
        self.workspace = new_workspace(size, batch_workspace_layout(n, self.cameras, self.settings, capacity),
                                       self.device)
        self.capacity, self.n = capacity, n

    def layout(self) -> L.Layout:
        return batch_workspace_layout(self.n, self.cameras, self.settings, self.capacity)

    def split(self, flat: torch.Tensor, channels: int):
        out, off = [], 0
        for c in self.cameras:
            hw = int(c.width) * int(c.height)
            out.append(flat[off * channels:(off + hw) * channels].view(channels, int(c.height), int(c.width))
                       if channels > 1 else flat[off:off + hw].view(int(c.height), int(c.width)))
            off += hw
        return out

    def forward(self, params: Dict[str, torch.Tensor], *, mode: int = 0, stream=None):
        """mode=FGS_FORWARD_NO_SYNC (once a synchronised forward has run): the
        depth sort covers the key bits that forward found varying, unless mode
        names its own FGS_FORWARD_DEPTH_BITS."""
        n = int(params["opacity_logits"].shape[0])
        if mode == L.FGS_FORWARD_NO_SYNC:
            mode = no_sync_mode(self.last_stats)
        self.ensure(n, max(self.capacity, 1024) if n == self.n else max(1024, 16 * n * len(self.cameras)))
        for _ in range(3):
            st = rasterize_forward_batch(params, self.cameras, self.times, self.settings, self.workspace,
                                         self.capacity, self.images, self.t_finals, self.lasts, mode=mode,
                                         sh_degree=self.sh_degree, stream=stream, raise_on_capacity=False)
            if st["status"] == L.FGS_OK:
                if not mode & L.FGS_FORWARD_NO_SYNC:  # the counts of a synchronised call
                    self.last_stats = st
                return self.images, self.t_finals, self.lasts
            self.ensure(n, int(st["n_instances"] * self.headroom) + 1024)
        raise RuntimeError("instance capacity could not be satisfied")

    def view(self, field: str, count: int, dtype=torch.int32, index: Optional[int] = None) -> torch.Tensor:
        lay = self.layout()
        off = getattr(lay, field)
        if index is not None:
            off = off[index]
        itemsize = torch.empty(0, dtype=dtype).element_size()
        return self.workspace[off:off + count * itemsize].view(dtype)

    def counters(self) -> torch.Tensor:
        """The workspace counter words (device): [0] visible, [4..5] I, [7] overflow."""
        return self.workspace[self.layout().counters:self.layout().counters + 64].view(torch.int32)

    def backward(self, params: Dict[str, torch.Tensor], dl_dimages: torch.Tensor,
                 grads: Optional[Dict[str, torch.Tensor]] = None, stream=None):
        if grads is None:
            grads = {k: torch.empty_like(v) for k, v in params.items()}
        rasterize_backward_batch(params, self.cameras, self.times, self.settings, self.workspace, self.capacity,
                                 self.images, self.lasts, dl_dimages.contiguous(), grads, sh_degree=self.sh_degree,
                                 stream=stream)
        return grads


def exported_symbols() -> Iterable[str]:
    return tuple(L.SIGNATURES)
