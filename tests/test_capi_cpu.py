"""The C ABI without a GPU: the library loads, exports every symbol the header
declares, and rejects invalid arguments before launching anything."""
import ctypes
import os
import re

import pytest

from paper_2602_09999_amd import _lib as L
from paper_2602_09999_amd import binding as B
import synthetic as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fastergs.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fgs_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    return L.load()


def test_every_declared_symbol_is_exported_and_bound(lib):
    names = declared_functions()
    assert len(names) >= 9
    for name in names:
        assert hasattr(lib, name), name
        assert name in L.SIGNATURES, name
    assert lib.fgs_abi_version() == 13 == L.ABI_VERSION


def test_default_settings_match_the_paper(lib):
    s = B.default_settings()
    assert s.tile == 16
    assert s.alpha_min == pytest.approx(1 / 255, rel=1e-7)
    assert s.alpha_max == pytest.approx(0.99, rel=1e-7)
    assert s.t_min == pytest.approx(1e-4, rel=1e-7)
    assert s.dilation == pytest.approx(0.3, rel=1e-7)
    assert s.quat_min == pytest.approx(1e-4, rel=1e-7) and s.det_min == pytest.approx(1e-6, rel=1e-7)


def test_single_view_layout_equals_one_view_batch(lib):
    # the synchronisation-free single-view forward goes through the batch
    # entry point with one view on the same workspace
    for name in ("c1", "c3"):
        cam = S.workload_camera(name)
        a = B.workspace_layout(20_000, cam, instance_capacity=300_000)
        b = B.batch_workspace_layout(20_000, [cam], instance_capacity=300_000)
        for f, _ in a._fields_:
            va, vb = getattr(a, f), getattr(b, f)
            if hasattr(va, "__len__"):
                va, vb = list(va), list(vb)
            assert va == vb, f


def test_workspace_size_and_layout(lib):
    cam = S.workload_camera("c1")
    a = B.workspace_size(10_000, cam, instance_capacity=100_000)
    b = B.workspace_size(10_000, cam, instance_capacity=200_000)
    assert b - a >= (2 * 2 + 2 * 4) * 100_000  # two 16-bit key and two value buffers
    lay = B.workspace_layout(10_000, cam, instance_capacity=100_000)
    offs = [lay.rec, lay.n_tiles, lay.depth_key, lay.counters, lay.vis_keys[0], lay.vis_ids[0],
            lay.dup_scan, lay.inst_keys[0], lay.inst_vals[0], lay.ranges, lay.accum, lay.marks, lay.touched,
            lay.touched_list, lay.slot_of, lay.sparse_grads, lay.queues, lay.scratch]
    assert lay.marks - lay.accum >= 9 * 4 * 10_000 and lay.touched - lay.marks >= 10_000
    assert lay.touched_list - lay.touched >= (10_000 + 3) // 4
    assert lay.slot_of - lay.touched_list >= 4 * 10_000 and lay.sparse_grads - lay.slot_of >= 4 * 10_000
    assert lay.queues - lay.sparse_grads >= 59 * 4 * 10_000 and lay.scratch - lay.queues >= 1024
    assert all(o % 256 == 0 for o in offs)
    assert lay.total == a and lay.tiles_x == 16 and lay.tiles_y == 16
    assert lay.inst_final == 1  # 256 tiles -> 8 key bits -> one radix pass
    assert lay.inst_key_bytes == 2
    lay2 = B.workspace_layout(10, S.workload_camera("c3"), instance_capacity=10)
    assert (lay2.tiles_x, lay2.tiles_y) == (100, 67) and lay2.inst_final == 0


def _status(fn, *args):
    return fn(*args)


def test_invalid_arguments_are_rejected_without_launching(lib):
    cam = B.make_camera(S.workload_camera("c1"))
    st = B.default_settings()
    size = ctypes.c_size_t()
    assert lib.fgs_workspace_size(-1, ctypes.byref(cam), ctypes.byref(st), 0, ctypes.byref(size)) == L.FGS_ERR_INVALID_ARGUMENT
    assert b"out of range" in lib.fgs_last_error()
    bad = B.make_camera(S.workload_camera("c1"))
    bad.width = 0
    assert lib.fgs_workspace_size(10, ctypes.byref(bad), ctypes.byref(st), 0, ctypes.byref(size)) == L.FGS_ERR_INVALID_ARGUMENT
    bad = B.make_camera(S.workload_camera("c1"))
    bad.fx = float("nan")
    assert lib.fgs_workspace_size(10, ctypes.byref(bad), ctypes.byref(st), 0, ctypes.byref(size)) == L.FGS_ERR_INVALID_ARGUMENT
    for t in (8, 16, 32):  # the three tile sizes are implemented
        stt = B.default_settings(tile=t)
        assert lib.fgs_workspace_size(10, ctypes.byref(cam), ctypes.byref(stt), 0, ctypes.byref(size)) == L.FGS_OK
    near0 = B.make_camera(S.workload_camera("c1"))
    near0.near_z = 0.0
    assert lib.fgs_workspace_size(10, ctypes.byref(near0), ctypes.byref(st), 0, ctypes.byref(size)) == L.FGS_ERR_INVALID_ARGUMENT
    # batched views: 1..16 cameras, every camera checked
    cams = (L.Camera * 17)(*([B.make_camera(S.workload_camera("c1"))] * 17))
    for v, want in ((0, L.FGS_ERR_INVALID_ARGUMENT), (1, L.FGS_OK), (16, L.FGS_OK), (17, L.FGS_ERR_INVALID_ARGUMENT)):
        assert lib.fgs_batch_workspace_size(10, cams, v, ctypes.byref(st), 0, ctypes.byref(size)) == want, v
    cams[3] = bad
    assert lib.fgs_batch_workspace_size(10, cams, 5, ctypes.byref(st), 0, ctypes.byref(size)) == L.FGS_ERR_INVALID_ARGUMENT
    one = ctypes.c_size_t()
    cams[3] = B.make_camera(S.workload_camera("c1"))
    assert lib.fgs_batch_workspace_size(1000, cams, 1, ctypes.byref(st), 500, ctypes.byref(one)) == L.FGS_OK
    assert lib.fgs_batch_workspace_size(1000, cams, 4, ctypes.byref(st), 500, ctypes.byref(size)) == L.FGS_OK
    assert size.value > 3 * one.value // 2
    st7 = B.default_settings(tile=7)
    assert lib.fgs_workspace_size(10, ctypes.byref(cam), ctypes.byref(st7), 0, ctypes.byref(size)) == L.FGS_ERR_INVALID_ARGUMENT
    stf = B.default_settings(flags=32)  # only bits 0-4 are defined
    assert lib.fgs_workspace_size(10, ctypes.byref(cam), ctypes.byref(stf), 0, ctypes.byref(size)) == L.FGS_ERR_INVALID_ARGUMENT
    for flags in (L.FGS_FLAG_FP64_CONIC, L.FGS_FLAG_LOOKBACK_FALLBACK, 3, L.FGS_FLAG_KEEP_ACCUM_ZERO, 31):
        st1 = B.default_settings(flags=flags)
        assert lib.fgs_workspace_size(10, ctypes.byref(cam), ctypes.byref(st1), 0, ctypes.byref(size)) == L.FGS_OK
    stb = B.default_settings(alpha_min=0.995)
    assert lib.fgs_workspace_size(10, ctypes.byref(cam), ctypes.byref(stb), 0, ctypes.byref(size)) == L.FGS_ERR_INVALID_ARGUMENT
    # no cap at 1: the backward divides by 1 - alpha
    st_cap = B.default_settings(alpha_max=1.0)
    assert lib.fgs_workspace_size(10, ctypes.byref(cam), ctypes.byref(st_cap), 0, ctypes.byref(size)) == L.FGS_ERR_INVALID_ARGUMENT
    assert b"alpha_max < 1" in lib.fgs_last_error()

    g = L.Gaussians()
    g.n = 5
    g.sh_dtype = L.FGS_F32
    g.sh_degree = 3
    stats = L.ForwardStats()
    # NULL parameter pointers
    r = lib.fgs_rasterize_forward(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(st), None, 0, 0, None, None, None,
                                  ctypes.byref(stats), None)
    assert r == L.FGS_ERR_INVALID_ARGUMENT
    # an unknown SH element type is rejected before any launch
    fake = 1 << 20
    for f in ("means", "log_scales", "quats", "opacity_logits", "sh_dc", "sh_rest"):
        setattr(g, f, fake)
    g.sh_dtype = 7
    r = lib.fgs_rasterize_forward(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(st), fake, 1 << 30, 0, fake, None,
                                  fake, ctypes.byref(stats), None)
    assert r == L.FGS_ERR_INVALID_ARGUMENT
    g.sh_dtype = L.FGS_F32
    g.sh_degree = 4
    r = lib.fgs_rasterize_forward(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(st), fake, 1 << 30, 0, fake, None,
                                  fake, ctypes.byref(stats), None)
    assert r == L.FGS_ERR_INVALID_ARGUMENT
    g.sh_degree = 3
    # workspace too small
    r = lib.fgs_rasterize_forward(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(st), fake, 16, 0, fake, None, fake,
                                  ctypes.byref(stats), None)
    assert r == L.FGS_ERR_INVALID_ARGUMENT and b"needed" in lib.fgs_last_error()
    # missing outputs
    r = lib.fgs_rasterize_forward(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(st), fake, 1 << 30, 0, None, None,
                                  None, ctypes.byref(stats), None)
    assert r == L.FGS_ERR_INVALID_ARGUMENT
    # backward without dl_dimage
    gr = L.GaussianGrads()
    r = lib.fgs_rasterize_backward(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(st), fake, 1 << 30, 0, fake, fake,
                                   None, ctypes.byref(gr), None)
    assert r == L.FGS_ERR_INVALID_ARGUMENT
    # dynamic Gaussians: velocity and accel together, and only through the batched calls
    g.velocity = fake
    cam1 = (L.Camera * 1)(B.make_camera(S.workload_camera("c1")))
    r = lib.fgs_rasterize_forward_batch(ctypes.byref(g), cam1, None, 1, ctypes.byref(st), fake, 1 << 40, 0, fake,
                                        None, fake, 0, ctypes.byref(stats), None)
    assert r == L.FGS_ERR_INVALID_ARGUMENT and b"together" in lib.fgs_last_error()
    g.accel = fake
    r = lib.fgs_rasterize_forward(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(st), fake, 1 << 30, 0, fake, None,
                                  fake, ctypes.byref(stats), None)
    assert r == L.FGS_ERR_INVALID_ARGUMENT and b"batch" in lib.fgs_last_error()
    times = (ctypes.c_float * 2)(0.0, float("inf"))
    cams2 = (L.Camera * 2)(B.make_camera(S.workload_camera("c1")), B.make_camera(S.workload_camera("c1")))
    r = lib.fgs_rasterize_forward_batch(ctypes.byref(g), cams2, times, 2, ctypes.byref(st), fake, 1 << 40, 0, fake,
                                        None, fake, 0, ctypes.byref(stats), None)
    assert r == L.FGS_ERR_INVALID_ARGUMENT and b"times[1]" in lib.fgs_last_error()
    r = lib.fgs_rasterize_forward_batch(ctypes.byref(g), cams2, None, 2, ctypes.byref(st), fake, 1 << 40, 0, fake,
                                        None, fake, 4, ctypes.byref(stats), None)
    assert r == L.FGS_ERR_INVALID_ARGUMENT and b"mode" in lib.fgs_last_error()
    # depth-bit hints: 1..31, only without synchronisation
    for mode, msg in ((L.FGS_FORWARD_DEPTH_BITS(20), b"NO_SYNC"),
                      (L.FGS_FORWARD_NO_SYNC | L.FGS_FORWARD_DEPTH_BITS(32), b"1..31"),
                      (L.FGS_FORWARD_NO_SYNC | L.FGS_FORWARD_DEPTH_BITS(64), b"mode bits")):
        r = lib.fgs_rasterize_forward_batch(ctypes.byref(g), cams2, None, 2, ctypes.byref(st), fake, 1 << 40, 0,
                                            fake, None, fake, mode, ctypes.byref(stats), None)
        assert r == L.FGS_ERR_INVALID_ARGUMENT and msg in lib.fgs_last_error(), (mode, lib.fgs_last_error())
    g.velocity = g.accel = None
    # conditional 4D Gaussians: all three extra planes or none, not with velocity, batched calls only
    g.mean_t = fake
    r = lib.fgs_rasterize_forward_batch(ctypes.byref(g), cam1, None, 1, ctypes.byref(st), fake, 1 << 40, 0, fake,
                                        None, fake, 0, ctypes.byref(stats), None)
    assert r == L.FGS_ERR_INVALID_ARGUMENT and b"quats_r" in lib.fgs_last_error()
    g.log_scale_t = g.quats_r = fake
    r = lib.fgs_rasterize_forward(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(st), fake, 1 << 30, 0, fake, None,
                                  fake, ctypes.byref(stats), None)
    assert r == L.FGS_ERR_INVALID_ARGUMENT and b"batch" in lib.fgs_last_error()
    g.velocity = g.accel = fake
    r = lib.fgs_rasterize_forward_batch(ctypes.byref(g), cam1, None, 1, ctypes.byref(st), fake, 1 << 40, 0, fake,
                                        None, fake, 0, ctypes.byref(stats), None)
    assert r == L.FGS_ERR_INVALID_ARGUMENT and b"no velocity" in lib.fgs_last_error()
    g.velocity = g.accel = None
    # the backward needs their gradients; the fused backward + Adam does not take them
    r = lib.fgs_rasterize_backward_batch(ctypes.byref(g), cam1, None, 1, ctypes.byref(st), fake, 1 << 40, 0, fake,
                                         fake, fake, ctypes.byref(gr), None)
    assert r == L.FGS_ERR_INVALID_ARGUMENT
    g.mean_t = g.log_scale_t = g.quats_r = None
    # fused backward + Adam: missing state, bad hyperparameters, non-finite lr
    mo = L.AdamMoments()
    r = lib.fgs_rasterize_backward_adam(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(st), fake, 1 << 30, 0, fake,
                                        fake, fake, None, 1, 0.9, 0.999, 1e-15, None)
    assert r == L.FGS_ERR_INVALID_ARGUMENT
    r = lib.fgs_rasterize_backward_adam(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(st), fake, 1 << 30, 0, fake,
                                        fake, fake, ctypes.byref(mo), 0, 0.9, 0.999, 1e-15, None)
    assert r == L.FGS_ERR_INVALID_ARGUMENT
    mo.lr[2] = float("nan")
    r = lib.fgs_rasterize_backward_adam(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(st), fake, 1 << 30, 0, fake,
                                        fake, fake, ctypes.byref(mo), 1, 0.9, 0.999, 1e-15, None)
    assert r == L.FGS_ERR_INVALID_ARGUMENT and b"lr[2]" in lib.fgs_last_error()
    mo.lr[2] = 1e-3
    r = lib.fgs_rasterize_backward_adam(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(st), fake, 1 << 30, 0, fake,
                                        fake, fake, ctypes.byref(mo), 1, 0.9, 0.999, 1e-15, None)
    assert r == L.FGS_ERR_INVALID_ARGUMENT and b"moment" in lib.fgs_last_error()
    # Adam argument checks
    arr = (L.AdamGroup * 1)()
    assert lib.fgs_adam_step(arr, 0, 1, 0.9, 0.999, 1e-15, None) == L.FGS_ERR_INVALID_ARGUMENT
    assert lib.fgs_adam_step(arr, 1, 0, 0.9, 0.999, 1e-15, None) == L.FGS_ERR_INVALID_ARGUMENT
    arr[0].numel = 4
    assert lib.fgs_adam_step(arr, 1, 1, 0.9, 0.999, 1e-15, None) == L.FGS_ERR_INVALID_ARGUMENT
    assert lib.fgs_adam_step(arr, 1, 1, 1.5, 0.999, 1e-15, None) == L.FGS_ERR_INVALID_ARGUMENT
    arr[0].param = arr[0].grad = arr[0].exp_avg = arr[0].exp_avg_sq = fake
    arr[0].dtype = 5
    assert lib.fgs_adam_step(arr, 1, 1, 0.9, 0.999, 1e-15, None) == L.FGS_ERR_INVALID_ARGUMENT
    assert lib.fgs_l1_loss_backward(None, None, 10, None, None, None) == L.FGS_ERR_INVALID_ARGUMENT
    # timing hook: known step names only, non-NULL events; NULL disarms
    assert lib.fgs_time_next_launch(b"no_such_step", fake, fake) == L.FGS_ERR_INVALID_ARGUMENT
    assert lib.fgs_time_next_launch(b"adam", None, fake) == L.FGS_ERR_INVALID_ARGUMENT
    assert lib.fgs_time_next_launch(None, None, None) == L.FGS_OK
    assert lib.fgs_status_string(2) == b"instance capacity exceeded"


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(FileNotFoundError):
        L._lib_backup = L._lib
        try:
            L._lib = None
            L.load(str(tmp_path / "nope.so"))
        finally:
            L._lib = L._lib_backup


def test_noalloc_sort_bounds_are_checked_before_any_device_call(lib):
    # the static scratch holds the workspace of the largest accepted sort
    for kb in (2, 4):
        assert B.sort_workspace_size(L.FGS_SORT_NOALLOC_MAX_PAIRS, kb) <= L.FGS_SORT_NOALLOC_SCRATCH_BYTES
    f = lib.fgs_sort_pairs_noalloc
    # rejected on the host: too many pairs, a bad width or bit count; nothing launched
    assert f(None, None, L.FGS_SORT_NOALLOC_MAX_PAIRS + 1, 4, 32, None) == L.FGS_ERR_INVALID_ARGUMENT
    assert b"static scratch" in lib.fgs_last_error()
    assert f(None, None, -1, 4, 32, None) == L.FGS_ERR_INVALID_ARGUMENT
    assert f(None, None, 10, 3, 8, None) == L.FGS_ERR_INVALID_ARGUMENT
    assert f(None, None, 10, 2, 17, None) == L.FGS_ERR_INVALID_ARGUMENT
    assert f(None, None, 10, 4, 8, None) == L.FGS_ERR_INVALID_ARGUMENT  # NULL arrays
    # nothing to sort: returns at once, before looking up the device array
    assert f(None, None, 0, 4, 32, None) == L.FGS_OK
    assert f(None, None, 10, 4, 0, None) == L.FGS_OK
