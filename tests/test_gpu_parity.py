"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bars: instance keys, sort and tile ranges bit-exact (pairs inside the FP32
borderline band of the key reference may go either way and are counted);
images and final transmittance within 1e-5 absolute of the FP64 oracle on
pixels without a borderline decision; the last contributor's index equal
there; gradients within 1e-3 relative L2 per parameter group, with the
upstream gradient zeroed on borderline pixels for both sides; Adam within
1e-6 relative of the FP64 update.
"""
import numpy as np
import pytest
import torch

import oracle as O
import synthetic as S
from paper_2602_09999_amd import binding as B
from paper_2602_09999_amd import _lib as L
from paper_2602_09999_amd.autograd import FusedAdam
from tests.gpu_util import (compare_lists, forward, last_ids, record, say, sorted_instances, to_gpu)

pytestmark = pytest.mark.gpu

IMG_TOL = 1e-5
GRAD_TOL = 1e-3
F64 = torch.float64


def rows64(sc):
    return {k: (v.to(F64).T.contiguous() if v.dim() == 2 else v.to(F64)) for k, v in sc.items()}


def rel_l2(a, b):
    a = a.double().cpu()
    b = b.double().cpu()
    den = float(b.norm())
    return float((a - b).norm()) / max(den, 1e-30)


CASES = {
    "c1": lambda: (S.make_scene(10_000, 0), S.workload_camera("c1")),
    "ragged_bg": lambda: (S.make_scene(3_000, 1), S.identity_camera(100, 75, 110.0, bg=(0.2, 0.5, 0.9))),
    "offcentre": lambda: (S.make_scene(4_000, 2), S.identity_camera(150, 130, 170.0, cx=40.0, cy=100.0,
                                                                     bg=(1.0, 0.0, 0.3))),
    "lookat": lambda: (S.make_scene(5_000, 3, z_range=(-1.0, 1.0)),
                       S.look_at_camera((0.5, -1.0, -4.0), (0.0, 0.0, 0.0), 120, 96, 130.0, bg=(0.1, 0.1, 0.1))),
    "dense": lambda: (S.make_scene(6_000, 4, log_scale_mean=-3.0), S.identity_camera(64, 48, 64.0)),
    # n % 4 != 0 exercises the per-element tails of the four-Gaussian kernels
    "ragged_n": lambda: (S.make_scene(2_999, 5), S.identity_camera(90, 70, 100.0, bg=(0.3, 0.1, 0.6))),
}


@pytest.mark.parametrize("case", list(CASES))
def test_preprocess_record_matches_oracle(case):
    sc, cam = CASES[case]()
    say("record", case)
    rz, params, *_ = forward(sc, cam)
    n = S.count(sc)
    rec = record(rz, n)
    n_tiles = rz.view("n_tiles", n).cpu().numpy().view(np.uint32)
    dkey = rz.view("depth_key", n).cpu().numpy().view(np.uint32)
    ref = O.keys_ref(sc, cam)
    assert np.array_equal(dkey, ref["depth"].view(np.uint32)), "depth keys must be bit-exact"
    nom, border = O.keys_ref_banded(sc, cam)
    bg = {g for _, g in border}
    mism = np.nonzero(n_tiles != ref["n_tiles"])[0]
    assert set(mism.tolist()) <= bg, f"tile counts differ off the borderline band: {mism[:10]}"
    pre = {k: (v.detach().numpy() if torch.is_tensor(v) else v) for k, v in O.preprocess64(rows64(sc), cam).items()}
    vis = n_tiles > 0
    assert vis.sum() > 0
    # mu2D = f * (x/z) + c in FP32: the rounding scale is |f x/z| + |c| <= 2|c| + |mu2D|
    for j, c in ((0, cam.cx), (1, cam.cy)):
        m = pre["mean2d"][vis, j]
        assert (np.abs(rec[vis, j] - m) / (np.abs(m) + 2 * abs(c) + 1.0)).max() < 2e-6
    assert np.abs(rec[vis, 2] - pre["opacity"][vis]).max() < 1e-6
    con = pre["conic"][vis]
    cs = np.abs(con).max(1)
    for j in range(3):
        assert (np.abs(rec[vis, 4 + j] - con[:, j]) / cs).max() < 1e-4
    assert np.abs(rec[vis, 8:11] - pre["rgb"][vis]).max() < 2e-6
    assert np.array_equal(rec[vis, 7], ref["depth"][vis])
    # fourth float4: packed tile rectangle and the instance count, as uint32 bits
    r3 = rz.view("rec", 16 * n, dtype=torch.float32).cpu().numpy().reshape(n, 16)[:, 12:15].view(np.uint32)
    assert np.array_equal(r3[vis, 2], n_tiles[vis])
    tx0, ty0, tx1, ty1, _ = O.tile_rect(O.record32(sc, cam), cam.width, cam.height, 16)
    sure = vis & ~np.isin(np.arange(n), list(bg))
    assert np.array_equal(r3[sure, 0], (tx0 | (ty0 << 16))[sure].astype(np.uint32))
    assert np.array_equal(r3[sure, 1], (tx1 | (ty1 << 16))[sure].astype(np.uint32))


@pytest.mark.parametrize("case", list(CASES))
def test_keys_sort_and_ranges_bit_exact(case):
    sc, cam = CASES[case]()
    if case == "dense":
        sc["means"][2, 100:400] = sc["means"][2, 50]  # many exact depth ties
    say("keys", case)
    rz, *_ = forward(sc, cam)
    keys, vals, ranges = sorted_instances(rz)
    nom, border = O.keys_ref_banded(sc, cam)
    assert rz.last_stats["n_instances"] == len(keys)
    flips = compare_lists(keys, vals, ranges, nom, border, depth=nom["depth"])
    say("  instances", len(keys), "borderline pairs", len(border), "flipped", flips)
    assert flips <= len(border)


@pytest.mark.parametrize("case", list(CASES))
def test_forward_image_matches_oracle(case):
    sc, cam = CASES[case]()
    say("forward", case)
    rz, params, image, t_final, last = forward(sc, cam)
    ref = O.render64(sc, cam)
    ok = ~ref["borderline"].numpy()
    img = image.cpu().double().numpy()
    err = np.abs(img - ref["image"].numpy()).max(0)
    terr = np.abs(t_final.cpu().double().numpy() - ref["t_final"].numpy())
    say("  exempt pixels", int((~ok).sum()), "of", ok.size, "max err", float(err[ok].max()), "T err",
        float(terr[ok].max()))
    assert (~ok).sum() <= max(4, ok.size // 100)
    assert err[ok].max() <= IMG_TOL
    assert terr[ok].max() <= IMG_TOL
    lid = last_ids(rz, last)
    assert np.array_equal(lid[ok], ref["last_id"].numpy()[ok])


@pytest.mark.parametrize("case", ["c1", "ragged_bg", "lookat", "dense", "ragged_n"])
def test_backward_gradients_match_oracle(case):
    sc, cam = CASES[case]()
    say("backward", case)
    dl = S.make_dl_dimage(cam.height, cam.width, seed=5)
    ref0 = O.render64(sc, cam)
    dl[:, ref0["borderline"]] = 0.0
    ref = O.render64(sc, cam, dl_dimage=dl)
    rz, params, image, t_final, last = forward(sc, cam)
    grads = rz.backward(params, image, last, dl.cuda())
    torch.cuda.synchronize()
    for k in B.PARAM_NAMES:
        e = rel_l2(grads[k], ref["grads"][k])
        say(f"  {k:15s} rel L2 {e:.2e}")
        assert e <= GRAD_TOL, (k, e)


def test_autograd_function_and_l1_gradient():
    sc, cam = CASES["ragged_bg"]()
    say("autograd")
    from paper_2602_09999_amd.autograd import rasterize
    rz = B.Rasterizer(cam)
    params = {k: v.clone().requires_grad_(True) for k, v in to_gpu(sc).items()}
    image, t_final, last = rasterize(params, rz)
    target = S.make_target(cam.height, cam.width, seed=1).cuda()
    dl = torch.empty_like(image)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    B.l1_loss_backward(image.detach(), target, dl, loss)
    image.backward(dl)
    torch.cuda.synchronize()
    # L1 term against the oracle (float64 reduction)
    l_ref, g_ref = O.l1_loss_grad64(image.detach().cpu(), target.cpu())
    assert abs(float(loss) - l_ref) <= 1e-12
    assert torch.equal(torch.sign(dl.cpu()), torch.sign(g_ref).float())
    assert torch.allclose(dl.cpu().double(), g_ref, rtol=1e-6, atol=0)
    # the autograd gradients equal a direct backward call
    rz2, p2, im2, t2, la2 = forward(sc, cam)
    direct = rz2.backward(p2, im2, la2, dl)
    for k in B.PARAM_NAMES:
        assert rel_l2(params[k].grad, direct[k]) <= 1e-6


def test_adam_matches_fp64_update():
    say("adam")
    g = torch.Generator().manual_seed(0)
    sizes = [30_000, 4_097, 3, 45 * 1000 + 1]
    lrs = [1.6e-4, 5e-3, 1e-3, 2.5e-2]
    p0 = [torch.randn(s, generator=g) for s in sizes]
    ps = [p.cuda() for p in p0]
    ms = [torch.zeros_like(p) for p in ps]
    vs = [torch.zeros_like(p) for p in ps]
    rp = [p.double() for p in p0]
    rm = [torch.zeros(s, dtype=F64) for s in sizes]
    rv = [torch.zeros(s, dtype=F64) for s in sizes]
    for step in range(1, 6):
        gr = [torch.randn(s, generator=g) for s in sizes]
        gr[1][::5] = 0.0
        B.adam_step([(ps[i], gr[i].cuda(), ms[i], vs[i], lrs[i]) for i in range(4)], step)
        for i in range(4):
            rp[i], rm[i], rv[i] = O.adam64(rp[i], gr[i].double(), rm[i], rv[i], step, lrs[i])
    torch.cuda.synchronize()
    for i in range(4):
        d = (ps[i].cpu().double() - rp[i]).abs()
        # 1e-6 relative to the larger of |p| and the total movement (each Adam
        # step moves p by at most ~lr); FP32 storage of p alone is ~6e-8 relative
        bound = 1e-6 * torch.clamp(rp[i].abs(), min=lrs[i] * 5)
        assert bool((d <= bound).all()), (i, float((d / bound).max()))
        assert rel_l2(ms[i], rm[i]) <= 1e-6
        assert rel_l2(vs[i], rv[i]) <= 1e-6


def test_empty_and_degenerate_inputs():
    say("empty")
    cam = S.identity_camera(40, 30, 50.0, bg=(0.25, 0.5, 0.75))
    empty = S.subset(S.make_scene(10, 0), slice(0, 0))
    rz, params, image, t_final, last = forward(empty, cam)
    bg = torch.tensor(cam.bg).view(3, 1, 1).expand(3, 30, 40)
    assert torch.equal(image.cpu(), bg)
    assert bool((t_final == 1).all()) and bool((last == 0).all())
    grads = rz.backward(params, image, last, torch.ones_like(image))
    # degenerate Gaussians: NaN / tiny quaternion, behind the camera, transparent
    sc = S.make_scene(6, 1)
    sc["quats"][:, 0] = float("nan")
    sc["quats"][:, 1] = 1e-6
    sc["means"][2, 2] = -1.0
    sc["opacity_logits"][3] = -30.0
    rz, params, image, t_final, last = forward(sc, cam)
    n_tiles = rz.view("n_tiles", 6).cpu().numpy()
    assert list(n_tiles[:4]) == [0, 0, 0, 0]
    assert bool(torch.isfinite(image).all())
    ref = O.render64(sc, cam)
    ok = ~ref["borderline"].numpy()
    assert np.abs(image.cpu().double().numpy() - ref["image"].numpy()).max(0)[ok].max() <= IMG_TOL
    grads = rz.backward(params, image, last, torch.ones_like(image))
    for k in B.PARAM_NAMES:
        assert bool(torch.isfinite(grads[k]).all())
        assert float(grads[k][..., :4].abs().max()) == 0.0


def test_forward_is_deterministic():
    sc, cam = CASES["c1"]()
    say("determinism")
    a = forward(sc, cam)
    b = forward(sc, cam)
    assert torch.equal(a[2], b[2]) and torch.equal(a[3], b[3]) and torch.equal(a[4], b[4])
    ka, va, ra = sorted_instances(a[0])
    kb, vb, rb = sorted_instances(b[0])
    assert np.array_equal(va, vb) and np.array_equal(ra, rb)


@pytest.mark.parametrize("case", ["c1", "ragged_n"])
def test_lookback_fallback_gives_the_same_lists(case):
    """The duplication's exact fallback (a workgroup sums the counts of all
    earlier entries itself), forced from the host for every workgroup after
    the first: the instance lists and the image equal those of the look-back,
    which the keys test checks against the oracle."""
    sc, cam = CASES[case]()
    say("look-back fallback", case)
    a = forward(sc, cam)
    b = forward(sc, cam, settings=B.default_settings(flags=L.FGS_FLAG_LOOKBACK_FALLBACK))
    nvis = a[0].last_stats["n_visible"]
    say("  visible", nvis, "slow-path workgroups", b[0].lookback_slow_count())
    assert a[0].lookback_slow_count() == 0
    assert b[0].lookback_slow_count() == (nvis + 255) // 256 - 1 > 0
    ka, va, ra = sorted_instances(a[0])
    kb, vb, rb = sorted_instances(b[0])
    assert np.array_equal(ka, kb) and np.array_equal(va, vb) and np.array_equal(ra, rb)
    assert torch.equal(a[2], b[2]) and torch.equal(a[4], b[4])


def test_capacity_overflow_reports_count_and_retry_succeeds():
    sc, cam = CASES["c1"]()
    say("capacity")
    params = to_gpu(sc)
    n = S.count(sc)
    cap = 100
    ws = torch.empty(B.workspace_size(n, cam, instance_capacity=cap), dtype=torch.uint8, device="cuda")
    image = torch.empty(3, cam.height, cam.width, device="cuda")
    last = torch.empty(cam.height, cam.width, dtype=torch.int32, device="cuda")
    st = B.rasterize_forward(params, cam, None, ws, cap, image, None, last, raise_on_capacity=False)
    assert st["status"] == L.FGS_ERR_CAPACITY
    need = st["n_instances"]
    assert need == len(O.keys_ref(sc, cam)["keys"]) or abs(need - len(O.keys_ref(sc, cam)["keys"])) < 20
    ws = torch.empty(B.workspace_size(n, cam, instance_capacity=need), dtype=torch.uint8, device="cuda")
    st = B.rasterize_forward(params, cam, None, ws, need, image, None, last)
    assert st["n_instances"] == need


@pytest.mark.parametrize("name", ["c2", "c3"])
def test_full_size_sampled_parity(name):
    """Full-size workloads, in the launch configuration the benchmark times:
    sampled tile lists bit-exact, a 64x64 crop of the image against the FP64
    oracle, all gradients with the upstream gradient confined to the crop; then
    the synchronisation-free forward and the fused backward + Adam of the
    benchmark's step against the checked synchronised forward and backward."""
    w = S.WORKLOADS[name]
    say("full size", name, w.n)
    sc = S.make_scene(w.n, seed=0)
    cam = S.workload_camera(name)
    rz, params, image, t_final, last = forward(sc, cam)
    keys, vals, ranges = sorted_instances(rz)
    say("  N_vis", rz.last_stats["n_visible"], "I", rz.last_stats["n_instances"])
    # the duplication's offsets came from its look-back, not its slow path
    assert rz.lookback_slow_count() == 0
    tiles_x = rz.layout().tiles_x
    rng = np.random.default_rng(0)
    sample = sorted(set(rng.integers(0, ranges.shape[0], 12).tolist()) | {0, ranges.shape[0] - 1,
                                                                          (ranges.shape[0] // 2) + tiles_x // 2})
    lists = O.tile_lists_for(sc, cam, sample, delta=1e-3)
    for t in sample:
        ref_list, band = lists[t]
        s, e = ranges[t]
        got = vals[s:e]
        assert np.all(keys[s:e] == t)
        a = [g for g in got.tolist() if g not in band]
        b = [g for g in ref_list.tolist() if g not in band]
        assert a == b, f"tile {t}"
    cx, cy = w.width // 2, w.height // 2
    crop = (cx - 32, cy - 32, cx + 32, cy + 32)
    dl_full = torch.zeros(3, w.height, w.width)
    dl_crop = S.make_dl_dimage(64, 64, seed=9)
    ref0 = O.render64(sc, cam, crop=crop)
    dl_crop[:, ref0["borderline"]] = 0.0
    dl_full[:, crop[1]:crop[3], crop[0]:crop[2]] = dl_crop
    ref = O.render64(sc, cam, crop=crop, dl_dimage=dl_crop)
    ok = ~ref["borderline"].numpy()
    img = image[:, crop[1]:crop[3], crop[0]:crop[2]].cpu().double().numpy()
    err = np.abs(img - ref["image"].numpy()).max(0)
    say("  crop exempt", int((~ok).sum()), "max err", float(err[ok].max()))
    assert err[ok].max() <= IMG_TOL
    lid = last_ids(rz, last)[crop[1]:crop[3], crop[0]:crop[2]]
    assert np.array_equal(lid[ok], ref["last_id"].numpy()[ok])
    grads = rz.backward(params, image, last, dl_full.cuda())
    torch.cuda.synchronize()
    for k in B.PARAM_NAMES:
        e = rel_l2(grads[k], ref["grads"][k])
        say(f"  {k:15s} rel L2 {e:.2e}")
        assert e <= GRAD_TOL, (k, e)
    # the benchmark's step: the forward without host synchronisation (same
    # outputs, bit for bit), then the backward fused with Adam against backward
    # then Adam from the same state.  Float atomics accumulate each Gaussian's
    # 2D gradients in a run-dependent order; at this size a Gaussian sums up to
    # thousands of fragments, and the log-scale gradient (conic terms of both
    # signs) moves most: measured 7e-6 relative, bound 1e-4 (the oracle bound
    # on each run's gradients is 1e-3)
    img2, tf2, last2 = rz.forward(params, sync=False)
    torch.cuda.synchronize()
    assert not rz.overflowed() and rz.lookback_slow_count() == 0
    assert torch.equal(img2, image) and torch.equal(tf2, t_final) and torch.equal(last2, last)
    dl = S.make_dl_dimage(w.height, w.width, seed=4).cuda()
    pa = {k: v.clone() for k, v in params.items()}
    pb = {k: v.clone() for k, v in params.items()}
    oa, ob = FusedAdam(pa, S.ADAM_LR), FusedAdam(pb, S.ADAM_LR)
    oa.step(rz.backward(pa, img2, last2, dl))
    rz.backward_adam(pb, img2, last2, dl, ob)
    torch.cuda.synchronize()
    # the fused path lists the Gaussians the blend backward marked: exactly
    # those whose accumulator row is nonzero
    rows = rz.view("accum", 9 * w.n, dtype=torch.float32).view(w.n, 9)
    n_rows = int(rows.ne(0).any(1).sum().item())
    n_listed = int(rz.view("counters", 16)[8].item())
    say("  Gaussians with a gradient", n_listed)
    assert n_listed == n_rows > 0
    for k in B.PARAM_NAMES:
        em = rel_l2(ob.exp_avg[k], oa.exp_avg[k])
        ev = rel_l2(ob.exp_avg_sq[k], oa.exp_avg_sq[k])
        ed = rel_l2(pb[k] - params[k], pa[k] - params[k])
        say(f"  fused {k:15s} m {em:.1e} v {ev:.1e} displacement {ed:.1e}")
        assert em <= 1e-4 and ev <= 1e-4 and ed <= 1e-3, (k, em, ev, ed)
