"""GPU tests of the batched forms: tile sizes 8 and 32, several views in one
pass (uneven resolutions, one depth sort, one tile sort, one blend launch),
the synchronisation-free mode and its graph capture, and dynamic (4D)
Gaussians whose means move with time.

A batched result must equal the per-view results: images and last
contributors bit-identical, keys per view bit-exact against the key
reference, gradients equal to the sum of the per-view gradients.  Dynamic
Gaussians: per timestep the oracle renders the means at that time, computed
in float32 in the kernel's order; the velocity and acceleration gradients
must equal sum_t t dL/dmean(t) and sum_t t^2 dL/dmean(t) of the oracle's
per-timestep mean gradients."""
import numpy as np
import pytest
import torch

import oracle as O
import synthetic as S
from paper_2602_09999_amd import _lib as L
from paper_2602_09999_amd import binding as B
from paper_2602_09999_amd.autograd import FusedAdam
from tests.gpu_util import (check_adam, check_grads, check_image, compare_lists, forward, last_ids, say,
                            sorted_instances, to_gpu)

pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    a, b = a.double().cpu(), b.double().cpu()
    return float((a - b).norm()) / max(float(b.norm()), 1e-30)


def small_views():
    """Three cameras on the radius-5 sphere around a recentred scene, uneven sizes."""
    cams = S.uniform_sphere_cameras(3, seed=11, w_range=(60, 140), h_range=(50, 120))
    return [c.copy(fx=0.9 * c.width, fy=0.9 * c.width) for c in cams]


@pytest.mark.parametrize("tile", [8, 32])
@pytest.mark.parametrize("case", ["c1", "ragged"])
def test_tile_sizes_keys_image_gradients(tile, case):
    if case == "c1":
        sc, cam = S.make_scene(10_000, 0), S.workload_camera("c1")
    else:
        sc, cam = S.make_scene(3_000, 1), S.identity_camera(100, 75, 110.0, bg=(0.2, 0.5, 0.9))
    say("tile", tile, case)
    st = B.default_settings(tile=tile)
    rz, params, image, t_final, last = forward(sc, cam, settings=st)
    keys, vals, ranges = sorted_instances(rz)
    nom, border = O.keys_ref_banded(sc, cam, tile=tile)
    flips = compare_lists(keys, vals, ranges, nom, border, depth=nom["depth"])
    say("  instances", len(keys), "borderline pairs", len(border), "flipped", flips)
    assert flips <= len(border)
    ref = O.render64(sc, cam, dl_dimage=S.make_dl_dimage(cam.height, cam.width, seed=5), mask_borderline=True)
    check_image(f"tile {tile} {case}", image, ref, t_final=t_final, last_ids_gpu=last_ids(rz, last))
    grads = rz.backward(params, image, last, ref["dl_used"].float().cuda())
    torch.cuda.synchronize()
    check_grads(f"tile {tile} {case}", grads, ref["grads"], exempt=ref["clip_border"].numpy())


def wide_views():
    """Three near-1080p cameras: at tile 8 the views hold >= 65536 tiles in
    all, so the batch sorts 32-bit tile keys while each view alone sorts
    16-bit ones."""
    cams = S.uniform_sphere_cameras(3, seed=12, w_range=(1900, 1920), h_range=(1060, 1080))
    return [c.copy(fx=0.9 * c.width, fy=0.9 * c.width) for c in cams]


def view_crops(cam, views):
    """Comparison windows of a view: the whole image for the small views; for
    the near-1080p views a 64x64 window at the centre and one on the bottom
    edge (the last, partial tile row at tile 8 when the height is not a
    multiple of 8)."""
    if views == "small":
        return [None]
    w, h = int(cam.width), int(cam.height)
    return [(w // 2 - 32, h // 2 - 32, w // 2 + 32, h // 2 + 32), (w // 2 + 100, h - 64, w // 2 + 164, h)]


@pytest.mark.parametrize("tile,views", [(16, "small"), (8, "small"), (8, "wide")])
def test_batch_matches_oracle_and_single_views(tile, views):
    """One batched pass over uneven views against the FP64 oracle per view
    (images on every view's comparison windows, gradients summed over the
    views with the upstream gradient confined to those windows), and against
    single-view runs of the same library (images and last contributors bit
    for bit, gradients the sum of the views').  At tile 8 the near-1080p views
    hold more than 65535 tiles together, so the batch sorts 32-bit tile keys."""
    sc = S.batch_scene(20_000, 3)
    cams = small_views() if views == "small" else wide_views()
    say("batch", [(c.width, c.height) for c in cams], "tile", tile)
    st = B.default_settings(tile=tile)
    params = to_gpu(sc)
    br = B.BatchRasterizer(cams, settings=st)
    images, t_finals, lasts = br.forward(params)
    lay = br.layout()
    say("  global tiles", lay.total_tiles, "key bytes", lay.inst_key_bytes)
    assert lay.inst_key_bytes == (4 if lay.total_tiles >= 65536 else 2)
    assert (views == "wide") == (lay.inst_key_bytes == 4)
    imgs, tfs, lss = br.split(images, 3), br.split(t_finals, 1), br.split(lasts, 1)
    # the oracle per view; the upstream gradient lives on the comparison windows
    dls, g_ref, exempt = [], None, []
    for k, cam in enumerate(cams):
        dl_full = torch.zeros(3, cam.height, cam.width)
        for j, crop in enumerate(view_crops(cam, views)):
            x0, y0, x1, y1 = crop if crop is not None else (0, 0, cam.width, cam.height)
            ref = O.render64(sc, cam, crop=crop, mask_borderline=True,
                             dl_dimage=S.make_dl_dimage(y1 - y0, x1 - x0, seed=20 + 7 * k + j))
            check_image(f"view {k} window {j}", imgs[k][:, y0:y1, x0:x1], ref, t_final=tfs[k][y0:y1, x0:x1])
            dl_full[:, y0:y1, x0:x1] = ref["dl_used"].float()
            g_ref = ref["grads"] if g_ref is None else {n: g_ref[n] + ref["grads"][n] for n in g_ref}
            exempt.append(ref["clip_border"].numpy())
        dls.append(dl_full)
    gb = br.backward(params, torch.cat([d.reshape(-1) for d in dls]).cuda())
    torch.cuda.synchronize()
    check_grads(f"batch tile {tile} {views}", gb, g_ref, exempt=np.concatenate(exempt))
    # the same library, one view at a time
    gsum = {k: torch.zeros_like(v, dtype=torch.float64) for k, v in params.items()}
    total = 0
    for k, cam in enumerate(cams):
        rz, p1, image, t_final, last = forward(sc, cam, settings=st)
        assert rz.layout().inst_key_bytes == 2
        assert torch.equal(imgs[k], image), k
        assert torch.equal(tfs[k], t_final), k
        assert torch.equal(lss[k], last), k
        total += rz.last_stats["n_instances"]
        g1 = rz.backward(p1, image, last, dls[k].cuda())
        for name in gsum:
            gsum[name] += g1[name].double()
    torch.cuda.synchronize()
    assert br.last_stats["n_instances"] == total
    for name in B.PARAM_NAMES:
        e = rel_l2(gb[name], gsum[name])
        say(f"  {name:15s} batch vs sum of views rel L2 {e:.1e}")
        assert e <= 1e-5, (name, e)


def test_batched_workload_full_size_sampled():
    """The 16-view workload at full size: 1.5M Gaussians around the origin, 16
    cameras on the radius-5 sphere with seeded resolutions in 640-1920 x
    480-1080, tile 16 (the benchmark's autotuner's choice).  On three views:
    sampled tile lists bit-exact against the key reference off the borderline
    band (entries of the right view, in canonical order), a 64x64 window at
    the view centre against the FP64 oracle, and every gradient summed over
    the three windows (the upstream gradient lives there only).  The
    synchronisation-free forward, as the captured step runs it, gives the
    same images bit for bit."""
    n = 1_500_000
    sc = S.batch_scene(n, 0)
    cams = S.uniform_sphere_cameras(16, seed=0)
    say("16-view workload", [(c.width, c.height) for c in cams])
    params = to_gpu(sc)
    br = B.BatchRasterizer(cams)
    images, t_finals, lasts = br.forward(params)
    images, t_finals = images.clone(), t_finals.clone()
    imgs, tfs = br.split(images, 3), br.split(t_finals, 1)
    keys, vals, ranges = sorted_instances(br)
    say("  instances", len(keys), "global tiles", br.layout().total_tiles)
    tiles_of = [((c.width + 15) // 16) * ((c.height + 15) // 16) for c in cams]
    base = np.concatenate([[0], np.cumsum(tiles_of)])
    rng = np.random.default_rng(4)
    views = [0, 7, 15]
    dls = [torch.zeros(3, c.height, c.width) for c in cams]
    g_ref, exempt = None, []
    for k in views:
        cam = cams[k]
        tx, ty = (cam.width + 15) // 16, (cam.height + 15) // 16
        sample = sorted(set(rng.integers(0, tiles_of[k], 3).tolist()) | {(ty // 2) * tx + tx // 2})
        lists = O.tile_lists_for(sc, cam, sample, delta=1e-3)
        for tl in sample:
            ref_list, band = lists[tl]
            s0, e0 = ranges[base[k] + tl]
            got = vals[s0:e0].astype(np.int64)
            assert np.all(got // n == k), (k, tl)
            got = (got % n).tolist()
            assert [g for g in got if g not in band] == [g for g in ref_list.tolist() if g not in band], (k, tl)
        say(f"  view {k}: tiles {sample} match ({sum(len(lists[t][0]) for t in sample)} entries)")
        crop = (cam.width // 2 - 32, cam.height // 2 - 32, cam.width // 2 + 32, cam.height // 2 + 32)
        x0, y0, x1, y1 = crop
        ref = O.render64(sc, cam, crop=crop, mask_borderline=True, dl_dimage=S.make_dl_dimage(64, 64, seed=40 + k))
        check_image(f"view {k} centre", imgs[k][:, y0:y1, x0:x1], ref, t_final=tfs[k][y0:y1, x0:x1])
        dls[k][:, y0:y1, x0:x1] = ref["dl_used"].float()
        g_ref = ref["grads"] if g_ref is None else {m: g_ref[m] + ref["grads"][m] for m in g_ref}
        exempt.append(ref["clip_border"].numpy())
    grads = br.backward(params, torch.cat([d.reshape(-1) for d in dls]).cuda())
    torch.cuda.synchronize()
    check_grads("16 views", grads, g_ref, exempt=np.concatenate(exempt))
    br.ensure(n, int(br.last_stats["n_instances"] * 1.3))
    images2, _, _ = br.forward(params, mode=L.FGS_FORWARD_NO_SYNC)
    torch.cuda.synchronize()
    assert int(br.counters().cpu()[7]) == 0
    assert torch.equal(images2, images)


def test_single_view_forward_without_synchronisation():
    sc, cam = S.make_scene(10_000, 0), S.workload_camera("c1")
    say("single-view no-sync forward")
    params = to_gpu(sc)
    rz = B.Rasterizer(cam)
    img, tf, last = rz.forward(params)
    img, tf, last = img.clone(), tf.clone(), last.clone()
    need = rz.last_stats["n_instances"]
    img2, tf2, last2 = rz.forward(params, sync=False)
    assert not rz.overflowed()
    assert torch.equal(img2, img) and torch.equal(tf2, tf) and torch.equal(last2, last)
    dl = S.make_dl_dimage(cam.height, cam.width, seed=3).cuda()
    g1 = rz.backward(params, img, last, dl)
    g1 = {k: v.clone() for k, v in g1.items()}
    rz.forward(params, sync=False)
    g2 = rz.backward(params, img, last, dl)
    for k in B.PARAM_NAMES:
        assert rel_l2(g2[k], g1[k]) <= 1e-6, k
    small = B.Rasterizer(cam)
    small._ensure(S.count(sc), need // 2)  # a workspace too small for this view
    small.forward(params, sync=False)
    say("  instances", need, "capacity", small.capacity, "overflow", small.overflowed())
    assert small.overflowed()


def test_forward_without_synchronisation_skips_constant_depth_digits():
    """A scene spread over a very thin depth range: the visible depth keys,
    offset by the smallest, span fewer than 2^16.  Without a depth-bits hint
    the synchronisation-free depth sort (four passes over 31 bits) skips its
    last two passes, taking the span from the device, and the duplication
    reads the sorted ids from the buffer the device noted; with the bits the
    synchronised forward reported (FGS_FORWARD_DEPTH_BITS, what the
    Rasterizer passes) it sorts only those.  Both equal the synchronised
    forward.  A hint four bits short sets bit 1 of the overflow word."""
    sc, cam = S.make_scene(8_000, 6, z_range=(3.0, 3.0005)), S.workload_camera("c1")
    say("no-sync forward, thin depth range")
    params = to_gpu(sc)
    rz = B.Rasterizer(cam)
    img, tf, last = (t.clone() for t in rz.forward(params))
    keys, vals, ranges = sorted_instances(rz)
    c = rz.view("counters", 16).cpu().numpy().view(np.uint32)
    kmin, kmax = int(c[1]), int(c[2])
    say("  visible", rz.last_stats["n_visible"], "depth key span", hex(kmax - kmin))
    assert rz.last_stats["n_visible"] > 256 and (kmax - kmin) >> 16 == 0 and (kmax - kmin) >> 8 != 0
    assert np.array_equal(c[10:12], [0, kmax - kmin])
    bits = rz.last_stats["depth_key_bits"]
    assert bits == (kmax - kmin).bit_length()
    say("  depth_key_bits", bits)
    for label, mode in (("hint", B.no_sync_mode(rz.last_stats)), ("no hint", L.FGS_FORWARD_NO_SYNC)):
        img2, tf2, last2 = torch.empty_like(img), torch.empty_like(tf), torch.empty_like(last)
        B.rasterize_forward_batch(params, [cam], None, rz.settings, rz.workspace, rz.capacity, img2.view(-1),
                                  tf2.view(-1), last2.view(-1), mode=mode)
        assert not rz.overflowed(), label
        assert torch.equal(img2, img) and torch.equal(tf2, tf) and torch.equal(last2, last), label
        keys2, vals2, ranges2 = sorted_instances(rz)
        assert np.array_equal(keys2, keys) and np.array_equal(vals2, vals) and np.array_equal(ranges2, ranges)
    img2, tf2, last2 = torch.empty_like(img), torch.empty_like(tf), torch.empty_like(last)
    B.rasterize_forward_batch(params, [cam], None, rz.settings, rz.workspace, rz.capacity, img2.view(-1),
                              tf2.view(-1), last2.view(-1),
                              mode=L.FGS_FORWARD_NO_SYNC | L.FGS_FORWARD_DEPTH_BITS(bits - 4))
    torch.cuda.synchronize()
    assert int(rz.view("counters", 8).cpu()[7]) == 2


def test_batch_without_synchronisation_and_overflow_flag():
    sc = S.batch_scene(20_000, 4)
    cams = small_views()
    say("no-sync batch")
    params = to_gpu(sc)
    br = B.BatchRasterizer(cams)
    images, t_finals, lasts = br.forward(params)
    ref_img, ref_last = images.clone(), lasts.clone()
    need = br.last_stats["n_instances"]
    images, t_finals, lasts = br.forward(params, mode=L.FGS_FORWARD_NO_SYNC)
    torch.cuda.synchronize()
    c = br.counters().cpu()
    assert int(c[7]) == 0 and int(c[4]) == need
    assert torch.equal(images, ref_img) and torch.equal(lasts, ref_last)
    # too small a capacity: the step completes, flags the overflow and writes
    # no instance beyond the capacity
    small = B.BatchRasterizer(cams)
    small.ensure(S.count(sc), need // 2)
    small.forward(params, mode=L.FGS_FORWARD_NO_SYNC)
    torch.cuda.synchronize()
    c = small.counters().cpu()
    say("  instances", need, "capacity", need // 2, "overflow flag", int(c[7]))
    assert int(c[7]) == 1 and int(c[4]) == need and int(c[6]) == need // 2


def test_graph_captured_batched_step_matches_eager():
    """forward (no synchronisation) + L1 + backward + Adam captured once and
    replayed; each replay is checked against the same step run eagerly."""
    sc = S.batch_scene(20_000, 5)
    cams = small_views()
    say("graph capture")
    npix = sum(B.view_pixels(cams))
    target = torch.rand(3 * npix, generator=torch.Generator().manual_seed(3)).cuda()
    pe, pg = to_gpu(sc), to_gpu(sc)
    be, bg = B.BatchRasterizer(cams), B.BatchRasterizer(cams)
    oe, og = FusedAdam(pe, S.ADAM_LR), FusedAdam(pg, S.ADAM_LR, device_step=True)
    dle, dlg = torch.empty(3 * npix, device="cuda"), torch.empty(3 * npix, device="cuda")
    ge = {k: torch.empty_like(v) for k, v in pe.items()}
    gg = {k: torch.empty_like(v) for k, v in pg.items()}
    for r in (be, bg):  # size the workspaces outside the capture
        r.forward(pe if r is be else pg)
        r.ensure(S.count(sc), int(r.last_stats["n_instances"] * 1.5))

    def step(r, p, o, dl, g):
        images, _, _ = r.forward(p, mode=L.FGS_FORWARD_NO_SYNC)
        B.l1_loss_backward(images, target, dl)
        r.backward(p, dl, g)
        o.step(g)

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step(bg, pg, og, dlg, gg)  # warm-up on the side stream, as torch's capture expects
    torch.cuda.current_stream().wait_stream(s)
    step(be, pe, oe, dle, ge)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step(bg, pg, og, dlg, gg)
    for rep in range(3):
        # both start the step from the same state (gradient atomics make the
        # two runs differ in the last bits, which would compound over steps)
        for k in pe:
            pg[k].copy_(pe[k])
            og.exp_avg[k].copy_(oe.exp_avg[k])
            og.exp_avg_sq[k].copy_(oe.exp_avg_sq[k])
        p0 = {k: v.clone() for k, v in pe.items()}
        step(be, pe, oe, dle, ge)
        graph.replay()
        torch.cuda.synchronize()
        assert int(bg.counters().cpu()[7]) == 0
        assert int(og.state[0].cpu()) == oe.t, "the device step counter advances with every replay"
        assert torch.equal(bg.images, be.images), rep
        for k in pe:
            em = rel_l2(og.exp_avg[k], oe.exp_avg[k])
            ed = rel_l2(pg[k] - p0[k], pe[k] - p0[k])
            assert em <= 1e-5 and ed <= 1e-3, (rep, k, em, ed)
        say(f"  replay {rep} (t = {oe.t}): images equal, moments within 1e-5, steps within 1e-3")


def test_graph_replay_matches_oracle_step():
    """A captured step (forward without synchronisation, backward of a fixed
    upstream gradient, Adam with the device step counter) replayed from a
    reset state, each replay against the oracle-driven step: render64
    gradients of every view summed, one adam64 step at t = 3 from seeded
    moments.  Eager library work and synchronisations run between the
    replays."""
    sc = S.batch_scene(20_000, 5)
    cams = small_views()
    say("graph replay vs oracle")
    dls, g_ref, exempt = [], None, []
    for k, cam in enumerate(cams):
        ref = O.render64(sc, cam, mask_borderline=True, dl_dimage=S.make_dl_dimage(cam.height, cam.width, 40 + k))
        dls.append(ref["dl_used"].float())
        g_ref = ref["grads"] if g_ref is None else {n: g_ref[n] + ref["grads"][n] for n in g_ref}
        exempt.append(ref["clip_border"].numpy())
    scales = {}
    for k, g in g_ref.items():
        rows = g.T if g.dim() == 2 else g[:, None]
        live = (rows != 0).any(dim=1)
        scales[k] = float(torch.sqrt((rows[live] ** 2).mean())) if bool(live.any()) else 1e-6
    m0, v0 = S.make_adam_state({k: tuple(v.shape) for k, v in sc.items()}, scales, seed=4)
    params = to_gpu(sc)
    p_start = {k: v.clone() for k, v in params.items()}
    br = B.BatchRasterizer(cams)
    br.forward(params)  # sizes the workspace outside the capture
    br.ensure(S.count(sc), int(br.last_stats["n_instances"] * 1.5))
    opt = FusedAdam(params, S.ADAM_LR, device_step=True)
    dl = torch.cat([d.reshape(-1) for d in dls]).cuda()
    grads = {k: torch.empty_like(v) for k, v in params.items()}

    def reset():
        for k in params:
            params[k].copy_(p_start[k])
            opt.exp_avg[k].copy_(m0[k])
            opt.exp_avg_sq[k].copy_(v0[k])
        opt.state.zero_()
        opt.state[0] = 2  # the replayed step is t = 3

    def step():
        br.forward(params, mode=L.FGS_FORWARD_NO_SYNC)
        br.backward(params, dl, grads)
        opt.step(grads)

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()  # warm-up on the side stream, as torch's capture expects
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    other = B.Rasterizer(cams[0])
    for rep in range(3):
        reset()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert int(br.counters().cpu()[7]) == 0 and int(opt.state[0].cpu()) == 3
        for k in B.PARAM_NAMES:
            check_adam(f"replay {rep}", k, p_start[k], params[k], opt.exp_avg[k], opt.exp_avg_sq[k], g_ref[k],
                       m0[k], v0[k], 3, S.ADAM_LR[k])
        # eager library work between the replays
        other.forward(p_start)
        torch.cuda.synchronize()


DYNAMIC = {
    # n, timesteps, camera, SH storage, comparison windows (None: whole frame)
    "small": (3_000, 3, lambda: S.identity_camera(96, 72, 100.0, bg=(0.1, 0.2, 0.3)), "f32", None),
    # the dynamic workload: 1M Gaussians, 8 timesteps of 1280x720, bfloat16 SH;
    # one 64x64 window per timestep, alternately at the centre and the bottom edge
    "c5": (1_000_000, 8, lambda: S.identity_camera(1280, 720, 1000.0), "bf16",
           [(608, 328, 672, 392), (1076, 656, 1140, 720)]),
}


@pytest.mark.parametrize("case", list(DYNAMIC))
def test_dynamic_gaussians_match_oracle_and_chain_rule(case):
    n, n_t, make_cam, sh, windows = DYNAMIC[case]
    sc = S.make_scene(n, 6)
    if sh == "bf16":
        sc = {k: (v.bfloat16().float() if k in ("sh_dc", "sh_rest") else v) for k, v in sc.items()}
    motion = S.make_motion(n, 6)
    cam = make_cam()
    times = S.timesteps(n_t)
    say("dynamic", case, n, "Gaussians", [round(t, 3) for t in times], sh)
    params = to_gpu(sc)
    if sh == "bf16":
        for k in ("sh_dc", "sh_rest"):
            params[k] = params[k].to(torch.bfloat16).contiguous()
    params.update({k: v.cuda() for k, v in motion.items()})
    br = B.BatchRasterizer([cam] * len(times), times=times)
    images, t_finals, lasts = br.forward(params)
    imgs, tfs = br.split(images, 3), br.split(t_finals, 1)
    # per timestep: the means the kernel sees, in float32 in its operation order
    mu0, vel, acc = sc["means"].numpy(), motion["velocity"].numpy(), motion["accel"].numpy()
    g_mean, dls, exempt = [], [], []
    gsum = {k: torch.zeros(v.shape, dtype=torch.float64) for k, v in sc.items()}
    keys, vals, ranges = sorted_instances(br)
    tiles_per_view = ranges.shape[0] // len(times)
    rng = np.random.default_rng(1)
    for k, t in enumerate(times):
        t32 = np.float32(t)
        mu_t = (mu0 + vel * t32) + acc * (t32 * t32)
        sk = dict(sc)
        sk["means"] = torch.from_numpy(mu_t.astype(np.float32))
        # keys of this view's tiles, shifted to local tile ids, entries j = k n + i
        lo = int(np.searchsorted(keys, k * tiles_per_view))
        hi = int(np.searchsorted(keys, (k + 1) * tiles_per_view))
        kv = vals[lo:hi].astype(np.int64)
        assert np.all(kv // n == k)
        view_ranges = ranges[k * tiles_per_view:(k + 1) * tiles_per_view].astype(np.int64)
        if windows is None:
            nom, border = O.keys_ref_banded(sk, cam)
            loc_ranges = view_ranges - lo
            loc_ranges[view_ranges[:, 1] == 0] = 0
            flips = compare_lists(keys[lo:hi] - k * tiles_per_view, (kv % n).astype(np.uint32),
                                  loc_ranges.astype(np.uint32), nom, border, depth=nom["depth"])
            assert flips <= len(border)
            crop = None
        else:
            # sampled tile lists of this timestep, bit-exact off the borderline band
            sample = sorted(set(rng.integers(0, tiles_per_view, 4).tolist()) | {tiles_per_view // 2})
            lists = O.tile_lists_for(sk, cam, sample, delta=1e-3)
            for tl in sample:
                ref_list, band = lists[tl]
                s0, e0 = view_ranges[tl]
                got = [int(g) % n for g in vals[s0:e0].tolist()]
                assert all(int(g) // n == k for g in vals[s0:e0].tolist())
                assert [g for g in got if g not in band] == [g for g in ref_list.tolist() if g not in band], (k, tl)
            crop = windows[k % len(windows)]
        x0, y0, x1, y1 = crop if crop is not None else (0, 0, cam.width, cam.height)
        ref = O.render64(sk, cam, crop=crop, mask_borderline=True,
                         dl_dimage=S.make_dl_dimage(y1 - y0, x1 - x0, seed=30 + k))
        check_image(f"t={t:.3f}", imgs[k][:, y0:y1, x0:x1], ref, t_final=tfs[k][y0:y1, x0:x1])
        dl = torch.zeros(3, cam.height, cam.width)
        dl[:, y0:y1, x0:x1] = ref["dl_used"].float()
        dls.append(dl)
        exempt.append(ref["clip_border"].numpy())
        g_mean.append(ref["grads"]["means"].double())
        for name in gsum:
            if name != "means":
                gsum[name] += ref["grads"][name].double()
    grads = {k: torch.empty_like(v) for k, v in params.items()}
    br.backward(params, torch.cat([d.reshape(-1) for d in dls]).cuda(), grads)
    torch.cuda.synchronize()
    want = {
        "means": sum(g_mean),
        "velocity": sum(t * g for t, g in zip(times, g_mean)),
        "accel": sum(t * t * g for t, g in zip(times, g_mean)),
    }
    want.update({k: v for k, v in gsum.items() if k != "means"})
    bf = ("sh_dc", "sh_rest") if sh == "bf16" else ()
    check_grads(f"dynamic {case}", grads, want, names=list(want), exempt=np.concatenate(exempt), bf16_groups=bf,
                rel_tol={k: 2.0 ** -8 for k in bf})


COND4D = {
    # n, timesteps, camera, comparison windows (None: whole frame)
    "small": (3_000, 3, lambda: S.identity_camera(96, 72, 100.0, bg=(0.1, 0.2, 0.3)), None),
    "720p": (200_000, 4, lambda: S.identity_camera(1280, 720, 1000.0), [(608, 328, 672, 392), (1076, 656, 1140, 720)]),
}


@pytest.mark.parametrize("case", list(COND4D))
def test_conditional_4d_gaussians_match_oracle(case):
    """Conditional 4D Gaussians (Sec. 3.4): every timestep is a view whose
    Gaussians are the conditional 3D Gaussians at its time, with opacities
    faded by the marginal factor.  Per timestep: the GPU's float32 depth keys
    within 1e-5 relative of the oracle's float64 conditional depth; tile lists
    against the key reference (whole frame: every list; 720p: sampled tiles)
    in the order of the GPU's keys, exact off the borderline band; the image
    against the FP64 oracle (rendered in that order); then every gradient,
    including those of the time mean, the temporal log-scale and the right
    quaternion, against the oracle's gradients summed over the timesteps."""
    n, n_t, make_cam, windows = COND4D[case]
    sc = S.make_scene(n, 8)
    sc.update(S.make_cond4d(sc, 8))
    cam = make_cam()
    times = S.timesteps(n_t)
    say("conditional 4D", case, n, "Gaussians", [round(t, 3) for t in times])
    params = to_gpu(sc)
    br = B.BatchRasterizer([cam] * n_t, times=times)
    images, t_finals, lasts = br.forward(params)
    imgs, tfs = br.split(images, 3), br.split(t_finals, 1)
    keys, vals, ranges = sorted_instances(br)
    dkeys = br.view("depth_key", n * n_t).cpu().numpy().view(np.float32).reshape(n_t, n)
    ntl = br.view("n_tiles", n * n_t).cpu().numpy().reshape(n_t, n)
    tiles_per_view = ranges.shape[0] // n_t
    rng = np.random.default_rng(2)
    rows = {k: (v.double().T.contiguous() if v.dim() == 2 else v.double()) for k, v in sc.items()}
    dls, g_sum, exempt = [], None, []
    for k, t in enumerate(times):
        vis = ntl[k] != 0
        with torch.no_grad():
            z64 = O.preprocess64(rows, cam, time=t, sh_degree=0)["cam_pos"][:, 2].numpy()
        rel = np.abs(dkeys[k][vis].astype(np.float64) - z64[vis]) / np.abs(z64[vis])
        say(f"  t={t:.3f}: visible {int(vis.sum())}, depth key max rel err {rel.max():.2e}")
        assert rel.max() <= 1e-5
        lo = int(np.searchsorted(keys, k * tiles_per_view))
        hi = int(np.searchsorted(keys, (k + 1) * tiles_per_view))
        kv = vals[lo:hi].astype(np.int64)
        assert np.all(kv // n == k)
        view_ranges = ranges[k * tiles_per_view:(k + 1) * tiles_per_view].astype(np.int64)
        if windows is None:
            nom, border = O.keys_ref_banded(sc, cam, time=t, depth=dkeys[k])
            loc_ranges = view_ranges - lo
            loc_ranges[view_ranges[:, 1] == 0] = 0
            flips = compare_lists(keys[lo:hi] - k * tiles_per_view, (kv % n).astype(np.uint32),
                                  loc_ranges.astype(np.uint32), nom, border, depth=dkeys[k])
            assert flips <= len(border)
            crop = None
        else:
            sample = sorted(set(rng.integers(0, tiles_per_view, 4).tolist()) | {tiles_per_view // 2})
            lists = O.tile_lists_for(sc, cam, sample, delta=1e-3, time=t, depth=dkeys[k])
            for tl in sample:
                ref_list, band = lists[tl]
                s0, e0 = view_ranges[tl]
                got = [int(g) % n for g in vals[s0:e0].tolist()]
                assert [g for g in got if g not in band] == [g for g in ref_list.tolist() if g not in band], (k, tl)
            crop = windows[k % len(windows)]
        x0, y0, x1, y1 = crop if crop is not None else (0, 0, cam.width, cam.height)
        ref = O.render64(sc, cam, crop=crop, time=t, order_keys=dkeys[k], mask_borderline=True,
                         dl_dimage=S.make_dl_dimage(y1 - y0, x1 - x0, seed=50 + k))
        check_image(f"t={t:.3f}", imgs[k][:, y0:y1, x0:x1], ref, t_final=tfs[k][y0:y1, x0:x1])
        dl = torch.zeros(3, cam.height, cam.width)
        dl[:, y0:y1, x0:x1] = ref["dl_used"].float()
        dls.append(dl)
        exempt.append(ref["clip_border"].numpy())
        g_sum = ref["grads"] if g_sum is None else {m: g_sum[m] + ref["grads"][m] for m in g_sum}
    grads = br.backward(params, torch.cat([d.reshape(-1) for d in dls]).cuda())
    torch.cuda.synchronize()
    assert set(g_sum) >= set(B.PARAM_NAMES) | set(B.COND4D_NAMES)
    check_grads(f"conditional 4D {case}", grads, g_sum, names=list(g_sum), exempt=np.concatenate(exempt))


@pytest.mark.parametrize("option", ["queue", "sort8192"])
@pytest.mark.parametrize("case", ["views", "c1", "wide"])
def test_schedule_and_blocking_options_match_the_defaults(case, option):
    """The autotuner's options change no result.  FGS_FLAG_BLEND_QUEUE runs the
    blend's per-tile code as persistent waves that take tiles from one queue
    per XCD; FGS_FLAG_SORT_LARGE_BLOCKS sorts the instances in blocks of 8192
    pairs.  Sorted instances, images, T and last ids are bit-identical to the
    defaults, gradients equal up to the order of their float atomics
    (relative L2 <= 1e-5 per group: float32 sums of up to a few hundred
    terms per Gaussian in another order, two runs of the defaults differ as
    much); run twice (the queues restart every
    launch), for several views, for one, and for 8x8 tiles of three 1920x1080
    views (129600 tiles: 32-bit tile keys)."""
    tile = 16
    if case == "views":
        sc, cams = S.batch_scene(20_000, 4), small_views()
    elif case == "c1":
        sc, cams = S.make_scene(10_000, 0), [S.workload_camera("c1")]
    else:
        sc, tile = S.make_scene(40_000, 9), 8
        cams = [S.identity_camera(1920, 1080, 1500.0, bg=(0.2, 0.3, 0.4))] * 3
    flag = L.FGS_FLAG_BLEND_QUEUE if option == "queue" else L.FGS_FLAG_SORT_LARGE_BLOCKS
    say("option", option, case)
    params = to_gpu(sc)
    npix = sum(B.view_pixels(cams))
    dl = torch.randn(3 * npix, generator=torch.Generator().manual_seed(7)).mul_(1e-3).cuda()
    out = {}
    for sched, flags in (("default", 0), (option, flag)):
        br = B.BatchRasterizer(cams, settings=B.default_settings(flags=flags, tile=tile))
        for rep in range(2):
            imgs, tfs, lasts = (t.clone() for t in br.forward(params))
            torch.cuda.synchronize()
            assert br.layout().inst_key_bytes == (4 if case == "wide" else 2)
            inst = sorted_instances(br)
            grads = {k: v.clone() for k, v in br.backward(params, dl).items()}
            torch.cuda.synchronize()
            out[(sched, rep)] = (imgs, tfs, lasts, grads, inst)
    noise = max(rel_l2(out[("default", 1)][3][k], out[("default", 0)][3][k]) for k in B.PARAM_NAMES)
    say(f"  two runs of the defaults: worst gradient rel L2 {noise:.2e}")
    for rep in range(2):
        gi, gt, gl, gg, ginst = out[("default", 0)]
        qi, qt, ql, qg, qinst = out[(option, rep)]
        assert all(np.array_equal(a, b) for a, b in zip(qinst, ginst)), rep
        assert torch.equal(qi, gi) and torch.equal(qt, gt) and torch.equal(ql, gl), rep
        worst = max(rel_l2(qg[k], gg[k]) for k in B.PARAM_NAMES)
        say(f"  rep {rep}: instances and images equal, worst gradient rel L2 {worst:.2e}")
        assert worst <= 1e-5


def accum_state(rz, vn):
    """(accum and marks all zero, the counters' accumulator-state words)."""
    acc = rz.view("accum", 9 * vn, dtype=torch.float32)
    marks = rz.view("marks", vn, dtype=torch.uint8)
    words = rz.view("counters", 14)[12:14].cpu().numpy().view(np.uint32)
    return bool((acc == 0).all().item() and (marks == 0).all().item()), (int(words[0]), int(words[1]))


ACCUM_CLEAN = 0x5A3C0F81


@pytest.mark.gpu
@pytest.mark.parametrize("form", ["views", "dynamic", "cond4d", "fused"])
def test_accumulators_kept_zero_between_backwards(form):
    """FGS_FLAG_KEEP_ACCUM_ZERO (the binding's default for the workspaces it
    owns): the chain rule clears every accumulator row and mark it reads and
    the next backward skips the clear.  Three backward passes in a row (with
    changing image gradients; fused: three training steps) equal those of a
    rasterizer that clears at every call, up to the order of the float atomics
    (relative L2 <= 1e-5); after each, accum and marks are all zero and the
    state words read {marker, tag}; without the flag the state words stay
    cleared.  The fused form compares Adam's first moment after one step
    from fresh moments, (1 - beta1) times the gradient."""
    if form == "fused":
        sc, cams = S.make_scene(30_000, 3), [S.workload_camera("c1")]
    else:
        sc, cams = S.batch_scene(20_000, 4), small_views()
    n = int(sc["opacity_logits"].shape[0])
    times = None
    if form == "dynamic":
        sc.update(S.make_motion(n, 4))
        times = S.timesteps(len(cams))
    elif form == "cond4d":
        sc.update(S.make_cond4d(sc, 4))
        times = S.timesteps(len(cams))
    say("keep accum zero", form, n, "Gaussians", len(cams), "views")
    npix = sum(B.view_pixels(cams))
    dls = [torch.randn(3 * npix, generator=torch.Generator().manual_seed(s)).mul_(1e-3).cuda() for s in (1, 2, 1)]
    vn = n * len(cams)
    out = {}
    for keep in (False, True):
        params = to_gpu(sc)
        if form == "fused":
            rz = B.Rasterizer(cams[0], keep_accum_zero=keep)
            res = []
            for call, dl in enumerate(dls):
                params = to_gpu(sc)
                opt = FusedAdam(params, S.ADAM_LR)
                image, _, last = rz.forward(params)
                rz.backward_adam(params, image, last, dl.view_as(image), opt)
                torch.cuda.synchronize()
                res.append({k: v.clone() for k, v in opt.exp_avg.items()})
                zero, words = accum_state(rz, vn)
                say(f"  keep={keep} step {call}: accum and marks zero {zero}, state words {words[0]:#x}")
                assert (zero and words[0] == ACCUM_CLEAN) if keep else words == (0, 0)
        else:
            br = B.BatchRasterizer(cams, times=times, keep_accum_zero=keep)
            br.forward(params)
            res = []
            for call, dl in enumerate(dls):
                res.append({k: v.clone() for k, v in br.backward(params, dl).items()})
                torch.cuda.synchronize()
                zero, words = accum_state(br, vn)
                say(f"  keep={keep} backward {call}: accum and marks zero {zero}, state words {words[0]:#x}")
                assert (zero and words[0] == ACCUM_CLEAN) if keep else words == (0, 0)
        out[keep] = res
    for call in range(3):
        worst = max(rel_l2(out[True][call][k], out[False][call][k]) for k in out[True][call])
        say(f"  call {call}: worst rel L2 against clearing at every call {worst:.2e}")
        assert worst <= 1e-5
    # the same image gradient twice: the same gradients
    assert max(rel_l2(out[True][2][k], out[True][0][k]) for k in out[True][0]) <= 1e-5


@pytest.mark.gpu
def test_accumulators_state_survives_a_workspace_regrow():
    """A forward whose instances outgrow the capacity allocates a new workspace,
    whose accumulator state words start cleared: the backward after it clears
    the new accumulators and matches a rasterizer that clears at every call."""
    sc, cams = S.batch_scene(20_000, 4), small_views()
    npix = sum(B.view_pixels(cams))
    dl = torch.randn(3 * npix, generator=torch.Generator().manual_seed(3)).mul_(1e-3).cuda()
    big = dict(sc, log_scales=sc["log_scales"] + 0.7)  # larger splats: more instances
    out = {}
    for keep in (True, False):
        br = B.BatchRasterizer(cams, keep_accum_zero=keep, headroom=1.0)
        br.ensure(20_000, 1024)  # a small workspace: the first forward regrows it too
        params = to_gpu(sc)
        br.forward(params)
        br.backward(params, dl)
        ws0, cap0 = br.workspace.data_ptr(), br.capacity
        params = to_gpu(big)
        br.forward(params)
        grown = br.capacity > cap0
        out[keep] = {k: v.clone() for k, v in br.backward(params, dl).items()}
        torch.cuda.synchronize()
        if keep:
            zero, words = accum_state(br, 20_000 * len(cams))
            say(f"  capacity {cap0} -> {br.capacity} (new workspace {br.workspace.data_ptr() != ws0}); "
                f"accum zero {zero}, state {words[0]:#x}")
            assert grown and zero and words[0] == ACCUM_CLEAN
    worst = max(rel_l2(out[True][k], out[False][k]) for k in out[True])
    say(f"  worst rel L2 against clearing at every call {worst:.2e}")
    assert worst <= 1e-5


@pytest.mark.gpu
@pytest.mark.parametrize("n", [3, 200])
def test_forward_without_synchronisation_few_pairs_in_a_large_capacity(n):
    """The radix passes band the chunks that hold pairs (read on the device)
    over the XCDs and leave the grid's other workgroups on their own empty
    chunks: a sync-free forward whose few instances fill fewer chunks than
    there are XCDs, in a workspace sized for far more, equals the synchronised
    forward bit for bit."""
    sc, cam = S.make_scene(n, 5), S.workload_camera("c1")
    params = to_gpu(sc)
    rz = B.Rasterizer(cam)
    rz._ensure(n, 200_000)  # 49 sort chunks of 4096 pairs
    img, tf, last = (t.clone() for t in rz.forward(params))
    need = rz.last_stats["n_instances"]
    img2, tf2, last2 = rz.forward(params, sync=False)
    torch.cuda.synchronize()
    say(f"  {n} Gaussians: {need} instances in a capacity of {rz.capacity}")
    assert need < 8 * 4096 and not rz.overflowed()
    assert torch.equal(img2, img) and torch.equal(tf2, tf) and torch.equal(last2, last)
