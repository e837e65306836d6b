"""Pins of the FP32 key reference (oracle.keys32).

* the canonical (tile, depth, index) order and the tile ranges against a
  brute-force ``sorted()`` of Python tuples;
* the exact per-tile test against a library box-constrained minimiser;
* conservativeness: every Gaussian whose FP64 alpha (oracle.render64's
  preprocess) reaches tau_alpha at a pixel is in that pixel's tile list;
* the FP32 record against the FP64 preprocess.
"""
import numpy as np
import pytest
import torch
from scipy.optimize import minimize

import oracle as O
from oracle import keys32 as K
import synthetic as S

F64 = torch.float64


def rows64(sc):
    return {k: (v.to(F64).T.contiguous() if v.dim() == 2 else v.to(F64)) for k, v in sc.items()}


def test_depth_key_identity_camera_is_z_exactly():
    sc = S.make_scene(1000, seed=3)
    cam = S.workload_camera("c1")
    assert np.array_equal(O.depth_key32(sc["means"], cam), sc["means"][2].numpy())


def test_sort_and_ranges_match_brute_force_tuples():
    sc = S.make_scene(300, seed=12)
    sc["means"][2, 10:40] = sc["means"][2, 5]      # many exact depth ties
    cam = S.identity_camera(100, 70, 90.0)          # ragged tile grid (7 x 5 tiles, partial)
    ref = O.keys_ref(sc, cam, tile=16)
    rec = ref["record"]
    tx0, ty0, tx1, ty1, ne = K.tile_rect(rec, 100, 70, 16)
    tiles_x = ref["tiles_x"]
    tuples = []
    for g in range(300):
        if not ne[g]:
            continue
        for ty in range(ty0[g], ty1[g] + 1):
            for tx in range(tx0[g], tx1[g] + 1):
                q = K.tile_min_q(rec["mx"][g:g + 1], rec["my"][g:g + 1], rec["a"][g:g + 1], rec["b"][g:g + 1],
                                 rec["c"][g:g + 1], np.array([tx]), np.array([ty]), 100, 70, 16)[0]
                if q <= rec["thr"][g]:
                    tuples.append((ty * tiles_x + tx, int(rec["depth"][g:g + 1].view(np.uint32)[0]), g))
    tuples.sort()
    assert [t[0] for t in tuples] == ref["keys"].tolist()
    assert [t[2] for t in tuples] == ref["vals"].tolist()
    lists = {}
    for i, t in enumerate(tuples):
        lists.setdefault(t[0], []).append(i)
    for tile in range(ref["ranges"].shape[0]):
        s, e = ref["ranges"][tile]
        if tile in lists:
            assert (s, e) == (lists[tile][0], lists[tile][-1] + 1)
        else:
            assert s == e == 0
    assert np.array_equal(np.bincount(ref["vals"], minlength=300), ref["n_tiles"])


def test_tile_min_matches_box_constrained_minimiser():
    rng = np.random.default_rng(1)
    for _ in range(300):
        A = rng.normal(size=(2, 2)) * rng.uniform(0.5, 12)
        cov = A @ A.T + 0.3 * np.eye(2)
        inv = np.linalg.inv(cov)
        a, b, c = (np.float32(inv[0, 0]), np.float32(inv[0, 1]), np.float32(inv[1, 1]))
        mx, my = np.float32(rng.uniform(-30, 90)), np.float32(rng.uniform(-30, 90))
        tx, ty = int(rng.integers(0, 4)), int(rng.integers(0, 4))
        q32 = K.tile_min_q(np.array([mx]), np.array([my]), np.array([a]), np.array([b]), np.array([c]),
                           np.array([tx]), np.array([ty]), 60, 60, 16)[0]
        x0, x1 = tx * 16 + 0.5, min(tx * 16 + 15, 59) + 0.5
        y0, y1 = ty * 16 + 0.5, min(ty * 16 + 15, 59) + 0.5
        Q = np.array([[a, b], [b, c]], dtype=np.float64)
        fun = lambda p: (p - [mx, my]) @ Q @ (p - [mx, my])
        jac = lambda p: 2 * Q @ (p - [mx, my])
        best = min(minimize(fun, x0=np.array(s), jac=jac, bounds=[(x0, x1), (y0, y1)], method="L-BFGS-B",
                            options={"ftol": 1e-15, "gtol": 1e-12}).fun
                   for s in [((x0 + x1) / 2, (y0 + y1) / 2), (x0, y0), (x1, y1), (x0, y1), (x1, y0)])
        assert abs(float(q32) - best) <= 1e-4 * max(1.0, best), (q32, best)


@pytest.mark.parametrize("seed,cam_kind", [(0, "c1"), (1, "offcentre")])
def test_tile_lists_cover_every_reaching_gaussian(seed, cam_kind):
    sc = S.make_scene(3000, seed=seed)
    cam = S.workload_camera("c1") if cam_kind == "c1" else S.identity_camera(200, 150, 230.0, cx=80.0, cy=60.0)
    ref = O.keys_ref(sc, cam)
    pre = {k: (v.detach() if torch.is_tensor(v) else v) for k, v in O.preprocess64(rows64(sc), cam).items()}
    tiles_x = ref["tiles_x"]
    members = {}
    for t in range(ref["ranges"].shape[0]):
        s, e = ref["ranges"][t]
        members[t] = set(ref["vals"][s:e].tolist())
    vi = torch.nonzero(pre["valid"]).flatten()
    m, c, o = pre["mean2d"][vi], pre["conic"][vi], pre["opacity"][vi]
    tau = O.DEFAULT_SETTINGS.tau_alpha
    missing = 0
    for py in range(0, cam.height, 3):
        for px in range(0, cam.width, 3):
            dx, dy = px + 0.5 - m[:, 0], py + 0.5 - m[:, 1]
            alpha = o * torch.exp(-0.5 * (c[:, 0] * dx * dx + 2 * c[:, 1] * dx * dy + c[:, 2] * dy * dy))
            reach = set(vi[alpha >= tau * (1 + 1e-3)].tolist())
            tile = (py // 16) * tiles_x + (px // 16)
            missing += len(reach - members[tile])
    assert missing == 0


def test_record32_agrees_with_fp64_preprocess():
    sc = S.make_scene(5000, seed=2)
    cam = S.workload_camera("c1")
    rec = K.record32(sc, cam)
    pre = {k: (v.detach().numpy() if torch.is_tensor(v) else v) for k, v in O.preprocess64(rows64(sc), cam).items()}
    assert np.array_equal(rec["valid"], pre["valid"])
    v = rec["valid"]
    rel = lambda a, b: np.abs(a - b) / np.maximum(np.abs(b), 1e-3)
    assert rel(rec["mx"][v], pre["mean2d"][v, 0]).max() < 1e-5
    assert rel(rec["my"][v], pre["mean2d"][v, 1]).max() < 1e-5
    for i, k in enumerate("abc"):
        assert (np.abs(rec[k][v] - pre["conic"][v, i]) / np.abs(pre["conic"][v]).max(1)).max() < 1e-4
    assert rel(rec["thr"][v], pre["thr"][v]).max() < 1e-4
    assert rel(rec["ext_x"][v], pre["extent"][v, 0]).max() < 1e-4


def test_banded_reference_brackets_nominal():
    sc = S.make_scene(10_000, seed=0)
    cam = S.workload_camera("c1")
    nom, border = O.keys_ref_banded(sc, cam, delta=1e-3)
    assert len(border) < 0.01 * len(nom["keys"])
    tight = O.keys_ref(sc, cam, thr_scale=1 - 1e-3, cull_slack=-1e-3)
    loose = O.keys_ref(sc, cam, thr_scale=1 + 1e-3, cull_slack=1e-3)
    p_nom = set(zip(nom["keys"].tolist(), nom["vals"].tolist()))
    p_t = set(zip(tight["keys"].tolist(), tight["vals"].tolist()))
    p_l = set(zip(loose["keys"].tolist(), loose["vals"].tolist()))
    assert p_t <= p_nom <= p_l


def test_tile_lists_for_matches_full_reference():
    sc = S.make_scene(4000, seed=6)
    cam = S.identity_camera(160, 120, 150.0)
    ref = O.keys_ref(sc, cam)
    tiles = [0, 7, 23, 40, 79]
    lists = O.tile_lists_for(sc, cam, tiles)
    for t in tiles:
        s, e = ref["ranges"][t]
        assert np.array_equal(lists[t], ref["vals"][s:e])
