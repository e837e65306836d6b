"""GPU tests of the fused backward + Adam entry point and of the precision
form (SH coefficients and their gradients stored as bfloat16).

The fused call must reproduce fgs_rasterize_backward followed by
fgs_adam_step bit for bit (same gradient arithmetic, same Adam element
update, every zero-gradient parameter updated too: Sec. 3.3 "Fusing Backward
and Optimizer").  The precision form is checked against the FP64 oracle run on
the bfloat16-rounded coefficients: every other input is identical, and all
blending and accumulation stays FP32, so the image bar is the FP32 one; the
SH gradients carry one bfloat16 rounding (relative 2^-8 at most).
"""
import numpy as np
import pytest
import torch

import oracle as O
import synthetic as S
from paper_2602_09999_amd import binding as B
from paper_2602_09999_amd.autograd import FusedAdam
from tests.gpu_util import check_grads, check_image, say, to_gpu

pytestmark = pytest.mark.gpu

BF16_REL = 2.0 ** -8  # one round-to-nearest bfloat16 rounding, relative
F64 = torch.float64

CASES = {
    "c1": lambda: (S.make_scene(10_000, 0), S.workload_camera("c1")),
    # n % 4 != 0: the four-Gaussian vector path falls back to per-element code
    "ragged_n": lambda: (S.make_scene(2_999, 5), S.identity_camera(90, 70, 100.0, bg=(0.3, 0.1, 0.6))),
}
SH = ("sh_dc", "sh_rest")


def rel_l2(a, b):
    a = a.double().cpu()
    b = b.double().cpu()
    return float((a - b).norm()) / max(float(b.norm()), 1e-30)


def bf16_scene(sc):
    """The scene with its SH coefficients rounded to bfloat16 (kept float32)."""
    out = dict(sc)
    for k in SH:
        out[k] = sc[k].bfloat16().float()
    return out


def gpu_params(sc, sh_dtype):
    p = to_gpu(sc)
    for k in SH:
        p[k] = p[k].to(sh_dtype).contiguous()
    return p


def one_tile_scene(n, seed, cam):
    """Small splats whose opacity-aware rectangles stay inside one 16x16 tile:
    centres within 2 px of a tile centre, 2D extent about 2 px.  Each Gaussian
    then gets its gradient from a single tile, i.e. one atomic add onto zero,
    so the accumulated gradients do not depend on the order of atomics."""
    sc = S.make_scene(n, seed, log_scale_mean=-6.5)
    g = torch.Generator().manual_seed(seed + 17)
    tx = torch.randint(0, cam.width // 16, (n,), generator=g)
    ty = torch.randint(0, cam.height // 16, (n,), generator=g)
    px = tx * 16 + 8 + (torch.rand(n, generator=g) * 4 - 2)
    py = ty * 16 + 8 + (torch.rand(n, generator=g) * 4 - 2)
    z = sc["means"][2].clamp(3.0, 6.0)
    sc["log_scales"] = sc["log_scales"].clamp(max=-5.5)
    sc["means"] = torch.stack([(px - cam.cx) * z / cam.fx, (py - cam.cy) * z / cam.fy, z]).float().contiguous()
    return sc


def train_both(sc, cam, sh_dtype, steps):
    """Steps of (backward; Adam) and of the fused call from the same start."""
    target = S.make_target(cam.height, cam.width, seed=3).cuda()
    pa = gpu_params(sc, sh_dtype)
    p0 = {k: v.clone() for k, v in pa.items()}
    pb = {k: v.clone() for k, v in pa.items()}
    ra, rb = B.Rasterizer(cam), B.Rasterizer(cam)
    oa, ob = FusedAdam(pa, S.ADAM_LR), FusedAdam(pb, S.ADAM_LR)
    touched = []
    for _ in range(steps):
        ia, _, la = ra.forward(pa)
        ib, _, lb = rb.forward(pb)
        da, db = torch.empty_like(ia), torch.empty_like(ib)
        B.l1_loss_backward(ia, target, da)
        B.l1_loss_backward(ib, target, db)
        grads = ra.backward(pa, ia, la, da)
        oa.step(grads)
        rb.backward_adam(pb, ib, lb, db, ob)
        torch.cuda.synchronize()
        touched.append(int((grads["opacity_logits"] != 0).sum()))
    assert oa.t == ob.t == steps
    return p0, pa, pb, oa, ob, ra, touched


@pytest.mark.parametrize("sh_dtype", [torch.float32, torch.bfloat16], ids=["f32", "bf16"])
@pytest.mark.parametrize("n", [4096, 2999])
def test_fused_backward_adam_bit_exact_when_accumulation_is_order_free(n, sh_dtype):
    cam = S.identity_camera(128, 96, 130.0, bg=(0.2, 0.3, 0.4))
    sc = one_tile_scene(n, 11, cam)
    say("fused exact", n, sh_dtype)
    p0, pa, pb, oa, ob, ra, touched = train_both(sc, cam, sh_dtype, 3)
    nt = ra.view("n_tiles", n).cpu().numpy()
    say(f"  Gaussians per tile count {np.bincount(nt, minlength=3)[:3].tolist()}, with a gradient {touched}")
    assert nt.max() == 1 and (nt == 1).sum() > n // 2, "the scene must put every Gaussian in one tile"
    assert min(touched) > n // 4
    for k in B.PARAM_NAMES:
        assert torch.equal(pa[k], pb[k]), (k, float((pa[k].float() - pb[k].float()).abs().max()))
        assert torch.equal(oa.exp_avg[k], ob.exp_avg[k]), k
        assert torch.equal(oa.exp_avg_sq[k], ob.exp_avg_sq[k]), k
        assert not torch.equal(pa[k], p0[k]), k


@pytest.mark.parametrize("sh_dtype", [torch.float32, torch.bfloat16], ids=["f32", "bf16"])
@pytest.mark.parametrize("case", list(CASES))
def test_fused_backward_adam_matches_on_overlapping_scenes(case, sh_dtype):
    """Gaussians spanning several tiles accumulate with float atomics in a
    run-dependent order, so the two paths agree to rounding: the moments to
    1e-5 relative; a parameter whose gradient is near zero may take an Adam
    step of either sign, so the parameter displacement is compared in L2."""
    sc, cam = CASES[case]()
    say("fused overlap", case, sh_dtype)
    p0, pa, pb, oa, ob, ra, touched = train_both(sc, cam, sh_dtype, 2)
    say("  with a gradient", touched)
    for k in B.PARAM_NAMES:
        em = rel_l2(ob.exp_avg[k], oa.exp_avg[k])
        ev = rel_l2(ob.exp_avg_sq[k], oa.exp_avg_sq[k])
        ed = rel_l2(pb[k].float() - p0[k].float(), pa[k].float() - p0[k].float())
        say(f"  {k:15s} m {em:.1e} v {ev:.1e} displacement {ed:.1e}")
        assert em <= 1e-5 and ev <= 1e-5, (k, em, ev)
        assert ed <= (2e-2 if k in SH and sh_dtype == torch.bfloat16 else 1e-3), (k, ed)


@pytest.mark.parametrize("case", list(CASES))
def test_bf16_sh_forward_and_backward_match_oracle(case):
    sc, cam = CASES[case]()
    say("bf16 sh", case)
    scb = bf16_scene(sc)
    ref = O.render64(scb, cam, dl_dimage=S.make_dl_dimage(cam.height, cam.width, seed=7), mask_borderline=True)
    params = gpu_params(sc, torch.bfloat16)
    assert torch.equal(params["sh_rest"].float().cpu(), scb["sh_rest"])
    rz = B.Rasterizer(cam)
    image, t_final, last = rz.forward(params)
    grads = rz.backward(params, image, last, ref["dl_used"].float().cuda())
    torch.cuda.synchronize()
    check_image(f"bf16 {case}", image, ref, t_final=t_final)
    for k in SH:
        assert grads[k].dtype == torch.bfloat16
    # SH gradients: one bfloat16 rounding of a float32-accurate value
    check_grads(f"bf16 {case}", grads, ref["grads"], exempt=ref["clip_border"].numpy(), bf16_groups=SH,
                rel_tol={k: BF16_REL for k in SH})


def test_adam_bf16_parameters_match_fp64_update():
    say("adam bf16")
    gen = torch.Generator().manual_seed(1)
    sizes = [4_096, 1_001, 45 * 257]
    lrs = [5e-3, 5e-3, 2.5e-2]
    p0 = [torch.randn(s, generator=gen).bfloat16() for s in sizes]
    ps = [p.cuda() for p in p0]
    ms = [torch.zeros(s, device="cuda") for s in sizes]
    vs = [torch.zeros(s, device="cuda") for s in sizes]
    rp = [p.double() for p in p0]
    rm = [torch.zeros(s, dtype=F64) for s in sizes]
    rv = [torch.zeros(s, dtype=F64) for s in sizes]
    worst = 0
    for step in range(1, 5):
        gr = [torch.randn(s, generator=gen).bfloat16() for s in sizes]
        gr[0][::3] = 0.0
        B.adam_step([(ps[i], gr[i].cuda(), ms[i], vs[i], lrs[i]) for i in range(3)], step)
        torch.cuda.synchronize()
        for i in range(3):
            p64, rm[i], rv[i] = O.adam64(rp[i], gr[i].double(), rm[i], rv[i], step, lrs[i])
            # the stored parameter is bfloat16: round the FP64 update, then continue from it
            rp[i] = p64.to(torch.bfloat16).double()
            got = ps[i].cpu().double()
            # a rounding boundary between the FP32 and FP64 updates moves the
            # result by at most one bfloat16 step (2^-7 relative)
            ulp = torch.maximum(rp[i].abs(), got.abs()) * 2.0 ** -7
            d = (got - rp[i]).abs()
            assert bool((d <= ulp * 1.0001).all()), (step, i)
            worst = max(worst, int((d > 0).sum()))
            # continue both from the GPU's parameters so differences do not compound
            rp[i] = got
    say("  elements one bfloat16 step off the FP64 update (worst step):", worst)
    for i in range(3):
        assert rel_l2(ms[i], rm[i]) <= 1e-6
        assert rel_l2(vs[i], rv[i]) <= 1e-6


@pytest.mark.parametrize("case", list(CASES))
def test_precision_form_fp64_conic_keys_and_image(case):
    """Precision form: bfloat16 SH plus the float64 determinant/inverse of the
    2x2 covariance.  Keys stay bit-exact against the key reference taking the
    same float64 steps; the image against the FP64 oracle."""
    from tests.gpu_util import compare_lists, sorted_instances
    sc, cam = CASES[case]()
    say("precision form", case)
    st = B.default_settings(flags=1)
    rz = B.Rasterizer(cam, settings=st)
    params = gpu_params(sc, torch.bfloat16)
    image, t_final, last = rz.forward(params)
    torch.cuda.synchronize()
    keys, vals, ranges = sorted_instances(rz)
    nom, border = O.keys_ref_banded(sc, cam, fp64_conic=True)
    flips = compare_lists(keys, vals, ranges, nom, border, depth=nom["depth"])
    say("  instances", len(keys), "borderline pairs", len(border), "flipped", flips)
    assert flips <= len(border)
    # the conic of the float64 path against the reference's float64 steps (the
    # float32 exp of the scales may differ by an ulp between the two sides)
    n = S.count(sc)
    rec = rz.view("rec", 16 * n, dtype=torch.float32).cpu().numpy().reshape(n, 16)
    vis = rz.view("n_tiles", n).cpu().numpy() > 0
    ref_con = np.stack([nom["record"][k][vis] for k in ("a", "b", "c")], 1).astype(np.float64)
    e = (np.abs(rec[vis, 4:7] - ref_con) / np.abs(ref_con).max(1, keepdims=True)).max()
    say("  conic max relative difference to the reference's float64 path", float(e))
    assert e < 1e-4
    ref = O.render64(bf16_scene(sc), cam)
    check_image(f"precision form {case}", image, ref, t_final=t_final)
