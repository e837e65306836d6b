"""The seeded input generator: determinism, layout and distributions."""
import numpy as np
import torch

import oracle as O
import synthetic as S


def test_scene_is_deterministic_and_soa():
    a = S.make_scene(5000, seed=7)
    b = S.make_scene(5000, seed=7)
    c = S.make_scene(5000, seed=8)
    for k in S.PARAM_NAMES:
        assert torch.equal(a[k], b[k])
        assert a[k].dtype == torch.float32 and a[k].is_contiguous()
    assert not torch.equal(a["means"], c["means"])
    assert a["means"].shape == (3, 5000) and a["sh_rest"].shape == (45, 5000)
    assert a["opacity_logits"].shape == (5000,)


def test_scene_distributions():
    s = S.make_scene(200_000, seed=0)
    m = s["means"].double()
    assert m[:2].min() >= -1 and m[:2].max() <= 1 and m[2].min() >= 2 and m[2].max() <= 6
    assert abs(float(s["log_scales"].double().mean()) + 4) < 0.01
    assert abs(float(s["log_scales"].double().std()) - 0.5) < 0.01
    assert torch.allclose(s["quats"].double().norm(dim=0), torch.ones(200_000, dtype=torch.float64), atol=1e-6)
    assert abs(float(s["sh_dc"].double().std()) - 0.3) < 0.01
    assert abs(float(s["sh_rest"].double().std()) - 0.05) < 0.001


def test_l1_gradient_matches_autograd_of_mean_abs():
    img = torch.rand(3, 8, 9, dtype=torch.float64)
    tgt = torch.rand(3, 8, 9, dtype=torch.float64)
    tgt[0, 0, 0] = img[0, 0, 0]  # sign(0) = 0
    loss, g = O.l1_loss_grad64(img, tgt)
    x = img.clone().requires_grad_(True)
    ref = (x - tgt).abs().mean()
    ref.backward()
    assert abs(loss - float(ref)) <= 1e-15
    assert torch.equal(g, x.grad)
    assert g[0, 0, 0] == 0
