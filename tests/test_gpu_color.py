"""Per-Gaussian colour covariance (FisherRF integration) on the GPU against
the FP64 oracle: maps, scores and argmax to the tolerances of the constant
covariance query (see test_gpu_parity), on seeded SH-coefficient variances."""
import math

import numpy as np
import pytest

import oracle
from paper_2605_30342_amd import scenes
from tests._gpu import compare_maps, gpu_query, oracle_params, say
from tests.test_gpu_parity import _check_argmax, _check_scores, _dsc, ctx  # noqa: F401

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tiny():
    return scenes.workload("tiny")


@pytest.fixture(scope="module")
def tiny_gamma(tiny):
    b = oracle.vf_build(tiny.scene, tiny.train, 2, oracle_params())
    return b["gamma"].astype(np.float32).astype(np.float64)


def _gpu_color(ctx, dsc, gamma_nk, L, n_train, var, cams, use_graph=0, gamma_dtype=None):
    import torch
    from paper_2605_30342_amd import _lib
    prm = _lib.default_uq_params()
    prm.use_graph = use_graph
    ws = ctx.query_workspace(dsc, cams, prm, L)
    g = torch.from_numpy(np.ascontiguousarray(np.asarray(gamma_nk, np.float32).T)).cuda()
    if gamma_dtype is not None:
        g = g.to(gamma_dtype)
    cv = torch.from_numpy(np.ascontiguousarray(var, np.float32)).cuda()
    scores, mp = ctx.vf_query_views_color(dsc, g, L, n_train, cv, cams, prm, ws, want_maps=True)
    st, counts = ctx.check_workspace(ws)
    torch.cuda.synchronize()
    assert st == 0 and counts[2] == 0, counts
    return scores.cpu().numpy().astype(np.float64), mp.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("Lc", [0, 1, 3])
def test_color_query_matches_oracle(ctx, tiny, tiny_gamma, Lc):
    say(f"case: vf_query_views_color tiny, colour SH degree {Lc}")
    var = scenes.color_sh_variances(tiny.scene.n, Lc, 7000 + Lc)
    prm = oracle_params()
    q = oracle.vf_query_color(tiny.scene, tiny_gamma, 2, tiny.train.n, var.astype(np.float64), Lc, tiny.cand, prm)
    s, mp = _gpu_color(ctx, _dsc(tiny.scene), tiny_gamma, 2, tiny.train.n, var, tiny.cand)
    worst, flagged = compare_maps(mp, q)
    say(f"  map worst ratio {worst:.3f}, flagged px {flagged:.5f}")
    assert worst <= 1.0 and flagged < 0.01
    _check_scores(s, q, mp)
    _check_argmax(ctx, s, q)


def test_constant_variance_equals_constant_covariance_query(ctx, tiny, tiny_gamma):
    """Variance only on Y_00, 4 pi sigma_c^2 in every channel: Q_c = sigma_c^2 I
    in every direction, so the result equals vf_query_views with that
    constant (up to FP32 rounding of the two summation orders)."""
    say("case: colour query with a direction-independent covariance")
    sig = 0.1
    var = np.zeros((3, 1, tiny.scene.n), np.float32)
    var[:] = 4 * math.pi * sig * sig
    s1, m1 = _gpu_color(ctx, _dsc(tiny.scene), tiny_gamma, 2, tiny.train.n, var, tiny.cand)
    s0, m0, _ = gpu_query(ctx, _dsc(tiny.scene), tiny_gamma, 2, tiny.train.n, tiny.cand, sigma_c=sig)
    scale = np.abs(m0).max()
    assert np.abs(m1 - m0).max() <= 2e-5 * scale
    np.testing.assert_allclose(s1, s0, rtol=2e-5)


def test_color_query_graph_replay_equals_eager(ctx, tiny, tiny_gamma):
    say("case: vf_query_views_color under hipGraph replay")
    var = scenes.color_sh_variances(tiny.scene.n, 2, 7100)
    dsc = _dsc(tiny.scene)
    s0, m0 = _gpu_color(ctx, dsc, tiny_gamma, 2, tiny.train.n, var, tiny.cand)
    for _ in range(3):
        s1, m1 = _gpu_color(ctx, dsc, tiny_gamma, 2, tiny.train.n, var, tiny.cand, use_graph=1)
        assert np.array_equal(m0, m1) and np.array_equal(s0, s1)


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_color_query_half_storage(ctx, dtype):
    """Colour covariance with the scene and the field stored in FP16 / BF16:
    equal to the oracle on the same dequantised attributes and field."""
    say(f"case: vf_query_views_color with {dtype} storage")
    import torch
    from paper_2605_30342_amd.api import DeviceScene
    from tests.test_gpu_parity import _dequantised
    w = scenes.workload("room", scale=0.05)
    sc = scenes.subset_scene(w.scene, scenes.morton_order(w.scene))
    deq = _dequantised(sc, dtype)
    prm = oracle_params()
    train = w.train.subset([0, 3])
    cand = w.cand.subset([0, 1])
    b = oracle.vf_build(deq, train, 3, prm)
    td = torch.float16 if dtype == "f16" else torch.bfloat16
    gh = torch.from_numpy(b["gamma"].astype(np.float32)).to(td).float().numpy().astype(np.float64)
    var = scenes.color_sh_variances(sc.n, 3, 7300)
    q = oracle.vf_query_color(deq, gh, 3, train.n, var.astype(np.float64), 3, cand, prm)
    s, mp = _gpu_color(ctx, DeviceScene(sc, dtype=dtype), gh, 3, train.n, var, cand, gamma_dtype=td)
    worst, flagged = compare_maps(mp, q)
    say(f"  map worst ratio {worst:.3f}, flagged px {flagged:.5f}")
    assert worst <= 1.0 and flagged < 0.02
    _check_scores(s, q, mp)
