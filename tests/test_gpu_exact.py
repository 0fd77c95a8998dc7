"""Exact-visibility validation mode on the GPU against the FP64 oracle.

vf_view_visibility: per-view v_p[g] of Alg. 2, |a - b| <= 1e-4 + 2 pert_p[g]
(pert = the oracle's first-order bound on the effect of near-tie decisions),
camera centres to FP32 rounding.  vf_query_views_exact: maps, scores and
argmax to the tolerances of the SH query (see test_gpu_parity), the oracle
taking the same FP32 per-view visibilities.
"""
import numpy as np
import pytest

import oracle
from paper_2605_30342_amd import scenes
from paper_2605_30342_amd.scenes import Scene
from tests._gpu import compare_maps, oracle_params, say
from tests.test_gpu_parity import _check_argmax, _check_scores, _dsc, ctx  # noqa: F401

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tiny():
    return scenes.workload("tiny")


def _gpu_exact(ctx, dsc, vis, centres, kappa, cams, sigma_c=0.1, use_graph=0):
    import torch
    from paper_2605_30342_amd import _lib
    prm = _lib.default_uq_params()
    prm.half_logdet_Qc = float(3.0 * np.log(sigma_c))
    prm.use_graph = use_graph
    ws = ctx.query_workspace(dsc, cams, prm, 0)
    v = torch.as_tensor(np.ascontiguousarray(vis, np.float32)).cuda()
    c = torch.as_tensor(np.ascontiguousarray(centres, np.float32)).cuda()
    scores, mp = ctx.vf_query_views_exact(dsc, v, c, kappa, cams, prm, ws, want_maps=True)
    st, counts = ctx.check_workspace(ws)
    torch.cuda.synchronize()
    assert st == 0 and counts[2] == 0, counts
    return scores.cpu().numpy().astype(np.float64), mp.cpu().numpy().astype(np.float64)


def test_view_visibility_matches_oracle(ctx, tiny):
    say("case: vf_view_visibility tiny, 8 training views 128x128")
    import torch
    vis, centres = ctx.view_visibility(_dsc(tiny.scene), tiny.train)
    torch.cuda.synchronize()
    vg = vis.cpu().numpy().astype(np.float64)
    prm = oracle_params()
    worst = 0.0
    for p in range(tiny.train.n):
        v, _, pert = oracle.single_view(tiny.scene, tiny.train, p, prm)
        worst = max(worst, float((np.abs(vg[p] - v) / (1e-4 + 2.0 * pert)).max()))
    say(f"  worst ratio {worst:.3f}")
    assert worst <= 1.0
    np.testing.assert_allclose(centres.cpu().numpy(), oracle.camera_centres(tiny.train), rtol=0, atol=2e-6)


def test_view_visibility_multi_pass(ctx, tiny):
    """Three views per pass gives the one-pass result: the same zero pattern
    (a record's pixel count is an integer) and values equal up to the order
    of the blend's floating-point atomic sums."""
    say("case: vf_view_visibility views_per_pass=3 equals one pass")
    import torch
    from paper_2605_30342_amd import _lib
    dsc = _dsc(tiny.scene)
    a, _ = ctx.view_visibility(dsc, tiny.train)
    b, _ = ctx.view_visibility(dsc, tiny.train, _lib.default_vf_params(views_per_pass=3))
    torch.cuda.synchronize()
    a, b = a.cpu().numpy(), b.cpu().numpy()
    assert np.array_equal(a == 0, b == 0)
    assert np.abs(a - b).max() <= 1e-5


def test_exact_query_matches_oracle(ctx, tiny):
    say("case: vf_query_views_exact tiny, 4 candidates 128x128, oracle per-view visibility")
    prm = oracle_params()
    b = oracle.vf_build(tiny.scene, tiny.train, 2, prm, want_views=True)
    vt = b["vview"].astype(np.float32).astype(np.float64)
    q = oracle.vf_query_exact(tiny.scene, vt, tiny.train, prm.kappa, tiny.cand, prm)
    s, mp = _gpu_exact(ctx, _dsc(tiny.scene), vt, oracle.camera_centres(tiny.train), prm.kappa, tiny.cand)
    worst, flagged = compare_maps(mp, q)
    say(f"  map worst ratio {worst:.3f}, flagged px {flagged:.5f}")
    assert worst <= 1.0 and flagged < 0.01
    _check_scores(s, q, mp)
    _check_argmax(ctx, s, q)


def test_exact_query_other_kappa_and_virtual_tail(ctx, tiny):
    say("case: vf_query_views_exact kappa = 3, virtual tail of 300")
    prm = oracle_params(kappa=3.0)
    sc = Scene(tiny.scene.means, tiny.scene.scales, tiny.scene.quats, tiny.scene.opacity, n_virtual=300)
    b = oracle.vf_build(sc, tiny.train, 0, prm, want_views=True)
    vt = b["vview"].astype(np.float32).astype(np.float64)
    q = oracle.vf_query_exact(sc, vt, tiny.train, prm.kappa, tiny.cand, prm)
    s, mp = _gpu_exact(ctx, _dsc(sc), vt, oracle.camera_centres(tiny.train), prm.kappa, tiny.cand)
    worst, _ = compare_maps(mp, q)
    say(f"  map worst ratio {worst:.3f}")
    assert worst <= 1.0
    _check_scores(s, q, mp)


def test_exact_query_without_views_equals_sh_query_without_views(ctx, tiny):
    """n_train = 0: every V is 0 in both modes, so the maps are bit-identical."""
    say("case: exact vs SH query with no training views")
    from tests._gpu import gpu_query
    dsc = _dsc(tiny.scene)
    s0, m0, _ = gpu_query(ctx, dsc, np.zeros((tiny.scene.n, 9)), 2, 0, tiny.cand)
    s1, m1 = _gpu_exact(ctx, dsc, np.zeros((0, tiny.scene.n)), np.zeros((0, 3)), 1.0, tiny.cand)
    assert np.array_equal(m0, m1) and np.array_equal(s0, s1)


def test_exact_query_graph_replay_equals_eager(ctx, tiny):
    say("case: vf_query_views_exact under hipGraph replay")
    prm = oracle_params()
    b = oracle.vf_build(tiny.scene, tiny.train, 0, prm, want_views=True)
    dsc = _dsc(tiny.scene)
    C = oracle.camera_centres(tiny.train)
    s0, m0 = _gpu_exact(ctx, dsc, b["vview"], C, 1.0, tiny.cand)
    for _ in range(3):
        s1, m1 = _gpu_exact(ctx, dsc, b["vview"], C, 1.0, tiny.cand, use_graph=1)
        assert np.array_equal(m0, m1) and np.array_equal(s0, s1)


def test_gpu_view_visibility_feeds_exact_query(ctx, tiny):
    """End to end on the GPU (per-view visibility -> exact query) against the
    oracle end to end (its own per-view visibilities -> exact query): the
    per-view visibilities agree to 1e-4 plus near-tie allowances, so maps are
    held to 1e-3 on unflagged pixels and scores to 1e-3 sum|H|.  The SH
    query of the GPU's own field is reported beside it."""
    say("case: GPU view visibility -> GPU exact query vs oracle end to end, tiny")
    import torch
    from tests._gpu import gpu_build, gpu_query
    prm = oracle_params()
    dsc = _dsc(tiny.scene)
    vis, centres = ctx.view_visibility(dsc, tiny.train)
    torch.cuda.synchronize()
    s, mp = _gpu_exact(ctx, dsc, vis.cpu().numpy(), centres.cpu().numpy(), 1.0, tiny.cand)
    b = oracle.vf_build(tiny.scene, tiny.train, 0, prm, want_views=True)
    q = oracle.vf_query_exact(tiny.scene, b["vview"], tiny.train, prm.kappa, tiny.cand, prm)
    worst, _ = compare_maps(mp, q, rel=1e-3)
    say(f"  map worst ratio at 1e-3: {worst:.3f}")
    assert worst <= 1.0
    off = 0
    for v, m in enumerate(q["maps"]):
        absH = np.abs(q["maps_flat"][off:off + m.size]).sum()
        assert abs(s[v] - q["scores"][v]) <= 1e-3 * absH
        off += m.size
    g = gpu_build(ctx, dsc, tiny.train, 2)
    s_sh, _, _ = gpu_query(ctx, dsc, g, 2, tiny.train.n, tiny.cand, maps=False)
    gap = np.abs(s_sh - s) / np.abs(s)
    say(f"  SH-query score gap to exact: max {gap.max():.4f}")
    assert np.all(np.isfinite(s_sh)) and np.all(np.isfinite(s))


def test_extension_arguments_are_rejected(ctx, tiny):
    """The exact, colour and depth entry points validate their arguments
    before enqueuing anything (errors come back as GvError, no launch)."""
    say("case: argument validation of the extension entry points")
    import ctypes
    import torch
    from paper_2605_30342_amd import _lib
    from paper_2605_30342_amd._lib import GvError, check
    dsc = _dsc(tiny.scene)
    prm = _lib.default_uq_params()
    ws = ctx.query_workspace(dsc, tiny.cand, prm, 2)
    n = tiny.scene.n
    vis = torch.zeros((2, n), device="cuda")
    cen = torch.zeros((2, 3), device="cuda")
    with pytest.raises(GvError):   # negative kappa
        ctx.vf_query_views_exact(dsc, vis, cen, -1.0, tiny.cand, prm, ws)
    with pytest.raises(ValueError):   # centres of the wrong shape (caught by the binding)
        ctx.vf_query_views_exact(dsc, vis, torch.zeros((3, 3), device="cuda"), 1.0, tiny.cand, prm, ws)
    cc = _lib.cameras_to_c(tiny.cand)
    scores = torch.empty(tiny.cand.n, device="cuda")
    with pytest.raises(GvError):   # NULL per-view visibility with training views (direct C call)
        check(ctx.L.vf_query_views_exact(ctx.h, ctypes.byref(dsc.c), None, ctypes.c_void_p(cen.data_ptr()), 2,
                                         1.0, cc, tiny.cand.n, ctypes.byref(prm),
                                         ctypes.c_void_p(scores.data_ptr()), None, ctypes.byref(ws.plan),
                                         ctypes.c_void_p(ws.buf.data_ptr()), None))
    g = torch.zeros((9, n), device="cuda")
    cv = torch.zeros((3, 25, n), device="cuda")   # colour degree 4: unsupported
    with pytest.raises(GvError):
        ctx.vf_query_views_color(dsc, g, 2, 8, cv, tiny.cand, prm, ws)
    bad = _lib.default_uq_params(write_depth=1)   # depth without maps
    with pytest.raises(GvError):
        check(ctx.L.vf_query_views(ctx.h, ctypes.byref(dsc.c), ctypes.c_void_p(g.data_ptr()), 0, 2, 8, cc,
                                   tiny.cand.n, ctypes.byref(bad), ctypes.c_void_p(scores.data_ptr()), None,
                                   ctypes.byref(ws.plan), ctypes.c_void_p(ws.buf.data_ptr()), None))
    torch.cuda.synchronize()


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_exact_query_half_storage(ctx, dtype):
    """The exact mode on half-stored attributes equals the oracle run on the
    same dequantised values (the per-view visibilities come from the oracle
    on those values too)."""
    say(f"case: vf_query_views_exact with {dtype} storage")
    from paper_2605_30342_amd.api import DeviceScene
    from tests.test_gpu_parity import _dequantised
    w = scenes.workload("room", scale=0.05)
    sc = scenes.subset_scene(w.scene, scenes.morton_order(w.scene))
    deq = _dequantised(sc, dtype)
    prm = oracle_params()
    train = w.train.subset([0, 2, 4])
    cand = w.cand.subset([0, 1])
    b = oracle.vf_build(deq, train, 0, prm, want_views=True)
    vt = b["vview"].astype(np.float32).astype(np.float64)
    q = oracle.vf_query_exact(deq, vt, train, prm.kappa, cand, prm)
    s, mp = _gpu_exact(ctx, DeviceScene(sc, dtype=dtype), vt, oracle.camera_centres(train), prm.kappa, cand)
    worst, flagged = compare_maps(mp, q)
    say(f"  map worst ratio {worst:.3f}, flagged px {flagged:.5f}")
    assert worst <= 1.0 and flagged < 0.02
    _check_scores(s, q, mp)
