"""GPU path vs the FP64 oracle, element by element, through the C ABI.

Tolerances (floating point, FP32 kernels vs FP64 oracle):
  maps     |a - b| <= 1e-4 (|b| + max|b_map|) on pixels the oracle does not
           flag as near ties (boundary pairs, transmittance at eps_T, equal
           depths); the flagged fraction is asserted small;
  gamma    |d gamma_gk| <= 1e-4 ||gamma_g||_inf + 2 allow_gk, where allow is the
           oracle's first-order bound on the effect of near-tie decisions;
  scores   |d S_v| <= 1e-4 sum_px |H| + the GPU-vs-oracle difference summed
           over flagged pixels;
  argmax   bit-exact, or inside the oracle's near-tie set when scores lie
           within 2e-4 max sum|H| of the best.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2605_30342_amd import scenes
from paper_2605_30342_amd.scenes import Cameras, Scene
from tests._cases import stress_scene, translucent_stack
from tests._gpu import (ALLOW_BAR, check_pair_count, compare_gamma, compare_maps, flag_bar, gpu_build, gpu_query,
                        oracle_params, say, score_slack)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2605_30342_amd.api import Context
    c = Context(0)
    yield c
    c.close()


def _dsc(scene, dtype="f32"):
    from paper_2605_30342_amd.api import DeviceScene
    return DeviceScene(scene, dtype=dtype)


def _check_scores(s_gpu, ora, mp_gpu):
    ref = ora["scores"]
    off = 0
    for v, m in enumerate(ora["maps"]):
        n = m.size
        absH = np.abs(ora["maps_flat"][off:off + n]).sum()
        f = ora["flags_flat"][off:off + n]
        flagged = np.abs(mp_gpu[off:off + n] - ora["maps_flat"][off:off + n])[f].sum() if mp_gpu is not None else 0.0
        assert abs(s_gpu[v] - ref[v]) <= 1e-4 * absH + flagged + 1e-6, (v, s_gpu[v], ref[v])
        off += n


def _check_argmax(ctx, s_gpu, ora):
    import torch
    best = ctx.select_next_view(torch.from_numpy(s_gpu.astype(np.float32)).cuda())
    absH = []
    off = 0
    for m in ora["maps"]:
        absH.append(np.abs(ora["maps_flat"][off:off + m.size]).sum())
        off += m.size
    near = oracle.near_tie_set(ora["scores"], absH)
    if len(near) == 1:
        assert best == oracle.argmax(ora["scores"])
    else:
        assert best in near


# ---------------------------------------------------------------- select_next_view

def test_select_next_view_ties_and_nan(ctx):
    import torch
    say("case: select_next_view small arrays")
    cases = [[1.0, 3.0, 3.0, 2.0], [float("nan"), -1.0, -1.0], [5.0], [0.0] * 7 + [1e-30],
             list(np.random.default_rng(3).standard_normal(3000))]
    for c in cases:
        s = torch.tensor(c, dtype=torch.float32, device="cuda")
        assert ctx.select_next_view(s) == oracle.argmax(np.asarray(c, np.float32).astype(np.float64))
    s = torch.tensor([float("nan")] * 4, dtype=torch.float32, device="cuda")
    assert ctx.select_next_view(s) == -1


# ---------------------------------------------------------------- tiny workload

@pytest.fixture(scope="module")
def tiny():
    return scenes.workload("tiny")


@pytest.fixture(scope="module")
def tiny_ref(tiny):
    prm = oracle_params()
    b = oracle.vf_build(tiny.scene, tiny.train, 2, prm)
    g32 = b["gamma"].astype(np.float32).astype(np.float64)
    q = oracle.vf_query(tiny.scene, g32, 2, tiny.train.n, tiny.cand, prm)
    return b, g32, q


def test_build_tiny_matches_oracle(ctx, tiny, tiny_ref):
    say("case: vf_build tiny 2000 Gaussians, 8 views 128x128, L=2")
    b, _, _ = tiny_ref
    g = gpu_build(ctx, _dsc(tiny.scene), tiny.train, 2)
    worst, frac = compare_gamma(g, b)
    say(f"  gamma worst ratio {worst:.3f}, allowance fraction {frac:.4f}")
    assert worst <= 1.0 and frac <= ALLOW_BAR
    assert frac <= ALLOW_BAR


def test_query_tiny_matches_oracle(ctx, tiny, tiny_ref):
    say("case: vf_query_views tiny, 4 views 128x128")
    _, g32, q = tiny_ref
    s, mp, _ = gpu_query(ctx, _dsc(tiny.scene), g32, 2, tiny.train.n, tiny.cand)
    worst, flagged = compare_maps(mp, q)
    say(f"  map worst ratio {worst:.3f}, flagged px {flagged:.5f}")
    assert worst <= 1.0
    assert flagged <= flag_bar(q["stats"])
    _check_scores(s, q, mp)
    _check_argmax(ctx, s, q)


def test_build_then_query_end_to_end(ctx, tiny, tiny_ref):
    """GPU build -> GPU query against oracle build -> oracle query.  The
    field's own error (1e-4 of its scale plus near-tie allowances) passes
    through the query, so maps are held to 1e-3 (the bound stated for composed
    forms against FP64) on unflagged pixels, scores to 1e-3 sum|H|, and the
    argmax to the oracle's near-tie set."""
    say("case: GPU build -> GPU query vs oracle build -> oracle query, tiny")
    _, _, q = tiny_ref
    dsc = _dsc(tiny.scene)
    g = gpu_build(ctx, dsc, tiny.train, 2)
    s, mp, _ = gpu_query(ctx, dsc, g, 2, tiny.train.n, tiny.cand)
    worst, _ = compare_maps(mp, q, rel=1e-3)
    say(f"  map worst ratio at 1e-3: {worst:.3f}")
    assert worst <= 1.0
    off = 0
    for v, m in enumerate(q["maps"]):
        absH = np.abs(q["maps_flat"][off:off + m.size]).sum()
        assert abs(s[v] - q["scores"][v]) <= 1e-3 * absH, (v, s[v], q["scores"][v])
        off += m.size
    _check_argmax(ctx, s, q)


def test_build_multi_pass_equals_single_pass(ctx, tiny, tiny_ref):
    say("case: vf_build views_per_pass=3 vs one pass")
    b, _, _ = tiny_ref
    dsc = _dsc(tiny.scene)
    g1 = gpu_build(ctx, dsc, tiny.train, 2)
    g3 = gpu_build(ctx, dsc, tiny.train, 2, views_per_pass=3)
    scale = np.abs(g1).max(1, keepdims=True) + 1e-30
    assert np.all(np.abs(g3 - g1) <= 1e-5 * scale)
    worst, _ = compare_gamma(g3, b)
    assert worst <= 1.0


@pytest.mark.parametrize("L", [0, 1, 3])
def test_build_and_query_other_degrees(ctx, tiny, L):
    say(f"case: degree L={L}")
    prm = oracle_params()
    sc = scenes.subset_scene(tiny.scene, np.arange(800))
    b = oracle.vf_build(sc, tiny.train, L, prm)
    g = gpu_build(ctx, _dsc(sc), tiny.train, L)
    assert compare_gamma(g, b)[0] <= 1.0
    g32 = b["gamma"].astype(np.float32).astype(np.float64)
    q = oracle.vf_query(sc, g32, L, tiny.train.n, tiny.cand.subset([0, 1]), prm)
    s, mp, _ = gpu_query(ctx, _dsc(sc), g32, L, tiny.train.n, tiny.cand.subset([0, 1]))
    assert compare_maps(mp, q)[0] <= 1.0


def test_kappa_zero_isotropic_on_gpu(ctx, tiny):
    say("case: kappa = 0 build")
    prm = oracle_params(kappa=0.0)
    sc = scenes.subset_scene(tiny.scene, np.arange(600))
    b = oracle.vf_build(sc, tiny.train, 2, prm)
    g = gpu_build(ctx, _dsc(sc), tiny.train, 2, kappa=0.0)
    assert np.all(g[:, 1:] == 0.0)
    assert compare_gamma(g, b)[0] <= 1.0


# ---------------------------------------------------------------- edge cases

def _ragged_cams(w):
    """Five views of mixed and ragged sizes (37x23, 1x1, 128x96, 200x17,
    16x16) from the first candidate's centre, looking at the origin."""
    C = w.cand.centers[:1].repeat(5, 0)
    sizes = [(37, 23), (1, 1), (128, 96), (200, 17), (16, 16)]
    return Cameras.concat([scenes.make_cameras(C[i:i + 1], np.zeros((1, 3)), ww, hh, 60.0)
                           for i, (ww, hh) in enumerate(sizes)])


def test_ragged_and_mixed_resolutions_in_one_call(ctx, tiny, tiny_ref):
    say("case: ragged/mixed resolutions 37x23, 1x1, 128x96, 200x17, 16x16")
    _, g32, _ = tiny_ref
    prm = oracle_params()
    cams = _ragged_cams(tiny)
    q = oracle.vf_query(tiny.scene, g32, 2, tiny.train.n, cams, prm)
    s, mp, _ = gpu_query(ctx, _dsc(tiny.scene), g32, 2, tiny.train.n, cams)
    assert compare_maps(mp, q)[0] <= 1.0
    _check_scores(s, q, mp)
    bo = oracle.vf_build(tiny.scene, cams, 2, prm)
    bg = gpu_build(ctx, _dsc(tiny.scene), cams, 2)
    assert compare_gamma(bg, bo)[0] <= 1.0


@pytest.mark.parametrize("n", [1024, 2048])
def test_scan_block_boundaries(ctx, tiny, n):
    """Scenes whose (Gaussian, view subset) entries fill the scans' 4096-value
    blocks exactly (1024 and 2048 Gaussians: 4096 and 8192 entries), so that
    the total lands in the first slot of a block of its own: build and query
    against the oracle."""
    say(f"case: scan block boundary, {n} Gaussians")
    sc = scenes.tiny_scene(n, seed=90 + n)
    prm = oracle_params()
    b = oracle.vf_build(sc, tiny.train, 2, prm)
    g = gpu_build(ctx, _dsc(sc), tiny.train, 2)
    assert compare_gamma(g, b)[0] <= 1.0
    g32 = b["gamma"].astype(np.float32).astype(np.float64)
    q = oracle.vf_query(sc, g32, 2, tiny.train.n, tiny.cand, prm)
    s, mp, _ = gpu_query(ctx, _dsc(sc), g32, 2, tiny.train.n, tiny.cand)
    worst, flagged = compare_maps(mp, q)
    assert worst <= 1.0 and flagged <= flag_bar(q["stats"])
    _check_scores(s, q, mp)


def _extreme_views():
    """Candidates at the largest image sizes the ABI accepts: 16384 x 16 and
    16 x 16384 pixels (1024 tiles along one axis), looking at the tiny scene."""
    wide = scenes.make_cameras([[3.0, 0.4, 0.3]], [[0.0, 0.0, 0.0]], 16384, 16, 120.0)
    tall = scenes.make_cameras([[-0.5, 2.9, 0.2]], [[0.0, 0.0, 0.0]], 16, 16384, 0.5)
    return Cameras.concat([wide, tall])


def test_maximum_image_sizes(ctx, tiny, tiny_ref):
    """Both largest image shapes in one call against the oracle, element by
    element (the packed tile-rectangle fields and int16 pixel anchors at their
    widest)."""
    say("case: query of a 16384x16 and a 16x16384 view in one call")
    _, g32, _ = tiny_ref
    cams = _extreme_views()
    q = oracle.vf_query(tiny.scene, g32, 2, tiny.train.n, cams, oracle_params())
    s, mp, _ = gpu_query(ctx, _dsc(tiny.scene), g32, 2, tiny.train.n, cams)
    worst, flagged = compare_maps(mp, q)
    say(f"  map worst ratio {worst:.3f}, flagged px {flagged:.5f}, "
        f"covered px {[int((m != 0).sum()) for m in q['maps']]}")
    assert worst <= 1.0 and flagged <= flag_bar(q["stats"])
    assert all((m != 0).sum() > 1000 for m in q["maps"])   # both views see the scene
    _check_scores(s, q, mp)


def test_no_training_views_means_invisible(ctx, tiny, tiny_ref):
    say("case: n_train = 0")
    _, g32, _ = tiny_ref
    prm = oracle_params()
    cams = tiny.cand.subset([0])
    q = oracle.vf_query(tiny.scene, g32, 2, 0, cams, prm)
    s, mp, _ = gpu_query(ctx, _dsc(tiny.scene), g32, 2, 0, cams)
    assert compare_maps(mp, q)[0] <= 1.0


def test_virtual_particles_query_zero(ctx, tiny, tiny_ref):
    say("case: virtual particle tail")
    _, g32, _ = tiny_ref
    prm = oracle_params()
    sc = Scene(tiny.scene.means, tiny.scene.scales, tiny.scene.quats, tiny.scene.opacity, n_virtual=300)
    cams = tiny.cand.subset([2])
    q = oracle.vf_query(sc, g32, 2, tiny.train.n, cams, prm)
    s, mp, _ = gpu_query(ctx, _dsc(sc), g32, 2, tiny.train.n, cams)
    assert compare_maps(mp, q)[0] <= 1.0


def test_everything_behind_camera_and_empty_scene(ctx, tiny, tiny_ref):
    say("case: all Gaussians behind the camera; empty scene")
    _, g32, _ = tiny_ref
    cams = scenes.make_cameras([[3.0, 0, 0]], [[6.0, 0.5, 0.2]], 64, 48, 60.0)   # looks away from the cloud
    s, mp, _ = gpu_query(ctx, _dsc(tiny.scene), g32, 2, tiny.train.n, cams)
    assert np.all(mp == 0.0) and s[0] == 0.0
    g = gpu_build(ctx, _dsc(tiny.scene), cams, 2)
    assert np.all(g == 0.0)
    empty = scenes.subset_scene(tiny.scene, np.arange(0))
    import torch
    from paper_2605_30342_amd import _lib
    from paper_2605_30342_amd.api import DeviceScene
    d = DeviceScene(empty)
    prm = _lib.default_uq_params()
    ws = ctx.query_workspace(d, tiny.cand, prm, 2)
    sc, mp2 = ctx.vf_query_views(d, torch.zeros((9, 0), device="cuda"), 2, 3, tiny.cand, prm, ws, want_maps=True)
    torch.cuda.synchronize()
    assert torch.all(sc == 0) and torch.all(mp2 == 0)


def test_invalid_arguments_are_rejected(ctx, tiny):
    say("case: argument validation")
    import torch
    from paper_2605_30342_amd import _lib
    from paper_2605_30342_amd._lib import GvError
    dsc = _dsc(tiny.scene)
    with pytest.raises(GvError):
        ctx.vf_build(dsc, tiny.train, 4, _lib.default_vf_params(sh_degree=4))
    bad = Cameras(tiny.cand.R[:1].copy(), tiny.cand.t[:1].copy(), tiny.cand.K[:1].copy(),
                  np.array([[0, 10]], np.int32))
    with pytest.raises(GvError):
        ctx.query_workspace(dsc, bad, _lib.default_uq_params(), 2)
    prm = _lib.default_uq_params()
    ws = ctx.query_workspace(dsc, tiny.cand.subset([0]), prm, 2)
    g = torch.zeros((9, tiny.scene.n), device="cuda")
    with pytest.raises(GvError):   # plan made for 1 view, called with 4
        ctx.vf_query_views(dsc, g, 2, 8, tiny.cand, prm, ws)


def test_capacity_overflow_is_reported(ctx, tiny, tiny_ref):
    say("case: workspace too small -> overflow flag, NaN scores, no fault")
    import torch
    from paper_2605_30342_amd import _lib
    _, g32, _ = tiny_ref
    dsc = _dsc(tiny.scene)
    prm = _lib.default_uq_params()
    ws = ctx.query_workspace(dsc, tiny.cand, prm, 2)
    ws.plan.max_instances = max(1, ws.plan.max_instances // 3)
    ws.plan.bytes = ctx.L.gv_workspace_bytes(__import__("ctypes").byref(ws.plan))
    g = torch.from_numpy(g32.T.astype(np.float32).copy()).cuda()
    s, _ = ctx.vf_query_views(dsc, g, 2, tiny.train.n, tiny.cand, prm, ws)
    st, counts = ctx.check_workspace(ws)
    assert st == _lib.GV_ERR_CAPACITY and counts[2] != 0
    assert torch.all(torch.isnan(s))


@pytest.mark.parametrize("fill", [0x00, 0xFF])
def test_record_overflow_over_stale_workspace_is_reported(ctx, tiny, tiny_ref, fill):
    """Record capacity a third of what the call needs, in a workspace whose
    bytes are all `fill` beforehand: the call skips the projection and sorts
    the workspace's stale contents (with 0xFF every packed sort value claims a
    saturated tile count and record 2^24 - 1).  Query and build both report
    GV_ERR_CAPACITY (the query also NaN scores), neither reading outside its
    workspace (every gathered record index is checked against the sorted
    count); calls with large enough workspaces afterwards still match the
    oracle."""
    say(f"case: record overflow over a workspace filled with {fill:#04x}")
    import ctypes
    import torch
    from paper_2605_30342_amd import _lib
    b, g32, q = tiny_ref
    dsc = _dsc(tiny.scene)
    prm = _lib.default_uq_params()
    full = ctx.query_workspace(dsc, tiny.cand, prm, 2)
    plan = ctx.query_plan(dsc, tiny.cand, 2, max(1, full.plan.max_records // 3), full.plan.max_instances)
    ws = ctx.alloc_workspace(plan)
    ws.buf.fill_(fill)
    g = torch.from_numpy(g32.T.astype(np.float32).copy()).cuda()
    s, _ = ctx.vf_query_views(dsc, g, 2, tiny.train.n, tiny.cand, prm, ws)
    st, counts = ctx.check_workspace(ws)
    torch.cuda.synchronize()
    assert st == _lib.GV_ERR_CAPACITY and (counts[2] & 1), (st, counts)
    assert torch.all(torch.isnan(s))
    vprm = _lib.default_vf_params(sh_degree=2)
    bws = ctx.build_workspace(dsc, tiny.train, vprm)
    bplan = bws.plan
    bplan.max_records = max(1, bplan.max_records // 3)
    bplan.bytes = ctx.L.gv_workspace_bytes(ctypes.byref(bplan))
    small = ctx.alloc_workspace(bplan)
    small.buf.fill_(fill)
    ctx.vf_build(dsc, tiny.train, 2, params=vprm, ws=small)
    st, counts = ctx.check_workspace(small)
    torch.cuda.synchronize()
    assert st == _lib.GV_ERR_CAPACITY and (counts[2] & 1), (st, counts)
    worst, _ = compare_gamma(gpu_build(ctx, dsc, tiny.train, 2), b)
    assert worst <= 1.0
    s2, mp, _ = gpu_query(ctx, dsc, g32, 2, tiny.train.n, tiny.cand)
    worst, flagged = compare_maps(mp, q)
    assert worst <= 1.0 and flagged <= flag_bar(q["stats"])


# ---------------------------------------------------------------- room scenes

@pytest.fixture(scope="module")
def room_small():
    return scenes.workload("room", scale=0.1)


def test_stress_geometry_matches_oracle(ctx):
    """Build and query on the stress scene (large, needle, opaque,
    transparent and near-plane Gaussians) against the oracle, element by
    element: the binning's band tests stay conservative and long tile lists
    run over several batches."""
    train = scenes.sphere_cameras(3, 7101, width=160, height=120)
    cand = scenes.sphere_cameras(3, 7102, width=160, height=120)
    sc = stress_scene(train)
    prm = oracle_params()
    say(f"case: stress geometry build, {sc.n} Gaussians, 3 views 160x120")
    b = oracle.vf_build(sc, train, 2, prm)
    dsc = _dsc(sc)
    g = gpu_build(ctx, dsc, train, 2)
    worst, frac = compare_gamma(g, b)
    say(f"  gamma worst ratio {worst:.3f}, allowance fraction {frac:.4f}")
    assert worst <= 1.0 and frac <= ALLOW_BAR
    say("case: stress geometry query, 3 views 160x120")
    g32 = b["gamma"].astype(np.float32).astype(np.float64)
    q = oracle.vf_query(sc, g32, 2, train.n, cand, prm)
    s, mp, _ = gpu_query(ctx, dsc, g32, 2, train.n, cand)
    worst, flagged = compare_maps(mp, q)
    say(f"  map worst ratio {worst:.3f}, flagged px {flagged:.5f}")
    assert worst <= 1.0 and flagged <= flag_bar(q["stats"])
    _check_scores(s, q, mp)
    _check_argmax(ctx, s, q)


def test_deep_translucent_stack_matches_oracle(ctx):
    """A fog of 4000 faint Gaussians (opacity 0.003) in a small cube: about
    19k tile instances per view over 16 tiles, up to about 3300 in one tile,
    so the blends run up to about 50 batches of 64 records per tile (the VF
    CONST blend flushing each one a batch late) with few pixels terminating;
    build and query against the oracle element by element."""
    sc, train, cand = translucent_stack()
    prm = oracle_params()
    say("case: translucent stack build, 4000 Gaussians of opacity 0.003, 2 views 96x96")
    b = oracle.vf_build(sc, train, 2, prm)
    dsc = _dsc(sc)
    g = gpu_build(ctx, dsc, train, 2)
    worst, frac = compare_gamma(g, b)
    say(f"  gamma worst ratio {worst:.3f}, allowance fraction {frac:.4f}")
    assert worst <= 1.0 and frac <= ALLOW_BAR
    say("case: translucent stack query, 2 views 96x96")
    g32 = b["gamma"].astype(np.float32).astype(np.float64)
    qo = oracle.vf_query(sc, g32, 2, train.n, cand, prm)
    s, mp, ws = gpu_query(ctx, dsc, g32, 2, train.n, cand)
    _, counts = ctx.check_workspace(ws)
    say(f"  instances {counts[1]}, map worst ratio {compare_maps(mp, qo)[0]:.3f}")
    assert counts[1] > 25000                 # tile instances of the two views
    worst, flagged = compare_maps(mp, qo)
    assert worst <= 1.0 and flagged <= flag_bar(qo["stats"])
    _check_scores(s, qo, mp)


def _pair_count_cases():
    w = scenes.workload("tiny")
    yield "tiny", w.scene, w.train, w.cand, 2
    tr = scenes.sphere_cameras(3, 7101, width=160, height=120)
    yield "stress", stress_scene(tr), tr, scenes.sphere_cameras(3, 7102, width=160, height=120), 2
    sc, tr, cd = translucent_stack()
    yield "translucent stack", sc, tr, cd, 2
    w = scenes.workload("room", scale=0.1)
    yield "room subset", w.scene, w.train.subset([0, 3, 7]), w.cand.subset([0, 1, 2, 3]), 3


@pytest.mark.parametrize("case", range(4))
def test_device_pair_counts_match_oracle(ctx, case):
    """The composited (pixel, Gaussian) pair counts the kernels report (the
    numerator of the blend rooflines) against the oracle's exact count
    (Alg. 2 for the build, Alg. 6 for the query): equal on every pixel
    without a near-tie flag; a flagged pixel may contribute anywhere
    between none and all of its list entries."""
    name, sc, train, cand, L = list(_pair_count_cases())[case]
    prm = oracle_params()
    say(f"case: pair counts, {name}: build over {train.n} views, query of {cand.n} views")
    b = oracle.vf_build(sc, train, L, prm)
    dsc = _dsc(sc)
    _, counts = gpu_build(ctx, dsc, train, L, want_counts=True)
    st = b["stats"]
    say(f"  build: device {counts[3]}, oracle {st[0]} (clean {st[4]}, flagged entries {st[5]})")
    check_pair_count(counts[3], st, 4, 5)
    g32 = b["gamma"].astype(np.float32).astype(np.float64)
    q = oracle.vf_query(sc, g32, L, train.n, cand, prm)
    _, _, ws = gpu_query(ctx, dsc, g32, L, train.n, cand, maps=False, count_pairs=True)
    _, counts = ctx.check_workspace(ws)
    st = q["stats"]
    say(f"  query: device {counts[3]}, oracle {st[0]} (clean {st[4]}, flagged entries {st[5]})")
    check_pair_count(counts[3], st, 4, 5)


def _with_emit_mode(ctx, ws, mode, instances=None):
    """The workspace re-planned for the given emission mode (and optionally a
    smaller instance capacity), with a buffer of the new size."""
    import ctypes
    plan = ws.plan
    plan.emit_mode = mode
    if instances is not None:
        plan.max_instances = instances
    plan.bytes = ctx.L.gv_workspace_bytes(ctypes.byref(plan))
    return ctx.alloc_workspace(plan)


@pytest.mark.parametrize("case", range(4))
def test_lookback_emission_matches_the_scanned_one_and_the_oracle(ctx, case):
    """The two ways the emission finds its output offsets (a scan of the tile
    counts gathered into depth order, or the emission's own single-pass scan
    with decoupled look-back, which the large workloads take) give the same
    instance lists: bit-identical query maps and scores, equal build fields
    to FP32 rounding, both equal to the oracle; a look-back emission whose
    instances exceed the workspace flags the overflow."""
    import torch
    from paper_2605_30342_amd import _lib
    name, sc, train, cand, L = list(_pair_count_cases())[case]
    say(f"case: emission modes, {name}")
    prm = oracle_params()
    b = oracle.vf_build(sc, train, L, prm)
    g32 = b["gamma"].astype(np.float32).astype(np.float64)
    q = oracle.vf_query(sc, g32, L, train.n, cand, prm)
    dsc = _dsc(sc)
    gd = torch.from_numpy(np.ascontiguousarray(g32.T.astype(np.float32))).cuda()
    uprm = _lib.default_uq_params()
    out = {}
    for mode in (1, 2):
        ws = _with_emit_mode(ctx, ctx.query_workspace(dsc, cand, uprm, L), mode)
        s_, m_ = ctx.vf_query_views(dsc, gd, L, train.n, cand, uprm, ws, want_maps=True)
        st_, cnt = ctx.check_workspace(ws)
        assert st_ == 0, cnt
        vprm = _lib.default_vf_params(sh_degree=L)
        wsb = _with_emit_mode(ctx, ctx.build_workspace(dsc, train, vprm), mode)
        gam = ctx.vf_build(dsc, train, L, vprm, wsb)
        torch.cuda.synchronize()
        out[mode] = (s_.cpu().numpy(), m_.cpu().numpy(), gam.cpu().numpy().T.astype(np.float64), cnt[1])
    assert out[1][3] == out[2][3]                          # instance totals
    assert np.array_equal(out[1][0], out[2][0]) and np.array_equal(out[1][1], out[2][1])
    worst, flagged = compare_maps(out[2][1].astype(np.float64), q)
    assert worst <= 1.0 and flagged <= flag_bar(q["stats"])
    scale = np.abs(out[1][2]).max(1, keepdims=True) + 1e-30
    assert np.all(np.abs(out[2][2] - out[1][2]) <= 1e-5 * scale)
    assert compare_gamma(out[2][2], b)[0] <= 1.0
    # overflow of the instance capacity in the look-back emission
    ws = _with_emit_mode(ctx, ctx.query_workspace(dsc, cand, uprm, L), 2, instances=max(1, out[2][3] // 3))
    s_, _ = ctx.vf_query_views(dsc, gd, L, train.n, cand, uprm, ws)
    st_, cnt = ctx.check_workspace(ws)
    assert st_ == _lib.GV_ERR_CAPACITY and (cnt[2] & 2) and cnt[1] == out[2][3]
    assert torch.all(torch.isnan(s_))


def test_scanned_emission_with_unpacked_tile_counts(ctx, tiny, tiny_ref):
    """Plans of 2^24 records and more keep the tile counts apart from the
    depth-sort values (the last depth pass gathers them): the same query and
    build with the record capacity raised to 2^24 give the results of the
    packed plan, bit-identical maps and gamma to FP32 rounding."""
    say("case: scanned emission with the record capacity at 2^24 (tile counts gathered)")
    import ctypes
    import torch
    from paper_2605_30342_amd import _lib
    _, g32, _ = tiny_ref
    dsc = _dsc(tiny.scene)
    gd = torch.from_numpy(np.ascontiguousarray(g32.T.astype(np.float32))).cuda()
    uprm = _lib.default_uq_params()
    vprm = _lib.default_vf_params(sh_degree=2)
    out = []
    for big in (False, True):
        wsq = ctx.query_workspace(dsc, tiny.cand, uprm, 2)
        wsb = ctx.build_workspace(dsc, tiny.train, vprm)
        if big:
            for ws in (wsq, wsb):
                ws.plan.max_records = 1 << 24
                ws.plan.emit_mode = 1
                ws.plan.bytes = ctx.L.gv_workspace_bytes(ctypes.byref(ws.plan))
            wsq, wsb = ctx.alloc_workspace(wsq.plan), ctx.alloc_workspace(wsb.plan)
        s_, m_ = ctx.vf_query_views(dsc, gd, 2, tiny.train.n, tiny.cand, uprm, wsq, want_maps=True)
        gam = ctx.vf_build(dsc, tiny.train, 2, vprm, wsb)
        torch.cuda.synchronize()
        assert ctx.check_workspace(wsq)[0] == 0 and ctx.check_workspace(wsb)[0] == 0
        out.append((s_.cpu().numpy(), m_.cpu().numpy(), gam.cpu().numpy().T.astype(np.float64)))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    scale = np.abs(out[0][2]).max(1, keepdims=True) + 1e-30
    assert np.all(np.abs(out[1][2] - out[0][2]) <= 1e-5 * scale)


def test_records_with_hundreds_of_tiles(ctx):
    """The stress scene seen at 640x480: its large Gaussians cover several
    hundred of the 1200 tiles, past the 255 that a packed depth-sort value
    can carry (their counts are read from the binning lines); build and
    query against the oracle."""
    say("case: records covering 255 tiles and more (stress scene at 640x480)")
    tr = scenes.sphere_cameras(2, 7201, width=640, height=480)
    cd = scenes.sphere_cameras(2, 7202, width=640, height=480)
    sc = stress_scene(tr)
    prm = oracle_params()
    # the test is only meaningful if some record spans at least 255 tiles
    p = oracle.project_view(sc, cd, 0, prm)
    ok = p["ok"] > 0
    rx, ry = np.sqrt(9.0 * p["sxx"][ok]), np.sqrt(9.0 * p["syy"][ok])
    tx = np.minimum(np.floor((p["ux"][ok] + rx) / 16), 39) - np.maximum(np.floor((p["ux"][ok] - rx) / 16), 0) + 1
    ty = np.minimum(np.floor((p["uy"][ok] + ry) / 16), 29) - np.maximum(np.floor((p["uy"][ok] - ry) / 16), 0) + 1
    assert (np.clip(tx, 0, None) * np.clip(ty, 0, None)).max() >= 255
    b = oracle.vf_build(sc, tr, 2, prm)
    g = gpu_build(ctx, _dsc(sc), tr, 2)
    worst_g, _ = compare_gamma(g, b)
    g32 = b["gamma"].astype(np.float32).astype(np.float64)
    q = oracle.vf_query(sc, g32, 2, tr.n, cd, prm)
    s_, mp, _ = gpu_query(ctx, _dsc(sc), g32, 2, tr.n, cd)
    worst, flagged = compare_maps(mp, q)
    say(f"  gamma worst {worst_g:.3f}; map worst {worst:.3f}, flagged {flagged:.5f}")
    assert worst_g <= 1.0 and worst <= 1.0 and flagged <= flag_bar(q["stats"])
    _check_scores(s_, q, mp)


def test_room_subset_build_and_query(ctx, room_small):
    say("case: room scene 20k Gaussians, L=3, 3 training views 800x800, 4 candidates 400x400")
    w = room_small
    prm = oracle_params()
    train = w.train.subset([0, 3, 7])
    b = oracle.vf_build(w.scene, train, 3, prm)
    g = gpu_build(ctx, _dsc(w.scene), train, 3)
    worst, frac = compare_gamma(g, b)
    say(f"  gamma worst {worst:.3f} allowance frac {frac:.4f}")
    assert worst <= 1.0 and frac <= ALLOW_BAR
    g32 = b["gamma"].astype(np.float32).astype(np.float64)
    cand = w.cand.subset([0, 1, 2, 3])
    q = oracle.vf_query(w.scene, g32, 3, train.n, cand, prm)
    s, mp, _ = gpu_query(ctx, _dsc(w.scene), g32, 3, train.n, cand)
    worst, flagged = compare_maps(mp, q)
    say(f"  map worst {worst:.3f} flagged {flagged:.5f}")
    assert worst <= 1.0 and flagged <= flag_bar(q["stats"])
    _check_scores(s, q, mp)
    _check_argmax(ctx, s, q)


def test_room_full_size_sampled(ctx):
    """The room workload at full size (200k Gaussians, 64 candidates 400x400,
    as the benchmark runs it, all views in one call): the oracle recomputes
    two of the views; the build is checked on two full-size training views."""
    w = scenes.workload("room")
    prm = oracle_params()
    say("case: room full size build on 2 of the 100 training views")
    train = w.train.subset([10, 60])
    b = oracle.vf_build(w.scene, train, 3, prm)
    dsc = _dsc(w.scene)
    g = gpu_build(ctx, dsc, train, 3)
    worst, frac = compare_gamma(g, b)
    say(f"  gamma worst {worst:.3f} allowance frac {frac:.4f}")
    assert worst <= 1.0 and frac <= ALLOW_BAR
    say("case: room full size query, 64 views in one call, oracle on views 5 and 40")
    g32 = b["gamma"].astype(np.float32).astype(np.float64)
    s, mp, _ = gpu_query(ctx, dsc, g32, 3, train.n, w.cand)
    sub = w.cand.subset([5, 40])
    q = oracle.vf_query(w.scene, g32, 3, train.n, sub, prm)
    npx = 400 * 400
    mp_sub = np.concatenate([mp[5 * npx:6 * npx], mp[40 * npx:41 * npx]])
    rep = {}
    worst, flagged = compare_maps(mp_sub, q, report=rep)
    say(f"  map worst {worst:.3f} flagged {flagged:.5f} worst pixel rel {rep['pixel_rel']:.2e}")
    assert worst <= 1.0 and flagged <= flag_bar(q["stats"])
    _check_scores(np.array([s[5], s[40]]), q, mp_sub)


def test_paper_geometry_full_size_sampled(ctx):
    """The room scene seen at the paper's image geometry (64 candidates of
    512x512, 90 degrees, all in one call): the oracle recomputes two of the
    views from an oracle field of one training view."""
    w = scenes.workload("ctx512")
    prm = oracle_params()
    say("case: 512x512 geometry, oracle field of training view 30")
    train = w.train.subset([30])
    b = oracle.vf_build(w.scene, train, 3, prm)
    g32 = b["gamma"].astype(np.float32).astype(np.float64)
    say("case: 512x512 geometry query, 64 views in one call, oracle on views 7 and 51")
    s, mp, _ = gpu_query(ctx, _dsc(w.scene), g32, 3, train.n, w.cand)
    sub = w.cand.subset([7, 51])
    q = oracle.vf_query(w.scene, g32, 3, train.n, sub, prm)
    npx = 512 * 512
    mp_sub = np.concatenate([mp[7 * npx:8 * npx], mp[51 * npx:52 * npx]])
    rep = {}
    worst, flagged = compare_maps(mp_sub, q, report=rep)
    say(f"  map worst {worst:.3f} flagged {flagged:.5f} worst pixel rel {rep['pixel_rel']:.2e}")
    assert worst <= 1.0 and flagged <= flag_bar(q["stats"])
    _check_scores(np.array([s[7], s[51]]), q, mp_sub)


def test_batched_full_size_sampled(ctx):
    """The batched workload at full size (1M Gaussians in two rooms; 256
    candidates of mixed 160x120 / 320x240 / 640x480 in one call, as the
    batched form runs): the build is checked on one full-size 1280x720
    training view, the query of all 256 views on one view of each size."""
    w = scenes.workload("batched")
    prm = oracle_params()
    say("case: batched full size build on training view 150 of 300 (1M Gaussians, 1280x720)")
    train = w.train.subset([150])
    b = oracle.vf_build(w.scene, train, 3, prm)
    dsc = _dsc(w.scene)
    g = gpu_build(ctx, dsc, train, 3)
    worst, frac = compare_gamma(g, b)
    say(f"  gamma worst {worst:.3f} allowance frac {frac:.4f}")
    assert worst <= 1.0 and frac <= ALLOW_BAR
    say("case: batched full size query, 256 mixed views in one call, oracle on one view per size")
    g32 = b["gamma"].astype(np.float32).astype(np.float64)
    s, mp, _ = gpu_query(ctx, dsc, g32, 3, train.n, w.cand)
    wh = w.cand.wh.astype(np.int64)
    starts = np.concatenate([[0], np.cumsum(wh[:, 0] * wh[:, 1])])
    idx = [int(np.nonzero(wh[:, 0] == x)[0][0]) for x in (160, 320, 640)]
    q = oracle.vf_query(w.scene, g32, 3, train.n, w.cand.subset(idx), prm)
    mp_sub = np.concatenate([mp[starts[i]:starts[i + 1]] for i in idx])
    rep = {}
    worst, flagged = compare_maps(mp_sub, q, report=rep)
    say(f"  views {idx}: map worst {worst:.3f} flagged {flagged:.5f} worst pixel rel {rep['pixel_rel']:.2e}")
    assert worst <= 1.0 and flagged <= flag_bar(q["stats"])
    _check_scores(s[idx], q, mp_sub)
    say("case: batched full size query as a captured hipGraph: capture, then replays, against the oracle")
    import torch
    from paper_2605_30342_amd import _lib
    gprm = _lib.default_uq_params(use_graph=1)
    ws = ctx.query_workspace(dsc, w.cand, gprm, 3)
    gd = torch.from_numpy(np.ascontiguousarray(g32.T.astype(np.float32))).cuda()
    for it in range(3):
        sg, mg = ctx.vf_query_views(dsc, gd, 3, train.n, w.cand, gprm, ws, want_maps=True)
        st_, _ = ctx.check_workspace(ws)
        assert st_ == 0
        sg, mg = sg.cpu().numpy().astype(np.float64), mg.cpu().numpy().astype(np.float64)
        mg_sub = np.concatenate([mg[starts[i]:starts[i + 1]] for i in idx])
        worst, _ = compare_maps(mg_sub, q)
        say(f"  graph call {it}: map worst {worst:.3f}")
        assert worst <= 1.0
        _check_scores(sg[idx], q, mg_sub)
        assert np.array_equal(sg, s) and np.array_equal(mg, mp)


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_precision_full_size_sampled(ctx, dtype):
    """The precision workload at full size (3M Gaussians, Morton ordered,
    attributes and gamma in FP16 / BF16, 512 candidates 320x240 in one call):
    equal to the FP64 oracle on the same dequantised values, the build on one
    training view, the query on two of the 512 views."""
    import torch
    from paper_2605_30342_amd.api import DeviceScene
    w = scenes.workload("precision")
    prm = oracle_params()
    say(f"case: precision full size {dtype} build on training view 100 of 300 (3M Gaussians)")
    deq = _dequantised(w.scene, dtype)
    dsc = DeviceScene(w.scene, dtype=dtype)
    train = w.train.subset([100])
    b = oracle.vf_build(deq, train, 3, prm)
    g = gpu_build(ctx, dsc, train, 3)
    worst, frac = compare_gamma(g, b)
    say(f"  gamma worst {worst:.3f} allowance frac {frac:.4f}")
    assert worst <= 1.0 and frac <= ALLOW_BAR
    say(f"case: precision full size {dtype} query, 512 views in one call, oracle on views 7 and 300")
    gh = torch.from_numpy(b["gamma"].astype(np.float32)).to(
        torch.float16 if dtype == "f16" else torch.bfloat16).float().numpy().astype(np.float64)
    s, mp, _ = gpu_query(ctx, dsc, gh, 3, train.n, w.cand, gamma_dtype=dtype)
    npx = 320 * 240
    idx = [7, 300]
    q = oracle.vf_query(deq, gh, 3, train.n, w.cand.subset(idx), prm)
    mp_sub = np.concatenate([mp[i * npx:(i + 1) * npx] for i in idx])
    rep = {}
    worst, flagged = compare_maps(mp_sub, q, report=rep)
    say(f"  map worst {worst:.3f} flagged {flagged:.5f} worst pixel rel {rep['pixel_rel']:.2e}")
    assert worst <= 1.0 and flagged <= flag_bar(q["stats"])
    _check_scores(s[idx], q, mp_sub)


# ---------------------------------------------------------------- batching: graph replay

def test_graph_replay_matches_eager(ctx, tiny, tiny_ref):
    """The whole multi-view query captured once in a hipGraph and replayed:
    every replay equals the eager call, also after the cameras change (same
    resolutions) and with other eager work queued between replays."""
    say("case: hipGraph capture/replay of vf_query_views")
    import torch
    from paper_2605_30342_amd import _lib
    _, g32, _ = tiny_ref
    dsc = _dsc(tiny.scene)
    g = torch.from_numpy(np.ascontiguousarray(g32.T.astype(np.float32))).cuda()
    prm_e = _lib.default_uq_params()
    prm_g = _lib.default_uq_params(use_graph=1)
    other = scenes.sphere_cameras(tiny.cand.n, 77, width=128, height=128)
    ws = ctx.query_workspace(dsc, Cameras.concat([tiny.cand, other]), prm_e, 2)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        for it, cams in enumerate([tiny.cand, tiny.cand, other, tiny.cand, other]):
            s_e, m_e = ctx.vf_query_views(dsc, g, 2, tiny.train.n, cams, prm_e, ws, want_maps=True)
            s_e, m_e = s_e.clone(), m_e.clone()
            junk = torch.randn(1 << 20, device="cuda").sum()          # unrelated eager work
            s_g, m_g = ctx.vf_query_views(dsc, g, 2, tiny.train.n, cams, prm_g, ws, want_maps=True)
            stream.synchronize()
            assert torch.equal(s_g, s_e), it
            assert torch.equal(m_g, m_e), it
            del junk
    # the default (legacy) stream works too: capture happens on a private stream
    s_e, _ = ctx.vf_query_views(dsc, g, 2, tiny.train.n, tiny.cand, prm_e, ws)
    s_e = s_e.clone()
    s_g, _ = ctx.vf_query_views(dsc, g, 2, tiny.train.n, tiny.cand, prm_g, ws)
    torch.cuda.synchronize()
    assert torch.equal(s_g, s_e)


def test_persistent_schedules_under_graph_replay(ctx, tiny, tiny_ref):
    """The persistent blend schedules (orders 3 and 4: workgroups draining a
    tile queue through counters that the call clears first) replayed from a
    captured graph several times, with eager work between the replays: every
    replay equals the eager call with the default one-tile schedule."""
    say("case: persistent tile-queue schedules under graph replay")
    import torch
    from paper_2605_30342_amd import _lib
    _, g32, _ = tiny_ref
    dsc = _dsc(tiny.scene)
    g = torch.from_numpy(np.ascontiguousarray(g32.T.astype(np.float32))).cuda()
    prm_e = _lib.default_uq_params()
    prm_g = _lib.default_uq_params(use_graph=1)
    ws = ctx.query_workspace(dsc, tiny.cand, prm_e, 2)
    t0 = ctx.get_tuning()
    try:
        s_ref, m_ref = ctx.vf_query_views(dsc, g, 2, tiny.train.n, tiny.cand, prm_e, ws, want_maps=True)
        s_ref, m_ref = s_ref.clone(), m_ref.clone()
        for order in (3, 4):
            ctx.set_tuning(t0["vis_batch"], t0["uq_batch"], t0["vis_order"], order)
            for it in range(3):
                s_g, m_g = ctx.vf_query_views(dsc, g, 2, tiny.train.n, tiny.cand, prm_g, ws, want_maps=True)
                s_g, m_g = s_g.clone(), m_g.clone()
                junk = torch.randn(1 << 20, device="cuda").sum()          # unrelated eager work
                torch.cuda.synchronize()
                assert torch.equal(s_g, s_ref), (order, it)
                assert torch.equal(m_g, m_ref), (order, it)
                del junk
    finally:
        ctx.set_tuning(**t0)


def test_graph_replay_follows_pixel_count_and_plan(ctx, tiny, tiny_ref):
    """Graph replays with expected-depth maps, alternating two camera sets of
    equal tile counts but different pixel counts (128x128 and 120x120, 8x8
    tiles each) into one preallocated maps buffer: the depth maps start
    right behind each call's entropy maps, so a replay captured for the other
    set must not be reused; every replay equals the eager call."""
    say("case: graph replay, equal tile counts, different pixel counts, depth maps")
    import torch
    from paper_2605_30342_amd import _lib
    _, g32, _ = tiny_ref
    dsc = _dsc(tiny.scene)
    g = torch.from_numpy(np.ascontiguousarray(g32.T.astype(np.float32))).cuda()
    a = tiny.cand
    b = scenes.make_cameras(a.centers, np.zeros((a.n, 3)), 120, 120, 60.0)
    tiles = lambda c: int(np.sum(((c.wh[:, 0] + 15) // 16) * ((c.wh[:, 1] + 15) // 16)))  # noqa: E731
    assert tiles(a) == tiles(b) and a.pixels() != b.pixels()
    prm_e = _lib.default_uq_params()
    prm_g = _lib.default_uq_params(use_graph=1)
    ws = ctx.query_workspace(dsc, Cameras.concat([a, b]), prm_e, 2)
    buf_e = torch.full((2 * a.pixels(),), -7.0, device="cuda")
    buf_g = torch.full((2 * a.pixels(),), -7.0, device="cuda")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        for it, cams in enumerate([a, b, a, b, b, a]):
            n2 = 2 * cams.pixels()
            s_e, _ = ctx.vf_query_views(dsc, g, 2, tiny.train.n, cams, prm_e, ws, maps=buf_e, want_depth=True)
            s_e = s_e.clone()
            s_g, _ = ctx.vf_query_views(dsc, g, 2, tiny.train.n, cams, prm_g, ws, maps=buf_g, want_depth=True)
            stream.synchronize()
            assert torch.equal(s_g, s_e), it
            assert torch.equal(buf_g[:n2], buf_e[:n2]), it
            assert torch.all(buf_g[n2:] == buf_e[n2:]), it       # nothing written past the call's maps


def test_batched_equals_per_view(ctx, tiny, tiny_ref):
    """All candidates in one call equal one call per candidate."""
    say("case: batched vs per-view query")
    import torch
    from paper_2605_30342_amd import _lib
    _, g32, _ = tiny_ref
    dsc = _dsc(tiny.scene)
    g = torch.from_numpy(np.ascontiguousarray(g32.T.astype(np.float32))).cuda()
    prm = _lib.default_uq_params()
    ws = ctx.query_workspace(dsc, tiny.cand, prm, 2)
    s_all, m_all = ctx.vf_query_views(dsc, g, 2, tiny.train.n, tiny.cand, prm, ws, want_maps=True)
    s_all, m_all = s_all.clone(), m_all.clone()
    off = 0
    for v in range(tiny.cand.n):
        s1, m1 = ctx.vf_query_views(dsc, g, 2, tiny.train.n, tiny.cand.subset([v]), prm, ws, want_maps=True)
        torch.cuda.synchronize()
        n = int(tiny.cand.wh[v, 0] * tiny.cand.wh[v, 1])
        assert torch.equal(m1, m_all[off:off + n])
        assert float(s1[0]) == pytest.approx(float(s_all[v]), rel=1e-6)
        off += n


# ---------------------------------------------------------------- precision: half storage

def _dequantised(scene, dtype):
    """The scene exactly as the half-storage kernels see it, rebuilt on the
    host from the FP32 inputs (block anchors + half offsets for the means,
    plain half values for the rest)."""
    import torch
    from paper_2605_30342_amd.api import half_storage
    _, _, deq = half_storage(scene.means, dtype)
    td = torch.float16 if dtype == "f16" else torch.bfloat16

    def rt(a):
        return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(td).float().numpy()
    return Scene(deq, rt(scene.scales), rt(scene.quats), rt(scene.opacity), scene.n_virtual, scene.extent)


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_half_storage_matches_oracle_on_dequantised_inputs(ctx, dtype):
    """FP16/BF16 attributes (means as half offsets from FP32 block anchors)
    and half gamma, FP32 arithmetic: equal to the FP64 oracle run on the same
    dequantised values, to the FP32 tolerances."""
    say(f"case: {dtype} storage, room scene subset")
    w = scenes.workload("room", scale=0.05)
    sc = scenes.subset_scene(w.scene, scenes.morton_order(w.scene))
    prm = oracle_params()
    from paper_2605_30342_amd.api import DeviceScene
    dsc = DeviceScene(sc, dtype=dtype)
    deq = _dequantised(sc, dtype)
    train = w.train.subset([0, 3])
    b = oracle.vf_build(deq, train, 3, prm)
    g = gpu_build(ctx, dsc, train, 3)
    worst, _ = compare_gamma(g, b)
    say(f"  gamma worst {worst:.3f}")
    assert worst <= 1.0
    # gamma stored in the same half type
    import torch
    gh = torch.from_numpy(b["gamma"].astype(np.float32)).to(
        torch.float16 if dtype == "f16" else torch.bfloat16).float().numpy().astype(np.float64)
    cand = w.cand.subset([0, 1])
    q = oracle.vf_query(deq, gh, 3, train.n, cand, prm)
    s, mp, _ = gpu_query(ctx, dsc, gh, 3, train.n, cand, gamma_dtype=dtype)
    worst, flagged = compare_maps(mp, q)
    say(f"  map worst {worst:.3f} flagged {flagged:.5f}")
    assert worst <= 1.0 and flagged <= flag_bar(q["stats"])
    # storage error against FP64 on the original FP32 inputs: reported, sanity-bounded
    q32 = oracle.vf_query(sc, b["gamma"], 3, train.n, cand, prm)
    rel = np.abs(s - q32["scores"]) / np.abs(q32["scores"])
    say(f"  score error vs FP32 inputs: {rel}")
    assert np.all(rel < 0.05)


def test_half_gamma_output_of_build(ctx, tiny):
    """vf_build writing gamma in FP16 / BF16 equals the FP32 result rounded."""
    say("case: half gamma output")
    import torch
    dsc = _dsc(tiny.scene)
    g32 = gpu_build(ctx, dsc, tiny.train, 2)
    for dt, tt in (("f16", torch.float16), ("bf16", torch.bfloat16)):
        gh = gpu_build(ctx, dsc, tiny.train, 2, gamma_dtype=dt).astype(np.float32)
        ref = torch.from_numpy(g32.astype(np.float32)).to(tt).float().numpy()
        # the two builds add float atomics in different orders, so an FP32
        # value next to a rounding boundary of the half format may round to
        # the neighbouring half value; everything else must match exactly
        mant, emin = (10, -14) if dt == "f16" else (7, -126)
        e = np.floor(np.log2(np.maximum(np.abs(ref), 2.0 ** emin)))
        ulp = np.exp2(e - mant)
        diff = np.abs(gh - ref)
        assert np.all(diff <= ulp), dt
        assert np.mean(diff == 0) >= 0.99, (dt, np.mean(diff == 0))


# ---------------------------------------------------------------- serving

def test_serving_results_alone_equal_results_in_the_mix(ctx):
    """Requests of three resident scenes (one stored in BF16 with a BF16
    field) with mixed view counts and resolutions, served with continuous
    batching on concurrent streams under a memory budget: every request's
    scores equal the scores of the same request run alone, and the first
    request of every scene matches the FP64 oracle (fields built by the
    oracle; the BF16 scene against the oracle on its dequantised values)."""
    say("case: continuous-batching server, alone vs mix, and against the oracle")
    import torch
    from paper_2605_30342_amd import _lib
    from paper_2605_30342_amd.api import DeviceScene
    from paper_2605_30342_amd.serve import DONE, GpuBackend, Server
    be = GpuBackend(ctx, n_slots=3)
    rng = np.random.default_rng(5)
    prm_o = oracle_params()
    ora_scene, ora_gamma = {}, {}
    for k in range(3):
        sc = scenes.tiny_scene(1500 + 500 * k, seed=50 + k)
        train = scenes.sphere_cameras(6, 60 + k, width=96, height=96)
        dt = "bf16" if k == 2 else "f32"
        dsc = DeviceScene(sc, dtype=dt)
        seen = _dequantised(sc, dt) if dt == "bf16" else sc
        b = oracle.vf_build(seen, train, 2, prm_o)
        td = torch.bfloat16 if dt == "bf16" else torch.float32
        g = torch.from_numpy(np.ascontiguousarray(b["gamma"].T.astype(np.float32))).to(td).cuda()
        ora_scene[k], ora_gamma[k] = seen, g.float().cpu().numpy().T.astype(np.float64)
        be.add_scene(k, dsc, g, 2, train.n)
    reqs = []
    for i in range(14):
        k = int(rng.integers(0, 3))
        res = [(32, 24), (64, 48), (96, 96)][int(rng.integers(0, 3))]
        cams = scenes.sphere_cameras(int(rng.integers(1, 6)), 100 + i, width=res[0], height=res[1])
        reqs.append((k, cams))
    srv = Server(be, memory_budget=64 << 20, n_slots=3, max_batch_views=12)
    rids = [srv.submit(k, c) for k, c in reqs]
    srv.run_until_idle(timeout=120.0)
    torch.cuda.synchronize()
    st = srv.stats()
    say(f"  {st}")
    assert st["merged_requests"] > 0
    prm = _lib.default_uq_params()
    checked = set()
    for rid, (k, c) in zip(rids, reqs):
        r = srv.requests[rid]
        assert r.status == DONE, r.error
        sc = be.scenes[k]
        s, _ = ctx.vf_query_views(sc.dsc, sc.gamma, 2, sc.n_train, c, prm)
        torch.cuda.synchronize()
        np.testing.assert_allclose(r.scores, s.cpu().numpy(), rtol=1e-6, atol=1e-6)
        if k not in checked:
            q = oracle.vf_query(ora_scene[k], ora_gamma[k], 2, sc.n_train, c, prm_o)
            slack = score_slack(q)
            err = np.abs(r.scores.astype(np.float64) - q["scores"])
            say(f"  scene {k} request {rid}: served vs oracle {err.max():.3e} (slack {slack.min():.3e})")
            assert np.all(err <= slack), (err, slack)
            checked.add(k)
    assert checked == {0, 1, 2}


def test_serving_relaunches_batches_whose_estimate_was_too_small(ctx):
    """With the backend's capacity estimates shrunk below the truth (slack
    0.3 of the learnt per-view rates), batches overflow their workspaces; the
    backend plans them exactly and launches them again on their slot, and
    every request still gets the scores of the same request run alone."""
    say("case: serving with estimates too small: overflow, exact re-plan, relaunch")
    import torch
    from paper_2605_30342_amd import _lib
    from paper_2605_30342_amd.api import DeviceScene
    from paper_2605_30342_amd.serve import DONE, GpuBackend, Server
    be = GpuBackend(ctx, n_slots=2, slack=0.3)
    sc = scenes.tiny_scene(2000, seed=70)
    train = scenes.sphere_cameras(6, 71, width=96, height=96)
    dsc = DeviceScene(sc)
    g = ctx.vf_build(dsc, train, 2)
    be.add_scene("s", dsc, g, 2, train.n)
    reqs = [scenes.sphere_cameras(3 + i % 3, 300 + i, width=64, height=48) for i in range(8)]
    srv = Server(be, memory_budget=1 << 30, n_slots=2, max_batch_views=8)
    rids = [srv.submit("s", c) for c in reqs]
    srv.run_until_idle(timeout=120.0)
    torch.cuda.synchronize()
    say(f"  relaunches {be.relaunches}, exact sizings {be.exact_sizings}, {srv.stats()}")
    assert be.relaunches > 0
    prm = _lib.default_uq_params()
    for rid, c in zip(rids, reqs):
        r = srv.requests[rid]
        assert r.status == DONE, r.error
        s_, _ = ctx.vf_query_views(dsc, g, 2, train.n, c, prm)
        torch.cuda.synchronize()
        np.testing.assert_allclose(r.scores, s_.cpu().numpy(), rtol=1e-6, atol=1e-6)


def test_serving_splits_a_request_larger_than_the_budget(ctx):
    """A request whose exact workspace exceeds the whole memory budget is
    served in chunks of its views; its scores equal the request run alone
    in one call, and a second request behind it is served too."""
    say("case: serving a request larger than the memory budget, in chunks")
    import torch
    from paper_2605_30342_amd import _lib
    from paper_2605_30342_amd.api import DeviceScene
    from paper_2605_30342_amd.serve import DONE, GpuBackend, Server
    be = GpuBackend(ctx, n_slots=2)
    sc = scenes.tiny_scene(2000, seed=80)
    train = scenes.sphere_cameras(6, 81, width=96, height=96)
    dsc = DeviceScene(sc)
    g = ctx.vf_build(dsc, train, 2)
    be.add_scene("s", dsc, g, 2, train.n)
    big = scenes.sphere_cameras(10, 82, width=96, height=96)
    small = scenes.sphere_cameras(2, 83, width=64, height=48)
    prm = _lib.default_uq_params()
    def exact(c):
        return int(ctx.query_plan_exact(dsc, c, prm, 2).bytes)
    full = exact(big)
    # the workspace has a part independent of the view count, so the budget
    # is set to what each half of the request needs
    budget = max(exact(big.subset(range(5))), exact(big.subset(range(5, 10))), exact(small))
    assert budget < full
    srv = Server(be, memory_budget=budget, n_slots=2, max_batch_views=16)
    rb, rs = srv.submit("s", big), srv.submit("s", small)
    srv.run_until_idle(timeout=120.0)
    torch.cuda.synchronize()
    st = srv.stats()
    say(f"  full request {full} bytes, budget {budget}: {st}")
    assert st["split_requests"] == 1 and st["requests_done"] == 2
    for rid, c in ((rb, big), (rs, small)):
        r = srv.requests[rid]
        assert r.status == DONE, r.error
        s_, _ = ctx.vf_query_views(dsc, g, 2, train.n, c, prm)
        torch.cuda.synchronize()
        np.testing.assert_allclose(r.scores, s_.cpu().numpy(), rtol=1e-6, atol=1e-6)


# ---------------------------------------------------------------- density control (Alg. 5)

def test_multiview_visibility_matches_oracle(ctx):
    """Virtual particles (opacity 0, scale s, uniform in the room) measured
    against a room scene from four training views: the GPU's
    1 - prod_p (1 - v_p) equals the oracle's."""
    say("case: density control multi-view visibility")
    import torch
    from paper_2605_30342_amd.api import DeviceScene
    w = scenes.workload("room", scale=0.05)
    train = scenes.ellipse_path_cameras(4, 2001, 200, 200)
    u = scenes.uniform_draws(8000, 2003)
    r = oracle.density_control(w.scene, train, u, [e[0] for e in w.scene.extent], [e[1] for e in w.scene.extent])
    from paper_2605_30342_amd.scenes import Scene
    nv = r["n_virt"]
    allp = Scene(np.concatenate([w.scene.means, r["means"].astype(np.float32)]),
                 np.concatenate([w.scene.scales, np.full((nv, 3), r["s"], np.float32)]),
                 np.concatenate([w.scene.quats, np.tile(np.array([1, 0, 0, 0], np.float32), (nv, 1))]),
                 np.concatenate([w.scene.opacity, np.zeros(nv, np.float32)]), 0, w.scene.extent)
    prm = oracle_params()
    vis_o, allow = oracle.multiview_visibility(allp, train, prm)
    vis_g = ctx.multiview_visibility(DeviceScene(allp), train)
    torch.cuda.synchronize()
    vg = vis_g.cpu().numpy().astype(np.float64)
    err = np.abs(vg - vis_o) / (1e-4 + 2.0 * allow)
    say(f"  worst {err.max():.3f}")
    assert err.max() <= 1.0


def test_density_control_through_the_abi_matches_oracle(ctx):
    """Alg. 5 end to end in the library (vf_density_control: N_virt and s,
    the particles from the uniform draws, their multi-view visibility, the
    eps_v prune and the packing of the kept particles behind the scene)
    against the oracle's Alg. 5 on the same draws: the same count and scale,
    visibility within the near-tie allowance, the same kept set away from
    eps_v, and the kept particles' attributes in the scene's tail."""
    say("case: vf_density_control against the oracle")
    from paper_2605_30342_amd import api
    w = scenes.workload("room", scale=0.05)
    train = scenes.ellipse_path_cameras(4, 2001, 200, 200)
    u = scenes.uniform_draws(8000, 2003)
    lo, hi = [e[0] for e in w.scene.extent], [e[1] for e in w.scene.extent]
    prm = oracle_params()
    r = oracle.density_control(w.scene, train, u.astype(np.float32).astype(np.float64), lo, hi, prm=prm)
    aug, vis, kept, n_virt = api.density_control(ctx, w.scene, train, u)
    say(f"  N_virt {n_virt} (oracle {r['n_virt']}), kept {len(kept)} (oracle {len(r['kept'])})")
    assert n_virt == r["n_virt"]
    assert np.float32(aug.scales[-1, 0] if aug.n_virtual else r["s"]) == np.float32(r["s"])
    err = np.abs(vis.astype(np.float64) - r["vis"]) / (1e-4 + 2.0 * r["allow"])
    say(f"  visibility worst ratio {err.max():.3f}")
    assert err.max() <= 1.0
    far = np.abs(r["vis"] - 0.95) > 1e-4 + 2.0 * r["allow"]
    ko, kg = set(r["kept"].tolist()), set(kept.tolist())
    assert {i for i in ko if far[i]} == {i for i in kg if far[i]}
    assert np.all(np.diff(kept) > 0) and aug.n_virtual == len(kept) and aug.n == w.scene.n + len(kept)
    assert np.array_equal(aug.means[:w.scene.n], w.scene.means)
    assert np.array_equal(aug.means[w.scene.n:], r["means"][kept].astype(np.float32))
    assert np.all(aug.opacity[w.scene.n:] == 0.0) and np.all(aug.quats[w.scene.n:] == [1, 0, 0, 0])


# ---------------------------------------------------------------- launch schedules

def test_schedule_variants_give_identical_results(ctx, tiny, tiny_ref):
    """Every staging batch size (64/128/256) and tile order (workgroup b takes
    tile b, contiguous runs of tiles per XCD, the longest tiles first, and
    persistent workgroups draining a tile queue in tile order or longest
    first) gives bit-identical query maps and gamma equal to FP32 rounding
    (float atomics add in another order); the autotuner picks one of them and
    records its timings."""
    say("case: blend batch-size variants and the autotuner")
    import torch
    from paper_2605_30342_amd import _lib
    from paper_2605_30342_amd.autotune import Autotuner
    _, g32, _ = tiny_ref
    dsc = _dsc(tiny.scene)
    g = torch.from_numpy(np.ascontiguousarray(g32.T.astype(np.float32))).cuda()
    prm = _lib.default_uq_params()
    ws = ctx.query_workspace(dsc, tiny.cand, prm, 2)
    t0 = ctx.get_tuning()
    maps, gams = [], []
    for b in (64, 128, 256):
        for order in (0, 1, 2, 3, 4):
            ctx.set_tuning(b, b, order, order)
            _, m = ctx.vf_query_views(dsc, g, 2, tiny.train.n, tiny.cand, prm, ws, want_maps=True)
            maps.append(m.clone())
            gams.append(gpu_build(ctx, dsc, tiny.train, 2))
    torch.cuda.synchronize()
    for m in maps[1:]:
        assert torch.equal(m, maps[0])
    for gg in gams[1:]:
        assert np.all(np.abs(gg - gams[0]) <= 1e-5 * (np.abs(gams[0]).max(1, keepdims=True) + 1e-30))
    ctx.set_tuning(**t0)
    tuner = Autotuner(ctx)
    r = tuner.tune_query(dsc, g, 2, tiny.train.n, tiny.cand, prm, ws)
    assert r["uq_batch"] in (64, 128, 256) and ctx.get_tuning()["uq_batch"] == r["uq_batch"]
    assert r["uq_order"] in (0, 1, 2, 3, 4) and ctx.get_tuning()["uq_order"] == r["uq_order"] and len(r["ms"]) == 15
    ctx.set_tuning(**t0)
