"""Expected-depth maps of the query (the per-pixel depth that eq. id's
spatial-correlation correction takes) on the GPU against the FP64 oracle:
|a - b| <= 1e-4 (|b| + max|b|) on unflagged pixels; the entropy maps and
scores do not change when the depth is requested."""
import numpy as np
import pytest

import oracle
from paper_2605_30342_amd import scenes
from tests._gpu import oracle_params, say
from tests.test_gpu_parity import _dsc, ctx  # noqa: F401

pytestmark = pytest.mark.gpu


def _query(ctx, dsc, gamma_nk, L, n_train, cams, depth, color_var=None):
    import torch
    from paper_2605_30342_amd import _lib
    prm = _lib.default_uq_params()
    ws = ctx.query_workspace(dsc, cams, prm, L)
    g = torch.from_numpy(np.ascontiguousarray(np.asarray(gamma_nk, np.float32).T)).cuda()
    if color_var is None:
        s, mp = ctx.vf_query_views(dsc, g, L, n_train, cams, prm, ws, want_maps=True, want_depth=depth)
    else:
        prm.write_depth = 1 if depth else 0
        cv = torch.from_numpy(np.ascontiguousarray(color_var, np.float32)).cuda()
        s, mp = ctx.vf_query_views_color(dsc, g, L, n_train, cv, cams, prm, ws, want_maps=True)
    st, counts = ctx.check_workspace(ws)
    torch.cuda.synchronize()
    assert st == 0 and counts[2] == 0, counts
    return s.cpu().numpy(), mp.cpu().numpy()


def _check_depth(d_gpu, q):
    ref, flags = q["depth_flat"], q["flags_flat"]
    tol = 1e-4 * (np.abs(ref) + np.abs(ref).max())
    ratio = np.abs(d_gpu.astype(np.float64) - ref) / tol
    ratio[flags] = 0.0
    return float(ratio.max())


@pytest.mark.parametrize("wl", ["tiny", "ragged"])
def test_depth_maps_match_oracle(ctx, wl):
    say(f"case: expected-depth maps, {wl}")
    w = scenes.workload("tiny")
    cams = w.cand
    if wl == "ragged":
        from tests.test_gpu_parity import _ragged_cams
        cams = _ragged_cams(w)
    prm = oracle_params()
    b = oracle.vf_build(w.scene, w.train, 2, prm)
    g32 = b["gamma"].astype(np.float32).astype(np.float64)
    q = oracle.vf_query(w.scene, g32, 2, w.train.n, cams, prm, want_depth=True)
    dsc = _dsc(w.scene)
    s1, m1 = _query(ctx, dsc, g32, 2, w.train.n, cams, True)
    npx = cams.pixels()
    assert m1.size == 2 * npx
    worst = _check_depth(m1[npx:], q)
    say(f"  depth worst ratio {worst:.3f}, flagged px {q['flags_flat'].mean():.5f}")
    assert worst <= 1.0
    s0, m0 = _query(ctx, dsc, g32, 2, w.train.n, cams, False)
    assert np.array_equal(m0, m1[:npx]) and np.array_equal(s0, s1)


def test_depth_with_color_covariance(ctx):
    """The weights do not depend on the colour term, so the colour query's
    depth maps equal the plain query's bit for bit."""
    say("case: expected depth with the per-Gaussian colour covariance")
    w = scenes.workload("tiny")
    b = oracle.vf_build(w.scene, w.train, 2, oracle_params())
    g32 = b["gamma"].astype(np.float32).astype(np.float64)
    dsc = _dsc(w.scene)
    var = scenes.color_sh_variances(w.scene.n, 1, 7200)
    _, mc = _query(ctx, dsc, g32, 2, w.train.n, w.cand, True, color_var=var)
    _, mp = _query(ctx, dsc, g32, 2, w.train.n, w.cand, True)
    npx = w.cand.pixels()
    assert np.array_equal(mc[npx:], mp[npx:])
    assert not np.array_equal(mc[:npx], mp[:npx])
