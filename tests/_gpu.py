"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
compare with the FP64 oracle on identical float32 inputs."""
import sys

import numpy as np

import oracle

# GPU parameters are float32; the oracle gets the same rounded values.
F = lambda x: float(np.float32(x))  # noqa: E731


def oracle_params(kappa=1.0, sigma_c=0.1):
    p = oracle.Params(kappa=F(kappa), eps_T=F(1e-4), znear=F(0.2), lowpass=F(0.3), cut=F(9.0), beta=F(0.5),
                      o0=F(0.15), half_logdet_Q0=0.0, sigma_c=sigma_c)
    return p


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_build(ctx, dsc, cams, L, kappa=1.0, views_per_pass=0, gamma_dtype="f32"):
    from paper_2605_30342_amd import _lib
    prm = _lib.default_vf_params(sh_degree=L, kappa=kappa, views_per_pass=views_per_pass)
    g = ctx.vf_build(dsc, cams, L, prm, gamma_dtype=gamma_dtype)
    import torch
    torch.cuda.synchronize()
    return g.float().cpu().numpy().T.astype(np.float64)     # [n][K]


def gpu_query(ctx, dsc, gamma_nk, L, n_train, cams, sigma_c=0.1, maps=True, gamma_dtype="f32"):
    import torch
    from paper_2605_30342_amd import _lib
    from paper_2605_30342_amd.api import TORCH_DTYPES, DTYPES
    prm = _lib.default_uq_params()
    prm.half_logdet_Qc = float(3.0 * np.log(sigma_c))
    g = torch.from_numpy(np.ascontiguousarray(np.asarray(gamma_nk, np.float32).T)).to(
        TORCH_DTYPES[DTYPES[gamma_dtype]]).cuda()
    ws = ctx.query_workspace(dsc, cams, prm, L)
    scores, mp = ctx.vf_query_views(dsc, g, L, n_train, cams, prm, ws, want_maps=maps)
    st, counts = ctx.check_workspace(ws)
    torch.cuda.synchronize()
    assert st == 0 and counts[2] == 0, counts
    return scores.cpu().numpy().astype(np.float64), (mp.cpu().numpy().astype(np.float64) if maps else None), ws


def compare_maps(gpu_flat, ora, rel=1e-4):
    """Per-pixel |a - b| <= rel (|b| + max|b_map|) on pixels the oracle does
    not flag as near ties.  Returns (worst ratio, flagged fraction)."""
    ref = ora["maps_flat"]
    flags = ora["flags_flat"]
    worst = 0.0
    off = 0
    for m in ora["maps"]:
        n = m.size
        b = ref[off:off + n]
        a = gpu_flat[off:off + n]
        f = flags[off:off + n]
        tol = rel * (np.abs(b) + np.abs(b).max() + 1e-30)
        ratio = np.abs(a - b) / tol
        ratio[f] = 0.0
        worst = max(worst, float(ratio.max()) if n else 0.0)
        off += n
    return worst, float(flags.mean()) if flags.size else 0.0


def compare_gamma(g_gpu, ora_build, rel=1e-4):
    """|d gamma_gk| <= rel ||gamma_g||_inf + 2 allow_gk (+ a tiny absolute
    floor).  Returns (worst ratio, fraction of Gaussians with an allowance)."""
    ref, allow = ora_build["gamma"], ora_build["allow"]
    scale = np.abs(ref).max(1, keepdims=True)
    floor = 1e-7 * max(float(np.abs(ref).max()), 1e-30)
    tol = rel * scale + 2.0 * allow + floor
    ratio = np.abs(g_gpu - ref) / tol
    return float(ratio.max()), float((allow.max(1) > rel * scale[:, 0]).mean())
