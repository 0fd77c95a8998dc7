"""FP64 reference checker for the GAVIS visibility-field path.

TEST INFRASTRUCTURE ONLY.  The product library never imports, links or runs
anything in this package; only the tests, the smoke check and the CPU-baseline
leg of the benchmark do.  It shares no code with the GPU path: the C source
`gavis_oracle.c` is compiled on its own with gcc (`build_oracle()`), and this
module only marshals numpy arrays into it.

Every function cites the part of the paper it follows; see gavis_oracle.c for
the step-by-step arithmetic.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gavis_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

_lib = None


def build_oracle(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, OpenMP over pixels)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build_oracle()
        L = ctypes.CDLL(LIB)
        d, i64, i32, vp = ctypes.c_double, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
        L.ora_bessel_i.argtypes = [ctypes.c_int, d]
        L.ora_bessel_i.restype = d
        L.ora_a_l.argtypes = [ctypes.c_int, d]
        L.ora_a_l.restype = d
        L.ora_sh_real.argtypes = [ctypes.c_int, vp, vp]
        L.ora_sh_real.restype = ctypes.c_int
        L.ora_num_threads.restype = ctypes.c_int
        L.ora_virtual_particles.argtypes = [vp, vp, d, d, vp, i64, vp, vp]
        L.ora_virtual_particles.restype = i64
        L.ora_project_view.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, d, d, d, vp]
        L.ora_project_view.restype = ctypes.c_int
        L.ora_vf_build.argtypes = [i64, vp, vp, vp, vp, i32, vp, vp, vp, vp, i32, d, d, d, d, d, i32,
                                   vp, vp, vp, vp]
        L.ora_vf_build.restype = ctypes.c_int
        L.ora_single_view.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, vp, d, d, d, d, i32, vp, vp, vp, vp, vp, vp]
        L.ora_single_view.restype = ctypes.c_int
        L.ora_query_visibility.argtypes = [vp, i32, i64, vp]
        L.ora_query_visibility.restype = d
        L.ora_vf_query.argtypes = [i64, vp, vp, vp, vp, i64, vp, i32, i64, i32, vp, vp, vp, vp,
                                   d, d, d, d, d, d, d, d, i32, vp, vp, vp, vp, vp]
        L.ora_vf_query.restype = ctypes.c_int
        L.ora_vf_query_instr.argtypes = [i64, vp, vp, vp, vp, i64, vp, i32, i64, i32, vp, vp, vp, vp,
                                         d, d, d, d, d, d, d, d, i32, vp, vp, vp, vp, vp, vp, vp]
        L.ora_vf_query_instr.restype = ctypes.c_int
        L.ora_exact_visibility.argtypes = [i64, vp, i64, vp, d, vp, vp]
        L.ora_exact_visibility.restype = d
        L.ora_vf_query_exact.argtypes = [i64, vp, vp, vp, vp, i64, vp, vp, i64, d, i32, vp, vp, vp, vp,
                                         d, d, d, d, d, d, d, d, i32, vp, vp, vp, vp, vp]
        L.ora_vf_query_exact.restype = ctypes.c_int
        L.ora_half_logdet_color.argtypes = [i32, vp, i64, vp]
        L.ora_half_logdet_color.restype = d
        L.ora_vf_query_color.argtypes = [i64, vp, vp, vp, vp, i64, vp, i32, i64, vp, i32, i32, vp, vp, vp, vp,
                                         d, d, d, d, d, d, d, i32, vp, vp, vp, vp, vp]
        L.ora_vf_query_color.restype = ctypes.c_int
        L.ora_vf_query_depth.argtypes = [i64, vp, vp, vp, vp, i64, vp, i32, i64, i32, vp, vp, vp, vp,
                                         d, d, d, d, d, d, d, d, i32, vp, vp, vp, vp, vp]
        L.ora_vf_query_depth.restype = ctypes.c_int
        L.ora_multiview_visibility.argtypes = [i64, vp, vp, vp, vp, i32, vp, vp, vp, vp, d, d, d, d, i32, vp, vp]
        L.ora_multiview_visibility.restype = ctypes.c_int
        L.ora_vf_build_f32.argtypes = [i64, vp, vp, vp, vp, i32, vp, vp, vp, vp, i32, d, d, d, d, d, vp, vp, vp]
        L.ora_vf_build_f32.restype = ctypes.c_int
        L.ora_vf_query_f32.argtypes = [i64, vp, vp, vp, vp, i64, vp, i32, i64, i32, vp, vp, vp, vp,
                                       d, d, d, d, d, d, d, d, vp, vp, vp]
        L.ora_vf_query_f32.restype = ctypes.c_int
        L.ora_argmax.argtypes = [vp, i32]
        L.ora_argmax.restype = i32
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


@dataclass
class Params:
    """Hyperparameters.  kappa = 1 and L = 2 are the paper's defaults; eps_T =
    1e-4, beta = 0.5, o0 = 0.15 and Q0 = I come with Alg. 2 / Alg. 6.  The rest
    are readings where the paper is silent: sigma_c = 0.1 for the constant
    colour covariance Q_c = sigma_c^2 I (so Q0 >= Q_c as the entropy bound
    requires), znear = 0.2, a 0.3 px^2 low-pass dilation of the 2D covariance
    and the 3-sigma overlap cut m <= 9."""
    kappa: float = 1.0
    eps_T: float = 1e-4
    znear: float = 0.2
    lowpass: float = 0.3
    cut: float = 9.0
    beta: float = 0.5
    o0: float = 0.15
    half_logdet_Q0: float = 0.0
    sigma_c: float = 0.1

    @property
    def half_logdet_Qc(self) -> float:
        return 3.0 * float(np.log(self.sigma_c))   # 1/2 log|sigma_c^2 I_3|


def num_threads() -> int:
    return int(lib().ora_num_threads())


def bessel_i(l: int, x: float) -> float:
    """Modified spherical Bessel function i_l(x) (eq. bl)."""
    return float(lib().ora_bessel_i(int(l), float(x)))


def a_l(l: int, kappa: float) -> float:
    """a_l = 4 pi exp(-kappa) i_l(kappa) (Alg. 3, eq. vis_gamma)."""
    return float(lib().ora_a_l(int(l), float(kappa)))


def sh_real(L: int, d) -> np.ndarray:
    """Real SH Y_lm(d), l <= L, index l^2 + l + m (Appendix, eq. vis_real)."""
    d = _f64(d)
    out = np.zeros((L + 1) ** 2)
    if lib().ora_sh_real(int(L), _p(d), _p(out)):
        raise ValueError("bad direction or degree")
    return out


def _cams(cams):
    R = _f64(cams.R.reshape(-1, 9))
    t = _f64(cams.t.reshape(-1, 3))
    K = _f64(cams.K.reshape(-1, 4))
    wh = np.ascontiguousarray(cams.wh.reshape(-1, 2), dtype=np.int32)
    return R, t, K, wh


def project_view(scene, cams, i, prm: Params = Params()):
    """EWA projection of every Gaussian into view i: dict of arrays."""
    R, t, K, wh = _cams(cams)
    m, s, q = _f64(scene.means), _f64(scene.scales), _f64(scene.quats)
    out = np.zeros((scene.n, 10))
    lib().ora_project_view(scene.n, _p(m), _p(s), _p(q), _p(R[i]), _p(t[i]), _p(K[i]), _p(wh[i]),
                           prm.znear, prm.lowpass, prm.cut, _p(out))
    keys = ("ok", "z", "ux", "uy", "ca", "cb", "cc", "sxx", "syy", "band")
    return {k: out[:, j] for j, k in enumerate(keys)}


def single_view(scene, cams, i, prm: Params = Params(), gather_mode: int = 0, want_pixels: bool = False):
    """Alg. 2 for view i: (v [n], count [n], near-tie allowance on v [n]);
    with want_pixels also a dict of per-pixel pairs composited and near-tie
    flags ([h, w]) and the view's counts (pairs, entries, pairs on unflagged
    pixels, entries of flagged pixels, flagged pixels, pixels)."""
    R, t, K, wh = _cams(cams)
    m, s, q, o = _f64(scene.means), _f64(scene.scales), _f64(scene.quats), _f64(scene.opacity)
    v = np.zeros(scene.n)
    c = np.zeros(scene.n, dtype=np.int64)
    pert = np.zeros(scene.n)
    w_, h_ = int(wh[i][0]), int(wh[i][1])
    pxp = np.zeros(w_ * h_, dtype=np.int32) if want_pixels else None
    pxf = np.zeros(w_ * h_, dtype=np.uint8) if want_pixels else None
    counts = np.zeros(6, dtype=np.int64)
    rc = lib().ora_single_view(scene.n, _p(m), _p(s), _p(q), _p(o), _p(R[i]), _p(t[i]), _p(K[i]), _p(wh[i]),
                               prm.eps_T, prm.znear, prm.lowpass, prm.cut, gather_mode, _p(v), _p(c), _p(pert),
                               _p(pxp), _p(pxf), _p(counts))
    if rc:
        raise RuntimeError("oracle single_view failed")
    if want_pixels:
        return v, c, pert, {"pairs": pxp.reshape(h_, w_), "flags": pxf.reshape(h_, w_).astype(bool),
                            "counts": counts}
    return v, c, pert


def vf_build(scene, cams, L: int, prm: Params = Params(), gather_mode: int = 0, want_views: bool = False):
    """Alg. 3 over all views in `cams`.  Returns dict: gamma [n][K], allow
    [n][K] (first-order near-tie allowance on each coefficient), stats
    (pairs composited, list entries, Gaussians with an allowance, views,
    pairs composited on pixels without a near-tie flag, list entries of the
    flagged pixels, flagged pixels, pixels) and vview [V][n] if asked."""
    R, t, K, wh = _cams(cams)
    m, s, q, o = _f64(scene.means), _f64(scene.scales), _f64(scene.quats), _f64(scene.opacity)
    Kc = (L + 1) ** 2
    gamma = np.zeros((scene.n, Kc))
    allow = np.zeros((scene.n, Kc))
    stats = np.zeros(8, dtype=np.int64)
    vview = np.zeros((cams.n, scene.n)) if want_views else None
    rc = lib().ora_vf_build(scene.n, _p(m), _p(s), _p(q), _p(o), cams.n, _p(R), _p(t), _p(K), _p(wh),
                            int(L), prm.kappa, prm.eps_T, prm.znear, prm.lowpass, prm.cut, gather_mode,
                            _p(gamma), _p(vview), _p(allow), _p(stats))
    if rc:
        raise RuntimeError("oracle vf_build failed")
    return {"gamma": gamma, "allow": allow, "stats": stats, "vview": vview}


def query_visibility(gamma_g, L: int, n_train: int, d) -> float:
    """Alg. 4 for one Gaussian (eq. vis_bound with V~ clamped to [0, |P|])."""
    g = _f64(gamma_g)
    d = _f64(d)
    return float(lib().ora_query_visibility(_p(g), int(L), int(n_train), _p(d)))


def vf_query(scene, gamma, L: int, n_train: int, cams, prm: Params = Params(), gather_mode: int = 0,
             want_maps: bool = True, want_vq: bool = False, want_depth: bool = False):
    """Alg. 4 + Alg. 6 for every view in `cams`.  gamma is [n][K] (float64 or
    float32; promoted).  Returns dict: scores [V], maps (list of [h, w]),
    flags (list of [h, w] bool), stats (pairs, entries, flagged px, px,
    pairs on unflagged px, list entries of flagged px), absmaps_flat (per
    pixel the sum of the magnitudes of H's terms), pxpairs_flat (pairs
    composited per pixel), vq,
    and with want_depth the expected-depth maps depth_flat (eq. id's d_p^mn:
    sum w* z / sum w* under the compositing weights, 0 without any)."""
    if want_depth:
        return _vf_query_depth(scene, gamma, L, n_train, cams, prm, gather_mode)
    R, t, K, wh = _cams(cams)
    m, s, q, o = _f64(scene.means), _f64(scene.scales), _f64(scene.quats), _f64(scene.opacity)
    g = _f64(gamma)
    npx = int(np.sum(wh[:, 0].astype(np.int64) * wh[:, 1]))
    maps = np.zeros(npx) if want_maps else None
    pflags = np.zeros(npx, dtype=np.uint8)
    scores = np.zeros(cams.n)
    stats = np.zeros(6, dtype=np.int64)
    vq = np.zeros((cams.n, scene.n)) if want_vq else None
    absmaps = np.zeros(npx) if want_maps else None
    pxpairs = np.zeros(npx, dtype=np.int32)
    rc = lib().ora_vf_query_instr(scene.n, _p(m), _p(s), _p(q), _p(o), int(scene.n_virtual), _p(g), int(L),
                                  int(n_train), cams.n, _p(R), _p(t), _p(K), _p(wh), prm.beta, prm.o0,
                                  prm.half_logdet_Q0, prm.half_logdet_Qc, prm.eps_T, prm.znear, prm.lowpass,
                                  prm.cut, gather_mode, _p(maps), _p(scores), _p(vq), _p(pflags), _p(stats),
                                  _p(absmaps), _p(pxpairs))
    if rc:
        raise RuntimeError("oracle vf_query failed")
    out_maps, out_flags, off = [], [], 0
    for (w, h) in wh:
        n = int(w) * int(h)
        if maps is not None:
            out_maps.append(maps[off:off + n].reshape(h, w))
        out_flags.append(pflags[off:off + n].reshape(h, w).astype(bool))
        off += n
    return {"scores": scores, "maps": out_maps, "flags": out_flags, "stats": stats, "vq": vq,
            "maps_flat": maps, "flags_flat": pflags.astype(bool), "absmaps_flat": absmaps, "pxpairs_flat": pxpairs}


def _vf_query_depth(scene, gamma, L, n_train, cams, prm, gather_mode):
    R, t, K, wh = _cams(cams)
    m, s, q, o = _f64(scene.means), _f64(scene.scales), _f64(scene.quats), _f64(scene.opacity)
    g = _f64(gamma)
    npx = int(np.sum(wh[:, 0].astype(np.int64) * wh[:, 1]))
    maps, depth = np.zeros(npx), np.zeros(npx)
    pflags = np.zeros(npx, dtype=np.uint8)
    scores = np.zeros(cams.n)
    stats = np.zeros(6, dtype=np.int64)
    rc = lib().ora_vf_query_depth(scene.n, _p(m), _p(s), _p(q), _p(o), int(scene.n_virtual), _p(g), int(L),
                                  int(n_train), cams.n, _p(R), _p(t), _p(K), _p(wh), prm.beta, prm.o0,
                                  prm.half_logdet_Q0, prm.half_logdet_Qc, prm.eps_T, prm.znear, prm.lowpass,
                                  prm.cut, gather_mode, _p(maps), _p(depth), _p(scores), _p(pflags), _p(stats))
    if rc:
        raise RuntimeError("oracle vf_query failed")
    out_maps, out_flags, off = [], [], 0
    for (w, h) in wh:
        n = int(w) * int(h)
        out_maps.append(maps[off:off + n].reshape(h, w))
        out_flags.append(pflags[off:off + n].reshape(h, w).astype(bool))
        off += n
    return {"scores": scores, "maps": out_maps, "flags": out_flags, "stats": stats, "vq": None,
            "maps_flat": maps, "flags_flat": pflags.astype(bool), "depth_flat": depth}


def camera_centres(cams) -> np.ndarray:
    """[V][3] camera centres C = -R^T t in FP64."""
    R = np.asarray(cams.R, dtype=np.float64).reshape(-1, 3, 3)
    t = np.asarray(cams.t, dtype=np.float64).reshape(-1, 3)
    return -np.einsum("vji,vj->vi", R, t)


def exact_visibility(vtrain_g, train_centres, kappa: float, x, C) -> float:
    """Exact multi-view visibility of one Gaussian at x seen from C (eq. vis_all
    with eq. vis_p): 1 - prod_p (1 - v_p exp(kappa (d.d_p - 1)))."""
    v = _f64(vtrain_g)
    tc = _f64(train_centres).reshape(-1, 3)
    return float(lib().ora_exact_visibility(len(v), _p(v), 1, _p(tc), float(kappa), _p(_f64(x)), _p(_f64(C))))


def vf_query_exact(scene, vtrain, train_cams, kappa: float, cams, prm: Params = Params(), gather_mode: int = 0,
                   want_maps: bool = True, want_vq: bool = False):
    """Alg. 6 for every view in `cams` with the exact multi-view visibility
    (eq. vis_all) in place of the SH query: vtrain [n_train][n] holds v_p of
    every Gaussian in every training view (as from vf_build(want_views=True)).
    Same outputs as vf_query."""
    R, t, K, wh = _cams(cams)
    m, s, q, o = _f64(scene.means), _f64(scene.scales), _f64(scene.quats), _f64(scene.opacity)
    vt = _f64(vtrain)
    tc = camera_centres(train_cams)
    npx = int(np.sum(wh[:, 0].astype(np.int64) * wh[:, 1]))
    maps = np.zeros(npx) if want_maps else None
    pflags = np.zeros(npx, dtype=np.uint8)
    scores = np.zeros(cams.n)
    stats = np.zeros(6, dtype=np.int64)
    vq = np.zeros((cams.n, scene.n)) if want_vq else None
    rc = lib().ora_vf_query_exact(scene.n, _p(m), _p(s), _p(q), _p(o), int(scene.n_virtual), _p(vt), _p(tc),
                                  int(train_cams.n), float(kappa), cams.n, _p(R), _p(t), _p(K), _p(wh), prm.beta,
                                  prm.o0, prm.half_logdet_Q0, prm.half_logdet_Qc, prm.eps_T, prm.znear,
                                  prm.lowpass, prm.cut, gather_mode, _p(maps), _p(scores), _p(vq), _p(pflags),
                                  _p(stats))
    if rc:
        raise RuntimeError("oracle vf_query_exact failed")
    out_maps, out_flags, off = [], [], 0
    for (w, h) in wh:
        n = int(w) * int(h)
        if maps is not None:
            out_maps.append(maps[off:off + n].reshape(h, w))
        out_flags.append(pflags[off:off + n].reshape(h, w).astype(bool))
        off += n
    return {"scores": scores, "maps": out_maps, "flags": out_flags, "stats": stats, "vq": vq,
            "maps_flat": maps, "flags_flat": pflags.astype(bool)}


def half_logdet_color(Lc: int, var_g, d) -> float:
    """1/2 log|Q_c(d)| of one Gaussian from the variances of its colour SH
    coefficients var_g [3][Kc] (Appendix, integration with FisherRF):
    Q_k(d) = sum_j Y_j(d)^2 var_g[k][j]."""
    v = _f64(var_g).reshape(3, -1)
    if v.shape[1] != (Lc + 1) ** 2:
        raise ValueError("var_g must be [3][(Lc+1)^2]")
    flat = np.ascontiguousarray(v.reshape(-1))
    return float(lib().ora_half_logdet_color(int(Lc), _p(flat), 1, _p(_f64(d))))


def vf_query_color(scene, gamma, L: int, n_train: int, color_var, Lc: int, cams, prm: Params = Params(),
                   gather_mode: int = 0, want_maps: bool = True, want_vq: bool = False):
    """vf_query with the constant colour covariance replaced per Gaussian and
    view by Q_c(d) from the colour SH-coefficient variances color_var
    [3][Kc][n] (Kc = (Lc+1)^2).  prm.sigma_c is not used."""
    R, t, K, wh = _cams(cams)
    m, s, q, o = _f64(scene.means), _f64(scene.scales), _f64(scene.quats), _f64(scene.opacity)
    g = _f64(gamma)
    cv = _f64(color_var)
    if cv.shape != (3, (Lc + 1) ** 2, scene.n):
        raise ValueError("color_var must be [3][(Lc+1)^2][n]")
    npx = int(np.sum(wh[:, 0].astype(np.int64) * wh[:, 1]))
    maps = np.zeros(npx) if want_maps else None
    pflags = np.zeros(npx, dtype=np.uint8)
    scores = np.zeros(cams.n)
    stats = np.zeros(6, dtype=np.int64)
    vq = np.zeros((cams.n, scene.n)) if want_vq else None
    rc = lib().ora_vf_query_color(scene.n, _p(m), _p(s), _p(q), _p(o), int(scene.n_virtual), _p(g), L, n_train,
                                  _p(cv), int(Lc), cams.n, _p(R), _p(t), _p(K), _p(wh), prm.beta, prm.o0,
                                  prm.half_logdet_Q0, prm.eps_T, prm.znear, prm.lowpass, prm.cut, gather_mode,
                                  _p(maps), _p(scores), _p(vq), _p(pflags), _p(stats))
    if rc:
        raise RuntimeError("oracle vf_query_color failed")
    out_maps, out_flags, off = [], [], 0
    for (w, h) in wh:
        n = int(w) * int(h)
        if maps is not None:
            out_maps.append(maps[off:off + n].reshape(h, w))
        out_flags.append(pflags[off:off + n].reshape(h, w).astype(bool))
        off += n
    return {"scores": scores, "maps": out_maps, "flags": out_flags, "stats": stats, "vq": vq,
            "maps_flat": maps, "flags_flat": pflags.astype(bool)}


def multiview_visibility(scene, cams, prm: Params = Params(), gather_mode: int = 0):
    """Alg. 5's multi-view visibility 1 - prod_p (1 - v_p[g]) for every
    Gaussian (v_p from Alg. 2).  Returns (vis [n], allowance [n])."""
    R, t, K, wh = _cams(cams)
    m, s, q, o = _f64(scene.means), _f64(scene.scales), _f64(scene.quats), _f64(scene.opacity)
    vis = np.zeros(scene.n)
    allow = np.zeros(scene.n)
    rc = lib().ora_multiview_visibility(scene.n, _p(m), _p(s), _p(q), _p(o), cams.n, _p(R), _p(t), _p(K), _p(wh),
                                        prm.eps_T, prm.znear, prm.lowpass, prm.cut, gather_mode, _p(vis), _p(allow))
    if rc:
        raise RuntimeError("oracle multiview_visibility failed")
    return vis, allow


def density_control_keep(vis, n_real: int, eps_v: float = 0.95):
    """Alg. 5's pruning rule: a virtual particle (index >= n_real) is kept
    when its multi-view visibility is at most eps_v."""
    vis = np.asarray(vis)
    return np.nonzero(vis[n_real:] <= eps_v)[0] + n_real


@dataclass
class _Gaussians:
    """Attribute arrays of a set of Gaussians (the fields the oracle reads)."""
    means: np.ndarray
    scales: np.ndarray
    quats: np.ndarray
    opacity: np.ndarray
    n_virtual: int = 0

    @property
    def n(self) -> int:
        return int(self.means.shape[0])


def virtual_particles(lo, hi, u, rho: float = 100.0, eta: float = 0.5):
    """Alg. 5's virtual particles in the box [lo, hi]: (means [N_virt][3],
    scale s).  N_virt = floor(rho * volume), positions lo + u (hi - lo) from
    the uniform draws u, scale s with (4/3) pi s^3 rho = 1 + eta."""
    lo, hi, u = _f64(np.asarray(lo)), _f64(np.asarray(hi)), _f64(np.asarray(u))
    n_draw = u.shape[0]
    out = np.zeros((max(n_draw, 1), 3))
    s = np.zeros(1)
    nv = lib().ora_virtual_particles(_p(lo), _p(hi), float(rho), float(eta), _p(u), n_draw, _p(out), _p(s))
    if nv < 0:
        raise ValueError("too few uniform draws for the box and density, or an empty box")
    return out[:nv].copy(), float(s[0])


def density_control(scene, cams, u, lo, hi, rho: float = 100.0, eta: float = 0.5, eps_v: float = 0.95,
                    prm: Params = Params(), stored_f32: bool = True):
    """Alg. 5 end to end: the virtual particles (transparent, identity
    rotation) appended to the scene, the multi-view visibility of everything
    (Alg. 2 per view, 1 - prod (1 - v_p)), and the particles kept (visibility
    at most eps_v).  With stored_f32 the particles' means and scale are
    rounded to FP32, the precision every Gaussian attribute is stored in,
    before they are measured.  Returns dict: n_virt, s, means [N_virt][3],
    vis and allow of the particles [N_virt], kept (particle indices,
    ascending)."""
    means, s = virtual_particles(lo, hi, u, rho, eta)
    if stored_f32:
        means, s = means.astype(np.float32).astype(np.float64), float(np.float32(s))
    nv = means.shape[0]
    allp = _Gaussians(np.concatenate([scene.means.astype(np.float64), means]),
                      np.concatenate([scene.scales.astype(np.float64), np.full((nv, 3), s)]),
                      np.concatenate([scene.quats.astype(np.float64), np.tile([1.0, 0.0, 0.0, 0.0], (nv, 1))]),
                      np.concatenate([scene.opacity.astype(np.float64), np.zeros(nv)]))
    vis, allow = multiview_visibility(allp, cams, prm)
    keep = density_control_keep(vis, scene.n, eps_v) - scene.n
    return {"n_virt": nv, "s": s, "means": means, "vis": vis[scene.n:], "allow": allow[scene.n:], "kept": keep}


def vf_build_f32(scene, cams, L: int, prm: Params = Params()):
    """Alg. 3 over `cams` with Alg. 2 evaluated per pixel in single precision
    (parity bookkeeping only: it checks that the FP64 oracle's near-tie flags
    and allowances cover what float arithmetic can change).  Returns dict:
    gamma [n][K], pxpairs (pairs composited per pixel, packed view after
    view), pairs."""
    R, t, K, wh = _cams(cams)
    m, s, q, o = _f64(scene.means), _f64(scene.scales), _f64(scene.quats), _f64(scene.opacity)
    gamma = np.zeros((scene.n, (L + 1) ** 2))
    pxp = np.zeros(cams.pixels(), dtype=np.int32)
    pairs = np.zeros(1, dtype=np.int64)
    rc = lib().ora_vf_build_f32(scene.n, _p(m), _p(s), _p(q), _p(o), cams.n, _p(R), _p(t), _p(K), _p(wh), int(L),
                                prm.kappa, prm.eps_T, prm.znear, prm.lowpass, prm.cut, _p(gamma), _p(pxp), _p(pairs))
    if rc:
        raise RuntimeError("oracle vf_build_f32 failed")
    return {"gamma": gamma, "pxpairs_flat": pxp, "pairs": int(pairs[0])}


def vf_query_f32(scene, gamma, L: int, n_train: int, cams, prm: Params = Params()):
    """Alg. 4 + Alg. 6 with every per-pixel quantity in single precision
    (parity bookkeeping only, as vf_build_f32).  Returns dict: maps_flat,
    pxpairs_flat, scores."""
    R, t, K, wh = _cams(cams)
    m, s, q, o = _f64(scene.means), _f64(scene.scales), _f64(scene.quats), _f64(scene.opacity)
    g = _f64(gamma)
    npx = cams.pixels()
    maps = np.zeros(npx)
    pxp = np.zeros(npx, dtype=np.int32)
    scores = np.zeros(cams.n)
    rc = lib().ora_vf_query_f32(scene.n, _p(m), _p(s), _p(q), _p(o), int(scene.n_virtual), _p(g), int(L),
                                int(n_train), cams.n, _p(R), _p(t), _p(K), _p(wh), prm.beta, prm.o0,
                                prm.half_logdet_Q0, prm.half_logdet_Qc, prm.eps_T, prm.znear, prm.lowpass, prm.cut,
                                _p(maps), _p(pxp), _p(scores))
    if rc:
        raise RuntimeError("oracle vf_query_f32 failed")
    return {"maps_flat": maps, "pxpairs_flat": pxp, "scores": scores}


def argmax(scores) -> int:
    """Next-best view (eq. i_gain): lowest index on exact ties."""
    s = _f64(scores)
    return int(lib().ora_argmax(_p(s), int(s.shape[0])))


def near_tie_set(scores, abs_h_sums, rel=2e-4):
    """Views whose oracle score lies within tau = rel * max_v sum|H| of the
    best; a GPU argmax inside this set is accepted."""
    s = np.asarray(scores, dtype=np.float64)
    tau = rel * float(np.max(abs_h_sums)) if len(abs_h_sums) else 0.0
    best = float(np.max(s))
    return set(int(i) for i in np.nonzero(s >= best - tau)[0])
