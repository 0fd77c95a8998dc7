"""Pins of the FP64 oracle against library routines, closed forms and exact
special cases (no GPU).  Each test names the part of the paper it pins."""
import math

import mpmath
import numpy as np
import pytest
import scipy.special as sp

import oracle
from oracle import Params
from tests._cases import axis_camera, stack_scene

RNG = np.random.default_rng(12345)


def _rand_dirs(n):
    d = RNG.standard_normal((n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


# ---------------------------------------------------------------- special functions

@pytest.mark.parametrize("kappa", [0.0, 0.1, 0.3, 1.0, 3.0, 10.0])
def test_bessel_i_matches_scipy_and_mpmath(kappa):
    """i_l(kappa) of eq. bl / eq. vmf_coeff against scipy and mpmath."""
    for l in range(6):
        ref = float(sp.spherical_in(l, kappa))
        got = oracle.bessel_i(l, kappa)
        assert got == pytest.approx(ref, rel=1e-12, abs=1e-300)
        if kappa > 0:
            mp = mpmath.sqrt(mpmath.pi / (2 * mpmath.mpf(kappa))) * mpmath.besseli(l + 0.5, kappa)
            assert got == pytest.approx(float(mp), rel=1e-12)


def test_bessel_closed_forms():
    """i_0 = sinh x / x, i_1 = (x cosh x - sinh x) / x^2."""
    for x in (0.1, 1.0, 3.0):
        assert oracle.bessel_i(0, x) == pytest.approx(math.sinh(x) / x, rel=1e-14)
        assert oracle.bessel_i(1, x) == pytest.approx((x * math.cosh(x) - math.sinh(x)) / x ** 2, rel=1e-12)


def test_a_l_table_kappa_1():
    """a_l = 4 pi e^{-kappa} i_l(kappa) (Alg. 3) at the paper's kappa = 1."""
    expect = [5.432848644, 1.700673326, 0.330828665, 0.04653000159, 0.005118653843, 4.621170039e-4]
    for l, e in enumerate(expect):
        assert oracle.a_l(l, 1.0) == pytest.approx(e, rel=1e-8)
    for l in range(6):
        ref = 4 * math.pi * math.exp(-1.0) * float(sp.spherical_in(l, 1.0))
        assert oracle.a_l(l, 1.0) == pytest.approx(ref, rel=1e-12)


# ---------------------------------------------------------------- real SH basis

def _real_sh_from_scipy(L, d):
    """The paper's real basis from the complex Y_l^m (eq. vis_real and the
    case split after it), with scipy's complex SH (Condon-Shortley phase)."""
    x, y, z = d
    theta = math.acos(max(-1.0, min(1.0, z)))
    phi = math.atan2(y, x)
    out = np.zeros((L + 1) ** 2)
    for l in range(L + 1):
        for m in range(-l, l + 1):
            if m < 0:
                v = math.sqrt(2) * (-1) ** m * np.imag(sp.sph_harm_y(l, -m, theta, phi))
            elif m == 0:
                v = np.real(sp.sph_harm_y(l, 0, theta, phi))
            else:
                v = math.sqrt(2) * (-1) ** m * np.real(sp.sph_harm_y(l, m, theta, phi))
            out[l * l + l + m] = v
    return out


def test_real_sh_matches_scipy():
    for d in _rand_dirs(50):
        np.testing.assert_allclose(oracle.sh_real(6, d), _real_sh_from_scipy(6, d), rtol=1e-10, atol=1e-12)


def test_real_sh_low_orders_closed_form():
    """l = 1: (Y_{1,-1}, Y_10, Y_11) = sqrt(3/4pi) (y, z, x); l = 2 standard forms."""
    c1 = math.sqrt(3 / (4 * math.pi))
    for x, y, z in _rand_dirs(10):
        Y = oracle.sh_real(2, (x, y, z))
        np.testing.assert_allclose(Y[1:4], c1 * np.array([y, z, x]), rtol=1e-12, atol=1e-14)
        c2 = 0.5 * math.sqrt(15 / math.pi)
        ref2 = [c2 * x * y, c2 * y * z, 0.25 * math.sqrt(5 / math.pi) * (3 * z * z - 1), c2 * x * z,
                0.25 * math.sqrt(15 / math.pi) * (x * x - y * y)]
        np.testing.assert_allclose(Y[4:9], ref2, rtol=1e-12, atol=1e-14)
    assert oracle.sh_real(0, (0, 0, 1))[0] == pytest.approx(0.5 / math.sqrt(math.pi), rel=1e-15)


def test_addition_theorem():
    """sum_m Y_lm(d) Y_lm(d') = (2l+1)/(4 pi) P_l(d . d')  (eq. add_theorem)."""
    for _ in range(20):
        d, e = _rand_dirs(2)
        Yd, Ye = oracle.sh_real(8, d), oracle.sh_real(8, e)
        for l in range(9):
            s = sum(Yd[l * l + l + m] * Ye[l * l + l + m] for m in range(-l, l + 1))
            ref = (2 * l + 1) / (4 * math.pi) * sp.eval_legendre(l, float(np.dot(d, e)))
            assert s == pytest.approx(ref, rel=1e-10, abs=1e-13)


@pytest.mark.parametrize("kappa", [0.3, 1.0, 3.0])
def test_vmf_expansion_converges_to_nu(kappa):
    """nu(d; d_p) = e^{-kappa} e^{kappa d.d_p} = sum_l sum_m a_l Y_lm(d) Y_lm(d_p)
    (eq. SH_vMF, eq. vis_real) -- truncated at l = 8."""
    for _ in range(10):
        d, dp = _rand_dirs(2)
        Yd, Yp = oracle.sh_real(8, d), oracle.sh_real(8, dp)
        s = sum(oracle.a_l(l, kappa) * Yd[l * l + l + m] * Yp[l * l + l + m]
                for l in range(9) for m in range(-l, l + 1))
        nu = math.exp(-kappa) * math.exp(kappa * float(np.dot(d, dp)))
        tail = math.exp(-kappa) * sum((2 * l + 1) * float(sp.spherical_in(l, kappa)) for l in range(9, 60))
        assert abs(s - nu) <= tail + 1e-14


def test_vmf_coefficients_by_quadrature():
    """Project nu(.; d_p) on the real basis by Gauss-Legendre x uniform-phi
    quadrature: the coefficient of Y_k equals a_l Y_k(d_p) (eq. vmf_coeff)."""
    kappa = 1.0
    dp = _rand_dirs(1)[0]
    nt, nphi = 40, 80
    xs, ws = np.polynomial.legendre.leggauss(nt)
    phis = (np.arange(nphi) + 0.5) * 2 * np.pi / nphi
    acc = np.zeros(16)
    for x, w in zip(xs, ws):
        st = math.sqrt(1 - x * x)
        for ph in phis:
            d = np.array([st * math.cos(ph), st * math.sin(ph), x])
            nu = math.exp(kappa * (float(d @ dp) - 1.0))
            acc += w * (2 * np.pi / nphi) * nu * oracle.sh_real(3, d)
    Yp = oracle.sh_real(3, dp)
    expect = np.array([oracle.a_l(l, kappa) * Yp[l * l + l + m] for l in range(4) for m in range(-l, l + 1)])
    np.testing.assert_allclose(acc, expect, rtol=1e-9, atol=1e-12)


# ---------------------------------------------------------------- projection

def test_projection_on_axis_isotropic():
    """EWA: an isotropic Gaussian of scale s at depth z on the optical axis
    projects to the principal point with covariance ((f s / z)^2 + lowpass) I."""
    f, s, z = 100.0, 0.05, 2.0
    cam = axis_camera(64, 48, f)
    sc = stack_scene([z], [0.5], scale=s)
    sc.quats[:] = np.array([0.3, -0.5, 0.2, 0.7], np.float32)   # rotation must not matter
    pr = oracle.project_view(sc, cam, 0, Params(lowpass=0.3))
    s32, f32, z32 = float(np.float32(s)), f, z
    var = (f32 * s32 / z32) ** 2 + 0.3
    assert pr["ok"][0] == 1 and pr["z"][0] == pytest.approx(z, rel=1e-15)
    assert pr["ux"][0] == pytest.approx(32.0) and pr["uy"][0] == pytest.approx(24.0)
    assert pr["ca"][0] == pytest.approx(1 / var, rel=1e-6)
    assert pr["cc"][0] == pytest.approx(1 / var, rel=1e-6)
    assert pr["cb"][0] == pytest.approx(0.0, abs=1e-12)


def test_projection_matches_numerical_jacobian():
    """Off-axis anisotropic Gaussian: Sigma_2D = J Sigma_3D J^T + lowpass I with
    J the Jacobian of the pinhole map, here taken by central differences."""
    from paper_2605_30342_amd.scenes import look_at, Cameras, Scene
    R, t = look_at((0.3, -2.0, 0.4), (0.1, 0.2, 0.0))
    f, cx, cy = 120.0, 40.0, 30.0
    cam = Cameras(R[None].astype(np.float32), t[None].astype(np.float32),
                  np.array([[f, f, cx, cy]], np.float32), np.array([[80, 60]], np.int32))
    mean = np.array([0.25, 0.1, -0.15])
    scale = np.array([0.07, 0.02, 0.04])
    q = np.array([0.8, 0.1, -0.4, 0.3]); q /= np.linalg.norm(q)
    sc = Scene(mean[None].astype(np.float32), scale[None].astype(np.float32), q[None].astype(np.float32),
               np.array([0.5], np.float32))
    Rc, tc = cam.R[0].astype(np.float64), cam.t[0].astype(np.float64)
    m64, s64, q64 = sc.means[0].astype(np.float64), sc.scales[0].astype(np.float64), sc.quats[0].astype(np.float64)
    q64 /= np.linalg.norm(q64)

    def pix(xw):
        p = Rc @ xw + tc
        return np.array([f * p[0] / p[2] + cx, f * p[1] / p[2] + cy])
    J = np.zeros((2, 3))
    h = 1e-6
    for k in range(3):
        e = np.zeros(3); e[k] = h
        J[:, k] = (pix(m64 + e) - pix(m64 - e)) / (2 * h)
    w, x, y, z = q64
    Rq = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                   [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                   [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
    S3 = Rq @ np.diag(s64 ** 2) @ Rq.T
    S2 = J @ S3 @ J.T + 0.3 * np.eye(2)
    conic = np.linalg.inv(S2)
    pr = oracle.project_view(sc, cam, 0, Params(lowpass=0.3))
    u = pix(m64)
    assert pr["ux"][0] == pytest.approx(u[0], rel=1e-12) and pr["uy"][0] == pytest.approx(u[1], rel=1e-12)
    np.testing.assert_allclose([pr["ca"][0], pr["cb"][0], pr["cc"][0]], [conic[0, 0], conic[0, 1], conic[1, 1]],
                               rtol=1e-6)
    np.testing.assert_allclose([pr["sxx"][0], pr["syy"][0]], [S2[0, 0], S2[1, 1]], rtol=1e-6)


def test_behind_camera_is_culled():
    cam = axis_camera(16, 16, 20.0)
    sc = stack_scene([-1.0, 0.1, 0.19, 0.21], [0.9] * 4)
    pr = oracle.project_view(sc, cam, 0, Params(znear=0.2))
    assert list(pr["ok"]) == [0, 0, 0, 1]


# ---------------------------------------------------------------- Alg. 2 / Alg. 3 special cases

def test_single_gaussian_unoccluded_has_visibility_one():
    """Nothing in front: every reached pixel has T = 1, so v = 1 (Alg. 2 with
    the pixel average) and gamma_k = a_l Y_k(d_p) (eq. vis_gamma)."""
    cam = axis_camera(32, 32, 60.0, center=(0.0, 0.0, -3.0))
    sc = stack_scene([0.0], [0.8], scale=0.1, x=0.05, y=-0.02)
    v, c, _ = oracle.single_view(sc, cam, 0)
    assert c[0] > 20 and v[0] == 1.0
    b = oracle.vf_build(sc, cam, 3)
    d = sc.means[0].astype(np.float64) - np.array([0, 0, -3.0])
    Y = oracle.sh_real(3, d)
    expect = np.array([oracle.a_l(l, 1.0) * Y[l * l + l + m] for l in range(4) for m in range(-l, l + 1)])
    np.testing.assert_allclose(b["gamma"][0], expect, rtol=1e-14, atol=1e-15)


def test_query_single_view_closed_form():
    """|P| = 1 and d = d_p: V = V~ = e^{-kappa} sum_{l<=L} (2l+1) i_l(kappa)
    (addition theorem), 0.9699708 for kappa = 1, L = 2 and 0.9958899 for L = 3."""
    cam = axis_camera(32, 32, 60.0, center=(0.0, 0.0, -3.0))
    sc = stack_scene([0.0], [0.8], scale=0.1)
    for L, expect in ((2, 0.9699708), (3, 0.9958899)):
        g = oracle.vf_build(sc, cam, L)["gamma"][0]
        V = oracle.query_visibility(g, L, 1, (0.0, 0.0, 1.0))
        closed = math.exp(-1.0) * sum((2 * l + 1) * float(sp.spherical_in(l, 1.0)) for l in range(L + 1))
        assert V == pytest.approx(closed, rel=1e-12)
        assert V == pytest.approx(expect, abs=5e-8)


def test_kappa_zero_is_isotropic():
    """kappa = 0 (the paper's isotropic ablation): only gamma_00 = 2 sqrt(pi)
    sum_p v_p is nonzero, and V~ is the same in every direction."""
    from paper_2605_30342_amd import scenes
    w = scenes.workload("tiny", scale=0.25)
    b = oracle.vf_build(w.scene, w.train, 2, Params(kappa=0.0), want_views=True)
    g = b["gamma"]
    assert np.all(g[:, 1:] == 0.0)
    np.testing.assert_allclose(g[:, 0], 2 * math.sqrt(math.pi) * b["vview"].sum(0), rtol=1e-13)
    nt = w.train.n
    for d in _rand_dirs(3):
        for i in range(5):
            Vt = g[i, 0] * oracle.sh_real(2, d)[0]
            expect = 1 - (1 - min(Vt, nt) / nt) ** nt
            assert oracle.query_visibility(g[i], 2, nt, d) == pytest.approx(expect, rel=1e-13, abs=1e-15)


def test_transmittance_stack_and_termination():
    """Gaussians centred on a 1x1 image's pixel (m = 0, alpha = o = 1/2): the
    k-th receives T = 2^{-(k-1)} (front to back by depth, whatever their
    index order); T < eps_T = 1e-4 first holds after the 14th (T = 2^-14), so
    the 15th and later are never reached and get v = 0 (Alg. 2)."""
    zs = np.arange(1.0, 17.0)[::-1]        # index 0 is the farthest
    sc = stack_scene(zs, [0.5] * 16, scale=0.01)
    cam = axis_camera(1, 1, 50.0)
    v, c, _ = oracle.single_view(sc, cam, 0)
    order = np.argsort(zs)
    for rank, g in enumerate(order):
        if rank < 14:
            assert c[g] == 1 and v[g] == 2.0 ** (-rank)
        else:
            assert c[g] == 0 and v[g] == 0.0


def test_full_occlusion_gives_zero():
    """Three large opaque occluders (o = 0.99) in front of a small target: T
    after them is 1e-6 < eps_T, so the target is never reached, v = 0 and its
    gamma is 0.  Also: a Gaussian off-image or behind the camera gets v = 0."""
    cam = axis_camera(24, 24, 40.0, center=(0.0, 0.0, -3.0))
    zs = [-1.0, -1.1, -1.2, 0.0, 0.0, -3.5]
    sc = stack_scene(zs, [0.99, 0.99, 0.99, 0.7, 0.7, 0.7], scale=0.05)
    sc.scales[:3] = 2.0                        # occluders cover the whole image
    sc.means[4, 0] = 50.0                      # far off-image
    v, c, _ = oracle.single_view(sc, cam, 0)
    assert c[3] == 0 and v[3] == 0.0
    assert c[4] == 0 and v[4] == 0.0 and c[5] == 0 and v[5] == 0.0
    assert np.all(v[:3] > 0)
    g = oracle.vf_build(sc, cam, 2)["gamma"]
    assert np.all(g[3:] == 0.0)


def test_two_gaussians_in_depth_order():
    """Front Gaussian (higher index) with alpha1 = 0.7 at the pixel centre: the
    one behind receives T = 1 - alpha1 (Alg. 2, sorted by increasing z)."""
    sc = stack_scene([3.0, 2.0], [0.4, 0.7], scale=0.01)
    cam = axis_camera(1, 1, 50.0)
    v, c, _ = oracle.single_view(sc, cam, 0)
    assert v[1] == 1.0 and v[0] == pytest.approx(1 - np.float32(0.7), rel=1e-15)


def test_pixel_average_of_transmittance():
    """A back Gaussian seen through a front one over part of its footprint:
    v = mean over its covered pixels of T, T = 1 - alpha_front(pixel) where the
    front one overlaps.  Checked by brute force against the definition."""
    from paper_2605_30342_amd.scenes import Scene
    cam = axis_camera(12, 12, 30.0)
    sc = Scene(np.array([[0.0, 0.0, 4.0], [0.05, 0.0, 2.0]], np.float32),
               np.array([[0.3, 0.3, 0.3], [0.04, 0.04, 0.04]], np.float32),
               np.tile(np.array([1, 0, 0, 0], np.float32), (2, 1)), np.array([0.6, 0.8], np.float32))
    prm = Params()
    v, c, _ = oracle.single_view(sc, cam, 0, prm)
    pr0 = oracle.project_view(sc, cam, 0, prm)
    tot, cnt = 0.0, 0
    for j in range(12):
        for i in range(12):
            q = np.array([i + 0.5, j + 0.5])

            def m_of(g):
                d = q - np.array([pr0["ux"][g], pr0["uy"][g]])
                C = np.array([[pr0["ca"][g], pr0["cb"][g]], [pr0["cb"][g], pr0["cc"][g]]])
                return float(d @ C @ d)
            if m_of(0) > 9:
                continue
            T = 1.0
            if m_of(1) <= 9:
                T = 1 - float(np.float32(0.8)) * math.exp(-0.5 * m_of(1))
            tot += T
            cnt += 1
    assert c[0] == cnt and v[0] == pytest.approx(tot / cnt, rel=1e-12)


# ---------------------------------------------------------------- AM-GM bound and truncation

def test_am_gm_is_a_lower_bound_and_tight_for_equal_views():
    """1 - (1 - sum V_p / |P|)^|P| <= 1 - prod (1 - V_p), equality when all
    V_p are equal (eq. vis_bound, Appendix derivation)."""
    for _ in range(50):
        P = int(RNG.integers(1, 12))
        Vp = RNG.uniform(0, 1, P)
        bound = 1 - (1 - Vp.sum() / P) ** P
        exact = 1 - np.prod(1 - Vp)
        assert bound <= exact + 1e-15
    Vp = np.full(7, 0.3)
    assert 1 - (1 - Vp.sum() / 7) ** 7 == pytest.approx(1 - np.prod(1 - Vp), rel=1e-14)
    assert 1 - np.prod(1 - Vp) == pytest.approx(0.9176457, abs=1e-7)


def test_query_equal_views_equals_exact_product():
    """|P| copies of the same training view: all V_p equal, so the oracle's
    query equals 1 - (1 - V_1)^|P| with V_1 the single-view query."""
    cam1 = axis_camera(32, 32, 60.0, center=(0.0, 0.0, -3.0))
    sc = stack_scene([0.0, -0.5], [0.8, 0.4], scale=0.1)
    from paper_2605_30342_amd.scenes import Cameras
    P = 5
    camP = Cameras(np.repeat(cam1.R, P, 0), np.repeat(cam1.t, P, 0), np.repeat(cam1.K, P, 0),
                   np.repeat(cam1.wh, P, 0))
    g1 = oracle.vf_build(sc, cam1, 2)["gamma"]
    gP = oracle.vf_build(sc, camP, 2)["gamma"]
    np.testing.assert_allclose(gP, P * g1, rtol=1e-13, atol=1e-15)
    for d in _rand_dirs(5):
        for g in range(2):
            V1 = oracle.query_visibility(g1[g], 2, 1, d)
            VP = oracle.query_visibility(gP[g], 2, P, d)
            assert VP == pytest.approx(1 - (1 - V1) ** P, rel=1e-12, abs=1e-15)


def test_truncation_bound():
    """|V~_L(d) - sum_p v_p nu(d; d_p)| <= |P| e^{-kappa} sum_{l>L} (2l+1) i_l(kappa)."""
    from paper_2605_30342_amd import scenes
    w = scenes.workload("tiny", scale=0.2)
    for L in (2, 3):
        b = oracle.vf_build(w.scene, w.train, L, want_views=True)
        C = w.train.centers
        tail = math.exp(-1.0) * sum((2 * l + 1) * float(sp.spherical_in(l, 1.0)) for l in range(L + 1, 60))
        for g in range(0, w.scene.n, 37):
            x = w.scene.means[g].astype(np.float64)
            for d in _rand_dirs(3):
                Vt = float(b["gamma"][g] @ oracle.sh_real(L, d))
                full = 0.0
                for p in range(w.train.n):
                    dp = x - C[p]
                    dp /= np.linalg.norm(dp)
                    full += b["vview"][p, g] * math.exp(-1.0) * math.exp(float(d @ dp))
                assert abs(Vt - full) <= w.train.n * tail + 1e-12


# ---------------------------------------------------------------- Alg. 6 closed forms

def _single_pixel_query(v_target, alpha, sigma_c):
    """1x1 image, one Gaussian on the pixel centre (alpha = o), |P| = 1 and
    gamma chosen so that V~ = v_target in every direction (gamma_00 only)."""
    sc = stack_scene([2.0], [alpha], scale=0.01)
    cam = axis_camera(1, 1, 50.0)
    g = np.zeros((1, 9))
    g[0, 0] = v_target / (0.5 / math.sqrt(math.pi))
    prm = Params(sigma_c=sigma_c)
    return oracle.vf_query(sc, g, 2, 1, cam, prm)["maps"][0][0, 0]


@pytest.mark.parametrize("sigma_c,expect", [(1.0, (1.964116820, 2.763358537, 2.860584734)),
                                            (0.1, (1.964116820, 1.079593188, -1.284068433))])
def test_uq_single_gaussian_closed_form(sigma_c, expect):
    """With T = 1: alpha* = (v + beta(1-v)) alpha + o0 (1-beta)(1-v) (eq.
    alpha_comp), x = alpha* v, y = alpha* (1 - v) and
    H = -x log x + x c_c - y log y + y c_0 (eq. huber, D = 3), c = 1/2 log|Q| +
    3/2 log(2 pi e); beta = 0.5, o0 = 0.15, Q0 = I (Alg. 6 defaults)."""
    alpha = float(np.float32(0.6))
    for v, e in zip((0.0, 0.5, 1.0), expect):
        a = (v + 0.5 * (1 - v)) * alpha + 0.15 * 0.5 * (1 - v)
        x, y = a * v, a * (1 - v)
        c3 = 1.5 * math.log(2 * math.pi * math.e)
        cc, c0 = 3 * math.log(sigma_c) + c3, c3

        def xl(t):
            return -t * math.log(t) if t > 0 else 0.0
        closed = xl(x) + x * cc + xl(y) + y * c0
        got = _single_pixel_query(v, alpha, sigma_c)
        assert got == pytest.approx(closed, rel=1e-12)
        assert got == pytest.approx(e, abs=2e-7)


def test_uq_invisible_everything_is_prior_only():
    """n_train = 0 gives V = 0 for every Gaussian: only the prior component
    w0 contributes, H = -w0 log w0 + w0 c_0 with w0 = 1 - T_end."""
    sc = stack_scene([2.0, 3.0], [0.6, 0.5], scale=0.01)
    cam = axis_camera(1, 1, 50.0)
    out = oracle.vf_query(sc, np.zeros((2, 9)), 2, 0, cam)
    a1 = 0.5 * float(np.float32(0.6)) + 0.075
    a2 = 0.5 * float(np.float32(0.5)) + 0.075
    w0 = a1 + (1 - a1) * a2
    c3 = 1.5 * math.log(2 * math.pi * math.e)
    assert out["maps"][0][0, 0] == pytest.approx(-w0 * math.log(w0) + w0 * c3, rel=1e-12)


def test_argmax_lowest_index_on_ties():
    assert oracle.argmax([1.0, 3.0, 3.0, 2.0]) == 1
    assert oracle.argmax([float("nan"), -1.0]) == 1
    assert oracle.argmax([-5.0]) == 0


# ---------------------------------------------------------------- density control (Alg. 5)

def test_virtual_particle_constants():
    """The oracle's Alg. 5 particles: N_virt = floor(rho Vol) (6 x 4 x 3 m at
    rho = 100: 7200; a 1.25 x 1 x 1 box: 125), the scale's
    defining identity (4/3) pi s^3 rho = 1 + eta and its value at rho = 100,
    eta = 0.5, and positions lo + u (hi - lo) (u = 0 at the low corner, u
    near 1 at the high one, a middle draw in the middle)."""
    lo, hi = (0.0, 0.0, 0.0), (6.0, 4.0, 3.0)
    u = np.full((7200, 3), 0.5)
    u[0] = 0.0
    u[1] = 1.0 - 2.0 ** -40
    means, s = oracle.virtual_particles(lo, hi, u, 100.0, 0.5)
    assert means.shape == (7200, 3)
    assert 4.0 / 3.0 * math.pi * s ** 3 * 100.0 == pytest.approx(1.5, rel=1e-12)
    assert s == pytest.approx(0.152992, abs=1e-6)
    assert np.array_equal(means[0], [0.0, 0.0, 0.0])
    assert np.allclose(means[1], hi, atol=1e-11) and np.all(means[1] < hi)
    assert np.array_equal(means[2], [3.0, 2.0, 1.5])
    m2, _ = oracle.virtual_particles((1.0, -2.0, 0.5), (2.25, -1.0, 1.5), np.full((200, 3), 0.25), 100.0, 0.5)
    assert m2.shape[0] == 125 and np.array_equal(m2[0], [1.3125, -1.75, 0.75])
    with pytest.raises(ValueError):
        oracle.virtual_particles(lo, hi, u[:7199], 100.0, 0.5)      # too few draws
    m3, s3 = oracle.virtual_particles(lo, hi, u, 10.0, 0.0)
    assert m3.shape[0] == 720 and 4.0 / 3.0 * math.pi * s3 ** 3 * 10.0 == pytest.approx(1.0, rel=1e-12)


def test_density_control_keeps_the_hidden_particles():
    """Alg. 5 end to end on a 1x1 view of a wall of three opaque occluders: a
    box that holds one particle in front of the wall (visible, multi-view
    visibility 1, pruned) and one behind it (never reached, 0, kept)."""
    from paper_2605_30342_amd.scenes import Cameras
    cam1 = axis_camera(1, 1, 50.0)
    cam2 = Cameras(np.repeat(cam1.R, 2, 0), np.repeat(cam1.t, 2, 0), np.repeat(cam1.K, 2, 0), np.repeat(cam1.wh, 2, 0))
    wall = stack_scene([1.0, 1.1, 1.2], [0.99, 0.99, 0.99], scale=0.01)
    # box 0.02 x 0.02 x 2.5 at rho = 2000 / (0.02 * 0.02 * 2.5) holds 2000 particles; two draws matter
    lo, hi = (-0.01, -0.01, 0.3), (0.01, 0.01, 2.8)
    rho = 2000.0 / (0.02 * 0.02 * 2.5) * (1 + 1e-9)
    u = np.full((2000, 3), 0.5)
    u[:, 2] = np.where(np.arange(2000) % 2 == 0, 0.1, 0.9)       # z = 0.55 (in front) or 2.55 (behind)
    r = oracle.density_control(wall, cam2, u, lo, hi, rho=rho, eta=0.5, eps_v=0.95)
    assert r["n_virt"] == 2000
    assert np.all(r["vis"][0::2] == 1.0) and np.all(r["vis"][1::2] == 0.0)
    assert np.array_equal(r["kept"], np.arange(1, 2000, 2))


def test_multiview_visibility_special_cases():
    """A transparent (opacity 0) particle alone in view has v = 1 (T = 1 on
    every reached pixel), so its multi-view visibility is 1 and it is pruned;
    behind a 50 % occluder on a single pixel it has v = 1/2 per view, so two
    identical views give 1 - (1/2)^2 = 3/4; behind three opaque occluders it
    is never reached (0, kept).  A particle of opacity 0 never occludes."""
    cam1 = axis_camera(1, 1, 50.0)
    from paper_2605_30342_amd.scenes import Cameras
    cam2 = Cameras(np.repeat(cam1.R, 2, 0), np.repeat(cam1.t, 2, 0), np.repeat(cam1.K, 2, 0), np.repeat(cam1.wh, 2, 0))
    sc = stack_scene([2.0], [0.0], scale=0.01)
    vis, _ = oracle.multiview_visibility(sc, cam2)
    assert vis[0] == 1.0
    sc = stack_scene([1.0, 2.0], [0.5, 0.0], scale=0.01)       # occluder alpha = 1/2 at the pixel centre
    vis, _ = oracle.multiview_visibility(sc, cam2)
    assert vis[1] == pytest.approx(0.75, rel=1e-12)
    sc = stack_scene([1.0, 1.1, 1.2, 2.0], [0.99, 0.99, 0.99, 0.0], scale=0.01)
    vis, _ = oracle.multiview_visibility(sc, cam2)
    assert vis[3] == 0.0
    assert list(oracle.density_control_keep(vis, 3)) == [3]
    sc = stack_scene([1.0, 2.0], [0.0, 0.7], scale=0.01)       # transparent in front of a real one
    v, c, _ = oracle.single_view(sc, cam1, 0)
    assert v[1] == 1.0


# ---------------------------------------------------------------- exact multi-view visibility (eq. vis_all)

def _unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


def test_exact_visibility_single_view_closed_forms():
    """One training view: V = v_p nu(d; d_p) = v_p e^{kappa (cos theta - 1)}.
    Gaussian at the origin, training camera on -z.  Queried from the same
    centre theta = 0 and V = v_p; from +x (theta = 90 deg) V = v_p e^{-kappa};
    from +z (theta = 180 deg) V = v_p e^{-2 kappa}.  v_p = 0.6, kappa = 1:
    0.6, 0.2207277, 0.0812012."""
    x = np.zeros(3)
    Cp = np.array([[0.0, 0.0, -3.0]])
    v = [0.6]
    for C, expect in (((0.0, 0.0, -2.0), 0.6), ((5.0, 0.0, 0.0), 0.2207277), ((0.0, 0.0, 4.0), 0.0812012)):
        got = oracle.exact_visibility(v, Cp, 1.0, x, C)
        assert got == pytest.approx(expect, abs=5e-8)
    # kappa = 0 is isotropic: V = v_p from every direction
    assert oracle.exact_visibility(v, Cp, 0.0, x, (0.0, 4.0, 0.0)) == pytest.approx(0.6, rel=1e-15)
    # a Gaussian at the querying centre has no direction: V = 0
    assert oracle.exact_visibility(v, Cp, 1.0, x, (0.0, 0.0, 0.0)) == 0.0


def test_exact_visibility_two_views_by_hand():
    """Two training views on -z and +x of a Gaussian at the origin, v = (0.5,
    0.3), queried from -z: view 1 is aligned (nu = 1), view 2 is at 90 deg
    (nu = e^{-1}), so V = 1 - 0.5 (1 - 0.3/e) = 0.5551819 (kappa = 1)."""
    Cp = np.array([[0.0, 0.0, -3.0], [2.0, 0.0, 0.0]])
    got = oracle.exact_visibility([0.5, 0.3], Cp, 1.0, np.zeros(3), (0.0, 0.0, -1.0))
    assert got == pytest.approx(0.5551819, abs=5e-8)
    # a view with v_p = 0 changes nothing; a view with v_p nu = 1 makes V = 1
    assert oracle.exact_visibility([0.5, 0.0], Cp, 1.0, np.zeros(3), (0.0, 0.0, -1.0)) == pytest.approx(0.5)
    assert oracle.exact_visibility([1.0, 0.3], Cp, 1.0, np.zeros(3), (0.0, 0.0, -1.0)) == 1.0


def test_sh_query_approaches_exact_for_identical_views():
    """|P| copies of one training view: all v_p nu_p are equal, so the AM-GM
    bound is tight (eq. vis_bound) and the SH query (Alg. 4) differs from the
    exact product only by the truncated tail: |V_L - V_exact| <= |P| e^{-kappa}
    sum_{l>L} (2l+1) i_l(kappa).  Ties the SH path (Bessel table, real SH,
    addition theorem) to the direct product."""
    from paper_2605_30342_amd.scenes import Cameras
    cam1 = axis_camera(32, 32, 60.0, center=(0.0, 0.0, -3.0))
    P = 4
    camP = Cameras(np.repeat(cam1.R, P, 0), np.repeat(cam1.t, P, 0), np.repeat(cam1.K, P, 0),
                   np.repeat(cam1.wh, P, 0))
    sc = stack_scene([0.0, -0.5], [0.8, 0.4], scale=0.1)
    Cp = oracle.camera_centres(camP)
    np.testing.assert_allclose(Cp, np.tile([0.0, 0.0, -3.0], (P, 1)), atol=1e-7)
    for L in (2, 3):
        b = oracle.vf_build(sc, camP, L, want_views=True)
        tail = math.exp(-1.0) * sum((2 * l + 1) * float(sp.spherical_in(l, 1.0)) for l in range(L + 1, 60))
        for g in range(2):
            x = sc.means[g].astype(np.float64)
            for d in _rand_dirs(6):
                C = x - 2.5 * _unit(d)                 # query camera seeing x along d
                Vq = oracle.query_visibility(b["gamma"][g], L, P, d)
                Ve = oracle.exact_visibility(b["vview"][:, g], Cp, 1.0, x, C)
                assert abs(Vq - Ve) <= P * tail + 1e-12


def test_exact_visibility_dominates_am_gm_of_exact_sum():
    """For distinct training views the exact product is never below the AM-GM
    bound of the same (untruncated) sum (eq. vis_bound): with S = sum_p v_p
    nu_p, 1 - (1 - S/|P|)^|P| <= V_exact.  The SH query at L = 3 follows the
    bound to within the truncation tail."""
    from paper_2605_30342_amd import scenes
    w = scenes.workload("tiny", scale=0.2)
    L = 3
    b = oracle.vf_build(w.scene, w.train, L, want_views=True)
    Cp = oracle.camera_centres(w.train)
    P = w.train.n
    tail = math.exp(-1.0) * sum((2 * l + 1) * float(sp.spherical_in(l, 1.0)) for l in range(L + 1, 60))
    checked = 0
    for g in range(0, w.scene.n, 41):
        x = w.scene.means[g].astype(np.float64)
        for d in _rand_dirs(3):
            C = x - 2.0 * _unit(d)
            Ve = oracle.exact_visibility(b["vview"][:, g], Cp, 1.0, x, C)
            Vq = oracle.query_visibility(b["gamma"][g], L, P, d)
            assert Vq <= Ve + P * tail + 1e-12
            checked += 1
    assert checked > 10


def test_vf_query_exact_single_pixel_closed_form():
    """1x1 image, one Gaussian on the pixel centre, one training view equal to
    the querying camera: V = v_p exactly, so the map matches the closed form of
    eq. alpha_comp / eq. huber with that v (as for the SH query; sigma_c = 1
    so that c_c = c_0)."""
    sc = stack_scene([2.0], [0.6], scale=0.01)
    cam = axis_camera(1, 1, 50.0)
    alpha = float(np.float32(0.6))
    c3 = 1.5 * math.log(2 * math.pi * math.e)

    def xl(t):
        return -t * math.log(t) if t > 0 else 0.0
    for v in (0.0, 0.25, 1.0):
        out = oracle.vf_query_exact(sc, np.array([[v]]), cam, 1.0, cam, Params(sigma_c=1.0), want_vq=True)
        assert out["vq"][0, 0] == pytest.approx(v, rel=1e-15)
        a = (v + 0.5 * (1 - v)) * alpha + 0.15 * 0.5 * (1 - v)
        closed = xl(a * v) + a * v * c3 + xl(a * (1 - v)) + a * (1 - v) * c3
        assert out["maps"][0][0, 0] == pytest.approx(closed, rel=1e-12)


def test_vf_query_exact_virtual_particles_and_no_views():
    """Virtual particles have V = 0 in the exact mode too, and with no training
    view every V is 0: the maps equal those of the SH query with n_train = 0."""
    from paper_2605_30342_amd import scenes
    w = scenes.workload("tiny", scale=0.25)
    nv = 40
    sc = scenes.Scene(w.scene.means, w.scene.scales, w.scene.quats, w.scene.opacity, n_virtual=nv)
    b = oracle.vf_build(sc, w.train, 2, want_views=True)
    out = oracle.vf_query_exact(sc, b["vview"], w.train, 1.0, w.cand, want_vq=True)
    assert np.all(out["vq"][:, sc.n - nv:] == 0.0) and np.any(out["vq"][:, :sc.n - nv] > 0.5)
    assert np.all(out["vq"] >= 0.0) and np.all(out["vq"] <= 1.0)
    empty = oracle.vf_query_exact(sc, np.zeros((0, sc.n)), scenes.Cameras(
        w.train.R[:0], w.train.t[:0], w.train.K[:0], w.train.wh[:0]), 1.0, w.cand)
    ref = oracle.vf_query(sc, np.zeros((sc.n, 9)), 2, 0, w.cand)
    np.testing.assert_allclose(empty["scores"], ref["scores"], rtol=1e-13)


# ---------------------------------------------------------------- colour covariance from SH variances (FisherRF hook)

def test_color_covariance_unsold_isotropy():
    """Equal variances s for every coefficient of degree <= Lc: by Unsold's
    theorem sum_m Y_lm(d)^2 = (2l+1)/(4 pi), so Q_k = s (Lc+1)^2 / (4 pi) in
    every direction; s = 0.05, Lc = 3: 1/2 log|Q_c| = -4.1312517."""
    for Lc in (0, 1, 2, 3):
        var = np.full((3, (Lc + 1) ** 2), 0.05)
        expect = 1.5 * math.log(0.05 * (Lc + 1) ** 2 / (4 * math.pi))
        for d in _rand_dirs(5):
            assert oracle.half_logdet_color(Lc, var, d) == pytest.approx(expect, rel=1e-13, abs=1e-13)
    assert oracle.half_logdet_color(3, np.full((3, 16), 0.05), (0.0, 0.0, 1.0)) == pytest.approx(-4.1312517, abs=1e-7)


def test_color_covariance_direction_dependence():
    """Variances on Y_00 (4 pi 0.01 c_k) and Y_10 (4 pi 0.02 c_k) only, channel
    factors c = (1, 2, 3): Y_00^2 = 1/(4 pi) and Y_10^2 = 3 z^2/(4 pi), so
    Q_k = c_k (0.01 + 0.06 z^2): 1/2 log|Q_c| = -3.0930103 along +-z and
    -6.0118755 in the xy-plane."""
    var = np.zeros((3, 4))
    for k, c in enumerate((1.0, 2.0, 3.0)):
        var[k, 0] = 4 * math.pi * 0.01 * c
        var[k, 2] = 4 * math.pi * 0.02 * c
    for d in ((0, 0, 1), (0, 0, -2)):
        assert oracle.half_logdet_color(1, var, d) == pytest.approx(-3.0930103, abs=1e-7)
    for d in ((1, 0, 0), (0.3, -0.7, 0)):
        assert oracle.half_logdet_color(1, var, d) == pytest.approx(-6.0118755, abs=1e-7)


def test_color_query_with_constant_variance_equals_constant_qc():
    """Only Y_00 carries variance, 4 pi sigma_c^2 in every channel: Q_c = sigma_c^2 I
    in every direction, so the query equals the constant-Q_c query."""
    from paper_2605_30342_amd import scenes
    w = scenes.workload("tiny", scale=0.25)
    b = oracle.vf_build(w.scene, w.train, 2)
    sig = 0.3
    var = np.zeros((3, 4, w.scene.n))
    var[:, 0, :] = 4 * math.pi * sig * sig
    ref = oracle.vf_query(w.scene, b["gamma"], 2, w.train.n, w.cand, Params(sigma_c=sig))
    got = oracle.vf_query_color(w.scene, b["gamma"], 2, w.train.n, var, 1, w.cand)
    np.testing.assert_allclose(got["maps_flat"], ref["maps_flat"], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(got["scores"], ref["scores"], rtol=1e-12)


def test_color_query_single_pixel_closed_form():
    """1x1 image looking along +z at one Gaussian (V = 1 from gamma_00, T = 1):
    H = -x log x + x c_c with x = alpha* = alpha, c_c = 1/2 log|Q_c(+z)| +
    1.5 log(2 pi e), Q_c from the direction-dependent variances above."""
    sc = stack_scene([2.0], [0.6], scale=0.01)
    cam = axis_camera(1, 1, 50.0)
    g = np.zeros((1, 9))
    g[0, 0] = 1.0 / (0.5 / math.sqrt(math.pi))
    var = np.zeros((3, 4, 1))
    for k, c in enumerate((1.0, 2.0, 3.0)):
        var[k, 0, 0] = 4 * math.pi * 0.01 * c
        var[k, 2, 0] = 4 * math.pi * 0.02 * c
    out = oracle.vf_query_color(sc, g, 2, 1, var, 1, cam)
    x = float(np.float32(0.6))
    closed = -x * math.log(x) + x * (-3.0930103207851394 + 1.5 * math.log(2 * math.pi * math.e))
    assert out["maps"][0][0, 0] == pytest.approx(closed, rel=1e-12)


# ---------------------------------------------------------------- expected depth (eq. id's d_p^mn)

def test_expected_depth_closed_forms():
    """Two Gaussians on a 1x1 image's pixel centre at z = 2 (o = 0.6) and z = 3
    (o = 0.5).  With V = 1 (gamma_00 only, |P| = 1): alpha* = alpha, weights
    0.6 and 0.5 (1 - 0.6) = 0.2, D = (0.6*2 + 0.2*3) / 0.8 = 2.25.  With no
    training view (V = 0): alpha* = alpha/2 + 0.075, weights 0.375 and
    0.325 * 0.625 = 0.203125, D = 2.3513514.  One Gaussian alone: D = z."""
    cam = axis_camera(1, 1, 50.0)
    sc = stack_scene([2.0, 3.0], [0.6, 0.5], scale=0.01)
    g = np.zeros((2, 9))
    g[:, 0] = 1.0 / (0.5 / math.sqrt(math.pi))
    out = oracle.vf_query(sc, g, 2, 1, cam, want_depth=True)
    assert out["depth_flat"][0] == pytest.approx(2.25, abs=1e-7)
    out = oracle.vf_query(sc, g, 2, 0, cam, want_depth=True)
    assert out["depth_flat"][0] == pytest.approx(2.3513514, abs=1e-7)
    one = stack_scene([4.5], [0.3], scale=0.01)
    out = oracle.vf_query(one, g[:1], 2, 1, cam, want_depth=True)
    assert out["depth_flat"][0] == pytest.approx(4.5, rel=1e-15)
    # the entropy maps are those of the plain query
    assert oracle.vf_query(sc, g, 2, 1, cam, want_depth=True)["maps_flat"][0] == \
        oracle.vf_query(sc, g, 2, 1, cam)["maps_flat"][0]


def test_expected_depth_empty_pixels_and_range():
    """Pixels no Gaussian reaches get D = 0; elsewhere D lies between the
    nearest and farthest depth in view (a convex combination)."""
    from paper_2605_30342_amd import scenes
    w = scenes.workload("tiny", scale=0.25)
    b = oracle.vf_build(w.scene, w.train, 2)
    out = oracle.vf_query(w.scene, b["gamma"], 2, w.train.n, w.cand, want_depth=True)
    D = out["depth_flat"]
    H = out["maps_flat"]
    assert np.all(D[H == 0.0] == 0.0)
    zmin, zmax = np.inf, 0.0
    for i in range(w.cand.n):
        pr = oracle.project_view(w.scene, w.cand, i)
        ok = pr["ok"] > 0
        zmin, zmax = min(zmin, pr["z"][ok].min()), max(zmax, pr["z"][ok].max())
    live = D > 0
    assert live.mean() > 0.3 and D[live].min() >= zmin * (1 - 1e-12) and D[live].max() <= zmax * (1 + 1e-12)


# ---------------------------------------------------------------- depth keys and near-tie flags

def test_depth_order_is_decided_on_float32_keys():
    """Reading of "sorted by increasing z" (Alg. 2 / Alg. 6): the order is
    decided on z rounded to FP32 (the precision of the sort keys), equal keys
    in index order.  Two Gaussians centred on a 1x1 image's pixel (alpha = o)
    whose FP64 depths differ, z0 = 2 + 3 2^-25 > z1 = 2 - 2^-25, but round to
    the same FP32 key 2: index 0 composites first, so v0 = 1 and v1 = 1 - o0,
    although FP64 order would give v1 = 1, v0 = 1 - o1.  Moving Gaussian 0 one
    FP32 key further (z0 = 2 + 2^-22 + 3 2^-25) restores depth order.  Neither
    depth lies near an FP32 rounding midpoint, so no pixel is flagged."""
    from paper_2605_30342_amd.scenes import Scene
    tz = np.float32(3.0 * 2.0 ** -25)
    cam = axis_camera(1, 1, 50.0, center=(0.0, 0.0, -float(tz)))
    assert cam.t[0, 2] == tz
    o = [0.5, 0.25]
    for m0, first in ((2.0, 0), (2.0 + 2.0 ** -22, 1)):
        means = np.array([[0.0, 0.0, m0], [0.0, 0.0, 2.0 - 2.0 ** -23]], np.float32)
        assert float(means[0, 2]) == m0 and float(means[1, 2]) == 2.0 - 2.0 ** -23
        z = means[:, 2].astype(np.float64) + float(tz)
        assert z[0] > z[1]
        assert (np.float32(z[0]) == np.float32(z[1])) == (first == 0)
        sc = Scene(means, np.full((2, 3), 0.01, np.float32), np.tile(np.array([1, 0, 0, 0], np.float32), (2, 1)),
                   np.array(o, np.float32))
        v, c, _, px = oracle.single_view(sc, cam, 0, want_pixels=True)
        second = 1 - first
        assert v[first] == 1.0 and v[second] == pytest.approx(1.0 - o[first], rel=1e-15)
        assert not px["flags"].any()
        q = oracle.vf_query(sc, np.zeros((2, 9)), 2, 0, cam)
        assert not q["flags_flat"].any()


def test_termination_near_eps_flags_the_pixel():
    """A stack of 15 Gaussians centred on a 1x1 image's pixel with equal
    opacity o: T after the 14th is (1 - o)^14.  With o chosen so that this
    lies within 1e-5 (relative) of eps_T, a float evaluation may stop before
    the 15th or not, so the oracle flags the pixel and gives the 15th an
    allowance; with (1 - o)^14 a few percent away from eps_T it does not."""
    eps = float(np.float32(1e-4))
    prm = Params(eps_T=eps)
    o_exact = 1.0 - eps ** (1.0 / 14.0)
    cands = np.float32(o_exact) + np.arange(-40, 41).astype(np.float32) * np.spacing(np.float32(o_exact))
    rel = np.abs((1.0 - cands.astype(np.float64)) ** 14 / eps - 1.0)
    o_near = cands[np.argmin(rel)]
    assert rel.min() < 1e-5
    zs = np.arange(1.0, 16.0)
    cam = axis_camera(1, 1, 50.0)
    for o, flagged in ((o_near, True), (np.float32(0.47), False), (np.float32(0.49), False)):
        sc = stack_scene(zs, [float(o)] * 15, scale=0.01)
        v, c, pert, px = oracle.single_view(sc, cam, 0, prm, want_pixels=True)
        assert bool(px["flags"][0, 0]) == flagged, o
        assert (pert[14] > 0) == flagged


def _boundary_scene(x):
    from paper_2605_30342_amd.scenes import Scene
    return Scene(np.array([[x, 0.0, 1.0]], np.float32), np.full((1, 3), 0.2, np.float32),
                 np.array([[1, 0, 0, 0]], np.float32), np.array([0.6], np.float32))


def test_overlap_boundary_flags_the_pixel():
    """One isotropic Gaussian whose 3-sigma ellipse (m = 9, C2) passes within
    1e-5 of the centre of pixel (0, 4) of a 9x9 image: the overlap decision
    there is a near tie, so the pixel is flagged in Alg. 2 and Alg. 6 and the
    Gaussian gets an allowance; moved by 5e-3 (m about 0.1 away) nothing is
    flagged."""
    cam = axis_camera(9, 9, 10.0)
    prm = Params()

    def m_at(x):
        p = oracle.project_view(_boundary_scene(x), cam, 0, prm)
        dx, dy = 0.5 - p["ux"][0], 4.5 - p["uy"][0]
        return p["ca"][0] * dx * dx + 2 * p["cb"][0] * dx * dy + p["cc"][0] * dy * dy
    lo, hi = 0.15, 0.35                  # m(lo) < 9 < m(hi): the ellipse's edge moves off the pixel
    assert m_at(lo) < 9.0 < m_at(hi)
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if m_at(mid) < 9.0 else (lo, mid)
    x0 = 0.5 * (lo + hi)
    xs = np.float32(x0) + np.arange(-20, 21).astype(np.float32) * np.spacing(np.float32(x0))
    ms = np.array([m_at(float(x)) for x in xs])
    x_near = float(xs[np.argmin(np.abs(ms - 9.0))])
    assert abs(m_at(x_near) - 9.0) < 1e-5
    for x, flagged in ((x_near, True), (x_near - 5e-3, False), (x_near + 5e-3, False)):
        sc = _boundary_scene(x)
        v, c, pert, px = oracle.single_view(sc, cam, 0, prm, want_pixels=True)
        assert bool(px["flags"][4, 0]) == flagged and int(px["flags"].sum()) == int(flagged)
        assert (pert[0] > 0) == flagged
        q = oracle.vf_query(sc, np.zeros((1, 9)), 2, 0, cam, prm)
        assert bool(q["flags"][0][4, 0]) == flagged and int(q["flags_flat"].sum()) == int(flagged)
