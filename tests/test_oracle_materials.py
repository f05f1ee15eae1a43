"""Pins of the oracle's materials, signed SVD and stiffness rule (CPU only).

Each test checks the oracle against something other than itself: calculus
(finite differences), invariances the energies must have, two independent
formulas of one energy, closed-form integrals of the stiffness rule, or a
textbook routine (numpy's polynomial least squares).
"""
import math

import numpy as np
import pytest

from oracle import materials as mat

KINDS = [mat.NEOHOOKEAN, mat.STVK, mat.SPLINE, mat.COROTATED, mat.POLYNOMIAL,
         mat.MOONEY_RIVLIN]
MU, LAM = 35714.28571428572, 142857.1428571429
MU2 = 0.4 * MU  # Mooney-Rivlin: shear modulus of the I2 term


def _d2(seed=0):
    rng = np.random.default_rng(seed)
    return MU * rng.uniform(0.5, 2.0, size=8)


def _extra(kind, seed=0):
    """The parameter beyond mu and lam: spline knot values, or mu2."""
    return MU2 if kind == mat.MOONEY_RIVLIN else _d2(seed)


def _random_F(n, seed, amp=0.3):
    rng = np.random.default_rng(seed)
    F = np.eye(3) + amp * rng.uniform(-1, 1, size=(n, 3, 3))
    F = F[np.linalg.det(F) > 0.2]
    return F


def _rot(seed):
    rng = np.random.default_rng(seed)
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    return q


@pytest.mark.parametrize("kind", KINDS)
def test_stress_is_energy_derivative(kind):
    """P = dPsi/dF by central differences (rel. err < 1e-7)."""
    F = _random_F(40, kind)
    d2 = _extra(kind)
    psi, P = mat.psi_and_P(kind, F, MU, LAM, d2)
    eps = 1e-6
    Pfd = np.zeros_like(P)
    for i in range(3):
        for j in range(3):
            Fp = F.copy(); Fp[:, i, j] += eps
            Fm = F.copy(); Fm[:, i, j] -= eps
            Pfd[:, i, j] = (mat.psi_and_P(kind, Fp, MU, LAM, d2)[0]
                            - mat.psi_and_P(kind, Fm, MU, LAM, d2)[0]) / (2 * eps)
    err = np.abs(Pfd - P).max() / np.abs(P).max()
    assert err < 1e-7, err


@pytest.mark.parametrize("kind", KINDS)
def test_rest_state_is_stress_free(kind):
    psi, P = mat.psi_and_P(kind, np.eye(3)[None], MU, LAM, _extra(kind))
    assert abs(psi[0]) < 1e-12 * MU
    assert np.abs(P).max() < 1e-12 * MU


@pytest.mark.parametrize("kind", KINDS)
def test_rotation_invariance(kind):
    """Psi(QF) = Psi(F), P(QF) = Q P(F) (world frame); Psi(FQ) = Psi(F) (isotropy)."""
    F = _random_F(30, 10 + kind)
    d2 = _extra(kind)
    psi, P = mat.psi_and_P(kind, F, MU, LAM, d2)
    for s in range(3):
        Q = _rot(100 + s)
        psi_l, P_l = mat.psi_and_P(kind, Q @ F, MU, LAM, d2)
        psi_r, _ = mat.psi_and_P(kind, F @ Q, MU, LAM, d2)
        scale = np.abs(psi).max()
        assert np.abs(psi_l - psi).max() < 1e-11 * scale
        assert np.abs(psi_r - psi).max() < 1e-11 * scale
        assert np.abs(P_l - Q @ P).max() < 1e-10 * np.abs(P).max()


@pytest.mark.parametrize("kind", [mat.NEOHOOKEAN, mat.STVK, mat.COROTATED, mat.MOONEY_RIVLIN])
def test_invariant_form_equals_valanis_landel_form(kind):
    """The closed invariant formula and the Valanis-Landel stretch form agree."""
    F = _random_F(50, 20 + kind)
    psi_a, P_a = mat.psi_and_P(kind, F, MU, LAM, MU2)
    psi_b, P_b = mat.psi_P_valanis_landel(kind, F, MU, LAM, MU2)
    assert np.abs(psi_a - psi_b).max() < 1e-10 * np.abs(psi_a).max()
    assert np.abs(P_a - P_b).max() < 1e-10 * np.abs(P_a).max()


def test_neohookean_inverted_is_infinite():
    F = np.diag([1.0, 1.0, -0.5])[None]
    psi, _ = mat.psi_and_P(mat.NEOHOOKEAN, F, MU, LAM)
    assert np.isinf(psi[0])
    psi, _ = mat.psi_and_P(mat.MOONEY_RIVLIN, F, MU, LAM, MU2)
    assert np.isinf(psi[0])


def test_mooney_rivlin_without_i2_term_is_neohookean():
    """mu2 = 0 leaves exactly the Neo-Hookean energy and stress."""
    F = _random_F(40, 31)
    psi_a, P_a = mat.psi_and_P(mat.MOONEY_RIVLIN, F, MU, LAM, 0.0)
    psi_b, P_b = mat.psi_and_P(mat.NEOHOOKEAN, F, MU, LAM)
    assert np.abs(psi_a - psi_b).max() <= 1e-12 * np.abs(psi_b).max()
    assert np.abs(P_a - P_b).max() <= 1e-12 * np.abs(P_b).max()


def test_mooney_rivlin_second_invariant_and_uniaxial_stress():
    """Uniaxial stretch F = diag(s, 1, 1), worked by hand: I1 = s^2 + 2,
    I2 = ((tr C)^2 - tr C^2)/2 = 2 s^2 + 1, J = s, so Psi(s) and its
    derivative P_11 = mu s + 2 mu2 s - (mu + 2 mu2)/s + lam log(s)/s."""
    for sv in (0.6, 0.9, 1.0, 1.3, 1.8):
        F = np.diag([sv, 1.0, 1.0])[None]
        psi, P = mat.psi_and_P(mat.MOONEY_RIVLIN, F, MU, LAM, MU2)
        ls = math.log(sv)
        p11 = MU * sv + 2 * MU2 * sv - (MU + 2 * MU2) / sv + LAM * ls / sv
        e = (0.5 * MU * (sv * sv - 1) + 0.5 * MU2 * (2 * sv * sv - 2)
             - (MU + 2 * MU2) * ls + 0.5 * LAM * ls * ls)
        assert P[0, 0, 0] == pytest.approx(p11, rel=1e-12, abs=1e-9 * MU)
        assert psi[0] == pytest.approx(e, rel=1e-12, abs=1e-9 * MU)


def test_signed_svd():
    rng = np.random.default_rng(3)
    F = rng.normal(size=(200, 3, 3))
    U, s, V = mat.signed_svd(F)
    rec = np.einsum("tij,tj,tkj->tik", U, s, V)
    assert np.abs(rec - F).max() < 1e-12
    assert np.allclose(np.linalg.det(U), 1.0) and np.allclose(np.linalg.det(V), 1.0)
    assert np.all(np.sign(s[:, 2]) == np.sign(np.linalg.det(F)))
    assert np.all(s[:, 0] >= s[:, 1]) and np.all(s[:, 1] >= np.abs(s[:, 2]))


def test_spline_term_is_c2_convex_and_anchored():
    d2 = _d2(5)
    sp = mat.StretchSpline(d2)
    a, da = sp.eval(np.array([1.0]))
    assert abs(a[0]) < 1e-12 * MU and abs(da[0]) < 1e-12 * MU
    # derivatives by central differences, across knots and beyond the ends
    s = np.linspace(-0.5, 3.8, 2001)
    eps = 1e-6
    a_p, da_p = sp.eval(s + eps)
    a_m, da_m = sp.eval(s - eps)
    a0, da0 = sp.eval(s)
    assert np.abs((a_p - a_m) / (2 * eps) - da0).max() < 1e-6 * MU
    assert np.abs((da_p - da_m) / (2 * eps) - sp.d2_at(s)).max() < 1e-5 * MU
    # continuity of a, a', a'' at every knot
    for kn in mat.SPLINE_KNOTS:
        lo, hi = sp.eval(np.array([kn - 1e-12, kn + 1e-12]))[0:2]
        assert abs(lo[0] - lo[1]) < 1e-9 * MU and abs(hi[0] - hi[1]) < 1e-9 * MU
    assert np.all(np.diff(da0) > 0)            # a' monotone (a convex)
    assert np.all(sp.d2_at(s) > 0)


# ---------------------------------------------------------------------------
# Stiffness rule: closed forms of the least-squares slope on [0.5, 1.5]
# ---------------------------------------------------------------------------
def test_stiffness_corotated_exact():
    """f(s) = (2 mu + lam)(s - 1) is linear, so k = 2 mu + lam exactly."""
    assert mat.stiffness(mat.COROTATED, MU, LAM) == pytest.approx(2 * MU + LAM, rel=1e-13)


def test_stiffness_polynomial_closed_form():
    """f(s) = 4 mu (s-1)^3: k = 12 * 4 mu * int_{-1/2}^{1/2} u^4 du = 0.6 mu.

    Also pins the paper's remark that the rest second derivative (0 here)
    would give zero stiffness.
    """
    assert mat.stiffness(mat.POLYNOMIAL, MU, 0.0) == pytest.approx(0.6 * MU, rel=1e-13)
    f = mat.stress_profile(mat.POLYNOMIAL, MU, 0.0)
    eps = 1e-4
    assert abs((f(1 + eps) - f(1 - eps)) / (2 * eps)) < 1e-6 * MU


def test_stiffness_stvk_closed_form():
    """f(s) = (mu + lam/2)(s^3 - s): k = 12 (mu + lam/2) (1/80 + 1/6) = 2.15 (mu + lam/2)."""
    assert mat.stiffness(mat.STVK, MU, LAM) == pytest.approx(2.15 * (MU + LAM / 2), rel=1e-13)


def test_stiffness_neohookean_closed_form():
    """f(s) = mu s + (-mu + lam log s)/s, integrated by hand on [0.5, 1.5]."""
    ln = math.log
    mu_coef = 1.0 + 12.0 * (ln(3.0) - 1.0)
    F = lambda s: s * ln(s) - s - 0.5 * ln(s) ** 2   # antiderivative of (s-1) ln(s)/s
    lam_coef = 12.0 * (F(1.5) - F(0.5))
    k = mat.stiffness(mat.NEOHOOKEAN, MU, LAM)
    assert k == pytest.approx(mu_coef * MU + lam_coef * LAM, rel=1e-13)
    # the value at E = 1e5, nu = 0.4
    assert k == pytest.approx(271342.6, abs=0.1)


def test_stiffness_spline_constant_curvature_reduces_to_linear():
    """Constant a'' = c mu makes a'(s) = c mu (s - 1): k = c mu + lam exactly."""
    d2 = np.full(8, 1.7 * MU)
    assert mat.stiffness(mat.SPLINE, MU, LAM, d2) == pytest.approx(1.7 * MU + LAM, rel=1e-12)


@pytest.mark.parametrize("kind", KINDS)
def test_stiffness_matches_discrete_least_squares(kind):
    """The continuous fit equals numpy's polyfit on a fine midpoint sample.

    Equal-weight samples at cell midpoints make the discrete least-squares sums
    midpoint-rule quadratures of the continuous ones (error O(N^-2)).
    """
    d2 = _extra(kind, 7)
    N = 200000
    s = 0.5 + (np.arange(N) + 0.5) / N
    f = mat.stress_profile(kind, MU, LAM, d2)(s)
    slope = np.polyfit(s, f, 1)[0]
    k = mat.stiffness(kind, MU, LAM, d2)
    assert k == pytest.approx(slope, rel=1e-8)


def test_stiffness_mooney_rivlin_is_neohookean_with_summed_shear():
    """f(s) = (mu + 2 mu2)(s - 1/s) + lam log(s)/s is the Neo-Hookean profile
    with shear modulus mu + 2 mu2, so k follows the same closed form."""
    ln = math.log
    mu_coef = 1.0 + 12.0 * (ln(3.0) - 1.0)
    F = lambda s: s * ln(s) - s - 0.5 * ln(s) ** 2
    lam_coef = 12.0 * (F(1.5) - F(0.5))
    k = mat.stiffness(mat.MOONEY_RIVLIN, MU, LAM, MU2)
    assert k == pytest.approx(mu_coef * (MU + 2 * MU2) + lam_coef * LAM, rel=1e-13)


def test_stiffness_positive_for_workload_materials():
    import workloads as W
    for kind in (W.NEOHOOKEAN, W.STVK, W.SPLINE, W.MOONEY_RIVLIN):
        m = W.make_material(kind, 1e5, 0.4)
        extra = m.mu2 if kind == W.MOONEY_RIVLIN else m.d2()
        assert mat.stiffness(m.type, m.mu, m.lam, extra) > 0


# ---------------------------------------------------------------------------
# Anisotropic fibre term (section 4, "Anisotropy"): kappa/2 (|F d| - 1)^2
# ---------------------------------------------------------------------------
KAPPA = 5.0 * MU
FDIR = np.array([1.0, 2.0, -0.5]) / np.linalg.norm([1.0, 2.0, -0.5])


def test_fiber_stress_is_energy_derivative():
    F = _random_F(40, 11)
    psi, P = mat.psi_P_fiber(F, KAPPA, FDIR)
    eps = 1e-6
    Pfd = np.zeros_like(P)
    for i in range(3):
        for j in range(3):
            Fp = F.copy(); Fp[:, i, j] += eps
            Fm = F.copy(); Fm[:, i, j] -= eps
            Pfd[:, i, j] = (mat.psi_P_fiber(Fp, KAPPA, FDIR)[0] - mat.psi_P_fiber(Fm, KAPPA, FDIR)[0]) / (2 * eps)
    assert np.abs(Pfd - P).max() / np.abs(P).max() < 1e-7


@pytest.mark.parametrize("lam_s", [0.6, 1.0, 1.7])
def test_fiber_uniaxial_closed_forms(lam_s):
    """Stretch lam along d: Psi = kappa/2 (lam - 1)^2, P = kappa (lam - 1) d d^T;
    stretch across d: no fibre energy or stress."""
    along = np.eye(3) + (lam_s - 1.0) * np.outer(FDIR, FDIR)
    psi, P = mat.psi_P_fiber(along[None], KAPPA, FDIR)
    assert psi[0] == pytest.approx(0.5 * KAPPA * (lam_s - 1.0) ** 2, rel=1e-13, abs=1e-9)
    assert np.abs(P[0] - KAPPA * (lam_s - 1.0) * np.outer(FDIR, FDIR)).max() < 1e-9 * KAPPA
    e = np.cross(FDIR, [0.0, 0.0, 1.0]); e /= np.linalg.norm(e)
    across = np.eye(3) + (lam_s - 1.0) * np.outer(e, e)
    psi, P = mat.psi_P_fiber(across[None], KAPPA, FDIR)
    assert abs(psi[0]) < 1e-20 * KAPPA and np.abs(P[0]).max() < 1e-12 * KAPPA


def test_fiber_invariances():
    """Frame invariance; invariance under rest rotations about the fibre axis
    only (the term is transversely isotropic, not isotropic)."""
    F = _random_F(20, 12)
    psi, P = mat.psi_P_fiber(F, KAPPA, FDIR)
    Q = _rot(3)
    psi_q, P_q = mat.psi_P_fiber(Q @ F, KAPPA, FDIR)
    assert np.abs(psi_q - psi).max() < 1e-12 * np.abs(psi).max()
    assert np.abs(P_q - Q @ P).max() < 1e-12 * np.abs(P).max()
    th = 0.7  # rotation about d (Rodrigues)
    K = np.array([[0, -FDIR[2], FDIR[1]], [FDIR[2], 0, -FDIR[0]], [-FDIR[1], FDIR[0], 0]])
    Rd = np.eye(3) + np.sin(th) * K + (1 - np.cos(th)) * K @ K
    assert np.abs(mat.psi_P_fiber(F @ Rd, KAPPA, FDIR)[0] - psi).max() < 1e-12 * np.abs(psi).max()
    assert np.abs(mat.psi_P_fiber(F @ _rot(4), KAPPA, FDIR)[0] - psi).max() > 1e-3 * np.abs(psi).max()
