"""Hyperelastic energy densities, first Piola stresses and the stiffness rule.

Oracle module (test infrastructure only; never used by the product path).

Paper passages followed:
* Section 4.1, Eq. valanis-landel: an isotropic energy written in the
  principal stretches s1, s2, s3 as
      Psi = sum_i a(s_i) + sum_{i<j} b(s_i s_j) + c(s1 s2 s3).
* Section 4.1, Eq. stiffness: the stress profile
      f(s) = a'(s) + 2 b'(s) + c'(s)
  (dPsi/ds1 with s2 = s3 = 1); the element stiffness k is the slope of the
  best linear approximation of f on [x_start, x_end] = [0.5, 1.5]
  (section 5, "Choice of stiffness parameters").
* Section 5: Neo-Hookean, St. Venant-Kirchhoff, corotated and spline-based
  materials; the polynomial material a(x) = mu (x - 1)^4, b = c = 0 of the
  squirrel-head example (section 4, figure caption; section 4.1).
* Section 4.1 names Mooney-Rivlin among the materials with a Valanis-Landel
  form (no formula or parameters are given).

Readings where the paper is silent:
* Material formulas (not written in the paper) are the standard ones:
    Neo-Hookean   Psi = mu/2 (I1 - 3) - mu log J + lam/2 (log J)^2, +inf for J <= 0
    StVK          Psi = mu tr(E^2) + lam/2 tr(E)^2,  E = (F^T F - I)/2
    corotated     Psi = mu |F - R|^2 + lam/2 tr(R^T F - I)^2
    Mooney-Rivlin Psi = mu/2 (I1 - 3) + mu2/2 (I2 - 3) - (mu + 2 mu2) log J
                        + lam/2 (log J)^2,  I2 = ((tr C)^2 - tr C^2)/2, C = F^T F,
                  +inf for J <= 0 (compressible form; the log J coefficient
                  makes the rest state stress-free; mu2 = 0 is Neo-Hookean)
  Their Valanis-Landel forms (derived by expanding in the stretches):
    Neo-Hookean   a(x) = mu/2 (x^2 - 1),                         b = 0,
                  c(J) = -mu log J + lam/2 (log J)^2
    StVK          a(x) = (mu/4 + lam/8)(x^2 - 1)^2 - lam/2 (x^2 - 1),
                  b(y) = lam/4 (y^2 - 1),                         c = 0
    corotated     a(x) = (mu + lam/2)(x - 1)^2 - 2 lam (x - 1),
                  b(y) = lam (y - 1),                             c = 0
    Mooney-Rivlin a(x) = mu/2 (x^2 - 1),  b(y) = mu2/2 (y^2 - 1),
                  c(J) = -(mu + 2 mu2) log J + lam/2 (log J)^2
* Spline material (the paper's spline curves are not given): a'' is the
  piecewise-linear interpolant of 8 values d2_j at knots 0.2 + 0.4 j
  (j = 0..7), constant beyond the end knots; a'(1) = a(1) = 0, so a is a
  convex C2 cubic spline. b = 0, c(J) = lam/2 (J - 1)^2.
* "Best linear approximation" = continuous least squares with a free
  intercept: k = 12 / L^3 * integral_{lo}^{hi} (s - mid) f(s) ds with
  L = hi - lo, mid = (lo + hi)/2, evaluated by composite Gauss-Legendre
  quadrature split at the spline knots.
* Signed SVD: F = U diag(s) V^T with det U = det V = +1; if numpy's SVD gives a
  reflection, the last column is flipped and s3 negated (Irving et al. 2004).
"""
from __future__ import annotations

import numpy as np

NEOHOOKEAN, STVK, SPLINE, COROTATED, POLYNOMIAL, MOONEY_RIVLIN = 0, 1, 2, 3, 4, 5

SPLINE_KNOTS = 0.2 + 0.4 * np.arange(8, dtype=np.float64)


# ---------------------------------------------------------------------------
# Signed SVD (section 4.1: energies in terms of principal stretches)
# ---------------------------------------------------------------------------
def signed_svd(F: np.ndarray):
    """F (..., 3, 3) = U diag(s) V^T with rotations U, V; s3 carries det F's sign."""
    U, s, Vt = np.linalg.svd(F)
    V = np.swapaxes(Vt, -1, -2).copy()
    U = U.copy()
    s = s.copy()
    detU = np.linalg.det(U)
    detV = np.linalg.det(V)
    fixU = detU < 0
    fixV = detV < 0
    U[fixU, :, 2] *= -1.0
    s[fixU, 2] *= -1.0
    V[fixV, :, 2] *= -1.0
    s[fixV, 2] *= -1.0
    return U, s, V


# ---------------------------------------------------------------------------
# Spline stretch term a(s) (reading of the spline-based material)
# ---------------------------------------------------------------------------
class StretchSpline:
    """a(s) with a'' piecewise linear through (knot_j, d2_j), a'(1) = a(1) = 0."""

    def __init__(self, d2):
        self.knots = SPLINE_KNOTS
        self.d2 = np.asarray(d2, dtype=np.float64)
        # Values of a' and a at every knot by exact integration of the
        # piecewise-linear a'', starting from s = 1 where both vanish.
        k = self.knots
        n = len(k)
        a1 = np.zeros(n)
        a0 = np.zeros(n)
        ref = int(np.argmin(np.abs(k - 1.0)))
        assert abs(k[ref] - 1.0) < 1e-15
        for j in range(ref, n - 1):          # integrate upwards
            dx = k[j + 1] - k[j]
            s0, s1 = self.d2[j], self.d2[j + 1]
            a1[j + 1] = a1[j] + dx * (s0 + s1) / 2.0
            a0[j + 1] = a0[j] + a1[j] * dx + dx * dx * (2.0 * s0 + s1) / 6.0
        for j in range(ref, 0, -1):          # integrate downwards
            dx = k[j] - k[j - 1]
            s0, s1 = self.d2[j - 1], self.d2[j]
            a1[j - 1] = a1[j] - dx * (s0 + s1) / 2.0
            # a(k[j-1]) = a(k[j]) - a'(k[j]) dx + dx^2 (s0 + 2 s1)/6 ... derived
            # from Taylor expansion about k[j] with a''' = (s1 - s0)/dx.
            a0[j - 1] = a0[j] - a1[j] * dx + dx * dx * (s0 + 2.0 * s1) / 6.0
        self.a1_knot = a1
        self.a0_knot = a0

    def _segment(self, s):
        k = self.knots
        j = np.clip(np.searchsorted(k, s, side="right") - 1, 0, len(k) - 2)
        return j

    def d2_at(self, s):
        s = np.asarray(s, dtype=np.float64)
        k, d2 = self.knots, self.d2
        j = self._segment(s)
        t = (s - k[j]) / (k[j + 1] - k[j])
        val = d2[j] + (d2[j + 1] - d2[j]) * t
        val = np.where(s < k[0], d2[0], val)
        val = np.where(s > k[-1], d2[-1], val)
        return val

    def eval(self, s):
        """Return (a(s), a'(s)) for an array of stretches (any sign)."""
        s = np.asarray(s, dtype=np.float64)
        k, d2, a0k, a1k = self.knots, self.d2, self.a0_knot, self.a1_knot
        j = self._segment(s)
        x = s - k[j]
        dx = k[j + 1] - k[j]
        slope = (d2[j + 1] - d2[j]) / dx
        a1 = a1k[j] + d2[j] * x + slope * x * x / 2.0
        a0 = a0k[j] + a1k[j] * x + d2[j] * x * x / 2.0 + slope * x ** 3 / 6.0
        lo = s < k[0]
        xl = s - k[0]
        a1 = np.where(lo, a1k[0] + d2[0] * xl, a1)
        a0 = np.where(lo, a0k[0] + a1k[0] * xl + d2[0] * xl * xl / 2.0, a0)
        hi = s > k[-1]
        xh = s - k[-1]
        a1 = np.where(hi, a1k[-1] + d2[-1] * xh, a1)
        a0 = np.where(hi, a0k[-1] + a1k[-1] * xh + d2[-1] * xh * xh / 2.0, a0)
        return a0, a1


# ---------------------------------------------------------------------------
# Valanis-Landel terms a, b, c and their derivatives (Eq. valanis-landel)
# ---------------------------------------------------------------------------
def vl_terms(kind: int, mu, lam, d2=None):
    """Return functions (a, da, b, db, c, dc) of the Valanis-Landel form.

    d2: the knot values a'' (SPLINE) or the second shear modulus mu2
    (MOONEY_RIVLIN); unused otherwise."""
    mu = np.asarray(mu, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    zero = lambda x: np.zeros_like(np.asarray(x, dtype=np.float64))  # noqa: E731
    if kind == NEOHOOKEAN:
        def c(J):
            with np.errstate(divide="ignore", invalid="ignore"):
                lj = np.log(J)
                return np.where(J > 0, -mu * lj + 0.5 * lam * lj * lj, np.inf)

        def dc(J):
            with np.errstate(divide="ignore", invalid="ignore"):
                return np.where(J > 0, (-mu + lam * np.log(J)) / J, np.nan)
        return (lambda x: 0.5 * mu * (x * x - 1.0), lambda x: mu * x,
                zero, zero, c, dc)
    if kind == STVK:
        A = mu / 4.0 + lam / 8.0
        return (lambda x: A * (x * x - 1.0) ** 2 - 0.5 * lam * (x * x - 1.0),
                lambda x: 4.0 * A * x * (x * x - 1.0) - lam * x,
                lambda y: 0.25 * lam * (y * y - 1.0),
                lambda y: 0.5 * lam * y,
                zero, zero)
    if kind == COROTATED:
        return (lambda x: (mu + 0.5 * lam) * (x - 1.0) ** 2 - 2.0 * lam * (x - 1.0),
                lambda x: (2.0 * mu + lam) * (x - 1.0) - 2.0 * lam,
                lambda y: lam * (y - 1.0),
                lambda y: lam + 0.0 * y,
                zero, zero)
    if kind == POLYNOMIAL:
        return (lambda x: mu * (x - 1.0) ** 4, lambda x: 4.0 * mu * (x - 1.0) ** 3,
                zero, zero, zero, zero)
    if kind == MOONEY_RIVLIN:
        mu2 = np.asarray(d2, dtype=np.float64)
        mue = mu + 2.0 * mu2

        def c(J):
            with np.errstate(divide="ignore", invalid="ignore"):
                lj = np.log(J)
                return np.where(J > 0, -mue * lj + 0.5 * lam * lj * lj, np.inf)

        def dc(J):
            with np.errstate(divide="ignore", invalid="ignore"):
                return np.where(J > 0, (-mue + lam * np.log(J)) / J, np.nan)
        return (lambda x: 0.5 * mu * (x * x - 1.0), lambda x: mu * x,
                lambda y: 0.5 * mu2 * (y * y - 1.0), lambda y: mu2 * y, c, dc)
    if kind == SPLINE:
        sp = StretchSpline(d2)
        return (lambda x: sp.eval(x)[0], lambda x: sp.eval(x)[1],
                zero, zero,
                lambda J: 0.5 * lam * (J - 1.0) ** 2,
                lambda J: lam * (J - 1.0))
    raise ValueError(f"unknown material type {kind}")


def psi_P_valanis_landel(kind: int, F: np.ndarray, mu, lam, d2=None):
    """Psi(F) and P(F) from the Valanis-Landel form through the signed SVD.

    dPsi/ds_i = a'(s_i) + sum_{j != i} b'(s_i s_j) s_j + c'(J) prod_{j != i} s_j
    and P = U diag(dPsi/ds) V^T (isotropic energies, section 4.1).
    """
    a, da, b, db, c, dc = vl_terms(kind, mu, lam, d2)
    U, s, V = signed_svd(F)
    s1, s2, s3 = s[..., 0], s[..., 1], s[..., 2]
    J = s1 * s2 * s3
    psi = (a(s1) + a(s2) + a(s3) + b(s1 * s2) + b(s2 * s3) + b(s1 * s3) + c(J))
    g1 = da(s1) + db(s1 * s2) * s2 + db(s1 * s3) * s3 + dc(J) * s2 * s3
    g2 = da(s2) + db(s1 * s2) * s1 + db(s2 * s3) * s3 + dc(J) * s1 * s3
    g3 = da(s3) + db(s1 * s3) * s1 + db(s2 * s3) * s2 + dc(J) * s1 * s2
    g = np.stack([g1, g2, g3], axis=-1)
    P = np.einsum("...ij,...j,...kj->...ik", U, g, V)
    return psi, P


# ---------------------------------------------------------------------------
# Anisotropic fibre term (section 4, "Anisotropy"): added to a base material,
#   Psi_f = kappa/2 (|F d| - 1)^2,  d the unit rest-pose fibre direction,
#   P_f = dPsi_f/dF = kappa (|F d| - 1) / |F d| * (F d) d^T.
# ---------------------------------------------------------------------------
def psi_P_fiber(F: np.ndarray, kappa, d):
    kappa = np.asarray(kappa, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    f = np.einsum("...ij,...j->...i", F, d)
    ln = np.sqrt(np.einsum("...i,...i->...", f, f))
    e = ln - 1.0
    psi = 0.5 * kappa * e * e
    P = (kappa * e / ln)[..., None, None] * np.einsum("...i,...j->...ij", f, d)
    return psi, P


# ---------------------------------------------------------------------------
# Invariant forms (standard definitions; no SVD)
# ---------------------------------------------------------------------------
def psi_P_neohookean(F, mu, lam):
    mu = np.asarray(mu, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    J = np.linalg.det(F)
    ok = J > 0
    Fs = np.where(ok[..., None, None], F, np.eye(3))
    Finv_T = np.swapaxes(np.linalg.inv(Fs), -1, -2)
    I1 = np.einsum("...ij,...ij->...", F, F)
    with np.errstate(divide="ignore", invalid="ignore"):
        logJ = np.log(np.where(ok, J, 1.0))
    psi = 0.5 * mu * (I1 - 3.0) - mu * logJ + 0.5 * lam * logJ * logJ
    psi = np.where(ok, psi, np.inf)
    P = mu[..., None, None] * (F - Finv_T) + (lam * logJ)[..., None, None] * Finv_T
    P = np.where(ok[..., None, None], P, np.nan)
    return psi, P


def psi_P_mooney_rivlin(F, mu, lam, mu2):
    """Invariant form: P = mu F + mu2 (I1 F - F C) + (lam log J - mu - 2 mu2) F^{-T}."""
    mu = np.asarray(mu, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    mu2 = np.asarray(mu2, dtype=np.float64)
    J = np.linalg.det(F)
    ok = J > 0
    Fs = np.where(ok[..., None, None], F, np.eye(3))
    Finv_T = np.swapaxes(np.linalg.inv(Fs), -1, -2)
    C = np.einsum("...ki,...kj->...ij", F, F)
    I1 = np.trace(C, axis1=-2, axis2=-1)
    I2 = 0.5 * (I1 * I1 - np.einsum("...ij,...ji->...", C, C))
    with np.errstate(divide="ignore", invalid="ignore"):
        logJ = np.log(np.where(ok, J, 1.0))
    mue = mu + 2.0 * mu2
    psi = 0.5 * mu * (I1 - 3.0) + 0.5 * mu2 * (I2 - 3.0) - mue * logJ + 0.5 * lam * logJ * logJ
    psi = np.where(ok, psi, np.inf)
    P = (mu[..., None, None] * F + mu2[..., None, None] * (I1[..., None, None] * F - F @ C)
         + (lam * logJ - mue)[..., None, None] * Finv_T)
    P = np.where(ok[..., None, None], P, np.nan)
    return psi, P


def psi_P_stvk(F, mu, lam):
    mu = np.asarray(mu, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    E = 0.5 * (np.einsum("...ki,...kj->...ij", F, F) - np.eye(3))
    trE = np.trace(E, axis1=-2, axis2=-1)
    psi = mu * np.einsum("...ij,...ij->...", E, E) + 0.5 * lam * trE * trE
    S = 2.0 * mu[..., None, None] * E + (lam * trE)[..., None, None] * np.eye(3)
    P = F @ S
    return psi, P


def psi_P_corotated(F, mu, lam):
    mu = np.asarray(mu, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    U, s, V = signed_svd(F)
    R = U @ np.swapaxes(V, -1, -2)
    D = F - R
    tr = np.einsum("...ki,...ki->...", R, F) - 3.0
    psi = mu * np.einsum("...ij,...ij->...", D, D) + 0.5 * lam * tr * tr
    P = 2.0 * mu[..., None, None] * D + (lam * tr)[..., None, None] * R
    return psi, P


def psi_and_P(kind: int, F: np.ndarray, mu, lam, d2=None):
    """Energy density Psi(F) (per unit rest volume) and first Piola stress P."""
    if kind == NEOHOOKEAN:
        return psi_P_neohookean(F, mu, lam)
    if kind == STVK:
        return psi_P_stvk(F, mu, lam)
    if kind == COROTATED:
        return psi_P_corotated(F, mu, lam)
    if kind == MOONEY_RIVLIN:
        return psi_P_mooney_rivlin(F, mu, lam, d2)
    if kind in (SPLINE, POLYNOMIAL):
        return psi_P_valanis_landel(kind, F, mu, lam, d2)
    raise ValueError(f"unknown material type {kind}")


# ---------------------------------------------------------------------------
# Stiffness rule (section 4.1, Eq. stiffness; section 5 interval [0.5, 1.5])
# ---------------------------------------------------------------------------
def stress_profile(kind: int, mu, lam, d2=None):
    """f(s) = a'(s) + 2 b'(s) + c'(s): dPsi/ds1 with s2 = s3 = 1."""
    a, da, b, db, c, dc = vl_terms(kind, mu, lam, d2)
    return lambda s: da(s) + 2.0 * db(s) + dc(s)


def stiffness(kind: int, mu: float, lam: float, d2=None, lo: float = 0.5,
              hi: float = 1.5, points: int = 64) -> float:
    """Least-squares slope of f(s) over [lo, hi] (continuous L2, free intercept)."""
    f = stress_profile(kind, mu, lam, d2)
    cuts = [lo]
    if kind == SPLINE:
        cuts += [kk for kk in SPLINE_KNOTS if lo < kk < hi]
    cuts.append(hi)
    xg, wg = np.polynomial.legendre.leggauss(points)
    mid = 0.5 * (lo + hi)
    L = hi - lo
    total = 0.0
    for x0, x1 in zip(cuts[:-1], cuts[1:]):
        s = 0.5 * (x1 - x0) * xg + 0.5 * (x1 + x0)
        total += 0.5 * (x1 - x0) * float(np.sum(wg * (s - mid) * f(s)))
    return 12.0 * total / L ** 3
