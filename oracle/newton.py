"""Projected Newton's method, iterated to convergence, for tiny meshes.

Oracle module (test infrastructure only; never used by the product path).

Section 5 compares against Newton's method with the per-element
definiteness fix (each element Hessian projected onto its positive
semi-definite part) and defines the relative error of an iterate as
    (g(x_k) - g(x*)) / (g(x_0) - g(x*)),   x_0 := y   (Eq. RelativeError),
where x* is Newton's method iterated until convergence. This module supplies
x* for the pins on small meshes. Element Hessians are central finite
differences of the analytic element gradients (12 x 12 per tetrahedron),
symmetrised and projected; the global system couples x, y and z (3n x 3n).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse
import scipy.sparse.linalg

from . import fem
from . import materials as mat


def _element_gradients_at(model, Fx):
    """Element gradient vectors (T, 12) at per-element vertex positions (T, 4, 3)."""
    P_ = Fx
    Ds = np.stack([P_[:, 1] - P_[:, 0], P_[:, 2] - P_[:, 0], P_[:, 3] - P_[:, 0]], axis=2)
    F = Ds @ model.Dm_inv
    T = F.shape[0]
    Pst = np.empty((T, 3, 3))
    for kind, ids, mu, lam, d2 in model.mat_groups:
        if mu is None:
            mu, lam = model.mu_t[ids], model.lam_t[ids]
        _, P = mat.psi_and_P(kind, F[ids], mu, lam, d2)
        Pst[ids] = P
    return fem.element_forces(model, Pst).reshape(T, 12)


def element_hessians(model, x, eps_rel=1e-6, project=True):
    X = x[model.tets]                               # (T, 4, 3)
    T = X.shape[0]
    scale = np.cbrt(model.vol * 6.0)[:, None, None]
    eps = eps_rel * scale
    H = np.empty((T, 12, 12))
    for c in range(12):
        a, i = divmod(c, 3)
        Xp = X.copy()
        Xm = X.copy()
        Xp[:, a, i] += eps[:, 0, 0]
        Xm[:, a, i] -= eps[:, 0, 0]
        H[:, :, c] = (_element_gradients_at(model, Xp)
                      - _element_gradients_at(model, Xm)) / (2.0 * eps[:, 0, :1])
    H = 0.5 * (H + np.swapaxes(H, 1, 2))
    if project:
        w, Q = np.linalg.eigh(H)
        w = np.maximum(w, 0.0)
        H = np.einsum("tij,tj,tkj->tik", Q, w, Q)
    return H


def newton_minimise(model, x0, y, tol=1e-10, max_iter=100, gamma=0.3):
    """Minimise g from x0 (pinned vertices held) with projected Newton + Armijo."""
    f = model.free
    nf = len(f)
    x = np.asarray(x0, dtype=np.float64).copy()
    dof = -np.ones((model.n, 3), dtype=np.int64)
    dof[f] = np.arange(3 * nf).reshape(nf, 3)
    edof = dof[model.tets].reshape(-1, 12)          # (T, 12)
    Mdiag = np.repeat(model.mass[f], 3) / model.h ** 2
    g = fem.objective(model, x, y)
    for it in range(max_iter):
        grad = fem.gradient(model, x, y).reshape(-1)
        if np.linalg.norm(grad) < tol:
            break
        He = element_hessians(model, x)
        r = np.repeat(edof, 12, axis=1).reshape(-1)
        c = np.tile(edof, (1, 12)).reshape(-1)
        v = He.reshape(-1)
        keep = (r >= 0) & (c >= 0)
        H = scipy.sparse.coo_matrix((v[keep], (r[keep], c[keep])), shape=(3 * nf, 3 * nf))
        H = (H + scipy.sparse.diags(Mdiag)).tocsc()
        d = -scipy.sparse.linalg.spsolve(H, grad)
        gtd = float(grad @ d)
        alpha = 1.0
        for _ in range(60):
            xt = x.copy()
            xt[f] = x[f] + alpha * d.reshape(nf, 3)
            gt = fem.objective(model, xt, y)
            if gt <= g + gamma * alpha * gtd:
                break
            alpha *= 0.5
        x, g = xt, gt
    return x, g


def relative_error(g_k: float, g_0: float, g_star: float) -> float:
    """Eq. RelativeError: (g(x_k) - g(x*)) / (g(x_0) - g(x*))."""
    return (g_k - g_star) / (g_0 - g_star)
