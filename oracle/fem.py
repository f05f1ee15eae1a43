"""Element precompute, the implicit-Euler objective g, its gradient, and A.

Oracle module (test infrastructure only; never used by the product path).

Paper passages followed:
* Section 3, Eq. PD: backward Euler as the minimisation of
      g(x) = 1/(2 h^2) tr((x - y)^T M (x - y)) + E(x),
  with M a lumped (diagonal) mass matrix and
      y = 2 q_l - q_{l-1} + h^2 M^{-1} f_ext = q_l + h v + h^2 M^{-1} f_ext.
* Section 3, Eq. PDenergy / PDtotalEnergy: G_i is the deformation-gradient
  operator of a tetrahedron; w_i = V_i k_i (rest volume times stiffness);
  section 4.1 infers k_i from the material (Eq. stiffness).
* Section 3, Eqs. PDmatrixForm and PDsolution: L = sum_i w_i G_i^T G_i and the
  constant SPD matrix M/h^2 + L, factorised once.
* Section 4, Eq. PDgrad2: the gradient of g is M (x - y)/h^2 + grad E(x); for
  a general material grad E is assembled from the element stresses.
* Section 3: the trace form decouples x, y, z, so every matrix is n x n and
  one factor serves the three coordinates.

Readings (paper silent or inconsistent):
* G_i x = F_i^T with F = Ds Dm^{-1} (deformation gradient of a linear tet),
  so G_i^T G_i per coordinate is the 4x4 matrix of dot products of the shape
  function gradients (rows of Dm^{-1}; vertex 0 gets minus their sum).
* The factor 1/2 of the projective energy: the paper writes |Gx - p|^2 in
  Eq. PDenergy but (1/2) x^T L x with L = sum w G^T G in Eq. PDmatrixForm and
  L x - J p in Eq. PDgrad; L = sum_i V_i k_i G_i^T G_i is used, so that k is
  the 1-D second derivative of the energy (section 4.1 "for linear materials").
* Lumped mass: each tet gives a quarter of rho V to each of its vertices.
* Pinned vertices are eliminated: they stay at their input positions, enter
  the element deformation gradients, and A, g's inertia term, the gradient and
  every solver vector live on the free vertices only.
* External force: a uniform body acceleration a (gravity) plus an optional
  per-vertex force, y = x + h v + h^2 (a + f_ext / m).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np
import scipy.linalg
import scipy.sparse
import scipy.sparse.linalg

from . import materials as mat


@dataclasses.dataclass
class Model:
    rest: np.ndarray
    tets: np.ndarray
    free: np.ndarray            # (n_f,) free vertex ids (ascending)
    pinned: np.ndarray          # (p,) pinned vertex ids
    free_of: np.ndarray         # (n,) free index of a vertex or -1
    Dm_inv: np.ndarray          # (T, 3, 3)
    vol: np.ndarray             # (T,)
    mass: np.ndarray            # (n,)
    k: np.ndarray               # (T,)
    mat_groups: list            # [(kind, tet_ids, mu, lam, d2)]
    mu_t: np.ndarray
    lam_t: np.ndarray
    kappa_t: np.ndarray         # (T,) fibre stiffness (0: no fibre term)
    fdir_t: np.ndarray          # (T, 3) unit fibre directions
    h: float
    gravity: np.ndarray
    A: scipy.sparse.csc_matrix  # (n_f, n_f)
    solve: object               # q (n_f, 3) -> A^{-1} q
    planes: np.ndarray = None   # (p, 4) colliders n . x >= c: unit n, c
    coll_k: float = 0.0         # weight of the collision terms

    @property
    def n(self):
        return self.rest.shape[0]

    @property
    def n_free(self):
        return self.free.shape[0]


def _extra(m):
    """The material's parameter beyond mu and lam: the spline's knot values
    a'' (SPLINE) or the second shear modulus mu2 (MOONEY_RIVLIN)."""
    if m.type == mat.MOONEY_RIVLIN:
        return float(getattr(m, "mu2", 0.0) or 0.0)
    return m.d2()


def element_rest_data(rest: np.ndarray, tets: np.ndarray):
    """Dm = [X1 - X0, X2 - X0, X3 - X0] (columns), V = |det Dm| / 6, Dm^{-1}."""
    X = rest[tets]                                   # (T, 4, 3)
    Dm = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
    det = np.linalg.det(Dm)
    vol = np.abs(det) / 6.0
    Dm_inv = np.linalg.inv(Dm)
    return Dm_inv, vol, det


def lumped_mass(n: int, tets: np.ndarray, vol: np.ndarray, rho: np.ndarray):
    m = np.zeros(n)
    for j in range(4):
        np.add.at(m, tets[:, j], rho * vol / 4.0)
    return m


def shape_gradients(Dm_inv: np.ndarray) -> np.ndarray:
    """(T, 4, 3): gradient of each vertex's linear shape function."""
    g123 = Dm_inv                                    # row j-1 = grad N_j
    g0 = -g123.sum(axis=1, keepdims=True)
    return np.concatenate([g0, g123], axis=1)


def assemble_A(n: int, tets, Dm_inv, vol, k, mass, h, free_of):
    """A = diag(m)/h^2 + sum_e V_e k_e G_e^T G_e on the free vertices."""
    B = shape_gradients(Dm_inv)                      # (T, 4, 3)
    Ke = np.einsum("tai,tbi->tab", B, B) * (vol * k)[:, None, None]
    rows = np.repeat(tets, 4, axis=1).reshape(-1)
    cols = np.tile(tets, (1, 4)).reshape(-1)
    vals = Ke.reshape(-1)
    fr = free_of[rows]
    fc = free_of[cols]
    keep = (fr >= 0) & (fc >= 0)
    nf = int((free_of >= 0).sum())
    L = scipy.sparse.coo_matrix((vals[keep], (fr[keep], fc[keep])), shape=(nf, nf))
    free_ids = np.nonzero(free_of >= 0)[0]
    Mdiag = scipy.sparse.diags(mass[free_ids] / (h * h))
    return (L + Mdiag).tocsc()


def make_solver(A: scipy.sparse.csc_matrix):
    """Factorise the constant SPD matrix once; return q -> A^{-1} q.

    Small systems: dense Cholesky (LAPACK). Large systems: reverse
    Cuthill-McKee reordering to a band, then LAPACK's banded Cholesky.
    """
    nf = A.shape[0]
    if nf <= 4000:
        c = scipy.linalg.cho_factor(A.toarray(), lower=True)
        return lambda q: scipy.linalg.cho_solve(c, q)
    from scipy.sparse.csgraph import reverse_cuthill_mckee
    p = reverse_cuthill_mckee(A.tocsr(), symmetric_mode=True)
    Ap = A.tocsr()[p][:, p].tocoo()
    lower = Ap.row >= Ap.col
    bw = int(np.max(Ap.row[lower] - Ap.col[lower]))
    band = np.zeros((bw + 1, nf))
    band[(Ap.row - Ap.col)[lower], Ap.col[lower]] = Ap.data[lower]
    c = scipy.linalg.cholesky_banded(band, lower=True)

    def solve(q):
        r = scipy.linalg.cho_solve_banded((c, True), np.asarray(q)[p])
        out = np.empty_like(r)
        out[p] = r
        return out
    return solve


def build_model(rest, tets, pinned, materials, tet_mat=None, h=1.0 / 30.0,
                gravity=(0.0, 0.0, -9.81), fit_lo=0.5, fit_hi=1.5, planes=None,
                coll_k=0.0) -> Model:
    rest = np.asarray(rest, dtype=np.float64)
    tets = np.asarray(tets, dtype=np.int64)
    n = rest.shape[0]
    T = tets.shape[0]
    if tet_mat is None:
        tet_mat = np.zeros(T, dtype=np.int64)
    tet_mat = np.asarray(tet_mat, dtype=np.int64)
    Dm_inv, vol, _ = element_rest_data(rest, tets)
    rho = np.array([materials[i].density for i in tet_mat])
    mass = lumped_mass(n, tets, vol, rho)

    # Stiffness per material (section 4.1, Eq. stiffness).
    kmat = np.array([mat.stiffness(m.type, m.mu, m.lam, _extra(m), fit_lo, fit_hi)
                     for m in materials])
    k = kmat[tet_mat]
    groups = []
    for mi, m in enumerate(materials):
        ids = np.nonzero(tet_mat == mi)[0]
        if len(ids):
            groups.append((m.type, ids, m.mu, m.lam, _extra(m)))
    # Merge groups of identical non-spline kind into one vectorised group with
    # per-tet parameters (plain bookkeeping, same arithmetic).
    mu_t = np.array([materials[i].mu for i in tet_mat])
    lam_t = np.array([materials[i].lam for i in tet_mat])
    # anisotropic fibre term per tet (kappa = 0: none); unit directions
    kap_m = np.array([float(getattr(m, "fiber_kappa", 0.0) or 0.0) for m in materials])
    dir_m = np.array([_unit(getattr(m, "fiber_dir", None)) for m in materials])
    kappa_t, fdir_t = kap_m[tet_mat], dir_m[tet_mat]
    merged = {}
    final = []
    for kind, ids, mu, lam, d2 in groups:
        if kind in (mat.SPLINE, mat.MOONEY_RIVLIN):
            final.append((kind, ids, mu, lam, d2))
        else:
            merged.setdefault(kind, []).append(ids)
    for kind, idl in merged.items():
        ids = np.sort(np.concatenate(idl))
        final.append((kind, ids, None, None, None))

    pinned = np.unique(np.asarray(pinned, dtype=np.int64))
    free_mask = np.ones(n, dtype=bool)
    free_mask[pinned] = False
    free = np.nonzero(free_mask)[0]
    free_of = -np.ones(n, dtype=np.int64)
    free_of[free] = np.arange(len(free))
    A = assemble_A(n, tets, Dm_inv, vol, k, mass, h, free_of)
    if planes is None or len(planes) == 0:
        planes = np.zeros((0, 4))
    planes = np.asarray(planes, dtype=np.float64).reshape(-1, 4).copy()
    nn = np.linalg.norm(planes[:, :3], axis=1, keepdims=True)
    planes /= nn                        # n . x >= c scaled to a unit normal
    return Model(planes=planes, coll_k=float(coll_k),
                 rest=rest, tets=tets, free=free, pinned=pinned, free_of=free_of,
                 Dm_inv=Dm_inv, vol=vol, mass=mass, k=k, mat_groups=final,
                 mu_t=mu_t, lam_t=lam_t, kappa_t=kappa_t, fdir_t=fdir_t, h=h,
                 gravity=np.asarray(gravity, dtype=np.float64), A=A,
                 solve=make_solver(A))


def _unit(d):
    if d is None:
        return np.array([1.0, 0.0, 0.0])
    d = np.asarray(d, dtype=np.float64)
    return d / np.linalg.norm(d)


def deformation_gradients(model: Model, x: np.ndarray) -> np.ndarray:
    """F_e = Ds_e Dm_e^{-1}, Ds = [x1 - x0, x2 - x0, x3 - x0]."""
    P = x[model.tets]
    Ds = np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]], axis=2)
    return Ds @ model.Dm_inv


def element_psi_P(model: Model, x: np.ndarray):
    """Per-tet energy density and first Piola stress at positions x (n, 3)."""
    F = deformation_gradients(model, x)
    T = F.shape[0]
    psi = np.empty(T)
    Pst = np.empty((T, 3, 3))
    for kind, ids, mu, lam, d2 in model.mat_groups:
        if mu is None:
            mu, lam = model.mu_t[ids], model.lam_t[ids]
        p, P = mat.psi_and_P(kind, F[ids], mu, lam, d2)
        psi[ids] = p
        Pst[ids] = P
    fib = np.nonzero(model.kappa_t > 0)[0]
    if len(fib):  # anisotropic fibre term on top of the base material
        p, P = mat.psi_P_fiber(F[fib], model.kappa_t[fib], model.fdir_t[fib])
        psi[fib] += p
        Pst[fib] += P
    return psi, Pst


def element_forces(model: Model, Pst: np.ndarray) -> np.ndarray:
    """(T, 4, 3) gradient of V Psi w.r.t. each vertex: V P Dm^{-T}, vertex 0 = -sum."""
    H = model.vol[:, None, None] * (Pst @ np.swapaxes(model.Dm_inv, 1, 2))  # (T,3,3) cols
    g123 = np.swapaxes(H, 1, 2)                     # row j = column j of H
    g0 = -g123.sum(axis=1, keepdims=True)
    return np.concatenate([g0, g123], axis=1)


def elastic_energy(model: Model, x: np.ndarray) -> float:
    psi, _ = element_psi_P(model, x)
    return float(np.sum(model.vol * psi))


def inertia_target(model: Model, x, v, f_ext=None):
    """y = x + h v + h^2 (a + f_ext/m) on free vertices, y = x on pinned ones."""
    h = model.h
    acc = np.broadcast_to(model.gravity, x.shape).copy()
    if f_ext is not None:
        acc += f_ext / model.mass[:, None]
    y = x + h * v + h * h * acc
    y[model.pinned] = x[model.pinned]
    return y


# ---------------------------------------------------------------------------
# Collisions (section 4.3): for each free vertex i in collision with a
# collider, the energy term ((S x - t)^T n)^2 with t the vertex's projection
# on the collider surface and n its normal, weighted by coll_k. For a plane
# n . x >= c this is coll_k (n . x_i - c)^2. The set of terms is chosen once
# at the start of an iteration and kept through its line search; the terms
# enter g and grad g but not A.
# ---------------------------------------------------------------------------
def contact_set(model: Model, x: np.ndarray, x_start: np.ndarray) -> np.ndarray:
    """Plane index per free vertex (-1: none): the vertex is in collision or
    contact (n . x <= c) and not separating (its velocity since the start of
    the step, (x - x_start)/h, does not point along n); the deepest plane."""
    f = model.free
    cset = -np.ones(len(f), dtype=np.int64)
    if len(model.planes) == 0:
        return cset
    n, c = model.planes[:, :3], model.planes[:, 3]
    depth = x[f] @ n.T - c                           # (n_f, p)
    moving = (x[f] - x_start[f]) @ n.T               # (n_f, p)
    ok = (depth <= 0.0) & ~(moving > 0.0)
    masked = np.where(ok, depth, np.inf)
    best = np.argmin(masked, axis=1)
    has = np.isfinite(masked[np.arange(len(f)), best])
    cset[has] = best[has]
    return cset


def contact_energy(model: Model, x: np.ndarray, cset) -> float:
    if cset is None or not np.any(cset >= 0):
        return 0.0
    idx = np.nonzero(cset >= 0)[0]
    pl = model.planes[cset[idx]]
    dep = np.einsum("ij,ij->i", x[model.free[idx]], pl[:, :3]) - pl[:, 3]
    return float(model.coll_k * np.sum(dep * dep))


def contact_gradient(model: Model, x: np.ndarray, cset) -> np.ndarray:
    g = np.zeros((len(model.free), 3))
    if cset is None or not np.any(cset >= 0):
        return g
    idx = np.nonzero(cset >= 0)[0]
    pl = model.planes[cset[idx]]
    dep = np.einsum("ij,ij->i", x[model.free[idx]], pl[:, :3]) - pl[:, 3]
    g[idx] = (2.0 * model.coll_k * dep)[:, None] * pl[:, :3]
    return g


def objective(model: Model, x: np.ndarray, y: np.ndarray, cset=None) -> float:
    """g(x) of Eq. PD restricted to the free vertices (pinned inertia is zero),
    plus the collision terms of cset."""
    f = model.free
    dx = x[f] - y[f]
    inertia = float(np.sum(model.mass[f][:, None] * dx * dx)) / (2.0 * model.h ** 2)
    return inertia + elastic_energy(model, x) + contact_energy(model, x, cset)


def gradient(model: Model, x: np.ndarray, y: np.ndarray, cset=None) -> np.ndarray:
    """Gradient of g on the free vertices, (n_f, 3)."""
    _, Pst = element_psi_P(model, x)
    fe = element_forces(model, Pst)
    gE = np.zeros_like(x)
    for j in range(4):
        np.add.at(gE, model.tets[:, j], fe[:, j])
    f = model.free
    return (model.mass[f][:, None] * (x[f] - y[f]) / model.h ** 2 + gE[f]
            + contact_gradient(model, x, cset))


def objective_and_gradient(model: Model, x, y):
    return objective(model, x, y), gradient(model, x, y)
