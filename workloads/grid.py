"""Seeded tetrahedral grid workloads.

Every mesh is a regular grid of cubes, each cube split into six tetrahedra
that share its main diagonal (the Kuhn / Freudenthal split), which conforms
across neighbouring cubes. The paper's own meshes are not available; these
grids stand in for them, with the sizes, materials and boundary conditions
of the workloads this project measures:

* cantilever: 10x3x3 cubes of 0.1 m (540 tets, 176 vertices), the x = 0 face
  pinned, rest vertices jittered by up to 1 % of the edge, released from rest
  under gravity;
* block: 40x40x40 cubes of 0.025 m (384,000 tets, 68,921 vertices), the
  z = 0 face pinned, started from a seeded random affine pre-stretch of 10 %;
* mixed cantilever: the cantilever mesh with a Young's modulus drawn per
  element, log-uniform in [1e4, 1e7] Pa;
* batch / pool: many independent grids of seeded sizes and materials.

Nothing here evaluates the method: no deformation gradients, volumes, masses,
stiffness fits, energies or solves.
"""
from __future__ import annotations

import dataclasses
import itertools
from typing import List, Optional, Sequence

import numpy as np

NEOHOOKEAN = 0
STVK = 1
SPLINE = 2
COROTATED = 3
POLYNOMIAL = 4
MOONEY_RIVLIN = 5
MATERIAL_NAMES = {
    NEOHOOKEAN: "neohookean",
    STVK: "stvk",
    SPLINE: "spline",
    COROTATED: "corotated",
    POLYNOMIAL: "polynomial",
    MOONEY_RIVLIN: "mooneyrivlin",
}

# Uniform body acceleration (m/s^2); the external force is M times this field.
GRAVITY = (0.0, 0.0, -9.81)


def lame_from_young(E: float, nu: float):
    """Lame parameters (mu, lambda) from Young's modulus and Poisson's ratio."""
    mu = E / (2.0 * (1.0 + nu))
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    return mu, lam


def spline_knots() -> np.ndarray:
    """Knots of the spline material's stretch term: 8 knots on [0.2, 3]."""
    return 0.2 + 0.4 * np.arange(8, dtype=np.float64)


def spline_d2_multipliers(seed: int) -> np.ndarray:
    """Seeded multipliers u_j ~ U[0.5, 2] of the spline's second derivative.

    The spline material's stretch term a(s) has a''(knot_j) = mu * u_j, is
    piecewise linear in between and constant beyond the end knots, so a is a
    convex C2 cubic spline with a monotone first derivative.
    """
    rng = np.random.default_rng(np.random.SeedSequence([0x5971, seed]))
    return rng.uniform(0.5, 2.0, size=8)


@dataclasses.dataclass
class Material:
    type: int
    mu: float
    lam: float
    density: float = 1000.0
    # a'' at the 8 knots (absolute values, Pa) for SPLINE; zeros otherwise.
    spline_d2: Optional[np.ndarray] = None
    # anisotropic fibre term kappa/2 (|F d| - 1)^2 on top (0: none)
    fiber_kappa: float = 0.0
    fiber_dir: Optional[np.ndarray] = None
    # second shear modulus of MOONEY_RIVLIN (the I2 term); 0 otherwise
    mu2: float = 0.0

    def d2(self) -> np.ndarray:
        if self.spline_d2 is None:
            return np.zeros(8)
        return np.asarray(self.spline_d2, dtype=np.float64)


def make_material(kind: int, E: float, nu: float, density: float = 1000.0,
                  spline_seed: int = 0) -> Material:
    """Material of the given type from Young's modulus and Poisson's ratio.
    Mooney-Rivlin splits the shear modulus mu into 0.7 mu on the I1 term and
    0.3 mu on the I2 term (their sum is the small-strain shear modulus)."""
    mu, lam = lame_from_young(E, nu)
    d2 = None
    if kind == SPLINE:
        d2 = mu * spline_d2_multipliers(spline_seed)
    if kind == MOONEY_RIVLIN:
        return Material(kind, 0.7 * mu, lam, density, None, mu2=0.3 * mu)
    return Material(kind, mu, lam, density, d2)


@dataclasses.dataclass
class Workload:
    name: str
    rest: np.ndarray          # (n, 3) float64 rest positions
    tets: np.ndarray          # (T, 4) int32 vertex indices
    pinned: np.ndarray        # (p,) int32 pinned vertex indices
    materials: List[Material]
    tet_mat: Optional[np.ndarray]  # (T,) int32 material index, None = all 0
    x0: np.ndarray            # (n, 3) initial positions
    v0: np.ndarray            # (n, 3) initial velocities
    h: float = 1.0 / 30.0
    gravity: Sequence[float] = GRAVITY
    dims: tuple = ()
    edge: float = 0.0

    @property
    def n_verts(self) -> int:
        return self.rest.shape[0]

    @property
    def n_tets(self) -> int:
        return self.tets.shape[0]


def kuhn_grid(nx: int, ny: int, nz: int, edge: float):
    """Vertices and Kuhn-split tetrahedra of an nx x ny x nz grid of cubes.

    Vertex (i, j, k) has index i + (nx+1) * (j + (ny+1) * k). Each cube with
    corner c is split into the six tetrahedra (c, c+e_a, c+e_a+e_b, c+(1,1,1))
    over the permutations (a, b, .) of the three axes.
    """
    gx, gy, gz = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1),
                             np.arange(nz + 1), indexing="ij")
    # index = i + (nx+1)*(j + (ny+1)*k): order vertices with i fastest
    ii = gx.transpose(2, 1, 0).reshape(-1)
    jj = gy.transpose(2, 1, 0).reshape(-1)
    kk = gz.transpose(2, 1, 0).reshape(-1)
    rest = np.stack([ii, jj, kk], axis=1).astype(np.float64) * edge

    def vid(i, j, k):
        return i + (nx + 1) * (j + (ny + 1) * k)

    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz),
                             indexing="ij")
    ci = ci.transpose(2, 1, 0).reshape(-1)
    cj = cj.transpose(2, 1, 0).reshape(-1)
    ck = ck.transpose(2, 1, 0).reshape(-1)
    unit = np.eye(3, dtype=np.int64)
    tets = []
    for perm in itertools.permutations(range(3)):
        a, b = unit[perm[0]], unit[perm[1]]
        p0 = (ci, cj, ck)
        p1 = (ci + a[0], cj + a[1], ck + a[2])
        p2 = (ci + a[0] + b[0], cj + a[1] + b[1], ck + a[2] + b[2])
        p3 = (ci + 1, cj + 1, ck + 1)
        tets.append(np.stack([vid(*p0), vid(*p1), vid(*p2), vid(*p3)], axis=1))
    # cube-major order: the six tets of one cube are adjacent
    tets = np.stack(tets, axis=1).reshape(-1, 4).astype(np.int32)
    return rest, tets


def pinned_face(rest: np.ndarray, axis: int, tol: float = 1e-9) -> np.ndarray:
    """Indices of the vertices on the minimum-coordinate face along `axis`."""
    lo = rest[:, axis].min()
    return np.nonzero(rest[:, axis] <= lo + tol)[0].astype(np.int32)


def _jitter(rest: np.ndarray, edge: float, frac: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(np.random.SeedSequence([0x717E, seed]))
    return rest + rng.uniform(-frac, frac, size=rest.shape) * edge


def _affine_prestretch(rest: np.ndarray, pinned: np.ndarray, amount: float,
                       seed: int) -> np.ndarray:
    """x0 = c + A (X - c), A = I + amount * R, R_ij ~ U[-1, 1].

    c is the centroid of the pinned face. The map is applied to every vertex,
    the pinned ones included, which are then held at their mapped positions:
    the whole block starts uniformly deformed, so no element starts inverted.
    """
    rng = np.random.default_rng(np.random.SeedSequence([0xAFF1, seed]))
    A = np.eye(3) + amount * rng.uniform(-1.0, 1.0, size=(3, 3))
    c = rest[pinned].mean(axis=0)
    return c + (rest - c) @ A.T


def workload_cantilever(jitter_seed: int = 0, dims=(10, 3, 3), edge: float = 0.1,
                        kind: int = NEOHOOKEAN, E: float = 1e5, nu: float = 0.4,
                        spline_seed: int = 0) -> Workload:
    """Cantilever bar: x = 0 face pinned, jittered rest shape, released from rest."""
    rest, tets = kuhn_grid(*dims, edge)
    pinned = pinned_face(rest, 0)
    rest = _jitter(rest, edge, 0.01, jitter_seed)
    mat = make_material(kind, E, nu, spline_seed=spline_seed)
    return Workload(
        name=f"cantilever{dims[0]}x{dims[1]}x{dims[2]}-{MATERIAL_NAMES[kind]}",
        rest=rest, tets=tets, pinned=pinned, materials=[mat], tet_mat=None,
        x0=rest.copy(), v0=np.zeros_like(rest), dims=tuple(dims), edge=edge)


def workload_block(kind: int = NEOHOOKEAN, n: int = 40, edge: float = 0.025,
                   prestretch_seed: int = 0, spline_seed: int = 0,
                   E: float = 1e5, nu: float = 0.4, dims=None) -> Workload:
    """Block of n^3 cubes, z = 0 face pinned, seeded 10 % affine pre-stretch."""
    dims = tuple(dims) if dims is not None else (n, n, n)
    rest, tets = kuhn_grid(*dims, edge)
    pinned = pinned_face(rest, 2)
    x0 = _affine_prestretch(rest, pinned, 0.1, prestretch_seed)
    mat = make_material(kind, E, nu, spline_seed=spline_seed)
    return Workload(
        name=f"block{dims[0]}x{dims[1]}x{dims[2]}-{MATERIAL_NAMES[kind]}",
        rest=rest, tets=tets, pinned=pinned, materials=[mat], tet_mat=None,
        x0=x0, v0=np.zeros_like(rest), dims=dims, edge=edge)


def workload_mixed_cantilever(E_seed: int = 0, jitter_seed: int = 0,
                              nu: float = 0.4) -> Workload:
    """Cantilever mesh with a Neo-Hookean E per element, log-uniform [1e4, 1e7]."""
    w = workload_cantilever(jitter_seed=jitter_seed)
    rng = np.random.default_rng(np.random.SeedSequence([0xE1E, E_seed]))
    Es = np.exp(rng.uniform(np.log(1e4), np.log(1e7), size=w.n_tets))
    w.materials = [make_material(NEOHOOKEAN, float(E), nu) for E in Es]
    w.tet_mat = np.arange(w.n_tets, dtype=np.int32)
    w.name = "cantilever10x3x3-neohookean-logE"
    return w


def workload_fiber_cantilever(jitter_seed: int = 0, kind: int = COROTATED, E: float = 1e5,
                              nu: float = 0.4, kappa_over_mu: float = 5.0,
                              direction=(1.0, 0.0, 1.0), dims=(10, 3, 3)) -> Workload:
    """Cantilever with an anisotropic fibre term kappa/2 (|F d| - 1)^2 on a
    base material (corotated, as in the paper's anisotropy example; kappa/mu
    = 5 there); d a fixed unit rest-pose direction."""
    w = workload_cantilever(jitter_seed=jitter_seed, dims=dims, kind=kind, E=E, nu=nu)
    m = w.materials[0]
    m.fiber_kappa = kappa_over_mu * m.mu
    d = np.asarray(direction, dtype=np.float64)
    m.fiber_dir = d / np.linalg.norm(d)
    w.name = w.name + "-fiber"
    return w


def cantilever_ground_planes(depth: float = 0.05, tilt: float = 0.1):
    """One collider under the cantilever: the plane n . x >= c with
    n = (tilt, 0, 1)/|.| through (0, 0, -depth) (the free end comes to rest on
    it under gravity)."""
    n = np.array([tilt, 0.0, 1.0])
    n = n / np.linalg.norm(n)
    return np.array([[n[0], n[1], n[2], float(n @ np.array([0.0, 0.0, -depth]))]])


def workload_batch(count: int = 256, seed: int = 0, lo: int = 4, hi: int = 30,
                   edge: float = 0.025) -> List[Workload]:
    """Independent blocks with per-axis sizes ~ U{lo..hi}, random materials."""
    rng = np.random.default_rng(np.random.SeedSequence([0xBA7C, seed]))
    out = []
    for i in range(count):
        dims = tuple(int(d) for d in rng.integers(lo, hi + 1, size=3))
        kind = int(rng.integers(0, 3))
        nu = float(rng.uniform(0.3, 0.48))
        w = workload_block(kind=kind, dims=dims, edge=edge,
                           prestretch_seed=seed * 100003 + i,
                           spline_seed=seed * 100003 + i, nu=nu)
        out.append(w)
    return out


def workload_pool(count: int = 2000, seed: int = 0, median_tets: float = 20000.0,
                  sigma: float = 1.0, lo: int = 500, hi: int = 400000,
                  edge: float = 0.025) -> List[dict]:
    """Lazy descriptions of a pool of simulations with lognormal tet counts.

    Returns dicts (dims, kind, nu, seed) so that a caller can build the mesh of
    a sim only when it is admitted. Grid dims satisfy 6*a*b*c ~= T with aspect
    ratios drawn from U[0.5, 2].
    """
    rng = np.random.default_rng(np.random.SeedSequence([0x9001, seed]))
    out = []
    for i in range(count):
        T = float(np.clip(np.exp(np.log(median_tets) + sigma * rng.normal()), lo, hi))
        r1, r2 = rng.uniform(0.5, 2.0, size=2)
        base = (T / 6.0 / (r1 * r2)) ** (1.0 / 3.0)
        dims = tuple(max(1, int(round(v))) for v in (base, base * r1, base * r2))
        kind = int(rng.integers(0, 3))
        nu = float(rng.uniform(0.3, 0.48))
        out.append(dict(dims=dims, kind=kind, nu=nu, seed=seed * 1000003 + i,
                        edge=edge))
    return out
