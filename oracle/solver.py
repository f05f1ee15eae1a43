"""One implicit-Euler time step: Algorithm 1 with Algorithm 2.

Oracle module (test infrastructure only; never used by the product path).

Paper passages followed:
* Section 4.1, Algorithm 1 (quasi-Newton solver): x_1 := y; for a fixed
  number of iterations: gradient, descent direction, backtracking line search
  starting from alpha = 1 and halving until the Armijo condition
      g(x_k + alpha d) <= g(x_k) + gamma alpha tr(grad g(x_k)^T d)
  holds, gamma = 0.3 (section 4.1, "Line search").
* Section 4.2, Algorithm 2 (L-BFGS two-loop recursion): q := -grad g;
  newest-to-oldest pass computing zeta_i = tr(s_i^T q)/rho_i and
  q -= zeta_i t_i; r := A_0^{-1} q with A_0 = M/h^2 + L (unscaled);
  oldest-to-newest pass with eta = tr(t_i^T r)/rho_i and r += s_i (zeta_i - eta);
  d := r. s_i = x_{i+1} - x_i, t_i = grad g(x_{i+1}) - grad g(x_i),
  rho_i = tr(t_i^T s_i), window m = 5. With m = 0 this is d = -A^{-1} grad g.
* Section 5, Table StatAll: 10 iterations per frame, m = 5, h = 1/30 s.

Readings (paper silent):
* The history holds the pairs of the current time step only (reset every
  step); the window is min(m, pairs stored).
* Curvature safeguard: a pair is stored only if rho > 1e-10 |s| |t| (this
  also skips s = t = 0). If the direction is not a descent direction
  (grad^T d >= 0 with grad != 0), the history is cleared and d = -A^{-1} grad.
* If g(y) is not finite (e.g. an inverted Neo-Hookean element), x_1 := x.
* The line search stops after 30 halvings; if no trial passes, the iterate
  stays x_k and the step's remaining iterations are skipped.
* Pinned vertices keep their input positions; their velocity becomes 0.
* Chebyshev direction (section 5, Algorithm 3, the comparison method):
  q = -A^{-1} grad g(x_k), x^_{k+1} = x_k + q, omega_{k+1} = 1 for k < S,
  2/(2 - rho^2) for k = S, 4/(4 - rho^2 omega_k) for k > S, and
  d = omega_{k+1} (x^_{k+1} - x_{k-1}) + x_{k-1} - x_k; k counts the step's
  iterations from 0 (so d = q while k < S). Readings: if d is not a descent
  direction the iteration uses d = q (counted as a fallback) and the omega
  recursion goes on; it needs history = 0 (no L-BFGS pairs).
* Collisions (section 4.3): the set of collision terms is chosen at the start
  of every iteration (before its gradient) at x_k, g(x_k) is re-evaluated
  with it, and it stays fixed through the iteration's line search; the step
  starts with no terms.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

from . import fem


def two_loop(grad: np.ndarray, pairs, solve) -> np.ndarray:
    """Algorithm 2: d = -B_k grad with pairs [(s, t, rho)] oldest first."""
    q = -grad
    zetas = []
    for s, t, rho in reversed(pairs):                 # i = k-1, ..., k-m
        zeta = float(np.sum(s * q)) / rho
        q = q - zeta * t
        zetas.append(zeta)
    r = solve(q)                                      # r := A_0^{-1} q
    for (s, t, rho), zeta in zip(pairs, reversed(zetas)):   # i = k-m, ..., k-1
        eta = float(np.sum(t * r)) / rho
        r = r + s * (zeta - eta)
    return r


@dataclasses.dataclass
class StepResult:
    x: np.ndarray
    v: np.ndarray
    iterations_run: int = 0
    ls_trials: int = 0
    ls_exhausted: int = 0
    lbfgs_skipped: int = 0
    fallbacks: int = 0
    g_first: float = 0.0
    g_last: float = 0.0
    grad_norm_first: float = 0.0
    grad_norm_last: float = float("nan")
    trace: list = dataclasses.field(default_factory=list)   # per iteration
    omegas: list = dataclasses.field(default_factory=list)  # Chebyshev weights per iteration
    iterates: list = dataclasses.field(default_factory=list)


def step(model: "fem.Model", x: np.ndarray, v: np.ndarray, f_ext=None,
         iterations: int = 10, history: int = 5, gamma: float = 0.3,
         backtrack: float = 0.5, max_halvings: int = 30,
         final_gradient: bool = False, keep_iterates: bool = False,
         x_init: Optional[np.ndarray] = None, direction: str = "lbfgs",
         cheb_delay: int = 10, cheb_rho: float = 0.9) -> StepResult:
    """Advance (x, v) by one step of size model.h; returns the new state."""
    x = np.asarray(x, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    f = model.free
    y = fem.inertia_target(model, x, v, f_ext)
    res = StepResult(x=None, v=None)

    xk = y.copy() if x_init is None else np.asarray(x_init, dtype=np.float64).copy()
    xk[model.pinned] = x[model.pinned]
    gk = fem.objective(model, xk, y)
    if not np.isfinite(gk):
        xk = x.copy()
        gk = fem.objective(model, xk, y)
        res.fallbacks += 1
    res.g_first = gk
    if keep_iterates:
        res.iterates.append(xk.copy())

    pairs: List[tuple] = []
    x_prev = grad_prev = None
    cset = None
    omega = 1.0
    if direction == "chebyshev" and cheb_delay < 1:
        raise ValueError("the Chebyshev delay S must be at least 1 (x_{k-1} is needed)")
    for k in range(iterations):
        if len(model.planes):
            cset = fem.contact_set(model, xk, x)
            gk = fem.objective(model, xk, y, cset)
        grad = fem.gradient(model, xk, y, cset)
        if k == 0:
            res.grad_norm_first = float(np.linalg.norm(grad))
        if x_prev is not None:
            s = xk[f] - x_prev[f]
            t = grad - grad_prev
            rho = float(np.sum(t * s))
            if rho > 1e-10 * np.linalg.norm(s) * np.linalg.norm(t):
                pairs.append((s, t, rho))
                if len(pairs) > history:
                    pairs.pop(0)
            else:
                res.lbfgs_skipped += 1
        if history == 0:
            pairs = []
        if direction == "chebyshev":
            q = model.solve(-grad)                       # q := -A^{-1} grad g(x_k)
            if k < cheb_delay:
                omega = 1.0
            elif k == cheb_delay:
                omega = 2.0 / (2.0 - cheb_rho ** 2)
            else:
                omega = 4.0 / (4.0 - cheb_rho ** 2 * omega)
            res.omegas.append(omega)
            if omega == 1.0:
                d = q
            else:                                        # x_{k-1} exists: k >= S >= 1
                x_hat = xk[f] + q
                d = omega * (x_hat - x_prev[f]) + x_prev[f] - xk[f]
            gtd = float(np.sum(grad * d))
            if gtd >= 0.0 and np.any(grad != 0.0):
                d = q
                gtd = float(np.sum(grad * d))
                res.fallbacks += 1
        else:
            d = two_loop(grad, pairs, model.solve)
            gtd = float(np.sum(grad * d))
            if gtd >= 0.0 and np.any(grad != 0.0):
                pairs = []
                d = model.solve(-grad)
                gtd = float(np.sum(grad * d))
                res.fallbacks += 1

        alpha = 1.0
        accepted = False
        margins = []
        for _ in range(max_halvings + 1):
            xt = xk.copy()
            xt[f] = xk[f] + alpha * d
            gt = fem.objective(model, xt, y, cset)
            res.ls_trials += 1
            bound = gk + gamma * alpha * gtd
            margins.append((alpha, gt, bound))
            if gt <= bound:
                accepted = True
                break
            alpha *= backtrack
        res.trace.append(dict(g=gk, gtd=gtd, alpha=alpha if accepted else 0.0,
                              margins=margins, pairs=len(pairs)))
        res.iterations_run += 1
        if not accepted:
            res.ls_exhausted = 1
            break
        x_prev, grad_prev = xk, grad
        xk, gk = xt, gt
        if keep_iterates:
            res.iterates.append(xk.copy())

    res.g_last = gk
    if final_gradient:
        res.grad_norm_last = float(np.linalg.norm(fem.gradient(model, xk, y, cset)))
    xk[model.pinned] = x[model.pinned]
    res.x = xk
    res.v = (xk - x) / model.h
    res.v[model.pinned] = 0.0
    return res


def simulate(model: "fem.Model", x0, v0, steps: int, **kw):
    """Run `steps` time steps; returns the list of positions and the results."""
    x, v = np.asarray(x0, dtype=np.float64), np.asarray(v0, dtype=np.float64)
    xs, results = [], []
    for _ in range(steps):
        r = step(model, x, v, **kw)
        x, v = r.x, r.v
        xs.append(x)
        results.append(r)
    return xs, results
