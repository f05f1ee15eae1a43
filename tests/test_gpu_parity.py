"""GPU parity: the HIP path against the FP64 oracle, through the C ABI.

Tolerances (FP64 everywhere on this path):
* per-element Psi and P: 1e-11 of the largest magnitude (the spline material
  goes through two different SVD algorithms);
* objective g: 1e-12 relative; gradient: 1e-11 of its largest entry;
* prefactored solve r = A^{-1} q: 1e-12 of the largest |r|;
* trajectories: eps(N) = |x_gpu(N) - x_ora(N)|_2 / |x_ora(N) - X|_2 <= 1e-9
  after every step (displacement-normalised, all vertices).
"""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle import fem

torch = pytest.importorskip("torch")
from paper_1604_07378_amd import qnsim  # noqa: E402

pytestmark = pytest.mark.gpu

KINDS = [W.NEOHOOKEAN, W.STVK, W.SPLINE, W.COROTATED, W.POLYNOMIAL, W.MOONEY_RIVLIN]


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _model(w):
    return oracle.build_model(w.rest, w.tets, w.pinned, w.materials, w.tet_mat, w.h, w.gravity)


def _perturbed(w, amp, seed):
    rng = np.random.default_rng(seed)
    x = w.rest + amp * w.edge * rng.uniform(-1, 1, size=w.rest.shape)
    x[w.pinned] = w.rest[w.pinned]
    return x


def _eps(x_gpu, x_ora, rest):
    return np.linalg.norm(x_gpu - x_ora) / max(np.linalg.norm(x_ora - rest), 1e-300)


def test_device_visible():
    assert torch.cuda.is_available(), "no HIP device visible"
    print("device:", torch.cuda.get_device_name(0), flush=True)


@pytest.mark.parametrize("kind", KINDS)
def test_element_energy_and_stress(kind):
    w = W.workload_cantilever(0, kind=kind)
    s = qnsim.sim_from_workload(w)
    m = _model(w)
    x = _perturbed(w, 0.15, 1)
    psi_ref, P_ref = fem.element_psi_P(m, x)
    psi = torch.empty(w.n_tets, dtype=torch.float64, device="cuda")
    P = torch.empty(w.n_tets, 9, dtype=torch.float64, device="cuda")
    s.element_stress_device(_dev(x), psi, P)
    torch.cuda.synchronize()
    psi, P = psi.cpu().numpy(), P.cpu().numpy().reshape(-1, 3, 3)
    assert np.abs(psi - psi_ref).max() <= 1e-11 * np.abs(psi_ref).max()
    assert np.abs(P - P_ref).max() <= 1e-11 * np.abs(P_ref).max()


@pytest.mark.parametrize("kind", KINDS)
def test_objective_and_gradient(kind):
    w = W.workload_cantilever(0, kind=kind)
    s = qnsim.sim_from_workload(w)
    m = _model(w)
    x = _perturbed(w, 0.1, 2)
    y = _perturbed(w, 0.1, 3)
    g_ref = fem.objective(m, x, y)
    grad_ref = np.zeros_like(x)
    grad_ref[m.free] = fem.gradient(m, x, y)
    grad = torch.empty(w.n_verts, 3, dtype=torch.float64, device="cuda")
    g = s.eval_device(_dev(x), _dev(y), grad)
    grad = grad.cpu().numpy()
    assert g == pytest.approx(g_ref, rel=1e-12)
    assert np.abs(grad - grad_ref).max() <= 1e-11 * np.abs(grad_ref).max()


# Solve schedules: every level of the unmerged tree through the per-level
# kernels; the bottom subtrees in one workgroup each; a small dense top block
# above them; merged levels without a top block; the defaults (small meshes:
# one dense block).
SCHEDULES = {"levels": dict(dense_top=0, subtree_cap=0, level_merge=0),
             "subtrees": dict(dense_top=0, subtree_cap=384, level_merge=0),
             "subtrees+top": dict(dense_top=64, subtree_cap=384, level_merge=0),
             "merged": dict(dense_top=0, subtree_cap=384, level_merge=1),
             "default": dict(dense_top=6144, subtree_cap=384, level_merge=1)}


@pytest.mark.parametrize("sched", list(SCHEDULES))
@pytest.mark.parametrize("dims", [(10, 3, 3), (7, 5, 3), (1, 1, 1), (16, 14, 12)])
def test_prefactored_solve(dims, sched):
    w = W.workload_cantilever(0, dims=dims)
    s = qnsim.sim_from_workload(w, **SCHEDULES[sched])
    m = _model(w)
    q = np.random.default_rng(4).normal(size=(w.n_verts, 3))
    r_ref = np.zeros_like(q)
    r_ref[m.free] = m.solve(q[m.free])
    r = torch.empty(w.n_verts, 3, dtype=torch.float64, device="cuda")
    s.solve_device(_dev(q), r)
    torch.cuda.synchronize()
    r = r.cpu().numpy()
    assert np.abs(r - r_ref).max() <= 1e-12 * np.abs(r_ref).max()


def _trajectory_parity(w, steps, tol=1e-9, history=5, check_stats=True, sched="default", **opt):
    m = _model(w)
    s = qnsim.sim_from_workload(w, history=history, **SCHEDULES[sched], **opt)
    x_o, v_o = w.x0.copy(), w.v0.copy()
    x_g, v_g = w.x0.copy(), w.v0.copy()
    worst = 0.0
    for k in range(steps):
        r = oracle.step(m, x_o, v_o, history=history)
        x_o, v_o = r.x, r.v
        x_g, v_g, st = s.step(x_g, v_g, w.h)
        e = _eps(x_g, x_o, w.rest)
        worst = max(worst, e)
        assert e <= tol, f"step {k}: eps {e:.3e}"
        if check_stats:
            assert st["iterations_run"] == r.iterations_run
            assert st["ls_trials"] == r.ls_trials, f"step {k}"
            assert st["lbfgs_skipped"] == r.lbfgs_skipped
            assert st["fallbacks"] == r.fallbacks, f"step {k}"
            assert st["g_last"] == pytest.approx(r.g_last, rel=1e-9)
    return worst


def _max_norm_ok(x_gpu, x_ora, rest, tol):
    """Per-vertex bound: the largest coordinate difference against the
    largest displacement, so that an error confined to a few vertices of a
    large mesh is not diluted by the 2-norm over all of them."""
    num = np.abs(x_gpu - x_ora).max()
    den = max(np.abs(x_ora - rest).max(), 1e-300)
    return num / den, num <= tol * den


@pytest.mark.parametrize("sched", list(SCHEDULES))
def test_cantilever_neohookean_100_steps(sched):
    """540-tet cantilever, Neo-Hookean E = 1e5, nu = 0.4, 100 steps from rest,
    under every solve schedule."""
    w = W.workload_cantilever(0)
    worst = _trajectory_parity(w, 100, sched=sched)
    print(f"cantilever NH 100 steps ({sched}): max eps {worst:.3e}", flush=True)


@pytest.mark.parametrize("seed", [1, 2])
def test_cantilever_other_jitter_seeds(seed):
    _trajectory_parity(W.workload_cantilever(seed), 30)


@pytest.mark.parametrize("kind", [W.STVK, W.SPLINE, W.COROTATED, W.POLYNOMIAL, W.MOONEY_RIVLIN])
def test_cantilever_materials(kind):
    _trajectory_parity(W.workload_cantilever(0, kind=kind), 30)


@pytest.mark.parametrize("tile", [128, 512])
@pytest.mark.parametrize("kind", [W.NEOHOOKEAN, W.STVK, W.MOONEY_RIVLIN])
def test_element_tiles(kind, tile):
    """Element-pass blocks of 128 and 512 tets: the 540-tet cantilever spans
    five blocks with a ragged tail, or one full block and a partial one."""
    _trajectory_parity(W.workload_cantilever(0, kind=kind), 20, elem_tile=tile)
    _trajectory_parity(W.workload_mixed_cantilever(0), 5, elem_tile=tile)


@pytest.mark.parametrize("history", [0, 1, 2, 8])
def test_history_window(history):
    _trajectory_parity(W.workload_cantilever(0), 20, history=history)
    _trajectory_parity(W.workload_cantilever(0), 10, history=history, sched="levels")
    _trajectory_parity(W.workload_cantilever(0), 10, history=history, sched="subtrees")


def test_ragged_small_meshes():
    for dims in [(1, 1, 1), (2, 1, 1), (5, 2, 1)]:
        _trajectory_parity(W.workload_cantilever(0, dims=dims), 10)


def test_per_element_young_modulus():
    w = W.workload_mixed_cantilever(0)
    _trajectory_parity(w, 20)


def test_determinism():
    w = W.workload_cantilever(0)
    s = qnsim.sim_from_workload(w)
    outs = []
    for _ in range(2):
        x, v = w.x0.copy(), w.v0.copy()
        for _ in range(5):
            x, v, _st = s.step(x, v, w.h)
        outs.append(x)
    assert np.array_equal(outs[0], outs[1])


def test_device_entry_points_agree_with_host_entry_point():
    w = W.workload_cantilever(0)
    s = qnsim.sim_from_workload(w)
    x, v = w.x0.copy(), w.v0.copy()
    for _ in range(3):
        x, v, _ = s.step(x, v, w.h)
    xd, vd = _dev(w.x0), _dev(w.v0)
    for _ in range(3):
        s.step_device(xd, vd, w.h)
    torch.cuda.synchronize()
    assert np.array_equal(xd.cpu().numpy(), x)
    xr, vr = _dev(w.x0), _dev(w.v0)
    s.run_device(xr, vr, w.h, 3)
    torch.cuda.synchronize()
    assert np.array_equal(xr.cpu().numpy(), x)


def test_step_errors():
    w = W.workload_cantilever(0)
    s = qnsim.sim_from_workload(w)
    with pytest.raises(qnsim.QnsimError) as e:
        s.step(w.x0, w.v0, w.h * 2)
    assert e.value.code == -7
    bad = w.x0.copy()
    bad[100] = bad[100] + np.array([0.0, 0.0, -0.5])   # flips tets through each other
    with pytest.raises(qnsim.QnsimError) as e:
        s.step(bad, w.v0, w.h)
    assert e.value.code == -4
    nanx = w.x0.copy()
    nanx[3, 1] = np.nan
    with pytest.raises(qnsim.QnsimError) as e:
        s.step(nanx, w.v0, w.h)
    assert e.value.code == -2
    x, v, st = s.step(w.x0, w.v0, w.h)           # context still usable
    assert st["iterations_run"] == 10


def test_infeasible_inertial_target_falls_back():
    """A fast vertex makes y invert a Neo-Hookean tet: x_1 := x (host path)."""
    w = W.workload_cantilever(0, dims=(3, 2, 2))
    m = _model(w)
    v = np.zeros_like(w.rest)
    v[m.free[0]] = [0.0, 0.0, -300.0]
    r = oracle.step(m, w.rest, v)
    s = qnsim.sim_from_workload(w)
    x, vv, st = s.step(w.rest, v, w.h)
    assert st["fallbacks"] == r.fallbacks >= 1
    assert _eps(x, r.x, w.rest) <= 1e-9


@pytest.mark.parametrize("sched", ["levels", "subtrees", "merged", "default"])
def test_block_solve_full_size(sched):
    """r = A^{-1} q on the 40^3 block (67,240 unknowns x 3) under the solve
    schedules, against the oracle's banded solve."""
    w = W.workload_block(W.NEOHOOKEAN, n=40)
    s = qnsim.sim_from_workload(w, **SCHEDULES[sched])
    info = s.factor_info()
    assert (info["dense_top_cols"] > 0) == (SCHEDULES[sched]["dense_top"] > 0)
    if sched in ("levels", "subtrees"):
        assert (info["subtree_levels"] > 0) == (sched == "subtrees")
    m = _model(w)
    q = np.random.default_rng(5).normal(size=(w.n_verts, 3))
    r_ref = np.zeros_like(q)
    r_ref[m.free] = m.solve(q[m.free])
    r = torch.empty(w.n_verts, 3, dtype=torch.float64, device="cuda")
    s.solve_device(_dev(q), r)
    torch.cuda.synchronize()
    r = r.cpu().numpy()
    err = np.abs(r - r_ref).max() / np.abs(r_ref).max()
    print(f"block solve {sched} (top {info['dense_top_cols']} cols, subtree levels "
          f"{info['subtree_levels']}, {info['n_levels']} levels): rel err {err:.3e}", flush=True)
    assert err <= 1e-12


@pytest.mark.timeout(600)
@pytest.mark.parametrize("kind", [W.NEOHOOKEAN, W.STVK, W.SPLINE])
def test_block_ten_steps_full_size(kind):
    """The 40^3 block (384,000 tets) at full size, in the benchmark's launch
    configuration (default options, captured step graph): ten free-running
    time steps against the oracle (section 4.1, Algorithm 1; section 4.2,
    Algorithm 2; banded LAPACK solve) at 1e-9, in the displacement-normalised
    2-norm and per vertex, with equal iteration, line-search, skipped-pair and
    fallback counts in every step."""
    w = W.workload_block(kind, n=40)
    s = qnsim.sim_from_workload(w)
    m = _model(w)
    x_o, v_o = w.x0.copy(), w.v0.copy()
    x_g, v_g = _dev(w.x0), _dev(w.v0)
    worst, worst_max = 0.0, 0.0
    for k in range(10):
        r = oracle.step(m, x_o, v_o)
        x_o, v_o = r.x, r.v
        st = s.step_device(x_g, v_g, w.h)
        torch.cuda.synchronize()
        x = x_g.cpu().numpy()
        e = _eps(x, x_o, w.rest)
        em, ok = _max_norm_ok(x, x_o, w.rest, 1e-9)
        worst, worst_max = max(worst, e), max(worst_max, em)
        assert e <= 1e-9, f"step {k}: eps {e:.3e}"
        assert ok, f"step {k}: per-vertex error {em:.3e}"
        assert st["iterations_run"] == r.iterations_run, f"step {k}"
        assert st["ls_trials"] == r.ls_trials, f"step {k}"
        assert st["lbfgs_skipped"] == r.lbfgs_skipped, f"step {k}"
        assert st["fallbacks"] == r.fallbacks, f"step {k}"
        assert st["g_last"] == pytest.approx(r.g_last, rel=1e-9)
    print(f"block {W.MATERIAL_NAMES[kind]} 10 steps: max eps {worst:.3e}, "
          f"max per-vertex {worst_max:.3e}", flush=True)
    s.close()


@pytest.mark.timeout(600)
def test_block_mixed_ten_steps_full_size():
    """Mixed precision on the 40^3 Neo-Hookean block: ten steps, each from the
    oracle's state, against the oracle's step (1e-4 in the 2-norm and per
    vertex) and against the FP64 GPU step from the same state."""
    w = W.workload_block(W.NEOHOOKEAN, n=40)
    s32 = qnsim.sim_from_workload(w, precision=qnsim.QNSIM_MIXED)
    s64 = qnsim.sim_from_workload(w)
    m = _model(w)
    x_o, v_o = w.x0.copy(), w.v0.copy()
    worst_o, worst_g = 0.0, 0.0
    for k in range(10):
        r = oracle.step(m, x_o, v_o)
        x_m, _, _ = s32.step(x_o, v_o, w.h)
        x_g, _, _ = s64.step(x_o, v_o, w.h)
        e_o, e_g = _eps(x_m, r.x, w.rest), _eps(x_m, x_g, w.rest)
        em, ok = _max_norm_ok(x_m, r.x, w.rest, 1e-4)
        assert e_o <= 1e-4 and ok, f"step {k}: eps {e_o:.3e}, per-vertex {em:.3e}"
        assert _eps(x_g, r.x, w.rest) <= 1e-9
        worst_o, worst_g = max(worst_o, e_o, em), max(worst_g, e_g)
        x_o, v_o = r.x, r.v
    print(f"block NH mixed, 10 steps from the oracle's states: max error vs oracle "
          f"{worst_o:.3e}, vs FP64 GPU {worst_g:.3e}", flush=True)
    s32.close()
    s64.close()


def test_chebyshev_ascent_fallback_against_oracle():
    """Algorithm 3's direction can point uphill when omega overshoots (rho
    near 1): the step then falls back to d = -A^{-1} grad g and counts it. With
    rho = 0.999 and S = 5 the cantilever's first steps take the fallback in
    their eighth iteration (cosine of the angle to -grad g about -0.1); the
    GPU must take the same fallbacks and stay on the oracle's trajectory. The
    L-BFGS reset of the same test cannot be reached: with every stored pair's
    rho positive, the two-loop operator is positive definite and d a descent
    direction."""
    w = W.workload_cantilever(0)
    opt = dict(iterations=10, history=0, direction=qnsim.DIR_CHEBYSHEV, cheb_delay=5,
               cheb_rho=0.999)
    m = _model(w)
    s = qnsim.sim_from_workload(w, **opt)
    x_o, v_o = w.x0.copy(), w.v0.copy()
    x_g, v_g = w.x0.copy(), w.v0.copy()
    total = 0
    for k in range(5):
        r = oracle.step(m, x_o, v_o, iterations=10, history=0, direction="chebyshev",
                        cheb_delay=5, cheb_rho=0.999)
        x_o, v_o = r.x, r.v
        x_g, v_g, st = s.step(x_g, v_g, w.h)
        assert _eps(x_g, x_o, w.rest) <= 1e-9, f"step {k}"
        assert st["fallbacks"] == r.fallbacks, f"step {k}"
        assert st["ls_trials"] == r.ls_trials, f"step {k}"
        total += st["fallbacks"]
    assert total >= 3
    s.close()


@pytest.mark.parametrize("kind", [W.MOONEY_RIVLIN])
def test_block_first_step_full_size(kind):
    """The 40^3 block (384,000 tets) at full size, in the benchmark's launch
    configuration: one time step against the oracle (banded LAPACK solve)."""
    w = W.workload_block(kind, n=40)
    s = qnsim.sim_from_workload(w)
    m = _model(w)
    r = oracle.step(m, w.x0, w.v0)
    x, v, st = s.step(w.x0, w.v0, w.h)
    e = _eps(x, r.x, w.rest)
    print(f"block {W.MATERIAL_NAMES[kind]}: eps {e:.3e} trials {st['ls_trials']} / {r.ls_trials}",
          flush=True)
    assert e <= 1e-9
    assert st["ls_trials"] == r.ls_trials


# ---------------------------------------------------------------------------
# Mixed precision (QNSIM_MIXED): FP32 element energies, stresses and force
# contributions; FP64 positions differences, energy sums, gradient gather,
# curvature dot products and solves. Stated tolerance against the FP64
# oracle: eps <= 1e-4 per step.
# ---------------------------------------------------------------------------
def _mixed_vs_oracle(w, steps, tol=1e-4, free_steps=0):
    """Per-step error of the mixed path: every step starts from the oracle's
    state, and the mixed and FP64 GPU results of that one step are compared
    with the oracle's. Also runs the first `free_steps` steps free (each
    implementation from its own state)."""
    m = _model(w)
    s64 = qnsim.sim_from_workload(w)
    s32 = qnsim.sim_from_workload(w, precision=qnsim.QNSIM_MIXED)
    x_o, v_o = w.x0.copy(), w.v0.copy()
    x_f, v_f = w.x0.copy(), w.v0.copy()
    worst_o, worst_g, worst_free = 0.0, 0.0, 0.0
    for k in range(steps):
        r = oracle.step(m, x_o, v_o)
        x_m, _, _ = s32.step(x_o, v_o, w.h)
        x_g, _, _ = s64.step(x_o, v_o, w.h)
        e_o = _eps(x_m, r.x, w.rest)
        e_g = _eps(x_m, x_g, w.rest)
        worst_o, worst_g = max(worst_o, e_o), max(worst_g, e_g)
        assert e_o <= tol, f"step {k}: mixed vs oracle eps {e_o:.3e}"
        if k < free_steps:
            x_f, v_f, _ = s32.step(x_f, v_f, w.h)
            e_f = _eps(x_f, r.x, w.rest)
            worst_free = max(worst_free, e_f)
            assert e_f <= tol, f"free-running step {k}: eps {e_f:.3e}"
        x_o, v_o = r.x, r.v
    return worst_o, worst_g, worst_free


def test_mixed_precision_cantilever_300_steps():
    """Per-element E log-uniform in [1e4, 1e7] Pa on the 540-tet cantilever,
    300 steps: the mixed path's per-step error against the FP64 oracle and the
    FP64 GPU path, and 60 free-running steps. (Beyond about 60 steps this
    floppy bar's motion is chaotic: even the FP64 GPU path and the FP64
    oracle separate by a factor ~10 every 8 steps from rounding differences,
    so free-running trajectories are compared only before that.)"""
    w = W.workload_mixed_cantilever(0)
    wo, wg, wf = _mixed_vs_oracle(w, 300, free_steps=60)
    print(f"mixed cantilever: per-step eps vs oracle max {wo:.3e}, vs FP64 GPU path {wg:.3e}; "
          f"free-running 60 steps {wf:.3e}", flush=True)


@pytest.mark.parametrize("kind", [W.NEOHOOKEAN, W.STVK, W.SPLINE])
def test_mixed_precision_block_first_step(kind):
    w = W.workload_block(kind, n=40)
    wo, wg, _ = _mixed_vs_oracle(w, 1)
    print(f"mixed block {W.MATERIAL_NAMES[kind]}: eps vs oracle {wo:.3e}, vs FP64 GPU {wg:.3e}",
          flush=True)


@pytest.mark.parametrize("amp", [0.15, 1e-4])
@pytest.mark.parametrize("kind", [W.NEOHOOKEAN, W.STVK, W.SPLINE])
def test_mixed_element_energy_and_stress(kind, amp):
    """The mixed path's FP32 element evaluation (from the displacement
    gradient H = F - I) against the FP64 oracle, at moderate strain and at
    strains of about 1e-4: the errors stay at FP32 level relative to the
    largest |Psi| and |P| of the mesh at either strain (1e-5). An FP32
    evaluation on F itself would lose about three digits at the small strain
    (relative error ~6e-8 / strain)."""
    w = W.workload_cantilever(0, kind=kind)
    s = qnsim.sim_from_workload(w, precision=qnsim.QNSIM_MIXED)
    m = _model(w)
    x = _perturbed(w, amp, 11)
    psi_ref, P_ref = fem.element_psi_P(m, x)
    psi = torch.empty(w.n_tets, dtype=torch.float64, device="cuda")
    P = torch.empty(w.n_tets, 9, dtype=torch.float64, device="cuda")
    s.element_stress_device(_dev(x), psi, P)
    torch.cuda.synchronize()
    psi, P = psi.cpu().numpy(), P.cpu().numpy().reshape(-1, 3, 3)
    ep = np.abs(psi - psi_ref).max() / np.abs(psi_ref).max()
    eP = np.abs(P - P_ref).max() / np.abs(P_ref).max()
    print(f"mixed {W.MATERIAL_NAMES[kind]} at amplitude {amp}: Psi {ep:.2e}, P {eP:.2e}", flush=True)
    assert ep <= 1e-5 and eP <= 1e-5
    s.close()


def test_mixed_precision_objective_and_gradient():
    """The mixed evaluation of g and its gradient against the FP64 oracle at a
    perturbed state (FP32 element terms: relative error ~1e-6 expected)."""
    w = W.workload_mixed_cantilever(0)
    m = _model(w)
    s = qnsim.sim_from_workload(w, precision=qnsim.QNSIM_MIXED)
    x = _perturbed(w, 0.05, 3)
    y = _perturbed(w, 0.02, 4)
    g_ref = fem.objective(m, x, y)
    grad_ref = np.zeros_like(x)
    grad_ref[m.free] = fem.gradient(m, x, y)
    grad = torch.empty(w.n_verts, 3, dtype=torch.float64, device="cuda")
    g = s.eval_device(_dev(x), _dev(y), grad)
    grad = grad.cpu().numpy()
    assert abs(g - g_ref) <= 1e-5 * abs(g_ref)
    assert np.abs(grad - grad_ref).max() <= 1e-4 * np.abs(grad_ref).max()


def test_step_graph_replays_equal_eager():
    """The captured step replayed 12 times (with eager probe kernels on the same
    buffers between replays) equals the step launched kernel by kernel, bit for
    bit, together with its statistics."""
    w = W.workload_cantilever(0)
    sg = qnsim.sim_from_workload(w, step_graph=1)
    se = qnsim.sim_from_workload(w, step_graph=0)
    xg, vg = _dev(w.x0), _dev(w.v0)
    xe, ve = _dev(w.x0), _dev(w.v0)
    grad = torch.empty(w.n_verts, 3, dtype=torch.float64, device="cuda")
    for k in range(12):
        a = sg.step_device(xg, vg, w.h, x_out=xg, v_out=vg)
        b = se.step_device(xe, ve, w.h, x_out=xe, v_out=ve)
        torch.cuda.synchronize()
        assert torch.equal(xg, xe) and torch.equal(vg, ve), f"step {k}"
        a.pop("grad_norm_last"); b.pop("grad_norm_last")   # not computed (NaN)
        assert a == b, f"step {k}: stats {a} vs {b}"
        sg.eval_device(xg, xg, grad)   # eager work on the context's buffers between replays
        torch.cuda.synchronize()


def test_fiber_element_objective_and_trajectory():
    """Corotated base + anisotropic fibre term (section 4, Anisotropy): element
    energies and stresses, g and its gradient, and 30 steps against the oracle."""
    w = W.workload_fiber_cantilever(0)
    s = qnsim.sim_from_workload(w)
    m = _model(w)
    x = _perturbed(w, 0.1, 5)
    psi_ref, P_ref = fem.element_psi_P(m, x)
    psi = torch.empty(w.n_tets, dtype=torch.float64, device="cuda")
    P = torch.empty(w.n_tets, 9, dtype=torch.float64, device="cuda")
    s.element_stress_device(_dev(x), psi, P)
    torch.cuda.synchronize()
    psi, P = psi.cpu().numpy(), P.cpu().numpy().reshape(-1, 3, 3)
    assert np.abs(psi - psi_ref).max() <= 1e-11 * np.abs(psi_ref).max()
    assert np.abs(P - P_ref).max() <= 1e-11 * np.abs(P_ref).max()
    y = _perturbed(w, 0.1, 6)
    grad = torch.empty(w.n_verts, 3, dtype=torch.float64, device="cuda")
    g = s.eval_device(_dev(x), _dev(y), grad)
    grad_ref = np.zeros_like(x)
    grad_ref[m.free] = fem.gradient(m, x, y)
    assert g == pytest.approx(fem.objective(m, x, y), rel=1e-12)
    assert np.abs(grad.cpu().numpy() - grad_ref).max() <= 1e-11 * np.abs(grad_ref).max()
    xo, vo = w.x0.copy(), w.v0.copy()
    xg, vg = w.x0.copy(), w.v0.copy()
    worst = 0.0
    for k in range(30):
        r = oracle.step(m, xo, vo)
        xo, vo = r.x, r.v
        xg, vg, st = s.step(xg, vg, w.h)
        assert st["ls_trials"] == r.ls_trials, f"step {k}: trials {st['ls_trials']} vs {r.ls_trials}"
        e = _eps(xg, xo, w.rest)
        worst = max(worst, e)
        assert e <= 1e-9, f"step {k}: eps {e:.3e}"
    print(f"fiber cantilever 30 steps: max eps {worst:.3e}", flush=True)


def test_collisions_with_a_plane_against_oracle():
    """The cantilever's free end falls onto a tilted plane and chatters on it
    (section 4.3): each of 25 steps, from the oracle's state, matches the
    oracle's step (1e-9, identical line-search trial counts); free-running
    trajectories are compared over the first 8 steps only (afterwards rounding
    differences flip contact decisions and the trajectories separate by about
    10x per step, in the oracle against itself as much as here). The collider
    is set after prepare, and removed again."""
    w = W.workload_cantilever(0)
    planes = W.cantilever_ground_planes()
    k = 1e5
    m = oracle.build_model(w.rest, w.tets, w.pinned, w.materials, w.tet_mat, w.h, w.gravity,
                           planes=planes, coll_k=k)
    s = qnsim.sim_from_workload(w)
    s.set_colliders(planes * 2.0, k)          # scaled rows: normalised by the library
    sf = qnsim.sim_from_workload(w)
    sf.set_colliders(planes, k)
    xo, vo = w.x0.copy(), w.v0.copy()
    xf, vf = w.x0.copy(), w.v0.copy()
    worst, worst_free, trials = 0.0, 0.0, 0
    for step in range(25):
        r = oracle.step(m, xo, vo)
        x1, _, st = s.step(xo, vo, w.h)
        assert st["ls_trials"] == r.ls_trials, f"step {step}: trials {st['ls_trials']} vs {r.ls_trials}"
        trials += st["ls_trials"]
        e = _eps(x1, r.x, w.rest)
        worst = max(worst, e)
        assert e <= 1e-9, f"step {step}: eps {e:.3e}"
        if step < 8:
            xf, vf, _ = sf.step(xf, vf, w.h)
            e = _eps(xf, r.x, w.rest)
            worst_free = max(worst_free, e)
            assert e <= 1e-9, f"free-running step {step}: eps {e:.3e}"
        xo, vo = r.x, r.v
    n, c = planes[0, :3], planes[0, 3]
    assert (xo[m.free] @ n - c).min() < 0.01
    print(f"collisions: 25 steps, per-step eps {worst:.3e}, free-running 8 steps {worst_free:.3e}, "
          f"{trials} line-search trials", flush=True)
    s.set_colliders(np.zeros((0, 4)), 0.0)    # removed: the plain step again
    r = oracle.step(_model(w), xo, vo)
    x1, _, _ = s.step(xo, vo, w.h)
    assert _eps(x1, r.x, w.rest) <= 1e-9


def test_chebyshev_direction_against_oracle():
    """Chebyshev semi-iterative direction (section 5, Algorithm 3) with 30
    iterations per step, S = 10, rho = 0.94: 5 steps against the oracle (1e-9,
    identical line-search trial counts and fallbacks)."""
    w = W.workload_cantilever(0)
    m = _model(w)
    opts = dict(iterations=30, history=0, direction=qnsim.DIR_CHEBYSHEV, cheb_delay=10,
                cheb_rho=0.94)
    s = qnsim.sim_from_workload(w, **opts)
    xo, vo = w.x0.copy(), w.v0.copy()
    xg, vg = w.x0.copy(), w.v0.copy()
    worst = 0.0
    for step in range(5):
        r = oracle.step(m, xo, vo, iterations=30, history=0, direction="chebyshev",
                        cheb_delay=10, cheb_rho=0.94)
        xo, vo = r.x, r.v
        xg, vg, st = s.step(xg, vg, w.h)
        assert (st["ls_trials"], st["fallbacks"]) == (r.ls_trials, r.fallbacks), f"step {step}"
        e = _eps(xg, xo, w.rest)
        worst = max(worst, e)
        assert e <= 1e-9, f"step {step}: eps {e:.3e}"
    print(f"chebyshev 5 steps x 30 iterations: max eps {worst:.3e}", flush=True)


def test_tune_single_context():
    """qnsim_tune on the 540-tet cantilever from a perturbed state: the state
    tensors stay as they were, every schedule and tile is timed, the tuned
    context steps as a fresh context created with the kept options (bit for
    bit) and as the oracle (1e-9); with the device factorisation and after a
    time-step change (A refactored on the device) the tile-only and the full
    tune keep oracle parity at the new h."""
    w = W.workload_cantilever(0)
    x0 = _perturbed(w, 0.05, 7)
    x, v = _dev(x0), _dev(w.v0)
    xc, vc = x.clone(), v.clone()
    s = qnsim.sim_from_workload(w)
    info = s.tune(x, v, w.h, reps=2)
    print(f"tune: {info}", flush=True)
    assert torch.equal(x, xc) and torch.equal(v, vc)
    assert np.isfinite(info["schedule_ms"]).all() and np.isfinite(info["tile_ms"]).all()
    assert np.isfinite(info["trials_ms"]).all() and info["trials_per_cycle"] in (1, 2, 3)
    kept = dict(dense_top=info["dense_top"], subtree_cap=info["subtree_cap"],
                level_merge=info["level_merge"], elem_tile=info["elem_tile"],
                trials_per_cycle=info["trials_per_cycle"])
    assert (kept["dense_top"], kept["subtree_cap"], kept["level_merge"]) in [
        (0, 0, 0), (0, 384, 0), (0, 384, 1), (6144, 384, 1)]
    assert kept["elem_tile"] in (128, 256, 512)
    fresh = qnsim.sim_from_workload(w, **kept)
    m = _model(w)
    xo, vo = x0.copy(), w.v0.copy()
    xa, va = x0.copy(), w.v0.copy()
    xb, vb = x0.copy(), w.v0.copy()
    for k in range(10):
        r = oracle.step(m, xo, vo)
        xo, vo = r.x, r.v
        xa, va, _ = s.step(xa, va, w.h)
        xb, vb, _ = fresh.step(xb, vb, w.h)
        assert np.array_equal(xa, xb) and np.array_equal(va, vb), f"step {k}"
        assert _eps(xa, xo, w.rest) <= 1e-9, f"step {k}"
    fresh.close()
    s.close()
    h2 = 1.0 / 60.0
    w2 = W.workload_cantilever(0)
    w2.h = h2
    m2 = _model(w2)
    for opts in (dict(device_factor=1), dict()):
        s = qnsim.sim_from_workload(w, **opts)
        s.refactor(h2)
        for sched in (False, True):
            info = s.tune(x, v, h2, reps=1, schedule=sched)
            assert np.isnan(info["schedule_ms"]).all() != sched
            xo, vo = x0.copy(), w.v0.copy()
            xa, va = x0.copy(), w.v0.copy()
            for k in range(5):
                r = oracle.step(m2, xo, vo)
                xo, vo = r.x, r.v
                xa, va, _ = s.step(xa, va, h2)
                assert _eps(xa, xo, w.rest) <= 1e-9, f"{opts} schedule {sched} step {k}"
        s.close()


def test_resume_from_saved_state():
    """The method keeps no state across steps (the L-BFGS window starts empty
    every step), so (x, v) is the whole checkpoint: 10 steps in one context
    equal 5 steps, a new context, and 5 more from the saved state, bit for bit."""
    w = W.workload_cantilever(0)
    s = qnsim.sim_from_workload(w)
    x, v = w.x0.copy(), w.v0.copy()
    traj = []
    for _ in range(10):
        x, v, _ = s.step(x, v, w.h)
        traj.append((x, v))
    s.close()
    s = qnsim.sim_from_workload(w)
    x, v = traj[4]
    s.close()
    s = qnsim.sim_from_workload(w)
    x, v = x.copy(), v.copy()
    for k in range(5, 10):
        x, v, _ = s.step(x, v, w.h)
        assert np.array_equal(x, traj[k][0]) and np.array_equal(v, traj[k][1]), f"step {k}"
    s.close()


@pytest.mark.parametrize("max_halvings", [0, 1, 4])
def test_line_search_exhaustion(max_halvings):
    """A StVK cantilever thrown with random 5 m/s vertex velocities: with at
    most 0, 1 or 4 halvings the first iteration's line search fails (up to 5
    trials, more than one cycle's budget of 2); the iterate stays where the
    iteration started and the step's remaining iterations are skipped. GPU
    and oracle agree on the statistics exactly and on the positions to 1e-9."""
    w = W.workload_cantilever(0, kind=W.STVK)
    m = _model(w)
    rng = np.random.default_rng(4)
    v0 = 5.0 * rng.normal(size=w.rest.shape)
    v0[w.pinned] = 0.0
    s = qnsim.sim_from_workload(w, max_halvings=max_halvings)
    x_o, v_o = w.rest.copy(), v0.copy()
    x_g, v_g = w.rest.copy(), v0.copy()
    for k in range(3):
        r = oracle.step(m, x_o, v_o, max_halvings=max_halvings)
        x_o, v_o = r.x, r.v
        x_g, v_g, st = s.step(x_g, v_g, w.h)
        assert r.ls_exhausted == 1, "the case must exhaust its line search"
        assert (st["ls_exhausted"], st["iterations_run"], st["ls_trials"]) == \
            (r.ls_exhausted, r.iterations_run, r.ls_trials), f"step {k}"
        assert _eps(x_g, x_o, w.rest) <= 1e-9, f"step {k}"
        assert np.abs(v_g - v_o).max() <= 1e-9 * max(np.abs(v_o).max(), 1.0)
    s.close()
