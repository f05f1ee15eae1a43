"""GPU: numeric refactorisation of A = M/h^2 + sum V k G^T G on the device
for a new time step (the matrix is constant for a fixed h and prefactored,
section 3, Eq. PDsolution; section 4.1, Eq. stiffness).

The refactored solve is checked against the oracle's solve with A assembled
for the new h, the steps that follow against the oracle's steps at that h, and
a round trip back to the prepared h against the host factor's solve. Every
solve schedule is covered: per-level kernels, bottom subtrees, merged levels
and the dense top block.
"""
import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
from paper_1604_07378_amd import qnsim  # noqa: E402

pytestmark = pytest.mark.gpu

SCHEDULES = {"levels": dict(dense_top=0, subtree_cap=0, level_merge=0),
             "subtrees+top": dict(dense_top=64, subtree_cap=384, level_merge=0),
             "merged": dict(dense_top=0, subtree_cap=384, level_merge=1),
             "default": dict(dense_top=6144, subtree_cap=384, level_merge=1)}


def _model(w, h):
    return oracle.build_model(w.rest, w.tets, w.pinned, w.materials, w.tet_mat, h, w.gravity)


def _solve(s, q):
    r = torch.empty(q.shape, dtype=torch.float64, device="cuda")
    s.solve_device(torch.from_numpy(np.ascontiguousarray(q)).cuda(), r)
    torch.cuda.synchronize()
    return r.cpu().numpy()


def _eps(x, ref, rest):
    return np.linalg.norm(x - ref) / max(np.linalg.norm(ref - rest), 1e-300)


@pytest.mark.parametrize("sched", list(SCHEDULES))
@pytest.mark.parametrize("dims", [(10, 3, 3), (16, 14, 12), (1, 1, 1)])
def test_refactor_solve_against_oracle(dims, sched):
    """Prepared at h = 1/30, refactored on the device for h = 1/90 and 1/8:
    r = A(h)^{-1} q against the oracle's solve with A assembled for h."""
    w = W.workload_cantilever(0, dims=dims)
    s = qnsim.sim_from_workload(w, **SCHEDULES[sched])
    q = np.random.default_rng(7).normal(size=(w.n_verts, 3))
    for h in (1.0 / 90.0, 1.0 / 8.0):
        ms = s.refactor(h)
        m = _model(w, h)
        r_ref = np.zeros_like(q)
        r_ref[m.free] = m.solve(q[m.free])
        r = _solve(s, q)
        err = np.abs(r - r_ref).max() / np.abs(r_ref).max()
        assert err <= 1e-11, f"h = {h}: rel err {err:.3e}"
        assert ms > 0.0
    s.close()


@pytest.mark.parametrize("mk", [lambda: W.workload_mixed_cantilever(0),
                                lambda: W.workload_block(W.SPLINE, dims=(6, 5, 4), prestretch_seed=1)],
                         ids=["logE-cantilever", "spline-block"])
def test_refactor_per_element_stiffness(mk):
    """Stiffness varying over three decades per element (log-uniform E), and
    the spline material's fitted k: the refactored solve at h = 1/120 against
    the oracle's."""
    w = mk()
    s = qnsim.sim_from_workload(w, dense_top=0, level_merge=0)
    q = np.random.default_rng(9).normal(size=(w.n_verts, 3))
    h = 1.0 / 120.0
    s.refactor(h)
    m = _model(w, h)
    r_ref = np.zeros_like(q)
    r_ref[m.free] = m.solve(q[m.free])
    r = _solve(s, q)
    err = np.abs(r - r_ref).max() / np.abs(r_ref).max()
    assert err <= 1e-11, f"rel err {err:.3e}"
    s.close()


@pytest.mark.parametrize("sched", ["levels", "default"])
def test_refactor_round_trip_and_steps(sched):
    """Refactor to h = 1/60, run five steps against the oracle at that h; a
    step with the old h is refused; refactoring back to 1/30 reproduces the
    host factor's solve and trajectory to rounding."""
    w = W.workload_block(W.NEOHOOKEAN, dims=(7, 6, 5), prestretch_seed=2)
    s = qnsim.sim_from_workload(w, **SCHEDULES[sched])
    ref = qnsim.sim_from_workload(w, **SCHEDULES[sched])
    q = np.random.default_rng(3).normal(size=(w.n_verts, 3))
    r0 = _solve(ref, q)
    h2 = 1.0 / 60.0
    s.refactor(h2)
    m2 = _model(w, h2)
    x_o, v_o = w.x0.copy(), w.v0.copy()
    x_g, v_g = w.x0.copy(), w.v0.copy()
    for k in range(5):
        r = oracle.step(m2, x_o, v_o)
        x_o, v_o = r.x, r.v
        x_g, v_g, _ = s.step(x_g, v_g, h2)
        e = _eps(x_g, x_o, w.rest)
        assert e <= 1e-9, f"step {k} at h = 1/60: eps {e:.3e}"
    with pytest.raises(qnsim.QnsimError):
        s.step(w.x0, w.v0, w.h)
    s.refactor(w.h)
    r1 = _solve(s, q)
    assert np.abs(r1 - r0).max() <= 1e-12 * np.abs(r0).max()
    xa, va = w.x0.copy(), w.v0.copy()
    xb, vb = w.x0.copy(), w.v0.copy()
    for k in range(3):
        xa, va, _ = s.step(xa, va, w.h)
        xb, vb, _ = ref.step(xb, vb, w.h)
        assert _eps(xa, xb, w.rest) <= 1e-10, f"step {k} after the round trip"
    s.close()
    ref.close()


def test_refactor_state_rules():
    w = W.workload_cantilever(0, dims=(6, 3, 3))
    s = qnsim.sim_from_workload(w, dense_top=0, level_merge=0)
    for bad in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(qnsim.QnsimError):
            s.refactor(bad)
    s.export_factor()                        # host factor valid before
    s.refactor(1.0 / 45.0)
    with pytest.raises(qnsim.QnsimError):
        s.export_factor()                    # host copy belongs to the analysed h
    s.prepare(1.0 / 45.0)                    # analysis again: host factor for 1/45
    s.export_factor()
    s.close()


@pytest.mark.parametrize("sched", ["levels", "default"])
def test_refactor_full_size(sched):
    """The 40^3 block (67,240 unknowns; top front about 1,600 columns):
    refactor for h = 1/60 against the oracle's solve at that h, then back to
    1/30 against the host factor's solve."""
    w = W.workload_block(W.NEOHOOKEAN, n=40)
    s = qnsim.sim_from_workload(w, **SCHEDULES[sched])
    q = np.random.default_rng(11).normal(size=(w.n_verts, 3))
    r0 = _solve(s, q)
    h2 = 1.0 / 60.0
    ms1 = s.refactor(h2)       # builds the plan, then refactors
    ms2 = s.refactor(h2)       # device work only
    m = _model(w, h2)
    r_ref = np.zeros_like(q)
    r_ref[m.free] = m.solve(q[m.free])
    r = _solve(s, q)
    err = np.abs(r - r_ref).max() / np.abs(r_ref).max()
    s.refactor(w.h)
    r1 = _solve(s, q)
    back = np.abs(r1 - r0).max() / np.abs(r0).max()
    print(f"40^3 refactor ({sched}): {ms1:.2f} / {ms2:.2f} ms on the device; "
          f"solve rel err vs oracle {err:.3e}; round trip {back:.3e}", flush=True)
    assert err <= 1e-11 and back <= 1e-12
    s.close()


@pytest.mark.parametrize("sched", ["levels", "subtrees+top", "default"])
def test_device_factor_at_prepare(sched):
    """device_factor = 1: the host orders and analyses, the device computes
    the numeric factor at prepare. Trajectory against the oracle (1e-9, same
    line-search counts) and against the host-factored context (1e-11)."""
    w = W.workload_block(W.STVK, dims=(8, 6, 5), prestretch_seed=4)
    s = qnsim.sim_from_workload(w, device_factor=1, **SCHEDULES[sched])
    ref = qnsim.sim_from_workload(w, **SCHEDULES[sched])
    with pytest.raises(qnsim.QnsimError):
        s.export_factor()                    # no host factor values
    assert s.factor_info()["factor_bytes"] == ref.factor_info()["factor_bytes"]
    m = _model(w, w.h)
    x_o, v_o = w.x0.copy(), w.v0.copy()
    x_g, v_g = w.x0.copy(), w.v0.copy()
    x_r, v_r = w.x0.copy(), w.v0.copy()
    for k in range(6):
        r = oracle.step(m, x_o, v_o)
        x_o, v_o = r.x, r.v
        x_g, v_g, st = s.step(x_g, v_g, w.h)
        x_r, v_r, _ = ref.step(x_r, v_r, w.h)
        assert _eps(x_g, x_o, w.rest) <= 1e-9, f"step {k}"
        assert st["ls_trials"] == r.ls_trials
        assert _eps(x_g, x_r, w.rest) <= 1e-11, f"step {k} vs host factor"
    s.prepare(w.h)                           # again: analysis kept, factor rebuilt
    x2, _, _ = s.step(w.x0, w.v0, w.h)
    x1, _, _ = ref.step(w.x0, w.v0, w.h)
    assert _eps(x2, x1, w.rest) <= 1e-11
    s.close()
    ref.close()


def test_refactor_with_colliders_and_mixed_precision():
    """The cantilever falling onto a tilted plane (section 4.3: the contact
    terms are not in A) after A is refactored for h = 1/45: each of 15 steps,
    from the oracle's state, against the oracle's step at that h (FP64:
    1e-9 with identical trial counts; the mixed path prepared with the device
    factorisation: 1e-4)."""
    w = W.workload_cantilever(0)
    planes = W.cantilever_ground_planes()
    k = 1e5
    h2 = 1.0 / 45.0
    m = oracle.build_model(w.rest, w.tets, w.pinned, w.materials, w.tet_mat, h2, w.gravity,
                           planes=planes, coll_k=k)
    s = qnsim.sim_from_workload(w)
    s.set_colliders(planes, k)
    s.refactor(h2)
    sm = qnsim.sim_from_workload(w, precision=qnsim.QNSIM_MIXED, device_factor=1, prepare=False)
    sm.prepare(h2)
    sm.set_colliders(planes, k)
    xo, vo = w.x0.copy(), w.v0.copy()
    for step in range(15):
        r = oracle.step(m, xo, vo)
        x1, _, st = s.step(xo, vo, h2)
        assert st["ls_trials"] == r.ls_trials, f"step {step}"
        assert _eps(x1, r.x, w.rest) <= 1e-9, f"step {step}"
        x2, _, _ = sm.step(xo, vo, h2)
        assert _eps(x2, r.x, w.rest) <= 1e-4, f"mixed step {step}"
        xo, vo = r.x, r.v
    n, c = planes[0, :3], planes[0, 3]
    assert (xo[m.free] @ n - c).min() < 0.001  # the bar is on the plane
    s.close()
    sm.close()
