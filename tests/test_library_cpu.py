"""CPU checks of the C-ABI library: it loads, exports every declared entry
point, and its host precompute (stiffness fit, lumped masses, the constant
matrix and its supernodal Cholesky factor) agrees with the oracle. No GPU.
"""
import ctypes
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workloads as W
from paper_1604_07378_amd import qnsim

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qnsim.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qnsim_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = qnsim.load_library()
    names = _declared()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(qnsim.SIGNATURES)


def test_defaults_are_the_paper_settings():
    o = qnsim.default_options()
    assert (o.iterations, o.history, o.max_halvings) == (10, 5, 30)
    assert (o.gamma, o.backtrack, o.fit_lo, o.fit_hi) == (0.3, 0.5, 0.5, 1.5)
    assert tuple(o.gravity) == (0.0, 0.0, -9.81)


def _model(w):
    return oracle.build_model(w.rest, w.tets, w.pinned, w.materials, w.tet_mat, w.h, w.gravity)


@pytest.mark.parametrize("kind", [W.NEOHOOKEAN, W.STVK, W.SPLINE, W.COROTATED, W.POLYNOMIAL,
                                  W.MOONEY_RIVLIN])
def test_host_stiffness_and_masses_match_oracle(kind):
    w = W.workload_cantilever(0, kind=kind)
    s = qnsim.sim_from_workload(w, prepare=False)
    m = _model(w)
    assert np.abs(s.stiffness() - m.k).max() <= 1e-13 * m.k.max()
    assert np.abs(s.masses() - m.mass).max() <= 1e-13 * m.mass.max()


def test_host_stiffness_per_element_materials():
    w = W.workload_mixed_cantilever(0)
    s = qnsim.sim_from_workload(w, prepare=False)
    m = _model(w)
    assert np.abs(s.stiffness() - m.k).max() <= 1e-13 * np.abs(m.k).max()


@pytest.mark.parametrize("merge", [(0, 0), (64, 0), (0, 1), (6144, 1)],
                         ids=["plain", "top", "levels", "default"])
@pytest.mark.parametrize("dims", [(10, 3, 3), (7, 5, 3), (1, 1, 1), (12, 10, 9), (20, 8, 8)])
def test_host_factor_reproduces_A(dims, merge):
    """L L^T equals the oracle's A (permuted) to rounding: the ordering,
    symbolic structure, amalgamation, level merging and dense top block (with
    their column renumbering) and numeric factorisation together."""
    w = W.workload_cantilever(0, dims=dims)
    s = qnsim.sim_from_workload(w, prepare=False, dense_top=merge[0], level_merge=merge[1])
    m = _model(w)
    perm, cp, ri, va = s.export_factor()
    nf = len(perm)
    assert sorted(perm.tolist()) == sorted(m.free.tolist())
    L = sp.csc_matrix((va, ri, cp), shape=(nf, nf))
    assert (sp.triu(L, 1).nnz == 0) or abs(sp.triu(L, 1)).max() == 0
    A = m.A.tocsr()[m.free_of[perm]][:, m.free_of[perm]]
    R = L @ L.T - A
    assert abs(R).max() <= 1e-13 * abs(A).max()
    info = s.factor_info()
    assert info["n_free"] == nf and info["nnz_L"] == len(va)
    assert info["nnz_L_exact"] <= info["nnz_L"]


def test_block_factor_statistics():
    """40^3 block: nested dissection keeps the fill near n^{4/3} scaling and the
    supernode tree shallow (the solve is level-scheduled)."""
    w = W.workload_block(W.NEOHOOKEAN, n=40)
    s = qnsim.sim_from_workload(w, prepare=False)
    info = s.factor_info()
    assert info["n_free"] == 67240
    assert info["nnz_L_exact"] < 40e6
    assert info["n_levels"] <= 20
    # the top separators are merged into one dense block of bounded size
    assert 0 < info["dense_top_cols"] <= 6144


def test_errors_are_reported_not_raised_across_the_abi():
    s = qnsim.Sim()
    with pytest.raises(qnsim.QnsimError) as e:
        s.prepare(1 / 30)
    assert e.value.code == -8                     # QNSIM_E_STATE
    rest = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1.0]])
    with pytest.raises(qnsim.QnsimError) as e:
        s.set_mesh(rest, np.array([[0, 1, 2, 7]]))
    assert e.value.code == -1                     # QNSIM_E_INVALID
    flat = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0.0]])
    s.set_mesh(flat, np.array([[0, 1, 2, 3]]))
    s.set_materials([dict(type=0, mu=1e4, lam=1e4, density=1e3)])
    with pytest.raises(qnsim.QnsimError) as e:
        s.analyze(1 / 30)
    assert e.value.code == -3                     # QNSIM_E_DEGENERATE
    s.set_mesh(rest, np.array([[0, 1, 2, 3]]))
    s.set_materials([dict(type=0, mu=1e4, lam=1e4, density=1e3)])
    with pytest.raises(qnsim.QnsimError):
        s.set_materials([dict(type=0, mu=np.nan, lam=1e4, density=1e3)])
    s.set_pinned([0, 1, 2, 3])
    with pytest.raises(qnsim.QnsimError) as e:
        s.analyze(1 / 30)
    assert e.value.code == -1                     # every vertex pinned
    s.set_pinned([0])
    s.analyze(1 / 30)
    assert s.factor_info()["n_free"] == 3
    with pytest.raises(qnsim.QnsimError) as e:
        s.refactor(1 / 60)                        # analysed, not prepared on a device
    assert e.value.code == -8                     # QNSIM_E_STATE
    # qnsim_tune checks its arguments and the prepared state before touching
    # the (never dereferenced) state pointers
    import ctypes
    info = qnsim.TuneInfo()
    fake = ctypes.c_void_p(64)
    assert s._lib.qnsim_tune(s._h, 1 / 30, fake, fake, 0, 0, ctypes.byref(info)) == -1
    assert s._lib.qnsim_tune(s._h, 1 / 30, fake, fake, 2, 8, ctypes.byref(info)) == -1
    assert s._lib.qnsim_tune(s._h, 1 / 30, None, fake, 2, 0, ctypes.byref(info)) == -1
    assert s._lib.qnsim_tune(s._h, 1 / 30, fake, fake, 2, 0, ctypes.byref(info)) == -8


@pytest.mark.parametrize("sched", [dict(dense_top=0, subtree_cap=0, level_merge=0),
                                   dict(dense_top=0, subtree_cap=384, level_merge=0),
                                   dict(dense_top=64, subtree_cap=384, level_merge=0),
                                   dict(dense_top=0, subtree_cap=384, level_merge=1), dict()],
                         ids=["levels", "subtrees", "subtrees+top", "merged", "default"])
@pytest.mark.parametrize("w", [W.workload_cantilever(0), W.workload_cantilever(0, dims=(1, 1, 1)),
                               W.workload_block(W.SPLINE, n=12), W.workload_block(W.SPLINE, n=20)],
                         ids=["cantilever", "one-cube", "block12", "block20"])
def test_solve_schedule_self_check_passes_on_host(w, sched):
    """qnsim_prepare builds the solve schedule (per-level items, bottom
    subtrees, dense top block) and checks it on the host before selecting a
    device; without a GPU it must get as far as hipSetDevice."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present: prepare succeeds instead")
    s = qnsim.sim_from_workload(w, prepare=False, **sched)
    with pytest.raises(qnsim.QnsimError) as e:
        s.prepare(w.h)
    assert "hipSetDevice" in str(e.value), str(e.value)


def _mesh_dict(w):
    return dict(rest=w.rest, tets=w.tets, pinned=w.pinned, tet_mat=w.tet_mat,
                materials=[dict(type=m.type, mu=m.mu, lam=m.lam, density=m.density,
                                spline_d2=m.d2()) for m in w.materials])


def test_pool_staging_and_validation_on_host():
    """Pool host side: parallel analysis stages simulations; an invalid
    description stages nothing; stepping or serving needs resident ones."""
    ws = W.workload_batch(count=5, seed=1, lo=3, hi=6)
    with pytest.raises(qnsim.QnsimError) as e:
        qnsim.Pool(ws[0].h, 0)
    assert e.value.code == -1
    p = qnsim.Pool(ws[0].h, 1 << 30)
    ids = p.add_workloads(ws)
    assert ids == list(range(5))
    info = p.info()
    assert (info["sims_staged"], info["sims_resident"], info["groups"]) == (5, 0, 0)
    bad = _mesh_dict(ws[0])
    bad["tets"] = ws[0].tets.copy()
    bad["tets"][3, 1] = ws[0].rest.shape[0]
    with pytest.raises(qnsim.QnsimError) as e:
        p.add([_mesh_dict(ws[1]), bad])
    assert e.value.code == -1 and "simulation 1" in str(e.value)
    assert p.info()["sims_staged"] == 5
    with pytest.raises(qnsim.QnsimError) as e:
        p.step([ids[0]])
    assert e.value.code == -1
    with pytest.raises(qnsim.QnsimError) as e:
        p.submit(ids[0])
    assert e.value.code == -8
    with pytest.raises(qnsim.QnsimError) as e:
        p.set_force(ids[0], np.zeros((ws[0].n_verts, 3)))   # staged, not resident
    assert e.value.code == -1
    assert p.tune() == ([], [])                   # no group yet: nothing to time
    import ctypes
    tiles = (ctypes.c_int32 * 1)()
    assert p._lib.qnsim_pool_tune(p._p, 8, 1, 1, tiles, None, None, None) == -1   # bad candidate mask
    assert p._lib.qnsim_pool_tune(p._p, 0, 0, 1, tiles, None, None, None) == -1   # reps < 1
    p.remove(ids[2])
    assert p.info()["sims_staged"] == 4
    p.close()


def test_pool_group_schedule_self_check_on_host():
    """A group of uneven meshes with mixed materials builds its combined solve
    schedule and block tables and checks them on the host before selecting a
    device; without a GPU the commit must get as far as hipSetDevice."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present: commit succeeds instead")
    ws = W.workload_batch(count=12, seed=2, lo=3, hi=9)
    p = qnsim.Pool(ws[0].h, 1 << 34)
    p.add_workloads(ws)
    with pytest.raises(qnsim.QnsimError) as e:
        p.commit(0)
    assert "hipSetDevice" in str(e.value), str(e.value)
    assert p.info()["sims_resident"] == 0
    p.close()


def test_fiber_material_validation():
    w = W.workload_fiber_cantilever(0, dims=(2, 1, 1))
    s = qnsim.sim_from_workload(w, prepare=False)
    mats = [dict(type=W.COROTATED, mu=1e4, lam=4e4, density=1000.0, fiber_kappa=5e4,
                 fiber_dir=[0.0, 0.0, 0.0])]
    with pytest.raises(qnsim.QnsimError) as e:
        s.set_materials(mats)
    assert e.value.code == -1
    mats[0]["fiber_dir"] = [0.0, 3.0, 4.0]     # normalised by the library
    s.set_materials(mats)
    mats[0]["fiber_kappa"] = -1.0
    with pytest.raises(qnsim.QnsimError) as e:
        s.set_materials(mats)
    assert e.value.code == -1


def test_bench_refuses_more_than_one_gpu():
    """The bench measures one GPU: asked for more it exits with status 2 and a
    message, before touching torch or the library."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2, r.stderr
    assert "measures one GPU" in r.stderr and r.stdout == ""


def test_bench_byte_accounting_and_traffic_gate(tmp_path, monkeypatch):
    """The bench's algorithmic bytes at 40^3 (the figures the profiles divide
    by), and the measured traffic is used only while the hash of the solve's
    sources matches the one recorded with it."""
    import importlib
    import sys
    sys.path.insert(0, ROOT)
    bench = importlib.import_module("bench")
    # exact factor of the 40^3 block: 25,061,779 entries; 67,240 free vertices
    assert bench.solve_bytes(25061779, 67240) == 404215984
    # 384,000 tets, 68,921 vertices, 67,240 free
    assert bench.element_bytes(384000, 68921, 67240) == 42283544
    fake = tmp_path / "traffic.md"
    fake.write_text("traffic_bytes_per_solve: 123\nsolve_source_sha256_16: 0000000000000000\n")
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(fake))
    assert bench.solve_traffic(40) is None          # sources do not match
    import hashlib
    h = hashlib.sha256()
    for f in bench.SOLVE_SOURCES:
        with open(os.path.join(ROOT, "paper_1604_07378_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    fake.write_text(f"traffic_bytes_per_solve: 123\nsolve_source_sha256_16: {h.hexdigest()[:16]}\n")
    assert bench.solve_traffic(40) == 123
    assert bench.solve_traffic(30) is None          # another workload
