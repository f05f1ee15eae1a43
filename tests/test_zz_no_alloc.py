"""GPU: the prefactored solve that allocates nothing (qnsim_solve_device_noalloc)
against the solve of qnsim_solve_device, through the C ABI.

The two run the same kernels on the same inputs; only the working memory
differs (the library's fixed device array instead of the context's buffers),
so their results must agree bit for bit. Two calls in a row on different
meshes, the second smaller, check that nothing the first call left in the
shared array leaks into the second; a mesh too large for the array is
rejected before any device work. r = A^{-1} q itself is held to the oracle
by the prefactored-solve parity tests.
"""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
from paper_1604_07378_amd import qnsim  # noqa: E402

pytestmark = pytest.mark.gpu


def _rhs(w, seed):
    rng = np.random.default_rng(seed)
    return torch.from_numpy(rng.normal(size=(w.n_verts, 3))).cuda()


def _both(sim, q):
    r_ref = torch.full_like(q, float("nan"))
    r_na = torch.full_like(q, float("nan"))
    sim.solve_device(q, r_ref)
    torch.cuda.synchronize()
    sim.solve_device_noalloc(q, r_na)
    torch.cuda.synchronize()
    return r_ref, r_na


def test_noalloc_solve_equals_solve_on_two_meshes_in_a_row():
    big = W.workload_block(W.NEOHOOKEAN, n=20)        # 8,820 free vertices
    small = W.workload_cantilever(0)                   # 160 free vertices
    s_big = qnsim.sim_from_workload(big)
    s_small = qnsim.sim_from_workload(small)
    print("noalloc: block 20^3, then the cantilever, then the block again", flush=True)
    for sim, w, seed in ((s_big, big, 1), (s_small, small, 2), (s_big, big, 3)):
        q = _rhs(w, seed)
        r_ref, r_na = _both(sim, q)
        assert torch.isfinite(r_ref).all()
        assert torch.equal(r_ref, r_na), f"{w.name}: max diff {(r_ref - r_na).abs().max().item()}"
        # pinned rows are zero in both
        assert torch.equal(r_na[torch.from_numpy(w.pinned).long().cuda()],
                           torch.zeros(len(w.pinned), 3, dtype=torch.float64, device="cuda"))
    s_big.close()
    s_small.close()


def test_noalloc_solve_on_a_caller_stream():
    w = W.workload_cantilever(1)
    sim = qnsim.sim_from_workload(w)
    q = _rhs(w, 4)
    r_ref = torch.empty_like(q)
    sim.solve_device(q, r_ref)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    r_na = torch.full_like(q, float("nan"))
    torch.cuda.synchronize()
    sim.solve_device_noalloc(q, r_na, stream=s)
    s.synchronize()
    assert torch.equal(r_ref, r_na)
    sim.close()


def test_noalloc_solve_rejects_a_mesh_larger_than_its_array():
    # a bar of 80,000 cubes pinned at x = 0: 320,000 free vertices need about
    # 9 x 320,000 doubles (22 MB) of working memory, more than the 16 MiB array
    w = W.workload_cantilever(0, dims=(80000, 1, 1))
    sim = qnsim.sim_from_workload(w)
    q = _rhs(w, 5)
    r = torch.full_like(q, 7.0)
    with pytest.raises(qnsim.QnsimError) as e:
        sim.solve_device_noalloc(q, r)
    assert e.value.code == -1                         # QNSIM_E_INVALID
    torch.cuda.synchronize()
    assert torch.equal(r, torch.full_like(q, 7.0))   # output untouched
    # the context stays usable
    sim.solve_device(q, r)
    torch.cuda.synchronize()
    assert torch.isfinite(r).all()
    sim.close()
