"""GPU: pools of resident simulations (batched and served steps).

A simulation stepped in a group (one concatenated device mesh, every phase
one launch over all stepping simulations, the element pass one launch per
material type) must give the result it gives alone, with the same options
(pools use dense_top = 0 and level_merge = 0), bit for bit. Small cases are
also checked against the FP64 oracle (1e-9).
"""
import threading

import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
from paper_1604_07378_amd import qnsim  # noqa: E402

pytestmark = pytest.mark.gpu


def _eps(x, ref, rest):
    return np.linalg.norm(x - ref) / max(np.linalg.norm(ref - rest), 1e-300)


def _alone(w, steps, **opt):
    """States after each of `steps` steps of w run alone (pool options)."""
    s = qnsim.sim_from_workload(w, dense_top=0, level_merge=0, **opt)
    x, v = w.x0.copy(), w.v0.copy()
    out = []
    for _ in range(steps):
        x, v, _ = s.step(x, v, w.h)
        out.append((x.copy(), v.copy()))
    s.close()
    return out


def _pool(ws, budget=1 << 34, group=0, **opt):
    p = qnsim.Pool(ws[0].h, budget, gravity=tuple(ws[0].gravity), **opt)
    ids = p.add_workloads(ws)
    assert p.commit(group) == len(ws)
    return p, ids


def test_batch_equals_alone_one_material():
    """Eight Neo-Hookean blocks of uneven size in one group, 12 steps."""
    ws = [W.workload_block(W.NEOHOOKEAN, dims=d, prestretch_seed=i)
          for i, d in enumerate([(3, 3, 3), (5, 3, 4), (4, 6, 3), (3, 3, 8),
                                 (6, 5, 4), (2, 7, 3), (4, 4, 4), (7, 3, 5)])]
    p, ids = _pool(ws)
    assert p.info()["groups"] == 1
    steps = 12
    ref = [_alone(w, steps) for w in ws]
    for k in range(steps):
        st = p.step(ids)
        assert all(s["iterations_run"] == 10 for s in st)
        for j, w in enumerate(ws):
            x, v = p.get_state(ids[j])
            assert np.array_equal(x, ref[j][k][0]), f"sim {j} step {k}: not bitwise equal"
            assert np.array_equal(v, ref[j][k][1])
    print(f"8 NH blocks, {steps} batched steps: bitwise equal to each block alone", flush=True)
    p.close()


def test_batch_mixed_materials_against_alone_and_oracle():
    """Blocks with NH / StVK / spline materials and per-block nu (the batched
    workload's generator at small sizes), 6 steps: each equals its run alone
    bit for bit; the first two also match the oracle."""
    ws = W.workload_batch(count=6, seed=3, lo=3, hi=6)
    p, ids = _pool(ws)
    steps = 6
    ref = [_alone(w, steps) for w in ws]
    for k in range(steps):
        p.step(ids)
        for j, w in enumerate(ws):
            x, v = p.get_state(ids[j])
            assert np.array_equal(x, ref[j][k][0]) and np.array_equal(v, ref[j][k][1]), \
                f"sim {j} step {k}: eps vs alone {_eps(x, ref[j][k][0], w.rest):.3e}"
    for j in range(2):
        w = ws[j]
        m = oracle.build_model(w.rest, w.tets, w.pinned, w.materials, w.tet_mat, w.h, w.gravity)
        x, v = w.x0.copy(), w.v0.copy()
        for k in range(steps):
            r = oracle.step(m, x, v)
            x, v = r.x, r.v
            e = _eps(ref[j][k][0], r.x, w.rest)
            assert e <= 1e-9, f"sim {j} step {k}: eps vs oracle {e:.3e}"
    print("mixed-material batch: bitwise equal to each mesh alone", flush=True)
    p.close()


@pytest.mark.timeout(600)
def test_batch_with_a_large_mesh_equals_alone_and_oracle():
    """A 22 x 20 x 21 block (55,440 tets: the per-level solve items and
    element blocks of the pool options at scale) among five small blocks of
    mixed materials, in one group. Steps alternate between the whole batch
    and partial batches (compacted launch lists) that include or leave out
    the large block; every simulation equals its run alone with as many
    steps, bit for bit, and the large block's first two steps match the
    oracle at 1e-9 (section 4.1, Algorithm 1)."""
    big = W.workload_block(W.NEOHOOKEAN, dims=(22, 20, 21), prestretch_seed=7)
    small = W.workload_batch(count=5, seed=11, lo=3, hi=6)
    ws = [small[0], small[1], big, small[2], small[3], small[4]]
    p, ids = _pool(ws)
    assert p.info()["groups"] == 1
    plan = [list(range(6)), [2, 0], list(range(6)), [1, 3, 4], [2, 5]]
    counts = [0] * 6
    for sub in plan:
        for j in sub:
            counts[j] += 1
    ref = [_alone(w, max(counts[j], 1)) for j, w in enumerate(ws)]
    done = [0] * 6
    for k, sub in enumerate(plan):
        p.step([ids[j] for j in sub])
        for j in sub:
            done[j] += 1
        for j in range(6):
            if done[j] == 0:
                continue
            x, v = p.get_state(ids[j])
            xr, vr = ref[j][done[j] - 1]
            assert np.array_equal(x, xr) and np.array_equal(v, vr), \
                f"batch step {k}, sim {j} ({ws[j].n_tets} tets) after {done[j]} steps: " \
                f"eps vs alone {_eps(x, xr, ws[j].rest):.3e}"
    m = oracle.build_model(big.rest, big.tets, big.pinned, big.materials, big.tet_mat, big.h,
                           big.gravity)
    x, v = big.x0.copy(), big.v0.copy()
    for k in range(2):
        r = oracle.step(m, x, v)
        x, v = r.x, r.v
        e = _eps(ref[2][k][0], r.x, big.rest)
        assert e <= 1e-9, f"large block step {k}: eps vs oracle {e:.3e}"
    print(f"large block in a batch of 6: bitwise equal alone over {plan}", flush=True)
    p.close()


def test_batch_with_mooney_rivlin_equals_alone():
    """Neo-Hookean, Mooney-Rivlin and spline blocks in one group (one element
    launch per material type), 5 steps: each equals its run alone, bit for
    bit, and the Mooney-Rivlin block matches the oracle."""
    kinds = [W.NEOHOOKEAN, W.MOONEY_RIVLIN, W.SPLINE, W.MOONEY_RIVLIN]
    ws = [W.workload_block(k, dims=(4 + i, 3, 4), prestretch_seed=30 + i) for i, k in enumerate(kinds)]
    p, ids = _pool(ws)
    steps = 5
    ref = [_alone(w, steps) for w in ws]
    for k in range(steps):
        p.step(ids)
        for j in range(len(ws)):
            x, v = p.get_state(ids[j])
            assert np.array_equal(x, ref[j][k][0]) and np.array_equal(v, ref[j][k][1]), \
                f"sim {j} step {k}"
    w = ws[1]
    m = oracle.build_model(w.rest, w.tets, w.pinned, w.materials, w.tet_mat, w.h, w.gravity)
    x, v = w.x0.copy(), w.v0.copy()
    for k in range(steps):
        r = oracle.step(m, x, v)
        x, v = r.x, r.v
        assert _eps(ref[1][k][0], r.x, w.rest) <= 1e-9, f"step {k}"
    p.close()


def test_subsets_and_groups():
    """Four groups of two; alternating subsets step; the others keep their state."""
    ws = [W.workload_block(W.STVK, dims=(3 + i % 3, 3, 4), prestretch_seed=10 + i) for i in range(8)]
    p, ids = _pool(ws, group=2)
    assert p.info()["groups"] == 4
    counts = [0] * 8
    ref = [_alone(w, 5) for w in ws]
    for rnd in range(6):
        sub = [ids[j] for j in range(8) if (j + rnd) % 3 != 0]
        before = {j: p.get_state(ids[j]) for j in range(8)}
        p.step(sub)
        for j in range(8):
            x, v = p.get_state(ids[j])
            if ids[j] in sub:
                counts[j] += 1
                if counts[j] <= 5:
                    assert np.array_equal(x, ref[j][counts[j] - 1][0]), f"sim {j} after {counts[j]} steps"
            else:
                assert np.array_equal(x, before[j][0]) and np.array_equal(v, before[j][1])
    info = p.info()
    assert info["steps_done"] == sum(counts)
    p.close()


def test_mixed_precision_pool_equals_alone():
    ws = [W.workload_block(W.NEOHOOKEAN, dims=(4, 3, 3), prestretch_seed=i) for i in range(3)]
    p, ids = _pool(ws, precision=qnsim.QNSIM_MIXED)
    ref = [_alone(w, 4, precision=qnsim.QNSIM_MIXED) for w in ws]
    for k in range(4):
        p.step(ids)
        for j in range(3):
            assert np.array_equal(p.get_state(ids[j])[0], ref[j][k][0])
    p.close()


def test_budget_admission_and_remove():
    ws = [W.workload_block(W.NEOHOOKEAN, dims=(4, 4, 4), prestretch_seed=i) for i in range(6)]
    probe = qnsim.Pool(ws[0].h, 1 << 34)
    probe.add_workloads(ws[:1])
    probe.commit(0)
    one = probe.info()["used_bytes"]
    probe.close()
    p = qnsim.Pool(ws[0].h, int(3.5 * one))
    ids = p.add_workloads(ws)
    admitted = p.commit(1)
    info = p.info()
    assert 1 <= admitted < 6 and info["sims_resident"] == admitted
    assert info["sims_staged"] == 6 - admitted and info["used_bytes"] <= info["budget_bytes"]
    with pytest.raises(qnsim.QnsimError):
        p.step([ids[-1]])                      # staged, not resident
    p.remove(ids[0])                           # frees its one-simulation group
    assert p.info()["used_bytes"] < info["used_bytes"]
    more = p.commit(1)
    assert more >= 1 and p.info()["sims_resident"] == admitted - 1 + more
    p.close()


def test_serving_results_equal_alone():
    """Requests from four client threads with random pacing over six
    simulations in three groups (two materials each); each simulation's final
    state equals its run alone with the same number of steps."""
    ws = [W.workload_block([W.NEOHOOKEAN, W.STVK, W.SPLINE][i % 3], dims=(3, 4, 3),
                           prestretch_seed=20 + i) for i in range(6)]
    p, ids = _pool(ws, group=2)
    p.serve_start(lanes=2)
    rng = np.random.default_rng(5)
    plan = [list(rng.integers(0, 6, size=8)) for _ in range(4)]
    lat = []
    lock = threading.Lock()

    def client(seq, seed):
        r = np.random.default_rng(seed)
        tickets = []
        for j in seq:
            tickets.append(p.submit(ids[int(j)]))
            if r.uniform() < 0.5:
                import time
                time.sleep(r.uniform(0, 0.003))
        for t in tickets:
            st, l = p.wait(t, 60.0)
            assert st["iterations_run"] == 10
            with lock:
                lat.append(l)

    th = [threading.Thread(target=client, args=(plan[i], i)) for i in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    p.serve_stop()
    counts = np.bincount(np.concatenate(plan).astype(int), minlength=6)
    assert len(lat) == counts.sum() and min(lat) > 0
    for j, w in enumerate(ws):
        if counts[j] == 0:
            continue
        ref = _alone(w, int(counts[j]))
        x, _ = p.get_state(ids[j])
        assert np.array_equal(x, ref[-1][0]), \
            f"sim {j}: served result differs from alone, eps {_eps(x, ref[-1][0], w.rest):.3e}"
    info = p.info()
    assert info["steps_done"] == counts.sum() and info["batches_done"] <= counts.sum()
    print(f"served {counts.sum()} requests in {info['batches_done']} batches; "
          f"latency p50 {np.median(lat) * 1e3:.2f} ms; each bitwise equal to alone", flush=True)
    p.close()


def test_commit_while_serving_results_equal_alone():
    """Live admission: while two lanes serve a steady stream of requests for
    four resident simulations, three new ones are added and committed (built
    and uploaded outside the pool's lock); requests for them follow as soon
    as they are resident. Every simulation's final state equals its run
    alone with the same number of steps, bit for bit."""
    import time
    old = [W.workload_block([W.NEOHOOKEAN, W.STVK][i % 2], dims=(3, 3 + i, 4),
                            prestretch_seed=60 + i) for i in range(4)]
    new = [W.workload_block([W.SPLINE, W.NEOHOOKEAN, W.STVK][i], dims=(4, 3, 3 + i),
                            prestretch_seed=70 + i) for i in range(3)]
    p, ids = _pool(old, group=2)
    p.serve_start(lanes=2)
    counts = {}
    stop = threading.Event()
    errors = []

    def client():
        try:
            k = 0
            while not stop.is_set() or k < 24:
                j = k % 4
                t = p.submit(ids[j])
                st, _ = p.wait(t, 60.0)
                assert st["iterations_run"] == 10
                counts[ids[j]] = counts.get(ids[j], 0) + 1
                k += 1
        except Exception as e:  # noqa: BLE001
            errors.append(e)

    th = threading.Thread(target=client)
    th.start()
    time.sleep(0.05)
    before = p.info()["steps_done"]
    nids = p.add_workloads(new)
    admitted = p.commit(0)
    during = p.info()["steps_done"] - before
    assert admitted == 3
    tickets = [(nid, p.submit(nid)) for nid in nids for _ in range(2)]
    for nid, t in tickets:
        st, _ = p.wait(t, 60.0)
        assert st["iterations_run"] == 10
        counts[nid] = counts.get(nid, 0) + 1
    stop.set()
    th.join()
    p.serve_stop()
    assert not errors, errors
    for j, w in enumerate(old + new):
        sid = (ids + nids)[j]
        ref = _alone(w, counts[sid])
        x, v = p.get_state(sid)
        assert np.array_equal(x, ref[-1][0]) and np.array_equal(v, ref[-1][1]), \
            f"sim {j} after {counts[sid]} served steps: eps vs alone {_eps(x, ref[-1][0], w.rest):.3e}"
    print(f"live admission: {during} requests completed while the commit ran; "
          f"{sum(counts.values())} served in all, each bitwise equal to alone", flush=True)
    p.close()


def test_commit_repacks_a_group_with_removed_members():
    """Two of four members of a group (holding more than half of its memory)
    are removed; the next commit rebuilds the group with the two live members
    (states copied on the device), returning memory to the budget; their
    later steps equal their runs alone bit for bit, and a force set before
    the rebuild still acts after it."""
    ws = [W.workload_block(W.NEOHOOKEAN, dims=d, prestretch_seed=80 + i)
          for i, d in enumerate([(3, 3, 3), (6, 5, 4), (3, 4, 3), (5, 6, 4)])]
    p, ids = _pool(ws)
    f = np.zeros((ws[2].n_verts, 3))
    f[:, 0] = 0.5
    p.set_force(ids[2], f)
    p.step(ids)
    p.step(ids)
    p.remove(ids[1])
    p.remove(ids[3])
    used = p.info()["used_bytes"]
    assert p.commit(0) == 0
    assert p.info()["used_bytes"] < used
    for _ in range(2):
        p.step([ids[0], ids[2]])
    ref0 = _alone(ws[0], 4)
    x, v = p.get_state(ids[0])
    assert np.array_equal(x, ref0[-1][0]) and np.array_equal(v, ref0[-1][1])
    s = qnsim.sim_from_workload(ws[2], dense_top=0, level_merge=0)
    x2, v2 = ws[2].x0.copy(), ws[2].v0.copy()
    for _ in range(4):
        x2, v2, _ = s.step(x2, v2, ws[2].h, f_ext=f)
    x, v = p.get_state(ids[2])
    assert np.array_equal(x, x2) and np.array_equal(v, v2)
    s.close()
    p.close()


def test_repack_while_serving_results_equal_alone():
    """A group is rebuilt without its two removed members while two lanes
    keep serving its two live members (the old group steps them until the
    new one, with their states copied over, replaces it); a third
    simulation in another group is served throughout. Every final state
    equals the simulation's run alone with the same number of steps, bit for
    bit, and the removed members' memory returns to the budget."""
    import time
    ws = [W.workload_block(W.NEOHOOKEAN, dims=d, prestretch_seed=90 + i)
          for i, d in enumerate([(4, 3, 3), (7, 6, 5), (3, 4, 4), (6, 7, 5)])]
    other = W.workload_block(W.STVK, dims=(4, 4, 3), prestretch_seed=95)
    p, ids = _pool(ws + [other], group=4)
    p.step(ids)
    p.remove(ids[1])
    p.remove(ids[3])
    used = p.info()["used_bytes"]
    p.serve_start(lanes=2)
    live = [ids[0], ids[2], ids[4]]
    counts = {sid: 1 for sid in live}  # the step before the removals
    stop = threading.Event()
    errors = []

    def client():
        try:
            k = 0
            while not stop.is_set() or k < 12:
                sid = live[k % 3]
                st, _ = p.wait(p.submit(sid), 60.0)
                assert st["iterations_run"] == 10
                counts[sid] += 1
                k += 1
        except Exception as e:  # noqa: BLE001
            errors.append(e)

    th = threading.Thread(target=client)
    th.start()
    time.sleep(0.05)
    before = p.info()["steps_done"]
    assert p.commit(0) == 0
    during = p.info()["steps_done"] - before
    time.sleep(0.05)
    stop.set()
    th.join()
    p.serve_stop()
    assert not errors, errors
    assert p.info()["used_bytes"] < used
    for j, sid in [(0, ids[0]), (2, ids[2])]:
        ref = _alone(ws[j], counts[sid])
        x, v = p.get_state(sid)
        assert np.array_equal(x, ref[-1][0]) and np.array_equal(v, ref[-1][1]), \
            f"member {j} after {counts[sid]} steps: eps vs alone {_eps(x, ref[-1][0], ws[j].rest):.3e}"
    ref = _alone(other, counts[ids[4]])
    x, v = p.get_state(ids[4])
    assert np.array_equal(x, ref[-1][0]) and np.array_equal(v, ref[-1][1])
    print(f"repack while serving: {during} requests completed while the commit ran; "
          f"steps {counts}", flush=True)
    p.close()


def test_pool_graph_replays_equal_eager():
    """Groups replaying their captured step (run flags changing between
    replays) equal groups launching kernel by kernel, bit for bit."""
    ws = W.workload_batch(count=5, seed=4, lo=3, hi=6)
    pg, ig = _pool(ws, step_graph=1)
    pe, ie = _pool(ws, step_graph=0)
    rng = np.random.default_rng(1)
    for k in range(8):
        sub = [j for j in range(5) if rng.uniform() < 0.7] or [0]
        a = pg.step([ig[j] for j in sub])
        b = pe.step([ie[j] for j in sub])
        drop = lambda st: [{k2: v for k2, v in d.items() if k2 != "grad_norm_last"} for d in st]
        assert drop(a) == drop(b), f"round {k}: stats differ"
        for j in range(5):
            xg, vg = pg.get_state(ig[j])
            xe, ve = pe.get_state(ie[j])
            assert np.array_equal(xg, xe) and np.array_equal(vg, ve), f"round {k}, sim {j}"
    pg.close()
    pe.close()


def test_pool_time_step_change():
    """qnsim_pool_set_h: four mixed-material simulations in two groups (one
    member removed from its group first) go to h = 1/60 with A refactored on
    the device; their steps match the oracle at 1/60 and a fresh pool built
    for 1/60 to rounding; a staged simulation is analysed again for 1/60."""
    ws = [W.workload_block([W.NEOHOOKEAN, W.STVK, W.MOONEY_RIVLIN, W.SPLINE][i], dims=(4, 3 + i, 4),
                           prestretch_seed=40 + i) for i in range(4)]
    extra = W.workload_block(W.STVK, dims=(5, 4, 3), prestretch_seed=50)
    p, ids = _pool(ws + [W.workload_block(W.NEOHOOKEAN, dims=(3, 3, 3))], group=3)
    p.remove(ids[4])                               # its group keeps the member's data
    sid = p.add_workloads([extra])[0]              # staged, analysed for 1/30
    h2 = 1.0 / 60.0
    ms = p.set_h(h2)
    assert ms > 0.0
    fresh = qnsim.Pool(h2, 1 << 34, gravity=tuple(ws[0].gravity))
    fids = fresh.add_workloads(ws)
    fresh.commit(3)
    for k in range(4):
        p.step(ids[:4])
        fresh.step(fids)
        for j in range(4):
            x, _ = p.get_state(ids[j])
            xf, _ = fresh.get_state(fids[j])
            assert _eps(x, xf, ws[j].rest) <= 1e-11, f"sim {j} step {k} vs fresh pool"
    w = ws[2]                                      # the Mooney-Rivlin member against the oracle
    m = oracle.build_model(w.rest, w.tets, w.pinned, w.materials, w.tet_mat, h2, w.gravity)
    x, v = w.x0.copy(), w.v0.copy()
    for k in range(4):
        r = oracle.step(m, x, v)
        x, v = r.x, r.v
    xg, _ = p.get_state(ids[2])
    assert _eps(xg, x, w.rest) <= 1e-9
    assert p.commit(0) == 1                        # the staged one, analysed for 1/60
    p.step([sid])
    s = qnsim.sim_from_workload(extra, dense_top=0, level_merge=0, prepare=False)
    s.prepare(h2)
    xs, _, _ = s.step(extra.x0, extra.v0, h2)
    assert np.array_equal(p.get_state(sid)[0], xs)
    s.close()
    p.close()
    fresh.close()


def _alone_from(w, x, v, steps, h=None, **opt):
    """States after each of `steps` steps of w alone from (x, v)."""
    h = w.h if h is None else h
    s = qnsim.sim_from_workload(w, dense_top=0, level_merge=0, prepare=False, **opt)
    s.prepare(h)
    out = []
    for _ in range(steps):
        x, v, _ = s.step(x, v, h)
        out.append((x.copy(), v.copy()))
    s.close()
    return out


def test_pool_tune_element_tiles():
    """qnsim_pool_tune on six mixed-material simulations in two groups.
    Restricted to 512, both groups are rebuilt, the members' states stay as
    they were, and later steps equal each simulation alone with elem_tile 512
    bit for bit; a full tune picks a tile per group, again equal to alone
    with that tile; after a time-step change (A refactored on the device) a
    rebuild to 128 steps as the simulation alone at the new h, to rounding."""
    kinds = [W.NEOHOOKEAN, W.STVK, W.MOONEY_RIVLIN, W.SPLINE, W.COROTATED, W.NEOHOOKEAN]
    ws = [W.workload_block(kinds[i], dims=(4 + i % 3, 3 + i, 4), prestretch_seed=60 + i)
          for i in range(6)]
    p, ids = _pool(ws, group=3)
    p.step(ids)
    before = [p.get_state(i) for i in ids]
    tiles, ms = p.tune(reps=2, candidates=(512,))
    assert tiles == [512, 512]
    for g in range(2):
        assert np.isnan(ms[g][0]) and np.isnan(ms[g][1]) and ms[g][2] > 0.0
    for j, i in enumerate(ids):
        x, v = p.get_state(i)
        assert np.array_equal(x, before[j][0]) and np.array_equal(v, before[j][1])
    ref = [_alone_from(w, *before[j], 3, elem_tile=512) for j, w in enumerate(ws)]
    for k in range(3):
        p.step(ids)
        for j in range(6):
            x, v = p.get_state(ids[j])
            assert np.array_equal(x, ref[j][k][0]), f"tile 512, sim {j} step {k}"
            assert np.array_equal(v, ref[j][k][1])
    start = [p.get_state(i) for i in ids]
    tiles, ms, trials, tms = p.tune(reps=2, trials=True)
    print(f"tune: tiles {tiles}, ms per step {ms}; trials per cycle {trials}, ms {tms}", flush=True)
    assert all(t in (128, 256, 512) for t in tiles)
    assert all(np.isfinite(m).all() and min(m) > 0.0 for m in ms)
    assert all(t in (1, 2, 3) for t in trials)
    assert all(np.isfinite(m).all() and min(m) > 0.0 for m in tms)
    for j, i in enumerate(ids):
        assert np.array_equal(p.get_state(i)[0], start[j][0])
    ref = [_alone_from(w, *start[j], 2, elem_tile=tiles[j // 3]) for j, w in enumerate(ws)]
    for k in range(2):
        p.step(ids)
        for j in range(6):
            x, _ = p.get_state(ids[j])
            assert np.array_equal(x, ref[j][k][0]), f"tile {tiles[j // 3]}, sim {j} step {k}"
    h2 = 1.0 / 60.0
    p.set_h(h2)
    start = [p.get_state(i) for i in ids]
    tiles, _ = p.tune(reps=1, candidates=(128,))
    assert tiles == [128, 128]
    ref = [_alone_from(w, *start[j], 2, h=h2, elem_tile=128) for j, w in enumerate(ws)]
    for k in range(2):
        p.step(ids)
        for j in range(6):
            x, _ = p.get_state(ids[j])
            assert _eps(x, ref[j][k][0], ws[j].rest) <= 1e-11, f"h 1/60, sim {j} step {k}"
    p.close()


def test_pool_external_force():
    """qnsim_pool_set_force: a force on one member of a group of four gives,
    bit for bit, that simulation's steps alone with the same f_ext (full and
    partial batches, a served request); the other members equal their steps
    alone without one; removing the force returns to gravity only.
    qnsim_pool_submit_force: the served step uses the request's force, and
    the next one the simulation's own force (or none) again."""
    ws = [W.workload_block(W.NEOHOOKEAN if i % 2 == 0 else W.STVK, dims=(3 + i, 4, 3),
                           prestretch_seed=70 + i) for i in range(4)]
    p, ids = _pool(ws)
    alone = [qnsim.sim_from_workload(w, dense_top=0, level_merge=0) for w in ws]
    rng = np.random.default_rng(5)
    m = alone[1].masses()
    f = m[:, None] * rng.normal(scale=4.0, size=(ws[1].n_verts, 3))  # about 4 m/s^2 per vertex
    p.set_force(ids[1], f)
    state = [(w.x0.copy(), w.v0.copy()) for w in ws]

    def advance(j, force):
        x, v, _ = alone[j].step(*state[j], ws[j].h, f_ext=force)
        state[j] = (x, v)

    def check(js, tag):
        for j in js:
            x, v = p.get_state(ids[j])
            assert np.array_equal(x, state[j][0]) and np.array_equal(v, state[j][1]), f"{tag}: sim {j}"

    for k in range(2):
        p.step(ids)
        for j in range(4):
            advance(j, f if j == 1 else None)
        check(range(4), f"batched step {k}")
    p.step([ids[1], ids[2]])
    advance(1, f)
    advance(2, None)
    check(range(4), "partial batch")
    p.serve_start(1)
    p.wait(p.submit(ids[1]))
    p.serve_stop()
    advance(1, f)
    check([1], "served request")
    p.set_force(ids[1], None)
    p.step(ids)
    for j in range(4):
        advance(j, None)
    check(range(4), "force removed")
    moved = np.linalg.norm(state[1][0] - ws[1].rest)
    assert moved > 0.0
    # a force for one served step only: in place of the simulation's own
    # force (sim 1), or of none (sim 2); later steps use their own again
    p.set_force(ids[1], f)
    f2 = -2.0 * f
    m2 = alone[2].masses()
    f3 = m2[:, None] * rng.normal(scale=4.0, size=(ws[2].n_verts, 3))
    p.serve_start(2)
    p.wait(p.submit_force(ids[1], f2))
    advance(1, f2)
    p.wait(p.submit_force(ids[2], f3))
    advance(2, f3)
    check([1, 2], "served step with its own force")
    p.wait(p.submit(ids[1]))
    p.wait(p.submit(ids[2]))
    p.serve_stop()
    advance(1, f)
    advance(2, None)
    check([1, 2], "served step after the request's force")
    for s in alone:
        s.close()
    p.close()
