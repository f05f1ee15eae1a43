#!/usr/bin/env python3
"""Throughput of the quasi-Newton / L-BFGS implicit-Euler step on one MI355X.

Workload: a 40 x 40 x 40 grid of 0.025 m cubes split into 384,000 tets
(68,921 vertices), bottom face pinned, released under gravity from a seeded
10 % random affine pre-stretch; three runs with Neo-Hookean, St. Venant-
Kirchhoff and spline materials (E = 1e5 Pa, nu = 0.4, rho = 1000 kg/m^3);
h = 1/30 s, 10 quasi-Newton iterations per step, L-BFGS window m = 5,
backtracking Armijo line search; all arithmetic in FP64.

A "step" is one full implicit-Euler step of the hot path (element passes,
gradient gather, two-loop recursion, prefactored solves, line search) with
the state resident in HBM. `value` is steps per second over the three
material runs (3 * steps / total time). Also reported: tet evaluations per
second, per-kernel HIP-event timings against the HBM roofline, and the FP64
NumPy oracle timed on the host on a bounded sample of the same workload.

Prints one JSON line. Runs on one GPU only.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector (and FP64 matrix) peak
METRIC = "timesteps/s and tet-evals/s at fixed L-BFGS residual; served p50/p99 step latency"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "solve_traffic_block40_neohookean.md")
SOLVE_SOURCES = ["trisolve.hip", "factor.cpp", "upload.cpp", "kernels.hpp", "wave.hpp"]


def solve_traffic(n):
    """HBM bytes of one solve measured with FETCH_SIZE / WRITE_SIZE (scaled by a copy
    kernel) for the 40^3 block, or None when the workload differs or the solve's
    sources changed since the counters were taken."""
    import hashlib
    if n != 40 or not os.path.exists(TRAFFIC_PROFILE):
        return None
    h = hashlib.sha256()
    for f in SOLVE_SOURCES:
        with open(os.path.join(ROOT, "paper_1604_07378_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    fields = {}
    for line in open(TRAFFIC_PROFILE):
        key, _, val = line.partition(":")
        fields[key.strip()] = val.strip()
    if fields.get("solve_source_sha256_16") != h.hexdigest()[:16]:
        return None
    return int(fields["traffic_bytes_per_solve"])


def element_bytes(T, n, nf):
    """Algorithmic HBM bytes of one FP64 line-search element pass.

    Per tet: 4 int32 vertex ids (16 B), Dm^{-1} (72 B), rest volume (8 B);
    per vertex once: x (24 B); per free vertex once: d (24 B), y (24 B) and
    the lumped mass (8 B) for the inertia term.
    """
    return T * (16 + 72 + 8) + n * 24 + nf * (24 + 24 + 8)


def solve_bytes(nnz_exact, nf):
    """Algorithmic HBM bytes of one prefactored solve (3 right-hand sides):
    the factor values read by the forward and by the backward sweep, plus the
    right-hand side read and the solution written (intermediate vectors are
    not algorithmic)."""
    return 2 * 8 * nnz_exact + 2 * 24 * nf


def run_material(kind, args, torch, W, qnsim, extra=None):
    w = W.workload_block(kind, n=args.n)
    t0 = time.time()
    sim = qnsim.sim_from_workload(w, **{**args.overrides, **(extra or {})})
    prep = time.time() - t0
    info = sim.factor_info()
    log(f"[bench] {w.name}: prepared in {prep:.2f}s, nnz(L)={info['nnz_L_exact']}, "
        f"levels={info['n_levels']}")
    x = torch.from_numpy(w.x0.copy()).cuda()
    v = torch.from_numpy(w.v0.copy()).cuda()
    if args.warmup:
        sim.run_device(x, v, w.h, args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = sim.run_device(x, v, w.h, args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log(f"[bench] {w.name}: {args.steps} steps in {dt:.3f}s ({args.steps / dt:.1f} steps/s), "
        f"trials {st['ls_trials']}, iterations {st['iterations_run']}")
    res = dict(material=W.MATERIAL_NAMES[kind], steps=args.steps, seconds=dt,
               steps_per_s=args.steps / dt, ls_trials=st["ls_trials"],
               iterations=st["iterations_run"], exhausted=st["ls_exhausted"],
               element_passes=st["ls_trials"] + args.steps, T=w.n_tets, n=w.n_verts,
               nf=info["n_free"], nnz_L=info["nnz_L_exact"], levels=info["n_levels"],
               prepare_s=prep)
    # per-kernel timings (HIP events on the library's stream)
    reps = 20
    el_ms = sim.time_kernel(qnsim.KERNEL_ELEMENT, reps)
    ga_ms = sim.time_kernel(qnsim.KERNEL_GATHER, reps)
    so_ms = sim.time_kernel(qnsim.KERNEL_SOLVE, reps)
    res["kernel_ms"] = dict(element=el_ms, gather=ga_ms, solve=so_ms)
    res["element_bytes"] = element_bytes(w.n_tets, w.n_verts, info["n_free"])
    res["solve_bytes"] = solve_bytes(info["nnz_L_exact"], info["n_free"])
    res["residual"] = gradient_reduction(sim, x, v, w.h, args.residual_steps)
    sim.close()
    return res


def gradient_reduction(sim, x, v, h, steps):
    """The "fixed L-BFGS residual" of the timed schedule: |grad g(x_final)| /
    |grad g(x_1)| per step (one extra gradient pass per step, untimed), over
    `steps` further steps from the state the timed run left."""
    import numpy as np
    if steps <= 0:
        return None
    sim.set_diagnostics(True)
    red = []
    for _ in range(steps):
        st = sim.step_device(x, v, h)
        red.append(st["grad_norm_last"] / st["grad_norm_first"])
    sim.set_diagnostics(False)
    r = np.array(red)
    return {"steps": steps, "grad_reduction_median": float(np.median(r)),
            "grad_reduction_max": float(r.max())}


def _pool_of(ws, qnsim, budget, group, **opt):
    t0 = time.time()
    p = qnsim.Pool(ws[0].h, budget, gravity=tuple(ws[0].gravity), **opt)
    ids = p.add_workloads(ws)
    t1 = time.time()
    admitted = p.commit(group)
    t2 = time.time()
    return p, ids, admitted, t1 - t0, t2 - t1


def batched_run(args, torch, W, qnsim, precision):
    """Many independent meshes of uneven size in one group: every phase of the
    step is one launch over all of them (one batched step = one step of each)."""
    ws = W.workload_batch(count=args.batch_count, seed=0)
    T = sum(w.n_tets for w in ws)
    p, ids, admitted, t_an, t_up = _pool_of(ws, qnsim, 200 * 10**9, 0, precision=precision)
    assert admitted == len(ws), "batch does not fit the budget"
    log(f"[bench] batch of {len(ws)} meshes ({T} tets): analysis {t_an:.1f}s, upload {t_up:.1f}s, "
        f"{p.info()['used_bytes'] / 1e9:.2f} GB")
    for _ in range(args.warmup):
        p.step(ids)
    tune = None
    if not args.no_tune:
        t_tu = time.perf_counter()
        tiles, tms, trials, trms = p.tune(reps=3, trials=True)
        tune = dict(elem_tile=tiles[0], step_ms={t: m for t, m in zip((128, 256, 512), tms[0])},
                    trials_per_cycle=trials[0],
                    trials_ms={t: m for t, m in zip((1, 2, 3), trms[0])},
                    seconds=time.perf_counter() - t_tu)
        log(f"[bench] tune: element tile {tiles[0]} (ms per batched step "
            + ", ".join(f"{t}: {m:.2f}" for t, m in tune["step_ms"].items())
            + f"), trials per cycle {trials[0]} ("
            + ", ".join(f"{t}: {m:.2f}" for t, m in tune["trials_ms"].items())
            + f"); {tune['seconds']:.1f}s")
        p.step(ids)
    torch.cuda.synchronize()
    evals, trials = 0, 0
    t0 = time.perf_counter()
    for _ in range(args.batch_steps):
        st = p.step(ids)
        for w, s in zip(ws, st):
            evals += w.n_tets * (s["ls_trials"] + 1)
            trials += s["ls_trials"]
    dt = time.perf_counter() - t0
    info = p.info()
    kern = {}
    for name, kid, nbytes in (
            ("element", qnsim.KERNEL_ELEMENT, element_bytes(T, sum(w.n_verts for w in ws), info["n_free"])),
            ("gather", qnsim.KERNEL_GATHER, None),
            ("solve", qnsim.KERNEL_SOLVE, solve_bytes(info["nnz_L"], info["n_free"]))):
        ms = p.time_kernel(0, kid, 10)
        kern[name] = {"ms": ms}
        if nbytes:
            kern[name].update(bytes=nbytes, GBs=nbytes / (ms * 1e-3) / 1e9,
                              frac=nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS)
    log(f"[bench] batch kernels: " + ", ".join(
        f"{k} {v['ms']:.3f} ms" + (f" ({v['GBs']:.0f} GB/s)" if "GBs" in v else "") for k, v in kern.items()))
    res = dict(meshes=len(ws), tets=T, verts=sum(w.n_verts for w in ws), nnz_L=info["nnz_L"],
               kernels=kern, precision="mixed" if precision else "f64", tune=tune,
               batched_steps_per_s=args.batch_steps / dt,
               mesh_steps_per_s=args.batch_steps * len(ws) / dt,
               tet_evals_per_s=evals / dt, ms_per_batched_step=1e3 * dt / args.batch_steps,
               ls_trials_per_mesh_step=trials / (args.batch_steps * len(ws)),
               device_gb=p.info()["used_bytes"] / 1e9, analysis_s=t_an, upload_s=t_up)
    log(f"[bench] batch ({res['precision']}): {res['batched_steps_per_s']:.1f} batched steps/s, "
        f"{res['mesh_steps_per_s']:.0f} mesh-steps/s, {res['tet_evals_per_s'] / 1e9:.2f} G tet-evals/s")
    p.close()
    return res


def served_run(args, torch, W, qnsim):
    """Request loop over a pool of resident simulations with lognormal sizes:
    Poisson step requests for uniformly drawn simulations at fractions of the
    pool's measured batched capacity; latency from submit to completion."""
    import numpy as np
    descs = W.workload_pool(count=args.pool_count, seed=0)
    ws = []
    for i, d in enumerate(descs):
        w = W.workload_block(d["kind"], dims=d["dims"], edge=d["edge"], prestretch_seed=d["seed"],
                             spline_seed=d["seed"], nu=d["nu"])
        ws.append(w)
    T = sum(w.n_tets for w in ws)
    group = args.pool_group or -(-len(ws) // args.pool_lanes)
    p, ids, admitted, t_an, t_up = _pool_of(ws, qnsim, int(args.pool_budget_gb * 10**9), group,
                                            precision=args.pool_precision)
    info = p.info()
    assert admitted == len(ids), "pool does not fit the budget"
    res_ids = ids
    log(f"[bench] pool of {len(ws)} sims ({T} tets), {admitted} admitted into {info['groups']} "
        f"groups, {info['used_bytes'] / 1e9:.2f} GB; analysis {t_an:.1f}s, upload {t_up:.1f}s")
    # capacity: every resident simulation stepped once, groups concurrently
    p.step(res_ids)
    tune = None
    if not args.no_tune:
        # line-search trials per cycle per group (the element tile stays at
        # 256: rebuilding groups of 500 simulations is not worth its time here)
        t_tu = time.perf_counter()
        _, _, trials, trms = p.tune(reps=2, candidates=(256,), trials=True)
        tune = dict(trials_per_cycle=trials, trials_ms=trms, seconds=time.perf_counter() - t_tu)
        log(f"[bench] pool tune: trials per cycle per group {trials} "
            f"({tune['seconds']:.1f}s; ms per group step for 1/2/3: "
            + "; ".join("/".join(f"{m:.0f}" for m in g) for g in trms) + ")")
        p.step(res_ids)
    t0 = time.perf_counter()
    p.step(res_ids)
    cap = len(res_ids) / (time.perf_counter() - t0)
    log(f"[bench] pool capacity (all resident sims, one batched step each): {cap:.0f} steps/s")
    rng = np.random.default_rng(np.random.SeedSequence([0x5E7, 0]))
    p.serve_start(lanes=args.pool_lanes)
    rates = []
    for frac in [float(f) for f in args.pool_load.split(",")]:
        rate = frac * cap
        n = args.pool_requests
        gaps = rng.exponential(1.0 / rate, size=n)
        who = rng.integers(0, len(res_ids), size=n)
        tickets = []
        t_start = time.perf_counter()
        t_next = t_start
        for g, j in zip(gaps, who):
            t_next += g
            while True:
                d = t_next - time.perf_counter()
                if d <= 0:
                    break
                time.sleep(min(d, 0.002) if d > 0.0005 else 0)
            tickets.append(p.submit(res_ids[int(j)]))
        lat = [p.wait(t, 120.0)[1] for t in tickets]
        wall = time.perf_counter() - t_start
        lat = np.array(lat)
        r = dict(load=frac, offered_steps_per_s=rate, requests=n,
                 achieved_steps_per_s=n / wall,
                 p50_ms=float(np.percentile(lat, 50) * 1e3),
                 p99_ms=float(np.percentile(lat, 99) * 1e3))
        rates.append(r)
        log(f"[bench] served load {frac:.2f} ({rate:.0f}/s offered): p50 {r['p50_ms']:.2f} ms, "
            f"p99 {r['p99_ms']:.2f} ms, {r['achieved_steps_per_s']:.0f} steps/s")
    p.serve_stop()
    info = p.info()
    # a time-step change of the whole served pool: A refactored on the device,
    # group by group (the first change also builds each group's plan)
    t0 = time.perf_counter()
    p.set_h(ws[0].h / 2)
    h_first_s = time.perf_counter() - t0
    h_ms = p.set_h(ws[0].h)
    log(f"[bench] pool time-step change: {h_ms:.1f} ms on the device for {info['groups']} groups "
        f"(first change {h_first_s:.1f} s with the plans)")
    p.close()
    return dict(sims=len(ws), admitted=admitted, tets=T, groups=info["groups"], group_size=group,
                precision="mixed" if args.pool_precision else "f64",
                device_gb=info["used_bytes"] / 1e9, budget_gb=args.pool_budget_gb,
                lanes=args.pool_lanes, capacity_steps_per_s=cap, tune=tune, rates=rates,
                batches=info["batches_done"], analysis_s=t_an, upload_s=t_up,
                set_h_device_ms=h_ms, set_h_first_s=h_first_s)


def admission_run(args, torch, W, qnsim, windows=6, per_window=1500, retire_frac=0.12):
    """Admission under a binding budget while serving: the 2,000 pool
    descriptions against a 20 GB budget, so that only part of them is
    resident. Poisson requests for the resident simulations run throughout;
    in each window a client thread retires the oldest resident simulations
    (waits for their requests, removes them) and commits, admitting staged
    simulations as the budget frees (groups whose removed members hold half
    of their memory are rebuilt first), while the main thread keeps
    submitting. Reports per window: resident count, device GB, admitted,
    commit seconds, requests completed during the commit, p50/p99."""
    import threading
    import numpy as np
    descs = W.workload_pool(count=args.pool_count, seed=0)
    ws = [W.workload_block(d["kind"], dims=d["dims"], edge=d["edge"], prestretch_seed=d["seed"],
                           spline_seed=d["seed"], nu=d["nu"]) for d in descs]
    budget = int(args.admission_budget_gb * 10**9)
    p, ids, admitted, t_an, t_up = _pool_of(ws, qnsim, budget, args.admission_group,
                                            precision=args.pool_precision)
    resident = [i for i in ids if p.status(i)[0] == "resident"]
    log(f"[bench] admission: budget {args.admission_budget_gb:.0f} GB, {admitted} of {len(ids)} "
        f"admitted ({p.info()['used_bytes'] / 1e9:.2f} GB; analysis {t_an:.1f}s, upload {t_up:.1f}s)")
    p.step(resident)
    t0 = time.perf_counter()
    p.step(resident)
    cap = len(resident) / (time.perf_counter() - t0)
    rate = args.admission_load * cap
    rng = np.random.default_rng(np.random.SeedSequence([0xAD1, 0]))
    p.serve_start(lanes=args.pool_lanes)
    outstanding = {}                      # sim -> tickets not yet waited for
    lock = threading.Lock()
    out = []
    t_run = time.perf_counter()
    for wnd in range(windows):
        active = list(resident)
        n_ret = max(1, int(retire_frac * len(active)))
        retire, keep = active[:n_ret], active[n_ret:]
        box = {}

        def churn(retire=retire, box=box):
            with lock:
                pend = [t for sid in retire for t in outstanding.pop(sid, [])]
            lats = [p.wait(t, 120.0)[1] for t in pend]
            for sid in retire:
                p.remove(sid)
            done0 = p.info()["steps_done"]
            c0 = time.perf_counter()
            box["admitted"] = p.commit(args.admission_group)
            box["commit_s"] = time.perf_counter() - c0
            box["during"] = p.info()["steps_done"] - done0
            box["lat"] = lats

        th = threading.Thread(target=churn)
        started = False
        tickets = []
        t_start = time.perf_counter()
        t_next = t_start
        who = rng.integers(0, len(keep), size=per_window)
        for k, g in enumerate(rng.exponential(1.0 / rate, size=per_window)):
            if k == per_window // 4 and not started:
                th.start()
                started = True
            t_next += g
            while True:
                d = t_next - time.perf_counter()
                if d <= 0:
                    break
                time.sleep(min(d, 0.002) if d > 0.0005 else 0)
            sid = keep[int(who[k])]
            t = p.submit(sid)
            with lock:
                outstanding.setdefault(sid, []).append(t)
            tickets.append((sid, t))
        th.join()
        lat = list(box["lat"])
        for sid, t in tickets:
            with lock:
                mine = t in outstanding.get(sid, [])
                if mine:
                    outstanding[sid].remove(t)
            if mine:
                lat.append(p.wait(t, 120.0)[1])
        lat = np.array(lat)
        resident = [i for i in ids if p.status(i)[0] == "resident"]
        info = p.info()
        r = dict(window=wnd, t_s=time.perf_counter() - t_run, resident=len(resident),
                 staged=info["sims_staged"], device_gb=info["used_bytes"] / 1e9,
                 retired=len(retire), admitted=box["admitted"], commit_s=box["commit_s"],
                 steps_during_commit=box["during"], requests=int(lat.size),
                 p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3))
        out.append(r)
        log(f"[bench] admission window {wnd}: resident {r['resident']} ({r['device_gb']:.2f} GB), "
            f"retired {r['retired']}, admitted {r['admitted']} in {r['commit_s']:.2f}s "
            f"({r['steps_during_commit']} steps served meanwhile), p50 {r['p50_ms']:.1f} ms, "
            f"p99 {r['p99_ms']:.1f} ms")
    p.serve_stop()
    p.close()
    return dict(sims=len(ws), budget_gb=args.admission_budget_gb, initial_admitted=admitted,
                group_size=args.admission_group, offered_steps_per_s=rate,
                capacity_steps_per_s=cap, windows=out)


def small_runs(args, torch, W, qnsim):
    """Latency-bound small meshes: the 540-tet cantilever (FP64, with and
    without the captured step graph) and the mixed-stiffness cantilever in
    mixed precision; steps/s and the per-step latency."""
    out = []
    cases = [("cantilever-neohookean-f64", W.workload_cantilever(0), dict(step_graph=1)),
             ("cantilever-neohookean-f64-nograph", W.workload_cantilever(0), dict(step_graph=0)),
             ("cantilever-logE-mixed", W.workload_mixed_cantilever(0),
              dict(step_graph=1, precision=qnsim.QNSIM_MIXED))]
    for name, w, opt in cases:
        sim = qnsim.sim_from_workload(w, **opt)
        x = torch.from_numpy(w.x0.copy()).cuda()
        v = torch.from_numpy(w.v0.copy()).cuda()
        sim.run_device(x, v, w.h, 10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = sim.run_device(x, v, w.h, args.small_steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out.append(dict(case=name, tets=w.n_tets, steps=args.small_steps,
                        steps_per_s=args.small_steps / dt, ms_per_step=1e3 * dt / args.small_steps,
                        ls_trials_per_step=st["ls_trials"] / args.small_steps))
        log(f"[bench] {name}: {args.small_steps / dt:.0f} steps/s ({1e3 * dt / args.small_steps:.3f} ms/step)")
        sim.close()
    return out


def relative_error_run(args, torch, W, qnsim, steps=100, k_star=300):
    """Eq. RelativeError (section 5) on the 540-tet Neo-Hookean cantilever:
    per step, (g(x_K) - g*) / (g(x_1) - g*) after the K = 10 iterations of the
    timed schedule, with g* from k_star iterations of the same method from the
    same state (converged: the relative gradient falls below 1e-9), plus the
    per-step gradient reduction |grad g(x_K)| / |grad g(x_1)|. Steps follow the
    10-iteration trajectory from rest."""
    import numpy as np
    w = W.workload_cantilever(0)
    run = qnsim.sim_from_workload(w)
    ref = qnsim.sim_from_workload(w, iterations=k_star)
    run.set_diagnostics(True)
    ref.set_diagnostics(True)
    x = torch.from_numpy(w.x0.copy()).cuda()
    v = torch.from_numpy(w.v0.copy()).cuda()
    xs, vs = torch.empty_like(x), torch.empty_like(v)
    rel, red, red_star = [], [], []
    for _ in range(steps):
        st_ref = ref.step_device(x, v, w.h, x_out=xs, v_out=vs)
        st = run.step_device(x, v, w.h)                # in place: the trajectory
        g_star = st_ref["g_last"]
        den = st["g_first"] - g_star
        rel.append((st["g_last"] - g_star) / den if den > 0 else 0.0)
        red.append(st["grad_norm_last"] / st["grad_norm_first"])
        red_star.append(st_ref["grad_norm_last"] / st_ref["grad_norm_first"])
    run.close()
    ref.close()
    rel, red = np.array(rel), np.array(red)
    out = {"workload": "cantilever 10x3x3 cubes (540 tets), Neo-Hookean, FP64, 100 steps from rest",
           "iterations": 10, "g_star_iterations": k_star,
           "relative_error_median": float(np.median(rel)), "relative_error_max": float(rel.max()),
           "grad_reduction_median": float(np.median(red)), "grad_reduction_max": float(red.max()),
           "g_star_grad_reduction_max": float(max(red_star))}
    log(f"[bench] relative error (Eq. RelativeError) on the cantilever: median "
        f"{out['relative_error_median']:.2e}, max {out['relative_error_max']:.2e}; gradient "
        f"reduction median {out['grad_reduction_median']:.2e}")
    return out


def mixed_error_run(args, torch, W, qnsim, steps=300):
    """Mixed precision on the mixed-stiffness cantilever (E log-uniform in
    [1e4, 1e7] Pa): per-step position error of the mixed path against the
    FP64 GPU path (which the parity tests hold to the FP64 oracle at 1e-9),
    both stepping from the FP64 trajectory's state, over `steps` steps; and the
    free-running separation of the two trajectories."""
    import numpy as np
    w = W.workload_mixed_cantilever(0)
    f64 = qnsim.sim_from_workload(w)
    mix = qnsim.sim_from_workload(w, precision=qnsim.QNSIM_MIXED)
    rest = torch.from_numpy(np.ascontiguousarray(w.rest, dtype=np.float64)).cuda()
    x = torch.from_numpy(w.x0.copy()).cuda()
    v = torch.from_numpy(w.v0.copy()).cuda()
    xf, vf = x.clone(), v.clone()          # free-running mixed trajectory
    xm, vm = torch.empty_like(x), torch.empty_like(v)
    per_step, free = [], {}
    flips = 0          # steps whose line searches took other decisions than FP64's
    for k in range(steps):
        sm = mix.step_device(x, v, w.h, x_out=xm, v_out=vm)
        sf = f64.step_device(x, v, w.h)                   # in place: the FP64 trajectory
        flips += int(sm["ls_trials"] != sf["ls_trials"] or sm["iterations_run"] != sf["iterations_run"])
        mix.step_device(xf, vf, w.h, stats=False)
        den = max(float(torch.linalg.norm(x - rest)), 1e-300)
        per_step.append(float(torch.linalg.norm(xm - x)) / den)
        if k + 1 in (10, 60, steps):
            free[k + 1] = float(torch.linalg.norm(xf - x)) / den
    f64.close()
    mix.close()
    e = np.array(per_step)
    out = dict(workload="cantilever 10x3x3 cubes (540 tets), Neo-Hookean, E log-uniform in [1e4, 1e7] Pa",
               steps=steps, reference="FP64 GPU path from the same state",
               per_step_error_max=float(e.max()), per_step_error_median=float(np.median(e)),
               free_running_error={str(k): v for k, v in free.items()}, tolerance=1e-4,
               steps_with_other_line_search=flips)
    log(f"[bench] mixed precision error over {steps} steps (vs FP64 GPU path, same state): "
        f"max {e.max():.2e}, median {np.median(e):.2e}; {flips} steps with other line-search "
        f"decisions; free-running "
        + ", ".join(f"step {k} {v:.1e}" for k, v in free.items()))
    return out


def convergence_run(args, torch, W, qnsim):
    """Relative error (g(x_k) - g*)/(g(x_0) - g*) of one frame of the Neo-Hookean
    block after K iterations for the plain PD direction (history 0), the
    Chebyshev direction (S = 10, rho estimated from a plain-PD run on the same
    frame) and L-BFGS with m = 2 and 5; g* from 200 L-BFGS iterations (section 5,
    convergence comparison, on the synthetic block)."""
    import numpy as np
    w = W.workload_block(W.NEOHOOKEAN, n=args.n)
    x0 = torch.from_numpy(w.x0.copy()).cuda()
    v0 = torch.from_numpy(w.v0.copy()).cuda()

    def frame(K, **opt):
        sim = qnsim.sim_from_workload(w, iterations=K, **opt)
        x, v = x0.clone(), v0.clone()
        st = sim.step_device(x, v, w.h)
        torch.cuda.synchronize()
        sim.close()
        return st, x.cpu().numpy()

    ref, _ = frame(200, history=5)
    gstar = ref["g_last"]
    pts = [frame(K, history=0)[1] for K in (38, 39, 40)]
    rho = float(np.linalg.norm(pts[2] - pts[1]) / np.linalg.norm(pts[1] - pts[0]))
    rho = min(max(rho, 0.05), 0.999)
    out = {"rho_estimate": rho, "g_star_iterations": 200, "relative_error": {}}
    methods = {"pd": dict(history=0),
               "chebyshev": dict(history=0, direction=qnsim.DIR_CHEBYSHEV, cheb_delay=10,
                                 cheb_rho=rho),
               "lbfgs_m2": dict(history=2), "lbfgs_m5": dict(history=5)}
    for name, opt in methods.items():
        errs = {}
        for K in (10, 20, 40):
            st, _ = frame(K, **opt)
            errs[str(K)] = (st["g_last"] - gstar) / (st["g_first"] - gstar)
        out["relative_error"][name] = errs
    log("[bench] convergence (relative error after 10/20/40 iterations): " + "; ".join(
        f"{k} " + "/".join(f"{v:.1e}" for v in e.values()) for k, e in out["relative_error"].items()))
    return out


def refactor_run(args, torch, W, qnsim):
    """Numeric refactorisation of A = M/h^2 + sum V k G^T G for a new time step
    on the device (the Neo-Hookean block, default solve schedule): device time
    per refactorisation once the plan exists, against the host's analysis and
    factorisation of the same matrix at prepare."""
    import time
    w = W.workload_block(W.NEOHOOKEAN, n=args.n)
    s = qnsim.sim_from_workload(w)
    info = s.factor_info()
    t0 = time.perf_counter()
    s.refactor(w.h / 2)
    first_wall = time.perf_counter() - t0
    ms = [s.refactor(w.h if k % 2 == 0 else w.h / 2) for k in range(6)]
    s.refactor(w.h)
    s.close()
    # prepare with the numeric factorisation on the device (host: ordering
    # and symbolic analysis only)
    s2 = qnsim.sim_from_workload(w, device_factor=1)
    dev_prep = s2.factor_info()["prepare_seconds"]
    s2.close()
    avg = sum(ms) / len(ms)
    flops = info["factor_flops"]
    out = {"workload": f"block {args.n}^3 Neo-Hookean, h = 1/30 <-> 1/60 s, default schedule "
                       f"(dense top {info['dense_top_cols']} columns)",
           "device_ms": avg, "first_call_wall_s": first_wall,
           "host_prepare_s": info["prepare_seconds"],
           "device_factor_prepare_s": dev_prep, "factor_flops_host_count": flops,
           "achieved_tflops": flops / (avg * 1e-3) / 1e12, "bound": "fp64 valu",
           "peak_tflops": FP64_PEAK_TFLOPS,
           "frac": flops / (avg * 1e-3) / 1e12 / FP64_PEAK_TFLOPS}
    log(f"[bench] refactor on the device: {avg:.2f} ms ({out['achieved_tflops']:.2f} TFLOP/s); "
        f"host prepare {info['prepare_seconds']:.2f} s, with the device factorisation "
        f"{dev_prep:.2f} s")
    return out


def tune_run(args, torch, W, qnsim):
    """qnsim_tune on the Neo-Hookean block: the four solve schedules, then the
    three element tiles with the fastest schedule, then 1-3 line-search trials
    per cycle (informational: the headline runs keep the default options)."""
    w = W.workload_block(W.NEOHOOKEAN, n=args.n)
    s = qnsim.sim_from_workload(w, **args.overrides)
    import numpy as np
    x = torch.from_numpy(np.ascontiguousarray(w.x0, dtype=np.float64)).cuda()
    v = torch.from_numpy(np.ascontiguousarray(w.v0, dtype=np.float64)).cuda()
    t0 = time.perf_counter()
    info = s.tune(x, v, w.h, reps=5)
    info["seconds"] = time.perf_counter() - t0
    s.close()
    names = ["levels", "subtrees", "merged", "merged+top"]
    log(f"[bench] tune block {args.n}^3: schedules " + ", ".join(
        f"{n} {m:.3f}" for n, m in zip(names, info["schedule_ms"])) + " ms/step; tiles " + ", ".join(
        f"{t} {m:.3f}" for t, m in zip((128, 256, 512), info["tile_ms"])) +
        f" ms/step; trials per cycle " + ", ".join(
        f"{t} {m:.3f}" for t, m in zip((1, 2, 3), info["trials_ms"])) +
        f" ms/step; kept dense_top {info['dense_top']}, subtree_cap {info['subtree_cap']}, "
        f"level_merge {info['level_merge']}, elem_tile {info['elem_tile']}, "
        f"trials_per_cycle {info['trials_per_cycle']} ({info['seconds']:.1f}s)")
    info["schedules"] = names
    return info


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _thread_pools():
    """The BLAS / OpenMP thread pools NumPy and SciPy run on, and the
    environment variables that size them."""
    pools = []
    try:
        from threadpoolctl import threadpool_info
        for p in threadpool_info():
            pools.append({"api": p.get("user_api"), "library": p.get("internal_api"),
                          "threads": p.get("num_threads")})
    except Exception:
        pass
    env = {k: os.environ[k] for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS",
                                      "MKL_NUM_THREADS", "BLIS_NUM_THREADS") if k in os.environ}
    return pools, env


def cpu_baseline(args, W):
    """The FP64 oracle on a bounded sample: a few steps of the Neo-Hookean block."""
    import numpy as np  # noqa: F401
    import oracle
    pools, env = _thread_pools()
    cores = max([p["threads"] or 1 for p in pools] + [1]) if pools else (os.cpu_count() or 1)
    w = W.workload_block(W.NEOHOOKEAN, n=args.n)
    t0 = time.time()
    m = oracle.build_model(w.rest, w.tets, w.pinned, w.materials, w.tet_mat, w.h, w.gravity)
    build = time.time() - t0
    t0 = time.perf_counter()
    steps = args.cpu_sample_steps
    x, v = w.x0, w.v0
    for _ in range(steps):
        r = oracle.step(m, x, v)
        x, v = r.x, r.v
    dt = time.perf_counter() - t0
    # the same oracle on one thread (BLAS/LAPACK pools limited to 1), one step
    one = None
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            oracle.step(m, w.x0, w.v0)
            one = 1.0 / (time.perf_counter() - t0)
    except Exception:
        one = None
    log(f"[bench] oracle: build {build:.1f}s, {steps} step(s) in {dt:.1f}s"
        + (f"; one thread {1.0 / one:.1f}s per step" if one else ""))
    return {"value": steps / dt, "unit": "timesteps/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{steps} step(s) of the Neo-Hookean {args.n}^3 block ({w.n_tets:,} tets) after an "
                      f"untimed {build:.1f}s model build and banded Cholesky factorisation",
            "seconds": dt, "value_one_thread": one, "cpu": _cpu_model(),
            "os_cpu_count": os.cpu_count(), "thread_pools": pools, "thread_env": env}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=40, help="cubes per axis of the block")
    ap.add_argument("--materials", default="neohookean,stvk,spline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-steps", type=int, default=5,
                    help="oracle steps of the CPU baseline (about 5-6 s each on 16 cores)")
    ap.add_argument("--residual-steps", type=int, default=3,
                    help="untimed steps per block run that report the gradient reduction")
    ap.add_argument("--no-convergence", action="store_true",
                    help="skip the convergence comparison of the direction methods")
    ap.add_argument("--no-refactor", action="store_true",
                    help="skip the device refactorisation measurement")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuners (batched run: default element tile)")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the extra mixed-precision Neo-Hookean run")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="run one plain device copy of this many MB first (a reference kernel of "
                         "known traffic for hardware-counter runs)")
    ap.add_argument("--small-steps", type=int, default=100,
                    help="steps of the small-mesh latency runs (0: skip them)")
    ap.add_argument("--batch-count", type=int, default=256,
                    help="meshes of the batched run (0: skip it)")
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--pool-count", type=int, default=2000,
                    help="simulations of the served run, the first of the 2,000-simulation "
                         "pool's descriptions (0: skip it)")
    ap.add_argument("--pool-group", type=int, default=0,
                    help="simulations per group (0: one group per lane)")
    ap.add_argument("--pool-lanes", type=int, default=4)
    ap.add_argument("--pool-budget-gb", type=float, default=200.0)
    ap.add_argument("--pool-requests", type=int, default=10000, help="requests per load level")
    ap.add_argument("--pool-load", default="0.25,0.5,0.8,1.2",
                    help="offered loads as fractions of the measured capacity")
    ap.add_argument("--pool-precision", type=int, default=1, help="1: mixed, 0: FP64")
    ap.add_argument("--admission-budget-gb", type=float, default=20.0,
                    help="budget of the admission run (0: skip it)")
    ap.add_argument("--admission-group", type=int, default=64,
                    help="simulations per group in the admission run")
    ap.add_argument("--admission-load", type=float, default=0.5,
                    help="offered load of the admission run, fraction of its capacity")
    ap.add_argument("--set", action="append", default=[], metavar="OPTION=INT",
                    help="override an integer solver option (e.g. level_merge=0, dense_top=0)")
    args = ap.parse_args()
    args.overrides = {}
    for item in args.set:
        key, _, val = item.partition("=")
        args.overrides[key.strip()] = int(val)
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(independent simulations would be sharded by simulation, one process per GPU); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    from paper_1604_07378_amd import qnsim

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_calibration_mb > 0:
        n = args.copy_calibration_mb * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {args.copy_calibration_mb} MB done")
        del src, dst
    names = {v: k for k, v in W.MATERIAL_NAMES.items()}
    kinds = [names[s] for s in args.materials.split(",")]
    runs = [run_material(k, args, torch, W, qnsim) for k in kinds]
    mixed = None
    if not args.no_mixed and W.NEOHOOKEAN in kinds:
        # informational: the mixed path (FP32 stresses) on the same workload
        mixed = run_material(W.NEOHOOKEAN, args, torch, W, qnsim, {"precision": qnsim.QNSIM_MIXED})

    small = small_runs(args, torch, W, qnsim) if args.small_steps > 0 else []
    relerr = relative_error_run(args, torch, W, qnsim) if args.small_steps > 0 else None
    mixed_err = mixed_error_run(args, torch, W, qnsim) if not args.no_mixed else None
    conv = convergence_run(args, torch, W, qnsim) if not args.no_convergence else None
    batched = []
    if args.batch_count > 0:
        batched = [batched_run(args, torch, W, qnsim, 0), batched_run(args, torch, W, qnsim, 1)]
    served = served_run(args, torch, W, qnsim) if args.pool_count > 0 else None
    admission = (admission_run(args, torch, W, qnsim)
                 if args.pool_count > 0 and args.admission_budget_gb > 0 else None)
    refac = refactor_run(args, torch, W, qnsim) if not args.no_refactor else None
    tuned = tune_run(args, torch, W, qnsim) if not args.no_tune else None

    total_steps = sum(r["steps"] for r in runs)
    total_s = sum(r["seconds"] for r in runs)
    tet_evals = sum(r["T"] * r["element_passes"] for r in runs)
    value = total_steps / total_s

    # dominant kernel: largest share of step time among the timed kernels
    nh = runs[0]
    per_step = {
        "element": nh["kernel_ms"]["element"] * nh["element_passes"] / nh["steps"],
        "gather": nh["kernel_ms"]["gather"] * nh["iterations"] / nh["steps"],
        "solve": nh["kernel_ms"]["solve"] * nh["iterations"] / nh["steps"],
    }
    dom = max(per_step, key=per_step.get)
    if dom == "solve":
        bytes_, ms = nh["solve_bytes"], nh["kernel_ms"]["solve"]
    else:
        bytes_, ms = nh["element_bytes"], nh["kernel_ms"]["element"]
        dom = "element"
    achieved = bytes_ / (ms * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "timesteps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * total_s / total_steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"block {args.n}^3 cubes x 6 tets ({nh['T']} tets, {nh['n']} verts), "
                        f"materials {args.materials}, FP64, h=1/30 s, 10 iterations, m=5",
            "tets": nh["T"], "verts": nh["n"], "free_verts": nh["nf"],
            "materials": args.materials.split(","),
            **({"options": args.overrides} if args.overrides else {}),
        },
        "tet_evals_per_s": tet_evals / total_s,
        "runs": [{k: r[k] for k in ("material", "steps_per_s", "ls_trials", "iterations",
                                    "exhausted", "kernel_ms", "nnz_L", "levels", "prepare_s",
                                    "residual")}
                 for r in runs],
        "step_time_share_ms": per_step,
        **({"mixed_precision_run": {k: mixed[k] for k in ("material", "steps_per_s", "ls_trials",
                                                         "iterations", "kernel_ms")}}
           if mixed else {}),
        **({"small_meshes": small} if small else {}),
        **({"relative_error": relerr} if relerr else {}),
        **({"mixed_precision_error": mixed_err} if mixed_err else {}),
        **({"convergence": conv} if conv else {}),
        **({"batched": batched} if batched else {}),
        **({"served": served} if served else {}),
        **({"admission": admission} if admission else {}),
        **({"refactor": refac} if refac else {}),
        **({"tune": tuned} if tuned else {}),
        "roofline": {
            "bound": "hbm",
            "kernel": dom,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": solve_traffic(args.n) if dom == "solve" else None,
            "algorithmic_bytes_per_launch": bytes_,
            "avg_launch_ms": ms,
        },
        "kernels": {
            "element": {"ms": nh["kernel_ms"]["element"], "bytes": nh["element_bytes"],
                        "GBs": nh["element_bytes"] / (nh["kernel_ms"]["element"] * 1e-3) / 1e9},
            "solve": {"ms": nh["kernel_ms"]["solve"], "bytes": nh["solve_bytes"],
                      "GBs": nh["solve_bytes"] / (nh["kernel_ms"]["solve"] * 1e-3) / 1e9},
            "gather_ms": nh["kernel_ms"]["gather"],
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args, W)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
