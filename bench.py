"""Benchmark: exact sparse permanents on one MI355X (gfx950).

Workload: 17 cubic graphs on 60 vertices (the truncated icosahedron and 16 seeded random
3-regular graphs of girth >= 5), expanded with expansion (2) down to jobs of order 20.

A step is the device part of the path over the whole batch with the job tables resident in
HBM: KKLLL keys, non-increasing-estimate queue, persistent R-NW kernels, exact recombination.
`value` is the R-NW subset-terms of the batch divided by the step time. Reported beside it:
per(A) wall time from host CSR to exact integers (expansion included, PCIe-inclusive), the
plain one-launch-per-job comparator in expansion order, other queue orders, the roofline of
the dominant kernel from HIP events (HBM traffic from the committed counter summary when it
matches the kernel source), the CPU oracle timed on a bounded sample, and a serving run
(continuous batching of mixed requests: capacity, then Poisson arrivals with p50/p99 latency).

    python bench.py [--steps K] [--warmup W] [--m-cut 20] [--no-cpu-baseline] [--no-plain]
                    [--no-serving] [--no-large] [--large-only c100|all] [--profile-split]
                    [--copy-probe]
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Full-rate 32-bit VALU lane operations per second: 256 CUs x 128 lanes per clock x 2.4 GHz,
# the same issue rate as the 157.3 TFLOP/s FP32 vector peak (an FMA counts two flops).
ALU_PEAK = 256 * 128 * 2.4e9


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def traffic_from_profile():
    """HBM bytes per launch of the dominant kernel from the committed counter summary, if it was
    taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "rnw_persistent_n60_counters.txt")
    src = os.path.join(ROOT, "paper_1112_6072_amd", "csrc", "kernels.hip")
    if not os.path.exists(path):
        return None
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    vals = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernels_hip_sha256_16") != digest:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_threads() -> int:
    """Host threads of the oracle: the job's CPU share (OMP_NUM_THREADS, set to the box's share),
    else every core."""
    n = os.cpu_count() or 1
    try:
        share = int(os.environ.get("OMP_NUM_THREADS", "0"))
    except ValueError:
        share = 0
    return max(1, min(n, share) if share > 0 else n)


def cpu_oracle_batch(mats, terms):
    """The oracle's C Algorithm H_per (oracle/hper_c.c) over the whole benchmark batch on the
    host's cores: its per(A) wall time, and the batch's R-NW subset-terms divided by it (the
    rate at which the oracle finishes the same work, in the metric's unit)."""
    from oracle import native
    threads = cpu_threads()
    native.hper_batch(mats[:1], threads=threads)   # load and warm the library
    t0 = time.time()
    vals = native.hper_batch(mats, threads=threads)
    dt = time.time() - t0
    return vals, {"value": terms / dt, "unit": "subset-terms/s", "cores": threads, "kind": "oracle",
                  "nproc": os.cpu_count(), "per_a_wall_ms_batch": dt * 1e3,
                  "sample": f"the whole benchmark batch (17 cubic graphs on 60 vertices) by the C H_per "
                            f"oracle on {threads} threads: per(A) of every problem in {dt:.2f} s; value = "
                            f"the batch's {terms:.3e} R-NW subset-terms of order-20 jobs / that time"}


def cpu_baseline(m_cut: int, budget_s: float = 20.0):
    """The C Ryser oracle on the first jobs (expansion order) of the truncated icosahedron."""
    import workloads as W
    from oracle import expand_leaves, native
    threads = cpu_threads()
    A = W.adjacency_matrix(W.truncated_icosahedron())
    leaves = expand_leaves(A, m_cut, limit=512)
    # size the sample from a one-job probe so the run stays near the budget
    t0 = time.time()
    native.ryser_batch(leaves[:1], threads=1)
    one = max(time.time() - t0, 1e-3)
    k = int(max(threads, min(len(leaves), budget_s * threads / one)))
    k = max(1, min(k, len(leaves)))
    sample = leaves[:k]
    t0 = time.time()
    native.ryser_batch(sample, threads=threads)
    dt = time.time() - t0
    terms = sum(1 << (len(x) - 1) for x in sample)
    return {"value": terms / dt, "unit": "subset-terms/s", "cores": threads, "kind": "oracle",
            "sample": f"plain C Ryser (oracle/ryser_c.c) on the first {k} order-{m_cut} jobs "
                      f"(expansion order) of the truncated icosahedron; {dt:.2f} s wall; terms "
                      f"counted as 2^(m-1) per job like the GPU path"}


def serving_leg(hp, W, n_requests: int = 48, seed: int = 7, n_lo: int = 30, n_hi: int = 100,
                limit_ms: int = 1000):
    """Continuous batching under a Poisson stream of mixed requests (3-regular, 4-regular and
    small-integer sparse matrices, n uniform in [n_lo, n_hi]). First the whole stream at once
    (capacity = served requests / makespan), then Poisson arrivals at half that rate; latencies
    are the library's submit-to-completion times of the served requests. Requests whose
    estimated work exceeds limit_ms are refused (HPERM_E_TOOBIG); integer requests whose
    expansion leaves the exact paths' entry range are served by residues (the device path modulo
    primes, CRT), counted apart, and refused (HPERM_E_RANGE) only beyond that path's reach."""
    import numpy as np
    reqs = [A for _, A in W.serving_requests(n_requests, seed, n_lo, n_hi)]
    ctx = hp.Context({"m_cut": 20, "trials": 32, "host_threads": 4, "serve_limit_ms": limit_ms})
    try:
        ctx.serve_start(4 * n_requests, 4 << 30)
        def collect(tickets):
            out = []
            for t in tickets:
                try:
                    out.append(ctx.wait(t, 600.0))
                except hp.HpermError as e:   # refused: beyond the work limit or the entry range
                    out.append((None, {"t_total_s": float("nan"), "error": e.status}))
            return out

        t0 = time.perf_counter()
        tickets = [ctx.submit(A) for A in reqs]
        burst = collect(tickets)
        makespan = time.perf_counter() - t0
        served = sum(v is not None for v, _ in burst)
        capacity = served / makespan
        rate = 0.5 * n_requests / makespan
        arrivals = W.poisson_arrivals(n_requests, rate, seed + 1)
        t0 = time.perf_counter()
        tickets = []
        for A, ta in zip(reqs, arrivals):
            delay = ta - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            tickets.append(ctx.submit(A))
        paced = collect(tickets)
        wall = time.perf_counter() - t0
        ctx.serve_stop()
    finally:
        ctx.close()
    lat = np.array([st["t_total_s"] for v, st in paced if v is not None]) * 1e3
    lat_b = np.array([st["t_total_s"] for v, st in burst if v is not None]) * 1e3
    errs = [st.get("error") for v, st in burst if v is None]
    same = [v for v, _ in burst] == [v for v, _ in paced]
    served_n = [A.shape[0] for A, (v, _) in zip(reqs, burst) if v is not None]
    by_res = [A.shape[0] for A, (v, st) in zip(reqs, burst) if v is not None and st.get("arith_mask") == 1 << 3]
    return {"requests": n_requests, "n_range": [n_lo, n_hi], "work_limit_ms": limit_ms,
            "served": served, "served_by_residues": len(by_res), "served_by_residues_n": sorted(by_res),
            "refused_work_limit": errs.count(-9), "refused_entry_range": errs.count(-2),
            "failed_other": len(errs) - errs.count(-9) - errs.count(-2),
            "served_n_max": max(served_n) if served_n else None,
            "mix": "1/3 each: 3-regular 0-1, 4-regular 0-1, 3-permutation union with values 1..4",
            "capacity_served_per_s": capacity,
            "poisson_rate_per_s": rate, "requests_per_s": n_requests / wall,
            "p50_ms": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_ms": float(np.percentile(lat, 99)) if lat.size else None,
            "burst_p50_ms": float(np.percentile(lat_b, 50)) if lat_b.size else None,
            "burst_p99_ms": float(np.percentile(lat_b, 99)) if lat_b.size else None,
            "burst_and_paced_results_identical": same}


def uneven_orders(hp, W, ctx, n_jobs: int = 600, seed: int = 11):
    """Queue orders on uneven jobs: n_jobs job-like matrices (unions of 3 to 6 random
    permutations, values 1..4) of orders uniform in 16..30, in one persistent launch per
    order bucket; R-NW milliseconds per order (the results are checked equal)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    mats = [W.permutation_union_matrix(int(rng.integers(16, 31)), int(rng.integers(3, 7)),
                                       int(rng.integers(0, 2 ** 31 - 1)), 1, 4) for _ in range(n_jobs)]
    J = ctx.jobs_from_dense(mats)
    keys = ctx.estimate(J, 32, 1)
    out, ref = {}, None
    for order in ("estimate", "exact_cost", "natural", "random"):
        tot, _, _ = ctx.run(J, order, True)
        ref = tot if ref is None else ref
        assert tot == ref
        out[order + "_ms"] = sum(L["ms"] for L in ctx.last_launches())
    d = J.describe()
    out["jobs"] = n_jobs
    out["subset_terms"] = int(d["terms"].astype(np.float64).sum())
    out["schedule_study"] = schedule_study(hp, ctx, J, keys)
    return out


def expansion_uneven(hp, W, ctx, mats, want, restore_m_cut, plain=True, m_cut=12, m_cap=24, s_leaf=3):
    """Queue orders on jobs of uneven order as the expansion produces them: the benchmark's 17
    graphs expanded with H_per's stop rule at s_leaf = 3 (a node whose lines all hold three or
    more nonzeros becomes a job once its order is at most m_cap; others are split down to
    m_cut), which leaves jobs of orders m_cut..m_cap in two rings. Persistent R-NW milliseconds
    in the paper's three orders (natural, exact cost, the estimate) and random; totals checked
    against the oracle's values; the scheduling study on the same jobs."""
    import numpy as np
    ctx.set_opts(m_cut=m_cut, m_cap=m_cap, s_leaf=s_leaf, split_order=0)
    try:
        J = ctx.expand(mats)
        keys = ctx.estimate(J, 32, 1)
        out = {"m_cut": m_cut, "m_cap": m_cap, "s_leaf": s_leaf}
        for order in ("estimate", "exact_cost", "natural", "random"):
            ms = []
            for _ in range(3):
                tot, _, _ = ctx.run(J, order, True)
                assert want is None or tot == want
                ms.append(sum(L["ms"] for L in ctx.last_launches()))
            out[order + "_ms"] = sorted(ms)[1]
        if plain:   # one launch per job in expansion order: the unbatched comparator
            tot, _, _ = ctx.run(J, "natural", False)
            assert want is None or tot == want
            out["plain_one_launch_per_job_ms"] = ctx.last_launches()[0]["ms"]
            out["lpt_vs_plain"] = out["plain_one_launch_per_job_ms"] / out["estimate_ms"]
        d = J.describe()
        vals, cnt = np.unique(d["m"], return_counts=True)
        out["jobs"] = int(d["m"].size)
        out["jobs_by_order"] = {int(v): int(c) for v, c in zip(vals, cnt)}
        out["jobs_by_ring"] = {name: int((d["arith"] == k).sum()) for k, name in ((1, "mod 2^64"), (2, "mod 2^128"), (3, "residues"))}
        out["subset_terms"] = int(d["terms"].astype(np.float64).sum())
        out["schedule_study"] = schedule_study(hp, ctx, J, keys)
    finally:   # the benchmark context's options (library defaults for m_cap and s_leaf)
        ctx.set_opts(m_cut=restore_m_cut, m_cap=36, s_leaf=5, split_order=0)
    return out


def autotune_leg(hp, W, ctx, jobs, trials, want):
    """The autotuner on the benchmark's jobs and on the 600 uneven jobs: its table, and the R-NW
    milliseconds of the whole persistent run (estimate order, median of 3) with the defaults and
    with the tuned lane chunks and grids (the values must not change)."""
    import numpy as np
    def rnw_ms(J):
        ms = []
        for _ in range(3):
            tot, _, _ = ctx.run(J, "estimate", True)
            ms.append(sum(L["ms"] for L in ctx.last_launches()))
        return sorted(ms)[1], tot
    out = {}
    rng = np.random.default_rng(11)
    uneven = [W.permutation_union_matrix(int(rng.integers(16, 31)), int(rng.integers(3, 7)),
                                         int(rng.integers(0, 2 ** 31 - 1)), 1, 4) for _ in range(600)]
    for name, J in (("n60", jobs), ("uneven", ctx.jobs_from_dense(uneven))):
        ctx.tune_clear()
        ctx.estimate(J, trials, 1)
        d_ms, d_tot = rnw_ms(J)
        t0 = time.perf_counter()
        table = ctx.autotune(J)
        tune_s = time.perf_counter() - t0
        t_ms, t_tot = rnw_ms(J)
        out[name] = {"default_rnw_ms": d_ms, "tuned_rnw_ms": t_ms, "tuning_s": tune_s, "table": table,
                     "values_equal": t_tot == d_tot and (name != "n60" or t_tot == want)}
    ctx.tune_clear()
    return out


def graph_leg(hp, W):
    """HIP graph replay against eager launches: wall time of one persistent run call on a
    resident job table (median of 9 after a warm-up; the first graph run captures), on the
    benchmark's jobs and on a small table of 64 jobs of order 16 (where launch and host
    overhead dominate); the values are checked equal."""
    import numpy as np
    import torch
    out = {}
    items = W.config_n60(16)
    small = [W.permutation_union_matrix(16, 3, 900 + i, 1, 3) for i in range(64)]
    for name, build in (("n60_jobs", lambda c: c.expand([A for _, A in items])),
                        ("small64_order16", lambda c: c.jobs_from_dense(small))):
        rec = {}
        ref = None
        for mode in ("eager", "graph"):
            c = hp.Context({"split_order": 0, "device_expand": 0, "use_graphs": int(mode == "graph")})
            try:
                J = build(c)
                c.run(J, "natural", True)
                walls = []
                for _ in range(9):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    tot, _, _ = c.run(J, "natural", True)
                    walls.append(time.perf_counter() - t0)
                ref = tot if ref is None else ref
                rec[f"{mode}_run_call_ms"] = sorted(walls)[4] * 1e3
                rec[f"{mode}_equal"] = tot == ref
            finally:
                c.close()
        out[name] = rec
    return out


def schedule_study(hp, ctx, jobs, keys, machines=(1, 2, 4, 8, 16, 32)):
    """The paper's load-balancing study on our jobs. One persistent run in natural order with
    per-job work timing gives T (work cycles), P (the exact job permanents) and, from the
    estimate, AP. Reports Kendall's tau (tie-corrected, with the paper's normal p-value) of T
    against P, AP and the subset-term count, and the parallel efficiency sum(T) / (k makespan)
    of list scheduling T on k machines in four orders: natural (PH Step 3), non-increasing T
    (the ideal one), non-increasing AP (the improved Step 3) and non-increasing 2^(m-1)."""
    import numpy as np
    ctx.set_opts(time_jobs=1)
    try:
        _, per_job, _ = ctx.run(jobs, "natural", True, per_job=True)
        T = jobs.cycles().astype(np.uint64)
    finally:
        ctx.set_opts(time_jobs=0)
    n = T.size
    P = np.array([math.log2(v) if v > 0 else -1.0 for v in per_job])
    AP = np.asarray(keys, dtype=np.float64)
    terms = jobs.describe()["terms"].astype(np.float64)
    tf = T.astype(np.float64)
    out = {"jobs": int(n), "time_unit": "shader-clock cycles of the job's work items",
           "cv_of_T": float(tf.std() / tf.mean()) if n else 0.0}
    for name, y in (("P", P), ("AP", AP), ("terms", terms)):
        try:
            tau, z, p = hp.kendall_tau(tf, y)
            out[f"tau_T_{name}"] = {"tau": tau, "z": z, "p": p}
        except hp.HpermError:   # every job tied in y (e.g. equal subset-term counts)
            out[f"tau_T_{name}"] = None
    nat = np.arange(n)
    desc = lambda v: np.lexsort((nat, -v))   # noqa: E731  non-increasing, ties by natural index
    orders = {"natural": nat, "time": desc(tf), "estimate": desc(AP), "exact_cost": desc(terms)}
    eff = {}
    for oname, order in orders.items():
        eff[oname] = {}
        for k in machines:
            ms, _ = hp.list_schedule(T, order, k)
            eff[oname][str(k)] = float(tf.sum() / (k * ms)) if ms else 1.0
    out["ls_efficiency"] = eff
    return out


def device_hper(hp, ctx, jobs, want, mats, golden_vals, keys, targets=(10, 12, 13, 14, 15, 16)):
    """The device continuation of H_per (split_order) on the resident jobs: each job is split on
    the device by expansion (2) down to the target order and its leaves evaluated there. Per
    target: the split launches' time (HIP events, median of 3), leaves, their subset-terms,
    splits, splits refused by the entry bounds, and whether the totals equal the R-NW run's.
    At the fastest target also the per(A) batch wall time and the scheduling study with T =
    each job's wave time."""
    import numpy as np
    import torch
    out = {"by_target": {}}
    for t in targets:
        ctx.set_opts(split_order=t)
        try:
            ms, walls, ok = [], [], True
            for _ in range(3):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                tot, _, _ = ctx.run(jobs, "natural", True)
                walls.append(time.perf_counter() - t0)
                L = [x for x in ctx.last_launches() if x["variant"] == 3][0]
                ms.append(L["ms"])
                ok = ok and tot == want
        finally:
            ctx.set_opts(split_order=0)
        out["by_target"][str(t)] = {
            "split_ms": sorted(ms)[1], "run_call_ms": sorted(walls)[1] * 1e3, "leaves": int(L["leaves"]),
            "leaf_terms": int(L["leaf_terms"]), "splits": int(L["splits"]),
            "refused_splits": int(L["split_stops"]), "jobs": int(L["n_jobs"]), "totals_equal_rnw": ok}
    main = min(targets, key=lambda t: out["by_target"][str(t)]["split_ms"])
    out["target_order"] = main
    ctx.set_opts(split_order=main)
    try:
        ctx.permanent_batch(mats)   # warm-up
        walls = []
        for _ in range(5):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            vals = ctx.permanent_batch(mats)
            walls.append(time.perf_counter() - t0)
        out["per_a_wall_ms_batch"] = sorted(walls)[2] * 1e3
        out["per_a_verified"] = bool(golden_vals) and vals == golden_vals
        st = schedule_study(hp, ctx, jobs, keys)
        st["time_unit"] = "shader-clock cycles of the job's wave (split, leaves and their walks)"
        out["schedule_study"] = st
    finally:
        ctx.set_opts(split_order=0)
    return out


def large_single(hp, W, seeds=(0,)):
    """The large single problems on the device path (expansion on the device to order 22, the
    device continuation of H_per to order 12): the paper's C100 (its printed per(A) is the
    check) and random cubic graphs on 100 vertices (checked against the Schrijver and Bregman
    bounds; their first jobs equal the oracle's in the tests). One run each."""
    import torch
    C100 = 149364113290700
    out = {}
    ctx = hp.Context({"split_order": 12, "device_expand": 22, "device_expand_mib": 16384})
    try:
        probs = [("c100", W.adjacency_matrix(W.read_appendix_adjacency("c100")))]
        probs += [(f"cubic100_seed{s}", W.random_cubic_matrix(100, s)) for s in seeds]
        for name, A in probs:
            log("large single problem", name)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            v, st = ctx.permanent_batch([A], with_stats=True)
            wall = time.perf_counter() - t0
            L = [l for l in ctx.last_launches() if l["variant"] == 4][-1]
            n = A.shape[0]
            rec = {"per": str(v[0]), "per_a_wall_s": wall, "jobs_order22": int(L["n_jobs"]),
                   "expansion_nodes": int(L["items"]), "device_hper_launches": int(L["row_updates"]),
                   "leaves": int(L["leaves"]), "leaf_subset_terms": int(L["leaf_terms"]),
                   "splits": int(L["splits"]), "device_hper_s": L["alg_slots"] * 1e-3}
            if name == "c100":
                rec["equals_paper"] = v[0] == C100
            else:
                rec["within_schrijver_bregman"] = (4 / 3) ** n <= v[0] <= 6 ** (n / 3)
            out[name] = rec
    finally:
        ctx.close()
    # random cubic graphs on 120 vertices: the library's own estimate of their trees (Knuth's
    # random descents) and the time it implies at the rate just measured
    rates = [r["leaves"] / r["device_hper_s"] for r in out.values() if r.get("device_hper_s")]
    rate = max(rates) if rates else None
    for s in (0, 1):
        A = W.random_cubic_matrix(120, s)
        _, lv = hp.tree_estimate(A, samples=20000, seed=3, split_order=12, device_expand=22)
        out[f"cubic120_seed{s}"] = {"run": False, "estimated_leaves": float(lv.sum()),
                                    "projected_s_at_measured_leaf_rate": float(lv.sum() / rate) if rate else None,
                                    "estimator": "20000 random descents of the expansion tree (hperm_tree_estimate)"}
    return out


def order_trials_study(hp, ctx, jobs, split=12, trial_set=(4, 8, 16, 32)):
    """The estimate's budget and the queue order on the device continuation of H_per, where a
    job is one wave's whole unit and its time follows its permanent: per trial budget the
    estimate call's time and Kendall's tau of the jobs' measured wave times against the keys;
    the device H_per launch time (median of 3) in estimate, natural, random and exact-cost
    order; and list-scheduling efficiency of the measured times on k = the launch's resident
    waves (the machines the queue actually feeds) as well as k = 32 (the paper's)."""
    import numpy as np
    out = {"split_order": split, "by_trials": {}, "launch_ms_by_order": {}}
    ctx.set_opts(split_order=split, time_jobs=1)
    try:
        ctx.run(jobs, "natural", True)
        T = jobs.cycles().astype(np.float64)
    finally:
        ctx.set_opts(time_jobs=0)
    split_jobs = T > 0   # the jobs the device continuation took
    for tr in trial_set:
        t0 = time.perf_counter()
        keys = ctx.estimate(jobs, tr, 1)
        est_ms = (time.perf_counter() - t0) * 1e3
        tau, z, _ = hp.kendall_tau(T[split_jobs], np.asarray(keys, np.float64)[split_jobs])
        out["by_trials"][str(tr)] = {"estimate_call_ms": est_ms, "tau_time_key": tau, "z": z}
    grid = 0
    for order in ("estimate", "natural", "random", "exact_cost"):
        ms = []
        for _ in range(3):
            ctx.run(jobs, order, True)
            L = [L for L in ctx.last_launches() if L["variant"] == 3][0]
            ms.append(L["ms"])
            grid = int(L["reserved"])   # the launch's resident waves
        out["launch_ms_by_order"][order] = sorted(ms)[1]
    ctx.set_opts(split_order=0)
    Tu = T[split_jobs].astype(np.uint64)
    n = Tu.size
    nat = np.arange(n)
    keys = np.asarray(ctx.estimate(jobs, 32, 1), np.float64)[split_jobs]
    desc = lambda v: np.lexsort((nat, -v))   # noqa: E731
    eff = {}
    for k in (32, grid):
        eff[str(k)] = {}
        for oname, order in (("natural", nat), ("estimate", desc(keys)), ("time", desc(Tu.astype(np.float64)))):
            ms, _ = hp.list_schedule(Tu, order, k)
            eff[str(k)][oname] = float(Tu.astype(np.float64).sum() / (k * ms)) if ms else 1.0
    out["ls_efficiency"] = eff
    out["machines_note"] = f"{grid} = the resident waves (one per block) of the device H_per launch"
    return out


def regression_study(hp, W, ctx, jobs, split=12, sample=20000, seed=5):
    """The regression of Section 3.1 (eqs. 4-6) on device-H_per times: T (the shader cycles of
    a job's wave in a timed run of the device continuation) against P = per, |D| = |det|, S =
    nonzeros, V1 and V2 = variances of the row and column sums; R^2 of the full model (Table
    T1's figure), the factors stepwise selection keeps (F-to-enter 4.0, F-to-remove 3.9) and R^2
    of T on P alone (eq. 6's form). Groups as in the paper: 100 random 0-1 matrices per (n, S)
    (each one job, run whole on the device), and a sample of the n60 workload's order-20 jobs.
    Factors constant within a group are left out (S of the n60 jobs varies; of a group, never)."""
    import numpy as np
    names = ["P", "|D|", "S", "V1", "V2"]

    def analyse(T, P, inv):
        X = np.column_stack([P, inv])
        cols = [i for i in range(5) if np.ptp(X[:, i]) > 0]
        _, r2 = hp.ols(X[:, cols], T)
        chosen = [names[cols[c]] for c in hp.stepwise(X[:, cols], T)]
        _, r2p = hp.ols(P[:, None], T)
        return {"jobs": int(T.size), "r2_all_factors": r2, "stepwise_keeps": chosen, "r2_P_only": r2p,
                "factors_left_out_as_constant": [names[i] for i in range(5) if i not in cols]}

    out = {"split_order": split, "groups": {}}
    ctx.set_opts(split_order=split, time_jobs=1)
    try:
        for n, mult in ((20, 4), (20, 5), (20, 6), (24, 4), (24, 5)):
            mats = [W.random_01_matrix(n, mult * n, 100000 * n + 1000 * mult + s) for s in range(100)]
            J = ctx.jobs_from_dense(mats)   # a matrix with an empty line gives no job
            d = J.describe()
            _, per_job, _ = ctx.run(J, "natural", True, per_job=True)
            T = J.cycles().astype(np.float64)
            sel = [j for j in range(len(per_job)) if d["arith"][j] == 1 and per_job[j] > 0]   # device H_per jobs
            inv = np.array([hp.matrix_invariants(mats[int(d["problem"][j])]) for j in sel])
            out["groups"][f"n{n}_S{mult}n"] = analyse(T[sel], np.array([float(per_job[j]) for j in sel]), inv)
        _, per_job, _ = ctx.run(jobs, "natural", True, per_job=True)
        T = jobs.cycles().astype(np.float64)
        rng = np.random.default_rng(seed)
        pick = np.sort(rng.choice(T.size, size=min(sample, T.size), replace=False))
        pick = [int(k) for k in pick if T[k] > 0]
        inv = np.array([hp.matrix_invariants(jobs.matrix(k)) for k in pick])
        out["groups"]["n60_order20_jobs_sample"] = analyse(T[pick], np.array([float(per_job[k]) for k in pick]), inv)
    finally:
        ctx.set_opts(split_order=0, time_jobs=0)
    return out


def split_profile_run():
    """A short fixed sequence for profiling the device continuation of H_per: the n60
    workload's order-20 host jobs at t = 12 five times (natural order), one timed run, then the
    per(A) batch on the default path (device expansion to 22, continuation to 12) six times;
    every total is checked against the oracle's stored values."""
    import torch
    import paper_1112_6072_amd as hp
    import workloads as W
    items = W.config_n60(16)
    mats = [A for _, A in items]
    golden = json.load(open(os.path.join(ROOT, "tests", "golden", "oracle_values.json")))
    want = [int(golden[n]) for n, _ in items]
    ctx = hp.Context({"split_order": 12, "device_expand": 0})
    out = {}
    try:
        J = ctx.expand(mats)
        ms = []
        for _ in range(5):
            tot, _, _ = ctx.run(J, "natural", True)
            assert tot == want, "totals"
            ms.append([L for L in ctx.last_launches() if L["variant"] == 3][0]["ms"])
        out["split_ms_n60_t12"] = sorted(ms)[2]
        ctx.set_opts(time_jobs=1)
        ctx.run(J, "natural", True)
        ctx.set_opts(time_jobs=0, device_expand=22)
        walls = []
        for _ in range(6):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            assert ctx.permanent_batch(mats) == want, "per(A)"
            walls.append(time.perf_counter() - t0)
        out["per_a_default_ms"] = sorted(walls[1:])[2] * 1e3
    finally:
        ctx.close()
    print(json.dumps(out), flush=True)


def n80_batch(hp, W, golden):
    """The batched configuration's eight cubic girth >= 5 graphs on 80 vertices, per(A) of the
    batch on the library's default path (median of 3 calls), checked against the oracle's
    stored values."""
    import torch
    items = W.config_n80(8)
    mats = [A for _, A in items]
    ctx = hp.Context({"device_expand_mib": 16384})
    try:
        walls, got, st = [], None, None
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            got, st = ctx.permanent_batch(mats, with_stats=True)
            walls.append(time.perf_counter() - t0)
        dev = [L for L in ctx.last_launches() if L["variant"] == 4]
    finally:
        ctx.close()
    return {"graphs": len(mats), "per_a_wall_ms_batch": sorted(walls)[1] * 1e3,
            "verified_vs_oracle": bool(golden) and got == [int(golden[n]) for n, _ in items],
            "jobs_order22": int(sum(L["n_jobs"] for L in dev)), "expansion_nodes": int(sum(L["items"] for L in dev)),
            "device_hper_launches": int(sum(L["row_updates"] for L in dev)),
            "note": "the host path at m_cut 20 expands this batch into 27.4 M jobs of order 20 "
                    "(1.3e13 subset-terms; its R-NW alone took 10.8 s)"}


def copy_probe(nbytes: int = 256 << 20, reps: int = 3):
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": nbytes, "copy_probe_bytes_written": nbytes, "reps": reps}))


def c60_primes() -> list:
    """The primes of the library's residue route for C60's permanental polynomial: the largest
    primes below 2^18 whose product passes the coefficient bound max_k C(60, k) g^k (g =
    (3!)^(1/3), Bregman's factor of a row with three ones) by more than a bit, then one more (the
    check): the six largest."""
    import math
    g = 6 ** (1 / 3)
    bound = max(math.log2(math.comb(60, k)) + k * math.log2(g) for k in range(61)) * (1 + 1e-9) + 1
    out, cover, q, done = [], 0.0, (1 << 18) - 1, False
    while True:
        if all(q % d for d in range(2, int(q ** 0.5) + 1)):
            out.append(q)
            if done:
                return out
            cover += math.log2(q)
            done = cover > bound + 1
        q -= 2


def c60_residues_part(j: int, out_dir: str, points=None, batch: int = 8):
    """per(xI + A) of C60 (the appendix's graph) modulo the j-th prime of c60_primes(), for
    x = 0..60 (or the given points), on the device path in modular arithmetic, `batch` points per
    call (a progress line after each); saved to <out_dir>/c60_residues_<j>.json for --c60-combine."""
    import numpy as np
    import paper_1112_6072_amd as hp
    import workloads as W
    primes = c60_primes()
    A = W.adjacency_matrix(W.read_appendix_adjacency("c60")).astype(np.uint32)
    eye = np.eye(60, dtype=np.uint32)
    ctx = hp.Context()
    res, device_s = [], 0.0
    try:
        pts = list(range(61)) if points is None else list(points)
        for b0 in range(0, len(pts), batch):
            xs = pts[b0:b0 + batch]
            t0 = time.perf_counter()
            res += ctx.permanent_mod_batch([A + np.uint32(x) * eye for x in xs], primes[j])
            dt = time.perf_counter() - t0
            device_s += dt
            log(f"C60 prime {j} ({primes[j]}): x = {xs[0]}..{xs[-1]} in {dt:.1f} s")
    finally:
        ctx.close()
    out = {"prime_index": j, "prime": primes[j], "points": pts, "residues": res, "seconds": device_s}
    os.makedirs(out_dir, exist_ok=True)
    with open(os.path.join(out_dir, f"c60_residues_{j}.json"), "w") as fh:
        json.dump(out, fh)
    print(json.dumps({k: v for k, v in out.items() if k != "residues"}), flush=True)


def c60_combine(out_dir: str):
    """C60's permanental polynomial from the saved residues of every prime (host step of the
    library: per-prime interpolation and the Chinese remainder theorem, checked against the last
    prime), against the oracle's stored coefficients."""
    import paper_1112_6072_amd as hp
    primes = c60_primes()
    parts = []
    for j in range(len(primes)):
        with open(os.path.join(out_dir, f"c60_residues_{j}.json")) as fh:
            parts.append(json.load(fh))
        assert parts[-1]["prime"] == primes[j] and parts[-1].get("points", list(range(61))) == list(range(61))
    coeffs = hp.polynomial_from_residues(primes, [p["residues"] for p in parts], alternate=True)
    with open(os.path.join(ROOT, "tests", "golden", "c60_permanental_polynomial.json")) as fh:
        want = [int(v) for v in json.load(fh)["coefficients"]]
    seconds = sum(p["seconds"] for p in parts)
    print(json.dumps({"graph": "C60 (appendix adjacency)", "primes": primes, "points": 61,
                      "device_seconds": seconds, "seconds_per_point": seconds / (61 * len(primes)),
                      "c60": coeffs[60], "c59": coeffs[59], "c58": coeffs[58], "c0": coeffs[0],
                      "equal_to_oracle": coeffs == want}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--m-cut", type=int, default=20)
    ap.add_argument("--trials", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-large", action="store_true", help="skip C100 and the random cubic n=100 problem")
    ap.add_argument("--large-only", choices=["c100", "all"], default=None,
                    help="only run the large single problems (C100, or C100 and random cubic n=100) and "
                         "print their record (for profiling)")
    ap.add_argument("--profile-split", action="store_true",
                    help="only the short fixed sequence used to profile the device continuation of H_per")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a device-to-device copy of 256 MiB three times (the reference kernel "
                         "that scales the FETCH_SIZE / WRITE_SIZE counters to bytes)")
    ap.add_argument("--c60-residues", type=int, default=None, metavar="J",
                    help="only per(xI + A) of C60 modulo the J-th of its polynomial's six primes, x = 0..60")
    ap.add_argument("--c60-combine", action="store_true",
                    help="only C60's permanental polynomial from the saved residues of all six primes")
    ap.add_argument("--out-dir", default=".", help="where --c60-residues saves and --c60-combine reads")
    ap.add_argument("--c60-points", default=None, metavar="X,Y",
                    help="with --c60-residues: only these points x (e.g. one point, for profiling)")
    args = ap.parse_args()
    if args.c60_residues is not None:
        pts = [int(v) for v in args.c60_points.split(",")] if args.c60_points else None
        c60_residues_part(args.c60_residues, args.out_dir, pts)
        return
    if args.c60_combine:
        c60_combine(args.out_dir)
        return
    if args.profile_split:
        split_profile_run()
        return
    if args.copy_probe:
        copy_probe()
        return
    if args.large_only:
        import paper_1112_6072_amd as hp
        import workloads as W
        import torch
        torch.cuda.set_device(0)
        print(json.dumps(large_single(hp, W, seeds=() if args.large_only == "c100" else (0,))), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (the path shards "
              f"its job list across GPUs only in design)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1112_6072_amd as hp
    import workloads as W

    torch.cuda.set_device(0)
    items = W.config_n60(16)
    names = [n for n, _ in items]
    mats = [A for _, A in items]
    golden_path = os.path.join(ROOT, "tests", "golden", "oracle_values.json")
    golden = json.load(open(golden_path)) if os.path.exists(golden_path) else {}

    # the R-NW measurements run with the device continuation of H_per off (split_order 0);
    # per(A) is timed on the library's default path (device expansion to order 22, device H_per
    # to order 12) and beside it on the host-expansion paths and the R-NW-only one
    ctx = hp.Context({"m_cut": args.m_cut, "trials": args.trials, "split_order": 0, "device_expand": 0})

    # ---- per(A) wall time, host CSR -> exact integers (expansion and copies included)
    def per_a_batch(split, m_cut=args.m_cut, dexp=0):
        ctx.set_opts(split_order=split, m_cut=m_cut, device_expand=dexp)
        try:
            ctx.permanent_batch(mats)   # warm-up
            walls = []
            for _ in range(5):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                v, st = ctx.permanent_batch(mats, with_stats=True)
                walls.append(time.perf_counter() - t0)
        finally:
            ctx.set_opts(split_order=0, m_cut=args.m_cut, device_expand=0)
        return sorted(walls)[2], v, st   # median of 5
    log("per(A) end to end")
    e2e, vals, _ = per_a_batch(12, dexp=22)          # the library default
    # the host expands to order 22 (fewer jobs: its time is linear in them), the device
    # continues H_per to order 12; the host to order 20; every job by R-NW
    e2e_h22, vals_h22, stats = per_a_batch(12, 22)
    e2e_m20, vals_m20, _ = per_a_batch(12)
    e2e_rnw, vals_rnw, _ = per_a_batch(0)
    exp_s = stats[0]["t_expand_s"]
    verified = (bool(golden) and all(int(golden[n]) == v for n, v in zip(names, vals)) and vals_rnw == vals
                and vals_m20 == vals and vals_h22 == vals)

    # ---- the timed step: jobs resident in HBM
    jobs = ctx.expand(mats)
    d = jobs.describe()
    n_jobs = int(d["m"].size)
    terms = int(d["terms"].astype(np.float64).sum())
    log(f"jobs {n_jobs}, subset-terms {terms:.3e}")
    for _ in range(args.warmup):
        ctx.estimate(jobs, args.trials, 1)
        ctx.run(jobs, "estimate", True)
    launches = []
    est_s = run_s = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ta = time.perf_counter()
        ctx.estimate(jobs, args.trials, 1)
        tb = time.perf_counter()
        tot, _, res = ctx.run(jobs, "estimate", True)
        tc = time.perf_counter()
        est_s += tb - ta
        run_s += tc - tb
        launches.append(ctx.last_launches())
    torch.cuda.synchronize()
    step_s = (time.perf_counter() - t0) / args.steps
    verified = verified and tot == vals

    # dominant kernel: the launch group with the most time; average over the steps
    groups = {}
    for ls in launches:
        for L in ls:
            key = (L["ring"], L["bucket"], L["variant"])
            g = groups.setdefault(key, {"ms": 0.0, "alg": 0.0, "terms": 0, "jobs": 0, "n": 0, "upd": 0})
            g["ms"] += L["ms"]
            g["upd"] += L["row_updates"]
            g["jobs"] += L["n_jobs"]
            g["alg"] += L["alg_slots"]
            g["terms"] += L["terms"]
            g["n"] += 1
    (ring, bucket, variant), dom = max(groups.items(), key=lambda kv: kv[1]["ms"])
    avg_ms = dom["ms"] / dom["n"]
    alg_per_launch = dom["alg"] / dom["n"]
    achieved = alg_per_launch / (avg_ms * 1e-3)
    # the launch's ring multiplies, recovered from its slot count (slots = mul x M + add x A + U
    # with A = one ring addition per term, or per two terms in the paired walk, U = the row
    # updates), and the same launch weighed with the half-rate multiplies at the issue costs a
    # probe measured for them (v_mul_lo_u32 2.5 and v_mad_u64_u32 3.8 full-rate slots instead
    # of 2 each; mod 2^64 only)
    WALK_NAMES = {0: "step-pair walk", 1: "paired walk, two-row column 0",
                  2: "paired walk, three-row column 0", 6: "four-step walk, two-row column 0",
                  7: "four-step walk, three-row column 0"}
    mul_slots, add_slots = {0: (5.0, 2.0), 1: (9.0, 4.0), 2: (33.0, 9.0)}[ring]
    adds = dom["terms"] / dom["n"] / {0: 1.0, 1: 2.0, 2: 2.0, 6: 4.0, 7: 4.0}[variant]
    # the four-step walks' full-rate block slots (FP32 products, conversions, 24-bit product)
    extra = dom["terms"] / dom["n"] / 4.0 * {6: 17.0, 7: 20.0}.get(variant, 0.0)
    mults = (alg_per_launch - add_slots * adds - dom["upd"] / dom["n"] - extra) / mul_slots
    probe_frac = ((alg_per_launch + mults * (2.5 + 3.8 - 4.0)) / (avg_ms * 1e-3) / ALU_PEAK
                  if ring == 0 else None)
    rnw_ms = sum(g["ms"] for g in groups.values()) / args.steps
    ring_name = {0: "mod 2^64", 1: "mod 2^128", 2: "residues"}[ring]

    # ---- comparators on the same resident jobs
    extra = {}
    for order in ("natural", "random", "exact_cost"):
        ctx.run(jobs, order, True)
        extra[f"persistent_{order}_rnw_ms"] = sum(L["ms"] for L in ctx.last_launches())
    extra["uneven_jobs"] = uneven_orders(hp, W, ctx)
    log("queue orders on jobs of uneven order from the expansion (s_leaf 3)")
    extra["expansion_uneven_n60"] = expansion_uneven(hp, W, ctx, mats, vals, args.m_cut, plain=not args.no_plain)
    extra["autotune"] = autotune_leg(hp, W, ctx, jobs, args.trials, tot)
    extra["hip_graphs"] = graph_leg(hp, W)
    # one problem alone: the truncated icosahedron (C60), median of 5 after a warm-up, on the
    # default path and on the R-NW-only one
    def c60_alone(split, dexp=0):
        ctx.set_opts(split_order=split, device_expand=dexp)
        try:
            ctx.permanent(mats[0])
            walls1 = []
            for _ in range(5):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                v = ctx.permanent(mats[0])
                walls1.append(time.perf_counter() - t0)
        finally:
            ctx.set_opts(split_order=0, device_expand=0)
        return sorted(walls1)[2], v
    e2e_c60, c60 = c60_alone(12, 22)
    e2e_c60_host, c60_host = c60_alone(12)
    e2e_c60_rnw, c60_rnw = c60_alone(0)
    verified = verified and c60 == vals[0] and c60_rnw == vals[0] and c60_host == vals[0]
    # permanental polynomial per(xI - A) of a random cubic graph on 24 vertices (25 exact
    # evaluations of per(xI + A) in one batch, then exact interpolation); median of 5
    G24 = W.random_cubic_matrix(24, 0)
    poly = ctx.permanental_polynomial(G24)
    wp = []
    for _ in range(5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.permanental_polynomial(G24)
        wp.append(time.perf_counter() - t0)
    extra["permanental_polynomial"] = {
        "graph": "random cubic, n=24, seed 0", "ms": sorted(wp)[2] * 1e3,
        "checks": {"leading_1": poly[24] == 1, "trace_0": poly[23] == 0, "edges_36": poly[22] == 36,
                   "constant_is_per": poly[0] == ctx.permanent(G24)}}
    log("scheduling study on the n60 jobs")
    keys = ctx.estimate(jobs, args.trials, 1)
    extra["schedule_study_n60"] = schedule_study(hp, ctx, jobs, keys)
    log("device continuation of H_per on the n60 jobs")
    golden_vals = [int(golden[n]) for n in names] if golden else None
    extra["device_hper_n60"] = device_hper(hp, ctx, jobs, tot, mats, golden_vals, keys)
    log("estimate budget and queue order on the device continuation of H_per")
    extra["order_trials_study_n60"] = order_trials_study(hp, ctx, jobs)
    log("regression study (Section 3.1)")
    extra["regression_study"] = regression_study(hp, W, ctx, jobs)
    log("the n80 batch (8 cubic graphs on 80 vertices) on the default path")
    extra["n80_batch"] = n80_batch(hp, W, golden)
    plain = None
    if not args.no_plain:
        log("plain: one launch per job, expansion order (best lane chunk of 3, 5, 7)")
        best = None
        for chunk in (3, 5, 7):
            ctx.set_opts(chunk_log2=chunk)
            ctx.run(jobs, "natural", False)
            ms = ctx.last_launches()[0]["ms"]
            extra[f"plain_rnw_ms_chunk{chunk}"] = ms
            best = ms if best is None else min(best, ms)
        ctx.set_opts(chunk_log2=0)
        plain = terms / (best * 1e-3)
        extra["plain_rnw_ms"] = best
        extra["plain_terms_per_s"] = plain
    lpt_rate = terms / (rnw_ms * 1e-3)

    serving = None
    if not args.no_serving:
        log("serving: burst, then Poisson arrivals at half the measured capacity")
        serving = serving_leg(hp, W)
        log("serving, the narrower mix (n 30..40, no work limit)")
        extra["serving_n30_40"] = serving_leg(hp, W, n_hi=40, limit_ms=0)

    large = None
    if not args.no_large:
        large = large_single(hp, W)

    cpu = cpu_ryser = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle): C H_per over the whole batch")
        cpu_vals, cpu = cpu_oracle_batch(mats, terms)
        verified = verified and cpu_vals == vals
        log("cpu baseline (oracle): plain Ryser on a sample of jobs")
        cpu_ryser = cpu_baseline(args.m_cut)

    out = {
        "metric": "Ryser subset-terms/sec + per(A) wall time (n=60 cubic), batched-LPT vs plain",
        "value": terms / step_s,
        "unit": "subset-terms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64/int128 (exact integer rings)",
        "data": "synthetic",
        "config": {"workload": "n60_cubic: truncated icosahedron + 16 seeded random 3-regular girth>=5 "
                               "graphs on 60 vertices; expansion to jobs of order "
                               f"{args.m_cut}; KKLLL keys with {args.trials} trials",
                   "n_problems": len(mats), "n_jobs": n_jobs, "subset_terms": terms,
                   "job_order": "non-increasing KKLLL estimate", "parallelism": "1 GPU"},
        "per_a_wall_ms_batch": e2e * 1e3,
        "per_a_wall_ms_per_problem": e2e * 1e3 / len(mats),
        "per_a_wall_ms_c60_alone": e2e_c60 * 1e3,
        "per_a_path": "the library default: expansion on the device to order 22, H_per continued on "
                      "the device to order 12",
        "per_a_wall_ms_batch_host22": e2e_h22 * 1e3,
        "per_a_wall_ms_batch_m_cut20": e2e_m20 * 1e3,
        "per_a_wall_ms_batch_rnw_only": e2e_rnw * 1e3,
        "per_a_wall_ms_batch_cpu_oracle": cpu["per_a_wall_ms_batch"] if cpu else None,
        "per_a_wall_ms_c60_alone_host22": e2e_c60_host * 1e3,
        "per_a_wall_ms_c60_alone_rnw_only": e2e_c60_rnw * 1e3,
        "host_expand_ms_batch": exp_s * 1e3,
        "rnw_ms_per_step": rnw_ms,
        "step_breakdown_ms": {"estimate_call": est_s * 1e3 / args.steps, "run_call": run_s * 1e3 / args.steps,
                              "rnw_kernels": rnw_ms,
                              "run_host_and_other": run_s * 1e3 / args.steps - rnw_ms},
        "lpt_persistent_terms_per_s": lpt_rate,
        "lpt_vs_plain": (lpt_rate / plain) if plain else None,
        "verified_vs_oracle": verified,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK,
                     "unit": "VALU lane-slots/s", "frac": achieved / ALU_PEAK,
                     "traffic": traffic_from_profile(),
                     "kernel": f"rnw_persistent ({ring_name}, orders <= {[16, 20, 24, 32, 40][bucket]}, "
                               f"{WALK_NAMES[variant]})",
                     "avg_launch_ms": avg_ms, "alg_slots_per_launch": alg_per_launch,
                     "jobs_per_launch": dom["jobs"] // dom["n"], "terms_per_launch": dom["terms"] // dom["n"],
                     "ring_multiplies_per_launch": mults, "frac_with_probe_multiply_weights": probe_frac},
        "cpu_baseline": cpu,
        "cpu_baseline_ryser_sample": cpu_ryser,
        "large_single_problems": large,
        "serving": serving,
    }
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
