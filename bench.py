"""Throughput of the two-phase PSL search's hot path on one MI355X.

Workload (default): the batched uniform configuration, 1024 independent walks
at L = 2^17 - 1 = 131071, each a random +-1 start from its own seed, full
neighbourhood (N_lmt = L), alpha_1 = 4 / alpha_2 = 13, a phase switch every 50
steps with FLIP_lmt = 10, FP64 fitness. One bench step is one iteration of the
loop of Algorithm 1 on every walk of the batch: neighbourhood evaluation,
selection, the O(L) flip, bookkeeping and (when due) the switch.

Prints one JSON line: flip-evals/s (whole job) with the roofline of the
dominant kernel (the neighbourhood evaluation, timed with HIP events on its
own stream) and the CPU oracle timed on a bounded sample of the same work.
Two secondary measurements ride along: the request loop under Poisson
arrivals of the serving workload's job mixture (p50/p99 time-to-budget and
aggregate flip-evals/s), and the same jobs served together against one walk
per launch sequence.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 64 lanes x 2.4 GHz of 32-bit / non-packed FP64 VALU issue
# (each CU issues one 64-lane VALU instruction per clock: 4 SIMDs, 4 clocks each).
PEAK_LANE_OPS = 256 * 64 * 2.4e9
# MI355X dense int8 matrix-core peak (v_mfma_i32_*_i8), ops/s (a multiply-add is 2).
PEAK_INT8_OPS = 5.0e15
# int8 ops of the split path's linear part per (element, neighbour) term: one
# multiply-add per digit of the quantized coefficient (8 digits).
LIN_OPS_PER_TERM = 2 * 8
# Shortest walk the split evaluation takes, and the fewest nominal updates of a
# launch that takes it by default.
SPLIT_MIN_L = 2048
SPLIT_MIN_WORK = 1 << 34
# VALU lane-ops per C_k-update of the direct form of the one-element flip: form
# C' (1), fold |C'| into the running max (1), select T(|C'|) (1), one FP64 add
# (1). The evaluation kernel needs fewer (it skips the unchanged shifts and
# resolves two or four shifts per table lookup), so this figure is reported
# beside the roofline, not as it.
OPS_PER_UPDATE_DIRECT = 4
# cfg2 (the batched uniform configuration) runs 100 steps per walk.
BATCHED_STEPS = 100
# Paper, Table 4 (A100 SXM4, N_lmt = 6912, one walk, alpha 4/10): context only.
PAPER_A100_NSE = {16383: 4678451, 32767: 2577101, 65535: 1258873, 131071: 638043,
                  262143: 326148, 524287: 167861, 1048575: 85062}


# Sources that define the evaluation kernel: a counter record is valid only for
# the exact text it was taken from.
KERNEL_SOURCES = ("paper_2107_09801_amd/csrc/psl_eval.hip", "paper_2107_09801_amd/csrc/psl_dev_util.h",
                  "paper_2107_09801_amd/csrc/psl_device.h", "paper_2107_09801_amd/csrc/psl_split.hip")


def kernel_source_digest() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counter_record(kind: str, tag: str, kernel: str = ""):
    """The `<kind>-record:` line of a committed rocprofv3 counter summary under
    profiles/ for workload `tag` (and kernel name prefix `kernel`, if given),
    as a dict of its key=value fields, or None when there is none or the
    evaluation kernels' sources changed since it was taken."""
    pdir = os.path.join(ROOT, "profiles")
    if not os.path.isdir(pdir):
        return None
    digest = kernel_source_digest()
    for name in sorted(os.listdir(pdir)):
        with open(os.path.join(pdir, name), encoding="utf-8", errors="replace") as f:
            for line in f:
                line = line.strip().strip("`")
                if not line.startswith(f"{kind}-record:"):
                    continue
                kv = dict(t.split("=", 1) for t in line.split()[1:] if "=" in t)
                if kv.get("workload") == tag and kv.get("source_sha256") == digest and \
                        kv.get("kernel", "").startswith(kernel):
                    return kv
    return None


def measured_traffic(tag: str, kernel: str = ""):
    """HBM bytes per launch of an evaluation kernel (k_eval or k_lin; any when
    empty) for workload `tag`, from the `traffic-record:` line (FETCH_SIZE and
    WRITE_SIZE, each scaled by what the counter reads for a copy of known
    size)."""
    kv = counter_record("traffic", tag, kernel)
    return None if kv is None else int(kv["fetch_bytes_per_launch"]) + int(kv["write_bytes_per_launch"])


def measured_valu(tag: str, kernel: str = "k_eval"):
    """VALU instructions (64-lane wavefront instructions, SQ_INSTS_VALU) per
    launch of the evaluation kernel for workload `tag`, from the
    `valu-record:` line."""
    kv = counter_record("valu", tag, kernel)
    return None if kv is None else float(kv["sq_insts_valu_per_launch"])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=BATCHED_STEPS,
                    help="timed steps (default: the batched configuration's 100 steps per walk)")
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--workload", default="batched",
                    choices=["batched", "single", "large", "uneven", "paper"],
                    help="batched: 1024 walks at L=131071 (the headline); single: one walk at "
                         "L=16383; large: one walk at L=1048575; uneven: L=2^m-1, m=14..20 with "
                         "512..8 walks; paper: Table 4 settings (N_lmt=6912, alpha 4/10, "
                         "LS_lmt=2000) at --L with --walks walks")
    ap.add_argument("--walks", type=int, default=0, help="override the walk count")
    ap.add_argument("--L", type=int, default=0, help="override L")
    ap.add_argument("--n-lmt", type=int, default=0, help="0 = full neighbourhood")
    ap.add_argument("--switch-period", type=int, default=50)
    ap.add_argument("--graph", action="store_true", help="replay a captured step per step")
    ap.add_argument("--autotune", action="store_true",
                    help="time every evaluation launch shape on the batch first and keep the fastest")
    ap.add_argument("--split", type=int, default=-1, choices=[-1, 0, 1, 2],
                    help="split evaluation (linear part on the matrix cores): -1 the library default "
                         "(2: for launches of at least 2^34 nominal updates), 0 off (table evaluation), "
                         "1 wherever L >= 2048")
    ap.add_argument("--tune-file", default="", help="evaluation launch shapes to load (psl_tune_load)")
    ap.add_argument("--eval-items", type=int, default=0,
                    help="minimum work items per evaluation launch (0 = the library default)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="target duration of the oracle sample, per mode (one thread; all cores)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=120.0,
                    help="arrival window of the serving run (0: skip it)")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="Poisson arrivals per second")
    ap.add_argument("--serve-nlmt", type=int, default=256,
                    help="N_lmt of served jobs (min(L, this))")
    ap.add_argument("--compare-jobs", type=int, default=48,
                    help="jobs in the served vs one-walk-per-launch comparison (0: skip)")
    ap.add_argument("--compare-uneven-steps", type=int, default=2,
                    help="uneven workload: steps of the batch-vs-one-walk-per-launch comparison (0 = off)")
    ap.add_argument("--study", default="", choices=["", "paper-sweep", "alpha-ablation", "restart", "serve"],
                    help="instead of the benchmark: the paper-settings speed sweep over L, the alpha ablation, "
                         "the restart protocol, or the serving run alone")
    ap.add_argument("--nse", type=float, default=1e9, help="alpha ablation: sequence evaluations per run")
    ap.add_argument("--runs", type=int, default=30, help="alpha ablation: runs per alpha pair")
    ap.add_argument("--rounds", type=int, default=4, help="restart study: rounds")
    ap.add_argument("--restart-nse", type=float, default=1e8,
                    help="restart study: sequence evaluations per walk and round")
    ap.add_argument("--sweep-seconds", type=float, default=4.0, help="paper sweep: seconds per L and mode")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="before the run, one device-to-device copy of this many MiB "
                         "(a known-size kernel to scale profiler byte counters)")
    return ap.parse_args()


def host_info() -> dict:
    """The host the oracle runs on: CPU model, logical CPUs, the CPUs this
    process may run on, and the OpenMP thread setting of the environment."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = os.cpu_count() or 1
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity_cpus": affinity,
            "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS")}


def all_core_threads(info: dict) -> int:
    """Every CPU this process may use, limited by OMP_NUM_THREADS when the
    environment sets it (the share of the host's cores given to one GPU)."""
    n = info["affinity_cpus"]
    omp = info["OMP_NUM_THREADS"]
    if omp and omp.isdigit() and int(omp) > 0:
        n = min(n, int(omp))
    return max(1, n)


def oracle_rate(L: int, n_lmt: int, alpha: int, target_s: float, max_walks: int, threads: int):
    """The oracle's Neighborhood for the first step of walks 0, 1, ... (their
    own seeds and starts), in scan-order slices, until about target_s seconds
    have passed. Only the evaluation is timed (the O(L^2) setup of each walk's
    C is not). Returns (neighbour evaluations, seconds, walks)."""
    import oracle
    import seeded_inputs as si
    done, walks, el = 0, 0, 0.0
    chunk = max(threads * 4, 16)
    for w in range(max_walks):
        seed = si.walk_seed(w)
        s = oracle.rand_pivot(seed, L)
        C = oracle.corr(s)
        start = oracle.draw(seed, 1 << 60) % L
        pos = 0
        while pos < n_lmt and el < target_s:
            m = min(chunk, n_lmt - pos)
            t0 = time.perf_counter()
            oracle.eval_neighbourhood(s, C, alpha, (start + pos) % L, m, nthreads=threads)
            el += time.perf_counter() - t0
            pos += m
            chunk = min(chunk * 2, n_lmt)
        done += pos
        walks += 1
        if el >= target_s:
            break
    return done, el, walks


def cpu_baseline(L: int, n_lmt: int, alpha: int, target_s: float, max_walks: int) -> dict:
    """The oracle timed in two modes on the host: one thread, and OpenMP over
    candidates on every core this process may use (see all_core_threads)."""
    info = host_info()
    threads = all_core_threads(info)
    d1, e1, w1 = oracle_rate(L, n_lmt, alpha, target_s, max_walks, 1)
    dn, en, wn = oracle_rate(L, n_lmt, alpha, target_s, max_walks, threads)
    return {"value": dn / en, "unit": "flip-evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{dn} neighbour evaluations from the first step of {wn} walk(s) at L={L} "
                      f"(alpha={alpha}), {en:.1f} s of evaluation, OpenMP over candidates on {threads} "
                      f"threads ({info['cpu_model']}, nproc {info['nproc']}, "
                      f"{info['affinity_cpus']} CPUs in this process's affinity, "
                      f"OMP_NUM_THREADS={info['OMP_NUM_THREADS']})",
            "C_k_updates_per_s": dn * (L - 1) / en,
            "single_thread": {"value": d1 / e1, "unit": "flip-evals/s", "cores": 1,
                              "C_k_updates_per_s": d1 * (L - 1) / e1,
                              "sample": f"{d1} neighbour evaluations from {w1} walk(s), {e1:.1f} s"},
            "host": info}


def run_serving(libpsl, seconds: float, rate: float, nlmt_cap: int, eval_items: int = 0) -> dict:
    """Poisson arrivals into the request loop; time-to-budget per job."""
    import numpy as np

    import seeded_inputs as si
    rng = np.random.Generator(np.random.PCG64(si.BASE_SEED))
    n = int(rng.poisson(rate * seconds))
    arrivals = np.sort(rng.uniform(0.0, seconds, size=n))
    jobs = si.serve_jobs(n, si.BASE_SEED + 1, nlmt_cap)
    ctx = libpsl.Context(0)
    if eval_items:
        ctx.set_option(libpsl.OPT_EVAL_ITEMS, eval_items)
    ctx.serve_start(hbm_budget=200 << 30, max_slots=4096)
    outstanding, results = set(), {}
    t0 = time.perf_counter()
    nxt = 0
    last_log = t0
    while nxt < n or len(results) < n:
        now = time.perf_counter() - t0
        while nxt < n and arrivals[nxt] <= now:
            j = jobs[nxt]
            outstanding.add(ctx.serve_submit(j["L"], j["seed"], j["budget"], alpha2=j["alpha2"],
                                             n_lmt=j["n_lmt"], switch_period=50, want_best=False))
            nxt += 1
        for t in list(outstanding):
            r = ctx.serve_poll(t)
            if r is not None:
                results[t] = r
                outstanding.discard(t)
        if time.perf_counter() - last_log > 5:
            last_log = time.perf_counter()
            log(f"serving: {nxt}/{n} submitted, {len(results)} done")
        time.sleep(0.0005)
    wall = time.perf_counter() - t0
    st = ctx.serve_stats()
    ctx.serve_stop(drain=True)
    ctx.close()
    ttb = np.array([(r["t_done_ns"] - r["t_arrive_ns"]) * 1e-9 for r in results.values()])
    queue = np.array([(r["t_admit_ns"] - r["t_arrive_ns"]) * 1e-9 for r in results.values()])
    offered = sum(j["budget"] * j["n_lmt"] * (j["L"] - 1) for j in jobs) / seconds
    return {"jobs": n, "arrival_rate": rate, "arrival_window_s": seconds, "wall_s": wall,
            "n_lmt": f"min(L, {nlmt_cap})",
            "time_to_budget_p50_s": float(np.percentile(ttb, 50)),
            "time_to_budget_p99_s": float(np.percentile(ttb, 99)),
            "queue_wait_p99_s": float(np.percentile(queue, 99)),
            "flip_evals_per_s": st["flip_evals"] / wall,
            "C_k_updates_per_s": st["ck_updates"] / wall,
            "offered_C_k_updates_per_s": offered,
            "failed": st["failed"], "peak_active": st["peak_active"],
            "iterations": st["iterations"]}


def run_compare(libpsl, n: int, nlmt_cap: int) -> dict:
    """The same jobs served together (all submitted at once) and run one walk
    per launch sequence, one job after the other (captured-graph steps)."""
    import seeded_inputs as si
    jobs = si.serve_jobs(n, si.BASE_SEED + 2, nlmt_cap)
    evals = sum(j["budget"] * j["n_lmt"] for j in jobs)
    ctx = libpsl.Context(0)
    ctx.serve_start(hbm_budget=200 << 30, max_slots=4096)
    t0 = time.perf_counter()
    tickets = [ctx.serve_submit(j["L"], j["seed"], j["budget"], alpha2=j["alpha2"],
                                n_lmt=j["n_lmt"], switch_period=50, want_best=False) for j in jobs]
    served, outstanding = {}, set(tickets)
    while outstanding:
        for t in list(outstanding):
            r = ctx.serve_poll(t)
            if r is not None:
                served[t] = r
                outstanding.discard(t)
        time.sleep(0.0005)
    t_served = time.perf_counter() - t0
    ctx.serve_stop(drain=True)
    solo = []
    t0 = time.perf_counter()
    for j in jobs:
        (w,) = ctx.init_walks(j["L"], 1, j["seed"], alpha2=j["alpha2"], n_lmt=j["n_lmt"],
                              switch_period=50)
        ctx.step_batch([w], j["budget"], graph=True)
        solo.append(ctx.read_walk(w, bits=False, C=False))
        ctx.free_walks([w])
    t_solo = time.perf_counter() - t0
    same = all(served[t]["psl_best"] == g["psl_best"] and served[t]["psl_final"] == g["psl_pivot"]
               for t, g in zip(tickets, solo))
    ctx.close()
    return {"jobs": n, "flip_evals": evals,
            "served_flip_evals_per_s": evals / t_served,
            "one_walk_per_launch_flip_evals_per_s": evals / t_solo,
            "speedup": t_solo / t_served, "results_identical": same}


def run_uneven_compare(libpsl, groups, steps: int, period: int) -> dict:
    """The uneven batch stepped in one launch sequence per step against every
    walk stepped alone (one launch sequence per walk), from the same seeds:
    wall time of `steps` steps each way, and whether every walk ends in the
    same state."""
    import torch

    import seeded_inputs as si
    ctx = libpsl.Context(0)
    batch, alone, base = [], [], 0
    for L, count in groups:
        kw = dict(alpha1=4, alpha2=si.alpha2_for(L), n_lmt=L, ls_lmt=2000, flip_lmt=10,
                  switch_period=period)
        batch += ctx.init_walks(L, count, si.BASE_SEED + 7 + base, **kw)
        for b in range(count):
            alone += ctx.init_walks(L, 1, si.BASE_SEED + 7 + base + b, **kw)
        base += count
    # warm single-walk timing per L: one more walk per L (same seed as the
    # first of its group), stepped alone with a captured graph
    warm, base = 0.0, 0
    for L, count in groups:
        (r,) = ctx.init_walks(L, 1, si.BASE_SEED + 7 + base, alpha1=4, alpha2=si.alpha2_for(L), n_lmt=L,
                              ls_lmt=2000, flip_lmt=10, switch_period=period)
        ctx.step_batch([r], 1, blocking=True, graph=True)
        t0 = time.perf_counter()
        ctx.step_batch([r], steps, blocking=True, graph=True)
        warm += count * (time.perf_counter() - t0)
        ctx.free_walks([r])
        base += count
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step_batch(batch, steps, blocking=True)
    t_batch = time.perf_counter() - t0
    t0 = time.perf_counter()
    for w in alone:
        ctx.step_batch([w], steps)
    ctx.sync()
    t_alone = time.perf_counter() - t0
    same = True
    for a, b in zip(alone, batch):
        ga, gb = ctx.read_walk(a, bits=False, C=False), ctx.read_walk(b, bits=False, C=False)
        same &= all(ga[k] == gb[k] for k in ("t", "last_k", "psl_best", "psl_pivot", "alpha",
                                               "unimproved"))
    ctx.close()
    return {"walks": len(batch), "steps": steps, "batch_s": t_batch,
            "one_walk_per_launch_s": t_alone, "speedup": t_alone / t_batch,
            "one_walk_per_launch_warm_graph_s": warm, "speedup_vs_warm_graph": warm / t_batch,
            "note": "one_walk_per_launch_s: every walk stepped alone, including its per-walk launch "
                    "set-up; warm_graph: per L, one walk's captured-graph step time times the walk count",
            "results_identical": bool(same)}


# Paper, Table 2 (L = 65535, 30 runs, NSE = 1e10, N_lmt = 6912): mean PSL.
PAPER_ALPHA_MEAN_PSL = {"4/13": 212.700, "4/4": 232.833, "13/13": 238.967}


def run_paper_sweep(libpsl, seconds: float) -> dict:
    """The paper's speed settings (N_lmt = 6912, alpha 4/10, LS_lmt = 2000,
    FLIP_lmt = 10, the switch rule of Algorithm 1) for every L = 2^m - 1,
    m = 14..20: one walk alone (captured-graph steps), and a batch of walks
    that fills the GPU; flip-evals/s against Table 4's A100 figure."""
    import seeded_inputs as si
    ctx = libpsl.Context(0)
    rows = []
    for m in range(14, 21):
        L = 2 ** m - 1
        kw = dict(alpha1=4, alpha2=10, n_lmt=6912, ls_lmt=2000, flip_lmt=10, switch_period=0)
        row = {"L": L, "A100_flip_evals_per_s": PAPER_A100_NSE[L]}
        for label, count in (("one_walk", 1), ("batch", 64 if m <= 18 else 16)):
            ids = ctx.init_walks(L, count, si.BASE_SEED + 500 * m, **kw)
            ctx.step_batch(ids, 3, blocking=True, graph=True)
            t0 = time.perf_counter()
            ctx.step_batch(ids, 3, blocking=True, graph=True)
            per = (time.perf_counter() - t0) / 3
            steps = max(3, int(seconds / 2 / max(per, 1e-6)))
            t0 = time.perf_counter()
            ctx.step_batch(ids, steps, blocking=True, graph=True)
            el = time.perf_counter() - t0
            rate = count * 6912 * steps / el
            row[label] = {"walks": count, "steps": steps, "flip_evals_per_s": rate,
                          "vs_A100": rate / PAPER_A100_NSE[L]}
            ctx.free_walks(ids)
        log(f"paper sweep L={L}: one walk {row['one_walk']['flip_evals_per_s']:.3g}, "
            f"batch {row['batch']['flip_evals_per_s']:.3g} flip-evals/s")
        rows.append(row)
    ctx.close()
    return {"study": "paper-settings speed sweep (Table 4 settings)", "rows": rows}


def run_alpha_ablation(libpsl, nse: float, runs: int) -> dict:
    """Table 2's alpha study at a reduced budget: L = 65535, N_lmt = 6912,
    LS_lmt = 2000, FLIP_lmt = 10, the switch rule of Algorithm 1; alpha_1 /
    alpha_2 = 4/13, 4/4 and 13/13, `runs` walks each (all stepped as one
    batch), each stopped after `nse` sequence evaluations. Reports the best
    PSL found per walk."""
    import numpy as np

    import seeded_inputs as si
    L, n_lmt = 65535, 6912
    configs = [(4, 13), (4, 4), (13, 13)]
    ctx = libpsl.Context(0)
    ids = {}
    for c, (a1, a2) in enumerate(configs):
        ids[(a1, a2)] = ctx.init_walks(L, runs, si.BASE_SEED + 10000 * (c + 1), alpha1=a1, alpha2=a2,
                                       n_lmt=n_lmt, ls_lmt=2000, flip_lmt=10, switch_period=0)
    every = [w for v in ids.values() for w in v]
    steps = int(nse // n_lmt)
    done, chunk = 0, 2000
    t0 = time.perf_counter()
    while done < steps:
        k = min(chunk, steps - done)
        ctx.step_batch(every, k, blocking=True, graph=True)
        done += k
        log(f"alpha ablation: {done}/{steps} steps, {time.perf_counter() - t0:.0f} s")
    el = time.perf_counter() - t0
    out = {"study": "alpha ablation (Table 2 settings, reduced budget)", "L": L, "n_lmt": n_lmt,
           "runs_per_config": runs, "nse_per_run": steps * n_lmt, "wall_s": el,
           "flip_evals_per_s": len(every) * n_lmt * steps / el, "configs": {}}
    for (a1, a2), ws in ids.items():
        p = np.array([ctx.read_walk(w, bits=False, C=False)["psl_best"] for w in ws])
        key = f"{a1}/{a2}"
        out["configs"][key] = {"psl_mean": float(p.mean()), "psl_std": float(p.std(ddof=1)) if len(p) > 1 else 0.0,
                               "psl_min": int(p.min()), "psl_max": int(p.max()),
                               "paper_psl_mean_at_1e10": PAPER_ALPHA_MEAN_PSL[key]}
    ctx.close()
    return out


def run_restart_study(libpsl, L: int, rounds: int, walks: int, nse: float) -> dict:
    """The restart protocol of Section 4 (the Table 5 runs), scaled down:
    Table 4's settings (N_lmt = 6912, alpha 4 / alpha2 by L, LS_lmt = 2000,
    FLIP_lmt = 10, the switch rule of Algorithm 1); round 0 starts `walks`
    walks from random sequences, every later round starts `walks` walks (new
    seeds) from the best sequence the previous round found. Each walk of a
    round is stopped after `nse` sequence evaluations."""
    import numpy as np

    import seeded_inputs as si
    n_lmt = min(L, 6912)
    steps = int(nse // n_lmt)
    ctx = libpsl.Context(0)
    out = {"study": "restart from the best sequence (Section 4 protocol, reduced budget)", "L": L,
           "n_lmt": n_lmt, "alpha1": 4, "alpha2": si.alpha2_for(L), "walks_per_round": walks,
           "nse_per_walk_per_round": steps * n_lmt, "rounds": []}
    best_bits, best_psl = None, None
    t_all = time.perf_counter()
    for r in range(rounds):
        init = None if best_bits is None else [best_bits] * walks
        ids = ctx.init_walks(L, walks, si.BASE_SEED + 20000 + 1000 * r, alpha1=4, alpha2=si.alpha2_for(L),
                             n_lmt=n_lmt, ls_lmt=2000, flip_lmt=10, switch_period=0, init_bits=init)
        start_psl = [ctx.read_walk(w, bits=False, C=False)["psl_best"] for w in ids]
        if best_psl is not None:
            # every walk of the round starts at the sequence it was given
            assert all(p == best_psl for p in start_psl), (best_psl, set(start_psl))
        t0 = time.perf_counter()
        done = 0
        while done < steps:
            k = min(2000, steps - done)
            ctx.step_batch(ids, k, blocking=True, graph=True)
            done += k
        el = time.perf_counter() - t0
        got = [ctx.read_walk(w, C=False) for w in ids]
        p = np.array([g["psl_best"] for g in got])
        b = int(np.argmin(p))
        best_psl, best_bits = int(p[b]), np.array(got[b]["best"], dtype=np.uint64)
        out["rounds"].append({"round": r, "start_psl": int(min(start_psl)), "psl_best": best_psl,
                              "psl_mean": float(p.mean()), "psl_max": int(p.max()), "wall_s": el})
        log(f"restart round {r}: start {min(start_psl)}, best {best_psl}, mean {p.mean():.1f} ({el:.0f} s)")
        ctx.free_walks(ids)
    out["wall_s"] = time.perf_counter() - t_all
    ctx.close()
    return out


def explicit_updates(groups, wl, n_lmt_arg, nominal_per_step, steps, el):
    """The nominal C_k-updates counted by `value`'s companion figure include
    the shifts k > max(j, L-1-j), where neither neighbour of j exists and C'_k
    = C_k: the evaluation takes them from suffix sums instead of visiting
    them. For full neighbourhoods (every j once) the remaining, explicitly
    evaluated (j, k) pairs number L(L-1) - sum_j min(j, L-1-j) per walk; with
    a limited neighbourhood the count depends on each step's start, and None
    is returned."""
    if wl == "paper" or n_lmt_arg:
        return None
    def skipped(L):
        m = L // 2
        return m * m if L % 2 else m * (m - 1)
    explicit = sum(c * (L * (L - 1) - skipped(L)) for L, c in groups)
    return {"per_step": explicit, "per_s": explicit * steps / el,
            "fraction_of_nominal": explicit / nominal_per_step,
            "note": "shifts with at least one neighbour of j in bounds; the rest come from suffix sums"}


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "libpsl runs walks on one GPU (walks shard across GPUs with no communication, but that is not built); --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    import seeded_inputs as si
    from paper_2107_09801_amd import libpsl

    assert torch.cuda.is_available(), "bench needs a GPU"
    if args.study == "paper-sweep":
        print(json.dumps(run_paper_sweep(libpsl, args.sweep_seconds)), flush=True)
        return
    if args.study == "alpha-ablation":
        print(json.dumps(run_alpha_ablation(libpsl, args.nse, args.runs)), flush=True)
        return
    if args.study == "serve":
        print(json.dumps(run_serving(libpsl, args.serve_seconds, args.serve_rate, args.serve_nlmt,
                                     args.eval_items)), flush=True)
        return
    if args.study == "restart":
        print(json.dumps(run_restart_study(libpsl, args.L or 65535, args.rounds, args.walks or 64,
                                           args.restart_nse)), flush=True)
        return
    UNEVEN = [(14, 512), (15, 256), (16, 128), (17, 64), (18, 32), (19, 16), (20, 8)]
    wl = args.workload
    period, ls_lmt = args.switch_period, 2000
    if wl == "batched":
        groups = [(args.L or 131071, args.walks or 1024)]
    elif wl == "single":
        groups = [(args.L or 16383, args.walks or 1)]
    elif wl == "large":
        groups = [(args.L or 1048575, args.walks or 1)]
    elif wl == "uneven":
        groups = [(2 ** m - 1, c) for m, c in UNEVEN]
    else:  # paper: Table 4 settings
        groups = [(args.L or 131071, args.walks or 64)]
        period = 0
    ctx = libpsl.Context(0)
    if args.eval_items:
        ctx.set_option(libpsl.OPT_EVAL_ITEMS, args.eval_items)
    if args.split >= 0:
        ctx.set_option(libpsl.OPT_SPLIT, args.split)
    if args.tune_file:
        ctx.tune_load(args.tune_file)
    ids, evals_per_step, updates_per_step = [], 0, 0
    for L, count in groups:
        a2 = 10 if wl == "paper" else si.alpha2_for(L)
        n_lmt = min(L, 6912) if wl == "paper" else min(L, args.n_lmt or L)
        ids += ctx.init_walks(L, count, si.BASE_SEED + len(ids), alpha1=4, alpha2=a2, n_lmt=n_lmt,
                              ls_lmt=ls_lmt, flip_lmt=10, switch_period=period)
        evals_per_step += count * n_lmt
        updates_per_step += count * n_lmt * (L - 1)
    nw = len(ids)
    L, n_lmt = groups[0][0], (min(groups[0][0], 6912) if wl == "paper" else min(groups[0][0], args.n_lmt or groups[0][0]))
    a2 = 10 if wl == "paper" else si.alpha2_for(L)
    log(f"{nw} walks initialised ({wl})")
    if wl == "large":   # per-step PSL and psl_best of the walk (trace ring)
        ctx.trace_enable(ids[0], args.warmup + args.steps)
    if args.calib_copy_mb:
        n = args.calib_copy_mb << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log(f"calibration copy of {args.calib_copy_mb} MiB done")
    tuned = ctx.autotune(ids) if args.autotune else None
    if tuned is not None:
        log(f"autotuned: {tuned}")
    warm_s = 0.0
    if args.warmup:
        t0 = time.perf_counter()
        ctx.step_batch(ids, args.warmup, blocking=True, graph=args.graph)
        warm_s = time.perf_counter() - t0
        log(f"{args.warmup} warmup step(s) done")
    torch.cuda.synchronize()
    tm = None
    if args.graph:
        t0 = time.perf_counter()
        ctx.step_batch(ids, args.steps, blocking=True, graph=True)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ctx.timing_enable(True)          # one eager pass for the kernel's duration
        ctx.step_batch(ids, min(args.steps, 8), blocking=True)
        tm = ctx.timing_read()
        ctx.timing_enable(False)
    else:
        ctx.timing_enable(True)
        t0 = time.perf_counter()
        ctx.step_batch(ids, args.steps, blocking=True)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        tm = ctx.timing_read()
        ctx.timing_enable(False)
    log(f"{args.steps} timed step(s) in {el:.3f} s")
    st = ctx.read_walk(ids[0], bits=False, C=False)
    whole = None
    if wl == "batched" and args.warmup + args.steps < BATCHED_STEPS:
        # the rest of the configuration's 100 steps (a phase switch after
        # steps 50 and 100), so its whole run is timed too
        rest = BATCHED_STEPS - args.warmup - args.steps
        t0 = time.perf_counter()
        ctx.step_batch(ids, rest, blocking=True, graph=args.graph)
        torch.cuda.synchronize()
        rest_s = time.perf_counter() - t0
        st_end = ctx.read_walk(ids[0], bits=False, C=False)
        total_s = warm_s + el + rest_s
        whole = {"steps": BATCHED_STEPS, "s": total_s, "ms_per_step": total_s / BATCHED_STEPS * 1e3,
                 "flip_evals_per_s": evals_per_step * BATCHED_STEPS / total_s,
                 "switches_after_steps": [t for t in range(1, BATCHED_STEPS + 1) if period and t % period == 0],
                 "walk0_after": {"t": st_end["t"], "q": st_end["q"], "psl_best": st_end["psl_best"],
                                 "alpha": st_end["alpha"]},
                 "note": "warmup, timed and remaining steps of the configuration's 100 steps, each "
                         "bracketed by a device sync (wall clock)"}
        log(f"whole run: {BATCHED_STEPS} steps in {total_s:.3f} s")

    value = evals_per_step * args.steps / el
    launches = max(1, tm["eval_launches"])
    eval_avg_s = tm["eval_ms"] / launches / 1e3
    lin_avg_s = tm["lin_ms"] / launches / 1e3
    prep_avg_s = tm["prep_ms"] / launches / 1e3
    split_work = sum(count * min(L_, args.n_lmt or L_) * (L_ - 1) for L_, count in groups if L_ >= SPLIT_MIN_L)
    if wl == "paper":
        split_work = sum(count * min(L_, 6912) * (L_ - 1) for L_, count in groups if L_ >= SPLIT_MIN_L)
    split_on = split_work > 0 and (args.split == 1 or (args.split in (-1, 2) and split_work >= SPLIT_MIN_WORK))
    tag = f"{wl}_L{'-'.join(str(g[0]) for g in groups)}_w{nw}" + ("" if split_on else "_table")
    valu = measured_valu(tag)
    if valu is not None:
        roof_eval = {"kernel": "k_eval", "bound": "alu", "achieved": valu * 64 / eval_avg_s / 1e12,
                     "peak": PEAK_LANE_OPS / 1e12, "unit": "Tlane-op/s",
                     "frac": valu * 64 / eval_avg_s / PEAK_LANE_OPS,
                     "traffic": measured_traffic(tag, "k_eval"), "traffic_unit": "B/launch",
                     "basis": "VALU lane-ops per launch (SQ_INSTS_VALU x 64, the valu-record of the "
                              "kernel's committed counter profile) / the launch time measured here"}
    else:
        roof_eval = {"kernel": "k_eval", "bound": "alu", "achieved": None, "peak": PEAK_LANE_OPS / 1e12,
                     "unit": "Tlane-op/s", "frac": None, "traffic": measured_traffic(tag, "k_eval"),
                     "traffic_unit": "B/launch",
                     "basis": "no SQ_INSTS_VALU record for these kernel sources and this workload"}
    roof_lin = None
    if split_on and lin_avg_s > 0:
        # algorithmic int8 ops of one launch: every (element, neighbour) term
        # of the evaluated elements of the split walks, 8 digit products each
        ops = LIN_OPS_PER_TERM * split_work
        roof_lin = {"kernel": "k_lin", "bound": "mfma", "achieved": ops / lin_avg_s / 1e12,
                    "peak": PEAK_INT8_OPS / 1e12, "unit": "TOP/s", "frac": ops / lin_avg_s / PEAK_INT8_OPS,
                    "traffic": measured_traffic(tag, "k_lin"), "traffic_unit": "B/launch",
                    "ops_per_launch": ops,
                    "basis": "16 int8 ops (8 digit multiply-adds) per (element, neighbour) term of the "
                             "linear part / the launch time measured here, against the dense int8 peak"}
    roofline = roof_eval if roof_lin is None or eval_avg_s >= lin_avg_s else roof_lin
    direct = OPS_PER_UPDATE_DIRECT * updates_per_step / eval_avg_s
    tiles, ks = ctx.eval_shape(L, n_lmt, nw)
    names = {"batched": "batched uniform", "single": "single walk", "large": "large single instance",
             "uneven": "uneven batch", "paper": "paper settings (Table 4)"}
    desc = (f"{names[wl]}: {nw} walks, L={'/'.join(str(g[0]) for g in groups)}, "
            f"N_lmt={'min(L,6912)' if wl == 'paper' else ('L' if not args.n_lmt else args.n_lmt)}, "
            f"alpha 4/{'10' if wl == 'paper' else 'by L'}, "
            f"{'paper switch rule LS_lmt=2000' if period == 0 else f'switch every {period} steps'}, "
            f"FLIP_lmt 10, FP64 F{', graph replay' if args.graph else ''}")

    out = {
        "metric": "flip-evals/s",
        "value": value,
        "unit": "flip-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i32+f64",
        "data": "synthetic",
        "config": {"workload": desc, "walks": nw, "L": [g[0] for g in groups],
                   "walks_per_L": [g[1] for g in groups], "n_lmt": n_lmt, "alpha1": 4,
                   "alpha2": a2, "switch_period": period, "eval_tiles": tiles, "eval_ksplit": ks,
                   **({"eval_items": args.eval_items} if args.eval_items else {})},
        "C_k_updates_per_s": updates_per_step * args.steps / el,
        "C_k_updates_explicit": explicit_updates(groups, wl, args.n_lmt, updates_per_step, args.steps, el),
        "eval_kernel": {"avg_ms": eval_avg_s * 1e3, "launches": tm["eval_launches"],
                        "updates_per_s": updates_per_step / eval_avg_s,
                        "split": split_on,
                        "split_prep_avg_ms": prep_avg_s * 1e3, "lin_avg_ms": lin_avg_s * 1e3,
                        "rest_of_step_avg_ms": tm["rest_ms"] / max(1, tm["steps"])},
        "roofline": roofline,
        "roofline_by_kernel": [r for r in (roof_eval, roof_lin) if r is not None],
        "vs_direct_form": {"direct_lane_ops_per_update": OPS_PER_UPDATE_DIRECT,
                           "nominal_updates_per_s": updates_per_step / eval_avg_s,
                           "ceiling_updates_per_s": PEAK_LANE_OPS / OPS_PER_UPDATE_DIRECT,
                           "ratio": direct / PEAK_LANE_OPS,
                           "lane_ops_per_nominal_update": (valu * 64 / updates_per_step) if valu else None,
                           "note": "nominal C_k-updates/s of the evaluation against the ceiling of the "
                                   "direct form (4 VALU lane-ops per update); above 1 because the kernel "
                                   "skips the unchanged shifts and resolves 2 or 4 shifts per table lookup"},
        "walk0_after": {"t": st["t"], "psl_best": st["psl_best"], "alpha": st["alpha"]},
    }
    if whole is not None:
        out["whole_run"] = whole
    if tuned is not None:
        out["autotune"] = tuned
    if wl == "large":
        out["walk0_trace"] = [{k: e[k] for k in ("t", "psl_k", "psl_best", "value_step", "alpha")}
                              for e in ctx.trace_read(ids[0], args.warmup + args.steps)]
    if L in PAPER_A100_NSE and len(groups) == 1:
        out["paper_context"] = {"A100_flip_evals_per_s": PAPER_A100_NSE[L],
                                "note": "paper Table 4: one walk, N_lmt=6912, alpha 4/10"}
        if wl == "paper":
            out["vs_paper_table4"] = value / PAPER_A100_NSE[L]
    ctx.close()
    if wl != "batched":
        args.serve_seconds, args.compare_jobs = 0, 0
    if args.serve_seconds > 0:
        log(f"serving run: {args.serve_rate:g} jobs/s for {args.serve_seconds:g} s")
        out["serving"] = run_serving(libpsl, args.serve_seconds, args.serve_rate, args.serve_nlmt)
    if args.compare_jobs > 0:
        log(f"served vs one-walk-per-launch on {args.compare_jobs} jobs")
        out["served_vs_single"] = run_compare(libpsl, args.compare_jobs, args.serve_nlmt)
    if wl == "uneven" and args.compare_uneven_steps > 0:
        log(f"uneven batch vs one-walk-per-launch, {args.compare_uneven_steps} step(s)")
        out["uneven_vs_single"] = run_uneven_compare(libpsl, groups, args.compare_uneven_steps, period)
    if not args.no_cpu_baseline:
        log("timing the oracle on a sample")
        out["cpu_baseline"] = cpu_baseline(L, n_lmt, 4, args.cpu_seconds, nw)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
