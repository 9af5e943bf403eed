"""Writes the full-size parity goldens: oracle trajectories of the benchmark
workloads at their real sizes, so the GPU tests compare against the oracle's
own arithmetic (its O(L^2) correlations included) without rerunning it.

Calls only the oracle (and the seeded input parameters). Every value written
comes from `oracle.Walk`, which follows Algorithm 1 step by step with Eq. (2)
by definition at init and after a switch, the one-element flip of Section 3
for every neighbour and move, and Eq. (5) by Neumaier summation.

    python tests/golden/make_fullsize.py [case ...]

Cases (each a JSON file beside this script):
  large    one walk at L = 2^20 - 1 (seed 210709801, alpha 4/10, full
           neighbourhood, a switch every 50 steps): its initial state and
           steps 1-3;
  uneven   the first walk of every length group of the uneven batch
           (L = 2^m - 1, m = 14..20, seed 210709801 + 1000 m, alpha 4 and
           alpha_2 by L, full neighbourhood, a switch every 50 steps): steps
           1-2;
  serve    the ten longest jobs of the 50-job serving-mixture sample
           (N_lmt = min(L, 256), a switch every 50 steps): the state after
           each job's step budget.

Per step it records the start, the move, F and PSL of the move, the minimum
F, the best-PSL neighbour, psl_best, alpha, unimproved, v_local, the oracle's
flags, and SHA-256 digests of C (int32, little-endian) and of the pivot,
local-best and best sequences (packed 64-bit words, little-endian). Floats
are written with Python's round-trip repr.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import seeded_inputs as si  # noqa: E402

MARGIN = 5e-13          # the ambiguity margin the parity tests use
THREADS = os.cpu_count() or 1


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).astype(a.dtype.newbyteorder("<")).tobytes()).hexdigest()


def state_record(w: oracle.Walk) -> dict:
    o = w.read()
    return {"t": o["t"], "q": o["q"], "alpha": o["alpha"], "psl_best": o["psl_best"],
            "psl_pivot": o["psl_pivot"], "unimproved": o["unimproved"],
            "value_local": o["value_local"], "F_pivot": o["F_pivot"],
            "sha_C": sha(o["C"]), "sha_pivot": sha(o["pivot"]),
            "sha_local_best": sha(o["local_best"]), "sha_best": sha(o["best"])}


def trajectory(cfg: oracle.WalkConfig, steps: int, label: str) -> dict:
    t0 = time.time()
    w = oracle.Walk(cfg, margin=MARGIN, nthreads=THREADS)
    rec = {"cfg": {"L": cfg.L, "seed": cfg.seed, "alpha1": cfg.alpha1, "alpha2": cfg.alpha2,
                   "n_lmt": cfg.n_lmt, "ls_lmt": cfg.ls_lmt, "flip_lmt": cfg.flip_lmt,
                   "switch_period": cfg.switch_period},
           "init": state_record(w), "steps": []}
    print(f"{label}: init in {time.time() - t0:.0f} s", flush=True)
    for t in range(steps):
        tr = w.step()
        step = {k: tr[k] for k in ("start", "k", "value_step", "F_min", "psl_k", "j_psl", "psl_min",
                                   "psl_best", "alpha", "unimproved", "value_local", "flags")}
        step["state"] = state_record(w)
        rec["steps"].append(step)
        print(f"{label}: step {t + 1} done at {time.time() - t0:.0f} s (flags {tr['flags']})", flush=True)
    return rec


def case_large() -> dict:
    L = 1048575
    cfg = oracle.WalkConfig(L=L, seed=si.walk_seed(0), alpha1=4, alpha2=si.alpha2_for(L), n_lmt=L,
                            ls_lmt=2000, flip_lmt=10, switch_period=50)
    return {"large_L1048575": trajectory(cfg, 3, "large")}


UNEVEN = [(14, 512), (15, 256), (16, 128), (17, 64), (18, 32), (19, 16), (20, 8)]


def case_uneven() -> dict:
    out = {}
    for m, _ in UNEVEN:
        L = 2 ** m - 1
        cfg = oracle.WalkConfig(L=L, seed=si.BASE_SEED + 1000 * m, alpha1=4, alpha2=si.alpha2_for(L),
                                n_lmt=L, ls_lmt=2000, flip_lmt=10, switch_period=50)
        out[f"m{m}"] = trajectory(cfg, 2, f"uneven m={m}")
    return out


def case_serve() -> dict:
    jobs = si.serve_mixture_50()
    order = sorted(range(len(jobs)), key=lambda i: (-jobs[i]["L"], i))[:10]
    out = {}
    for i in order:
        j = jobs[i]
        cfg = oracle.WalkConfig(L=j["L"], seed=j["seed"], alpha1=4, alpha2=j["alpha2"], n_lmt=j["n_lmt"],
                                ls_lmt=2000, flip_lmt=min(10, j["L"]), switch_period=50)
        t0 = time.time()
        w = oracle.Walk(cfg, margin=MARGIN, nthreads=THREADS)
        flags = 0
        for _ in range(j["budget"]):
            flags |= w.step()["flags"]
        rec = {"job_index": i, "L": j["L"], "seed": j["seed"], "budget": j["budget"], "n_lmt": j["n_lmt"],
               "alpha2": j["alpha2"], "flags_or": flags, "final": state_record(w)}
        out[f"job{i}"] = rec
        print(f"serve job {i} (L={j['L']}, {j['budget']} steps) in {time.time() - t0:.0f} s", flush=True)
    return out


CASES = {"large": case_large, "uneven": case_uneven, "serve": case_serve}


def main(argv):
    names = argv or list(CASES)
    for name in names:
        data = CASES[name]()
        path = os.path.join(HERE, f"fullsize_{name}.json")
        with open(path + ".tmp", "w") as f:
            json.dump({"generator": "tests/golden/make_fullsize.py", "oracle": "oracle/psl_oracle.c",
                       "cases": data}, f, indent=1, sort_keys=True)
            f.write("\n")
        os.replace(path + ".tmp", path)
        print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
