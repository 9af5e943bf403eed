"""Parity at the benchmark workloads' full sizes, in the launch shapes the bench
uses, against the oracle: run live where it finishes in seconds, else from
the committed goldens (tests/golden/fullsize_*.json, written from the oracle
alone by tests/golden/make_fullsize.py, its O(L^2) correlations included).

* L = 16383, one walk, full neighbourhood, alpha 4/13, switch every 50 steps:
  the 200-step trajectory in lockstep with the oracle.
* L = 131071, 1024 walks: walks 0, 511 and 1023 after steps 1, 2 and 3.
* L = 131071, 64 walks at Table 4's settings (N_lmt = 6912, alpha 4/10, the
  switch rule of Algorithm 1): walks 0 and 63 after steps 1, 2 and 3.
* L = 1048575, one walk, alpha 4/10: the initial C, pivot, F and PSL and
  steps 1-3 against the oracle's goldens (C and the sequences by SHA-256);
  then sampled neighbours of the next step against the oracle on the C the
  goldens pinned, and the choice against the full F/PSL arrays.
* The uneven batch (L = 2^m - 1, m = 14..20, 512..8 walks) in one launch per
  step: the first walk of every m after steps 1 and 2 against the goldens,
  and the same walks stepped alone equal to the walks in the batch.
"""
import numpy as np
import pytest

import goldens
import oracle
import seeded_inputs as si
from lockstep import run_lockstep

pytestmark = pytest.mark.gpu

F_RTOL = 1e-12
MARGIN = 5e-13
THREADS = 16


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2107_09801_amd import libpsl
    assert torch.cuda.is_available()
    c = libpsl.Context(0)
    yield c
    c.close()


def _check_against_oracle(g, ow_state, tr, t):
    assert g["last_start"] == tr["start"], t
    assert g["last_k"] == tr["k"], t
    assert abs(g["last_value_step"] - tr["value_step"]) <= F_RTOL * tr["value_step"], t
    assert g["psl_best"] == tr["psl_best"] and g["alpha"] == tr["alpha"], t
    assert g["unimproved"] == tr["unimproved"], t
    if ow_state is not None:
        for key in ("pivot", "C", "local_best", "best"):
            assert np.array_equal(g[key], ow_state[key]), (t, key)


def test_single_walk_L16383_200_steps_lockstep(ctx):
    L, seed = 16383, si.walk_seed(0)
    (w,) = ctx.init_walks(L, 1, seed, alpha1=4, alpha2=13, n_lmt=0, flip_lmt=10, switch_period=50)
    ow = oracle.Walk(oracle.WalkConfig(L=L, seed=seed, alpha1=4, alpha2=13, n_lmt=L, flip_lmt=10,
                                       switch_period=50), margin=MARGIN, nthreads=THREADS)
    compared, imposed = run_lockstep(ctx, w, ow, 200, check_every=10)
    assert compared + imposed == 200 and compared >= 190
    ctx.free_walks([w])


def test_batch_1024_L131071_sampled_walks(ctx):
    L, nw = 131071, 1024
    ids = ctx.init_walks(L, nw, si.BASE_SEED, alpha1=4, alpha2=13, n_lmt=0, flip_lmt=10,
                         switch_period=50)
    sample = [0, 511, 1023]
    ows = {b: oracle.Walk(oracle.WalkConfig(L=L, seed=si.walk_seed(b), alpha1=4, alpha2=13, n_lmt=L,
                                            flip_lmt=10, switch_period=50),
                          margin=MARGIN, nthreads=THREADS) for b in sample}
    for b in sample:
        g = ctx.read_walk(ids[b])
        o = ows[b].read()
        assert np.array_equal(g["pivot"], o["pivot"]) and np.array_equal(g["C"], o["C"])
    for t in range(3):
        ctx.step_batch(ids, 1)
        for b in sample:
            tr = ows[b].step()
            assert not tr["flags"] & (oracle.AMBIG_ARGMIN | oracle.AMBIG_COMPARE)
            _check_against_oracle(ctx.read_walk(ids[b]), ows[b].read(), tr, (b, t))
    ctx.free_walks(ids)


def test_paper_settings_64_walks_L131071_sampled(ctx):
    """The limited neighbourhood at full size: 6912 candidates from a random
    start, 16-wavefront blocks and many k-splits per walk."""
    L, nw, n_lmt = 131071, 64, 6912
    ids = ctx.init_walks(L, nw, si.BASE_SEED, alpha1=4, alpha2=10, n_lmt=n_lmt, ls_lmt=2000, flip_lmt=10,
                         switch_period=0)
    sample = [0, 63]
    ows = {b: oracle.Walk(oracle.WalkConfig(L=L, seed=si.walk_seed(b), alpha1=4, alpha2=10, n_lmt=n_lmt,
                                            ls_lmt=2000, flip_lmt=10, switch_period=0),
                          margin=MARGIN, nthreads=THREADS) for b in sample}
    for t in range(3):
        ctx.step_batch(ids, 1)
        for b in sample:
            tr = ows[b].step()
            assert not tr["flags"] & (oracle.AMBIG_ARGMIN | oracle.AMBIG_COMPARE)
            _check_against_oracle(ctx.read_walk(ids[b]), ows[b].read(), tr, (b, t))
    ctx.free_walks(ids)


def test_single_walk_L1048575_goldens(ctx):
    """The large single instance against the oracle's own trajectory: its
    initial state (C from the O(L^2) definition) and steps 1-3."""
    import torch
    gold = goldens.load("large")["large_L1048575"]
    cfg = gold["cfg"]
    L, seed = cfg["L"], cfg["seed"]
    assert (L, seed, cfg["alpha2"], cfg["switch_period"]) == (1048575, si.walk_seed(0), 10, 50)
    (w,) = ctx.init_walks(L, 1, seed, alpha1=cfg["alpha1"], alpha2=cfg["alpha2"], n_lmt=0,
                          ls_lmt=cfg["ls_lmt"], flip_lmt=cfg["flip_lmt"], switch_period=cfg["switch_period"])
    goldens.check_state(ctx.read_walk(w), gold["init"], F_RTOL, "init")
    for t, step in enumerate(gold["steps"]):
        assert not step["flags"] & (oracle.AMBIG_ARGMIN | oracle.AMBIG_COMPARE), t
        ctx.step_batch([w], 1)
        goldens.check_step(ctx.read_walk(w), step, F_RTOL, t + 1)
    # the next step's full neighbourhood: sampled neighbours against the
    # oracle on the C the goldens pinned, the choice against the full arrays
    g = ctx.read_walk(w)
    assert goldens.sha(g["C"]) == gold["steps"][-1]["state"]["sha_C"]
    s = si.to_pm1(g["pivot"], L)
    C = g["C"]
    alpha = g["alpha"]
    start = oracle.draw(seed, (1 << 60) | g["t"]) % L
    F = torch.empty(L, dtype=torch.float64, device="cuda:0")
    P = torch.empty(L, dtype=torch.int32, device="cuda:0")
    ch = ctx.eval_neighbourhood(w, start, L, F, P)
    Fg, Pg = F.cpu().numpy(), P.cpu().numpy()
    for i0 in (0, 1, L // 3, L // 2 - 3, max(0, L - 1 - start - 2), L - 9):
        Fo, Po = oracle.eval_neighbourhood(s, C, alpha, (start + i0) % L, 8, nthreads=THREADS)
        assert np.array_equal(Pg[i0:i0 + 8], Po), i0
        assert np.max(np.abs(Fg[i0:i0 + 8] - Fo) / Fo) <= F_RTOL, i0
    fmin = Fg.min()
    inband = np.nonzero(Fg <= fmin * (1 + oracle.TAU))[0]
    assert ch["i_best"] == inband[0] and ch["F_min"] == fmin
    assert ch["psl_min"] == Pg.min() and ch["j_psl"] == (start + int(np.argmin(Pg)) + 1) % L
    Fo, Po = oracle.eval_neighbourhood(s, C, alpha, (start + ch["i_best"]) % L, 1, nthreads=1)
    assert abs(Fo[0] - ch["F_best"]) <= F_RTOL * Fo[0] and Po[0] == ch["psl_k"]
    ctx.free_walks([w])


UNEVEN = [(14, 512), (15, 256), (16, 128), (17, 64), (18, 32), (19, 16), (20, 8)]


def test_uneven_batch_goldens_and_alone(ctx):
    """The uneven batch in one launch sequence per step: the first walk of
    every length group against the oracle's goldens after steps 1 and 2, and
    the same walks stepped alone equal to the walks in the batch."""
    gold = goldens.load("uneven")
    ids, first = [], {}
    for m, count in UNEVEN:
        L = 2 ** m - 1
        w = ctx.init_walks(L, count, si.BASE_SEED + 1000 * m, alpha1=4, alpha2=si.alpha2_for(L),
                           n_lmt=0, flip_lmt=10, switch_period=50)
        first[m] = w[0]
        ids += w
        cfg = gold[f"m{m}"]["cfg"]
        assert (cfg["L"], cfg["seed"], cfg["alpha2"]) == (L, si.BASE_SEED + 1000 * m, si.alpha2_for(L))
    alone = {}
    for m, _ in UNEVEN:
        L = 2 ** m - 1
        (a,) = ctx.init_walks(L, 1, si.BASE_SEED + 1000 * m, alpha1=4, alpha2=si.alpha2_for(L),
                              n_lmt=0, flip_lmt=10, switch_period=50)
        alone[m] = a
    for m, _ in UNEVEN:
        goldens.check_state(ctx.read_walk(first[m]), gold[f"m{m}"]["init"], F_RTOL, (m, "init"))
    for t in range(2):
        ctx.step_batch(ids, 1)
        for m, _ in UNEVEN:
            ctx.step_batch([alone[m]], 1)
        for m, _ in UNEVEN:
            step = gold[f"m{m}"]["steps"][t]
            assert not step["flags"] & (oracle.AMBIG_ARGMIN | oracle.AMBIG_COMPARE), (m, t)
            gb = ctx.read_walk(first[m])
            goldens.check_step(gb, step, F_RTOL, (m, t + 1))
            ga = ctx.read_walk(alone[m])
            for key in ("pivot", "C", "best", "local_best"):
                assert np.array_equal(ga[key], gb[key]), (m, t, key)
            assert ga["last_k"] == gb["last_k"] and ga["psl_best"] == gb["psl_best"], (m, t)
            assert abs(ga["last_value_step"] - gb["last_value_step"]) <= F_RTOL * ga["last_value_step"]
    ctx.free_walks(ids + list(alone.values()))
