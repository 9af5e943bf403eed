"""Parity at the benchmark workloads' full sizes, in the launch shapes the bench
uses, against the oracle on sampled outputs or on properties that hold at any
size.

* L = 16383, one walk, full neighbourhood, alpha 4/13, switch every 50 steps:
  the 200-step trajectory in lockstep with the oracle.
* L = 131071, 1024 walks: walks 0, 511 and 1023 after steps 1, 2 and 3.
* L = 131071, 64 walks at Table 4's settings (N_lmt = 6912, alpha 4/10, the
  switch rule of Algorithm 1): walks 0 and 63 after steps 1, 2 and 3.
* L = 1048575, one walk, alpha 4/10: sampled neighbours of step 1 against the
  oracle, the choice against the full F/PSL arrays, the O(L) flip against the
  oracle's formula tier, and the correlation invariants.
* The uneven batch (L = 2^m - 1, m = 14..20, 512..8 walks): one walk per m
  stepped alone equals the same walk stepped inside the batch; for m <= 16
  also equal to the oracle.
"""
import numpy as np
import pytest

import oracle
import seeded_inputs as si

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
    compared = 0
    for t in range(200):
        ctx.step_batch([w], 1)
        tr = ow.step()
        if tr["flags"] & (oracle.AMBIG_ARGMIN | oracle.AMBIG_COMPARE):
            print(f"step {t}: oracle flags an ambiguous decision; stop comparing")
            break
        full = (t % 10 == 9) or (tr["flags"] & oracle.SWITCHED)
        g = ctx.read_walk(w, bits=bool(full), C=bool(full))
        _check_against_oracle(g, ow.read() if full else None, tr, t)
        compared += 1
    assert compared >= 190
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


def test_single_walk_L1048575_step1(ctx):
    import torch
    L, seed = 1048575, si.walk_seed(0)
    (w,) = ctx.init_walks(L, 1, seed, alpha1=4, alpha2=10, n_lmt=0, flip_lmt=10, switch_period=50)
    g0 = ctx.read_walk(w)
    s = oracle.rand_pivot(seed, L)
    assert np.array_equal(g0["pivot"], oracle.seq_to_bits(s))
    C0 = g0["C"].astype(np.int64)
    # invariants of Eq. (2) for the device's C (a from-scratch C is O(L^2))
    k = np.arange(L)
    assert C0[0] == L and C0[L - 1] == int(s[0]) * int(s[L - 1])
    assert np.all((C0 - (L - k)) % 2 == 0) and np.all(np.abs(C0) <= L - k)
    assert int(s.astype(np.int64).sum()) ** 2 == L + 2 * int(C0[1:].sum())
    C0 = C0.astype(np.int32)
    # the full neighbourhood of step 1, as the step evaluates it
    start = oracle.draw(seed, 1 << 60) % L
    F = torch.empty(L, dtype=torch.float64, device="cuda:0")
    P = torch.empty(L, dtype=torch.int32, device="cuda:0")
    ch = ctx.eval_neighbourhood(w, start, L, F, P)
    Fg, Pg = F.cpu().numpy(), P.cpu().numpy()
    for i0 in (0, 1, L // 3, L // 2 - 3, max(0, L - 1 - start - 2), L - 9):
        Fo, Po = oracle.eval_neighbourhood(s, C0, 4, (start + i0) % L, 8, nthreads=THREADS)
        assert np.array_equal(Pg[i0:i0 + 8], Po), i0
        assert np.max(np.abs(Fg[i0:i0 + 8] - Fo) / Fo) <= F_RTOL, i0
    # the choice, by the band rule over the full arrays
    fmin = Fg.min()
    inband = np.nonzero(Fg <= fmin * (1 + oracle.TAU))[0]
    assert ch["i_best"] == inband[0] and ch["F_min"] == fmin
    assert ch["psl_min"] == Pg.min() and ch["j_psl"] == (start + int(np.argmin(Pg)) + 1) % L
    Fo, Po = oracle.eval_neighbourhood(s, C0, 4, (start + ch["i_best"]) % L, 1, nthreads=1)
    assert abs(Fo[0] - ch["F_best"]) <= F_RTOL * Fo[0] and Po[0] == ch["psl_k"]
    # one step: the move and the O(L) flip
    ctx.step_batch([w], 1)
    g1 = ctx.read_walk(w)
    kb = ch["j_best"]
    assert g1["last_k"] == kb and g1["last_start"] == start
    assert np.array_equal(g1["C"], oracle.flip_corr_formula(s, C0, kb))
    s1 = s.copy()
    s1[kb] = -s1[kb]
    assert np.array_equal(g1["pivot"], oracle.seq_to_bits(s1))
    assert g1["psl_best"] == min(oracle.psl(C0), ch["psl_min"])
    assert g1["psl_pivot"] == oracle.psl(g1["C"]) == ch["psl_k"]
    ctx.free_walks([w])


UNEVEN = [(14, 512), (15, 256), (16, 128), (17, 64), (18, 32), (19, 16), (20, 8)]


def test_uneven_batch_alone_equals_mixed(ctx):
    ids, first = [], {}
    for m, count in UNEVEN:
        L = 2 ** m - 1
        w = ctx.init_walks(L, count, si.BASE_SEED + 1000 * m, alpha1=4, alpha2=si.alpha2_for(L),
                           n_lmt=0, flip_lmt=10, switch_period=50)
        first[m] = w[0]
        ids += w
    alone = {}
    for m, _ in UNEVEN:
        L = 2 ** m - 1
        (a,) = ctx.init_walks(L, 1, si.BASE_SEED + 1000 * m, alpha1=4, alpha2=si.alpha2_for(L),
                              n_lmt=0, flip_lmt=10, switch_period=50)
        alone[m] = a
    for t in range(2):
        ctx.step_batch(ids, 1)
        for m, _ in UNEVEN:
            ctx.step_batch([alone[m]], 1)
        for m, _ in UNEVEN:
            ga, gb = ctx.read_walk(alone[m]), ctx.read_walk(first[m])
            for key in ("pivot", "C", "best", "local_best"):
                assert np.array_equal(ga[key], gb[key]), (m, t, key)
            assert ga["last_k"] == gb["last_k"] and ga["psl_best"] == gb["psl_best"], (m, t)
            assert abs(ga["last_value_step"] - gb["last_value_step"]) <= F_RTOL * ga["last_value_step"]
    # oracle trajectories for the smaller sizes
    for m in (14, 15, 16):
        L = 2 ** m - 1
        ow = oracle.Walk(oracle.WalkConfig(L=L, seed=si.BASE_SEED + 1000 * m, alpha1=4,
                                           alpha2=si.alpha2_for(L), n_lmt=L, flip_lmt=10,
                                           switch_period=50), margin=MARGIN, nthreads=THREADS)
        tr = [ow.step(), ow.step()]
        assert not any(x["flags"] & (oracle.AMBIG_ARGMIN | oracle.AMBIG_COMPARE) for x in tr)
        _check_against_oracle(ctx.read_walk(first[m]), ow.read(), tr[1], m)
    ctx.free_walks(ids + list(alone.values()))
