"""GPU parity of libpsl against the CPU oracle (through the C-ABI).

Bars: C, PSL, bits and moves bit-exact; F within a relative 1e-12. A step
flagged ambiguous (a value within 5e-13 relative of a band edge) must carry
the same flag on both sides, and is resolved by imposing the oracle's state
on the GPU walk (tests/lockstep.py).
"""
import numpy as np
import pytest

import oracle
import seeded_inputs as si
from lockstep import run_lockstep as _lockstep

pytestmark = pytest.mark.gpu

F_RTOL = 1e-12
MARGIN = 5e-13


@pytest.fixture(scope="module", params=["auto", "dense"])
def ctx(request):
    """Two contexts: automatic PSL mode (near-peak list) and the in-loop max."""
    import torch
    from paper_2107_09801_amd import libpsl
    assert torch.cuda.is_available()
    c = libpsl.Context(0)
    if request.param == "dense":
        c.set_option(libpsl.OPT_NEAR_LIMIT, 0)
        c._dense = True
    yield c
    c.close()


def _dev(n, dtype):
    import torch
    return torch.empty(max(n, 1), dtype=dtype, device="cuda:0")


def _oracle_state(L, seed=None, bits=None):
    s = oracle.rand_pivot(seed, L) if bits is None else si.to_pm1(bits, L)
    return s, oracle.corr(s)


def _rel(a, b):
    return np.max(np.abs(np.asarray(a) - np.asarray(b)) / np.maximum(np.abs(np.asarray(b)), 1e-300))


# ------------------------------------------------------------------- init

@pytest.mark.parametrize("L", [2, 3, 4, 5, 13, 31, 63, 64, 65, 127, 1001, 4097, 16383])
def test_init_random_pivot_matches_oracle(ctx, L):
    seed = si.BASE_SEED + L
    (w,) = ctx.init_walks(L, 1, seed, alpha1=4, alpha2=13)
    g = ctx.read_walk(w)
    s, C = _oracle_state(L, seed)
    assert np.array_equal(g["pivot"], oracle.seq_to_bits(s))
    assert np.array_equal(g["C"], C)
    assert np.array_equal(g["local_best"], g["pivot"]) and np.array_equal(g["best"], g["pivot"])
    assert g["psl_best"] == oracle.psl(C) == g["psl_pivot"]
    F = oracle.fitness(C, 4)
    assert abs(g["value_local"] - F) <= F_RTOL * F and g["F_pivot"] == g["value_local"]
    assert g["alpha"] == 4 and g["t"] == 0 and g["unimproved"] == 0
    ctx.free_walks([w])


@pytest.mark.parametrize("kind", ["plus", "alternating", "biased", "random"])
@pytest.mark.parametrize("L", [2, 70, 3001])
def test_init_given_bits(ctx, L, kind):
    bits = {"plus": si.all_plus_bits(L), "alternating": si.alternating_bits(L),
            "biased": si.biased_bits(L, 5, 0.2), "random": si.random_bits(L, 6)}[kind]
    (w,) = ctx.init_walks(L, 1, 1, init_bits=[bits])
    g = ctx.read_walk(w)
    assert np.array_equal(g["pivot"], bits)
    assert np.array_equal(g["C"], oracle.corr(si.to_pm1(bits, L)))
    ctx.free_walks([w])


# -------------------------------------------------------- neighbourhood

EVAL_CASES = []
for L in [2, 3, 4, 5, 13, 31, 63, 64, 65, 127, 1001, 4097, 16383]:
    for start in sorted({0, L - 1, L // 2}):
        for n_lmt in sorted({1, min(7, L), min(256, L), L}):
            EVAL_CASES.append((L, start, n_lmt))


@pytest.mark.parametrize("L,start,n_lmt", EVAL_CASES)
def test_eval_neighbourhood_random_pivot(ctx, L, start, n_lmt):
    import torch
    seed = 77 + L
    alpha = 4 if (L + start) % 2 else 13
    (w,) = ctx.init_walks(L, 1, seed, alpha1=alpha, alpha2=4)
    F, P = _dev(n_lmt, torch.float64), _dev(n_lmt, torch.int32)
    ch = ctx.eval_neighbourhood(w, start, n_lmt, F, P)
    s, C = _oracle_state(L, seed)
    Fo, Po = oracle.eval_neighbourhood(s, C, alpha, start, n_lmt, nthreads=8)
    Fg, Pg = F.cpu().numpy()[:n_lmt], P.cpu().numpy()[:n_lmt]
    assert np.array_equal(Pg, Po)
    assert _rel(Fg, Fo) <= F_RTOL
    oc = oracle.select(Fo, Po, margin=MARGIN)
    assert ch["psl_min"] == oc.psl_min and ch["j_psl"] == (start + oc.i_psl + 1) % L
    if not oc.flags & oracle.AMBIG_ARGMIN:
        assert ch["i_best"] == oc.i_best
        assert ch["j_best"] == (start + oc.i_best + 1) % L
    assert ch["F_best"] == Fg[ch["i_best"]] and ch["psl_k"] == Pg[ch["i_best"]]
    assert ch["F_min"] == Fg.min()
    # pure: the walk is unchanged
    g = ctx.read_walk(w)
    assert np.array_equal(g["C"], C) and g["t"] == 0
    ctx.free_walks([w])


@pytest.mark.parametrize("kind", ["plus", "alternating", "biased"])
@pytest.mark.parametrize("alpha", [1, 2, 4, 10, 13, 16])
@pytest.mark.parametrize("L", [2, 33, 300, 2049])
def test_eval_structured_pivots(ctx, L, alpha, kind):
    import torch
    bits = {"plus": si.all_plus_bits(L), "alternating": si.alternating_bits(L),
            "biased": si.biased_bits(L, 11, 0.25)}[kind]
    (w,) = ctx.init_walks(L, 1, 1, alpha1=alpha, alpha2=4, init_bits=[bits])
    start = (L * 7) // 11
    F, P = _dev(L, torch.float64), _dev(L, torch.int32)
    ctx.eval_neighbourhood(w, start, L, F, P)
    s, C = _oracle_state(L, bits=bits)
    Fo, Po = oracle.eval_neighbourhood(s, C, alpha, start, L, nthreads=8)
    assert np.array_equal(P.cpu().numpy()[:L], Po)
    assert _rel(F.cpu().numpy()[:L], Fo) <= F_RTOL
    ctx.free_walks([w])


# ------------------------------------------------------------------ flip

@pytest.mark.parametrize("L", [2, 5, 64, 65, 1000, 16383])
def test_apply_flip_matches_formula(ctx, L):
    seed = 5 + L
    (w,) = ctx.init_walks(L, 1, seed, alpha1=13, alpha2=4)
    s, C = _oracle_state(L, seed)
    for j in sorted({0, L - 1, L // 3, (2 * L) // 3}):
        ctx.apply_flip(w, j)
        C = oracle.flip_corr_formula(s, C, j)
        s[j] = -s[j]
        g = ctx.read_walk(w)
        assert np.array_equal(g["C"], C)
        assert np.array_equal(g["pivot"], oracle.seq_to_bits(s))
        F = oracle.fitness(C, 13)
        assert abs(g["F_pivot"] - F) <= F_RTOL * F and g["psl_pivot"] == oracle.psl(C)
    assert np.array_equal(C, oracle.corr(s))
    ctx.free_walks([w])


# ------------------------------------------------------------ trajectories

@pytest.mark.parametrize("L,n_lmt,period,ls,steps", [
    (257, 257, 5, 2000, 60), (1001, 1001, 50, 2000, 120), (1001, 300, 0, 3, 80),
    (64, 64, 0, 2, 100), (2, 2, 3, 2000, 20), (5, 3, 0, 1, 40), (4097, 4097, 50, 2000, 60)])
def test_step_lockstep_with_oracle(ctx, L, n_lmt, period, ls, steps):
    seed = si.BASE_SEED + 3 * L + period
    flip = min(10, L)
    (w,) = ctx.init_walks(L, 1, seed, alpha1=4, alpha2=13, n_lmt=n_lmt, ls_lmt=ls,
                          flip_lmt=flip, switch_period=period)
    ow = oracle.Walk(oracle.WalkConfig(L=L, seed=seed, alpha1=4, alpha2=13, n_lmt=n_lmt,
                                       ls_lmt=ls, flip_lmt=flip, switch_period=period),
                     margin=MARGIN, nthreads=8)
    n, imposed = _lockstep(ctx, w, ow, steps)
    assert n + imposed == steps and n >= steps * 0.9
    ctx.free_walks([w])


@pytest.mark.parametrize("margin_fs", [10 ** 11, 10 ** 12])
@pytest.mark.parametrize("L,n_lmt,period,alpha2", [(257, 257, 7, 13), (1001, 300, 0, 4), (64, 64, 5, 2)])
def test_lockstep_imposes_oracle_on_flagged_steps(ctx, L, n_lmt, period, alpha2, margin_fs):
    """With a wide ambiguity margin (1e-4 or 1e-3 relative, on both sides)
    many steps are flagged: the GPU's flags must equal the oracle's, and the
    harness resolves each flagged step by imposing the oracle's state, after
    which the walks go on in lockstep."""
    from paper_2107_09801_amd import libpsl
    margin = margin_fs * 1e-15
    seed = si.BASE_SEED + 5 * L + alpha2
    flip = min(10, L)
    ctx.set_option(libpsl.OPT_AMBIG_MARGIN, margin_fs)
    try:
        (w,) = ctx.init_walks(L, 1, seed, alpha1=4, alpha2=alpha2, n_lmt=n_lmt, ls_lmt=3,
                              flip_lmt=flip, switch_period=period)
        ow = oracle.Walk(oracle.WalkConfig(L=L, seed=seed, alpha1=4, alpha2=alpha2, n_lmt=n_lmt,
                                           ls_lmt=3, flip_lmt=flip, switch_period=period),
                         margin=margin, nthreads=8)
        n, imposed = _lockstep(ctx, w, ow, 60, margin=margin)
        assert n + imposed == 60
        assert imposed >= 1, "the wide margin flagged no step"
        ctx.free_walks([w])
    finally:
        ctx.set_option(libpsl.OPT_AMBIG_MARGIN, -1)


@pytest.mark.parametrize("margin_fs", [0, 500, 10 ** 9, 10 ** 11, 10 ** 12, 10 ** 13])
@pytest.mark.parametrize("L,n_lmt,alpha", [(4097, 4097, 4), (16383, 16383, 13), (3001, 700, 2),
                                           (100000, 20000, 10)])
def test_choice_ambiguity_flag(ctx, L, n_lmt, alpha, margin_fs):
    """psl_choice.flags against the definition (some F within m*F_min of the
    band edge), evaluated on the GPU's own F array and on the oracle's; the
    margins run from 0 (exact hits only) to 1e-2, so both answers occur, and
    L up to 100000 puts the candidates in many combine blocks."""
    import torch
    from paper_2107_09801_amd import libpsl
    margin = margin_fs * 1e-15
    seed = 9000 + L + margin_fs % 97
    start = (L * 5) // 7
    ctx.set_option(libpsl.OPT_AMBIG_MARGIN, margin_fs)
    try:
        (w,) = ctx.init_walks(L, 1, seed, alpha1=alpha, alpha2=4)
        F, P = _dev(n_lmt, torch.float64), _dev(n_lmt, torch.int32)
        ch = ctx.eval_neighbourhood(w, start, n_lmt, F, P)
        Fg = F.cpu().numpy()[:n_lmt]
        thr = Fg.min() * (1 + oracle.TAU)
        want = bool(np.any(np.abs(Fg - thr) <= margin * Fg.min()))
        assert bool(ch["flags"] & libpsl.CHOICE_AMBIGUOUS_ARGMIN) == want
        s, C = _oracle_state(L, seed)
        Fo, Po = oracle.eval_neighbourhood(s, C, alpha, start, n_lmt, nthreads=8)
        oc = oracle.select(Fo, Po, margin=margin)
        if bool(oc.flags & oracle.AMBIG_ARGMIN) != want:
            # only a value at the window's edge, within the F tolerance, may differ
            edge = np.abs(np.abs(Fo - oc.F_min * (1 + oracle.TAU)) - margin * oc.F_min)
            assert np.min(edge) <= 1e-11 * oc.F_min
        if not want and not oc.flags & oracle.AMBIG_ARGMIN:
            assert ch["i_best"] == oc.i_best
        ctx.free_walks([w])
    finally:
        ctx.set_option(libpsl.OPT_AMBIG_MARGIN, -1)


def test_ambig_margin_option_range(ctx):
    from paper_2107_09801_amd import libpsl
    for bad in (-2, 10 ** 15 + 1):
        with pytest.raises(libpsl.PslError):
            ctx.set_option(libpsl.OPT_AMBIG_MARGIN, bad)
    for ok in (0, 10 ** 15, -1):
        ctx.set_option(libpsl.OPT_AMBIG_MARGIN, ok)


def test_batch_matches_single_walks(ctx):
    Ls = [2, 65, 257, 1001, 3000]
    solo, mixed = [], []
    for L in Ls:
        solo += ctx.init_walks(L, 1, 99 + L, n_lmt=0, switch_period=7, flip_lmt=min(3, L))
    for L in Ls:
        mixed += ctx.init_walks(L, 1, 99 + L, n_lmt=0, switch_period=7, flip_lmt=min(3, L))
    for w in solo:
        ctx.step_batch([w], 15)
    ctx.step_batch(mixed, 15)
    for a, b in zip(solo, mixed):
        ga, gb = ctx.read_walk(a), ctx.read_walk(b)
        for key in ("pivot", "C", "best", "local_best"):
            assert np.array_equal(ga[key], gb[key]), key
        for key in ("psl_best", "alpha", "unimproved", "t", "q", "last_k"):
            assert ga[key] == gb[key], key
        assert abs(ga["value_local"] - gb["value_local"]) <= F_RTOL * ga["value_local"]
    ctx.free_walks(solo + mixed)


@pytest.mark.parametrize("flip", [0, 1, 10, 40, 64, 65, 90])
def test_switch_every_step_against_oracle(ctx, flip):
    """Every walk of a mixed batch switches after every step, so every step
    rebuilds C from local_best's C through the pending list (FLIP_lmt <= 64:
    one-flip updates plus the fix-up of the shifts earlier flips touched;
    above 64: the full correlation). Each walk follows its oracle walk."""
    Ls = [70, 129, 500, 1200]
    ids, ows = [], []
    for L in Ls:
        seed = si.BASE_SEED + 11 * L + flip
        fl = min(flip, L)
        ids += ctx.init_walks(L, 1, seed, alpha1=4, alpha2=13, n_lmt=0, flip_lmt=fl, switch_period=1)
        ows.append(oracle.Walk(oracle.WalkConfig(L=L, seed=seed, alpha1=4, alpha2=13, n_lmt=L,
                                                 flip_lmt=fl, switch_period=1), margin=MARGIN, nthreads=8))
    for t in range(8):
        ctx.step_batch(ids, 1)
        for w, ow in zip(ids, ows):
            tr = ow.step()
            if tr["flags"] & (oracle.AMBIG_ARGMIN | oracle.AMBIG_COMPARE):
                pytest.skip("the oracle flags an ambiguous decision")
            assert tr["flags"] & oracle.SWITCHED
            g, o = ctx.read_walk(w), ow.read()
            for key in ("pivot", "C", "local_best", "best"):
                assert np.array_equal(g[key], o[key]), (t, key)
            assert g["alpha"] == o["alpha"] and g["psl_pivot"] == o["psl_pivot"], t
            assert abs(g["value_local"] - o["value_local"]) <= F_RTOL * o["value_local"], t
    ctx.free_walks(ids)


def test_invalid_arguments(ctx):
    from paper_2107_09801_amd import libpsl
    with pytest.raises(libpsl.PslError):
        ctx.init_walks(1, 1, 0)
    with pytest.raises(libpsl.PslError):
        ctx.init_walks(10, 1, 0, n_lmt=11)
    with pytest.raises(libpsl.PslError):
        ctx.init_walks(10, 1, 0, alpha1=0)
    (w,) = ctx.init_walks(10, 1, 0)
    with pytest.raises(libpsl.PslError):
        ctx.eval_neighbourhood(w, 10, 5)
    with pytest.raises(libpsl.PslError):
        ctx.eval_neighbourhood(w, 0, 11)
    with pytest.raises(libpsl.PslError):
        ctx.apply_flip(w, 10)
    with pytest.raises(libpsl.PslError):
        ctx.step_batch([w, w], 1)
    ctx.free_walks([w])
    with pytest.raises(libpsl.PslError):
        ctx.read_walk(w)


def test_empty_batches_and_range_edges(ctx):
    """Empty inputs are no-ops; configuration limits are enforced on the host."""
    from paper_2107_09801_amd import libpsl
    assert ctx.init_walks(1001, 0, 5) == []
    ctx.step_batch([], 3)
    (w,) = ctx.init_walks(1001, 1, 5)
    before = ctx.read_walk(w)
    ctx.step_batch([w], 0)
    after = ctx.read_walk(w)
    assert after["t"] == 0 and np.array_equal(after["C"], before["C"])
    assert np.array_equal(after["pivot"], before["pivot"])
    for bad in (dict(L=libpsl.L_MAX + 1), dict(L=1001, alpha1=17), dict(L=1001, alpha2=0),
                dict(L=1001, flip_lmt=1002), dict(L=3000, flip_lmt=1025)):
        L = bad.pop("L")
        with pytest.raises(libpsl.PslError):
            ctx.init_walks(L, 1, 5, **bad)
    # the limits themselves are accepted
    ids = ctx.init_walks(2, 1, 5, flip_lmt=2, alpha1=16, alpha2=1)
    ids += ctx.init_walks(3000, 1, 5, flip_lmt=1024)
    ctx.step_batch(ids, 2)
    for x in ids:
        g = ctx.read_walk(x)
        assert g["t"] == 2
        assert np.array_equal(g["C"], oracle.corr(si.to_pm1(g["pivot"], g["L"])))
    ctx.free_walks(ids + [w])


def test_eval_items_option_keeps_results(ctx):
    """More or fewer evaluation work items change only how the shifts are cut
    (the k-splits) and so F by rounding: PSL and the chosen move stay."""
    import torch
    from paper_2107_09801_amd import libpsl
    L, n_lmt, start = 20001, 20001, 777
    (w,) = ctx.init_walks(L, 1, 4242, alpha1=13, alpha2=4)
    s, C = _oracle_state(L, 4242)
    Fo, Po = oracle.eval_neighbourhood(s, C, 13, start, n_lmt, nthreads=8)
    oc = oracle.select(Fo, Po, margin=MARGIN)
    splits = set()
    try:
        for v in (1, 128, 4096, 65536, 262144):
            ctx.set_option(libpsl.OPT_EVAL_ITEMS, v)
            splits.add(ctx.eval_shape(L, n_lmt, 1)[1])
            F, P = _dev(n_lmt, torch.float64), _dev(n_lmt, torch.int32)
            ch = ctx.eval_neighbourhood(w, start, n_lmt, F, P)
            assert np.array_equal(P.cpu().numpy(), Po), v
            assert _rel(F.cpu().numpy(), Fo) <= F_RTOL, v
            assert ch["psl_min"] == oc.psl_min
            if not oc.flags & oracle.AMBIG_ARGMIN:
                assert ch["i_best"] == oc.i_best, v
        for bad in (0, -2, 262145):
            with pytest.raises(libpsl.PslError):
                ctx.set_option(libpsl.OPT_EVAL_ITEMS, bad)
    finally:
        ctx.set_option(libpsl.OPT_EVAL_ITEMS, -1)
    assert len(splits) >= 3          # the option reached the layout
    ctx.free_walks([w])


@pytest.mark.parametrize("L,n_lmt,items,ks_min", [(65535, 256, 0, 129), (131071, 64, 0, 257),
                                                   (262143, 64, 65536, 513)])
def test_eval_many_splits_small_neighbourhood(ctx, L, n_lmt, items, ks_min):
    """Few candidates over a long sequence (the serving shape) cut into many
    k-splits, which the combine adds with 16, 32 and 64 lanes per candidate
    (each lane's splits in order, then a fixed tree): F and PSL against the
    oracle, candidate by candidate."""
    import torch
    from paper_2107_09801_amd import libpsl
    seed, start, alpha = 900 + L % 97, L // 3, 13 if L % 2 else 4
    (w,) = ctx.init_walks(L, 1, seed, alpha1=alpha, alpha2=4)
    try:
        if items:
            ctx.set_option(libpsl.OPT_EVAL_ITEMS, items)
        assert ctx.eval_shape(L, n_lmt, 1)[1] >= ks_min
        F, P = _dev(n_lmt, torch.float64), _dev(n_lmt, torch.int32)
        ch = ctx.eval_neighbourhood(w, start, n_lmt, F, P)
    finally:
        ctx.set_option(libpsl.OPT_EVAL_ITEMS, -1)
    s, C = _oracle_state(L, seed)
    Fo, Po = oracle.eval_neighbourhood(s, C, alpha, start, n_lmt, nthreads=8)
    assert np.array_equal(P.cpu().numpy()[:n_lmt], Po)
    assert _rel(F.cpu().numpy()[:n_lmt], Fo) <= F_RTOL
    oc = oracle.select(Fo, Po, margin=MARGIN)
    assert ch["psl_min"] == oc.psl_min
    if not oc.flags & oracle.AMBIG_ARGMIN:
        assert ch["i_best"] == oc.i_best
    ctx.free_walks([w])


def test_graph_replays_match_eager(ctx):
    """One captured step replayed many times, with eager work and syncs between
    replays, equals the eager path after every replay."""
    Ls = [2, 257, 1001, 5000]
    eager, graph = [], []
    for L in Ls:
        eager += ctx.init_walks(L, 1, 4242 + L, n_lmt=0, switch_period=4, flip_lmt=min(3, L))
    for L in Ls:
        graph += ctx.init_walks(L, 1, 4242 + L, n_lmt=0, switch_period=4, flip_lmt=min(3, L))
    other = ctx.init_walks(300, 2, 7, n_lmt=0)
    for r in range(9):
        ctx.step_batch(eager, 1)
        ctx.step_batch(graph, 1 + (r % 2), graph=True)
        if r % 2 == 1:
            ctx.step_batch(eager, 1)
        ctx.step_batch(other, 1)          # eager work between replays
        ctx.sync()
        for a, b in zip(eager, graph):
            ga, gb = ctx.read_walk(a), ctx.read_walk(b)
            assert ga["t"] == gb["t"]
            for key in ("pivot", "C", "best", "local_best"):
                assert np.array_equal(ga[key], gb[key]), (r, key)
            for key in ("psl_best", "alpha", "unimproved", "q", "last_k", "value_local"):
                assert ga[key] == gb[key], (r, key)
    ctx.free_walks(eager + graph + other)


def test_autotune_shapes_keep_results(ctx, tmp_path):
    """Every launch shape the autotuner may pick gives the same walks: a batch
    stepped under the tuned shape equals the same batch under the defaults
    (fresh context), and the tuning file round-trips."""
    from paper_2107_09801_amd import libpsl
    Ls = [64, 513, 2000, 4097, 9000]

    def batch(c):
        ids = []
        for L in Ls:
            ids += c.init_walks(L, 2, 31 + L, n_lmt=0, switch_period=6, flip_lmt=min(5, L))
        return ids

    ids = batch(ctx)
    choice = ctx.autotune(ids)
    assert choice["waves"] in (4, 8, 16) and choice["persistent"] in (0, 1)
    assert choice["eval_items"] in (2048, 4096, 8192, 16384)     # x/2 .. 4x of the default
    assert choice["eval_ms"] > 0 and choice["eval_ms"] <= choice["default_ms"] * 1.0001
    ctx.step_batch(ids, 12)
    path = str(tmp_path / "tune.txt")
    ctx.tune_save(path)
    fields = open(path).read().split()
    assert len(fields) % 5 == 0 and int(fields[4]) == choice["eval_items"]
    other = libpsl.Context(0)
    ref = batch(other)
    other.step_batch(ref, 12)
    for a, b in zip(ids, ref):
        ga, gb = ctx.read_walk(a), other.read_walk(b)
        for key in ("pivot", "C", "best", "local_best"):
            assert np.array_equal(ga[key], gb[key]), key
        assert abs(ga["value_local"] - gb["value_local"]) <= F_RTOL * ga["value_local"]
    other.tune_load(path)
    assert other.autotune(ref)["waves"] in (4, 8, 16)
    other.close()
    ctx.free_walks(ids)


def test_every_launch_shape_gives_the_same_walks(ctx, tmp_path):
    """Each evaluation launch shape (4, 8 or 16 wavefronts; one block per
    item, or a persistent grid of 1..6 blocks per CU over the per-XCD
    queues), forced through a tuning file, steps a mixed batch (ragged
    tiles, L from 2 to 9000, several k-splits) to the same walks as the
    untuned default, which the oracle pins elsewhere."""
    from paper_2107_09801_amd import libpsl
    Ls = [2, 65, 257, 1001, 3000, 9000]

    def batch(c):
        ids = []
        for L in Ls:
            ids += c.init_walks(L, 2, 57 + L, n_lmt=0, switch_period=4, flip_lmt=min(5, L))
        return ids

    ref_ctx = libpsl.Context(0)
    ref = batch(ref_ctx)
    ref_ctx.step_batch(ref, 9)
    want = [ref_ctx.read_walk(w) for w in ref]
    ref_ctx.close()
    # the batch's tuning key, as the library writes it
    probe = libpsl.Context(0)
    pids = batch(probe)
    probe.autotune(pids)
    probe.tune_save(str(tmp_path / "key.txt"))
    key = open(tmp_path / "key.txt").read().split()[0]
    probe.close()
    shapes = [(16, 0, 0), (16, 1, 1), (16, 1, 2), (8, 0, 0), (8, 1, 1), (8, 1, 2), (8, 1, 3),
              (4, 0, 0), (4, 1, 1), (4, 1, 3), (4, 1, 6)]
    for waves, pers, bpc in shapes:
        c = libpsl.Context(0)
        if ctx_is_dense(ctx):
            c.set_option(libpsl.OPT_NEAR_LIMIT, 0)
        f = tmp_path / "shape.txt"
        f.write_text(f"{key} {waves} {pers} {bpc}\n")
        c.tune_load(str(f))
        ids = batch(c)
        c.step_batch(ids, 9)
        for w, o in zip(ids, want):
            g = c.read_walk(w)
            for k in ("pivot", "C", "best", "local_best"):
                assert np.array_equal(g[k], o[k]), (waves, pers, bpc, k)
            assert g["psl_best"] == o["psl_best"] and g["t"] == o["t"]
            assert abs(g["value_local"] - o["value_local"]) <= F_RTOL * o["value_local"]
        c.close()


def ctx_is_dense(ctx):
    return getattr(ctx, "_dense", False)


def test_checkpoint_restore_continues_exactly(ctx):
    """N steps, checkpoint, restore into another walk, M steps == N + M steps."""
    L, seed, N, M = 2000, 77, 17, 13
    kw = dict(alpha1=4, alpha2=11, n_lmt=0, ls_lmt=4, flip_lmt=7, switch_period=0)
    (a,) = ctx.init_walks(L, 1, seed, **kw)
    (b,) = ctx.init_walks(L, 1, seed, **kw)
    ctx.step_batch([a], N + M)
    ctx.step_batch([b], N)
    ck = ctx.checkpoint(b)
    ctx.free_walks([b])
    (c,) = ctx.init_walks(L, 1, 999, alpha1=13, alpha2=13, n_lmt=100, switch_period=3)
    ctx.restore(c, ck)
    ctx.step_batch([c], M)
    ga, gc = ctx.read_walk(a), ctx.read_walk(c)
    for key in ("pivot", "C", "local_best", "best"):
        assert np.array_equal(ga[key], gc[key]), key
    for key in ("t", "q", "alpha", "psl_best", "unimproved", "psl_pivot", "last_k", "value_local"):
        assert ga[key] == gc[key], key
    ctx.free_walks([a, c])


def test_trace_ring_matches_oracle(ctx):
    L, seed, steps, cap = 1001, 4321, 40, 16
    (w,) = ctx.init_walks(L, 1, seed, alpha1=4, alpha2=13, n_lmt=0, flip_lmt=10, switch_period=9)
    ctx.trace_enable(w, cap)
    ow = oracle.Walk(oracle.WalkConfig(L=L, seed=seed, alpha1=4, alpha2=13, n_lmt=L, flip_lmt=10,
                                       switch_period=9), margin=MARGIN, nthreads=8)
    ctx.step_batch([w], steps)
    trs = [ow.step() for _ in range(steps)]
    got = ctx.trace_read(w, 100)
    assert [e["t"] for e in got] == list(range(steps - cap, steps))
    for e in got:
        tr = trs[e["t"]]
        assert e["start"] == tr["start"] and e["k"] == tr["k"]
        assert abs(e["value_step"] - tr["value_step"]) <= F_RTOL * tr["value_step"]
        assert e["psl_k"] == tr["psl_k"] and e["psl_best"] == tr["psl_best"]
        assert e["alpha"] == tr["alpha"]
        assert bool(e["flags"] & 4) == bool(tr["flags"] & oracle.SWITCHED)
    ctx.trace_enable(w, 0)
    ctx.free_walks([w])
