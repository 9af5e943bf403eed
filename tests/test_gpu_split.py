"""The split evaluation (linear part of Eq. (5) on the matrix cores as exact
integer sums, the both-neighbour remainder on the vector units) against the
table evaluation and against the oracle, through the C-ABI: the same PSL and
moves, F within 1e-12 relative (it agrees to about 1e-14)."""
import numpy as np
import pytest

import oracle
import seeded_inputs as si
from lockstep import run_lockstep

pytestmark = pytest.mark.gpu

F_RTOL = 1e-12


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2107_09801_amd import libpsl
    assert torch.cuda.is_available()
    c = libpsl.Context(0)
    yield c
    c.close()


def _eval(ctx, w, start, n_lmt, split):
    import torch
    from paper_2107_09801_amd import libpsl
    ctx.set_option(libpsl.OPT_SPLIT, 1 if split else 0)
    try:
        F = torch.empty(n_lmt, dtype=torch.float64, device="cuda:0")
        P = torch.empty(n_lmt, dtype=torch.int32, device="cuda:0")
        ch = ctx.eval_neighbourhood(w, start, n_lmt, F, P)
        return ch, F.cpu().numpy(), P.cpu().numpy()
    finally:
        ctx.set_option(libpsl.OPT_SPLIT, -1)


@pytest.mark.parametrize("L,alpha,start,n_lmt", [
    (2049, 4, 0, 2049), (2049, 13, 1000, 2049), (4097, 13, 4096, 4097), (3001, 10, 17, 700),
    (16383, 13, 5, 16383), (16383, 4, 9000, 6912), (65535, 13, 123, 65535), (100000, 10, 99990, 3000)])
def test_split_equals_table_and_oracle(ctx, L, alpha, start, n_lmt):
    seed = si.BASE_SEED + 31 * L + alpha
    (w,) = ctx.init_walks(L, 1, seed, alpha1=alpha, alpha2=4)
    ch_s, Fs, Ps = _eval(ctx, w, start, n_lmt, True)
    ch_t, Ft, Pt = _eval(ctx, w, start, n_lmt, False)
    assert np.array_equal(Ps, Pt)
    assert np.max(np.abs(Fs - Ft) / Ft) <= 1e-13
    for key in ("i_best", "j_best", "j_psl", "psl_min", "psl_k", "flags"):
        assert ch_s[key] == ch_t[key], key
    s = oracle.rand_pivot(seed, L)
    C = oracle.corr(s)
    idx = np.unique(np.linspace(0, n_lmt - 1, 24).astype(int))
    for i0 in idx:
        Fo, Po = oracle.eval_neighbourhood(s, C, alpha, (start + int(i0)) % L, 1, nthreads=8)
        assert Ps[i0] == Po[0]
        assert abs(Fs[i0] - Fo[0]) <= F_RTOL * Fo[0], i0
    ctx.free_walks([w])


@pytest.mark.parametrize("L,n_lmt,period", [(4097, 4097, 7), (16383, 16383, 50), (3001, 900, 0)])
def test_split_steps_lockstep_with_oracle(ctx, L, n_lmt, period):
    from paper_2107_09801_amd import libpsl
    seed = si.BASE_SEED + 7 * L
    ctx.set_option(libpsl.OPT_SPLIT, 1)
    try:
        (w,) = ctx.init_walks(L, 1, seed, alpha1=4, alpha2=13, n_lmt=n_lmt, ls_lmt=5, flip_lmt=10,
                              switch_period=period)
        ow = oracle.Walk(oracle.WalkConfig(L=L, seed=seed, alpha1=4, alpha2=13, n_lmt=n_lmt, ls_lmt=5,
                                           flip_lmt=10, switch_period=period), margin=5e-13, nthreads=8)
        compared, imposed = run_lockstep(ctx, w, ow, 30, check_every=5)
        assert compared + imposed == 30 and compared >= 27
        ctx.free_walks([w])
    finally:
        ctx.set_option(libpsl.OPT_SPLIT, -1)


def test_split_mixed_batch_equals_table_batch(ctx):
    """A batch with walks the split path takes (L >= 2048) and walks it does
    not, stepped with the split path on and off: identical walks."""
    from paper_2107_09801_amd import libpsl
    Ls = [1001, 2049, 4097, 9999, 16383]
    walks = {}
    for mode in (1, 0):
        ctx.set_option(libpsl.OPT_SPLIT, mode)
        try:
            ids = []
            for L in Ls:
                ids += ctx.init_walks(L, 2, si.BASE_SEED + L, alpha1=4, alpha2=13, switch_period=4, flip_lmt=10)
            ctx.step_batch(ids, 9)
            walks[mode] = [ctx.read_walk(w) for w in ids]
            ctx.free_walks(ids)
        finally:
            ctx.set_option(libpsl.OPT_SPLIT, -1)
    for a, b in zip(walks[1], walks[0]):
        for key in ("pivot", "C", "best", "local_best"):
            assert np.array_equal(a[key], b[key]), key
        assert a["psl_best"] == b["psl_best"] and a["last_k"] == b["last_k"]
        assert abs(a["value_local"] - b["value_local"]) <= 1e-13 * b["value_local"]
