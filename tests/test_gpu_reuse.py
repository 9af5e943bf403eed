"""Unit-under-test calls that repeat: psl_eval_neighbourhood on the same walk
and N_lmt reuses its layout (only the start changes) and psl_apply_flip its
batch entry, so neither allocates device memory after the first call, and
the reused evaluations still equal the oracle's."""
import numpy as np
import pytest

import oracle
import seeded_inputs as si

pytestmark = pytest.mark.gpu

F_RTOL = 1e-12


@pytest.fixture()
def ctx():
    import torch
    from paper_2107_09801_amd import libpsl
    assert torch.cuda.is_available()
    c = libpsl.Context(0)
    yield c
    c.close()


def _free():
    import torch
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info(0)[0]


@pytest.mark.parametrize("L,n_lmt", [(4097, 500), (3001, 3001)])
def test_eval_reuses_its_layout_across_starts(ctx, L, n_lmt):
    import torch
    seed = si.BASE_SEED + 17 * L
    (w,) = ctx.init_walks(L, 1, seed, alpha1=4, alpha2=13)
    F = torch.empty(n_lmt, dtype=torch.float64, device="cuda:0")
    P = torch.empty(n_lmt, dtype=torch.int32, device="cuda:0")
    ctx.eval_neighbourhood(w, 0, n_lmt, F, P)            # the first call lays out the evaluation
    F.cpu(), P.cpu()                                     # (the runtime's own first-copy set-up)
    free0 = _free()
    outs = []
    for start in (17, L - 1, L // 2, 17, 0):
        ch = ctx.eval_neighbourhood(w, start, n_lmt, F, P)
        outs.append((start, ch, F.cpu().numpy().copy(), P.cpu().numpy().copy()))
    assert _free() == free0                              # the repeats allocate nothing
    s = oracle.rand_pivot(seed, L)
    C = oracle.corr(s)
    for start, ch, Fg, Pg in outs:
        Fo, Po = oracle.eval_neighbourhood(s, C, 4, start, n_lmt, nthreads=8)
        assert np.array_equal(Pg, Po), start
        assert np.max(np.abs(Fg - Fo) / Fo) <= F_RTOL, start
        oc = oracle.select(Fo, Po, margin=5e-13)
        assert ch["psl_min"] == oc.psl_min and ch["j_psl"] == (start + oc.i_psl + 1) % L
        if not oc.flags & oracle.AMBIG_ARGMIN:
            assert ch["j_best"] == (start + oc.i_best + 1) % L
    # a different N_lmt lays out again and is still right
    ch = ctx.eval_neighbourhood(w, 5, n_lmt - 1, F, P)
    Fo, Po = oracle.eval_neighbourhood(s, C, 4, 5, n_lmt - 1, nthreads=8)
    assert np.array_equal(P.cpu().numpy()[:n_lmt - 1], Po)
    assert np.max(np.abs(F.cpu().numpy()[:n_lmt - 1] - Fo) / Fo) <= F_RTOL
    ctx.free_walks([w])


def test_eval_after_free_and_reinit_lays_out_again(ctx):
    import torch
    F = torch.empty(900, dtype=torch.float64, device="cuda:0")
    P = torch.empty(900, dtype=torch.int32, device="cuda:0")
    (w,) = ctx.init_walks(1001, 1, si.walk_seed(21))
    ctx.eval_neighbourhood(w, 3, 900, F, P)
    ctx.free_walks([w])
    # the same walk id, now of another length: the old layout must not be reused
    (w2,) = ctx.init_walks(2049, 1, si.walk_seed(22), alpha1=13, alpha2=4)
    ctx.eval_neighbourhood(w2, 3, 900, F, P)
    s = oracle.rand_pivot(si.walk_seed(22), 2049)
    Fo, Po = oracle.eval_neighbourhood(s, oracle.corr(s), 13, 3, 900, nthreads=8)
    assert np.array_equal(P.cpu().numpy(), Po)
    assert np.max(np.abs(F.cpu().numpy() - Fo) / Fo) <= F_RTOL
    ctx.free_walks([w2])


def test_apply_flip_allocates_once(ctx):
    L = 1001
    seed = si.BASE_SEED + 5
    (w,) = ctx.init_walks(L, 1, seed, alpha1=4, alpha2=13)
    s = oracle.rand_pivot(seed, L)
    ctx.apply_flip(w, 3)
    s[3] = -s[3]
    ctx.read_walk(w)
    free0 = _free()
    for j in (10, 500, 999, 3):
        ctx.apply_flip(w, j)
        s[j] = -s[j]
    assert _free() == free0
    g = ctx.read_walk(w)
    assert np.array_equal(g["C"], oracle.corr(s))
    assert np.array_equal(g["pivot"], oracle.seq_to_bits(s))
    ctx.free_walks([w])
