"""psl_eval_neighbourhood_noalloc against psl_eval_neighbourhood, through the
C-ABI: the same F (within 1e-12 relative), PSL, choice and flags on two calls
in a row, the second on a smaller input, so the fixed scratch the first call
left behind is reused; the small case also against the oracle; a request
whose scratch exceeds the fixed array is refused with nothing launched."""
import numpy as np
import pytest

import oracle
import seeded_inputs as si

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


def _pair(ctx, w, start, n_lmt):
    import torch
    F_a = torch.full((n_lmt,), -1.0, dtype=torch.float64, device="cuda:0")
    P_a = torch.full((n_lmt,), -1, dtype=torch.int32, device="cuda:0")
    F_b = torch.empty(n_lmt, dtype=torch.float64, device="cuda:0")
    P_b = torch.empty(n_lmt, dtype=torch.int32, device="cuda:0")
    ch_a = ctx.eval_neighbourhood_noalloc(w, start, n_lmt, F_a, P_a)
    ch_b = ctx.eval_neighbourhood(w, start, n_lmt, F_b, P_b)
    return ch_a, F_a.cpu().numpy(), P_a.cpu().numpy(), ch_b, F_b.cpu().numpy(), P_b.cpu().numpy()


def _same(ch_a, Fa, Pa, ch_b, Fb, Pb):
    assert np.array_equal(Pa, Pb)
    assert np.max(np.abs(Fa - Fb) / Fb) <= F_RTOL
    for key in ("i_best", "j_best", "j_psl", "psl_min", "psl_k", "flags"):
        assert ch_a[key] == ch_b[key], key
    for key in ("F_best", "F_min"):
        assert abs(ch_a[key] - ch_b[key]) <= F_RTOL * ch_b[key], key


def test_noalloc_equals_eval_neighbourhood_twice(ctx):
    (wa,) = ctx.init_walks(16383, 1, si.walk_seed(3), alpha1=13, alpha2=4)
    (wb,) = ctx.init_walks(3001, 1, si.walk_seed(4), alpha1=4, alpha2=13)
    # first call: a full neighbourhood of the larger walk
    _same(*_pair(ctx, wa, 5, 16383))
    # second call, smaller: a limited neighbourhood that wraps past L - 1
    ch_a, Fa, Pa, ch_b, Fb, Pb = _pair(ctx, wb, 2999, 700)
    _same(ch_a, Fa, Pa, ch_b, Fb, Pb)
    s = oracle.rand_pivot(si.walk_seed(4), 3001)
    Fo, Po = oracle.eval_neighbourhood(s, oracle.corr(s), 4, 2999, 700, nthreads=8)
    assert np.array_equal(Pa, Po) and np.max(np.abs(Fa - Fo) / Fo) <= F_RTOL
    oc = oracle.select(Fo, Po)
    assert ch_a["i_best"] == oc.i_best and ch_a["psl_min"] == oc.psl_min
    ctx.free_walks([wa, wb])


def test_noalloc_refuses_what_exceeds_its_scratch(ctx):
    import torch
    from paper_2107_09801_amd import libpsl
    (w,) = ctx.init_walks(131071, 1, si.walk_seed(5))
    ctx.set_option(libpsl.OPT_EVAL_ITEMS, 1 << 18)
    try:
        F = torch.empty(131071, dtype=torch.float64, device="cuda:0")
        P = torch.empty(131071, dtype=torch.int32, device="cuda:0")
        with pytest.raises(libpsl.PslError) as e:
            ctx.eval_neighbourhood_noalloc(w, 0, 131071, F, P)
        assert e.value.status == libpsl.E_NOMEM
    finally:
        ctx.set_option(libpsl.OPT_EVAL_ITEMS, -1)
    # a request that fits still works after the refusal
    (w2,) = ctx.init_walks(1001, 1, si.walk_seed(6))
    _same(*_pair(ctx, w2, 17, 1001))
    ctx.free_walks([w, w2])
