"""Pins of the oracle's Algorithm 1 step against the algorithm's stated effects.

Each property is checked with definition-tier arithmetic (Eq. (2) recomputed,
Eq. (5) as an exact integer) rather than the oracle's own code paths.
"""
import numpy as np
import pytest

import oracle
import seeded_inputs as si

U = 2.0 ** -53


def _exact_F_of_bits(bits, L, alpha):
    s = si.to_pm1(bits, L)
    return oracle.fitness_exact(oracle.corr_exact(s), alpha)


def _exact_psl_of_bits(bits, L):
    C = oracle.corr_exact(si.to_pm1(bits, L))
    return max(abs(c) for c in C[1:])


def _hamming(a, b, L):
    return int(np.sum(si.unpack(a, L) != si.unpack(b, L)))


@pytest.mark.parametrize("L,n_lmt,period,ls", [(23, 23, 5, 2000), (40, 9, 0, 3),
                                                (31, 31, 0, 1), (64, 20, 7, 2000)])
def test_walk_step_properties(L, n_lmt, period, ls):
    cfg = oracle.WalkConfig(L=L, seed=424242 + L, alpha1=4, alpha2=13, n_lmt=n_lmt,
                            ls_lmt=ls, flip_lmt=3, switch_period=period)
    w = oracle.Walk(cfg)
    st = w.read()
    # initial state (readings R7, R11)
    assert st["alpha"] == 4 and st["unimproved"] == 0
    assert np.array_equal(st["local_best"], st["pivot"])
    assert np.array_equal(st["best"], st["pivot"])
    assert st["psl_best"] == _exact_psl_of_bits(st["pivot"], L)
    ex = _exact_F_of_bits(st["pivot"], L, 4)
    assert abs(st["value_local"] - ex) <= 8 * U * ex
    n_switch = 0
    for t in range(60):
        prev = st
        tr = w.step()
        st = w.read()
        alpha_prev = prev["alpha"]
        # start of the limited neighbourhood
        assert tr["start"] == oracle.draw(cfg.seed, (1 << 60) | t) % L
        # candidates, their exact F and PSL, recomputed by definition
        s_prev = si.to_pm1(prev["pivot"], L)
        cand = [(tr["start"] + i) % L for i in range(1, n_lmt + 1)]
        Fx, Px = [], []
        for j in cand:
            u = s_prev.copy()
            u[j] = -u[j]
            Cn = oracle.corr_exact(u)
            Fx.append(oracle.fitness_exact(Cn, alpha_prev))
            Px.append(max(abs(c) for c in Cn[1:]))
        fmin = min(Fx)
        first_min = cand[Fx.index(fmin)]
        assert tr["k"] == first_min        # no near-ties at these sizes
        assert abs(tr["value_step"] - fmin) <= 8 * U * fmin
        assert tr["psl_k"] == Px[Fx.index(fmin)]
        assert tr["psl_min"] == min(Px) and tr["j_psl"] == cand[Px.index(min(Px))]
        # best-PSL neighbour kept only on strict improvement
        want_best = min(prev["psl_best"], min(Px))
        assert st["psl_best"] == want_best
        assert _exact_psl_of_bits(st["best"], L) == want_best
        if min(Px) < prev["psl_best"]:
            # the first best-PSL neighbour in scan order replaces solution_best
            jb = cand[Px.index(min(Px))]
            nb = prev["pivot"].copy()
            nb[jb // 64] ^= np.uint64(1) << np.uint64(jb % 64)
            assert np.array_equal(st["best"], nb)
        else:
            # ties and worse leave solution_best as it was
            assert np.array_equal(st["best"], prev["best"])
        switched = bool(tr["flags"] & oracle.SWITCHED)
        improved = tr["value_step"] < prev["value_local"] * (1 - oracle.TAU)
        worse = tr["value_step"] > prev["value_local"] * (1 + oracle.TAU)
        assert bool(tr["flags"] & oracle.IMPROVED) == improved
        assert bool(tr["flags"] & oracle.WORSE) == worse
        moved = prev["pivot"].copy()
        moved[tr["k"] // 64] ^= np.uint64(1) << np.uint64(tr["k"] % 64)
        if period:
            want_switch = (t + 1) % period == 0
        else:
            want_switch = worse and prev["unimproved"] + 1 > ls
        assert switched == want_switch
        if not switched:
            # Flip(pivot, k): exactly one element changes; C is Eq. (2) of it
            assert np.array_equal(st["pivot"], moved)
            assert np.array_equal(st["C"], np.array(oracle.corr_exact(si.to_pm1(moved, L))))
            assert st["alpha"] == alpha_prev
            if improved:
                assert st["unimproved"] == 0 and st["value_local"] == tr["value_step"]
                assert np.array_equal(st["local_best"], moved)
            elif worse:
                assert st["unimproved"] == prev["unimproved"] + 1
            else:
                assert st["unimproved"] == prev["unimproved"]
        else:
            n_switch += 1
            lb = st["local_best"]
            if improved:
                assert np.array_equal(lb, moved)
            else:
                assert np.array_equal(lb, prev["local_best"])
            assert _hamming(st["pivot"], lb, L) == cfg.flip_lmt
            assert st["alpha"] == (13 if alpha_prev == 4 else 4)
            assert st["unimproved"] == 0
            ex = _exact_F_of_bits(st["pivot"], L, st["alpha"])
            assert abs(st["value_local"] - ex) <= 16 * U * ex
            assert np.array_equal(st["C"], np.array(oracle.corr_exact(si.to_pm1(st["pivot"], L))))
    if period:
        assert n_switch == 60 // period


def test_rand_flip_positions_are_the_first_distinct_draws():
    L, seed = 16, 99
    cfg = oracle.WalkConfig(L=L, seed=seed, alpha1=4, alpha2=13, n_lmt=L,
                            ls_lmt=2000, flip_lmt=12, switch_period=1)
    w = oracle.Walk(cfg)
    st0 = w.read()
    tr = w.step()
    st = w.read()
    assert tr["flags"] & oracle.SWITCHED
    lb = st["local_best"]
    want = set()
    r = 0
    while len(want) < 12:
        want.add(oracle.draw(seed, (2 << 60) | (0 << 24) | r) % L)
        r += 1
    diff = set(np.nonzero(si.unpack(st["pivot"], L) != si.unpack(lb, L))[0].tolist())
    assert diff == want
    del st0


def test_walk_given_initial_bits():
    L = 50
    bits = si.random_bits(L, 3)
    w = oracle.Walk(oracle.WalkConfig(L=L, seed=1, n_lmt=L), init_bits=bits)
    st = w.read()
    assert np.array_equal(st["pivot"], bits)
    assert np.array_equal(st["C"], np.array(oracle.corr_exact(si.to_pm1(bits, L))))


def test_walk_rejects_bad_config():
    with pytest.raises(ValueError):
        oracle.Walk(oracle.WalkConfig(L=1, seed=0))
    with pytest.raises(ValueError):
        oracle.Walk(oracle.WalkConfig(L=10, seed=0, n_lmt=11))
    with pytest.raises(ValueError):
        oracle.Walk(oracle.WalkConfig(L=10, seed=0, alpha1=17))


def test_corr_self_check_catches_planted_errors():
    """The walk's per-step check of C (identities of Eq. (2), plus the full
    recomputation) accepts a true C and rejects planted mistakes."""
    rng = np.random.default_rng(11)
    for L in (2, 3, 17, 64, 101):
        s = (1 - 2 * rng.integers(0, 2, L)).astype(np.int8)
        C = np.array(oracle.corr_exact(s), dtype=np.int32)
        assert oracle.check_corr(s, C) and oracle.check_corr(s, C, full=True)
        if L < 4:
            continue
        bad = C.copy(); bad[0] += 2                 # C_0 != L
        assert not oracle.check_corr(s, bad)
        bad = C.copy(); bad[L - 1] = -bad[L - 1]    # wrong end term
        assert not oracle.check_corr(s, bad)
        bad = C.copy(); bad[2] += 1                 # parity of L-k broken
        assert not oracle.check_corr(s, bad)
        bad = C.copy(); bad[1] += 2                 # sum identity broken
        if abs(bad[1]) <= L - 1:
            assert not oracle.check_corr(s, bad)
        # a change the identities cannot see: +2 at one shift, -2 at another
        bad = C.copy(); k1, k2 = 1, 3
        if abs(C[k1] + 2) <= L - k1 and abs(C[k2] - 2) <= L - k2:
            bad[k1] += 2; bad[k2] -= 2
            assert oracle.check_corr(s, bad)
            assert not oracle.check_corr(s, bad, full=True)


def test_walk_runs_its_self_check_past_64_steps():
    L = 40
    w = oracle.Walk(oracle.WalkConfig(L=L, seed=5, alpha1=4, alpha2=13, n_lmt=L, flip_lmt=3,
                                      switch_period=7))
    for _ in range(130):
        tr = w.step()
        assert not tr["flags"] & oracle.SELFCHECK_FAILED
