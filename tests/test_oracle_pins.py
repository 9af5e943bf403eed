"""Pins of the CPU oracle against what the paper and mathematics fix.

Nothing here compares the oracle with itself: every check uses a closed form,
an invariant, a library routine, exact integer arithmetic, a symmetry, a
published value or brute force.
"""
import math
import os

import numpy as np
import pytest

import oracle
import seeded_inputs as si

pytestmark = pytest.mark.filterwarnings("ignore")
HERE = os.path.dirname(os.path.abspath(__file__))
U = 2.0 ** -53


# ----------------------------------------------------------------- RNG

def test_splitmix64_reference_outputs():
    """Counter form equals the published SplitMix64 stream from state 0."""
    with open(os.path.join(HERE, "golden", "splitmix64_state0.txt")) as f:
        want = [int(x) for x in f.read().split("\n") if x and not x.startswith("#")]
    got = [oracle.draw(0, c) for c in range(len(want))]
    assert got == want


def test_rand_pivot_uses_word_bits():
    L = 200
    s = oracle.rand_pivot(77, L)
    for i in range(L):
        w = oracle.draw(77, i // 64)
        assert s[i] == (-1 if (w >> (i % 64)) & 1 else 1)


# ------------------------------------------------------------- Eq. (2)

@pytest.mark.parametrize("L", [2, 3, 5, 64, 65, 127, 1001])
def test_corr_matches_numpy_correlate(L):
    s = si.to_pm1(si.random_bits(L, 1000 + L), L)
    C = oracle.corr(s)
    ref = np.correlate(s.astype(np.int64), s.astype(np.int64), mode="full")[L - 1:]
    assert np.array_equal(C, ref)


@pytest.mark.parametrize("L", [2, 3, 4, 17, 100, 511, 2047])
def test_corr_invariants(L):
    s = si.to_pm1(si.random_bits(L, 7 * L + 1), L)
    C = oracle.corr(s).astype(np.int64)
    k = np.arange(L)
    assert C[0] == L
    assert C[L - 1] == int(s[0]) * int(s[L - 1])
    assert np.all((C - (L - k)) % 2 == 0)
    assert int(s.astype(np.int64).sum()) ** 2 == L + 2 * int(C[1:].sum())
    assert np.all(np.abs(C) <= L - k)


@pytest.mark.parametrize("L", [2, 9, 64, 333])
def test_corr_closed_forms(L):
    k = np.arange(L)
    C1 = oracle.corr(si.to_pm1(si.all_plus_bits(L), L))
    assert np.array_equal(C1, L - k)
    Ca = oracle.corr(si.to_pm1(si.alternating_bits(L), L))
    assert np.array_equal(Ca, ((-1) ** k) * (L - k))


@pytest.mark.parametrize("L", [5, 40, 257])
def test_corr_symmetries(L):
    s = si.to_pm1(si.random_bits(L, 99 + L), L)
    C = oracle.corr(s)
    assert np.array_equal(oracle.corr(-s), C)
    assert np.array_equal(oracle.corr(s[::-1].copy()), C)
    alt = (s * np.where(np.arange(L) % 2 == 0, 1, -1)).astype(np.int8)
    assert np.array_equal(oracle.corr(alt), C * ((-1) ** np.arange(L)))


# ------------------------------------------------------------- Eq. (3)

def test_psl_all_plus_is_L_minus_1():
    for L in (2, 3, 10, 100):
        assert oracle.psl(oracle.corr(si.to_pm1(si.all_plus_bits(L), L))) == L - 1


# Minimum PSL over all binary sequences of length L (Eq. (4)), as published:
# Barker sequences (PSL 1) exist for L in {2,3,4,5,7,11,13} and for no other
# L up to far beyond 24; every other L <= 21 has minimum PSL 2, and
# 22 <= L <= 48 has minimum PSL 3 (Turyn 1968; Lindner 1975; Coxson & Russo
# 2005, the exhaustive-search work the paper cites in Section 1).
BARKER = {2, 3, 4, 5, 7, 11, 13}


def published_min_psl(L):
    if L in BARKER:
        return 1
    return 2 if L <= 21 else 3


@pytest.mark.parametrize("L", list(range(2, 25)))
def test_bruteforce_min_psl_matches_literature(L):
    best, count = oracle.min_psl_bruteforce(L)
    assert best == published_min_psl(L)
    assert count >= 1


def _orbit(seq):
    """All sequences equivalent under negation, reversal and alternation."""
    s = np.array(seq, dtype=np.int8)
    alt = np.where(np.arange(len(s)) % 2 == 0, 1, -1).astype(np.int8)
    out = set()
    for a in (s, s[::-1]):
        for b in (a, a * alt):
            for c in (b, -b):
                out.add(tuple(int(x) for x in c))
    return out


@pytest.mark.parametrize("code", [
    [1, 1, 1, -1, -1, 1, -1],                                # Barker 7
    [1, 1, 1, -1, -1, -1, 1, -1, -1, 1, -1],                 # Barker 11
    [1, 1, 1, 1, 1, -1, -1, 1, 1, -1, 1, -1, 1],             # Barker 13
])
def test_psl_one_sequences_are_the_barker_orbit(code):
    L = len(code)
    orbit = {o for o in _orbit(code) if o[0] == 1}
    best, count = oracle.min_psl_bruteforce(L)
    assert best == 1 and count == len(orbit)
    for o in orbit:
        assert oracle.psl(oracle.corr(np.array(o, dtype=np.int8))) == 1


# ------------------------------------------------------------- Eq. (5)

@pytest.mark.parametrize("alpha", [1, 2, 4, 10, 11, 13, 16])
def test_power_table_against_exact_powers(alpha):
    n = 3000
    T = oracle.power_table(alpha, n)
    assert T[0] == 0.0
    for c in list(range(0, 50)) + list(range(50, n, 37)):
        exact = c ** alpha
        assert abs(T[c] - exact) <= (alpha - 1) * 1.0000001 * U * exact


@pytest.mark.parametrize("L,alpha", [(2, 4), (13, 4), (64, 13), (50, 2), (40, 11), (33, 1)])
def test_fitness_against_exact_integer(L, alpha):
    s = si.to_pm1(si.random_bits(L, 3 * L + alpha), L)
    C = oracle.corr(s)
    exact = oracle.fitness_exact(oracle.corr_exact(s), alpha)
    F = oracle.fitness(C, alpha)
    assert abs(F - exact) <= (alpha + 2) * U * exact


def _faulhaber(n, alpha):
    # textbook closed forms of sum_{m=1}^{n} m^alpha
    return {1: n * (n + 1) // 2,
            2: n * (n + 1) * (2 * n + 1) // 6,
            3: (n * (n + 1) // 2) ** 2,
            4: n * (n + 1) * (2 * n + 1) * (3 * n * n + 3 * n - 1) // 30}[alpha]


@pytest.mark.parametrize("alpha", [1, 2, 3, 4])
@pytest.mark.parametrize("L", [2, 7, 300, 4096])
def test_fitness_all_plus_faulhaber(L, alpha):
    C = oracle.corr(si.to_pm1(si.all_plus_bits(L), L))
    exact = _faulhaber(L - 1, alpha)
    F = oracle.fitness(C, alpha)
    assert abs(F - exact) <= (alpha + 2) * U * exact


def test_fitness_alpha2_merit_factor_relation():
    # MF = L^2 / (2 sum C_k^2) (Section 2): for Barker 13, sum C_k^2 = 6.
    s = np.array([1, 1, 1, 1, 1, -1, -1, 1, 1, -1, 1, -1, 1], dtype=np.int8)
    F = oracle.fitness(oracle.corr(s), 2)
    assert F == 6.0
    assert math.isclose(13 ** 2 / (2 * F), 14.083333333333334)


# --------------------------------------------- one-element flip (Section 3)

@pytest.mark.parametrize("L", [2, 3, 4, 31, 64, 65, 200])
def test_flip_formula_equals_definition(L):
    s = si.to_pm1(si.random_bits(L, 11 * L + 5), L)
    C = oracle.corr(s)
    for j in range(L):
        assert np.array_equal(oracle.flip_corr_formula(s, C, j),
                              oracle.flip_corr_definition(s, j)), j


@pytest.mark.parametrize("L", [2, 5, 70])
def test_flip_all_plus_closed_form(L):
    s = si.to_pm1(si.all_plus_bits(L), L)
    C = oracle.corr(s)
    k = np.arange(L)
    for j in range(L):
        want = (L - k) - 2 * ((j + k < L).astype(int) + (j - k >= 0).astype(int))
        want[0] = L
        assert np.array_equal(oracle.flip_corr_formula(s, C, j), want)


# ------------------------------------------ Neighborhood (Algorithm 1)

@pytest.mark.parametrize("L,alpha,start,n_lmt", [
    (2, 4, 0, 2), (3, 13, 2, 3), (17, 4, 5, 17), (40, 13, 39, 40), (40, 10, 3, 7),
    (64, 11, 63, 64), (65, 4, 0, 1)])
def test_neighbourhood_against_definition(L, alpha, start, n_lmt):
    s = si.to_pm1(si.random_bits(L, 1234 + L + start), L)
    C = oracle.corr(s)
    F, P = oracle.eval_neighbourhood(s, C, alpha, start, n_lmt)
    for i in range(1, n_lmt + 1):
        j = (start + i) % L
        t = s.copy()
        t[j] = -t[j]
        Cn = oracle.corr_exact(t)
        exact = oracle.fitness_exact(Cn, alpha)
        assert abs(F[i - 1] - exact) <= (alpha + 2) * U * exact
        assert P[i - 1] == max(abs(c) for c in Cn[1:])


def test_full_neighbourhood_covers_every_element_once_start_last():
    L, start = 37, 11
    s = si.to_pm1(si.random_bits(L, 5), L)
    C = oracle.corr(s)
    F, P = oracle.eval_neighbourhood(s, C, 4, start, L)
    js = [(start + i) % L for i in range(1, L + 1)]
    assert sorted(js) == list(range(L)) and js[-1] == start
    for i, j in enumerate(js):
        exact = oracle.fitness_exact(oracle.flip_corr_definition(s, j), 4)
        assert abs(F[i] - exact) <= 6 * U * exact


def test_neighbourhood_thread_count_invariant():
    L = 500
    s = si.to_pm1(si.random_bits(L, 8), L)
    C = oracle.corr(s)
    F1, P1 = oracle.eval_neighbourhood(s, C, 13, 17, L, nthreads=1)
    F4, P4 = oracle.eval_neighbourhood(s, C, 13, 17, L, nthreads=4)
    assert np.array_equal(F1, F4) and np.array_equal(P1, P4)


# ------------------------------------------------------- selection

def test_select_strict_first_minimum_in_scan_order():
    F = np.array([5.0, 3.0, 4.0, 3.0, 3.5])
    P = np.array([9, 7, 7, 8, 6], dtype=np.int32)
    ch = oracle.select(F, P)
    assert ch.i_best == 1 and ch.F_best == 3.0 and ch.F_min == 3.0
    assert ch.i_psl == 4 and ch.psl_min == 6
    P2 = np.array([9, 7, 7, 8, 7], dtype=np.int32)
    assert oracle.select(F, P2).i_psl == 1


def test_select_band_takes_first_in_scan_order():
    base = 1.0e20
    F = np.array([base * (1 + 5e-13), base, base * (1 + 2e-12)])
    P = np.ones(3, dtype=np.int32)
    ch = oracle.select(F, P, tau=1e-12)
    assert ch.i_best == 0            # within the band, earlier in scan order
    ch = oracle.select(F, P, tau=0.0)
    assert ch.i_best == 1            # exact rule


def test_select_flags_band_edge():
    base = 1.0e10
    F = np.array([base, base * (1 + 1e-12 + 1e-14)])
    P = np.ones(2, dtype=np.int32)
    assert oracle.select(F, P, 1e-12, 5e-13).flags & oracle.AMBIG_ARGMIN
    F = np.array([base, base * (1 + 5e-12)])
    assert not oracle.select(F, P, 1e-12, 5e-13).flags & oracle.AMBIG_ARGMIN
