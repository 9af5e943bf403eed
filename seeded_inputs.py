"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module holds none of the method's arithmetic: it only makes packed +-1
sequences (64-bit words, element i in bit i%64 of word i/64, bit 1 = -1) and
the workload parameters. The method's own random draws (the initial pivot of
Algorithm 1, the start of each limited neighbourhood, the positions flipped at
a phase switch) are not made here: each side implements the counter-based
generator it is defined by.
"""
from __future__ import annotations

import numpy as np

BASE_SEED = 210709801


def n_words(L: int) -> int:
    return (L + 63) // 64


def _clear_tail(bits: np.ndarray, L: int) -> np.ndarray:
    r = L % 64
    if r:
        bits[-1] &= np.uint64((1 << r) - 1)
    return bits


def random_bits(L: int, seed: int) -> np.ndarray:
    """i.i.d. uniform +-1 elements from numpy's PCG64 stream `seed`."""
    rng = np.random.Generator(np.random.PCG64(seed))
    bits = rng.integers(0, 2**63, size=n_words(L), dtype=np.uint64) * np.uint64(2)
    bits ^= rng.integers(0, 2, size=n_words(L), dtype=np.uint64)
    return _clear_tail(bits, L)


def biased_bits(L: int, seed: int, p_minus: float) -> np.ndarray:
    """Elements are -1 with probability p_minus (skewed sums, large |C_k|)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    neg = rng.random(L) < p_minus
    return pack(neg)


def all_plus_bits(L: int) -> np.ndarray:
    return np.zeros(n_words(L), dtype=np.uint64)


def alternating_bits(L: int) -> np.ndarray:
    """s_i = (-1)^i with the paper's 1-based i: element 0 (s_1) is -1,
    element 1 (s_2) is +1, and so on."""
    neg = (np.arange(L) % 2) == 0
    return pack(neg)


def pack(neg: np.ndarray) -> np.ndarray:
    """Pack a boolean array (True = -1) into 64-bit words."""
    L = len(neg)
    padded = np.zeros(n_words(L) * 64, dtype=np.uint64)
    padded[:L] = neg.astype(np.uint64)
    words = padded.reshape(-1, 64)
    shifts = np.arange(64, dtype=np.uint64)
    return np.bitwise_or.reduce(words << shifts, axis=1).astype(np.uint64)


def unpack(bits: np.ndarray, L: int) -> np.ndarray:
    """Boolean array (True = -1) of the first L elements."""
    shifts = np.arange(64, dtype=np.uint64)
    b = (np.asarray(bits, dtype=np.uint64)[:, None] >> shifts) & np.uint64(1)
    return b.reshape(-1)[:L].astype(bool)


def to_pm1(bits: np.ndarray, L: int) -> np.ndarray:
    """int8 +-1 view of a packed sequence."""
    return np.where(unpack(bits, L), -1, 1).astype(np.int8)


def walk_seed(w: int) -> int:
    """Seed of walk w in the batched workloads."""
    return BASE_SEED + w


# Paper exponents: alpha_1 = 4; alpha_2 = 13 up to L = 2^17-1, 11 at 2^18-1,
# 10 above (Section 4.2 and Table 3).
def alpha2_for(L: int) -> int:
    if L <= 131071:
        return 13
    if L <= 262143:
        return 11
    return 10


def serve_jobs(n: int, seed: int, nlmt_cap: int) -> list[dict]:
    """The serving workload's job mixture: half L = 2^m - 1 (m = 14..20
    uniform), half odd L uniform in [1001, 1048575]; step budget uniform in
    [50, 500]; N_lmt = min(L, nlmt_cap); job i has seed BASE_SEED + i."""
    rng = np.random.Generator(np.random.PCG64(seed))
    jobs = []
    for i in range(n):
        if rng.random() < 0.5:
            L = 2 ** int(rng.integers(14, 21)) - 1
        else:
            L = 2 * int(rng.integers(500, 524288)) + 1
        budget = int(rng.integers(50, 501))
        jobs.append({"L": L, "budget": budget, "n_lmt": min(L, nlmt_cap),
                     "alpha2": alpha2_for(L), "seed": BASE_SEED + i})
    return jobs


def serve_mixture_50() -> list[dict]:
    """The 50-job sample of the serving mixture that the serving parity test
    submits in waves: budgets cut to 5..60 steps so the check stays short."""
    rng = np.random.default_rng(2107)
    jobs = serve_jobs(50, BASE_SEED + 7, 256)
    for j in jobs:
        j["budget"] = int(rng.integers(5, 61))
    return jobs
