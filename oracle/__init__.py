"""CPU oracle for the two-phase PSL search (arXiv 2107.09801).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the bench's
CPU-baseline leg are the only callers. The product library never imports this
package, and this package imports nothing from the product.

The arithmetic lives in ``psl_oracle.c`` (plain loops that follow Eq. (2),
Eq. (3), Eq. (5) and Algorithm 1, with the readings listed at the top of that
file). This module compiles it with gcc, loads it with ctypes and adds a few
exact pure-Python helpers (Python integers) used to pin it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "psl_oracle.c")
LIB_PATH = os.path.join(HERE, "_build", "libpsl_oracle.so")

TAU = 1e-12          # relative width of the best-neighbour band (reading R5/R6)

AMBIG_ARGMIN = 1
AMBIG_COMPARE = 2
IMPROVED = 4
WORSE = 8
SWITCHED = 16
PSL_IMPROVED = 32
SELFCHECK_FAILED = 64


def build(verbose: bool = False) -> str:
    """Compile psl_oracle.c into a shared library (gcc, -O2, OpenMP)."""
    os.makedirs(os.path.dirname(LIB_PATH), exist_ok=True)
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
           "-fvisibility=hidden", "-o", tmp, SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


class Choice(ctypes.Structure):
    _fields_ = [("i_best", ctypes.c_uint32), ("F_best", ctypes.c_double),
                ("F_min", ctypes.c_double), ("i_psl", ctypes.c_uint32),
                ("psl_min", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class Trace(ctypes.Structure):
    _fields_ = [("start", ctypes.c_uint32), ("k", ctypes.c_uint32),
                ("value_step", ctypes.c_double), ("F_min", ctypes.c_double),
                ("psl_k", ctypes.c_int32), ("j_psl", ctypes.c_uint32),
                ("psl_min", ctypes.c_int32), ("psl_best", ctypes.c_int32),
                ("alpha", ctypes.c_int32), ("unimproved", ctypes.c_uint32),
                ("value_local", ctypes.c_double), ("flags", ctypes.c_uint32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


def lib() -> ctypes.CDLL:
    """The compiled oracle; built on first use when no library exists yet."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build()
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    u32, i32, u64, dbl, cint = (ctypes.c_uint32, ctypes.c_int32, ctypes.c_uint64,
                                ctypes.c_double, ctypes.c_int)
    sig = {
        "oc_draw": (u64, [u64, u64]),
        "oc_rand_pivot": (None, [u64, cint, P]),
        "oc_bits_to_seq": (None, [P, cint, P]),
        "oc_seq_to_bits": (None, [P, cint, P]),
        "oc_corr": (None, [P, cint, P]),
        "oc_check_corr": (cint, [P, P, cint, cint]),
        "oc_psl": (i32, [P, cint]),
        "oc_power_table": (None, [cint, cint, P]),
        "oc_fitness": (dbl, [P, cint, P]),
        "oc_flip_corr_definition": (None, [P, cint, cint, P]),
        "oc_flip_corr_formula": (None, [P, P, cint, cint, P]),
        "oc_eval_neighbourhood": (None, [P, P, cint, P, u32, u32, P, P, cint]),
        "oc_select": (None, [P, P, u32, dbl, dbl, ctypes.POINTER(Choice)]),
        "oc_walk_create": (P, [cint, u64, cint, cint, u32, u32, u32, u32, P]),
        "oc_walk_destroy": (None, [P]),
        "oc_walk_step": (None, [P, dbl, dbl, cint, i32, ctypes.POINTER(Trace)]),
        "oc_walk_read": (None, [P, P, P, P, P, P, P]),
        "oc_walk_last_neighbourhood": (None, [P, P, P]),
        "oc_min_psl_bruteforce": (i32, [cint, ctypes.POINTER(u64), cint]),
        "oc_max_threads": (cint, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _p(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def n_words(L: int) -> int:
    return (L + 63) // 64


# --------------------------------------------------------------- wrappers

def draw(seed: int, ctr: int) -> int:
    return int(lib().oc_draw(seed & (2**64 - 1), ctr & (2**64 - 1)))


def rand_pivot(seed: int, L: int) -> np.ndarray:
    s = np.empty(L, dtype=np.int8)
    lib().oc_rand_pivot(seed, L, _p(s))
    return s


def bits_to_seq(bits: np.ndarray, L: int) -> np.ndarray:
    bits = np.ascontiguousarray(bits, dtype=np.uint64)
    s = np.empty(L, dtype=np.int8)
    lib().oc_bits_to_seq(_p(bits), L, _p(s))
    return s


def seq_to_bits(s: np.ndarray) -> np.ndarray:
    s = np.ascontiguousarray(s, dtype=np.int8)
    bits = np.empty(n_words(len(s)), dtype=np.uint64)
    lib().oc_seq_to_bits(_p(s), len(s), _p(bits))
    return bits


def corr(s: np.ndarray) -> np.ndarray:
    s = np.ascontiguousarray(s, dtype=np.int8)
    C = np.empty(len(s), dtype=np.int32)
    lib().oc_corr(_p(s), len(s), _p(C))
    return C


def check_corr(s: np.ndarray, C: np.ndarray, full: bool = False) -> bool:
    """The identities of Eq. (2) that every C satisfies (and, with full, C
    equal to Eq. (2) recomputed): the walk's per-step self-check."""
    s = np.ascontiguousarray(s, dtype=np.int8)
    C = np.ascontiguousarray(C, dtype=np.int32)
    return bool(lib().oc_check_corr(_p(s), _p(C), len(s), 1 if full else 0))


def psl(C: np.ndarray) -> int:
    C = np.ascontiguousarray(C, dtype=np.int32)
    return int(lib().oc_psl(_p(C), len(C)))


def power_table(alpha: int, n: int) -> np.ndarray:
    T = np.empty(n, dtype=np.float64)
    lib().oc_power_table(alpha, n, _p(T))
    return T


def fitness(C: np.ndarray, alpha: int) -> float:
    C = np.ascontiguousarray(C, dtype=np.int32)
    T = power_table(alpha, len(C) + 1)
    return float(lib().oc_fitness(_p(C), len(C), _p(T)))


def flip_corr_definition(s: np.ndarray, j: int) -> np.ndarray:
    s = np.ascontiguousarray(s, dtype=np.int8)
    Cn = np.empty(len(s), dtype=np.int32)
    lib().oc_flip_corr_definition(_p(s), len(s), j, _p(Cn))
    return Cn


def flip_corr_formula(s: np.ndarray, C: np.ndarray, j: int) -> np.ndarray:
    s = np.ascontiguousarray(s, dtype=np.int8)
    C = np.ascontiguousarray(C, dtype=np.int32)
    Cn = np.empty(len(s), dtype=np.int32)
    lib().oc_flip_corr_formula(_p(s), _p(C), len(s), j, _p(Cn))
    return Cn


def eval_neighbourhood(s: np.ndarray, C: np.ndarray, alpha: int, start: int,
                       n_lmt: int, nthreads: int = 1):
    """F and PSL of neighbours j = (start+i) mod L, i = 1..n_lmt (entry i-1)."""
    L = len(s)
    s = np.ascontiguousarray(s, dtype=np.int8)
    C = np.ascontiguousarray(C, dtype=np.int32)
    T = power_table(alpha, L + 1)
    F = np.empty(n_lmt, dtype=np.float64)
    P = np.empty(n_lmt, dtype=np.int32)
    lib().oc_eval_neighbourhood(_p(s), _p(C), L, _p(T), start, n_lmt, _p(F), _p(P),
                                nthreads)
    return F, P


def select(F: np.ndarray, P: np.ndarray, tau: float = TAU, margin: float = 0.0) -> Choice:
    F = np.ascontiguousarray(F, dtype=np.float64)
    P = np.ascontiguousarray(P, dtype=np.int32)
    ch = Choice()
    lib().oc_select(_p(F), _p(P), len(F), tau, margin, ctypes.byref(ch))
    return ch


def min_psl_bruteforce(L: int, nthreads: int = 0):
    cnt = ctypes.c_uint64(0)
    nt = nthreads or os.cpu_count() or 1
    best = lib().oc_min_psl_bruteforce(L, ctypes.byref(cnt), nt)
    return int(best), int(cnt.value)


def max_threads() -> int:
    return int(lib().oc_max_threads())


@dataclass
class WalkConfig:
    L: int
    seed: int
    alpha1: int = 4
    alpha2: int = 13
    n_lmt: int = 0            # 0 = full neighbourhood (L)
    ls_lmt: int = 2000
    flip_lmt: int = 10
    switch_period: int = 0


class Walk:
    """One run of Algorithm 1 held by the oracle."""

    def __init__(self, cfg: WalkConfig, init_bits: np.ndarray | None = None,
                 tau: float = TAU, margin: float = 0.0, nthreads: int = 1):
        self.cfg = cfg
        self.L = cfg.L
        self.n_lmt = cfg.n_lmt or cfg.L
        self.tau = tau
        self.margin = margin
        self.nthreads = nthreads
        self._bits_keep = None
        ptr = None
        if init_bits is not None:
            self._bits_keep = np.ascontiguousarray(init_bits, dtype=np.uint64)
            ptr = _p(self._bits_keep)
        self._w = lib().oc_walk_create(cfg.L, cfg.seed & (2**64 - 1), cfg.alpha1, cfg.alpha2,
                                       self.n_lmt, cfg.ls_lmt, cfg.flip_lmt,
                                       cfg.switch_period, ptr)
        if not self._w:
            raise ValueError(f"invalid walk configuration {cfg}")

    def __del__(self):
        w = getattr(self, "_w", None)
        if w:
            lib().oc_walk_destroy(w)
            self._w = None

    def step(self, force_k: int = -1) -> dict:
        tr = Trace()
        lib().oc_walk_step(self._w, self.tau, self.margin, self.nthreads, force_k,
                           ctypes.byref(tr))
        d = tr.as_dict()
        if d["flags"] & SELFCHECK_FAILED:
            raise RuntimeError(f"oracle walk: C fails its Eq. (2) self-check after step {self.read()['t']}")
        return d

    def read(self) -> dict:
        nw = n_words(self.L)
        pivot = np.empty(nw, np.uint64)
        local_best = np.empty(nw, np.uint64)
        best = np.empty(nw, np.uint64)
        C = np.empty(self.L, np.int32)
        sf = np.empty(2, np.float64)
        si = np.empty(6, np.int64)
        lib().oc_walk_read(self._w, _p(pivot), _p(local_best), _p(best), _p(C), _p(sf), _p(si))
        return {"pivot": pivot, "local_best": local_best, "best": best, "C": C,
                "value_local": float(sf[0]), "F_pivot": float(sf[1]),
                "alpha": int(si[0]), "psl_best": int(si[1]), "unimproved": int(si[2]),
                "t": int(si[3]), "q": int(si[4]), "psl_pivot": int(si[5])}

    def last_neighbourhood(self):
        F = np.empty(self.n_lmt, np.float64)
        P = np.empty(self.n_lmt, np.int32)
        lib().oc_walk_last_neighbourhood(self._w, _p(F), _p(P))
        return F, P


# ----------------------------------------------- exact pure-Python helpers

def corr_exact(s) -> list[int]:
    """Eq. (2) with Python integers (small L only)."""
    L = len(s)
    return [sum(int(s[i]) * int(s[i + k]) for i in range(L - k)) for k in range(L)]


def fitness_exact(C, alpha: int) -> int:
    """Eq. (5) as an exact integer, for integer alpha."""
    return sum(abs(int(c)) ** alpha for c in C[1:])
