"""Thin ctypes binding of libpsl (include/psl.h).

Argument marshalling only: every step of the search runs in the HIP kernels of
``_build/libpsl.so``. PyTorch is used for device buffers and streams. There is
no fallback: if the library is missing, importing this module fails.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "_build", "libpsl.so")

OK, E_INVAL, E_NOMEM, E_HIP, E_STATE, E_AGAIN, E_FULL = 0, -1, -2, -3, -4, -5, -6
STEP_BLOCKING = 1
STEP_GRAPH = 2
STEP_IMPROVED, STEP_WORSE, STEP_SWITCHED, STEP_PSL_IMPROVED = 1, 2, 4, 8
STEP_AMBIG_ARGMIN, STEP_AMBIG_COMPARE = 16, 32
CHOICE_AMBIGUOUS_ARGMIN = 1
L_MAX = 1048575

EXPORTS = ["psl_ctx_create", "psl_ctx_destroy", "psl_last_error", "psl_sync", "psl_init_walks",
           "psl_free_walks", "psl_eval_neighbourhood", "psl_eval_neighbourhood_noalloc", "psl_apply_flip", "psl_step_batch",
           "psl_read_walk", "psl_eval_shape", "psl_version", "psl_timing_enable",
           "psl_timing_read", "psl_set_option", "psl_serve_start", "psl_serve_submit",
           "psl_serve_poll", "psl_serve_stats_read", "psl_serve_stop", "psl_serve_footprint",
           "psl_autotune", "psl_tune_save", "psl_tune_load", "psl_trace_enable",
           "psl_trace_read", "psl_restore_walk"]
OPT_NEAR_LIMIT = 1
OPT_EVAL_ITEMS = 2
OPT_AMBIG_MARGIN = 3      # value in units of 1e-15 (-1: the default, 5e-13)
OPT_SPLIT = 4             # split evaluation: 2 (default) by launch work, 1 wherever L >= 2048, 0 never
OPT_TEST_FAIL_ADMIT = 5   # test hook: serving admission n (>= 1) fails as a HIP error would; 0: off


class PslError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libpsl status {status}: {msg}")
        self.status = status


class WalkCfg(ctypes.Structure):
    _fields_ = [("L", ctypes.c_uint32), ("alpha1", ctypes.c_uint32), ("alpha2", ctypes.c_uint32),
                ("n_lmt", ctypes.c_uint32), ("ls_lmt", ctypes.c_uint32),
                ("flip_lmt", ctypes.c_uint32), ("switch_period", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("seed", ctypes.c_uint64)]


class Choice(ctypes.Structure):
    _fields_ = [("j_best", ctypes.c_uint32), ("i_best", ctypes.c_uint32),
                ("F_best", ctypes.c_double), ("F_min", ctypes.c_double),
                ("j_psl", ctypes.c_uint32), ("psl_min", ctypes.c_int32),
                ("psl_k", ctypes.c_int32), ("flags", ctypes.c_uint32)]

    def as_dict(self) -> dict:
        return {n: getattr(self, n) for n, _ in self._fields_}


class WalkState(ctypes.Structure):
    _fields_ = [("L", ctypes.c_uint32), ("alpha1", ctypes.c_uint32), ("alpha2", ctypes.c_uint32),
                ("alpha", ctypes.c_uint32), ("n_lmt", ctypes.c_uint32), ("ls_lmt", ctypes.c_uint32),
                ("flip_lmt", ctypes.c_uint32), ("switch_period", ctypes.c_uint32),
                ("seed", ctypes.c_uint64), ("t", ctypes.c_uint64), ("q", ctypes.c_uint64),
                ("value_local", ctypes.c_double), ("F_pivot", ctypes.c_double),
                ("psl_pivot", ctypes.c_int32), ("psl_best", ctypes.c_int32),
                ("unimproved", ctypes.c_uint32), ("last_k", ctypes.c_uint32),
                ("last_value_step", ctypes.c_double), ("last_start", ctypes.c_uint32),
                ("last_flags", ctypes.c_uint32)]

    def as_dict(self) -> dict:
        return {n: getattr(self, n) for n, _ in self._fields_}


class ServeCfg(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_uint64), ("max_slots", ctypes.c_uint32),
                ("flags", ctypes.c_uint32)]


class Job(ctypes.Structure):
    _fields_ = [("cfg", WalkCfg), ("step_budget", ctypes.c_uint64),
                ("best_bits_out", ctypes.c_void_p)]


class JobResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("psl_best", ctypes.c_int32),
                ("psl_final", ctypes.c_int32), ("alpha_final", ctypes.c_uint32),
                ("F_final", ctypes.c_double), ("steps", ctypes.c_uint64),
                ("t_arrive_ns", ctypes.c_uint64), ("t_admit_ns", ctypes.c_uint64),
                ("t_done_ns", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {n: getattr(self, n) for n, _ in self._fields_}


class ServeStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("failed", ctypes.c_uint64), ("active", ctypes.c_uint64),
                ("queued", ctypes.c_uint64), ("iterations", ctypes.c_uint64),
                ("flip_evals", ctypes.c_uint64), ("ck_updates", ctypes.c_uint64),
                ("busy_s", ctypes.c_double), ("peak_active", ctypes.c_uint64),
                ("peak_used", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {n: getattr(self, n) for n, _ in self._fields_}


class TraceEntry(ctypes.Structure):
    _fields_ = [("t", ctypes.c_uint64), ("start", ctypes.c_uint32), ("k", ctypes.c_uint32),
                ("value_step", ctypes.c_double), ("psl_k", ctypes.c_int32),
                ("psl_best", ctypes.c_int32), ("alpha", ctypes.c_uint32), ("flags", ctypes.c_uint32)]

    def as_dict(self) -> dict:
        return {n: getattr(self, n) for n, _ in self._fields_}


class TuneChoice(ctypes.Structure):
    _fields_ = [("waves", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("eval_items", ctypes.c_int32),
                ("eval_ms", ctypes.c_double), ("default_ms", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {n: getattr(self, n) for n, _ in self._fields_}


class Timing(ctypes.Structure):
    _fields_ = [("eval_ms", ctypes.c_double), ("eval_launches", ctypes.c_uint64),
                ("rest_ms", ctypes.c_double), ("steps", ctypes.c_uint64),
                ("prep_ms", ctypes.c_double), ("lin_ms", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {n: getattr(self, n) for n, _ in self._fields_}


_lib = None


def lib() -> ctypes.CDLL:
    """The compiled library. Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libpsl is not built ({LIB_PATH} missing); run "
                          "`python -c 'import __graft_entry__ as g; g.build()'`")
    L = ctypes.CDLL(LIB_PATH)
    P, u32, u64, i32, sz = (ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32,
                            ctypes.c_size_t)
    sig = {
        "psl_ctx_create": (i32, [ctypes.c_int, P, P, sz, ctypes.POINTER(P)]),
        "psl_ctx_destroy": (None, [P]),
        "psl_last_error": (ctypes.c_char_p, [P]),
        "psl_sync": (i32, [P]),
        "psl_init_walks": (i32, [P, ctypes.POINTER(WalkCfg), u32, P, P]),
        "psl_free_walks": (i32, [P, P, u32]),
        "psl_eval_neighbourhood": (i32, [P, u32, u32, u32, P, P, ctypes.POINTER(Choice)]),
        "psl_eval_neighbourhood_noalloc": (i32, [P, u32, u32, u32, P, P, ctypes.POINTER(Choice)]),
        "psl_apply_flip": (i32, [P, u32, u32]),
        "psl_step_batch": (i32, [P, P, u32, u32, u32]),
        "psl_read_walk": (i32, [P, u32, ctypes.POINTER(WalkState), P, P, P, P]),
        "psl_eval_shape": (i32, [P, u32, u32, u32, ctypes.POINTER(u32), ctypes.POINTER(u32)]),
        "psl_version": (ctypes.c_char_p, []),
        "psl_timing_enable": (i32, [P, ctypes.c_int]),
        "psl_timing_read": (i32, [P, ctypes.POINTER(Timing)]),
        "psl_set_option": (i32, [P, ctypes.c_int, ctypes.c_int64]),
        "psl_serve_start": (i32, [P, ctypes.POINTER(ServeCfg)]),
        "psl_serve_submit": (i32, [P, ctypes.POINTER(Job), ctypes.POINTER(u64)]),
        "psl_serve_poll": (i32, [P, u64, ctypes.POINTER(JobResult)]),
        "psl_serve_stats_read": (i32, [P, ctypes.POINTER(ServeStats)]),
        "psl_serve_stop": (i32, [P, ctypes.c_int]),
        "psl_serve_footprint": (i32, [ctypes.POINTER(WalkCfg), ctypes.POINTER(u64)]),
        "psl_autotune": (i32, [P, P, u32, ctypes.POINTER(TuneChoice)]),
        "psl_tune_save": (i32, [P, ctypes.c_char_p]),
        "psl_tune_load": (i32, [P, ctypes.c_char_p]),
        "psl_trace_enable": (i32, [P, u32, u32]),
        "psl_trace_read": (i32, [P, u32, ctypes.POINTER(TraceEntry), u32, ctypes.POINTER(u32)]),
        "psl_restore_walk": (i32, [P, u32, ctypes.POINTER(WalkState), P, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def n_words(L: int) -> int:
    return (L + 63) // 64


class Context:
    """A libpsl context on one HIP device (default: torch's current stream)."""

    def __init__(self, device: int = 0, stream=None, arena=None):
        import torch
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self._stream = stream
        self._arena = arena          # a torch uint8 tensor kept alive by the context
        h = ctypes.c_void_p()
        arena_ptr = arena.data_ptr() if arena is not None else None
        arena_bytes = arena.numel() * arena.element_size() if arena is not None else 0
        st = lib().psl_ctx_create(device, ctypes.c_void_p(stream.cuda_stream), arena_ptr,
                                  arena_bytes, ctypes.byref(h))
        if st != OK:
            raise PslError(st, "psl_ctx_create failed")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().psl_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, st: int):
        if st != OK:
            raise PslError(st, lib().psl_last_error(self._h).decode())

    def last_error(self) -> str:
        return lib().psl_last_error(self._h).decode()

    def sync(self):
        self._check(lib().psl_sync(self._h))

    def init_walks(self, L: int, n: int, seed: int, alpha1: int = 4, alpha2: int = 13,
                   n_lmt: int = 0, ls_lmt: int = 2000, flip_lmt: int | None = None,
                   switch_period: int = 0, init_bits=None) -> list[int]:
        if flip_lmt is None:          # the paper's FLIP_lmt = 10, capped by L
            flip_lmt = min(10, L)
        cfg = WalkCfg(L=L, alpha1=alpha1, alpha2=alpha2, n_lmt=n_lmt, ls_lmt=ls_lmt,
                      flip_lmt=flip_lmt, switch_period=switch_period, reserved=0,
                      seed=seed & (2**64 - 1))
        ids = np.zeros(n, dtype=np.uint32)
        arr = None
        keep = []
        if init_bits is not None:
            arr = (ctypes.c_void_p * n)()
            for w in range(n):
                b = init_bits[w]
                if b is None:
                    arr[w] = None
                else:
                    b = np.ascontiguousarray(b, dtype=np.uint64)
                    keep.append(b)
                    arr[w] = b.ctypes.data
        st = lib().psl_init_walks(self._h, ctypes.byref(cfg), n,
                                  ctypes.cast(arr, ctypes.c_void_p) if arr is not None else None,
                                  _ptr(ids))
        self._check(st)
        return [int(x) for x in ids]

    def free_walks(self, ids):
        a = np.ascontiguousarray(ids, dtype=np.uint32)
        self._check(lib().psl_free_walks(self._h, _ptr(a), len(a)))

    def eval_neighbourhood(self, walk: int, start: int, n_lmt: int, F_out=None, psl_out=None):
        """F_out / psl_out: optional torch device tensors (float64 / int32, n_lmt)."""
        ch = Choice()
        fp = F_out.data_ptr() if F_out is not None else None
        pp = psl_out.data_ptr() if psl_out is not None else None
        if F_out is not None:
            assert F_out.is_cuda and F_out.dtype.itemsize == 8 and F_out.numel() >= n_lmt
        if psl_out is not None:
            assert psl_out.is_cuda and psl_out.dtype.itemsize == 4 and psl_out.numel() >= n_lmt
        self._check(lib().psl_eval_neighbourhood(self._h, walk, start, n_lmt, fp, pp,
                                                 ctypes.byref(ch)))
        return ch.as_dict()

    def eval_neighbourhood_noalloc(self, walk: int, start: int, n_lmt: int, F_out, psl_out):
        """psl_eval_neighbourhood_noalloc: F_out / psl_out are required torch
        device tensors (float64 / int32, at least n_lmt entries)."""
        assert F_out.is_cuda and F_out.dtype.itemsize == 8 and F_out.numel() >= n_lmt
        assert psl_out.is_cuda and psl_out.dtype.itemsize == 4 and psl_out.numel() >= n_lmt
        ch = Choice()
        self._check(lib().psl_eval_neighbourhood_noalloc(self._h, walk, start, n_lmt, F_out.data_ptr(),
                                                         psl_out.data_ptr(), ctypes.byref(ch)))
        return ch.as_dict()

    def apply_flip(self, walk: int, j: int):
        self._check(lib().psl_apply_flip(self._h, walk, j))

    def step_batch(self, ids, steps: int, blocking: bool = True, graph: bool = False):
        a = np.ascontiguousarray(ids, dtype=np.uint32)
        flags = (STEP_BLOCKING if blocking else 0) | (STEP_GRAPH if graph else 0)
        self._check(lib().psl_step_batch(self._h, _ptr(a), len(a), steps, flags))

    def read_walk(self, walk: int, bits: bool = True, C: bool = True) -> dict:
        st = WalkState()
        self._check(lib().psl_read_walk(self._h, walk, ctypes.byref(st), None, None, None, None))
        d = st.as_dict()
        if bits or C:
            nw = n_words(d["L"])
            piv = np.zeros(nw, np.uint64) if bits else None
            lb = np.zeros(nw, np.uint64) if bits else None
            best = np.zeros(nw, np.uint64) if bits else None
            Cv = np.zeros(d["L"], np.int32) if C else None
            self._check(lib().psl_read_walk(self._h, walk, None,
                                            _ptr(piv) if bits else None,
                                            _ptr(lb) if bits else None,
                                            _ptr(best) if bits else None,
                                            _ptr(Cv) if C else None))
            d.update(pivot=piv, local_best=lb, best=best, C=Cv)
        return d

    def eval_shape(self, L: int, n_lmt: int, n_walks: int = 1):
        t, k = ctypes.c_uint32(), ctypes.c_uint32()
        self._check(lib().psl_eval_shape(self._h, L, n_lmt, n_walks, ctypes.byref(t),
                                         ctypes.byref(k)))
        return int(t.value), int(k.value)


    # ------------------------------------------------------------ serving

    def serve_start(self, hbm_budget: int, max_slots: int):
        self._served = {}
        cfg = ServeCfg(hbm_budget=hbm_budget, max_slots=max_slots, flags=0)
        self._check(lib().psl_serve_start(self._h, ctypes.byref(cfg)))

    def serve_submit(self, L: int, seed: int, step_budget: int, alpha1: int = 4,
                     alpha2: int = 13, n_lmt: int = 0, ls_lmt: int = 2000,
                     flip_lmt: int | None = None, switch_period: int = 0,
                     want_best: bool = True) -> int:
        """Queue a job; returns its ticket. Raises PslError on a non-OK status."""
        if flip_lmt is None:
            flip_lmt = min(10, L)
        best = np.zeros(n_words(L), np.uint64) if want_best else None
        job = Job(cfg=WalkCfg(L=L, alpha1=alpha1, alpha2=alpha2, n_lmt=n_lmt, ls_lmt=ls_lmt,
                              flip_lmt=flip_lmt, switch_period=switch_period, reserved=0,
                              seed=seed & (2**64 - 1)),
                  step_budget=step_budget, best_bits_out=best.ctypes.data if want_best else None)
        t = ctypes.c_uint64()
        st = lib().psl_serve_submit(self._h, ctypes.byref(job), ctypes.byref(t))
        if st != OK:
            raise PslError(st, "psl_serve_submit")
        self._served[int(t.value)] = best      # the buffer lives until polled
        return int(t.value)

    def serve_poll(self, ticket: int):
        """The job's result dict (with 'best' bits) when done, else None."""
        r = JobResult()
        st = lib().psl_serve_poll(self._h, ticket, ctypes.byref(r))
        if st == E_AGAIN:
            return None
        if st != OK:
            raise PslError(st, "psl_serve_poll")
        d = r.as_dict()
        d["best"] = self._served.pop(ticket, None)
        return d

    def serve_stats(self) -> dict:
        s = ServeStats()
        self._check(lib().psl_serve_stats_read(self._h, ctypes.byref(s)))
        return s.as_dict()

    def serve_stop(self, drain: bool = True):
        self._check(lib().psl_serve_stop(self._h, 1 if drain else 0))

    def trace_enable(self, walk: int, capacity: int):
        self._check(lib().psl_trace_enable(self._h, walk, capacity))

    def trace_read(self, walk: int, max_entries: int) -> list[dict]:
        buf = (TraceEntry * max(max_entries, 1))()
        n = ctypes.c_uint32()
        self._check(lib().psl_trace_read(self._h, walk, buf, max_entries, ctypes.byref(n)))
        return [buf[i].as_dict() for i in range(n.value)]

    def checkpoint(self, walk: int) -> dict:
        """Everything psl_restore_walk needs: the state struct and the three bit sets."""
        st = WalkState()
        self._check(lib().psl_read_walk(self._h, walk, ctypes.byref(st), None, None, None, None))
        nw = n_words(st.L)
        piv, lb, best = (np.zeros(nw, np.uint64) for _ in range(3))
        self._check(lib().psl_read_walk(self._h, walk, None, _ptr(piv), _ptr(lb), _ptr(best), None))
        return {"state": st, "pivot": piv, "local_best": lb, "best": best}

    def restore(self, walk: int, ck: dict):
        self._check(lib().psl_restore_walk(self._h, walk, ctypes.byref(ck["state"]),
                                           _ptr(ck["pivot"]), _ptr(ck["local_best"]),
                                           _ptr(ck["best"])))

    def autotune(self, ids) -> dict:
        a = np.ascontiguousarray(ids, dtype=np.uint32)
        c = TuneChoice()
        self._check(lib().psl_autotune(self._h, _ptr(a), len(a), ctypes.byref(c)))
        return c.as_dict()

    def tune_save(self, path: str):
        self._check(lib().psl_tune_save(self._h, path.encode()))

    def tune_load(self, path: str):
        self._check(lib().psl_tune_load(self._h, path.encode()))

    def set_option(self, option: int, value: int):
        self._check(lib().psl_set_option(self._h, option, value))

    def timing_enable(self, on: bool = True):
        self._check(lib().psl_timing_enable(self._h, 1 if on else 0))

    def timing_read(self) -> dict:
        t = Timing()
        self._check(lib().psl_timing_read(self._h, ctypes.byref(t)))
        return t.as_dict()


def serve_footprint(L: int, n_lmt: int = 0) -> int:
    """Bytes a served job of length L (and N_lmt) counts against the budget."""
    cfg = WalkCfg(L=L, alpha1=4, alpha2=13, n_lmt=n_lmt, ls_lmt=0, flip_lmt=0, switch_period=0,
                  reserved=0, seed=0)
    out = ctypes.c_uint64()
    st = lib().psl_serve_footprint(ctypes.byref(cfg), ctypes.byref(out))
    if st != OK:
        raise PslError(st, "psl_serve_footprint")
    return int(out.value)


def version() -> str:
    return lib().psl_version().decode()
