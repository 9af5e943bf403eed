"""Readers of the committed oracle goldens (tests/golden/*.json, written by
tests/golden/make_fullsize.py from the oracle alone) and the digests they
hold."""
import hashlib
import json
import os

import numpy as np

GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name: str) -> dict:
    with open(os.path.join(GOLDEN_DIR, f"fullsize_{name}.json")) as f:
        return json.load(f)["cases"]


def sha(a: np.ndarray) -> str:
    """SHA-256 of an array's little-endian bytes (C as int32, sequences as
    packed 64-bit words), as the generator writes it."""
    a = np.ascontiguousarray(a)
    return hashlib.sha256(a.astype(a.dtype.newbyteorder("<")).tobytes()).hexdigest()


def check_state(g: dict, want: dict, rtol: float, where):
    """A libpsl read_walk() dict against a golden state record."""
    assert g["t"] == want["t"] and g["q"] == want["q"], where
    assert g["alpha"] == want["alpha"] and g["psl_best"] == want["psl_best"], where
    assert g["psl_pivot"] == want["psl_pivot"] and g["unimproved"] == want["unimproved"], where
    assert abs(g["value_local"] - want["value_local"]) <= rtol * want["value_local"], where
    assert abs(g["F_pivot"] - want["F_pivot"]) <= rtol * want["F_pivot"], where
    if "C" in g and g["C"] is not None:
        assert sha(g["C"]) == want["sha_C"], (where, "C")
    if "pivot" in g and g["pivot"] is not None:
        assert sha(g["pivot"]) == want["sha_pivot"], (where, "pivot")
        assert sha(g["local_best"]) == want["sha_local_best"], (where, "local_best")
        assert sha(g["best"]) == want["sha_best"], (where, "best")


def check_step(g: dict, step: dict, rtol: float, where):
    """The last step of a libpsl walk against a golden step record."""
    assert g["last_start"] == step["start"], where
    assert g["last_k"] == step["k"], where
    assert abs(g["last_value_step"] - step["value_step"]) <= rtol * step["value_step"], where
    check_state(g, step["state"], rtol, where)
