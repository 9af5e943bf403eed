"""CPU checks of bench.py's host-side arithmetic (no GPU): the count of
explicitly evaluated (j, k) pairs and the traffic-record lookup."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("L", [2, 3, 4, 5, 16, 17, 100, 101])
def test_explicit_updates_closed_form_against_brute_force(L):
    # (j, k) pairs, k = 1..L-1, where at least one neighbour j+k < L or j-k >= 0
    # exists, for every candidate j of a full neighbourhood
    brute = sum(1 for j in range(L) for k in range(1, L) if j + k < L or j - k >= 0)
    nominal = L * (L - 1)
    got = bench.explicit_updates([(L, 1)], "batched", 0, nominal, 1, 1.0)
    assert got["per_step"] == brute
    assert got["fraction_of_nominal"] == pytest.approx(brute / nominal)


def test_explicit_updates_unknown_for_limited_neighbourhoods():
    assert bench.explicit_updates([(1001, 1)], "paper", 0, 1, 1, 1.0) is None
    assert bench.explicit_updates([(1001, 1)], "batched", 500, 1, 1, 1.0) is None


def test_traffic_record_is_keyed_by_workload_and_source_digest(tmp_path, monkeypatch):
    digest = bench.kernel_source_digest()
    assert len(digest) == 64
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "a.md").write_text(
        f"`traffic-record: workload=w1 kernel=k source_sha256={digest} "
        f"fetch_bytes_per_launch=10 write_bytes_per_launch=5`\n"
        f"traffic-record: workload=w2 kernel=k source_sha256={'0' * 64} "
        f"fetch_bytes_per_launch=1 write_bytes_per_launch=1\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: digest)
    assert bench.measured_traffic("w1") == 15
    assert bench.measured_traffic("w2") is None       # recorded for other kernel sources
    assert bench.measured_traffic("w3") is None       # no record
