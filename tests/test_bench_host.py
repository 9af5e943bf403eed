"""CPU checks of bench.py's host-side parts (no GPU): the count of explicitly
evaluated (j, k) pairs, the counter-record lookups and the oracle baseline's
two modes."""
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
        f"`traffic-record: workload=w1 kernel=k_eval_persistent<16> source_sha256={digest} "
        f"fetch_bytes_per_launch=10 write_bytes_per_launch=5`\n"
        f"`traffic-record: workload=w1 kernel=k_lin source_sha256={digest} "
        f"fetch_bytes_per_launch=100 write_bytes_per_launch=7`\n"
        f"traffic-record: workload=w2 kernel=k_eval source_sha256={'0' * 64} "
        f"fetch_bytes_per_launch=1 write_bytes_per_launch=1\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: digest)
    assert bench.measured_traffic("w1", "k_eval") == 15
    assert bench.measured_traffic("w1", "k_lin") == 107
    assert bench.measured_traffic("w1", "k_combine") is None
    assert bench.measured_traffic("w2") is None       # recorded for other kernel sources
    assert bench.measured_traffic("w3") is None       # no record


def test_valu_record_is_keyed_by_workload_and_source_digest(tmp_path, monkeypatch):
    digest = bench.kernel_source_digest()
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "b.md").write_text(
        f"`valu-record: workload=w1 kernel=k_eval_persistent<16> source_sha256={digest} "
        f"sq_insts_valu_per_launch=2.5e11`\n"
        f"`valu-record: workload=w2 kernel=k_eval source_sha256={'1' * 64} sq_insts_valu_per_launch=7`\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: digest)
    assert bench.measured_valu("w1") == 2.5e11
    assert bench.measured_valu("w2") is None
    assert bench.measured_valu("w3") is None


def test_kernel_digest_covers_the_evaluation_sources():
    for rel in bench.KERNEL_SOURCES:
        assert os.path.exists(os.path.join(ROOT, rel)), rel
    assert any(rel.endswith("psl_eval.hip") for rel in bench.KERNEL_SOURCES)
    assert any(rel.endswith("psl_split.hip") for rel in bench.KERNEL_SOURCES)


def test_all_core_threads_follows_affinity_and_omp(monkeypatch):
    info = {"affinity_cpus": 64, "OMP_NUM_THREADS": None}
    assert bench.all_core_threads(info) == 64
    assert bench.all_core_threads(dict(info, OMP_NUM_THREADS="16")) == 16
    assert bench.all_core_threads(dict(info, OMP_NUM_THREADS="128")) == 64
    assert bench.all_core_threads(dict(info, OMP_NUM_THREADS="x")) == 64
    h = bench.host_info()
    assert h["nproc"] >= 1 and h["affinity_cpus"] >= 1


def test_cpu_baseline_has_both_modes():
    out = bench.cpu_baseline(257, 257, 4, 0.05, 2)
    assert out["kind"] == "oracle" and out["unit"] == "flip-evals/s" and out["value"] > 0
    assert out["single_thread"]["cores"] == 1 and out["single_thread"]["value"] > 0
    assert out["cores"] == bench.all_core_threads(bench.host_info())
    assert "cpu_model" in out["host"]
