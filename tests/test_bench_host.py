"""Host logic of bench.py (no GPU): the one-GPU guard, the closed forms of the algorithmic
work, and the reader of the committed HBM-traffic records (source hash check, scaling of
a sweep's record to the run's fraction of non-identity proposals)."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_sv_flops_and_bytes_closed_forms():
    n, N, M = 7, 3, 5
    # complex: z = sigma V (8 n N M), y and w (16 n M), the visible term (4 n N)
    assert bench.sv_flops(n, N, M, True) == 8 * n * N * M + 16 * n * M + 4 * n * N
    assert bench.sv_flops(n, N, M, False) == 4 * n * N * M + 6 * n * M + 4 * n * N
    P = N + M + N * M
    assert bench.sv_bytes(n, N, M, True, True) == n * M * 8 + 8 * n + 2 * P * 16
    assert bench.sv_bytes(n, N, M, False, False) == n * M * 4 + n * N + 2 * P * 8


def _record(tmp_path, src_text, digest, extra=""):
    (tmp_path / "profiles").mkdir()
    (tmp_path / "src.hip").write_text(src_text)
    (tmp_path / "profiles" / "traffic_k_x_w.md").write_text(
        "# record\n\n- sources: `src.hip`\n- sources_sha256: `%s`\n%s"
        "- hbm_bytes_per_launch: `1000`\n" % (digest, extra))


def test_recorded_traffic_checks_the_source_hash(tmp_path, monkeypatch):
    good = hashlib.sha256(b"kernel v1").hexdigest()
    _record(tmp_path, "kernel v1", good)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.recorded_traffic("k_x", "w") == 1000.0
    assert bench.recorded_traffic("k_y", "w") is None          # no record
    (tmp_path / "src.hip").write_text("kernel v2")             # sources changed
    assert bench.recorded_traffic("k_x", "w") is None


def test_recorded_sweep_traffic_scales_with_the_proposal_fraction(tmp_path, monkeypatch):
    good = hashlib.sha256(b"sweep").hexdigest()
    _record(tmp_path, "sweep", good, "- real_move_fraction: `0.5`\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.recorded_traffic("k_x", "w") == 1000.0
    assert bench.recorded_traffic("k_x", "w", 0.6) == pytest.approx(1200.0)


@pytest.mark.parametrize("name", sorted(f for f in os.listdir(os.path.join(ROOT, "profiles"))
                                        if f.startswith("traffic_")))
def test_committed_traffic_records_match_the_sources(name):
    kernel_workload = name[len("traffic_"):-len(".md")]
    # the kernel name is the record name up to the workload (workloads start with a model)
    for w in list(bench.WORKLOADS):
        if kernel_workload.endswith("_" + w):
            kernel = kernel_workload[:-len(w) - 1]
            assert bench.recorded_traffic(kernel, w) is not None, name
            return
    pytest.fail("no workload for " + name)
