"""Host-side pieces of bench.py that need no GPU: the one-GPU guard, the
rocprofv3 summaries written to profiles/, the traffic figures read back
from them, and the operation count that scales the oracle's CPU rate."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_oracle_operation_count():
    """Multiply-adds of the direct oracle, counted pair by pair on small sizes:
    the chain of convolutions x * x * ..., the correlation with h for y, and
    x * w then the dot product with h for alpha."""
    for n, m in [(1, 2), (5, 2), (7, 3), (4, 5), (9, 4)]:
        count, lw = 0, n
        for _ in range(m - 2):
            count += sum(1 for k in range(lw + n - 1) for j in range(lw) if 0 <= k - j < n)
            lw += n - 1
        dh = m * (n - 1) + 1
        count += sum(1 for i in range(n) for k in range(lw) if i + k < dh)
        count += sum(1 for k in range(lw + n - 1) for j in range(lw) if 0 <= k - j < n) + dh
        assert bench.oracle_macs_per_product(n, m) == count, (n, m)


def test_summarize_stats(tmp_path):
    d = tmp_path / "trace" / "host"
    d.mkdir(parents=True)
    (d / "run_kernel_stats.csv").write_text(
        '"Name","Calls","TotalDurationNs","AverageNs","Percentage","MinNs","MaxNs","StdDev"\n'
        '"small_kernel",10,1000,100,10.0,90,110,1\n'
        '"big_kernel",3,9000,3000,90.0,2900,3100,5\n')
    txt = bench.summarize_stats(str(tmp_path / "trace"), "the command", "a title")
    lines = txt.splitlines()
    assert lines[0] == "# a title" and "the command" in lines[1]
    rows = [ln for ln in lines if ln.startswith("| `")]
    assert rows[0].startswith("| `big_kernel` | 3 | 3.00 |")   # most total time first
    assert rows[1].startswith("| `small_kernel` | 10 | 0.10 |")


def test_committed_traffic_profile_reads_back():
    """The committed per-pass traffic summary parses; when it was taken on the
    current kernel sources, the traffic of each pass is within 5 % of its
    algorithmic bytes (the passes read and write each byte once)."""
    t = bench.load_traffic("c64")
    if t is None:
        pytest.skip("the traffic summary was taken on other kernel sources")
    n_bytes = {"pass_a": (bench.DH + bench.NVEC + 2 * bench.NFFT) * 8, "pass_b": 3 * bench.NFFT * 8,
               "pass_d": (bench.NFFT + bench.NVEC) * 8}
    for k, alg in n_bytes.items():
        assert 0.95 * alg <= t[k] <= 1.05 * alg, (k, t[k], alg)
