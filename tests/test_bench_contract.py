"""CPU checks of bench.py's host logic: the HBM traffic and MFMA-busy figures
it reports come from the committed rocprofv3 summary of the headline kernel
and read as null once that kernel's sources differ from the ones the
counters were taken on; runs on more than one GPU are refused."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_profile_figures_match_the_committed_sources():
    assert bench.profiled_traffic() is not None and bench.profiled_traffic() > 0
    busy = bench.profiled("mfma_busy_fraction")
    assert busy is not None and 0.0 < busy < 1.0


def test_profile_figures_are_null_for_other_sources(tmp_path):
    text = open(bench.PROFILE_X3).read()
    lines = []
    for line in text.splitlines():
        if line.startswith("source_sha256: "):
            line = "source_sha256: " + "0" * 64
        lines.append(line)
    stale = tmp_path / "stale.md"
    stale.write_text("\n".join(lines) + "\n")
    assert bench.profiled_traffic(str(stale)) is None
    assert bench.profiled("mfma_busy_fraction", str(stale)) is None
    assert bench.profiled_traffic(str(tmp_path / "missing.md")) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr and r.stdout == ""
