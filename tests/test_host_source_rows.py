"""Host logic of the tile plan: the source-row lists the host makes for range
tiles match the node metadata the kernel builds (checked by a small C++
program compiled against the plan sources; no GPU)."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2004_03701_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc is not installed")
def test_range_tile_source_rows_match_kernel_metadata(tmp_path):
    exe = str(tmp_path / "check_source_rows")
    subprocess.check_call([HIPCC, "-O2", "-std=c++17", "-I", CSRC, "-o", exe,
                           os.path.join(HERE, "host", "check_source_rows.cpp"),
                           os.path.join(CSRC, "ffa_plan.cpp")],
                          stderr=subprocess.DEVNULL)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.startswith("ok:"), out.stdout
