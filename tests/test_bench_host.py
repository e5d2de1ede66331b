"""Host-side logic of bench.py (no GPU): the code hash that keys the stored
HBM counters, and the refusal of multi-GPU runs."""
import os
import shutil
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2404_08371_amd", "csrc")


def _copy_sources(tmp_path):
    for name in bench.KERNEL_SOURCES:
        shutil.copy(os.path.join(CSRC, name), tmp_path / name)
    return str(tmp_path)


def test_code_hash_ignores_comments_and_whitespace(tmp_path):
    d = _copy_sources(tmp_path)
    h0 = bench.kernel_code_hash(csrc=d)
    assert h0 == bench.kernel_code_hash()
    p = tmp_path / bench.KERNEL_SOURCES[0]
    txt = p.read_text()
    p.write_text("// a new leading comment\n/* and a block\n   comment */\n" + txt.replace("\n", "\n\n", 5))
    assert bench.kernel_code_hash(csrc=d) == h0


def test_code_hash_follows_code_edits(tmp_path):
    d = _copy_sources(tmp_path)
    h0 = bench.kernel_code_hash(csrc=d)
    for name in bench.KERNEL_SOURCES:
        p = tmp_path / name
        txt = p.read_text()
        p.write_text(txt + "\nnamespace tmf { constexpr int kHashProbe = 1; }\n")
        assert bench.kernel_code_hash(csrc=d) != h0
        p.write_text(txt)
    assert bench.kernel_code_hash(csrc=d) == h0


def test_multi_gpu_request_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, env=dict(os.environ, PYTHONPATH=ROOT))
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""

