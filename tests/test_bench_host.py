"""Host-side logic of bench.py (no GPU): the one-GPU contract and the
roofline's algorithmic bytes per pass."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


class FakeSim:
    """Resident bytes after the basis encode and after each gate."""

    def __init__(self, resident):
        self.resident = list(resident)
        self.k = -1

    def set_basis(self, x):
        self.k = 0

    def apply(self, g):
        self.k += 1

    def stats(self):
        return {"resident_bytes": self.resident[self.k]}


def test_pass_stream_bytes_counts_streams_in_and_out_plus_metadata():
    # n = 12, b = 8: s = 8, 16 segments, 32 planes; metadata per pass
    # 12 B per plane (two 4-byte record offsets, one size word) + 8 B per
    # segment = 384 + 128 = 512 B
    n, b = 12, 8
    res = [1000, 3000, 2000]  # after the basis encode, gate 1, gate 2
    total = bench.pass_stream_bytes(FakeSim(res), 0, ["g1", "g2"], n, b)
    meta = 12 * 32 + 8 * 16
    want = (1000 + meta) + (1000 + 3000 + meta) + (3000 + 2000 + meta)
    assert total == want
