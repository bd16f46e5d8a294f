"""Host-side checks of bench.py (no GPU): the committed traffic summary belongs to the current
kernel sources, the byte model of a loop round, and the one-GPU rule."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402  (imports no GPU module at load time)


def test_traffic_summary_matches_the_kernel_sources():
    # the x-pass traffic the benchmark line carries comes from counters taken with the sources
    # in the tree (their digest is recorded in the summary); a kernel change without new
    # counters would leave the line's traffic empty
    n = 512
    M = n * n * (n // 2 + 1)
    alg = bench.pass_bytes("x_pass", n ** 3, M, 4, 8)
    t = bench.measured_traffic("x_pass", 0)
    assert t is not None, "profiles/ traffic summary was taken with other kernel sources"
    assert 1.0 <= t / alg <= 1.1, t / alg  # row padding only: rows of 257 entries at a pitch of 272


def test_round_byte_model():
    # a loop round reads and writes the half spectrum once per pass: 8 M c (the model of the
    # steady-round figure)
    n = 256
    M = n * n * (n // 2 + 1)
    assert sum(bench.pass_bytes(k, n ** 3, M, 4, 8) for k in bench.LOOP_KINDS) == 8 * M * 8
    assert bench.pass_bytes("verify_x", n ** 3, M, 4, 8) == M * 16


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, env={**os.environ, "WORLD_SIZE": "1"})
    assert r.returncode != 0
    assert "one GPU" in r.stderr
