"""Host-side checks of the benchmark's bookkeeping: the operator applications
it counts per step, the rank of the split adjoint's phase product that its
VALU-inclusive bound uses, and its refusal of more than one GPU.  No GPU is
used."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_applications_per_step():
    """20 power steps (A and A^H each), the Rayleigh quotient (FP32: one A;
    split forms: A and A^H), the lambda rule's A^H (also iteration 0's
    gradient) and A + A^H in the other 49 of 50 iterations."""
    assert bench.applications("fp32", 50) == 40 + 1 + 1 + 98 == 140
    assert bench.applications("bf16", 50) == bench.applications("fp16", 50) == 40 + 2 + 1 + 98 == 141
    assert bench.applications("bf16", 1, n_power=0) == 3


def _rank_brute(n):
    """Average rank by walking the padded row-major pixel index block by
    block: 6 for a 32-pixel block inside one row, 10 for one that continues
    into the next row."""
    nxq = 16 * ((n + 15) // 16)
    total, ranks = nxq * n, []
    for start in range(0, total, 32):
        rows = {(start + k) // nxq for k in range(32)}
        ranks.append(6 if len(rows) == 1 else 10)
    return sum(ranks) / len(ranks)


@pytest.mark.parametrize("n", [20, 32, 148, 170, 200])
def test_adjoint_phase_rank(n):
    assert bench.adjoint_phase_rank(n) == pytest.approx(_rank_brute(n), abs=1e-12)


def test_adjoint_phase_rank_benchmark_grids():
    # 148 px rows pad to 160 = 5 blocks: every block stays in its row
    assert bench.adjoint_phase_rank(148) == 6.0
    # 200 px rows pad to 208 = 6.5 blocks: one block in 13 continues
    assert bench.adjoint_phase_rank(200) == pytest.approx(6 + 4 / 13)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""
