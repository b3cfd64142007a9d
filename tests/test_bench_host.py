"""bench.py's host-side contract, without a GPU: one GPU only (any other
count exits with a message), and the algorithmic bytes of one fused step
launch as the per-unit figures state them."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stdout + r.stderr


def test_step_bytes_per_launch():
    import bench
    nf, nl, nif = 6_695_295, 12_829_908, 2_791_773     # the 256^3 sphere packing
    nt, rw = 105_600, 256 * 256 * 4
    # per fluid node: Q read + Q written for each lattice (FP32) and its dense
    # index and link base (8 B); per link: coefficient read, exchange written;
    # per fluid interface node: solid fraction read and written (FP64); per
    # launch every task record (32 B) and row word (16 B) once
    per_node = (19 + 19) * 4 * 2 + 8
    expect = nf * per_node + nl * (4 + 4) + nif * 16 + nt * 32 + rw * 16
    assert bench.kernel_bytes(19, 4, nf, nl, nif, n_tasks=nt, n_row_words=rw) == expect
    assert bench.kernel_bytes(19, 4, nf, nl, nif) == nf * per_node + nl * 8 + nif * 16
    # the solute on D3Q7: 7 populations instead of 19
    per_node7 = (19 + 7) * 4 * 2 + 8
    assert bench.kernel_bytes(19, 4, nf, 3_397_116, 1_000_000, qs=7) == \
        nf * per_node7 + 3_397_116 * 8 + 1_000_000 * 16
    # FP64 storage doubles the population and link terms
    assert bench.kernel_bytes(9, 8, 100, 10, 5) == 100 * ((9 + 9) * 8 * 2 + 8) + 10 * 16 + 5 * 16


def test_adjoint_bytes_per_launch():
    import bench
    # recomputation: QS read + QS written per node, beta read and the source
    # value written per link; transposed step: the same per node, beta +
    # source read and the step's dL/dbeta term written per link; fold: per
    # link a segment's terms read and the FP64 dL/dbeta read and written
    sol, adj, fold = bench.adjoint_kernel_bytes(19, 4, 939_011, 1_000_000, seg=100)
    assert sol == 939_011 * 19 * 8 + 1_000_000 * 8
    assert adj == 939_011 * 19 * 8 + 1_000_000 * 12
    assert fold == 1_000_000 * (100 * 4 + 16)


if __name__ == "__main__":
    sys.exit(pytest.main([__file__, "-q"]))
