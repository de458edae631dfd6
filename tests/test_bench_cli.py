"""Host checks of bench.py (no GPU): the one-GPU refusal, the algorithmic
byte counts of the timed kernels at the 2049 x 2049 sizes, and the reading
of the committed counter records."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_no_gpu_exits_with_a_message():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "1"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 1 and "no GPU" in r.stderr


def test_algorithmic_bytes_at_2049():
    # 2049^2 fine mesh, k = 3: 4,198,401 fine nodes and 29,372,417 nonzeros;
    # 257^2 pressure mesh: 131,072 triangles, 197,120 edges, 66,049 vertices
    nf, zf, t, e, v = 4198401, 29372417, 131072, 197120, 66049
    mass = bench.KERNELS["mass_spmv"][1]
    # lattice size 8: the step over the coarse-edge and vertex nodes, from the
    # even node at or below the 21 t interior nodes
    r = nf - 21 * t
    assert r == 7 * e + v and (21 * t) % 2 == 0
    assert mass(nf, zf, 3, t, e, v, 3) == (96 * r + r + 360 * t + 16 * e + 32 * t
                                           + 12 * (2 * e + v)) == 200308845
    # other lattice sizes: the step over every node
    assert mass(nf, zf, 3, t, e, v, 2) == 422221941
    pair = bench.KERNELS["mass_pair"][1]
    assert pair(nf, zf, 3, t, e, v, 3) == 21 * t * 121 + 7 * e * 48 + 32 * t == 403480576
    # the interior and edge ranges cover the vector
    assert 21 * t + 7 * e + v == nf
    mom = bench.KERNELS["mom_spmv"][1]
    assert mom(nf, zf, 3, t, e, v, 3) == 12 * zf + 4 * (nf + 1) + 48 * nf == 570785860
    pcg = bench.KERNELS["coarse_spmv"][1]
    # the fine-scale calibration: the 2049^2 square as the Poisson mesh
    assert pcg(nf, zf, 0, 0, 0, 0, 0) == 738721900


def test_counter_records_are_read_or_declined():
    for (workload, kernel), (name, sources) in bench.TRAFFIC_RECORDS.items():
        assert os.path.exists(os.path.join(ROOT, "profiles", name)), name
        for f in sources:
            assert os.path.exists(os.path.join(ROOT, "paper_1812_00185_amd", "csrc", f)), f
        traffic, src = bench.stored_traffic(workload, kernel)
        if traffic is None:
            assert "changed" in src
        else:
            assert traffic > 0 and src == f"profiles/{name}"
    assert bench.stored_traffic("nowhere", "mass_spmv")[0] is None
