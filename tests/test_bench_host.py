"""Host logic of bench.py (no GPU): the algorithmic byte counts behind the
roofline lines and the rule that counter traffic is reported only for the
kernel sources and the workload it was measured on."""
import json
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

N1M, NE1M = 970299, 5821794


def test_algorithmic_bytes_at_the_1m_node_cube():
    # the method's count per elastic CG iteration: connectivity 16 B per tet,
    # FP64 coordinates 24 B per node, nine passes over 3-vectors
    assert bench.cg_iteration_bytes(N1M, NE1M, 8) == 16 * NE1M + 24 * N1M + 216 * N1M
    assert abs(bench.cg_iteration_bytes(N1M, NE1M, 8) / 1e6 - 326.0) < 0.1
    assert abs(bench.cg_iteration_bytes(N1M, NE1M, 4) / 1e6 - 221.2) < 0.1
    assert abs(bench.ms_matvec_bytes(N1M, NE1M, 4) / 1e6 - 124.2) < 0.1
    # at exactly six tetrahedra per node: 336 and 228 B per node (elastic), 192 and 156 (GS)
    n = 1000
    assert bench.cg_iteration_bytes(n, 6 * n, 8) == 336 * n
    assert bench.cg_iteration_bytes(n, 6 * n, 4) == 228 * n
    assert bench.gs_iteration_bytes(n, 6 * n, 8) == 192 * n
    assert bench.gs_iteration_bytes(n, 6 * n, 4) == 156 * n
    # the fused GS iteration on three components: the magnetic tets' connectivity and the coordinates once,
    # nine passes per component, the Jacobi diagonal once (5,811,637 magnetic tets at the 1M-node cube)
    nem = 5811637
    assert bench.gs3_iteration_bytes(N1M, nem, 4, jacobi=True) == 16 * nem + 24 * N1M + 27 * 4 * N1M + 4 * N1M
    assert bench.gs3_iteration_bytes(N1M, nem, 4, jacobi=True) == 224946856
    assert bench.gs3_iteration_bytes(N1M, nem, 8, jacobi=False) == 16 * nem + 24 * N1M + 27 * 8 * N1M


def test_step_bytes_in_both_precisions():
    n, ne = 1000, 6000
    base = 3 * (16 * ne + 96 * n) + 200 * n                 # three RHS passes (192 B/node) + node passes
    assert bench.step_bytes(n, ne, 0, 0) == base
    # FP64 path: 150 elastic and 40 GS iterations at 336 and 192 B per node
    assert bench.step_bytes(n, ne, 150, 40, 8) == base + 150 * 336 * n + 40 * 192 * n
    # mixed path: inner iterations at FP32 bytes, refinements at FP64
    ref3 = 16 * ne + 24 * n + 3 * 56 * n
    ref1 = 16 * ne + 24 * n + 56 * n
    got = bench.step_bytes(n, ne, 150, 40, 4, mech_refinements=2, other_refinements=8)
    assert got == base + 150 * 228 * n + 40 * 156 * n + 2 * ref3 + 8 * ref1
    # the FP32 step moves fewer bytes than the FP64 one at equal iteration counts
    assert bench.step_bytes(n, ne, 150, 40, 4) < bench.step_bytes(n, ne, 150, 40, 8)


@pytest.mark.parametrize("family,path", [("elastic", "mixed"), ("gs", "mixed+precond")])
def test_traffic_is_tied_to_sources_and_workload(tmp_path, monkeypatch, family, path):
    rel, sources = bench.TRAFFIC[family]
    with open(os.path.join(bench.ROOT, rel)) as f:
        t = json.load(f)
    assert t["workload"].startswith("cube100_ellipsoids ")
    current = t["kernel_hash"] == bench.kernel_hash(family)
    fake = dict(t)
    tmp = tmp_path / "traffic.json"
    tmp.write_text(json.dumps(fake))
    monkeypatch.setitem(bench.TRAFFIC, family, (str(tmp), sources))
    got = bench.traffic_from_profile(family, path)
    assert (got == fake[path]["bytes_per_launch"]) if current else got is None
    assert bench.traffic_from_profile(family, path, "cube144_ellipsoids") is None
    fake["kernel_hash"] = "0" * 16
    tmp.write_text(json.dumps(fake))
    assert bench.traffic_from_profile(family, path) is None


def test_rotation_of_the_bench_path_is_app_d_frame():
    R = bench.R111
    assert np.allclose(R @ R.T, np.eye(3), atol=1e-15) and abs(np.linalg.det(R) - 1.0) < 1e-15
    assert np.allclose(R[0], np.ones(3) / np.sqrt(3.0))


def test_more_than_one_gpu_is_refused_with_a_message():
    import subprocess
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_preconditioned_step_bytes_and_grid():
    import workloads as w
    case = w.cube10_random()
    g = bench.precond_grid(case.mesh.lo, case.mesh.hi, 729)
    assert g == [9, 9, 9]
    n, ne = 1000, 6000
    plain = bench.step_bytes(n, ne, 100, 40, 4)
    pc = bench.step_bytes(n, ne, 100, 40, 4, precond=True, grid=(10, 10, 10))
    # each preconditioned iteration adds the preconditioner, and the Jacobi diagonal to the GS ones
    per_it = bench.pcg_matvec_bytes(n, ne, 4) + 60 * n + bench.precond_bytes(n, (10, 10, 10), 4)
    assert pc - plain == 100 * (per_it - bench.cg_iteration_bytes(n, ne, 4)) + 40 * 4 * n
    assert bench.gs3_iteration_bytes(n, ne, 4, jacobi=False) == 16 * ne + 24 * n + 108 * n
    assert bench.gs3_iteration_bytes(n, ne, 4) == 16 * ne + 24 * n + 112 * n
