"""Host logic of the tet-strip operators: the segment encoding that mesh
upload builds (compiled from the library's mesh_prep.cpp with a small host
checker; no GPU) decodes to exactly each block's element list."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import workloads as w

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2510_09812_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("strips")
    exe = str(d / "strip_check")
    subprocess.check_call([hipcc, "-O2", "-std=c++17", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
                           os.path.join(ROOT, "tests", "host", "strip_check.cpp"), os.path.join(CSRC, "mesh_prep.cpp"),
                           "-o", exe], stderr=subprocess.DEVNULL)
    return exe, d


def _dump(mesh, path):
    with open(path, "wb") as f:
        np.array([mesh.xyz.shape[0], mesh.tets.shape[0]], np.int64).tofile(f)
        np.asarray(mesh.lo, np.float64).tofile(f)
        np.asarray(mesh.hi, np.float64).tofile(f)
        mesh.xyz.astype(np.float64).tofile(f)
        mesh.tets.astype(np.int32).tofile(f)
        mesh.tags.astype(np.uint8).tofile(f)


@pytest.mark.parametrize("name,mesh,nb", [
    ("ragged9_sphere_shuffled", lambda: w.small_cube(9, seed=5, L=8e-8, jitter=0.15, sphere=0.3, shuffle=True).mesh, 64),
    ("ragged9_sphere_shuffled", lambda: w.small_cube(9, seed=5, L=8e-8, jitter=0.15, sphere=0.3, shuffle=True).mesh, 1024),
    ("cube10", lambda: w.cube10_random().mesh, 256),
    ("ragged23_sphere", lambda: w.small_cube(23, seed=6, L=1e-7, jitter=0.15, sphere=0.25).mesh, 256),
    ("five17_sphere_shuffled", lambda: w.small_cube(17, seed=8, L=1e-7, jitter=0.15, sphere=0.3, shuffle=True,
                                                    split="five").mesh, 256),
])
def test_strip_segments_decode_to_the_element_lists(checker, name, mesh, nb):
    exe, d = checker
    path = str(d / f"{name}.bin")
    _dump(mesh(), path)
    r = subprocess.run([exe, path, str(nb)], capture_output=True, text=True)
    print(r.stdout.strip())
    assert r.returncode == 0, r.stdout
    loads = float(r.stdout.split("loads/elem ")[1].split()[0])
    assert loads < 2.0       # strips share faces: far fewer than 4 loads per element (short segments at nb 64)


@pytest.mark.parametrize("reorder", [1, 2])
def test_strips_under_the_other_node_orders(checker, reorder):
    """The caller's order (1) and reverse Cuthill-McKee (2) give other owner
    blocks and halos; the encoding must still decode to the element lists."""
    exe, d = checker
    path = str(d / f"order{reorder}.bin")
    _dump(w.small_cube(15, seed=7, L=1e-7, jitter=0.15, sphere=0.3).mesh, path)
    r = subprocess.run([exe, path, "256", str(reorder)], capture_output=True, text=True)
    print(r.stdout.strip())
    assert r.returncode == 0, r.stdout
