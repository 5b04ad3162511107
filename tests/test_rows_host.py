"""Host logic of the GS operator's row form: the rows that mesh upload
assembles (compiled from the library's mesh_prep.cpp and gs_rows.cpp with a
small host checker; no GPU) decode to a symmetric operator whose product
equals the element-by-element sum over the magnetic tets."""
import os
import shutil
import subprocess

import pytest

import workloads as w

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2510_09812_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("rows")
    exe = str(d / "rows_check")
    subprocess.check_call([hipcc, "-O2", "-std=c++17", "-pthread", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
                           os.path.join(ROOT, "tests", "host", "rows_check.cpp"), os.path.join(CSRC, "mesh_prep.cpp"),
                           os.path.join(CSRC, "gs_rows.cpp"), "-o", exe], stderr=subprocess.DEVNULL)
    return exe, d


def _dump(mesh, path):
    import numpy as np
    with open(path, "wb") as f:
        np.array([mesh.xyz.shape[0], mesh.tets.shape[0]], np.int64).tofile(f)
        np.asarray(mesh.lo, np.float64).tofile(f)
        np.asarray(mesh.hi, np.float64).tofile(f)
        mesh.xyz.astype(np.float64).tofile(f)
        mesh.tets.astype(np.int32).tofile(f)
        mesh.tags.astype(np.uint8).tofile(f)


@pytest.mark.parametrize("name,mesh,nb,reorder,nb_rows", [
    ("ragged9_sphere_shuffled", lambda: w.small_cube(9, seed=5, L=8e-8, jitter=0.15, sphere=0.3, shuffle=True).mesh,
     64, 0, 0),
    ("ragged9_sphere_shuffled_rows128", lambda: w.small_cube(9, seed=5, L=8e-8, jitter=0.15, sphere=0.3,
                                                             shuffle=True).mesh, 64, 0, 128),
    ("ragged23_sphere", lambda: w.small_cube(23, seed=6, L=1e-7, jitter=0.15, sphere=0.25).mesh, 256, 0, 0),
    ("ragged23_sphere_rows512", lambda: w.small_cube(23, seed=6, L=1e-7, jitter=0.15, sphere=0.25).mesh, 256, 0, 512),
    ("ragged23_sphere_blocks1024", lambda: w.small_cube(23, seed=6, L=1e-7, jitter=0.15, sphere=0.25).mesh, 1024, 0,
     0),
    ("five17_sphere_shuffled_rows512", lambda: w.small_cube(17, seed=8, L=1e-7, jitter=0.15, sphere=0.3, shuffle=True,
                                                            split="five").mesh, 256, 0, 512),
    ("callers_order", lambda: w.small_cube(15, seed=7, L=1e-7, jitter=0.15, sphere=0.3).mesh, 256, 1, 0),
    ("rcm_order_rows512", lambda: w.small_cube(15, seed=7, L=1e-7, jitter=0.15, sphere=0.3).mesh, 256, 2, 512),
])
def test_gs_rows_decode_to_the_assembled_operator(checker, name, mesh, nb, reorder, nb_rows):
    exe, d = checker
    path = str(d / f"{name}.bin")
    _dump(mesh(), path)
    r = subprocess.run([exe, path, str(nb), str(reorder), str(nb_rows)], capture_output=True, text=True)
    print(r.stdout.strip())
    assert r.returncode == 0, r.stdout
