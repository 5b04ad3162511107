"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the library's mesh preparation and row assembly (mesh_prep.cpp, gs_rows.cpp,
driven by the strip and row checkers) and the oracle (driven by a small C
program through two plain steps, one with both preconditioners and one with
the local magnetostatic potential).  Any invalid access, leak or undefined
operation aborts the run."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import workloads as w

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2510_09812_amd", "csrc")
HOST = os.path.join(ROOT, "tests", "host")
# host-only sanitizer flags for hipcc (each placed after -Xarch_host)
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all"]
HIPCC_SAN = [x for f in SAN for x in ("-Xarch_host", f)]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="2")


def _dump(mesh, path):
    with open(path, "wb") as f:
        np.array([mesh.xyz.shape[0], mesh.tets.shape[0]], np.int64).tofile(f)
        np.asarray(mesh.lo, np.float64).tofile(f)
        np.asarray(mesh.hi, np.float64).tofile(f)
        mesh.xyz.astype(np.float64).tofile(f)
        mesh.tets.astype(np.int32).tofile(f)
        mesh.tags.astype(np.uint8).tofile(f)


@pytest.fixture(scope="module")
def tools(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    gcc = shutil.which("gcc")
    if not os.path.exists(hipcc) or gcc is None:
        pytest.skip("compilers not available")
    d = tmp_path_factory.mktemp("san")
    inc = ["-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
    exes = {}
    for name in ("strip_check", "rows_check"):
        exe = str(d / name)
        subprocess.check_call([hipcc, "-O1", "-g", "-fno-omit-frame-pointer", "-std=c++17", "-pthread"] + HIPCC_SAN +
                              inc + [os.path.join(HOST, name + ".cpp"), os.path.join(CSRC, "mesh_prep.cpp"),
                                     os.path.join(CSRC, "gs_rows.cpp"), "-o", exe], stderr=subprocess.DEVNULL)
        exes[name] = exe
    exe = str(d / "oracle_check")
    subprocess.check_call([gcc, "-O1", "-g", "-fno-omit-frame-pointer", "-std=gnu11", "-fopenmp"] + SAN +
                          ["-I" + os.path.join(ROOT, "oracle"), os.path.join(HOST, "oracle_check.c"),
                           os.path.join(ROOT, "oracle", "gspm_oracle.c"), "-lm", "-o", exe])
    exes["oracle_check"] = exe
    return exes, d


MESHES = {
    "ragged9_sphere_shuffled": lambda: w.small_cube(9, seed=5, L=8e-8, jitter=0.15, sphere=0.3, shuffle=True).mesh,
    "five9_sphere": lambda: w.small_cube(9, seed=9, L=1e-7, jitter=0.15, sphere=0.3, split="five").mesh,
}


@pytest.mark.parametrize("name", list(MESHES))
def test_mesh_preparation_under_sanitizers(tools, name):
    exes, d = tools
    path = str(d / f"{name}.bin")
    _dump(MESHES[name](), path)
    for exe, args in (("strip_check", ["64"]), ("strip_check", ["256", "2"]), ("rows_check", ["64", "0", "128"]),
                      ("rows_check", ["256", "1"])):
        r = subprocess.run([exes[exe], path] + args, capture_output=True, text=True, env=ENV)
        print(exe, args, r.stdout.strip()[-300:])
        assert r.returncode == 0, r.stdout + r.stderr[-3000:]
        assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]


@pytest.mark.parametrize("name", list(MESHES))
def test_oracle_under_sanitizers(tools, name):
    exes, d = tools
    path = str(d / f"o_{name}.bin")
    _dump(MESHES[name](), path)
    r = subprocess.run([exes["oracle_check"], path], capture_output=True, text=True, env=ENV, timeout=600)
    print(r.stdout.strip())
    assert r.returncode == 0, r.stdout + r.stderr[-3000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]
