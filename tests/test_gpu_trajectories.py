"""The configured trajectory lengths (Alg. B.1 run for the workloads' step
counts), against the oracle and between the precisions.

  - The 100k-node cube with a sphere (200 steps of 5 ps, CG tolerance 1e-8):
    the FP64 path, the mixed path and the mixed path with both
    preconditioners after all 200 steps against the oracle's state (stored by
    tests/golden/make_trajectory_checkpoints.py, which calls only the
    oracle): m and mean-removed u within 1e-6, the energies within 1e-6, the
    per-step elastic iteration totals of the FP64 path within 1%.
  - The 1M-node cube (10 steps of 10 ps): the FP64 path against the oracle's
    state at 4096 sampled nodes (the full state is too large to store) and its
    cell averages and energies, which the oracle computed over the whole mesh.
  - The 1M-node cube over 500 steps: mixed, mixed with both preconditioners,
    and the same with the corrected GS start (the bench's fastest path)
    against FP64 at steps 20, 100 and 500, within 1e-6 on m and u.
  - The 1M-node cube with the local magnetostatic potential over 25 steps:
    mixed against FP64 within 1e-6 on m, u and U~.
"""
import os

import numpy as np
import pytest

import workloads as w
from paper_2510_09812_amd import gspm

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ENERGY_KEYS = ("exchange", "anisotropy", "zeeman", "magnetoelastic", "stress", "demag_far", "total")


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _demean(u):
    return u - u.mean(axis=0)


def _golden(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not generated (tests/golden/make_trajectory_checkpoints.py)")
    return np.load(path)


def _sim(case, precision, precond=False, **kw):
    p = dict(case.params)
    if precond:
        p["elastic_precond"] = gspm.GSPM_PRECOND_GREEN
        p["gs_precond"] = gspm.GSPM_PRECOND_JACOBI
    sim = gspm.Simulation(case.mesh, p, hext=case.hext, precision=precision, **kw)
    sim.set_m(case.m0)
    return sim


@pytest.mark.parametrize("path", ["fp64", "mixed", "mixed+precond"])
def test_cube47_sphere_200_steps_against_oracle(path):
    ref = _golden("cube47_sphere_oracle.npz")
    case = w.cube47_sphere()
    sim = _sim(case, gspm.GSPM_FP64 if path == "fp64" else gspm.GSPM_MIXED, precond=path.endswith("+precond"))
    mech = []
    for k in range(case.steps):
        mech.append(sim.step(case.dt, 1)["mech_iters"])
    m, u = sim.get_m(), sim.get_u()
    em, eu = _rel(m, ref["m200"]), _rel(_demean(u), _demean(ref["u200"]))
    eg = sim.energies()
    er = dict(zip(ENERGY_KEYS, ref["energies"][-1]))
    ee = max(abs(eg[q] - er[q]) for q in ENERGY_KEYS) / abs(er["total"])
    mbar, _ = sim.averages()
    print(f"[traj] cube47_sphere {path}, 200 steps: m {em:.2e} u {eu:.2e} energies {ee:.2e} "
          f"|dmbar| {np.abs(mbar - ref['mbar'][-1]).max():.2e}; elastic iterations {sum(mech)} "
          f"(oracle {int(ref['mech_iters'].sum())})", flush=True)
    assert em < 1e-6 and eu < 1e-6 and ee < 1e-6
    assert np.abs(mbar - ref["mbar"][-1]).max() < 1e-6
    if path == "fp64":
        assert abs(sum(mech) - int(ref["mech_iters"].sum())) <= 0.01 * int(ref["mech_iters"].sum())
    sim.close()


def test_cube100_ten_steps_against_oracle_sample():
    ref = _golden("cube100_ellipsoids_oracle_sample.npz")
    case = w.cube100_ellipsoids()
    sim = _sim(case, gspm.GSPM_FP64)
    sample = ref["sample"]
    for k in range(1, 11):
        st = sim.step(case.dt, 1)
        mbar, ebar = sim.averages()
        e = sim.energies()
        er = ref["energies"][k - 1]
        de = max(abs(e[q] - er[i]) for i, q in enumerate(ENERGY_KEYS)) / abs(er[-1])
        print(f"[traj] cube100 step {k}: elastic {st['mech_iters']} (oracle {int(ref['mech_iters'][k - 1])}), "
              f"|dmbar| {np.abs(mbar - ref['mbar'][k - 1]).max():.2e}, energies {de:.2e}", flush=True)
        assert np.abs(mbar - ref["mbar"][k - 1]).max() < 1e-8
        assert np.abs(ebar - ref["ebar"][k - 1]).max() < 1e-8 * case.material["lambda100"]
        assert de < 1e-8
        assert abs(st["mech_iters"] - int(ref["mech_iters"][k - 1])) <= 2
        if k in (5, 10):
            m, u = sim.get_m()[sample], sim.get_u()[sample]
            em = _rel(m, ref[f"m{k}"])
            eu = np.abs(u - ref[f"u{k}"]).max() / np.abs(ref[f"u{k}"]).max()
            print(f"[traj] cube100 step {k}: sampled m {em:.2e}, sampled u max {eu:.2e}", flush=True)
            assert em < 1e-8 and eu < 1e-6
    sim.close()


def test_cube100_500_steps_mixed_against_fp64():
    case = w.cube100_ellipsoids()
    sims = {"fp64": _sim(case, gspm.GSPM_FP64), "mixed": _sim(case, gspm.GSPM_MIXED),
            "mixed+precond": _sim(case, gspm.GSPM_MIXED, precond=True),
            "mixed+precond+gscorr": _sim(case, gspm.GSPM_MIXED, precond=True)}
    sims["mixed+precond+gscorr"].set_gs_start(gspm.GSPM_GS_START_CORRECTED)
    done = 0
    for mark in (20, 100, 500):
        for s in sims.values():
            s.step(case.dt, mark - done)
        done = mark
        ref_m, ref_u = sims["fp64"].get_m(), _demean(sims["fp64"].get_u())
        for name in ("mixed", "mixed+precond", "mixed+precond+gscorr"):
            em = _rel(sims[name].get_m(), ref_m)
            eu = _rel(_demean(sims[name].get_u()), ref_u)
            print(f"[traj] cube100 step {mark}: {name} vs fp64 m {em:.2e} u {eu:.2e}", flush=True)
            assert em < 1e-6 and eu < 1e-6
    for s in sims.values():
        s.close()


def test_cube100_local_magnetostatics_mixed_against_fp64():
    case = w.cube100_ellipsoids()
    sims = {p: _sim(case, p, local_demag=True) for p in (gspm.GSPM_FP64, gspm.GSPM_MIXED)}
    for p, s in sims.items():
        st = s.step(case.dt, 25)
        print(f"[traj] cube100 local_demag {'mixed' if p else 'fp64'}: 25 steps, K^ms iterations {st['ms_iters']}",
              flush=True)
    a, b = sims[gspm.GSPM_MIXED], sims[gspm.GSPM_FP64]
    em, eu = _rel(a.get_m(), b.get_m()), _rel(_demean(a.get_u()), _demean(b.get_u()))
    eud = _rel(a.get_ud(), b.get_ud())
    print(f"[traj] cube100 local_demag, 25 steps, mixed vs fp64: m {em:.2e} u {eu:.2e} U~ {eud:.2e}", flush=True)
    assert em < 1e-6 and eu < 1e-6 and eud < 1e-6
    for s in sims.values():
        s.close()
