"""The mixed form (FP64 iterative refinement around FP32 inner CG) against the
FP64 oracle.  Both stop at ||b - A x|| <= tol ||b||; the mixed form tests the
true FP64 residual.  Bounds: m and mean-removed u within 1e-6 relative at
the workload CG tolerance 1e-8 (the stated accuracy target of the mixed
form); the energy functional, which the mixed form evaluates in FP64, within
1e-9 of the oracle's on the same state."""
import numpy as np
import pytest

import oracle as O
import workloads as w
from paper_2510_09812_amd import gspm

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _demean(u):
    return u - u.mean(axis=0)


@pytest.mark.parametrize("seed", [201, 202])
def test_mixed_solves_reach_true_residual(seed):
    case = w.small_cube(11, seed=seed, L=1e-7, jitter=0.15, sphere=0.25, shuffle=True)
    orc = O.Oracle.from_mesh(case.mesh)
    orc.set_params(case.params)
    sim = gspm.Simulation(case.mesh, case.params, precision=gspm.GSPM_MIXED)
    rng = np.random.default_rng(seed)
    nmap = orc.node_map()
    for op, oop, eps in ((gspm.GSPM_OP_GS, O.OP_GS, 3e-17), (gspm.GSPM_OP_ELASTIC, O.OP_ELASTIC, 0.0)):
        b = case.mesh.per_site(rng.standard_normal((case.mesh.n_sites, 3)))
        bu = np.zeros((orc.n, 3)); bu[nmap] = b
        x, it = sim.solve(op, b, None, eps, tol=1e-10)
        xr, itr = orc.solve(oop, bu, None, eps, tol=1e-13)
        xu = np.zeros((orc.n, 3)); xu[nmap] = x
        r = orc.apply(oop, xu, eps) - bu
        if oop == O.OP_ELASTIC:
            r[orc.pinned_node()] = 0.0; bu[orc.pinned_node()] = 0.0
        else:
            mag = orc.lumped_weights() > 0
            r[~mag] = 0.0; bu[~mag] = 0.0
        cols = [0] if oop == O.OP_ELASTIC else [0, 1, 2]
        for c in cols:
            rc = r if oop == O.OP_ELASTIC else r[:, c]
            bc = bu if oop == O.OP_ELASTIC else bu[:, c]
            assert np.linalg.norm(rc) <= 1e-10 * np.linalg.norm(bc) * 1.0001
        err = _rel(x, xr[nmap])
        print(f"mixed solve {op}: iters {it} (fp64 oracle {itr}) rel err vs tight oracle {err:.2e}", flush=True)
        assert err < 1e-6
    sim.close()


@pytest.mark.parametrize("name,steps", [("cube10_random", 20), ("cube47_sphere", 10)])
def test_mixed_steps_match_fp64_oracle(name, steps):
    case = w.CASES[name]()
    orc = O.Oracle.from_mesh(case.mesh)
    orc.set_params(case.params, hext=case.hext)
    orc.set_m(case.m0)
    sim = gspm.Simulation(case.mesh, case.params, hext=case.hext, precision=gspm.GSPM_MIXED)
    sim.set_m(case.m0)
    st = sim.step(case.dt, steps)
    ost = orc.step(case.dt, steps)
    m, u = sim.get_m(), sim.get_u()
    em = _rel(m, orc.get_m())
    eu = _rel(_demean(u), _demean(orc.get_u()))
    eg, er = sim.energies(), orc.energies()
    e_traj = abs(eg["total"] - er["total"]) / abs(er["total"])
    # the energy functional on the mixed run's own state, evaluated by the oracle
    orc2 = O.Oracle.from_mesh(case.mesh)
    orc2.set_params(case.params, hext=case.hext)
    orc2.set_m(m)
    orc2.set_u(u)
    e2 = orc2.energies()
    e_state = max(abs(eg[k] - e2[k]) / abs(e2["total"]) for k in e2)
    print(f"{name}: m {em:.2e} u {eu:.2e} energy along trajectory {e_traj:.2e} energy on state {e_state:.2e} | "
          f"inner iters mech {st['mech_iters']} gs {st['gs_iters']} refinements {st['refinements']} | "
          f"fp64 oracle mech {ost['mech_iters']} gs {sum(ost['gs_iters'])}", flush=True)
    assert em < 1e-6 and eu < 1e-6
    assert e_state < 1e-9
    r = np.linalg.norm(m, axis=1)
    assert np.abs(r[r > 0] - 1.0).max() < 1e-14
    sim.close()
