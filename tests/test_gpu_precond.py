"""The elastic solve with the Green's-operator preconditioner
(elastic_precond = GSPM_PRECOND_GREEN) against the oracle's own
implementation of the same preconditioner and solve.

  - the preconditioner B = Q A_g^+ Q^T + (1/2) D^-1 applied to a vector:
    within 1e-12 of the oracle (FP64; the oracle builds the grid operator's
    symbol from its own stencil and transforms by plain DFTs, the library by
    its own stencil, a symbol kernel and batched FFTs);
  - preconditioned solves at tol 1e-12: within 1e-9 of the oracle's, with the
    iteration count within 1;
  - steps at tol 1e-12 with the preconditioned elastic solve: m and u within
    1e-9 of the oracle's, elastic iterations within 1 per step;
  - the mixed form with the preconditioner against the FP64 plain path over
    several steps at the workloads' tolerance: within the 1e-6 target;
  - the rotated crystal (general stiffness) through the same checks.
"""
import numpy as np
import pytest

import oracle as O
import workloads as w
from paper_2510_09812_amd import gspm

pytestmark = pytest.mark.gpu

H = 200e-9 / 46
R111 = np.array([[1, 1, 1], [-1, 1, 0], [-1, -1, 2]], dtype=np.float64) / np.sqrt([[3.0], [2.0], [6.0]])


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _params(case, rotated=False, tol=None):
    p = dict(case.params)
    p["elastic_precond"] = gspm.GSPM_PRECOND_GREEN
    if rotated:
        p["crystal_rot"] = R111
    if tol is not None:
        p["cg_tol"] = tol
    return p


CASES = {
    "jittered9_sphere_shuffled": lambda: w.small_cube(9, seed=111, L=8 * H, jitter=0.15, sphere=0.3, shuffle=True),
    "regular8": lambda: w.small_cube(8, seed=112, L=7 * H, jitter=0.0),
    "jittered17_sphere": lambda: w.small_cube(17, seed=113, L=16 * H, jitter=0.15, sphere=0.25),
    "five13_sphere_shuffled": lambda: w.small_cube(13, seed=117, L=12 * H, jitter=0.15, sphere=0.3, shuffle=True,
                                                   split="five"),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    print(f"[case {request.param}]", flush=True)
    return CASES[request.param]()


@pytest.mark.parametrize("rotated", [False, True])
def test_preconditioner_matches_oracle(case, rotated):
    p = _params(case, rotated)
    orc = O.Oracle.from_mesh(case.mesh)
    orc.set_params(p)
    sim = gspm.Simulation(case.mesh, p)
    rng = np.random.default_rng(9)
    x = case.mesh.per_site(rng.standard_normal((case.mesh.n_sites, 3)))
    nmap = orc.node_map()
    xu = np.zeros((orc.n, 3)); xu[nmap] = x
    y = sim.apply(gspm.GSPM_OP_PRECOND, x)
    ref = orc.precond_apply(xu)[nmap]
    err = np.abs(y - ref).max() / np.abs(ref).max()
    print(f"B x: grid {orc.precond_grid()}, max rel err {err:.2e}", flush=True)
    assert err < 1e-12
    sim.close()


@pytest.mark.parametrize("rotated", [False, True])
def test_preconditioned_solve_matches_oracle(case, rotated):
    p = _params(case, rotated)
    orc = O.Oracle.from_mesh(case.mesh)
    orc.set_params(p)
    sim = gspm.Simulation(case.mesh, p)
    rng = np.random.default_rng(10)
    b = case.mesh.per_site(rng.standard_normal((case.mesh.n_sites, 3)))
    x0 = case.mesh.per_site(rng.standard_normal((case.mesh.n_sites, 3)) * 1e-3)
    nmap = orc.node_map()
    bu = np.zeros((orc.n, 3)); bu[nmap] = b
    xu0 = np.zeros((orc.n, 3)); xu0[nmap] = x0
    xg, itg = sim.solve(gspm.GSPM_OP_ELASTIC, b, x0, tol=1e-12)
    xo, ito = orc.solve(O.SOLVE_ELASTIC_GREEN, bu, xu0, tol=1e-12)
    err = _rel(xg, xo[nmap])
    _, itp = orc.solve(O.OP_ELASTIC, bu - bu.mean(0), xu0, tol=1e-12)
    print(f"preconditioned solve: iterations gpu {itg} oracle {ito} (plain CG {itp}), rel err {err:.2e}", flush=True)
    assert err < 1e-9
    assert abs(itg - ito) <= 1
    assert np.abs(xg[0]).max() == 0.0          # pinned at the caller's node 0
    sim.close()


def test_steps_with_preconditioner_match_oracle(case):
    p = _params(case, tol=1e-12)
    H_ext = (-0.5 * case.material["Ms"], 0.0, 0.0)
    orc = O.Oracle.from_mesh(case.mesh)
    orc.set_params(p, hext=H_ext)
    orc.set_m(case.m0)
    sim = gspm.Simulation(case.mesh, p, hext=H_ext)
    sim.set_m(case.m0)
    for k in range(3):
        sg = sim.step(2e-12, 1)
        so = orc.step(2e-12, 1)
        em, eu = _rel(sim.get_m(), orc.get_m()), _rel(sim.get_u(), orc.get_u())
        print(f"step {k}: elastic iterations gpu {sg['mech_iters']} oracle {so['mech_iters']}; "
              f"rel err m {em:.2e} u {eu:.2e}", flush=True)
        assert abs(sg["mech_iters"] - so["mech_iters"]) <= 1
        assert em < 1e-9 and eu < 1e-9
    sim.close()


def test_mixed_preconditioned_against_fp64_plain():
    case = w.small_cube(21, seed=114, L=20 * H, jitter=0.15, sphere=0.3, m="noisy_x")
    H_ext = (-0.5 * case.material["Ms"], 0.0, 0.0)
    ref = gspm.Simulation(case.mesh, case.params, hext=H_ext)
    ref.set_m(case.m0)
    mix = gspm.Simulation(case.mesh, _params(case), hext=H_ext, precision=gspm.GSPM_MIXED)
    mix.set_m(case.m0)
    sr = ref.step(1e-11, 10)
    sm = mix.step(1e-11, 10)
    um = lambda u: u - u.mean(axis=0)
    em, eu = _rel(mix.get_m(), ref.get_m()), _rel(um(mix.get_u()), um(ref.get_u()))
    print(f"10 steps: elastic iterations plain FP64 {sr['mech_iters']}, preconditioned mixed {sm['mech_iters']}; "
          f"rel err m {em:.2e} u {eu:.2e}", flush=True)
    assert em < 1e-6 and eu < 1e-6
    assert sm["mech_iters"] < sr["mech_iters"] / 3
    ref.close()
    mix.close()


def test_preconditioner_argument_checks():
    case = w.small_cube(5, seed=115, L=4 * H, jitter=0.15)
    sim = gspm.Simulation(case.mesh, case.params)
    with pytest.raises(gspm.GspmError) as e:
        sim.apply(gspm.GSPM_OP_PRECOND, np.zeros((case.mesh.n_nodes, 3)))
    assert e.value.status == gspm.GSPM_E_STATE
    bad = dict(case.params); bad["elastic_precond"] = 7
    with pytest.raises(gspm.GspmError) as e:
        sim.set_params(bad)
    assert e.value.status == gspm.GSPM_E_ARG
    sim.close()
    mix = gspm.Simulation(case.mesh, _params(case), precision=gspm.GSPM_MIXED)
    with pytest.raises(gspm.GspmError) as e:
        mix.apply(gspm.GSPM_OP_PRECOND, np.zeros((case.mesh.n_nodes, 3)))
    assert e.value.status == gspm.GSPM_E_STATE
    mix.close()


# ------------------------------------------------- Jacobi-preconditioned GS

def _gs_eps(case, dt=1e-11):
    p = case.params
    return 2 * p["A"] / (p["mu0"] * p["Ms"] ** 2) * p["gamma0"] * p["Ms"] * dt


def test_jacobi_gs_solve_matches_oracle(case):
    p = dict(case.params); p["gs_precond"] = gspm.GSPM_PRECOND_JACOBI
    orc = O.Oracle.from_mesh(case.mesh)
    orc.set_params(p)
    sim = gspm.Simulation(case.mesh, p)
    eps = _gs_eps(case)
    rng = np.random.default_rng(14)
    b = case.mesh.per_site(rng.standard_normal((case.mesh.n_sites, 3)))
    nmap = orc.node_map()
    bu = np.zeros((orc.n, 3)); bu[nmap] = b
    xg, itg = sim.solve(gspm.GSPM_OP_GS, b, eps=eps, tol=1e-12)
    xo, ito = orc.solve(O.OP_GS, bu, eps=eps, tol=1e-12)
    err = _rel(xg, xo[nmap])
    print(f"Jacobi GS solve (3 components): iterations gpu {itg} oracle {ito}, rel err {err:.2e}", flush=True)
    assert err < 1e-9
    assert abs(itg - ito) <= 3
    sim.close()


def test_steps_with_both_preconditioners_match_oracle(case):
    p = _params(case, tol=1e-12); p["gs_precond"] = gspm.GSPM_PRECOND_JACOBI
    H_ext = (-0.5 * case.material["Ms"], 0.0, 0.0)
    orc = O.Oracle.from_mesh(case.mesh)
    orc.set_params(p, hext=H_ext)
    orc.set_m(case.m0)
    sim = gspm.Simulation(case.mesh, p, hext=H_ext)
    sim.set_m(case.m0)
    for k in range(3):
        sg = sim.step(5e-12, 1)
        so = orc.step(5e-12, 1)
        em, eu = _rel(sim.get_m(), orc.get_m()), _rel(sim.get_u(), orc.get_u())
        print(f"step {k}: elastic {sg['mech_iters']}/{so['mech_iters']}, GS {sg['gs_iters']}/{sum(so['gs_iters'])} "
              f"(gpu/oracle); rel err m {em:.2e} u {eu:.2e}", flush=True)
        assert abs(sg["mech_iters"] - so["mech_iters"]) <= 1
        assert abs(sg["gs_iters"] - sum(so["gs_iters"])) <= 8
        assert em < 1e-9 and eu < 1e-9
    sim.close()


def test_mixed_with_both_preconditioners_against_fp64_plain():
    case = w.small_cube(21, seed=116, L=20 * H, jitter=0.15, sphere=0.3, m="noisy_x")
    H_ext = (-0.5 * case.material["Ms"], 0.0, 0.0)
    ref = gspm.Simulation(case.mesh, case.params, hext=H_ext)
    ref.set_m(case.m0)
    p = _params(case); p["gs_precond"] = gspm.GSPM_PRECOND_JACOBI
    mix = gspm.Simulation(case.mesh, p, hext=H_ext, precision=gspm.GSPM_MIXED)
    mix.set_m(case.m0)
    sr = ref.step(1e-11, 10)
    sm = mix.step(1e-11, 10)
    um = lambda u: u - u.mean(axis=0)
    em, eu = _rel(mix.get_m(), ref.get_m()), _rel(um(mix.get_u()), um(ref.get_u()))
    print(f"10 steps: GS iterations plain FP64 {sr['gs_iters']}, preconditioned mixed {sm['gs_iters']}; "
          f"rel err m {em:.2e} u {eu:.2e}", flush=True)
    assert em < 1e-6 and eu < 1e-6
    assert sm["gs_iters"] < 0.8 * sr["gs_iters"]
    ref.close()
    mix.close()
