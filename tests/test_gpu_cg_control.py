"""Control paths of the CG solves, against the CPU oracle's CG (Sec. 2.5,
stopping rule of Sec. 3.1).

The elastic solve runs single-reduction CG (one fused launch per iteration,
the stopping test one launch behind, the last permitted iteration completed
by a final launch); the GS solves run the two-launch form.  These tests pin
the edge cases of that control on a small mesh with an inclusion:

  - an iteration budget that runs out: status GSPM_E_NOCONV and the iterate
    after exactly maxit CG updates, which equals the oracle's iterate after
    the same budget (1e-9 relative: the two CGs take the same steps);
  - a zero right-hand side: x = 0 exactly, no iteration;
  - a start that already meets the tolerance: no iteration, x unchanged;
  - tolerances from loose to tight: the oracle's iteration count (within 1)
    and its solution (0.1 tol relative at equal counts, 100 tol one apart).

The elastic cases run in FP64 and in the mixed form (zero right-hand side and
converged start only: the mixed form's iterates differ from FP64 CG's by
design).
"""
import ctypes

import numpy as np
import pytest

import oracle as O
import workloads as w
from paper_2510_09812_amd import gspm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def case():
    return w.small_cube(8, seed=31, L=8e-8, jitter=0.15, sphere=0.3)


def _site_vector(mesh, rng, scale=1.0):
    return mesh.per_site(rng.standard_normal((mesh.n_sites, 3)) * scale)


def _gpu_solve(sim, op, b, x0, eps, tol, maxit):
    """The C-ABI call itself: status, x and iterations also on failure."""
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.ascontiguousarray(x0, dtype=np.float64).copy()
    it = ctypes.c_int32(0)
    st = gspm.load().gspm_solve(sim.ctx, op, eps, gspm._dp(b), gspm._dp(x), b.shape[0], tol, maxit,
                                ctypes.byref(it))
    return st, x, it.value


def _oracle_solve(orc, which, b, x0, eps, tol, maxit):
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.ascontiguousarray(x0, dtype=np.float64).copy()
    it = ctypes.c_int32(0)
    rc = orc._lib.or_solve(orc._h, which, eps, O._dp(b), O._dp(x), tol, maxit, ctypes.byref(it))
    return rc, x, it.value


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


OPS = [("elastic", gspm.GSPM_OP_ELASTIC, O.OP_ELASTIC, 0.0), ("gs", gspm.GSPM_OP_GS, O.OP_GS, 3e-17)]


@pytest.mark.parametrize("name,op,oop,eps", OPS)
@pytest.mark.parametrize("maxit", [1, 2, 7, 20])
def test_budget_exhaustion_returns_the_oracle_iterate(case, name, op, oop, eps, maxit):
    mesh = case.mesh
    orc = O.Oracle.from_mesh(mesh)
    orc.set_params(case.params)
    nmap = orc.node_map()
    sim = gspm.Simulation(mesh, case.params)
    rng = np.random.default_rng(40 + maxit)
    b = _site_vector(mesh, rng)
    x0 = _site_vector(mesh, rng, 0.1)
    bu = np.zeros((orc.n, 3)); bu[nmap] = b
    xu = np.zeros((orc.n, 3)); xu[nmap] = x0
    st, x, it = _gpu_solve(sim, op, b, x0, eps, 1e-14, maxit)
    if op == gspm.GSPM_OP_ELASTIC:
        rc, xr, itr = _oracle_solve(orc, oop, bu, xu, eps, 1e-14, maxit)
        errs = [_rel(x, xr[nmap])]
        rcs = [rc]
    else:
        # the oracle's GS call stops at the first component that runs out of
        # iterations: give it each component alone, in the first slot
        errs, rcs = [], []
        for c in range(3):
            bc = np.zeros_like(bu); bc[:, 0] = bu[:, c]
            xc = np.zeros_like(xu); xc[:, 0] = xu[:, c]
            rc, xr, itr = _oracle_solve(orc, oop, bc, xc, eps, 1e-14, maxit)
            errs.append(_rel(x[:, c], xr[nmap][:, 0]))
            rcs.append(rc)
    print(f"{name} maxit {maxit}: status {st} oracle {rcs} iters {it} rel err {max(errs):.2e}", flush=True)
    assert st == gspm.GSPM_E_NOCONV and all(rc == -5 for rc in rcs)
    assert max(errs) < 1e-9
    sim.close()


@pytest.mark.parametrize("precision", [gspm.GSPM_FP64, gspm.GSPM_MIXED])
@pytest.mark.parametrize("name,op,oop,eps", OPS)
def test_zero_rhs_and_converged_start(case, precision, name, op, oop, eps):
    mesh = case.mesh
    sim = gspm.Simulation(mesh, case.params, precision=precision)
    rng = np.random.default_rng(50)
    x0 = _site_vector(mesh, rng, 0.1)
    st, x, it = _gpu_solve(sim, op, np.zeros_like(x0), x0, eps, 1e-8, 1000)
    assert st == gspm.GSPM_OK and it == 0
    assert np.all(x == 0.0)
    # a start at the solution of a tighter solve needs no iteration and stays as it is
    b = _site_vector(mesh, rng)
    st, xs, it1 = _gpu_solve(sim, op, b, x0, eps, 1e-12, 100000)
    assert st == gspm.GSPM_OK and it1 > 0
    st, x2, it2 = _gpu_solve(sim, op, b, xs, eps, 1e-6, 100000)
    print(f"{name} precision {precision}: tight solve {it1} iterations, restart {it2}", flush=True)
    assert st == gspm.GSPM_OK and it2 == 0
    assert np.array_equal(x2, xs)
    sim.close()


@pytest.mark.parametrize("tol", [1e-4, 1e-7, 1e-10])
def test_elastic_iterations_and_solution_match_oracle(case, tol):
    mesh = case.mesh
    orc = O.Oracle.from_mesh(mesh)
    orc.set_params(case.params)
    nmap = orc.node_map()
    sim = gspm.Simulation(mesh, case.params)
    rng = np.random.default_rng(60)
    b = _site_vector(mesh, rng)
    x0 = _site_vector(mesh, rng, 0.1)
    bu = np.zeros((orc.n, 3)); bu[nmap] = b
    xu = np.zeros((orc.n, 3)); xu[nmap] = x0
    st, x, it = _gpu_solve(sim, gspm.GSPM_OP_ELASTIC, b, x0, 0.0, tol, 100000)
    rc, xr, itr = _oracle_solve(orc, O.OP_ELASTIC, bu, xu, 0.0, tol, 100000)
    err = _rel(x, xr[nmap])
    print(f"tol {tol:.0e}: iters gpu {it} oracle {itr} rel err {err:.2e}", flush=True)
    assert st == gspm.GSPM_OK and rc == 0
    assert abs(it - itr) <= 1
    # the same iteration count: the same steps up to rounding (summation
    # orders differ), which moves an iterate by a small fraction of its
    # remaining error (of order tol); one apart (a residual within rounding of
    # the threshold): both meet the tolerance and differ by one step
    assert err < (0.1 * tol if it == itr else 100 * tol)
    sim.close()
