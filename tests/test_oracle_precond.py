"""Jacobi-preconditioned CG on the elastic system in the oracle (the
preconditioning the paper leaves aside, Sec. 2.5), and the measurement that
decided not to build it on the GPU.

  - it converges to the same solution as a dense solve and as plain CG;
  - on the regular Kuhn lattice the diagonal of K^mech is one constant, so the
    preconditioned iteration is plain CG rescaled: the same iteration count
    (up to one iteration where rounding moves the stopping test's crossing);
  - on a jittered 13,824-node mesh with a spherical inclusion (the bench's
    lattice spacing), Jacobi saves only a few percent of the iterations.
"""
import numpy as np

import oracle as O
import workloads as w


def _rhs(orc, case, seed):
    rng = np.random.default_rng(seed)
    b = np.zeros((orc.n, 3))
    b[orc.node_map()] = case.mesh.per_site(rng.standard_normal((case.mesh.n_sites, 3)))
    b[orc.pinned_node()] = 0.0
    return b


def test_jacobi_pcg_solves_the_elastic_system():
    case = w.small_cube(5, seed=71, L=4e-8, jitter=0.15, sphere=0.3)
    orc = O.Oracle.from_mesh(case.mesh)
    orc.set_params(case.params)
    b = _rhs(orc, case, 1)
    xj, itj = orc.solve(O.SOLVE_ELASTIC_JACOBI, b, tol=1e-13)
    xc, itc = orc.solve(O.OP_ELASTIC, b, tol=1e-13)
    # dense reference on the free DOFs
    n = orc.n
    A = np.zeros((3 * n, 3 * n))
    for j in range(3 * n):
        e = np.zeros(3 * n); e[j] = 1.0
        A[:, j] = orc.apply(O.OP_ELASTIC, e.reshape(n, 3)).ravel()
    free = np.ones(3 * n, bool); free[3 * orc.pinned_node():3 * orc.pinned_node() + 3] = False
    xd = np.zeros(3 * n)
    xd[free] = np.linalg.solve(A[np.ix_(free, free)], b.ravel()[free])
    assert np.abs(xj.ravel() - xd).max() < 1e-9 * np.abs(xd).max()
    assert np.abs(xj - xc).max() < 1e-9 * np.abs(xc).max()
    assert itj > 0 and itc > 0


def test_constant_diagonal_gives_plain_cg():
    case = w.small_cube(7, seed=72, L=6e-8, jitter=0.0)
    orc = O.Oracle.from_mesh(case.mesh)
    orc.set_params(case.params)
    b = _rhs(orc, case, 2)
    # In exact arithmetic the two iterations coincide.  The stopping test
    # compares a residual norm with a threshold, so rounding (the OpenMP
    # reduction order depends on the runtime loaded) can move the crossing by
    # one iteration; a wrong diagonal or scaling moves it by many.
    for tol in (1e-6, 1e-8, 1e-10, 1e-12):
        xj, itj = orc.solve(O.SOLVE_ELASTIC_JACOBI, b, tol=tol)
        xc, itc = orc.solve(O.OP_ELASTIC, b, tol=tol)
        assert abs(itj - itc) <= 1, (tol, itj, itc)
        assert np.abs(xj - xc).max() < 10 * tol * np.abs(xc).max()


def test_jacobi_saves_little_on_the_bench_lattice():
    h = 200e-9 / 46
    case = w.small_cube(25, seed=5, L=24 * h, jitter=0.15, sphere=0.3)
    orc = O.Oracle.from_mesh(case.mesh)
    orc.set_params(case.params)
    b = _rhs(orc, case, 3)
    _, itj = orc.solve(O.SOLVE_ELASTIC_JACOBI, b, tol=1e-8)
    _, itc = orc.solve(O.OP_ELASTIC, b, tol=1e-8)
    print(f"elastic CG {itc} iterations, Jacobi PCG {itj} ({100 * (itc - itj) / itc:.1f}% fewer), {orc.n} nodes")
    assert itj <= itc
    assert itc - itj < 0.15 * itc
