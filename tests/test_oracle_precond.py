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


# ------------------------------------------- Green's-operator preconditioner

H_BENCH = 200e-9 / 46


def _green(case, omega=None):
    orc = O.Oracle.from_mesh(case.mesh)
    p = dict(case.params)
    p["elastic_precond"] = 1
    orc.set_params(p)
    if omega is not None:
        orc.set_precond_omega(omega)
    return orc


def _zero_mean(v):
    return v - v.mean(axis=0)


def test_green_operator_inverts_the_regular_lattice():
    """On an unjittered periodic Kuhn lattice the auxiliary grid is the
    lattice itself (trilinear weights 0/1) and the grid operator is the mesh's
    own K^mech, so without the diagonal term B is its pseudo-inverse:
    B K x = x - mean(x) for every x, and the preconditioned solve converges in
    one iteration to the dense solution."""
    case = w.small_cube(7, seed=81, L=6 * H_BENCH, jitter=0.0)
    orc = _green(case, omega=0.0)
    assert orc.precond_grid() == (6, 6, 6)
    rng = np.random.default_rng(4)
    x = rng.standard_normal((orc.n, 3))
    Kx = orc.apply(O.OP_ELASTIC, x)
    # OP_ELASTIC zeroes the pinned rows: put the periodic row back (rows sum to zero)
    Kx[orc.pinned_node()] = -np.delete(Kx, orc.pinned_node(), axis=0).sum(axis=0)
    z = orc.precond_apply(Kx)
    assert np.abs(z - _zero_mean(x)).max() < 1e-10 * np.abs(x).max()
    b = _rhs(orc, case, 5)
    xg, it = orc.solve(O.SOLVE_ELASTIC_GREEN, b, tol=1e-10)
    assert it == 1
    xc, _ = orc.solve(O.OP_ELASTIC, _zero_mean(b), tol=1e-13)
    assert np.abs(xg - xc).max() < 1e-9 * np.abs(xc).max()


def test_green_operator_is_symmetric_and_positive():
    """B = Q A^+ Q^T + omega D^-1 on a jittered, shuffled mesh with an
    inclusion: symmetric, and positive on random vectors."""
    case = w.small_cube(6, seed=82, L=5 * H_BENCH, jitter=0.15, sphere=0.3, shuffle=True)
    orc = _green(case)
    rng = np.random.default_rng(6)
    u = rng.standard_normal((orc.n, 3))
    v = rng.standard_normal((orc.n, 3))
    Bu, Bv = orc.precond_apply(u), orc.precond_apply(v)
    assert abs(np.sum(u * Bv) - np.sum(v * Bu)) < 1e-12 * np.sqrt(np.sum(u * Bu) * np.sum(v * Bv))
    for _ in range(5):
        x = rng.standard_normal((orc.n, 3))
        assert np.sum(x * orc.precond_apply(x)) > 0.0


def test_green_pcg_matches_dense_solve():
    case = w.small_cube(5, seed=83, L=4 * H_BENCH, jitter=0.15, sphere=0.3, shuffle=True)
    orc = _green(case)
    b = _zero_mean(_rhs(orc, case, 7))
    x, it = orc.solve(O.SOLVE_ELASTIC_GREEN, b, tol=1e-13)
    n, p0 = orc.n, orc.pinned_node()
    A = np.zeros((3 * n, 3 * n))
    for j in range(3 * n):
        e = np.zeros(3 * n); e[j] = 1.0
        A[:, j] = orc.apply(O.OP_ELASTIC, e.reshape(n, 3)).ravel()
    free = np.ones(3 * n, bool); free[3 * p0:3 * p0 + 3] = False
    xd = np.zeros(3 * n)
    xd[free] = np.linalg.solve(A[np.ix_(free, free)], b.ravel()[free])
    assert np.abs(x.ravel() - xd).max() < 1e-9 * np.abs(xd).max()
    assert np.abs(x[p0]).max() == 0.0


def test_green_iterations_do_not_grow_with_the_mesh():
    """Plain CG on the pinned system needs more iterations as the mesh is
    refined at fixed spacing; with the Green's-operator preconditioner the
    count stays flat (jittered meshes, bench spacing, spherical inclusion)."""
    plain, green = [], []
    for n in (9, 14, 19):
        case = w.small_cube(n, seed=84, L=(n - 1) * H_BENCH, jitter=0.15, sphere=0.3)
        orc = _green(case)
        b = _zero_mean(_rhs(orc, case, 8))
        _, itg = orc.solve(O.SOLVE_ELASTIC_GREEN, b, tol=1e-8)
        _, itp = orc.solve(O.OP_ELASTIC, b, tol=1e-8)
        plain.append(itp); green.append(itg)
    print(f"plain CG {plain}, Green-preconditioned CG {green}")
    assert plain[2] > 1.6 * plain[0]
    assert max(green) <= 25 and max(green) - min(green) <= 4


def test_green_step_reproduces_the_plain_step():
    """A step with the preconditioned elastic solve and a step with plain CG
    reach the same state at a tight tolerance (the pinned solution differs
    from the periodic one only by the translation the solve removes)."""
    case = w.small_cube(7, seed=85, L=6 * H_BENCH, jitter=0.15, sphere=0.3, shuffle=True)
    out = []
    for pc in (0, 1):
        orc = O.Oracle.from_mesh(case.mesh)
        p = dict(case.params); p["cg_tol"] = 1e-12; p["elastic_precond"] = pc
        orc.set_params(p, hext=(-2e5, 0.0, 0.0))
        orc.set_m(case.m0)
        st = orc.step(5e-12, 3)
        out.append((orc.get_m(), orc.get_u(), st["mech_iters"]))
    (m0, u0, it0), (m1, u1, it1) = out
    print(f"elastic iterations over 3 steps: plain {it0}, preconditioned {it1}")
    assert np.abs(m1 - m0).max() < 1e-10
    assert np.abs(u1 - u0).max() < 1e-9 * np.abs(u0).max()
    assert it1 < it0 / 3


# ------------------------------------------- Jacobi-preconditioned GS solves

def _gs_case(n, seed, jitter=0.15, sphere=0.3):
    case = w.small_cube(n, seed=seed, L=(n - 1) * H_BENCH, jitter=jitter, sphere=sphere)
    p = dict(case.params)
    dtau = p["gamma0"] * p["Ms"] * 1e-11
    eps = 2 * p["A"] / (p["mu0"] * p["Ms"] ** 2) * dtau
    return case, p, eps


def _gs_oracles(case, p):
    out = []
    for gp in (0, 2):
        orc = O.Oracle.from_mesh(case.mesh)
        q = dict(p); q["gs_precond"] = gp
        orc.set_params(q)
        out.append(orc)
    return out


def test_gs_jacobi_matches_dense_solve():
    case, p, eps = _gs_case(7, 91, sphere=0.35)
    plain, jac = _gs_oracles(case, p)
    rng = np.random.default_rng(11)
    mag = jac.lumped_weights() > 0
    assert (~mag).any()
    b = rng.standard_normal((jac.n, 3)) * mag[:, None]
    xj, _ = jac.solve(O.OP_GS, b, eps=eps, tol=1e-13)
    n = jac.n
    A = np.zeros((n, n))
    for j in range(n):
        e = np.zeros((n, 3)); e[j, 0] = 1.0
        A[:, j] = jac.apply(O.OP_GS, e, eps)[:, 0]
    for c in range(3):
        xd = np.zeros(n)
        xd[mag] = np.linalg.solve(A[np.ix_(mag, mag)], b[mag, c])
        assert np.abs(xj[:, c] - xd).max() < 1e-10 * np.abs(xd).max()
    assert np.abs(xj[~mag]).max() == 0.0


def test_gs_jacobi_with_a_constant_diagonal_is_plain_cg():
    """On the regular lattice without inclusions the GS operator's diagonal is
    one constant, so Jacobi-preconditioned CG is plain CG rescaled: the same
    iteration count (within one, where rounding moves the test's crossing)."""
    case, p, eps = _gs_case(8, 92, jitter=0.0, sphere=0.0)
    plain, jac = _gs_oracles(case, p)
    rng = np.random.default_rng(12)
    b = rng.standard_normal((jac.n, 3))
    for tol in (1e-6, 1e-10):
        xp, itp = plain.solve(O.OP_GS, b, eps=eps, tol=tol)
        xj, itj = jac.solve(O.OP_GS, b, eps=eps, tol=tol)
        assert abs(itp - itj) <= 3, (tol, itp, itj)       # three components summed
        assert np.abs(xj - xp).max() < 10 * tol * np.abs(xp).max()


def test_gs_jacobi_cuts_iterations_on_jittered_meshes_with_inclusions():
    case, p, eps = _gs_case(16, 93)
    plain, jac = _gs_oracles(case, p)
    rng = np.random.default_rng(13)
    mag = jac.lumped_weights() > 0
    b = rng.standard_normal((jac.n, 3)) * mag[:, None]
    xp, itp = plain.solve(O.OP_GS, b, eps=eps, tol=1e-8)
    xj, itj = jac.solve(O.OP_GS, b, eps=eps, tol=1e-8)
    print(f"GS solves (3 components): plain CG {itp} iterations, Jacobi PCG {itj}")
    assert itj < 0.75 * itp
    assert np.abs(xj - xp).max() < 1e-6 * np.abs(xp).max()


def test_gs_jacobi_step_reproduces_the_plain_step():
    case, p, eps = _gs_case(7, 94)
    out = []
    for gp in (0, 2):
        orc = O.Oracle.from_mesh(case.mesh)
        q = dict(p); q["cg_tol"] = 1e-12; q["gs_precond"] = gp
        orc.set_params(q, hext=(-2e5, 0.0, 0.0))
        orc.set_m(case.m0)
        st = orc.step(1e-11, 3)
        out.append((orc.get_m(), orc.get_u(), sum(st["gs_iters"])))
    (m0, u0, it0), (m1, u1, it1) = out
    print(f"GS iterations over 3 steps: plain {it0}, Jacobi {it1}")
    assert np.abs(m1 - m0).max() < 1e-10
    assert np.abs(u1 - u0).max() < 1e-9 * np.abs(u0).max()
    assert it1 < it0
