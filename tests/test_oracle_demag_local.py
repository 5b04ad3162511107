"""Pins of the oracle's local magnetostatic solve (Eq. demag, weak form
(weak_demag), K^ms and F^ms of Eqs. (LHS), (RHS_F), (RHS_b)).

Each check rests on something other than the oracle itself:
  - closed forms: a uniform magnetisation carries no charge; a transverse
    modulation is divergence-free; a longitudinal sinusoid m_x = a sin(kx) has
    h~_d = -m~_x and energy density mu0 Ms^2 a^2 / 4, approached at first order
    (element field) and second order (energy) under refinement;
  - the Lorentz cavity field: a spherical hole in a uniformly magnetised host
    on a cubic lattice (volume fraction f) sees h~_d = (1 - f) / 3 along m;
  - an FFT solve of the circulant periodic Laplacian on a regular lattice;
  - the field as the energy gradient (central finite differences of the
    energy, which is quadratic in m, so the difference quotient is exact up
    to rounding);
  - invariants of the step: damping-only steps lower the total energy, and
    a charge-free state reproduces the step without the local solve (to
    rounding).
"""
import numpy as np
import pytest

import oracle as O
import workloads as w
from workloads.mesh import Inclusion, kuhn_cube, tag_inclusions

MAT = dict(w.MATERIAL_FEGA)
L = 100e-9


def _setup(n, jitter=0.0, sphere=0.0, seed=1, periodic=True):
    mesh = kuhn_cube(n, L, jitter=jitter, rng=np.random.default_rng(seed) if jitter > 0 else None)
    if sphere:
        tag_inclusions(mesh, [Inclusion(center=np.full(3, L / 2), semi=np.full(3, sphere * L))])
    orc = O.Oracle.from_mesh(mesh, periodic=periodic)
    orc.set_params(MAT)
    xu = np.zeros((orc.n, 3))
    xu[orc.node_map()] = mesh.xyz
    return mesh, orc, xu


def test_uniform_and_transverse_magnetisation_carry_no_charge():
    mesh, orc, xu = _setup(13)
    m = np.zeros((orc.n, 3)); m[:, 0] = 1.0
    assert np.abs(orc.ms_rhs(m)).max() == 0.0
    # m_y(x): on the unjittered Kuhn lattice its P1 interpolant depends on x
    # only, so div m_h = 0 element by element
    m = np.zeros((orc.n, 3)); m[:, 1] = 0.3 * np.sin(2 * np.pi * xu[:, 0] / L); m[:, 2] = 1.0
    scale = MAT["Ms"] * (L / 12) ** 2
    assert np.abs(orc.ms_rhs(m)).max() < 1e-12 * scale


def test_longitudinal_sinusoid_converges_to_closed_form():
    a, k = 0.3, 2 * np.pi / L
    e_exact = 0.25 * MAT["mu0"] * MAT["Ms"] ** 2 * a ** 2
    field_err, energy_err = [], []
    for n in (9, 17, 33):
        mesh, orc, xu = _setup(n, jitter=0.15)
        m = np.zeros((orc.n, 3)); m[:, 0] = a * np.sin(k * xu[:, 0]); m[:, 2] = 1.0
        U, it = orc.ms_solve(m, tol=1e-12)
        hd = orc.ms_field(U)
        vol, _ = orc.geometry()
        xc = mesh.xyz[mesh.tets].mean(axis=1)         # unwrapped mesh: centroids are plain means
        exact = -a * np.sin(k * xc[:, 0])
        field_err.append(np.sqrt(np.sum(vol * (hd[:, 0] - exact) ** 2) / np.sum(vol * exact ** 2)))
        energy_err.append(abs(orc.ms_energy(U) - e_exact) / e_exact)
        assert it > 0
    print("field L2 errors", field_err, "energy errors", energy_err)
    assert field_err[-1] < 0.05 and energy_err[-1] < 0.015
    for r in (field_err[0] / field_err[1], field_err[1] / field_err[2]):
        assert 1.7 < r < 2.4                      # first order: the P1 gradient
    for r in (energy_err[0] / energy_err[1], energy_err[1] / energy_err[2]):
        assert 3.3 < r < 4.7                      # second order: the energy


def test_cg_matches_fft_solve_on_periodic_lattice():
    case = w.small_cube(9, seed=0, L=8e-8, jitter=0.0)
    orc = O.Oracle.from_mesh(case.mesh)
    orc.set_params(MAT)
    nmap = orc.node_map()
    m = case.mesh.n_axis - 1
    s2u = np.full(m ** 3, -1)
    s2u[case.mesh.site] = nmap
    delta = np.zeros((orc.n, 3)); delta[s2u[0], 0] = 1.0
    sym = np.fft.fftn(orc.apply(O.OP_LAPLACE_ALL, delta)[s2u, 0].reshape(m, m, m))
    rng = np.random.default_rng(8)
    B = rng.standard_normal((m, m, m))
    B -= B.mean()                                 # the singular system is solvable
    Bf = np.fft.fftn(B)
    sym[0, 0, 0] = 1.0
    Bf[0, 0, 0] = 0.0
    Xf = np.real(np.fft.ifftn(Bf / sym))
    b = np.zeros((orc.n, 3)); b[s2u, 0] = B.ravel()
    x, it = orc.solve(O.OP_MS, b, tol=1e-13)
    p0 = orc.pinned_node()
    assert x[p0, 0] == 0.0
    ref = Xf.ravel() - Xf.ravel()[np.where(s2u == p0)[0][0]]
    assert np.abs(x[s2u, 0] - ref).max() < 1e-9 * np.abs(ref).max()
    # the pinned operator: the pinned row is zero, the rest is the Laplacian
    y = orc.apply(O.OP_MS, b)
    yall = orc.apply(O.OP_LAPLACE_ALL, b)
    assert np.all(y[p0] == 0.0) and np.array_equal(np.delete(y, p0, 0), np.delete(yall, p0, 0))


def test_energy_pairs_with_the_right_hand_side():
    # int |grad U|^2 = U . b for the exact discrete solution (weak form with v = U)
    mesh, orc, xu = _setup(8, jitter=0.15, sphere=0.3, seed=5)
    rng = np.random.default_rng(9)
    m = rng.standard_normal((orc.n, 3))
    U, _ = orc.ms_solve(m, tol=1e-13)
    e1 = orc.ms_energy(U)
    e2 = 0.5 * MAT["mu0"] * float(U @ orc.ms_rhs(m)) / orc.total_volume()
    assert abs(e1 - e2) < 1e-10 * e1


def test_field_is_minus_the_energy_gradient():
    # E(m) = (mu0 / 2 V_c) int |grad U(m)|^2; dE/dm_ja = -(mu0 Ms^2 / V_c) sum_{e ni j} V_e / 4 h~_d,e,a
    mesh, orc, xu = _setup(6, jitter=0.15, sphere=0.3, seed=6)
    rng = np.random.default_rng(10)
    m = rng.standard_normal((orc.n, 3))
    U, _ = orc.ms_solve(m, tol=1e-14)
    hd = orc.ms_field(U)
    vol, _ = orc.geometry()
    tets_u = orc.node_map()[mesh.tets]
    grad = np.zeros((orc.n, 3))
    for j in range(4):
        np.add.at(grad, tets_u[:, j], (vol / 4)[:, None] * hd)
    grad *= -MAT["mu0"] * MAT["Ms"] ** 2 / orc.total_volume()
    for node, a in ((3, 0), (17, 1), (40, 2), (orc.n - 1, 0)):
        d = 1e-3
        mp = m.copy(); mp[node, a] += d
        mm = m.copy(); mm[node, a] -= d
        ep = orc.ms_energy(orc.ms_solve(mp, U0=U, tol=1e-14)[0])
        em = orc.ms_energy(orc.ms_solve(mm, U0=U, tol=1e-14)[0])
        fd = (ep - em) / (2 * d)
        assert abs(fd - grad[node, a]) < 1e-6 * np.abs(grad).max(), (node, a, fd, grad[node, a])


def test_spherical_cavity_sees_the_lorentz_field():
    mesh, orc, xu = _setup(25, jitter=0.15, sphere=0.25, seed=2)
    m0 = np.zeros((mesh.n_nodes, 3)); m0[:, 0] = 1.0
    orc.set_m(m0)
    mu = np.zeros((orc.n, 3)); mu[orc.node_map()] = orc.get_m()
    U, _ = orc.ms_solve(mu, tol=1e-10)
    hd = orc.ms_field(U)
    vol, _ = orc.geometry()
    xc = mesh.xyz[mesh.tets].mean(axis=1)
    inside = np.linalg.norm(xc - L / 2, axis=1) < 0.125 * L
    f = vol[mesh.tags == 0].sum() / vol.sum()
    hin = (vol[inside, None] * hd[inside]).sum(0) / vol[inside].sum()
    print("cavity: f", f, "mean field inside", hin, "Lorentz", (1 - f) / 3)
    assert abs(hin[0] / ((1 - f) / 3) - 1.0) < 0.04
    assert abs(hin[1]) < 0.03 and abs(hin[2]) < 0.03


def test_damping_steps_lower_the_energy_with_local_magnetostatics():
    case = w.small_cube(7, seed=43, L=6e-8, jitter=0.15, sphere=0.35)
    orc = O.Oracle.from_mesh(case.mesh)
    orc.set_params(case.params, precession=False, local_demag=True)
    orc.set_m(case.m0)
    nmap = orc.node_map()

    def energy():
        mu = np.zeros((orc.n, 3)); mu[nmap] = orc.get_m()
        U, _ = orc.ms_solve(mu, tol=1e-12)
        return orc.energies()["total"] - orc.demag_local_energy() + orc.ms_energy(U), U

    e_prev, U_before = energy()
    for k in range(6):
        st = orc.step(1e-12, 1)
        assert st["ms_iters"] > 0
        if k == 0:
            # the stored potential is the solve at the step's starting state
            Us = np.zeros(orc.n); Us[nmap] = orc.get_ud()
            assert np.abs(Us - U_before).max() < 1e-6 * np.abs(U_before).max()
        e, _ = energy()
        assert e < e_prev
        e_prev = e


def test_charge_free_state_matches_the_step_without_the_solve():
    case = w.small_cube(6, seed=12, L=6e-8, jitter=0.15)
    m0 = np.tile([0.6, 0.8, 0.0], (case.mesh.n_nodes, 1))
    out = []
    for ld in (False, True):
        orc = O.Oracle.from_mesh(case.mesh)
        orc.set_params(case.params, local_demag=ld)
        orc.set_m(m0)
        st = orc.step(2e-12, 2)
        out.append((orc.get_m(), st))
    # the charge is zero up to rounding of the gradient sums (the solve then
    # only sees noise), so the trajectories agree to rounding
    assert out[0][1]["ms_iters"] == 0
    assert np.abs(out[0][0] - out[1][0]).max() < 1e-13


def test_stored_potential_enters_the_field_rhs_and_energy():
    case = w.small_cube(6, seed=13, L=6e-8, jitter=0.15, sphere=0.3)
    orc = O.Oracle.from_mesh(case.mesh)
    orc.set_params(case.params, local_demag=True)
    orc.set_m(case.m0)
    rng = np.random.default_rng(14)
    ud = case.mesh.per_site(rng.standard_normal(case.mesh.n_sites)) * 1e-3
    orc.set_ud(ud)
    assert np.array_equal(orc.get_ud(), ud)
    e_on = orc.energies()["total"]
    b_on, ch_on = orc.field_rhs(1.0)
    Uu = np.zeros(orc.n); Uu[orc.node_map()] = ud
    assert abs(orc.demag_local_energy() - orc.ms_energy(Uu)) == 0.0
    orc.set_params(case.params, local_demag=False)
    e_off = orc.energies()["total"]
    b_off, ch_off = orc.field_rhs(1.0)
    assert abs((e_on - e_off) - orc.ms_energy(Uu)) < 1e-12 * abs(e_on)
    # the field enters as M^e h~_d on magnetic elements: sum over nodes of the
    # difference is sum_e chi_e V_e h~_d,e
    hd = orc.ms_field(Uu)
    vol, _ = orc.geometry()
    mag = case.mesh.tags != 0
    expect = (vol[mag, None] * hd[mag]).sum(0)
    assert np.allclose((ch_on - ch_off).sum(0), expect, rtol=1e-10, atol=1e-12 * np.abs(expect).max())


def test_local_magnetostatics_needs_a_periodic_mesh():
    mesh, orc, xu = _setup(5, periodic=False)
    with pytest.raises(O.OracleError):
        orc.set_params(MAT, local_demag=True)
