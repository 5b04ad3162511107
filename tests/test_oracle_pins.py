"""Pins of the CPU oracle against what the paper and mathematics fix.

None of these compares the oracle with itself: each check uses a closed form,
a value printed in or worked from the paper (tests/golden), an independent
route to the same quantity (finite-difference Hessians of an energy written in
Voigt form, quadrature, numpy dense solves, FFT solves of circulant systems),
or an invariant of the method.
"""
import os

import numpy as np
import pytest

import oracle as O
import workloads as w

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
MAT = dict(w.MATERIAL_FEGA)


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def _voigt_C(p):
    c11, c12, c44 = p["c11"], p["c12"], p["c44"]
    C = np.zeros((6, 6))
    C[:3, :3] = c12
    np.fill_diagonal(C[:3, :3], c11)
    C[3, 3] = C[4, 4] = C[5, 5] = c44
    return C


def _eng(e6):
    """Tensor strain (xx yy zz yz xz xy) -> engineering Voigt vector."""
    e = np.asarray(e6, float).copy()
    e[3:] *= 2.0
    return e


def _site_map(case, orc):
    """unique id of each periodic lattice site, and the lattice shape."""
    nmap = orc.node_map()
    m = case.mesh.n_axis - 1
    s2u = np.full(m ** 3, -1)
    s2u[case.mesh.site] = nmap
    assert (s2u >= 0).all()
    return s2u, m


def _single_tet(seed=0):
    rng = np.random.default_rng(seed)
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float) * 1e-8
    xyz += rng.uniform(-2e-9, 2e-9, size=(4, 3))
    tets = np.array([[0, 1, 2, 3]], np.int32)
    if np.linalg.det(xyz[1:] - xyz[0]) < 0:
        tets = np.array([[0, 2, 1, 3]], np.int32)
    return xyz, tets


# --------------------------------------------------------------- geometry

def test_geometry_identities():
    case = w.small_cube(7, seed=11, L=1e-7, jitter=0.15, shuffle=True)
    orc = O.Oracle.from_mesh(case.mesh)
    vol, grad = orc.geometry()
    assert np.isclose(vol.sum(), 1e-21, rtol=1e-12)
    assert np.abs(grad.sum(axis=1)).max() < 1e-6 * np.abs(grad).max()
    X = case.mesh.xyz[case.mesh.tets]            # unwrapped generator coordinates
    d = X - X[:, :1]
    prod = np.einsum("eia,eja->eij", grad, d)    # grad lambda_i . (x_j - x_0)
    target = np.zeros((4, 4)); target[1:, 1:] = np.eye(3); target[0, 1:] = -1.0
    assert np.abs(prod - target).max() < 1e-9


def test_periodic_identification_matches_sites():
    case = w.small_cube(6, seed=2, L=1.0, jitter=0.15, shuffle=True)
    orc = O.Oracle.from_mesh(case.mesh)
    assert orc.n == case.mesh.n_sites
    nmap = orc.node_map()
    # same site <-> same unique node (a bijection)
    pairs = set(zip(case.mesh.site.tolist(), nmap.tolist()))
    assert len(pairs) == orc.n


def test_mesh_errors():
    case = w.small_cube(5, seed=2, L=1.0, jitter=0.0)
    xyz = case.mesh.xyz.copy()
    on_max_x = np.isclose(xyz[:, 0], 1.0) & (xyz[:, 1] > 0.1) & (xyz[:, 1] < 0.9)
    xyz[np.argmax(on_max_x), 1] += 1e-3            # breaks the face match
    with pytest.raises(O.OracleError, match="unmatched"):
        O.Oracle(xyz, case.mesh.tets, case.mesh.tags, case.mesh.lo, case.mesh.hi)
    xyz = case.mesh.xyz.copy(); xyz[0, 0] = -0.5
    with pytest.raises(O.OracleError):
        O.Oracle(xyz, case.mesh.tets, case.mesh.tags, case.mesh.lo, case.mesh.hi)
    tets = case.mesh.tets.copy(); tets[0, 3] = tets[0, 2]
    with pytest.raises(O.OracleError):
        O.Oracle(case.mesh.xyz, tets, case.mesh.tags, case.mesh.lo, case.mesh.hi)


# ------------------------------------------------------- scalar operators

def test_laplacian_is_h_times_seven_point_stencil():
    case = w.small_cube(9, seed=0, L=1e-7, jitter=0.0)
    orc = O.Oracle.from_mesh(case.mesh)
    s2u, m = _site_map(case, orc)
    h = 1e-7 / 8
    stencil = [(int(r[0]), int(r[1]), int(r[2]), float(r[3])) for r in _read_golden("kuhn_laplacian_stencil.txt")]
    rng = np.random.default_rng(0)
    X = rng.standard_normal((m, m, m))            # indexed [z, y, x]
    x = np.zeros((orc.n, 3)); x[s2u, 0] = X.ravel()
    y = orc.apply(O.OP_LAPLACE_ALL, x)[s2u, 0].reshape(m, m, m)
    ref = np.zeros_like(X)
    for dx, dy, dz, c in stencil:
        ref += c * h * np.roll(X, shift=(-dz, -dy, -dx), axis=(0, 1, 2))
    assert np.abs(y - ref).max() < 1e-12 * np.abs(ref).max()


def test_laplacian_kernel_symmetry_psd():
    case = w.small_cube(6, seed=3, L=1e-7, jitter=0.15, sphere=0.25)
    orc = O.Oracle.from_mesh(case.mesh)
    ones = np.ones((orc.n, 3))
    assert np.abs(orc.apply(O.OP_LAPLACE, ones)).max() < 1e-22
    rng = np.random.default_rng(1)
    x, y = rng.standard_normal((2, orc.n, 3))
    for op in (O.OP_LAPLACE, O.OP_MASS, O.OP_GS):
        a = np.sum(x * orc.apply(op, y, eps=1e-17)); b = np.sum(y * orc.apply(op, x, eps=1e-17))
        assert abs(a - b) < 1e-12 * abs(a)
        assert np.sum(x * orc.apply(op, x, eps=1e-17)) > 0


def test_laplacian_patch_test_unwrapped():
    case = w.small_cube(7, seed=4, L=1e-7, jitter=0.15)
    orc = O.Oracle.from_mesh(case.mesh, periodic=False)
    X = case.mesh.xyz
    interior = np.all((X > 1e-12) & (X < 1e-7 - 1e-12), axis=1)
    G = np.array([[0.3, -1.2, 2.0]])
    x = np.repeat(X @ G.T + 0.7e-7, 3, axis=1)
    y = orc.apply(O.OP_LAPLACE, x)
    edge = np.abs(y[~interior]).max()            # boundary rows are not zero: the test bites
    assert edge > 0.0
    assert np.abs(y[interior]).max() < 1e-10 * edge


def test_mass_matrix_against_quadrature():
    xyz, tets = _single_tet(5)
    orc = O.Oracle(xyz, tets, np.ones(1, np.uint8), xyz.min(0) - 1e-9, xyz.max(0) + 1e-9, periodic=False)
    V = abs(np.linalg.det(xyz[tets[0]][1:] - xyz[tets[0]][0])) / 6.0
    a, b = 0.5854101966249685, 0.1381966011250105     # 4-point rule, exact for degree 2
    pts = np.full((4, 4), b) + np.eye(4) * (a - b)
    rng = np.random.default_rng(2)
    for _ in range(5):
        u = rng.standard_normal(4)
        quad = V / 4.0 * np.sum((pts @ u[tets[0] * 0 + np.arange(4)]) ** 2)
        x = np.zeros((4, 3)); x[tets[0], 0] = u
        y = orc.apply(O.OP_MASS, x)
        assert np.isclose(np.sum(x[:, 0] * y[:, 0]), quad, rtol=1e-12)


# ------------------------------------------------------------- elasticity

def _elastic_energy_fd_hessian(xyz, tet, p):
    """Hessian of W(u) = (V/2) eps_v . C_v eps_v (Voigt, engineering shear) by
    central differences; exact for a quadratic up to rounding."""
    X = xyz[tet]
    D = (X[1:] - X[0]).T
    V = abs(np.linalg.det(D)) / 6.0
    Dinv = np.linalg.inv(D)
    Cv = _voigt_C(p)

    def W(u):
        U = u.reshape(4, 3)
        H = (U[1:] - U[0]).T @ Dinv          # grad u
        e = 0.5 * (H + H.T)
        ev = np.array([e[0, 0], e[1, 1], e[2, 2], 2 * e[1, 2], 2 * e[0, 2], 2 * e[0, 1]])
        return 0.5 * V * ev @ Cv @ ev

    n = 12
    Hs = np.zeros((n, n))
    d = 1e-9
    for i in range(n):
        for j in range(n):
            ei = np.zeros(n); ei[i] = d
            ej = np.zeros(n); ej[j] = d
            Hs[i, j] = (W(ei + ej) - W(ei - ej) - W(-ei + ej) + W(-ei - ej)) / (4 * d * d)
    return Hs


def test_elastic_element_matrix_is_energy_hessian():
    xyz, tets = _single_tet(7)
    orc = O.Oracle(xyz, tets, np.ones(1, np.uint8), xyz.min(0) - 1e-9, xyz.max(0) + 1e-9, periodic=False)
    orc.set_params(MAT)
    Hs = _elastic_energy_fd_hessian(xyz, tets[0], MAT)
    # oracle K applied to unit vectors (the pinned node 0's rows are zero)
    K = np.zeros((12, 12))
    for k in range(12):
        x = np.zeros((4, 3)); x[tets[0][k // 3], k % 3] = 1.0
        y = orc.apply(O.OP_ELASTIC, x)
        K[:, k] = y[tets[0]].reshape(12)
    rows = [r for r in range(12) if tets[0][r // 3] != 0]
    assert np.abs(K[rows] - Hs[rows]).max() < 1e-6 * np.abs(Hs).max()


def test_elastic_patch_and_rigid_modes():
    case = w.small_cube(6, seed=9, L=1e-7, jitter=0.15)
    orc = O.Oracle.from_mesh(case.mesh, periodic=False)
    orc.set_params(MAT)
    X = case.mesh.xyz
    interior = np.all((X > 1e-12) & (X < 1e-7 - 1e-12), axis=1)
    rng = np.random.default_rng(3)
    scale = np.abs(orc.apply(O.OP_ELASTIC, rng.standard_normal((orc.n, 3)) * 1e-9)).max()
    G = rng.standard_normal((3, 3)) * 1e-3
    y = orc.apply(O.OP_ELASTIC, X @ G.T)
    assert np.abs(y[interior]).max() < 1e-9 * scale
    omega = np.array([0.2, -0.5, 0.9]) * 1e-3
    y = orc.apply(O.OP_ELASTIC, np.cross(omega, X))
    assert np.abs(y).max() < 1e-9 * scale
    per = O.Oracle.from_mesh(case.mesh, periodic=True); per.set_params(MAT)
    y = per.apply(O.OP_ELASTIC, np.tile([1e-9, -2e-9, 3e-9], (per.n, 1)))
    assert np.abs(y).max() < 1e-9 * scale


# ------------------------------------------------------------------ solvers

def _dense(orc, op, eps, comps):
    n = orc.n
    A = np.zeros((n * comps, n * comps))
    for k in range(n * comps):
        x = np.zeros((n, 3))
        if comps == 1:
            x[k, 0] = 1.0
            A[:, k] = orc.apply(op, x, eps)[:, 0]
        else:
            x[k // 3, k % 3] = 1.0
            A[:, k] = orc.apply(op, x, eps).reshape(-1)
    return A


def test_gs_cg_matches_dense_direct_solve():
    case = w.small_cube(5, seed=21, L=4e-8, jitter=0.15, sphere=0.2)
    orc = O.Oracle.from_mesh(case.mesh)
    eps = 3e-18
    A = _dense(orc, O.OP_GS, eps, 1)
    mag = orc.lumped_weights() > 0
    rng = np.random.default_rng(4)
    b = rng.standard_normal((orc.n, 3)); b[~mag] = 0.0
    x, it = orc.solve(O.OP_GS, b, eps=eps, tol=1e-14)
    for c in range(3):
        ref = np.zeros(orc.n)
        ref[mag] = np.linalg.solve(A[np.ix_(mag, mag)], b[mag, c])
        assert np.abs(x[:, c] - ref).max() < 1e-10 * np.abs(ref).max()


def test_elastic_cg_matches_dense_direct_solve():
    case = w.small_cube(4, seed=22, L=4e-8, jitter=0.15)
    orc = O.Oracle.from_mesh(case.mesh)
    orc.set_params(MAT)
    A = _dense(orc, O.OP_ELASTIC, 0.0, 3)
    p0 = orc.pinned_node()
    free = np.ones(orc.n * 3, bool); free[p0 * 3:p0 * 3 + 3] = False
    rng = np.random.default_rng(5)
    b = rng.standard_normal((orc.n, 3)) * 1e-3
    x, it = orc.solve(O.OP_ELASTIC, b, tol=1e-14)
    ref = np.zeros(orc.n * 3)
    ref[free] = np.linalg.solve(A[np.ix_(free, free)], b.reshape(-1)[free])
    assert np.abs(x.reshape(-1) - ref).max() < 1e-9 * np.abs(ref).max()


def test_gs_cg_matches_fft_solve_on_periodic_lattice():
    case = w.small_cube(9, seed=0, L=8e-8, jitter=0.0)
    orc = O.Oracle.from_mesh(case.mesh)
    s2u, m = _site_map(case, orc)
    eps = 5e-17
    delta = np.zeros((orc.n, 3)); delta[s2u[0], 0] = 1.0
    st = orc.apply(O.OP_GS, delta, eps)[s2u, 0].reshape(m, m, m)
    sym = np.fft.fftn(st)
    rng = np.random.default_rng(6)
    B = rng.standard_normal((m, m, m))
    Xf = np.real(np.fft.ifftn(np.fft.fftn(B) / sym))
    b = np.zeros((orc.n, 3)); b[s2u, 0] = B.ravel()
    x, it = orc.solve(O.OP_GS, b, eps=eps, tol=1e-13)
    assert np.abs(x[s2u, 0].reshape(m, m, m) - Xf).max() < 1e-9 * np.abs(Xf).max()


def test_elastic_cg_matches_fft_solve_on_periodic_lattice():
    case = w.small_cube(9, seed=0, L=8e-8, jitter=0.0)
    orc = O.Oracle.from_mesh(case.mesh)
    orc.set_params(MAT)
    s2u, m = _site_map(case, orc)
    c0 = (m // 2) * (1 + m + m * m)               # a site away from the pinned corner
    sym = np.zeros((m, m, m, 3, 3), complex)
    for bcol in range(3):
        x = np.zeros((orc.n, 3)); x[s2u[c0], bcol] = 1.0
        y = orc.apply(O.OP_ELASTIC, x)[s2u].reshape(m, m, m, 3)
        y = np.roll(y, shift=(-(m // 2),) * 3, axis=(0, 1, 2))
        for a in range(3):
            sym[..., a, bcol] = np.fft.fftn(y[..., a])
    rng = np.random.default_rng(7)
    B = rng.standard_normal((m, m, m, 3)) * 1e-3
    B -= B.mean(axis=(0, 1, 2))
    Bf = np.stack([np.fft.fftn(B[..., a]) for a in range(3)], axis=-1)
    Xf = np.zeros_like(Bf)
    mask = np.ones((m, m, m), bool); mask[0, 0, 0] = False
    Xf[mask] = np.linalg.solve(sym[mask], Bf[mask][..., None])[..., 0]
    Xs = np.stack([np.real(np.fft.ifftn(Xf[..., a])) for a in range(3)], axis=-1)
    p0 = orc.pinned_node()
    p0_site = int(np.where(s2u == p0)[0][0])
    Xs -= Xs.reshape(-1, 3)[p0_site]
    b = np.zeros((orc.n, 3)); b[s2u] = B.reshape(-1, 3)
    x, it = orc.solve(O.OP_ELASTIC, b, tol=1e-13)
    assert np.abs(x[s2u].reshape(m, m, m, 3) - Xs).max() < 1e-8 * np.abs(Xs).max()


# ------------------------------------------------------------------ demag

def test_demag_sphere_and_trace():
    assert np.allclose(O.demag_factors(1.0, 1.0, 1.0), 1.0 / 3.0, atol=1e-10)
    N = O.demag_factors(3.0, 1.3, 0.6)
    assert abs(N.sum() - 1.0) < 1e-10
    assert N[0] < N[1] < N[2]


@pytest.mark.parametrize("ratio", [1.5, 3.0, 10.0])
def test_demag_prolate_oblate_closed_forms(ratio):
    mm = ratio
    # prolate spheroid, long axis a = ratio, b = c = 1
    Na = (mm / np.sqrt(mm * mm - 1) * np.log(mm + np.sqrt(mm * mm - 1)) - 1.0) / (mm * mm - 1)
    N = O.demag_factors(mm, 1.0, 1.0)
    assert abs(N[0] - Na) < 1e-9 and abs(N[1] - (1 - Na) / 2) < 1e-9
    # oblate spheroid a = b = ratio, short axis c = 1
    Nc = mm * mm / (mm * mm - 1) * (1.0 - np.arcsin(np.sqrt(mm * mm - 1) / mm) / np.sqrt(mm * mm - 1))
    N = O.demag_factors(mm, mm, 1.0)
    assert abs(N[2] - Nc) < 1e-9 and abs(N[0] - (1 - Nc) / 2) < 1e-9


# ------------------------------------------------------- local field terms

def test_local_field_is_energy_derivative():
    rng = np.random.default_rng(8)
    scale = 1.0 / (MAT["mu0"] * MAT["Ms"] ** 2)
    for _ in range(10):
        m = rng.standard_normal(3)
        E = rng.standard_normal(6) * 3e-4
        H = rng.standard_normal(3) * 1e5
        h = O.h_local(MAT, m, E, np.zeros(3), hext=H)
        fd = np.zeros(3)
        d = 1e-6
        for k in range(3):
            mp = m.copy(); mp[k] += d
            mn = m.copy(); mn[k] -= d
            fd[k] = -(O.energy_density_local(MAT, mp, E, H) - O.energy_density_local(MAT, mn, E, H)) / (2 * d)
        assert np.allclose(h, scale * fd, rtol=1e-6, atol=1e-9 * np.abs(h).max())
    # far field: h changes by -Nd mbar
    p = dict(MAT); p["Nd"] = np.diag([0.2, 0.3, 0.5]).reshape(9)
    m = np.array([0.6, 0.0, 0.8]); E = np.zeros(6); mb = np.array([0.5, -0.25, 0.1])
    dh = O.h_local(p, m, E, mb) - O.h_local(p, m, E, np.zeros(3))
    assert np.allclose(dh, -np.diag([0.2, 0.3, 0.5]) @ mb, atol=1e-15)


def test_anisotropy_special_directions():
    for name, coeff in _read_golden("anisotropy_special.txt"):
        m = np.array([float(c) for c in name]); m /= np.linalg.norm(m)
        p = dict(MAT); p["lambda100"] = 0.0; p["lambda111"] = 0.0
        val = O.energy_density_local(p, m, np.zeros(6))
        assert np.isclose(val, float(coeff) * MAT["K1"], rtol=1e-12, atol=1e-9)


def _uniform_case(direction, sigma=(0.0,) * 6):
    case = w.small_cube(5, seed=31, L=4e-8, jitter=0.15)
    orc = O.Oracle.from_mesh(case.mesh)
    orc.set_params(MAT, sigma_ext=sigma)
    m = np.tile(direction / np.linalg.norm(direction), (case.mesh.n_nodes, 1))
    orc.set_m(m)
    return case, orc


def test_uniform_strain_reproduction_and_spontaneous_strain():
    for row in _read_golden("spontaneous_strain.txt"):
        direction = np.array([float(c) for c in row[0]])
        a = np.array([float(v) for v in row[1:7]]); b = np.array([float(v) for v in row[7:13]])
        case, orc = _uniform_case(direction)
        rhs = orc.elastic_rhs()
        scale = MAT["c11"] * MAT["lambda100"] * (4e-8 / 4) ** 2
        assert np.abs(rhs).max() < 1e-12 * scale
        mbar, ebar = orc.averages()
        assert np.allclose(ebar, a * MAT["lambda100"] + b * MAT["lambda111"], atol=1e-15)
        orc.step(1e-12, 1)
        assert np.abs(orc.get_u()).max() < 1e-12 * MAT["lambda100"] * 4e-8   # displacement scale lambda L


def test_homogeneous_strain_under_applied_stress():
    sigma = np.array([6e6, -2e6, 1e6, 0.5e6, 0.0, -1e6])
    d = np.array([1.0, 0.0, 0.0])
    case, orc = _uniform_case(d, sigma)
    mbar, ebar = orc.averages()
    E0 = np.array([1.0, -0.5, -0.5, 0, 0, 0]) * MAT["lambda100"]
    assert np.allclose(_voigt_C(MAT) @ _eng(ebar - E0), sigma, rtol=1e-10, atol=1e-3)


# --------------------------------------------------------- step invariants

def _macrospin(dt, steps, axis, theta0=1.0, hmag=0.05):
    """Uniform m in a constant field h along `axis`: the LL equation of App. B,
    dm/dtau = -m x h - alpha m x (m x h), has the closed form
    tan(theta/2) = tan(theta0/2) exp(-alpha |h| tau), phi = |h| tau about h."""
    case = w.small_cube(4, seed=41, L=3e-8, jitter=0.15)
    p = dict(MAT); p["K1"] = 0.0; p["lambda100"] = 0.0; p["lambda111"] = 0.0; p["cg_tol"] = 1e-12
    d = np.eye(3)[axis]; e1 = np.eye(3)[(axis + 1) % 3]; e2 = np.cross(d, e1)
    orc = O.Oracle.from_mesh(case.mesh)
    orc.set_params(p, hext=hmag * p["Ms"] * d)
    orc.set_m(np.tile(np.sin(theta0) * e1 + np.cos(theta0) * d, (case.mesh.n_nodes, 1)))
    orc.step(dt, steps)
    m = orc.get_m()
    assert np.ptp(m, axis=0).max() < 1e-12            # stays uniform
    tau = p["gamma0"] * p["Ms"] * dt * steps
    theta = 2 * np.arctan(np.tan(theta0 / 2) * np.exp(-p["alpha"] * hmag * tau))
    phi = hmag * tau
    exact = np.cos(theta) * d + np.sin(theta) * (np.cos(phi) * e1 + np.sin(phi) * e2)
    return np.linalg.norm(m[0] - exact)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_macrospin_first_order_convergence_to_ll_closed_form(axis):
    dt = 2e-13
    e1 = _macrospin(dt, 100, axis)
    e2 = _macrospin(dt / 2, 200, axis)
    e3 = _macrospin(dt / 4, 400, axis)
    assert e1 < 0.05
    assert 1.6 < e1 / e2 < 2.4 and 1.6 < e2 / e3 < 2.4


def test_fixed_point_along_easy_axis():
    case = w.small_cube(5, seed=42, L=4e-8, jitter=0.15)
    orc = O.Oracle.from_mesh(case.mesh)
    orc.set_params(MAT, hext=(0.3 * MAT["Ms"], 0.0, 0.0))
    orc.set_m(np.tile([1.0, 0.0, 0.0], (case.mesh.n_nodes, 1)))
    orc.step(5e-12, 3)
    assert np.abs(orc.get_m() - [1.0, 0.0, 0.0]).max() < 1e-13


def test_unit_length_and_monotone_decay_without_precession():
    case = w.small_cube(7, seed=43, L=6e-8, jitter=0.15, sphere=0.35)
    orc = O.Oracle.from_mesh(case.mesh)
    assert (orc.lumped_weights() == 0).any()     # some nodes lie inside the inclusion only
    orc.set_params(case.params, precession=False)
    orc.set_m(case.m0)
    e_prev = orc.energies()["total"]
    mag = orc.lumped_weights() > 0
    nmap = orc.node_map()
    for _ in range(8):
        orc.step(1e-12, 1)
        m = orc.get_m()
        r = np.linalg.norm(m, axis=1)
        assert np.abs(r[mag[nmap]] - 1.0).max() < 1e-14
        assert np.abs(m[~mag[nmap]]).max() == 0.0
        e = orc.energies()["total"]
        assert e < e_prev
        e_prev = e


def test_exchange_energy_equals_laplacian_quadratic_form():
    case = w.small_cube(6, seed=44, L=6e-8, jitter=0.15, sphere=0.2)
    orc = O.Oracle.from_mesh(case.mesh)
    orc.set_params(case.params)
    orc.set_m(case.m0)
    mq = orc.get_m()
    # unique-order copy of m
    mu = np.zeros((orc.n, 3)); mu[orc.node_map()] = mq
    ex = MAT["A"] * np.sum(mu * orc.apply(O.OP_LAPLACE, mu)) / orc.total_volume()
    assert np.isclose(orc.energies()["exchange"], ex, rtol=1e-12)


def test_noconv_and_bad_calls():
    case = w.small_cube(5, seed=45, L=4e-8, jitter=0.15)
    orc = O.Oracle.from_mesh(case.mesh)
    with pytest.raises(O.OracleError):
        orc.step(1e-12, 1)                       # no params / m yet
    p = dict(case.params); p["cg_maxit"] = 1
    orc.set_params(p)
    orc.set_m(case.m0)
    with pytest.raises(O.OracleError, match="converge"):
        orc.step(1e-12, 1)
    m = case.m0.copy(); m[0, 0] = np.nan
    with pytest.raises(O.OracleError):
        orc.set_m(m)


def test_mass_is_kuhn_stencil():
    case = w.small_cube(7, seed=0, L=6e-8, jitter=0.0)
    orc = O.Oracle.from_mesh(case.mesh)
    s2u, m = _site_map(case, orc)
    h = 1e-8
    rng = np.random.default_rng(9)
    X = rng.standard_normal((m, m, m))
    x = np.zeros((orc.n, 3)); x[s2u, 1] = X.ravel()
    y = orc.apply(O.OP_MASS, x)[s2u, 1].reshape(m, m, m)
    ref = np.zeros_like(X)
    for r in _read_golden("kuhn_mass_stencil.txt"):
        dx, dy, dz, c = int(r[0]), int(r[1]), int(r[2]), float(r[3])
        ref += c * h ** 3 * np.roll(X, shift=(-dz, -dy, -dx), axis=(0, 1, 2))
    assert np.abs(y - ref).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("kvec", [(1, 0, 0), (1, 2, 0), (2, 1, 3)])
def test_damping_stage_decay_matches_lattice_symbols(kvec):
    """Without precession and with h = 0 the step is m** = (eps3 K + M)^-1 M m
    followed by the unit-length projection.  On an unjittered periodic Kuhn
    lattice a small transverse Fourier mode is scaled by mu/(mu + eps3 kappa),
    kappa and mu the symbols of the pinned Laplacian and mass stencils."""
    n, L = 9, 8e-8
    case = w.small_cube(n, seed=0, L=L, jitter=0.0)
    p = dict(MAT); p["K1"] = 0.0; p["lambda100"] = 0.0; p["lambda111"] = 0.0
    p["Nd"] = np.zeros(9); p["cg_tol"] = 1e-13
    orc = O.Oracle.from_mesh(case.mesh)
    orc.set_params(p, precession=False)
    h = L / (n - 1)
    k = 2 * np.pi * np.asarray(kvec) / L
    X = case.mesh.xyz
    delta = 1e-5
    mx = delta * np.cos(X @ k)
    m0 = np.stack([mx, np.zeros_like(mx), np.ones_like(mx)], axis=1)
    m0 /= np.linalg.norm(m0, axis=1, keepdims=True)
    orc.set_m(m0)
    dt = 5e-12
    orc.step(dt, 1)
    m1 = orc.get_m()
    ratio = (m1[:, 0] @ m0[:, 0]) / (m0[:, 0] @ m0[:, 0])
    th = k * h
    kappa = h * np.sum(2 - 2 * np.cos(th))
    mu = h ** 3 * (0.4 + 0.1 * np.sum(np.cos(th))
                   + (np.cos(th[0] + th[1]) + np.cos(th[0] + th[2]) + np.cos(th[1] + th[2])) / 15.0
                   + 0.1 * np.cos(th.sum()))
    dtau = p["gamma0"] * p["Ms"] * dt
    eps3 = p["alpha"] * 2 * p["A"] / (p["mu0"] * p["Ms"] ** 2) * dtau
    assert abs(ratio - mu / (mu + eps3 * kappa)) < 1e-8


def test_averages_weight_by_magnetic_volume():
    case = w.small_cube(8, seed=51, L=7e-8, jitter=0.15, sphere=0.3)
    x = case.mesh.xyz[case.mesh.tets]
    vol = np.abs(np.linalg.det(x[:, 1:] - x[:, :1])) / 6.0
    frac = vol[case.mesh.tags != 0].sum() / vol.sum()
    assert 0.5 < frac < 0.95
    d = np.array([1.0, 1.0, 1.0]) / np.sqrt(3.0)
    orc = O.Oracle.from_mesh(case.mesh)
    orc.set_params(MAT)
    orc.set_m(np.tile(d, (case.mesh.n_nodes, 1)))
    mbar, ebar = orc.averages()
    assert np.allclose(mbar, frac * d, rtol=1e-12)
    e0 = np.array([0, 0, 0, 0.5, 0.5, 0.5]) * MAT["lambda111"]     # golden [111] row
    assert np.allclose(ebar, frac * e0, rtol=1e-10, atol=1e-18)


def test_elastic_rhs_is_energy_gradient():
    """b of Eq. (RHS_b) is minus the gradient at u = 0 of
    W(u) = 1/2 int (E(u) - E0_h) : C (E(u) - E0_h), E0_h the P1 interpolant of
    E0(m) on magnetic elements; W is written here in Voigt form with numpy
    geometry and differentiated by central differences."""
    case = w.small_cube(4, seed=52, L=3e-8, jitter=0.15, sphere=0.3, shuffle=True)
    orc = O.Oracle.from_mesh(case.mesh, periodic=False)
    orc.set_params(MAT)
    orc.set_m(case.m0)
    b = orc.elastic_rhs()
    m = orc.get_m()
    l1, l2 = MAT["lambda100"], MAT["lambda111"]
    E0 = np.stack([1.5 * l1 * (m[:, 0] ** 2 - 1 / 3), 1.5 * l1 * (m[:, 1] ** 2 - 1 / 3), 1.5 * l1 * (m[:, 2] ** 2 - 1 / 3),
                   1.5 * l2 * m[:, 1] * m[:, 2], 1.5 * l2 * m[:, 0] * m[:, 2], 1.5 * l2 * m[:, 0] * m[:, 1]], axis=1)
    Cv = _voigt_C(MAT)
    X = case.mesh.xyz
    tets, tags = case.mesh.tets, case.mesh.tags
    Dinv = np.linalg.inv(np.transpose(X[tets[:, 1:]] - X[tets[:, :1]], (0, 2, 1)))
    V = np.abs(np.linalg.det(X[tets[:, 1:]] - X[tets[:, :1]])) / 6.0
    E0e = np.where(tags[:, None] != 0, E0[tets].mean(axis=1), 0.0)

    def grad_W_at_zero(node, comp):
        inc = np.where((tets == node).any(axis=1))[0]
        def W(t):
            tot = 0.0
            for e in inc:
                U = np.zeros((4, 3)); U[tets[e] == node, comp] = t
                H = (U[1:] - U[0]).T @ Dinv[e]
                eps = 0.5 * (H + H.T)
                r = np.array([eps[0, 0], eps[1, 1], eps[2, 2], eps[1, 2], eps[0, 2], eps[0, 1]]) - E0e[e]
                tot += 0.5 * V[e] * _eng(r) @ Cv @ _eng(r)
            return tot
        d = 1e-12
        return (W(d) - W(-d)) / (2 * d)

    rng = np.random.default_rng(10)
    nmap = orc.node_map()
    p0 = orc.pinned_node()
    checked = 0
    for node in rng.choice(case.mesh.n_nodes, 25, replace=False):
        if nmap[node] == p0:
            continue
        for comp in range(3):
            ref = -grad_W_at_zero(node, comp)
            assert abs(b[nmap[node], comp] - ref) < 1e-6 * np.abs(b).max()
            checked += 1
    assert checked >= 60


def test_field_rhs_sees_only_symmetric_strain():
    """A rigid rotation u = omega x x leaves the field right-hand side unchanged,
    and a linear displacement u = G x acts exactly like the applied stress
    C sym(G) that shifts the homogeneous strain by sym(G)."""
    case = w.small_cube(5, seed=53, L=4e-8, jitter=0.15, sphere=0.25)
    X = case.mesh.xyz
    G = np.array([[1.0, 2.0, -0.5], [0.3, -1.0, 0.7], [-2.0, 0.4, 0.2]]) * 2e-4
    S = 0.5 * (G + G.T)
    sigma = _voigt_C(MAT) @ _eng([S[0, 0], S[1, 1], S[2, 2], S[1, 2], S[0, 2], S[0, 1]])
    res = {}
    for name, u, sig in (("zero", 0 * X, np.zeros(6)), ("rot", np.cross([2e-4, -1e-4, 3e-4], X), np.zeros(6)),
                         ("lin", X @ G.T, np.zeros(6)), ("stress", 0 * X, sigma)):
        orc = O.Oracle.from_mesh(case.mesh, periodic=False)
        orc.set_params(MAT, sigma_ext=sig)
        orc.set_m(case.m0)
        orc.set_u(u)
        res[name] = orc.field_rhs(0.7)[1]
    scale = np.abs(res["zero"]).max()
    assert np.abs(res["rot"] - res["zero"]).max() < 1e-10 * scale
    assert np.abs(res["lin"] - res["stress"]).max() < 1e-9 * scale
    assert np.abs(res["lin"] - res["zero"]).max() > 1e-6 * scale


@pytest.mark.parametrize("direction", ["100", "1-23"])
def test_lumped_gs_start_is_exact_for_uniform_m(direction):
    """Reading R14: the GS start y + (sum_e M^e c h^e) / w is the exact
    solution of (eps K + M) g = b when m is uniform: h is then the same at
    every magnetic vertex, the mass rows over magnetic elements sum to the
    lumped weights w, and K annihilates a field that is constant on every
    magnetic element (inclusion-only nodes carry zero and touch no magnetic
    element).  So the start has a rounding-level residual and CG takes no
    iteration, while the start without the field term does not."""
    case = w.small_cube(9, seed=57, L=8e-8, jitter=0.15, sphere=0.3)
    d = {"100": [1.0, 0.0, 0.0], "1-23": [1.0, -2.0, 3.0]}[direction]
    d = np.asarray(d) / np.linalg.norm(d)
    orc = O.Oracle.from_mesh(case.mesh)
    orc.set_params(MAT, hext=(2e5, -1e5, 5e4), sigma_ext=(1e7, 0, -2e7, 0, 3e6, 0))
    orc.set_m(case.mesh.per_site(np.tile(d, (case.mesh.n_sites, 1))))
    c, eps = 0.37, 2.5e-17
    b, ch = orc.field_rhs(c)
    wts = orc.lumped_weights()
    mag = wts > 0
    m = np.zeros((orc.n, 3)); m[mag] = d
    h = ch[mag] / (c * wts[mag, None])
    assert np.abs(h - h.mean(axis=0)).max() <= 1e-12 * np.abs(h).max()   # one field at every magnetic node
    g0 = np.where(mag[:, None], m + ch / np.where(mag, wts, 1.0)[:, None], 0.0)
    res = np.linalg.norm(b - orc.apply(O.OP_GS, g0, eps)) / np.linalg.norm(b)
    res_plain = np.linalg.norm(b - orc.apply(O.OP_GS, m, eps)) / np.linalg.norm(b)
    g, its = orc.solve(O.OP_GS, b, g0, eps, tol=1e-12)
    assert res < 1e-14 and its == 0
    assert res_plain > 1e-6
    assert np.abs(g - g0).max() == 0.0


# ------------------------------------------------- energy terms, dm_avg

def _e0_closed(p, m):
    """App. A: E0 = (3/2)[lambda100 (m_i^2 - 1/3) on the diagonal, lambda111
    m_i m_j off it], order xx yy zz yz xz xy."""
    m = np.asarray(m, float)
    l1, l2 = p["lambda100"], p["lambda111"]
    return 1.5 * np.array([l1 * (m[0] ** 2 - 1 / 3), l1 * (m[1] ** 2 - 1 / 3), l1 * (m[2] ** 2 - 1 / 3),
                           l2 * m[1] * m[2], l2 * m[0] * m[2], l2 * m[0] * m[1]])


def _cubic_compliance_closed(p, s):
    """Tensor strain of a stress for cubic C in closed form: normal part
    s11 sigma_ii + s12 (sum of the other two), s11 = (c11 + c12) / D,
    s12 = -c12 / D, D = (c11 - c12)(c11 + 2 c12); shear sigma_ij / (2 c44)."""
    c11, c12, c44 = p["c11"], p["c12"], p["c44"]
    D = (c11 - c12) * (c11 + 2 * c12)
    s11, s12 = (c11 + c12) / D, -c12 / D
    s = np.asarray(s, float)
    tr = s[:3].sum()
    return np.concatenate([s11 * s[:3] + s12 * (tr - s[:3]), s[3:] / (2 * c44)])


def _tensor_contract(a6, b6):
    """a : b of two symmetric tensors in xx yy zz yz xz xy order."""
    return a6[:3] @ b6[:3] + 2.0 * (a6[3:] @ b6[3:])


@pytest.mark.parametrize("direction", ["100", "111", "1-23"])
def test_energy_terms_closed_forms_for_uniform_m_with_inclusion(direction):
    """Eq. (MicromagneticsEnergy) with R16's quadrature on a uniform state:
    the vertex rule integrates constants exactly, so with magnetic volume
    fraction f the anisotropy is f kappa1 (m1^2 m2^2 + ...) (0 along [100],
    kappa1/3 along [111]), the Zeeman term -mu0 Ms f H.m, the far field
    (mu0 Ms^2 / 2) mbar.N mbar with mbar = f m, the stress work -sigma:Ebar
    with Ebar = f E0(m) + C^-1 sigma, and exchange 0."""
    case = w.small_cube(8, seed=61, L=7e-8, jitter=0.15, sphere=0.3, shuffle=True)
    x = case.mesh.xyz[case.mesh.tets]
    vol = np.abs(np.linalg.det(x[:, 1:] - x[:, :1])) / 6.0
    f = vol[case.mesh.tags != 0].sum() / vol.sum()
    assert 0.5 < f < 0.95
    d = {"100": [1.0, 0, 0], "111": [1.0, 1.0, 1.0], "1-23": [1.0, -2.0, 3.0]}[direction]
    d = np.asarray(d) / np.linalg.norm(d)
    p = dict(MAT)
    N = np.diag([0.2, 0.3, 0.5]); N[0, 1] = N[1, 0] = 0.05
    p["Nd"] = N.reshape(9)
    H = np.array([3e4, -1e4, 2e4])
    sigma = np.array([4e7, -1e7, 2e7, 5e6, -3e6, 1e7])
    orc = O.Oracle.from_mesh(case.mesh)
    orc.set_params(p, hext=H, sigma_ext=sigma)
    orc.set_m(np.tile(d, (case.mesh.n_nodes, 1)))
    e = orc.energies()
    Ms, mu0, K1 = p["Ms"], p["mu0"], p["K1"]
    anis = f * K1 * (d[0] ** 2 * d[1] ** 2 + d[1] ** 2 * d[2] ** 2 + d[2] ** 2 * d[0] ** 2)
    if direction == "100":
        assert anis == 0.0
    if direction == "111":
        assert np.isclose(anis, f * K1 / 3, rtol=1e-14)
    mbar = f * d
    ebar = f * _e0_closed(p, d) + _cubic_compliance_closed(p, sigma)
    scale = K1
    assert abs(e["exchange"]) < 1e-12 * scale
    assert abs(e["anisotropy"] - anis) < 1e-12 * scale
    assert abs(e["zeeman"] - (-mu0 * Ms * f * H @ d)) < 1e-12 * abs(mu0 * Ms * H @ d)
    assert abs(e["demag_far"] - 0.5 * mu0 * Ms ** 2 * mbar @ N @ mbar) < 1e-12 * mu0 * Ms ** 2
    work = -_tensor_contract(sigma, ebar)
    assert abs(e["stress"] - work) < 1e-10 * abs(work)
    m_av, e_av = orc.averages()
    assert np.allclose(m_av, mbar, rtol=1e-12, atol=1e-15)
    assert np.allclose(e_av, ebar, rtol=1e-10, atol=1e-16)
    parts = sum(e[k] for k in ("exchange", "anisotropy", "zeeman", "magnetoelastic", "stress", "demag_far"))
    assert abs(e["total"] - parts) < 1e-12 * abs(e["total"])


@pytest.mark.parametrize("direction", ["100", "111"])
def test_magnetoelastic_energy_of_uniform_state_under_stress(direction):
    """All-magnetic cell, uniform m, applied stress: E0 is uniform, so the
    periodic displacement vanishes (Eq. elasticity has a zero right-hand
    side), E - E0 = C^-1 sigma everywhere and the magnetoelastic density is
    (1/2) sigma : C^-1 sigma; a rigid translation of u changes nothing."""
    case = w.small_cube(6, seed=62, L=5e-8, jitter=0.15, shuffle=True)
    d = np.array([1.0, 0, 0]) if direction == "100" else np.ones(3) / np.sqrt(3)
    sigma = np.array([-3e7, 1e7, 2e7, -4e6, 6e6, 2e6])
    orc = O.Oracle.from_mesh(case.mesh)
    orc.set_params(MAT, sigma_ext=sigma)
    orc.set_m(np.tile(d, (case.mesh.n_nodes, 1)))
    b = orc.elastic_rhs()
    assert np.abs(b).max() < 1e-12 * MAT["c11"] * MAT["lambda100"] * (5e-8 / 5) ** 2
    eps = _cubic_compliance_closed(MAT, sigma)
    me = 0.5 * _tensor_contract(sigma, eps)
    e = orc.energies()
    assert abs(e["magnetoelastic"] - me) < 1e-11 * me
    orc.set_u(np.tile([3e-10, -1e-10, 2e-10], (case.mesh.n_nodes, 1)))
    assert abs(orc.energies()["magnetoelastic"] - me) < 1e-11 * me
    # the step keeps u = 0 up to the CG tolerance
    orc.set_u(np.zeros((case.mesh.n_nodes, 3)))
    orc.step(1e-12, 1)
    u = orc.get_u()
    assert np.abs(u - u.mean(0)).max() < 1e-12 * MAT["lambda100"] * 5e-8


def test_dm_avg_is_the_mean_over_magnetic_nodes():
    """Sec. 3.2's convergence measure, the mean over the magnetic nodes of
    |m^{n+1} - m^n|: a uniform macrospin (no magnetostriction, so the
    inclusion exerts no strain field) moves every magnetic node by the same
    chord, so dm_avg must equal that chord even though some nodes lie inside
    the inclusion only (and stay at zero)."""
    case = w.small_cube(7, seed=63, L=6e-8, jitter=0.15, sphere=0.35, shuffle=True)
    p = dict(MAT); p["lambda100"] = 0.0; p["lambda111"] = 0.0; p["cg_tol"] = 1e-12
    orc = O.Oracle.from_mesh(case.mesh)
    mag = orc.lumped_weights() > 0
    assert (~mag).sum() > 0
    mag_user = mag[orc.node_map()]
    d0 = np.array([1.0, 0.4, -0.3]); d0 /= np.linalg.norm(d0)
    orc.set_params(p, hext=(0.0, 0.2 * p["Ms"], 0.0))
    orc.set_m(np.tile(d0, (case.mesh.n_nodes, 1)))
    st = orc.step(3e-12, 1)
    m1 = orc.get_m()
    assert np.ptp(m1[mag_user], axis=0).max() < 1e-13
    assert np.abs(m1[~mag_user]).max() == 0.0
    chord = np.linalg.norm(m1[mag_user][0] - d0)
    assert chord > 1e-3
    assert abs(st["dm_avg"] - chord) < 1e-12 * chord


# ------------------------------------ a second tetrahedralization (valence)

def test_five_tet_split_geometry_and_patch_tests():
    """The five-tetrahedron split (variable valence: 8 or 32 tetrahedra per
    node) through the same identities: volumes sum to the cell, the Laplacian
    and the elastic operator vanish on linear fields at interior nodes."""
    case = w.small_cube(7, seed=14, L=1e-7, jitter=0.15, split="five")
    cnt = np.bincount(case.mesh.site[case.mesh.tets].ravel(), minlength=case.mesh.n_sites)
    assert set(np.unique(cnt)) == {8, 32}
    orc = O.Oracle.from_mesh(case.mesh)
    vol, _ = orc.geometry()
    assert np.isclose(vol.sum(), 1e-21, rtol=1e-12)
    un = O.Oracle.from_mesh(case.mesh, periodic=False)
    un.set_params(MAT)
    X = case.mesh.xyz
    interior = np.all((X > 1e-12) & (X < 1e-7 - 1e-12), axis=1)
    G = np.array([[0.3, -1.2, 2.0], [1.1, 0.4, -0.5], [-0.2, 0.9, 0.6]])
    lin = X @ G.T + 0.7e-7
    for op, x in ((O.OP_LAPLACE, np.repeat(lin[:, :1], 3, axis=1)), (O.OP_ELASTIC, lin)):
        y = un.apply(op, x)
        edge = np.abs(y[~interior]).max()
        assert edge > 0.0
        assert np.abs(y[interior]).max() < 1e-10 * edge
