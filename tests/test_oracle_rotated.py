"""Pins of the oracle's rotated crystal frame (App. D).

The mesh, fields and loads live in the sample frame; the cubic crystal is
turned by R (v_sample = R v_crystal).  Checks against what the paper and the
mathematics fix:
  - the stiffness in the sample frame equals M C M^T with the Bond matrix M
    printed in App. D, for the paper's R (axes <111>, <-110>, <11-2>);
  - the spontaneous strain of a sample-frame m equals M E0(R^T m) with the
    closed form of App. A;
  - a rotation in the cubic point group changes nothing, on a full mesh;
  - a uniform state (a macrospin: no exchange, no displacement) has the same
    energy in the rotated crystal with rotated loads, and under the damping
    stage alone evolves exactly as R times the unrotated evolution (the
    precession stages of Algorithm B.1 update the components in a fixed
    order, so the full step is not covariant under a rotation of the axes);
  - the local field is minus the energy gradient in the rotated frame.
"""
import numpy as np
import pytest

import oracle as O
import workloads as w

MAT = dict(w.MATERIAL_FEGA)
S3, S2, S6 = np.sqrt(3.0), np.sqrt(2.0), np.sqrt(6.0)
R111 = np.array([[1 / S3, 1 / S3, 1 / S3], [-1 / S2, 1 / S2, 0.0], [-1 / S6, -1 / S6, 2 / S6]])


def _bond(R):
    """The Voigt rotation matrix of App. D, entry by entry as printed
    (order xx yy zz yz xz xy)."""
    (xx, xy, xz), (yx, yy, yz), (zx, zy, zz) = R
    return np.array([
        [xx ** 2, xy ** 2, xz ** 2, 2 * xy * xz, 2 * xx * xz, 2 * xx * xy],
        [yx ** 2, yy ** 2, yz ** 2, 2 * yy * yz, 2 * yx * yz, 2 * yx * yy],
        [zx ** 2, zy ** 2, zz ** 2, 2 * zy * zz, 2 * zx * zz, 2 * zx * zy],
        [yx * zx, yy * zy, yz * zz, yy * zz + yz * zy, yx * zz + yz * zx, yx * zy + yy * zx],
        [xx * zx, xy * zy, xz * zz, xy * zz + xz * zy, xx * zz + xz * zx, xx * zy + xy * zx],
        [xx * yx, xy * yy, xz * yz, xy * yz + xz * yy, xx * yz + xz * yx, xx * yy + xy * yx],
    ])


def _cubic_voigt(p):
    C = np.zeros((6, 6))
    C[:3, :3] = p["c12"]
    np.fill_diagonal(C[:3, :3], p["c11"])
    C[3, 3] = C[4, 4] = C[5, 5] = p["c44"]
    return C


def _e0_crystal(p, mc):
    """App. A, tensor components (xx yy zz yz xz xy)."""
    a, b = 1.5 * p["lambda100"], 1.5 * p["lambda111"]
    return np.array([a * (mc[0] ** 2 - 1 / 3), a * (mc[1] ** 2 - 1 / 3), a * (mc[2] ** 2 - 1 / 3),
                     b * mc[1] * mc[2], b * mc[0] * mc[2], b * mc[0] * mc[1]])


def _rot(R):
    p = dict(MAT)
    p["crystal_rot"] = np.asarray(R, float)
    return p


def test_paper_rotation_is_proper():
    assert np.allclose(R111 @ R111.T, np.eye(3), atol=1e-15) and abs(np.linalg.det(R111) - 1) < 1e-15


def test_stiffness_is_bond_rotated():
    M = _bond(R111)
    ref = M @ _cubic_voigt(MAT) @ M.T
    C = O.stiffness_voigt(_rot(R111))
    assert np.abs(C - ref).max() < 1e-12 * np.abs(ref).max()
    # the unrotated stiffness is the cubic Voigt matrix, and rotation keeps the invariants
    assert np.array_equal(O.stiffness_voigt(MAT), _cubic_voigt(MAT))
    assert abs(np.trace(C[:3, :3]) + 2 * np.trace(C[3:, 3:]) - np.trace(_cubic_voigt(MAT)[:3, :3])
               - 2 * np.trace(_cubic_voigt(MAT)[3:, 3:])) < 1e-9 * MAT["c11"]


def test_spontaneous_strain_rotates_with_the_bond_matrix():
    rng = np.random.default_rng(3)
    M = _bond(R111)
    for _ in range(5):
        m = rng.standard_normal(3); m /= np.linalg.norm(m)
        ref = M @ _e0_crystal(MAT, R111.T @ m)
        assert np.abs(O.spont_strain(_rot(R111), m) - ref).max() < 1e-17
    # along the crystal's [111] (the sample's x axis) the strain is lambda111 along x
    e = O.spont_strain(_rot(R111), np.array([1.0, 0.0, 0.0]))
    assert abs(e[0] - MAT["lambda111"]) < 1e-18


def test_rotated_local_field_is_energy_gradient():
    rng = np.random.default_rng(4)
    p = _rot(R111)
    scale = 1.0 / (MAT["mu0"] * MAT["Ms"] ** 2)
    for _ in range(6):
        m = rng.standard_normal(3)
        E = rng.standard_normal(6) * 3e-4
        H = rng.standard_normal(3) * 1e5
        h = O.h_local(p, m, E, np.zeros(3), hext=H)
        fd = np.zeros(3)
        for k in range(3):
            d = 1e-6
            mp = m.copy(); mp[k] += d
            mn = m.copy(); mn[k] -= d
            fd[k] = -(O.energy_density_local(p, mp, E, H) - O.energy_density_local(p, mn, E, H)) / (2 * d)
        assert np.allclose(h, scale * fd, rtol=1e-6, atol=1e-9 * np.abs(h).max())
    # along the rotated easy axes, at the matching spontaneous strain, the
    # anisotropy and magnetoelastic energies vanish; off them they do not
    for ax in np.eye(3):
        m = R111 @ ax
        assert abs(O.energy_density_local(p, m, O.spont_strain(p, m))) < 1e-9
    m = np.array([1.0, 0.0, 0.0])                 # the crystal's [111]: a hard axis for K1 > 0
    assert abs(O.energy_density_local(p, m, O.spont_strain(p, m)) - MAT["K1"] / 3) < 1e-9 * MAT["K1"]


def test_cubic_symmetry_rotation_changes_nothing():
    case = w.small_cube(7, seed=61, L=6e-8, jitter=0.15, sphere=0.3)
    rz = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    out = []
    for p in (case.params, {**case.params, "crystal_rot": rz}):
        orc = O.Oracle.from_mesh(case.mesh)
        orc.set_params(p, hext=(2e4, -1e4, 5e3), sigma_ext=(1e7, 0, -2e7, 3e6, 0, 1e6))
        orc.set_m(case.m0)
        orc.step(5e-12, 3)
        out.append((orc.get_m(), orc.get_u(), orc.energies()["total"]))
    assert np.abs(out[0][0] - out[1][0]).max() < 1e-12
    # the rotated stiffness equals the cubic one up to rounding, which CG
    # carries into u at the 1e-11 level
    assert np.abs(out[0][1] - out[1][1]).max() < 1e-9 * np.abs(out[0][1]).max()
    assert abs(out[0][2] - out[1][2]) < 1e-12 * abs(out[0][2])


@pytest.mark.parametrize("precession", [True, False])
def test_macrospin_in_the_rotated_crystal(precession):
    case = w.small_cube(5, seed=62, L=4e-8, jitter=0.15)
    m0 = np.array([0.3, 0.8, -0.52]); m0 /= np.linalg.norm(m0)
    H = np.array([-3e4, 1e4, 2e4])
    sig = np.array([[2e7, 3e6, -1e6], [3e6, -1e7, 4e6], [-1e6, 4e6, 5e6]])
    Nd = np.diag([0.2, 0.3, 0.5])
    voigt = lambda S: (S[0, 0], S[1, 1], S[2, 2], S[1, 2], S[0, 2], S[0, 1])
    res = []
    for R in (np.eye(3), R111):
        p = {**case.params, "crystal_rot": R, "Nd": (R @ Nd @ R.T).reshape(9)}
        orc = O.Oracle.from_mesh(case.mesh)
        orc.set_params(p, hext=tuple(R @ H), sigma_ext=voigt(R @ sig @ R.T), precession=precession)
        orc.set_m(np.tile(R @ m0, (case.mesh.n_nodes, 1)))
        e0 = orc.energies()["total"]
        orc.step(1e-11, 4)
        m = orc.get_m()
        assert np.abs(m - m[0]).max() < 1e-13          # it stays uniform
        res.append((R, m[0], e0, orc.energies()["total"]))
    (_, m_ref, e0_ref, e_ref), (R, m_rot, e0_rot, e_rot) = res
    assert np.linalg.norm(m_ref - m0) > 1e-3              # it moved
    assert abs(e0_rot - e0_ref) < 1e-10 * abs(e0_ref)
    if not precession:
        assert np.abs(m_rot - R @ m_ref).max() < 1e-12
        assert abs(e_rot - e_ref) < 1e-10 * abs(e_ref)
    else:
        # the precession stages differ, but both runs stay unit-length macrospins
        assert abs(np.linalg.norm(m_rot) - 1.0) < 1e-14


def test_improper_orientation_is_rejected():
    case = w.small_cube(4, seed=63, L=4e-8, jitter=0.0)
    orc = O.Oracle.from_mesh(case.mesh)
    with pytest.raises(O.OracleError):
        orc.set_params({**case.params, "crystal_rot": np.diag([1.0, 1.0, -1.0])})
    with pytest.raises(O.OracleError):
        orc.set_params({**case.params, "crystal_rot": 1.01 * np.eye(3)})
