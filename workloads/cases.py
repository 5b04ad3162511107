"""Named, seeded workloads.

Each workload is a synthetic stand-in for the meshes of the paper's benchmarks
(Sec. 3): a periodic cube meshed with linear tetrahedra, optionally jittered,
with nonmagnetic spherical or ellipsoidal inclusions, at 1e3 to 3e6 nodes.  The
paper's COMSOL meshes and NiFe constants are not available, so a cubic Fe-Ga
material stands in.  Every random draw comes from
numpy.random.default_rng(SeedSequence(seed).spawn(k)).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .mesh import Inclusion, Mesh, five_tet_cube, kuhn_cube, random_rotation, tag_inclusions

MU0 = 4e-7 * np.pi
# Gyromagnetic ratio of the dimensionless time tau = gamma0 * Ms * t, in m/(A s).
GAMMA0 = MU0 * 1.76085963e11

MATERIAL_FEGA = dict(
    Ms=1.36e6, A=1.5e-11, K1=1.3e4, lambda100=2e-4, lambda111=-2e-5,
    c11=196e9, c12=156e9, c44=123e9, alpha=0.5, mu0=MU0, gamma0=GAMMA0,
)

# Lattice spacing of the 200 nm, 47-node cube; larger cubes keep it.
H_C2 = 200e-9 / 46


@dataclass
class Case:
    name: str
    mesh: Mesh
    material: dict
    m0: np.ndarray                 # (n0, 3) initial magnetisation, unit where magnetic
    hext: np.ndarray               # (3,) applied field [A/m]
    dt: float                      # time step [s]
    steps: int
    cg_tol: float = 1e-8
    sigma_ext: np.ndarray = field(default_factory=lambda: np.zeros(6))  # Voigt-ordered xx yy zz yz xz xy [Pa]
    nd: np.ndarray = field(default_factory=lambda: np.eye(3) / 3.0)      # body demag tensor (sphere)
    field_sweep: np.ndarray | None = None                                # (k, 3) fields for a hysteresis sweep

    @property
    def params(self) -> dict:
        p = dict(self.material)
        p["Nd"] = np.asarray(self.nd, dtype=np.float64).reshape(9)
        p["cg_tol"] = self.cg_tol
        return p


def _unit_rows(v: np.ndarray) -> np.ndarray:
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _m_random(mesh: Mesh, rng: np.random.Generator) -> np.ndarray:
    xi = rng.standard_normal((mesh.n_sites, 3))
    return mesh.per_site(_unit_rows(xi))


def _m_noisy_x(mesh: Mesh, rng: np.random.Generator, noise: float = 0.01) -> np.ndarray:
    xi = rng.standard_normal((mesh.n_sites, 3))
    v = np.array([1.0, 0.0, 0.0]) + noise * xi
    return mesh.per_site(_unit_rows(v))


def _random_ellipsoids(rng: np.random.Generator, k: int, L: float, lo_nm=10.0, hi_nm=40.0):
    out = []
    for _ in range(k):
        semi = rng.uniform(lo_nm, hi_nm, size=3) * 1e-9
        rot = random_rotation(rng)
        center = rng.uniform(0.0, L, size=3)
        out.append(Inclusion(center=center, semi=semi, rot=rot))
    return out


def _shuffle_nodes(mesh: Mesh, rng: np.random.Generator) -> Mesh:
    perm = rng.permutation(mesh.n_nodes)          # new id -> old id
    inv = np.empty_like(perm)
    inv[perm] = np.arange(mesh.n_nodes)
    return Mesh(xyz=mesh.xyz[perm].copy(), tets=inv[mesh.tets].astype(np.int32), tags=mesh.tags,
                lo=mesh.lo, hi=mesh.hi, n_axis=mesh.n_axis, site=mesh.site[perm].copy())


def cube10_random(seed: int = 1) -> Case:
    """100 nm cube, 10x10x10 nodes (4374 tets), all magnetic, random unit m,
    no applied field, dt = 1 ps, 20 steps, CG tolerance 1e-8."""
    s_m, = np.random.SeedSequence(seed).spawn(1)
    mesh = kuhn_cube(10, 100e-9)
    m0 = _m_random(mesh, np.random.default_rng(s_m))
    return Case("cube10_random", mesh, dict(MATERIAL_FEGA), m0, np.zeros(3), 1e-12, 20)


def cube47_sphere(seed: int = 2) -> Case:
    """200 nm cube, 47^3 nodes jittered by +-15% of h, a centred nonmagnetic
    sphere of radius 30 nm; m = [100] + 1% noise; H = -0.5 Ms [100];
    dt = 5 ps, 200 steps."""
    s_mesh, s_m = np.random.SeedSequence(seed).spawn(2)
    L = 200e-9
    mesh = kuhn_cube(47, L, jitter=0.15, rng=np.random.default_rng(s_mesh))
    tag_inclusions(mesh, [Inclusion(center=np.full(3, L / 2), semi=np.full(3, 30e-9))])
    m0 = _m_noisy_x(mesh, np.random.default_rng(s_m))
    hext = np.array([-0.5 * MATERIAL_FEGA["Ms"], 0.0, 0.0])
    return Case("cube47_sphere", mesh, dict(MATERIAL_FEGA), m0, hext, 5e-12, 200)


def cube100_ellipsoids(seed: int = 3) -> Case:
    """1M-node cube: 100^3 nodes at the 200/46 nm spacing (L = 430.4 nm),
    jittered, three random ellipsoids (semi-axes U(10, 40) nm, uniform random
    orientation and centre); m = [100] + 1% noise; H = -0.5 Ms [100];
    dt = 10 ps, 500 steps."""
    s_mesh, s_inc, s_m = np.random.SeedSequence(seed).spawn(3)
    n = 100
    L = (n - 1) * H_C2
    mesh = kuhn_cube(n, L, jitter=0.15, rng=np.random.default_rng(s_mesh))
    tag_inclusions(mesh, _random_ellipsoids(np.random.default_rng(s_inc), 3, L))
    m0 = _m_noisy_x(mesh, np.random.default_rng(s_m))
    hext = np.array([-0.5 * MATERIAL_FEGA["Ms"], 0.0, 0.0])
    return Case("cube100_ellipsoids", mesh, dict(MATERIAL_FEGA), m0, hext, 10e-12, 500)


def cube144_ellipsoids(seed: int = 4) -> Case:
    """3M-node cube: 144^3 nodes at the 200/46 nm spacing (L = 621.7 nm), eight
    random ellipsoids; hysteresis sweep H_k = (1 - 0.05 k) Ms [100], k = 0..40,
    200 steps of 10 ps per field."""
    s_mesh, s_inc, s_m = np.random.SeedSequence(seed).spawn(3)
    n = 144
    L = (n - 1) * H_C2
    mesh = kuhn_cube(n, L, jitter=0.15, rng=np.random.default_rng(s_mesh))
    tag_inclusions(mesh, _random_ellipsoids(np.random.default_rng(s_inc), 8, L))
    m0 = _m_noisy_x(mesh, np.random.default_rng(s_m))
    Ms = MATERIAL_FEGA["Ms"]
    sweep = np.array([[(1.0 - 0.05 * k) * Ms, 0.0, 0.0] for k in range(41)])
    return Case("cube144_ellipsoids", mesh, dict(MATERIAL_FEGA), m0, sweep[0], 10e-12, 200,
                field_sweep=sweep)


def small_cube(n: int, seed: int, L: float = 40e-9, jitter: float = 0.15, sphere: float = 0.0,
               m: str = "random", hext=(0.0, 0.0, 0.0), dt: float = 2e-12, steps: int = 5,
               shuffle: bool = False, split: str = "kuhn") -> Case:
    """Small test meshes of arbitrary (ragged) size; optional centred sphere of
    radius `sphere` (fraction of L), seeded node shuffling, and the cell split
    ("kuhn": six tetrahedra per cell; "five": five, alternating by parity,
    n - 1 even)."""
    s_mesh, s_m, s_perm = np.random.SeedSequence(seed).spawn(3)
    gen = five_tet_cube if split == "five" else kuhn_cube
    mesh = gen(n, L, jitter=jitter, rng=np.random.default_rng(s_mesh) if jitter > 0 else None)
    if sphere > 0.0:
        tag_inclusions(mesh, [Inclusion(center=np.full(3, L / 2), semi=np.full(3, sphere * L))])
    if shuffle:
        mesh = _shuffle_nodes(mesh, np.random.default_rng(s_perm))
    rng = np.random.default_rng(s_m)
    m0 = _m_random(mesh, rng) if m == "random" else _m_noisy_x(mesh, rng)
    return Case(f"small_cube{n}", mesh, dict(MATERIAL_FEGA), m0, np.asarray(hext, float), dt, steps)


def warm_start_training(seed: int, n: int = 47, inclusions: int = 3) -> Case:
    """Training family of the learned elastic warm start: n^3 nodes at the
    1M-node cube's spacing (47^3 ~ 100k nodes), jittered, `inclusions` random
    ellipsoids; m = [100] + 1% noise; H = -0.5 Ms [100]; dt = 10 ps."""
    s_mesh, s_inc, s_m = np.random.SeedSequence(seed).spawn(3)
    L = (n - 1) * H_C2
    mesh = kuhn_cube(n, L, jitter=0.15, rng=np.random.default_rng(s_mesh))
    tag_inclusions(mesh, _random_ellipsoids(np.random.default_rng(s_inc), inclusions, L))
    m0 = _m_noisy_x(mesh, np.random.default_rng(s_m))
    hext = np.array([-0.5 * MATERIAL_FEGA["Ms"], 0.0, 0.0])
    return Case(f"warm_start_training{n}_s{seed}", mesh, dict(MATERIAL_FEGA), m0, hext, 10e-12, 60)


CASES = {
    "cube10_random": cube10_random,
    "cube47_sphere": cube47_sphere,
    "cube100_ellipsoids": cube100_ellipsoids,
    "cube144_ellipsoids": cube144_ellipsoids,
}
