"""Structured-then-jittered tetrahedral meshes of a periodic cube.

A cube [0, L]^3 carries n nodes per axis (both faces included), so the
periodic box has (n-1)^3 distinct lattice sites.  Every cell is split into six
tetrahedra around its main diagonal (the Kuhn split), which gives a conforming
mesh with 6 (n-1)^3 tetrahedra.  Interior nodes (those on no box face) may be
moved by a seeded uniform jitter; face nodes stay put so that opposite faces
still match node for node, which is what the periodic identification of the
paper (Sec. 2.5) needs.  Nonmagnetic inclusions are tagged by element centroid.

The mesh is returned unwrapped, exactly as a mesh generator would hand it to a
solver: the max-face copies of the min-face nodes are separate nodes.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from itertools import permutations

import numpy as np


@dataclass
class Inclusion:
    """Ellipsoid {x : |R^T (x - center) / semi| <= 1}; R's columns are its axes."""
    center: np.ndarray
    semi: np.ndarray
    rot: np.ndarray = field(default_factory=lambda: np.eye(3))


@dataclass
class Mesh:
    xyz: np.ndarray        # (n0, 3) float64 node coordinates [m]
    tets: np.ndarray       # (ne, 4) int32 node ids, positively oriented
    tags: np.ndarray       # (ne,) uint8, 0 = nonmagnetic inclusion, 1 = magnetic host
    lo: np.ndarray         # (3,) box min corner [m]
    hi: np.ndarray         # (3,) box max corner [m]
    n_axis: int            # nodes per axis of the source lattice
    site: np.ndarray       # (n0,) int64 periodic lattice site of every node

    @property
    def n_nodes(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_tets(self) -> int:
        return int(self.tets.shape[0])

    @property
    def n_sites(self) -> int:
        return (self.n_axis - 1) ** 3

    def per_site(self, values: np.ndarray) -> np.ndarray:
        """Broadcast one value per periodic site to every node, so that the
        copies of a node on opposite faces carry identical values."""
        return np.ascontiguousarray(values[self.site])


def kuhn_cube(n: int, L: float, jitter: float = 0.0, rng: np.random.Generator | None = None,
              lo: float = 0.0) -> Mesh:
    """n nodes per axis on [lo, lo+L]^3, Kuhn-split into 6 (n-1)^3 tetrahedra.

    jitter is the half-width of the uniform interior displacement as a fraction
    of the lattice spacing h = L/(n-1).
    """
    if n < 2:
        raise ValueError("need at least 2 nodes per axis")
    h = L / (n - 1)
    kk, jj, ii = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ii = ii.ravel(); jj = jj.ravel(); kk = kk.ravel()
    xyz = np.stack([ii, jj, kk], axis=1).astype(np.float64) * h + lo
    if jitter > 0.0:
        if rng is None:
            raise ValueError("jitter needs a seeded generator")
        interior = ((ii > 0) & (ii < n - 1) & (jj > 0) & (jj < n - 1) & (kk > 0) & (kk < n - 1))
        d = rng.uniform(-jitter * h, jitter * h, size=(int(interior.sum()), 3))
        xyz[interior] += d
    m = n - 1
    site = (ii % m) + m * ((jj % m) + m * (kk % m))

    cz, cy, cx = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    base = (cx.ravel() + n * (cy.ravel() + n * cz.ravel())).astype(np.int64)
    unit = np.eye(3, dtype=np.int64)
    stride = np.array([1, n, n * n], dtype=np.int64)
    tets = []
    for perm in permutations(range(3)):
        a, b, c = perm
        path = [np.zeros(3, np.int64), unit[a], unit[a] + unit[b], unit[a] + unit[b] + unit[c]]
        offs = [int(p @ stride) for p in path]
        sign = np.linalg.det(np.stack([path[1], path[2], path[3]], axis=1).astype(float))
        if sign < 0:
            offs[2], offs[3] = offs[3], offs[2]
        tets.append(base[:, None] + np.array(offs, dtype=np.int64)[None, :])
    tets = np.stack(tets, axis=1).reshape(-1, 4).astype(np.int32)
    tags = np.ones(tets.shape[0], dtype=np.uint8)
    return Mesh(xyz=xyz, tets=tets, tags=tags, lo=np.full(3, lo), hi=np.full(3, lo + L),
                n_axis=n, site=site.astype(np.int64))


# Five-tetrahedron split of a unit cell (corner bits x | y << 1 | z << 2): a
# central tetrahedron on four alternate corners and one tetrahedron cutting off
# each of the other four.  Cells alternate between the two mirror images by
# the parity of i + j + k, so that neighbouring cells split their shared face
# along the same diagonal.
_FIVE_EVEN = [(0, 3, 5, 6), (1, 0, 3, 5), (2, 0, 3, 6), (4, 0, 5, 6), (7, 3, 5, 6)]
_FIVE_ODD = [(1, 2, 4, 7), (0, 1, 2, 4), (3, 1, 2, 7), (5, 1, 4, 7), (6, 2, 4, 7)]


def five_tet_cube(n: int, L: float, jitter: float = 0.0, rng: np.random.Generator | None = None,
                  lo: float = 0.0) -> Mesh:
    """n nodes per axis on [lo, lo+L]^3 (n - 1 even, so the alternation also
    matches across the periodic faces), each cell split into five tetrahedra:
    5 (n-1)^3 tetrahedra; half the nodes carry 8 tetrahedra and 6 edge
    neighbours, the other half 32 and 18 (the Kuhn split gives every node 24
    and 14).  Jitter as in kuhn_cube."""
    if n < 3 or (n - 1) % 2:
        raise ValueError("the five-tetrahedron split needs an even number of cells per axis")
    h = L / (n - 1)
    kk, jj, ii = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ii = ii.ravel(); jj = jj.ravel(); kk = kk.ravel()
    xyz = np.stack([ii, jj, kk], axis=1).astype(np.float64) * h + lo
    if jitter > 0.0:
        if rng is None:
            raise ValueError("jitter needs a seeded generator")
        interior = ((ii > 0) & (ii < n - 1) & (jj > 0) & (jj < n - 1) & (kk > 0) & (kk < n - 1))
        xyz[interior] += rng.uniform(-jitter * h, jitter * h, size=(int(interior.sum()), 3))
    m = n - 1
    site = (ii % m) + m * ((jj % m) + m * (kk % m))
    cz, cy, cx = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    cx = cx.ravel(); cy = cy.ravel(); cz = cz.ravel()
    base = (cx + n * (cy + n * cz)).astype(np.int64)
    corner = np.array([(b & 1) + n * (((b >> 1) & 1) + n * (b >> 2)) for b in range(8)], dtype=np.int64)
    odd = (cx + cy + cz) % 2 == 1
    tets = np.empty((base.shape[0], 5, 4), dtype=np.int64)
    for t in range(5):
        te = corner[list(_FIVE_EVEN[t])]
        to = corner[list(_FIVE_ODD[t])]
        tets[:, t, :] = base[:, None] + np.where(odd[:, None], to[None, :], te[None, :])
    tets = tets.reshape(-1, 4)
    # positive orientation on the unjittered lattice
    X = (np.stack([ii, jj, kk], axis=1).astype(np.float64))[tets]
    det = np.linalg.det(X[:, 1:] - X[:, :1])
    flip = det < 0
    tets[flip, 2], tets[flip, 3] = tets[flip, 3].copy(), tets[flip, 2].copy()
    tags = np.ones(tets.shape[0], dtype=np.uint8)
    return Mesh(xyz=xyz, tets=tets.astype(np.int32), tags=tags, lo=np.full(3, lo), hi=np.full(3, lo + L),
                n_axis=n, site=site.astype(np.int64))


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniformly distributed rotation from a normalised Gaussian quaternion."""
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def tag_inclusions(mesh: Mesh, inclusions: list[Inclusion], chunk: int = 1 << 20) -> None:
    """Set tag 0 on every element whose centroid lies in an inclusion.

    Offsets from an inclusion centre use the nearest periodic image, so an
    inclusion that crosses a box face continues on the opposite face.
    """
    L = mesh.hi - mesh.lo
    for s in range(0, mesh.n_tets, chunk):
        t = mesh.tets[s:s + chunk]
        c = mesh.xyz[t].mean(axis=1)
        inside = np.zeros(t.shape[0], dtype=bool)
        for inc in inclusions:
            d = c - inc.center
            d -= L * np.round(d / L)
            q = (d @ inc.rot) / inc.semi
            inside |= np.einsum("ij,ij->i", q, q) <= 1.0
        mesh.tags[s:s + chunk][inside] = 0
