"""The seeded input generator: sizes, orientation, periodic faces, tags."""
import numpy as np
import pytest

import workloads as w


def _det(mesh):
    x = mesh.xyz[mesh.tets]
    return np.linalg.det(x[:, 1:] - x[:, :1])


@pytest.mark.parametrize("n", [3, 4, 7, 10])
def test_kuhn_counts_and_volume(n):
    mesh = w.kuhn_cube(n, 1.0)
    assert mesh.n_nodes == n ** 3
    assert mesh.n_tets == 6 * (n - 1) ** 3
    d = _det(mesh)
    assert (d > 0).all()
    assert np.isclose(d.sum() / 6.0, 1.0, rtol=1e-12)


def test_cube10_sizes():
    c = w.cube10_random()
    assert c.mesh.n_nodes == 1000 and c.mesh.n_tets == 4374 and c.mesh.n_sites == 729
    assert np.allclose(np.linalg.norm(c.m0, axis=1), 1.0)


def test_jitter_keeps_faces_and_orientation():
    c = w.small_cube(8, seed=5, L=1.0, jitter=0.15)
    mesh = c.mesh
    assert (_det(mesh) > 0).all()
    ref = w.kuhn_cube(8, 1.0)
    on_face = np.any((ref.xyz == 0.0) | (np.isclose(ref.xyz, 1.0)), axis=1)
    assert np.array_equal(mesh.xyz[on_face], ref.xyz[on_face])
    assert not np.allclose(mesh.xyz[~on_face], ref.xyz[~on_face])
    # periodic copies of a site carry the same initial m
    for s in np.unique(mesh.site)[:50]:
        rows = c.m0[mesh.site == s]
        assert np.ptp(rows, axis=0).max() == 0.0


def test_sphere_inclusion_volume():
    c = w.small_cube(21, seed=1, L=1.0, jitter=0.0, sphere=0.3)
    d = _det(c.mesh) / 6.0
    v_inc = d[c.mesh.tags == 0].sum()
    assert abs(v_inc - 4.0 / 3.0 * np.pi * 0.3 ** 3) < 0.05 * 4.0 / 3.0 * np.pi * 0.3 ** 3


def test_seeded_reproducible():
    a = w.small_cube(6, seed=3, shuffle=True)
    b = w.small_cube(6, seed=3, shuffle=True)
    assert np.array_equal(a.mesh.xyz, b.mesh.xyz) and np.array_equal(a.mesh.tets, b.mesh.tets)
    assert np.array_equal(a.m0, b.m0)
