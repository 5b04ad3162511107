"""The largest configuration: the 3M-node cube (2,924,207 unique nodes,
17,545,242 tetrahedra, eight ellipsoidal inclusions), where the CPU oracle
would take minutes per step, checked through properties that hold at any
size (the oracle parity at this size is the 1M-node test's):

  - after two steps without precession (damping only) the total energy has
    not increased (the oracle pins monotone decay on small cells);
  - |m| = 1 on magnetic nodes to 1e-14, m = 0 on nodes inside inclusions only,
    every value finite;
  - the mixed form agrees with FP64 to 1e-6 (m and mean-removed u), the
    mixed form's bound.
"""
import numpy as np
import pytest

import workloads as w
from paper_2510_09812_amd import gspm

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_largest_cube_two_steps_properties_and_mixed_vs_fp64():
    print("[largest] building the 3M-node cube", flush=True)
    case = w.cube144_ellipsoids()
    out = {}
    for precision in (gspm.GSPM_FP64, gspm.GSPM_MIXED):
        print(f"[largest] precision {precision}: upload", flush=True)
        sim = gspm.Simulation(case.mesh, case.params, hext=tuple(case.hext), precession=False, precision=precision)
        sim.set_m(case.m0)
        e0 = sim.energies()["total"]
        st = sim.step(case.dt, 2)
        e1 = sim.energies()["total"]
        m, u = sim.get_m(), sim.get_u()
        info = sim.mesh_info()
        print(f"[largest] precision {precision}: {info['n_unique']} nodes, {info['n_tets']} tets, "
              f"mech iters {st['mech_iters']}, energy {e0:.6e} -> {e1:.6e}", flush=True)
        assert info["n_unique"] == 2924207 and info["n_tets"] == 17545242
        assert np.all(np.isfinite(m)) and np.all(np.isfinite(u))
        r = np.linalg.norm(m, axis=1)
        mag = r > 0
        assert np.abs(r[mag] - 1.0).max() < 1e-14
        assert mag.mean() > 0.5            # inclusions are a minority of the cell
        assert e1 <= e0 + 1e-12 * abs(e0)
        out[precision] = (m, u)
        sim.close()
    (m64, u64), (m32, u32) = out[gspm.GSPM_FP64], out[gspm.GSPM_MIXED]
    dm = _rel(m32, m64)
    du = _rel(u32 - u32.mean(axis=0), u64 - u64.mean(axis=0))
    print(f"[largest] mixed vs FP64: m {dm:.2e} u {du:.2e}", flush=True)
    assert dm < 1e-6 and du < 1e-6
