"""Create options of the C ABI: the internal node order (Morton curve, the
caller's order, reverse Cuthill-McKee) changes the owner blocks and halos but
not the result, and a caller-supplied device allocator (PyTorch's caching
allocator here) holds every device buffer of the context."""
import numpy as np
import pytest

import workloads as w
from paper_2510_09812_amd import gspm

pytestmark = pytest.mark.gpu


def _run(case, **kw):
    p = dict(case.params)
    p["cg_tol"] = 1e-12
    sim = gspm.Simulation(case.mesh, p, hext=(-3e5, 0.0, 0.0), **kw)
    sim.set_m(case.m0)
    st = sim.step(2e-12, 3)
    out = sim.get_m(), sim.get_u(), st, sim.mesh_info()
    sim.close()
    return out


@pytest.mark.parametrize("reorder", [gspm.GSPM_REORDER_NONE, gspm.GSPM_REORDER_RCM])
def test_node_orders_give_the_same_steps(reorder):
    case = w.small_cube(13, seed=121, L=1.2e-7, jitter=0.15, sphere=0.3)
    m0, u0, s0, i0 = _run(case)
    m1, u1, s1, i1 = _run(case, reorder=reorder)
    em = np.abs(m1 - m0).max()
    eu = np.abs(u1 - u0).max() / np.abs(u0).max()
    print(f"order {reorder}: element copies {i1['n_elem_copies']} (Morton {i0['n_elem_copies']}), "
          f"m {em:.1e} u {eu:.1e}, elastic iterations {s1['mech_iters']} / {s0['mech_iters']}", flush=True)
    assert em < 1e-12 and eu < 1e-10
    assert abs(s1["mech_iters"] - s0["mech_iters"]) <= 3


def test_torch_allocator_holds_the_context_memory():
    import torch
    case = w.small_cube(17, seed=122, L=1.6e-7, jitter=0.15, sphere=0.3)
    m0, u0, _, _ = _run(case)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated(0)
    alloc = gspm.torch_allocator(0)
    p = dict(case.params)
    p["cg_tol"] = 1e-12
    p["elastic_precond"] = gspm.GSPM_PRECOND_GREEN        # its buffers come from the allocator too
    sim = gspm.Simulation(case.mesh, p, hext=(-3e5, 0.0, 0.0), allocator=alloc)
    held = torch.cuda.memory_allocated(0) - before
    sim.set_params(dict(case.params, cg_tol=1e-12), hext=(-3e5, 0.0, 0.0))
    sim.set_m(case.m0)
    sim.step(2e-12, 3)
    m1, u1 = sim.get_m(), sim.get_u()
    n = sim.mesh_info()["n_unique"]
    print(f"allocator: {held} bytes held through PyTorch for {n} nodes", flush=True)
    assert held > 18 * 3 * 8 * n                       # at least the arena's 3-vectors
    sim.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated(0) == before     # every buffer went back
    assert np.abs(m1 - m0).max() < 1e-12
    assert np.abs(u1 - u0).max() < 1e-10 * np.abs(u0).max()
