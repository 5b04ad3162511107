"""Per-phase device times (profile mode) and the final relative residual of
each solve reported in the step statistics."""
import numpy as np
import pytest

import workloads as w
from paper_2510_09812_amd import gspm

pytestmark = pytest.mark.gpu


def _case():
    return w.small_cube(13, seed=121, L=1.2e-7, jitter=0.15, sphere=0.3, m="noisy_x")


@pytest.mark.parametrize("precision", [gspm.GSPM_FP64, gspm.GSPM_MIXED])
@pytest.mark.parametrize("precond", [False, True])
def test_phase_times_and_final_residuals(precision, precond):
    case = _case()
    p = dict(case.params)
    p["cg_tol"] = 1e-8
    if precond:
        p["elastic_precond"] = gspm.GSPM_PRECOND_GREEN
        p["gs_precond"] = gspm.GSPM_PRECOND_JACOBI
    sim = gspm.Simulation(case.mesh, p, hext=(-0.3 * case.material["Ms"], 0.0, 0.0), local_demag=True,
                          precision=precision)
    sim.set_m(case.m0)
    sim.step(case.dt, 1)
    sim.set_profile(True)
    st = sim.step(case.dt, 3)
    ph, res = st["phase_ms"], st["final_residual"]
    total = sum(ph.values())
    print(f"precision {precision} precond {precond}: phases " + ", ".join(f"{k} {v:.2f}" for k, v in ph.items()) +
          f" ms (sum {total:.2f} of {st['elapsed_ms']:.2f}); residuals " +
          ", ".join(f"{k} {v:.2e}" for k, v in res.items()), flush=True)
    assert all(v >= 0.0 for v in ph.values())
    assert ph["elastic"] > 0 and ph["gs_stage1"] > 0 and ph["gs_stage3"] > 0 and ph["magnetostatic"] > 0
    # the phases tile each step up to the host's read of the commit check
    assert 0.7 * st["elapsed_ms"] <= total <= 1.01 * st["elapsed_ms"]
    ms_tol = max(1e-3 * p["cg_tol"], 1e-12)
    for k in ("elastic", "gs_stage1", "gs_stage2", "gs_stage3"):
        assert 0.0 < res[k] <= p["cg_tol"] * (1 + 1e-9), k
    assert 0.0 < res["magnetostatic"] <= ms_tol * (1 + 1e-9)
    # without profile mode the phases are not timed; the residuals still are
    sim.set_profile(False)
    st2 = sim.step(case.dt, 1)
    assert all(v == 0.0 for v in st2["phase_ms"].values())
    assert 0.0 < st2["final_residual"]["elastic"] <= p["cg_tol"] * (1 + 1e-9)
    sim.close()
