"""The deterministic create option: fixed-order sums (per-workgroup slots
added in a fixed order, element passes gathered per owned node) make steps
bitwise reproducible: repeated runs agree bit for bit, and 2n steps equal n
steps, a save and restore of the state into a fresh context, and n more.
Also checked against the oracle (the gather form computes the same
operators)."""
import numpy as np
import pytest

import oracle as O
import workloads as w
from paper_2510_09812_amd import gspm

pytestmark = pytest.mark.gpu

H_BENCH = 430.4e-9 / 99


def _case():
    return w.small_cube(17, seed=131, L=16 * H_BENCH, jitter=0.15, sphere=0.3, shuffle=True, m="noisy_x")


CONFIGS = {
    "fp64": dict(precision=gspm.GSPM_FP64, precond=False, local_demag=False),
    "fp64+precond": dict(precision=gspm.GSPM_FP64, precond=True, local_demag=False),
    "mixed+precond": dict(precision=gspm.GSPM_MIXED, precond=True, local_demag=False),
    "mixed+local_demag": dict(precision=gspm.GSPM_MIXED, precond=False, local_demag=True),
}


def _sim(case, cfg, m=None, u=None, ud=None):
    p = dict(case.params)
    p["cg_tol"] = 1e-8
    if cfg["precond"]:
        p["elastic_precond"] = gspm.GSPM_PRECOND_GREEN
        p["gs_precond"] = gspm.GSPM_PRECOND_JACOBI
    sim = gspm.Simulation(case.mesh, p, hext=(-0.4 * case.material["Ms"], 0.02 * case.material["Ms"], 0.0),
                          sigma_ext=(3e6, 0, 0, 0, 0, 0), local_demag=cfg["local_demag"], precision=cfg["precision"],
                          deterministic=True)
    sim.set_m(case.m0 if m is None else m)
    if u is not None:
        sim.set_u(u)
    if ud is not None:
        sim.set_ud(ud)
    return sim


def _state(sim, cfg):
    s = [sim.get_m(), sim.get_u()]
    if cfg["local_demag"]:
        s.append(sim.get_ud())
    return s


@pytest.mark.parametrize("name", list(CONFIGS))
def test_repeat_and_split_runs_are_bitwise_identical(name):
    cfg = CONFIGS[name]
    case = _case()
    n = 3
    a = _sim(case, cfg)
    sa = a.step(case.dt, 2 * n)
    ref = _state(a, cfg)
    a.close()
    b = _sim(case, cfg)
    b.step(case.dt, 2 * n)
    again = _state(b, cfg)
    b.close()
    c = _sim(case, cfg)
    c.step(case.dt, n)
    mid = _state(c, cfg)
    c.close()
    d = _sim(case, cfg, *mid)
    d.step(case.dt, n)
    split = _state(d, cfg)
    d.close()
    print(f"{name}: {2 * n} steps, elastic iterations {sa['mech_iters']}, GS {sa['gs_iters']}, "
          f"magnetostatic {sa['ms_iters']}; max |diff| repeat "
          f"{max(np.abs(x - y).max() for x, y in zip(ref, again)):.1e}, split "
          f"{max(np.abs(x - y).max() for x, y in zip(ref, split)):.1e}", flush=True)
    for x, y in zip(ref, again):
        assert np.array_equal(x, y)
    for x, y in zip(ref, split):
        assert np.array_equal(x, y)


def test_deterministic_steps_match_oracle():
    case = _case()
    cfg = CONFIGS["fp64+precond"]
    sim = _sim(case, cfg)
    p = dict(case.params)
    p["cg_tol"] = 1e-12
    p["elastic_precond"] = gspm.GSPM_PRECOND_GREEN
    p["gs_precond"] = gspm.GSPM_PRECOND_JACOBI
    hext = (-0.4 * case.material["Ms"], 0.02 * case.material["Ms"], 0.0)
    sig = (3e6, 0, 0, 0, 0, 0)
    sim.set_params(p, hext=hext, sigma_ext=sig)
    orc = O.Oracle.from_mesh(case.mesh)
    orc.set_params(p, hext=hext, sigma_ext=np.array(sig))
    orc.set_m(case.m0)
    sg = sim.step(case.dt, 3)
    so = orc.step(case.dt, 3)
    em = np.linalg.norm(sim.get_m() - orc.get_m()) / np.linalg.norm(orc.get_m())
    ug, uo = sim.get_u(), orc.get_u()
    ug, uo = ug - ug.mean(axis=0), uo - uo.mean(axis=0)
    eu = np.linalg.norm(ug - uo) / np.linalg.norm(uo)
    print(f"deterministic vs oracle: m {em:.2e} u {eu:.2e}; elastic {sg['mech_iters']}/{so['mech_iters']}, "
          f"GS {sg['gs_iters']}/{sum(so['gs_iters'])}", flush=True)
    assert em < 1e-9 and eu < 1e-9
    assert abs(sg["mech_iters"] - so["mech_iters"]) <= 3
    sim.close()


def test_network_starts_are_refused():
    case = _case()
    sim = _sim(case, CONFIGS["fp64"])
    with pytest.raises(gspm.GspmError) as e:
        sim.set_warm_start(gspm.GSPM_WARM_EXTRAPOLATE)
    assert e.value.status == gspm.GSPM_E_STATE
    sim.close()
