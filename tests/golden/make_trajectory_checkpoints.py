"""Writes the oracle checkpoints of the long trajectory tests (run once; calls
only oracle/ and the seeded workloads).

  cube47_sphere_oracle.npz: the 100k-node cube with a sphere (200 steps of
    5 ps, CG tolerance 1e-8), m and u in the caller's node order after step
    200, and per step the elastic and GS iteration counts, dm_avg, mbar and
    the energies.
  cube100_ellipsoids_oracle_sample.npz: the 1M-node cube with three
    ellipsoids (10 steps of 10 ps, tolerance 1e-8); the full state is too
    large to store, so m and u after steps 5 and 10 are kept at 4096 seeded
    sample nodes, with per-step iteration counts, dm_avg, mbar, ebar and the
    energies (which the oracle computes over the whole mesh).

Usage: python tests/golden/make_trajectory_checkpoints.py [c2|c3|all]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
import workloads as w  # noqa: E402

ENERGY_KEYS = ("exchange", "anisotropy", "zeeman", "magnetoelastic", "stress", "demag_far", "total")
SAMPLE_SEED, SAMPLE_SIZE = 2024, 4096


def sample_nodes(n0: int) -> np.ndarray:
    return np.sort(np.random.default_rng(SAMPLE_SEED).choice(n0, size=SAMPLE_SIZE, replace=False))


def run(case, steps, keep, sample=None):
    orc = O.Oracle.from_mesh(case.mesh)
    orc.set_params(case.params, hext=case.hext)
    orc.set_m(case.m0)
    rows = {k: [] for k in ("mech_iters", "gs_iters", "dm_avg", "mbar", "ebar", "energies")}
    out = {}
    t0 = time.time()
    for k in range(1, steps + 1):
        st = orc.step(case.dt, 1)
        mbar, ebar = orc.averages()
        e = orc.energies()
        rows["mech_iters"].append(st["mech_iters"])
        rows["gs_iters"].append(sum(st["gs_iters"]))
        rows["dm_avg"].append(st["dm_avg"])
        rows["mbar"].append(mbar)
        rows["ebar"].append(ebar)
        rows["energies"].append([e[q] for q in ENERGY_KEYS])
        if k in keep:
            m, u = orc.get_m(), orc.get_u()
            if sample is not None:
                m, u = m[sample], u[sample]
            out[f"m{k}"] = m
            out[f"u{k}"] = u
        print(f"{case.name}: step {k} ({st['mech_iters']} elastic iterations, {time.time() - t0:.0f} s)", flush=True)
    for key, v in rows.items():
        out[key] = np.asarray(v)
    out["threads"] = np.int64(O.num_threads())
    return out


def main():
    which = sys.argv[1] if len(sys.argv) > 1 else "all"
    if which in ("c2", "all"):
        out = run(w.cube47_sphere(), 200, (200,))
        np.savez_compressed(os.path.join(HERE, "cube47_sphere_oracle.npz"), **out)
    if which in ("c3", "all"):
        case = w.cube100_ellipsoids()
        sample = sample_nodes(case.mesh.n_nodes)
        out = run(case, 10, (5, 10), sample)
        out["sample"] = sample
        np.savez_compressed(os.path.join(HERE, "cube100_ellipsoids_oracle_sample.npz"), **out)


if __name__ == "__main__":
    main()
