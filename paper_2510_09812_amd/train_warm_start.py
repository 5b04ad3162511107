"""Train the learned elastic warm start with the library's own GPU kernels.

Samples come from the library's FP64 time step on meshes of the training
family (`workloads.warm_start_training`: ~100k nodes at the 1M-node cube's
spacing, random ellipsoidal inclusions, m = [100] + noise, H = -0.5 Ms [100],
dt = 10 ps).  Step n of a trajectory gives the sample (m^{n-1}, m^n,
u^n - u^{n-1}), u^n being the elastic solution at m^n.  Training runs Adam
on the mean-removed MSE (gspm_mpnn_train_step: forward, loss, backward and
update all in the library's HIP kernels), one mesh at a time.  The held-out
trajectory reports the K-norm error left by the learned start, as a fraction
of the previous-step start's.

    python -m paper_2510_09812_amd.train_warm_start --out paper_2510_09812_amd/weights/warm_start.f32
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import workloads as w  # noqa: E402
from paper_2510_09812_amd import gspm  # noqa: E402

DEFAULT_OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "warm_start.f32")


def init_params(seed: int) -> np.ndarray:
    """Gaussian weights scaled by 1/sqrt(fan-in), zero biases, a small decoder."""
    rng = np.random.default_rng(seed)
    parts = []

    def mat(o, i, scale=1.0):
        parts.append((rng.standard_normal((o, i)) * scale / np.sqrt(i)).ravel())

    def vec(k):
        parts.append(np.zeros(k))

    mat(64, 7); vec(64)
    for _ in range(3):
        mat(64, 64); mat(64, 64); mat(64, 3); vec(64); mat(64, 128, 0.5); vec(64)
    mat(3, 64, 0.1); vec(3)
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == gspm.GSPM_MPNN_PARAMS
    return p


def trajectory(sim, case, steps: int):
    """Samples (m^{n-1}, m^n, u^n - u^{n-1}) of `steps` FP64 steps from m0."""
    sim.set_m(case.m0)
    sim.set_u(np.zeros_like(case.m0))
    ms, us = [sim.get_m()], []
    for _ in range(steps):
        sim.step(case.dt, 1)
        us.append(sim.get_u())       # solution at ms[-1]
        ms.append(sim.get_m())
    return [(ms[k - 1], ms[k], us[k] - us[k - 1]) for k in range(1, steps)]


def knorm_ratio(sim, samples, u_prev_list):
    """sqrt(e1' K e1 / e0' K e0): e0 the previous-step start's error, e1 the learned start's."""
    out = []
    for (mp, m, du), up in zip(samples, u_prev_list):
        sim.set_m(m)
        sim.set_u(up)
        u0, s = sim.mpnn_warm_start(mp)
        e0 = du
        e1 = (up + du) - u0
        k0 = float(np.sum(e0 * sim.apply(gspm.GSPM_OP_ELASTIC, e0)))
        k1 = float(np.sum(e1 * sim.apply(gspm.GSPM_OP_ELASTIC, e1)))
        out.append(np.sqrt(k1 / k0) if k0 > 0 else 1.0)
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--meshes", type=int, default=2, help="training meshes (one more is held out)")
    ap.add_argument("--n", type=int, default=47, help="nodes per axis of the training meshes")
    ap.add_argument("--steps", type=int, default=40, help="GSPM steps per trajectory")
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=7)
    args = ap.parse_args()

    params = init_params(args.seed)
    rng = np.random.default_rng(args.seed)
    t0 = time.perf_counter()
    log = {"train_loss": [], "heldout_knorm_ratio": None}
    for mi in range(args.meshes):
        case = w.warm_start_training(100 + mi, n=args.n)
        sim = gspm.Simulation(case.mesh, case.params, hext=case.hext)
        samples = trajectory(sim, case, args.steps)
        print(f"[train] mesh {mi}: {len(samples)} samples in {time.perf_counter() - t0:.1f} s", flush=True)
        sim.mpnn_set_params(params)
        for ep in range(args.epochs):
            losses = []
            for k in rng.permutation(len(samples)):
                mp, m, du = samples[k]
                losses.append(sim.mpnn_train_step(mp, m, du, lr=args.lr)[0])
            log["train_loss"].append(float(np.mean(losses)))
            if ep % 5 == 0 or ep == args.epochs - 1:
                print(f"[train] mesh {mi} epoch {ep}: mean loss {np.mean(losses):.4e}", flush=True)
        params = sim.mpnn_get_params()
        sim.close()
    # held-out mesh
    case = w.warm_start_training(100 + args.meshes, n=args.n)
    sim = gspm.Simulation(case.mesh, case.params, hext=case.hext)
    sim.set_m(case.m0)
    sim.set_u(np.zeros_like(case.m0))
    ms, us = [sim.get_m()], []
    for _ in range(args.steps):
        sim.step(case.dt, 1)
        us.append(sim.get_u())
        ms.append(sim.get_m())
    samples = [(ms[k - 1], ms[k], us[k] - us[k - 1]) for k in range(1, args.steps)]
    sim.mpnn_set_params(params)
    ratios = knorm_ratio(sim, samples, [us[k - 1] for k in range(1, args.steps)])
    sim.close()
    log["heldout_knorm_ratio"] = [float(r) for r in ratios]
    print(f"[train] held-out K-norm error ratio learned/previous: median {np.median(ratios):.3f}, "
          f"mean {np.mean(ratios):.3f} over {len(ratios)} steps; {time.perf_counter() - t0:.1f} s", flush=True)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    params.astype(np.float32).tofile(args.out)
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump({"args": vars(args), **log}, f)
    return 0


if __name__ == "__main__":
    sys.exit(main())
