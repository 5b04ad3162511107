"""Train the learned elastic warm start with the library's own GPU kernels.

Samples come from the library's FP64 time step on meshes of the training
family (`workloads.warm_start_training`: ~100k nodes at the 1M-node cube's
spacing, random ellipsoidal inclusions, m = [100] + noise, H = -0.5 Ms [100],
dt = 10 ps).  Step n of a trajectory gives the sample (m^{n-1}, m^n,
u^n - u^{n-1}), u^n being the elastic solution at m^n.  Training runs Adam
on the mean-removed MSE (gspm_mpnn_train_step: forward, loss, backward and
update all in the library's HIP kernels), one mesh at a time.  The held-out
trajectory reports, for the network start, the extrapolated start and the
learned start (both directions), the K-norm error and the residual 2-norm
each leaves, as a fraction of the previous-step start's.  With --eval-only
the same evaluation of existing weights is written into their .json log.

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


def trajectory(sim, case, steps: int, target: str = "du"):
    """Samples (m^{n-1}, m^n, t) of `steps` FP64 steps from m0, t = u^n - u^{n-1}
    (target "du"), or that minus the previous increment u^{n-1} - u^{n-2}
    (target "du-e": what the extrapolated start leaves, the part the learned
    start's second direction cannot supply)."""
    sim.set_m(case.m0)
    sim.set_u(np.zeros_like(case.m0))
    ms, us = [sim.get_m()], []
    for _ in range(steps):
        sim.step(case.dt, 1)
        us.append(sim.get_u())       # solution at ms[-1]
        ms.append(sim.get_m())
    if target == "du":
        return [(ms[k - 1], ms[k], us[k] - us[k - 1]) for k in range(1, steps)]
    return [(ms[k - 1], ms[k], (us[k] - us[k - 1]) - (us[k - 1] - us[k - 2])) for k in range(2, steps)]


def training_case(seed: int, n: int, vary: bool):
    """The training family; with vary, 1 to 3 inclusions by seed."""
    return w.warm_start_training(seed, n=n, inclusions=1 + seed % 3 if vary else 3)


def solver_params(case, precond: bool) -> dict:
    """The case's parameters; with precond both preconditioners (same solutions to the CG tolerance)."""
    p = dict(case.params)
    if precond:
        p["elastic_precond"] = gspm.GSPM_PRECOND_GREEN
        p["gs_precond"] = gspm.GSPM_PRECOND_JACOBI
    return p


def start_ratios(sim, ms, us):
    """For held-out steps n >= 2, the K-norm error and the residual 2-norm of
    three starts, each relative to the previous-step start's: the network
    increment alone, the previous increment alone (extrapolation) and both
    (the learned start).  The network starts come from the library; the
    extrapolated start takes the same residual-minimising coefficient the
    library would, c = (K e).r0 / |K e|^2 with r0 = K (u^n - u^{n-1})
    (u^n solves the step's system to the CG tolerance)."""
    out = {"knorm": {"network": [], "extrapolated": [], "learned": []},
           "residual": {"network": [], "extrapolated": [], "learned": []}}
    K = lambda v: sim.apply(gspm.GSPM_OP_ELASTIC, v)
    for n in range(2, len(us)):
        m_prev, m, u_prev, u_prev2, u_sol = ms[n - 1], ms[n], us[n - 1], us[n - 2], us[n]
        e0 = u_sol - u_prev
        r0 = K(e0)
        k0, n0 = float(np.sum(e0 * r0)), float(np.linalg.norm(r0))
        if k0 <= 0 or n0 <= 0:
            continue
        sim.set_m(m)
        sim.set_u(u_prev)
        u_net, _ = sim.mpnn_warm_start(m_prev)
        u_both, _ = sim.mpnn_warm_start(m_prev, u_prev2)
        e = u_prev - u_prev2
        ke = K(e)
        kk = float(np.sum(ke * ke))
        c = float(np.sum(ke * r0)) / kk if kk > 0 else 0.0   # (a settled trajectory: no previous increment)
        for key, u0 in (("network", u_net), ("learned", u_both), ("extrapolated", u_prev + c * e)):
            err = u_sol - u0
            kerr = K(err)
            out["knorm"][key].append(float(np.sqrt(max(float(np.sum(err * kerr)), 0.0) / k0)))
            out["residual"][key].append(float(np.linalg.norm(kerr)) / n0)
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
    ap.add_argument("--eval-only", default="", help="evaluate these weights on the held-out mesh, no training")
    ap.add_argument("--passes", type=int, default=1, help="passes over all training meshes (trajectories regenerated)")
    ap.add_argument("--target", choices=("du", "du-e"), default="du",
                    help="training target: the displacement increment, or its change from the previous one")
    ap.add_argument("--vary-inclusions", action="store_true", help="1 to 3 inclusions per mesh")
    ap.add_argument("--no-precond", action="store_true", help="generate trajectories with the unpreconditioned solves")
    args = ap.parse_args()
    precond = not args.no_precond

    params = init_params(args.seed)
    if args.eval_only:
        params = np.fromfile(args.eval_only, dtype=np.float32)
    rng = np.random.default_rng(args.seed)
    t0 = time.perf_counter()
    log = {"train_loss": [], "heldout": None}
    n_samples = 0
    for ps in range(0 if args.eval_only else args.passes):
        for mi in range(args.meshes):
            case = training_case(100 + mi, args.n, args.vary_inclusions)
            sim = gspm.Simulation(case.mesh, solver_params(case, precond), hext=case.hext)
            samples = trajectory(sim, case, args.steps, args.target)
            n_samples += len(samples)
            sim.mpnn_set_params(params)
            for ep in range(args.epochs):
                losses = []
                for k in rng.permutation(len(samples)):
                    mp, m, du = samples[k]
                    losses.append(sim.mpnn_train_step(mp, m, du, lr=args.lr)[0])
                log["train_loss"].append(float(np.mean(losses)))
            print(f"[train] pass {ps} mesh {mi}: {len(samples)} samples ({n_samples} so far), mean loss "
                  f"{log['train_loss'][-1]:.4e}, {time.perf_counter() - t0:.1f} s", flush=True)
            params = sim.mpnn_get_params()
            sim.close()
    log["samples"] = n_samples
    # held-out mesh
    case = training_case(100 + args.meshes, args.n, args.vary_inclusions)
    sim = gspm.Simulation(case.mesh, solver_params(case, precond), hext=case.hext)
    sim.set_m(case.m0)
    sim.set_u(np.zeros_like(case.m0))
    ms, us = [sim.get_m()], []
    for _ in range(args.steps):
        sim.step(case.dt, 1)
        us.append(sim.get_u())
        ms.append(sim.get_m())
    sim.mpnn_set_params(params)
    ratios = start_ratios(sim, ms, us)
    sim.close()
    for metric, per in ratios.items():
        for key, v in per.items():
            print(f"[train] held-out {metric} ratio {key}/previous: median {np.median(v):.3f}, "
                  f"mean {np.mean(v):.3f} over {len(v)} steps", flush=True)
    print(f"[train] {time.perf_counter() - t0:.1f} s", flush=True)
    if args.eval_only:
        logf = os.path.splitext(args.eval_only)[0] + ".json"
        prev = {}
        if os.path.exists(logf):
            with open(logf) as f:
                prev = json.load(f)
        prev.pop("heldout_knorm_ratio", None)
        prev["heldout"] = ratios
        with open(logf, "w") as f:
            json.dump(prev, f)
        return 0
    log["heldout"] = ratios
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    params.astype(np.float32).tofile(args.out)
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump({"args": vars(args), **log}, f)
    return 0


if __name__ == "__main__":
    sys.exit(main())
