"""CPU FP64 oracle of the learned elastic warm start -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this module; the product library never does.  Plain numpy in FP64,
with an optional emulation of BF16 storage (round-to-nearest-even to 8
significand bits) at the points where the GPU network stores activations and
weights.

The paper does not describe a learned warm start; the network is the reading
this project takes for it (a message-passing net that predicts the elastic
displacement increment from the magnetisation increment):

  node input   x_i = tag_i [dm_i / s_m, m_i, 1]                  (7 values)
               s_m = sqrt(sum_i w_i |dm_i|^2 / sum_i w_i), dm = m^n - m^{n-1},
               tag_i = 1 on magnetic nodes (w_i > 0), else 0 (m is zero on
               the other nodes, so the mask only fixes what arbitrary inputs
               give there)
  encoder      h_i = SiLU(W0 x_i + b0)                              (64)
  3 layers     z_ij = Wa h_i + Wb h_j + We e_ij + c   over directed mesh edges,
               e_ij = nearest-image (x_j - x_i) / hbar,  hbar = (6 mean V_e)^(1/3)
               a_i  = mean_{j in N(i)} SiLU(z_ij)
               h_i <- h_i + Wu [h_i ; a_i] + bu
  decoder      y_i = Wd h_i + bd                                    (3)
  increment    d = (lambda100 hbar s_m) (y - y_p0)   (zero at the pinned node)
  start        u0 = u_prev + s d,  s = (K d).r0 / |K d|^2,  r0 = b - K u_prev
               (the step along d that minimises the residual 2-norm, the
               quantity CG's stopping test measures: |b - K u0| <= |r0|);
               with the previous increment e = u_prev - u_prev2 also
               available, u0 = u_prev + a d + c e with (a, c) minimising
               |r0 - a K d - c K e| (least squares on span{K d, K e})

Training minimises the mean squared difference between the mean-removed
network output and the mean-removed normalised target
t = (u^n - u^{n-1}) / (lambda100 hbar s_m), with Adam.

Parameter vector (float, this order; matrices row-major, out x in):
  W0[64][7] b0[64] | 3 x (Wa[64][64] Wb[64][64] We[64][3] c[64] Wu[64][128] bu[64]) | Wd[3][64] bd[3]
"""
from __future__ import annotations

import numpy as np

F_IN, HID, N_LAYERS, F_OUT = 7, 64, 3, 3


def param_shapes():
    shapes = [("W0", (HID, F_IN)), ("b0", (HID,))]
    for l in range(N_LAYERS):
        shapes += [(f"Wa{l}", (HID, HID)), (f"Wb{l}", (HID, HID)), (f"We{l}", (HID, 3)), (f"c{l}", (HID,)),
                   (f"Wu{l}", (HID, 2 * HID)), (f"bu{l}", (HID,))]
    shapes += [("Wd", (F_OUT, HID)), ("bd", (F_OUT,))]
    return shapes


def param_count() -> int:
    return int(sum(np.prod(s) for _, s in param_shapes()))


def unpack(vec):
    """Flat parameter vector -> dict of FP64 arrays (copies)."""
    vec = np.asarray(vec, dtype=np.float64)
    assert vec.size == param_count()
    out, o = {}, 0
    for name, shp in param_shapes():
        k = int(np.prod(shp))
        out[name] = vec[o:o + k].reshape(shp).copy()
        o += k
    return out


def pack(p) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in param_shapes()])


# ------------------------------------------------------------------ BF16

def bf16_round(a):
    """Round to the nearest BF16 value (ties to even), returned as FP64.

    Works on the FP32 bit pattern: BF16 keeps the top 16 bits; adding 0x7FFF
    plus the lowest kept bit before truncating rounds to nearest, ties to even.
    Inputs are first rounded to FP32 (the GPU stores FP32 accumulators)."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isfinite(f), out, f.astype(np.float64))


def _ident(a):
    return np.asarray(a, dtype=np.float64)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


# ------------------------------------------------------------------ graph

class Graph:
    """Directed edge graph of a periodic tetrahedral mesh on its unique nodes.

    Every pair of distinct unique nodes that share a tetrahedron is joined in
    both directions.  Edges are stored by source node (CSR: ptr, nbr) with
    the nearest-image edge vector divided by hbar."""

    def __init__(self, n, tets_unique, coords, box, vol_mean):
        self.n = int(n)
        t = np.asarray(tets_unique, dtype=np.int64)
        pairs = []
        for a in range(4):
            for b in range(4):
                if a != b:
                    pairs.append(np.stack([t[:, a], t[:, b]], axis=1))
        e = np.concatenate(pairs)
        e = e[e[:, 0] != e[:, 1]]
        e = np.unique(e, axis=0)                       # sorted by (source, target)
        self.src, self.dst = e[:, 0], e[:, 1]
        self.ptr = np.zeros(self.n + 1, dtype=np.int64)
        np.add.at(self.ptr, self.src + 1, 1)
        self.ptr = np.cumsum(self.ptr)
        self.deg = np.diff(self.ptr).astype(np.float64)
        self.hbar = (6.0 * vol_mean) ** (1.0 / 3.0)
        box = np.asarray(box, dtype=np.float64)
        d = coords[self.dst] - coords[self.src]
        d -= box * np.round(d / box)
        self.evec = d / self.hbar

    @classmethod
    def from_oracle(cls, orc, mesh):
        """Graph on the oracle's unique nodes (its periodic identification)."""
        nmap = orc.node_map()
        coords = np.zeros((orc.n, 3))
        coords[nmap] = mesh.xyz
        box = np.asarray(mesh.hi) - np.asarray(mesh.lo)
        return cls(orc.n, nmap[mesh.tets], coords, box, orc.total_volume() / mesh.tets.shape[0])


# ------------------------------------------------------------------ network

def features(m, m_prev, w):
    """Node inputs and the increment scale s_m (weighted rms of dm over the
    magnetic nodes)."""
    dm = np.asarray(m, np.float64) - np.asarray(m_prev, np.float64)
    w = np.asarray(w, np.float64)
    sm = np.sqrt(np.sum(w[:, None] * dm * dm) / np.sum(w))
    tag = (w > 0).astype(np.float64)
    x = np.zeros((m.shape[0], F_IN))
    if sm > 0:
        x[:, 0:3] = tag[:, None] * dm / sm
    x[:, 3:6] = tag[:, None] * np.asarray(m, np.float64)
    x[:, 6] = tag
    return x, sm


def forward(p, x, g: Graph, bf16=False):
    """Network output y (n x 3) and the cache the backward pass needs."""
    r = bf16_round if bf16 else _ident
    P = {k: r(v) for k, v in p.items()}
    X = r(x)
    pre0 = X @ P["W0"].T + P["b0"]
    h = r(silu(pre0))
    cache = {"X": X, "pre0": pre0, "layers": [], "P": P}
    for l in range(N_LAYERS):
        A = r(h @ P[f"Wa{l}"].T)
        B = r(h @ P[f"Wb{l}"].T)
        z = A[g.src] + B[g.dst] + g.evec @ P[f"We{l}"].T + P[f"c{l}"]
        s = silu(z)
        agg = np.zeros((g.n, HID))
        np.add.at(agg, g.src, s)
        a = r(agg / np.maximum(g.deg, 1.0)[:, None])
        ha = np.concatenate([h, a], axis=1)
        hn = r(h + ha @ P[f"Wu{l}"].T + P[f"bu{l}"])
        cache["layers"].append({"h": h, "z": z, "ha": ha})
        h = hn
    y = h @ P["Wd"].T + P["bd"]
    cache["hL"] = h
    return y, cache


def loss_and_grad_y(y, t):
    """Mean squared difference of the mean-removed output and target, and its
    gradient with respect to y."""
    d = (y - y.mean(axis=0)) - (t - t.mean(axis=0))
    n = y.shape[0] * y.shape[1]
    L = float(np.sum(d * d) / n)
    gy = 2.0 * d / n
    gy = gy - gy.mean(axis=0)
    return L, gy


def backward(p, cache, gy, g: Graph):
    """Gradients of sum(gy * y) with respect to every parameter (the rounding
    of the forward pass is treated as identity)."""
    P = cache["P"]
    G = {}
    h = cache["hL"]
    G["Wd"] = gy.T @ h
    G["bd"] = gy.sum(axis=0)
    gh = gy @ P["Wd"]
    for l in reversed(range(N_LAYERS)):
        L = cache["layers"][l]
        G[f"Wu{l}"] = gh.T @ L["ha"]
        G[f"bu{l}"] = gh.sum(axis=0)
        gha = gh @ P[f"Wu{l}"]
        gh_prev = gh + gha[:, :HID]
        ga = gha[:, HID:]
        gz = (ga / np.maximum(g.deg, 1.0)[:, None])[g.src] * dsilu(L["z"])
        gA = np.zeros((g.n, HID))
        gB = np.zeros((g.n, HID))
        np.add.at(gA, g.src, gz)
        np.add.at(gB, g.dst, gz)
        G[f"We{l}"] = gz.T @ g.evec
        G[f"c{l}"] = gz.sum(axis=0)
        G[f"Wa{l}"] = gA.T @ L["h"]
        G[f"Wb{l}"] = gB.T @ L["h"]
        gh = gh_prev + gA @ P[f"Wa{l}"] + gB @ P[f"Wb{l}"]
    gpre = gh * dsilu(cache["pre0"])
    G["W0"] = gpre.T @ cache["X"]
    G["b0"] = gpre.sum(axis=0)
    return G


def increment(y, sm, lambda100, hbar, p0):
    """Displacement increment d from the network output, zero at the pinned
    node."""
    return (lambda100 * hbar * sm) * (y - y[p0])


def start_scale(r0, Kd):
    """Step length along d minimising the residual 2-norm |r0 - s K d|:
    s = (K d).r0 / (K d).(K d) (0 if K d vanishes)."""
    den = float(np.sum(Kd * Kd))
    return float(np.sum(Kd * r0)) / den if den > 0 else 0.0


def start_scale2(r0, Kd, Ke):
    """Coefficients (a, c) minimising |r0 - a K d - c K e| (normal equations
    of the 2-column least-squares problem).  When K d and K e are nearly
    parallel (determinant below 1e-10 of the diagonal product) the one of the
    two single-direction steps that lowers the residual more is taken."""
    dd, de, ee = float(np.sum(Kd * Kd)), float(np.sum(Kd * Ke)), float(np.sum(Ke * Ke))
    dr, er = float(np.sum(Kd * r0)), float(np.sum(Ke * r0))
    det = dd * ee - de * de
    if dd > 0 and ee > 0 and det > 1e-10 * dd * ee:
        return (dr * ee - er * de) / det, (er * dd - dr * de) / det
    gain_d = dr * dr / dd if dd > 0 else 0.0
    gain_e = er * er / ee if ee > 0 else 0.0
    if gain_d >= gain_e:
        return (dr / dd if dd > 0 else 0.0), 0.0
    return 0.0, er / ee


def adam(vec, grad, m1, m2, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba, Algorithm 1) on flat FP64 arrays; t >= 1."""
    m1 = beta1 * m1 + (1 - beta1) * grad
    m2 = beta2 * m2 + (1 - beta2) * grad * grad
    mh = m1 / (1 - beta1 ** t)
    vh = m2 / (1 - beta2 ** t)
    return vec - lr * mh / (np.sqrt(vh) + eps), m1, m2
