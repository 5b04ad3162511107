"""Pins of the learned-warm-start oracle (CPU).

The network itself is a reading (the paper is silent on it), so its pins fix
what the reading defines: the graph of a Kuhn lattice (14 neighbours along
the 7 lattice directions), BF16 rounding against torch's conversion and hand
values, mean aggregation and the i/j roles against a per-edge brute force,
equivariance under node relabelling, the backward pass against central
differences, the residual-minimising start steps against dense least squares, and Adam's first step
against its closed form."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as w
from oracle import mpnn_oracle as N


def _graph(n=5, seed=301, shuffle=False, jitter=0.15, sphere=0.0):
    case = w.small_cube(n, seed=seed, L=4e-8, jitter=jitter, sphere=sphere, shuffle=shuffle)
    orc = O.Oracle.from_mesh(case.mesh)
    return case, orc, N.Graph.from_oracle(orc, case.mesh)


def _params(seed=0, scale=1.0):
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in N.param_shapes():
        fan_in = shp[1] if len(shp) == 2 else 8
        p[name] = rng.standard_normal(shp) * scale / np.sqrt(fan_in)
    return p


def test_bf16_round_matches_torch_and_hand_values():
    assert N.bf16_round(1.0 + 2.0 ** -8) == 1.0                      # tie -> even
    assert N.bf16_round(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6      # tie -> even (upwards)
    assert N.bf16_round(1.0 + 2.0 ** -7) == 1.0 + 2.0 ** -7          # representable
    assert N.bf16_round(-3.0) == -3.0
    rng = np.random.default_rng(1)
    v = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.uniform(-30, 30, 20000),
                        [0.0, -0.0, 1e-40, -1e-39, 3.4e38, np.inf, -np.inf]]).astype(np.float32)
    ref = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    got = N.bf16_round(v)
    assert np.array_equal(got, ref)


def test_kuhn_graph_has_fourteen_lattice_neighbours():
    n = 6
    case, orc, g = _graph(n, jitter=0.0)
    assert g.n == (n - 1) ** 3
    assert np.all(g.deg == 14) and g.src.size == 14 * g.n
    dirs = {tuple(v) for v in np.round(g.evec).astype(int)}
    base = {(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, 0, 1), (0, 1, 1), (1, 1, 1)}
    assert dirs == base | {tuple(-np.array(d)) for d in base}
    assert np.allclose(g.evec, np.round(g.evec), atol=1e-9)           # hbar is the lattice spacing
    # symmetric: (i, j) present iff (j, i) present
    fwd = set(zip(g.src.tolist(), g.dst.tolist()))
    assert all((j, i) in fwd for i, j in fwd)


def test_features_scale_and_tag():
    case, orc, g = _graph(5, sphere=0.3)
    wts = orc.lumped_weights()
    m = np.zeros((g.n, 3)); m[:, 0] = 1.0
    v = np.array([0.003, -0.004, 0.0])
    x, sm = N.features(m, m - v, wts)
    mag = wts > 0
    assert np.isclose(sm, 0.005)
    assert np.allclose(x[mag, 0:3], v / 0.005) and np.allclose(x[mag, 3:6], m[mag])
    assert np.array_equal(x[:, 6], mag.astype(float))
    assert (~mag).any() and np.all(x[~mag] == 0.0)          # inputs vanish off the magnetic nodes
    x0, sm0 = N.features(m, m, wts)
    assert sm0 == 0 and np.all(x0[:, 0:3] == 0)


def test_layer_against_per_edge_brute_force():
    """One layer written as explicit loops over nodes and their neighbour
    lists on a tiny graph; checks mean (not sum) aggregation and that Wa acts
    on the receiving node and Wb on the sending neighbour."""
    case, orc, g = _graph(4, seed=302, sphere=0.3)
    rng = np.random.default_rng(3)
    p = _params(4)
    x = rng.standard_normal((g.n, N.F_IN))
    y, cache = N.forward(p, x, g)
    h = cache["layers"][0]["h"]
    nbrs = {i: [] for i in range(g.n)}
    for s, d, e in zip(g.src, g.dst, g.evec):
        nbrs[int(s)].append((int(d), e))
    h1 = np.zeros_like(h)
    for i in range(g.n):
        acc = np.zeros(N.HID)
        for j, e in nbrs[i]:
            z = p["Wa0"] @ h[i] + p["Wb0"] @ h[j] + p["We0"] @ e + p["c0"]
            acc += z / (1.0 + np.exp(-z))
        a = acc / len(nbrs[i])
        h1[i] = h[i] + p["Wu0"] @ np.concatenate([h[i], a]) + p["bu0"]
    assert np.allclose(cache["layers"][1]["h"], h1, rtol=1e-12, atol=1e-12)


def test_equivariant_under_node_relabelling():
    case_a, orc_a, ga = _graph(5, seed=303, sphere=0.3)
    case_b, orc_b, gb = _graph(5, seed=303, sphere=0.3, shuffle=True)
    # the same physical nodes: match by coordinates
    def coords(orc, case):
        c = np.zeros((orc.n, 3)); c[orc.node_map()] = case.mesh.xyz
        return c
    ca, cb = coords(orc_a, case_a), coords(orc_b, case_b)
    key = lambda c: np.round(np.mod(c, 4e-8) / 4e-8 * 1e6).astype(np.int64) % 1000000   # periodic copies agree
    ia = {tuple(k): i for i, k in enumerate(key(ca))}
    perm = np.array([ia[tuple(k)] for k in key(cb)])              # b index -> a index
    rng = np.random.default_rng(5)
    x = rng.standard_normal((ga.n, N.F_IN))
    p = _params(6)
    ya, _ = N.forward(p, x, ga)
    yb, _ = N.forward(p, x[perm], gb)
    assert np.allclose(yb, ya[perm], rtol=1e-10, atol=1e-12)


def test_backward_matches_central_differences():
    case, orc, g = _graph(4, seed=304, sphere=0.3)
    rng = np.random.default_rng(7)
    p = _params(8, scale=0.7)
    x = rng.standard_normal((g.n, N.F_IN))
    t = rng.standard_normal((g.n, 3))
    y, cache = N.forward(p, x, g)
    L, gy = N.loss_and_grad_y(y, t)
    G = N.backward(p, cache, gy, g)
    for name, shp in N.param_shapes():
        idx = [tuple(rng.integers(0, s) for s in shp) for _ in range(4)]
        for ix in idx:
            q = {k: v.copy() for k, v in p.items()}
            hstep = 1e-6 * max(1.0, abs(p[name][ix]))
            q[name][ix] = p[name][ix] + hstep
            Lp, _ = N.loss_and_grad_y(N.forward(q, x, g)[0], t)
            q[name][ix] = p[name][ix] - hstep
            Lm, _ = N.loss_and_grad_y(N.forward(q, x, g)[0], t)
            fd = (Lp - Lm) / (2 * hstep)
            # central differences carry ~1e-10 of rounding noise at this step
            assert abs(G[name][ix] - fd) <= 1e-5 * abs(fd) + 1e-9, (name, ix, G[name][ix], fd)


def test_loss_ignores_constant_offsets():
    rng = np.random.default_rng(9)
    y, t = rng.standard_normal((50, 3)), rng.standard_normal((50, 3))
    L1, g1 = N.loss_and_grad_y(y, t)
    L2, g2 = N.loss_and_grad_y(y + np.array([1.0, -2.0, 3.0]), t - 5.0)
    assert np.isclose(L1, L2) and np.allclose(g1, g2)
    assert np.allclose(g1.sum(axis=0), 0.0, atol=1e-14)


def test_start_step_minimises_the_residual():
    rng = np.random.default_rng(10)
    Q = rng.standard_normal((40, 40))
    K = Q @ Q.T + 40 * np.eye(40)
    b = rng.standard_normal(40)
    xs = np.linalg.solve(K, b)
    u = xs + 0.3 * rng.standard_normal(40)
    d = (xs - u) + 0.2 * rng.standard_normal(40)
    r0 = b - K @ u
    s = N.start_scale(r0, K @ d)
    res = lambda v: np.linalg.norm(b - K @ v)
    grid = np.linspace(s - 1, s + 1, 2001)
    assert res(u + s * d) <= min(res(u + q * d) for q in grid) + 1e-12
    assert res(u + s * d) <= res(u)
    assert N.start_scale(r0, np.zeros(40)) == 0.0


def test_two_direction_start_is_the_least_squares_residual():
    rng = np.random.default_rng(14)
    Q = rng.standard_normal((50, 50))
    K = Q @ Q.T + 50 * np.eye(50)
    b = rng.standard_normal(50)
    xs = np.linalg.solve(K, b)
    u = xs + 0.3 * rng.standard_normal(50)
    d = (xs - u) + 0.3 * rng.standard_normal(50)
    e = 0.5 * (xs - u) + 0.3 * rng.standard_normal(50)
    r0 = b - K @ u
    a, c = N.start_scale2(r0, K @ d, K @ e)
    # least squares on span{K d, K e}, by a dense solver
    coef, *_ = np.linalg.lstsq(np.stack([K @ d, K @ e], axis=1), r0, rcond=None)
    assert np.allclose([a, c], coef, rtol=1e-10)
    res = lambda v: np.linalg.norm(b - K @ v)
    assert res(u + a * d + c * e) <= min(res(u), res(u + N.start_scale(r0, K @ d) * d)) + 1e-12
    # parallel directions fall back to one step
    a2, c2 = N.start_scale2(r0, K @ d, 2 * (K @ d))
    assert np.isclose(a2 + 2 * c2, N.start_scale(r0, K @ d))


def test_increment_zero_at_pinned_node():
    rng = np.random.default_rng(11)
    y = rng.standard_normal((30, 3))
    d = N.increment(y, 0.01, 2e-4, 4e-9, 7)
    assert np.all(d[7] == 0)
    assert np.allclose(d[3], 0.01 * 2e-4 * 4e-9 * (y[3] - y[7]))


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(12)
    v, gr = rng.standard_normal(100), rng.standard_normal(100)
    out, m1, m2 = N.adam(v, gr, np.zeros(100), np.zeros(100), 1, 1e-3)
    assert np.allclose(out, v - 1e-3 * gr / (np.abs(gr) + 1e-8), rtol=1e-12, atol=1e-15)
    assert np.allclose(m1, 0.1 * gr) and np.allclose(m2, 0.001 * gr * gr)
    # constant gradient: every bias-corrected step is lr * g / (|g| + eps)
    m1 = m2 = np.zeros(100)
    x = v
    for t in range(1, 6):
        x2, m1, m2 = N.adam(x, gr, m1, m2, t, 1e-3)
        assert np.allclose(x - x2, 1e-3 * gr / (np.abs(gr) + 1e-8), rtol=1e-9)
        x = x2


def test_param_layout_round_trip():
    p = _params(13)
    vec = N.pack(p)
    assert vec.size == N.param_count() == 50819
    q = N.unpack(vec)
    assert all(np.array_equal(p[k], q[k]) for k in p)
