"""Python binding of the C ABI in include/gspm.h (argument marshalling only).

Every function here has the name of the C entry point it calls and does no
arithmetic of its own; all numerical work runs in libgspm.so's HIP kernels.
The library must be built (paper_2510_09812_amd.build) -- a missing library
is an error, never a fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgspm.so")

GSPM_OK, GSPM_E_ARG, GSPM_E_MESH, GSPM_E_STATE, GSPM_E_DEVICE, GSPM_E_NOCONV, GSPM_E_NONFINITE, GSPM_E_OOM = \
    0, -1, -2, -3, -4, -5, -6, -7
GSPM_FP64, GSPM_MIXED = 0, 1
GSPM_FIELD_M, GSPM_FIELD_U, GSPM_FIELD_UD = 0, 1, 2
GSPM_OP_LAPLACE, GSPM_OP_MASS, GSPM_OP_GS, GSPM_OP_ELASTIC, GSPM_OP_MS, GSPM_OP_PRECOND = 0, 1, 2, 3, 4, 5
GSPM_PRECOND_NONE, GSPM_PRECOND_GREEN, GSPM_PRECOND_JACOBI = 0, 1, 2
GSPM_PERIODIC = 1
GSPM_WARM_PREVIOUS, GSPM_WARM_LEARNED, GSPM_WARM_EXTRAPOLATE = 0, 1, 2
GSPM_GS_START_LUMPED, GSPM_GS_START_CORRECTED = 0, 1
GSPM_SWEEP_STOP_ON_REVERSAL, GSPM_SWEEP_CONTINUE = 1, 2
GSPM_REORDER_MORTON, GSPM_REORDER_NONE, GSPM_REORDER_RCM = 0, 1, 2
GSPM_MPNN_PARAMS = 50819

STATUS_NAMES = {0: "GSPM_OK", -1: "GSPM_E_ARG", -2: "GSPM_E_MESH", -3: "GSPM_E_STATE", -4: "GSPM_E_DEVICE",
                -5: "GSPM_E_NOCONV", -6: "GSPM_E_NONFINITE", -7: "GSPM_E_OOM"}

EXPORTS = ("gspm_create", "gspm_destroy", "gspm_upload_mesh", "gspm_set_params", "gspm_set_field",
           "gspm_get_field", "gspm_step", "gspm_energies", "gspm_averages", "gspm_apply", "gspm_solve",
           "gspm_mesh_info", "gspm_demag_factors", "gspm_time_operator", "gspm_last_error",
           "gspm_set_warm_start", "gspm_mpnn_set_params", "gspm_mpnn_get_params", "gspm_mpnn_forward",
           "gspm_mpnn_train_step", "gspm_mpnn_warm_start", "gspm_set_profile", "gspm_relax", "gspm_sweep",
           "gspm_demag_local_energy", "gspm_averages_noalloc", "gspm_set_gs_start")


class GspmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


DEV_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
DEV_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class gspm_create_opts(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("precision", ctypes.c_int32), ("block_nodes", ctypes.c_int32),
                ("profile", ctypes.c_int32), ("stream", ctypes.c_void_p), ("reorder", ctypes.c_int32),
                ("dev_alloc", DEV_ALLOC_FN), ("dev_free", DEV_FREE_FN), ("alloc_user", ctypes.c_void_p),
                ("deterministic", ctypes.c_int32)]


class gspm_params(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in
                ("Ms", "A", "K1", "lambda100", "lambda111", "c11", "c12", "c44", "alpha", "mu0", "gamma0")] + [
        ("Nd", ctypes.c_double * 9), ("hext", ctypes.c_double * 3), ("sigma_ext", ctypes.c_double * 6),
        ("cg_tol", ctypes.c_double), ("cg_maxit", ctypes.c_int32), ("precession", ctypes.c_int32),
        ("local_demag", ctypes.c_int32), ("crystal_rot", ctypes.c_double * 9), ("elastic_precond", ctypes.c_int32),
        ("gs_precond", ctypes.c_int32), ("ms_tol", ctypes.c_double)]


class gspm_step_stats(ctypes.Structure):
    _fields_ = [("steps_done", ctypes.c_int32), ("failed_step", ctypes.c_int32), ("mech_iters", ctypes.c_int64),
                ("gs_iters", ctypes.c_int64), ("gs_iters_stage", ctypes.c_int64 * 8), ("dm_avg", ctypes.c_double),
                ("elapsed_ms", ctypes.c_double), ("matvec_ms", ctypes.c_double),
                ("matvec_launches", ctypes.c_int64), ("refinements", ctypes.c_int64),
                ("learned_starts", ctypes.c_int64), ("minres_starts", ctypes.c_int64),
                ("warm_coef", ctypes.c_double * 2), ("ms_iters", ctypes.c_int64),
                ("mech_refinements", ctypes.c_int64), ("gs_matvec_ms", ctypes.c_double),
                ("gs_matvec_launches", ctypes.c_int64), ("phase_ms", ctypes.c_double * 8),
                ("final_residual", ctypes.c_double * 5)]

PHASES = ("averages", "elastic", "magnetostatic", "gs_stage1", "gs_stage2", "averages_mstar", "gs_stage3",
          "projection")
RESIDUAL_SOLVES = ("elastic", "gs_stage1", "gs_stage2", "gs_stage3", "magnetostatic")


_lib = None


def load() -> ctypes.CDLL:
    """Load libgspm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FileNotFoundError(f"{LIB_PATH} is missing: run paper_2510_09812_amd.build.build() first")
    lib = ctypes.CDLL(LIB_PATH)
    P, dp, i64 = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int64
    S = ctypes.c_int
    lib.gspm_create.argtypes = [ctypes.POINTER(P), ctypes.POINTER(gspm_create_opts)]; lib.gspm_create.restype = S
    lib.gspm_destroy.argtypes = [P]; lib.gspm_destroy.restype = None
    lib.gspm_upload_mesh.argtypes = [P, i64, dp, i64, P, P, dp, dp, ctypes.c_uint32]; lib.gspm_upload_mesh.restype = S
    lib.gspm_set_params.argtypes = [P, ctypes.POINTER(gspm_params)]; lib.gspm_set_params.restype = S
    lib.gspm_set_field.argtypes = [P, ctypes.c_int, dp, i64]; lib.gspm_set_field.restype = S
    lib.gspm_get_field.argtypes = [P, ctypes.c_int, dp, i64]; lib.gspm_get_field.restype = S
    lib.gspm_step.argtypes = [P, ctypes.c_double, ctypes.c_int32, ctypes.POINTER(gspm_step_stats)]
    lib.gspm_step.restype = S
    lib.gspm_relax.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.POINTER(gspm_step_stats)]
    lib.gspm_relax.restype = S
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.gspm_sweep.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_int32, dp, dp,
                               ctypes.c_uint32, dp, i32p, i32p, i32p]
    lib.gspm_sweep.restype = S
    lib.gspm_energies.argtypes = [P, dp]; lib.gspm_energies.restype = S
    lib.gspm_demag_local_energy.argtypes = [P, dp]; lib.gspm_demag_local_energy.restype = S
    lib.gspm_averages.argtypes = [P, dp, dp]; lib.gspm_averages.restype = S
    lib.gspm_averages_noalloc.argtypes = [P, P, P]; lib.gspm_averages_noalloc.restype = S
    lib.gspm_apply.argtypes = [P, ctypes.c_int, ctypes.c_double, dp, dp, i64]; lib.gspm_apply.restype = S
    lib.gspm_solve.argtypes = [P, ctypes.c_int, ctypes.c_double, dp, dp, i64, ctypes.c_double, ctypes.c_int32,
                               ctypes.POINTER(ctypes.c_int32)]
    lib.gspm_solve.restype = S
    lib.gspm_mesh_info.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64),
                                   ctypes.POINTER(i64), dp]
    lib.gspm_mesh_info.restype = S
    lib.gspm_demag_factors.argtypes = [ctypes.c_double] * 3 + [dp]; lib.gspm_demag_factors.restype = S
    lib.gspm_time_operator.argtypes = [P, ctypes.c_int, ctypes.c_double, ctypes.c_int32, dp]
    lib.gspm_time_operator.restype = S
    lib.gspm_last_error.argtypes = [P]; lib.gspm_last_error.restype = ctypes.c_char_p
    fp = ctypes.POINTER(ctypes.c_float)
    lib.gspm_set_warm_start.argtypes = [P, ctypes.c_int32]; lib.gspm_set_warm_start.restype = S
    lib.gspm_set_gs_start.argtypes = [P, ctypes.c_int32]; lib.gspm_set_gs_start.restype = S
    lib.gspm_set_profile.argtypes = [P, ctypes.c_int32]; lib.gspm_set_profile.restype = S
    lib.gspm_mpnn_set_params.argtypes = [P, fp, i64]; lib.gspm_mpnn_set_params.restype = S
    lib.gspm_mpnn_get_params.argtypes = [P, fp, i64]; lib.gspm_mpnn_get_params.restype = S
    lib.gspm_mpnn_forward.argtypes = [P, dp, dp, i64, dp, dp]; lib.gspm_mpnn_forward.restype = S
    lib.gspm_mpnn_train_step.argtypes = [P, dp, dp, dp, i64, ctypes.c_float, ctypes.c_int32, dp, fp]
    lib.gspm_mpnn_train_step.restype = S
    lib.gspm_mpnn_warm_start.argtypes = [P, dp, dp, i64, dp, dp]; lib.gspm_mpnn_warm_start.restype = S
    _lib = lib
    return lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a, shape=None) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a.reshape(shape) if shape is not None else a


def _check(ctx, status: int):
    if status != GSPM_OK:
        raise GspmError(status, gspm_last_error(ctx))


def gspm_last_error(ctx) -> str:
    return load().gspm_last_error(ctx).decode()


def torch_allocator(device: int = 0):
    """A (dev_alloc, dev_free) pair of C callbacks that take the context's
    device memory from PyTorch's caching allocator on `device` (keep the pair
    alive as long as the context)."""
    import torch

    def alloc(nbytes, _user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device)
        except Exception:
            return None

    def free(ptr, _user):
        torch.cuda.caching_allocator_delete(ptr)

    return DEV_ALLOC_FN(alloc), DEV_FREE_FN(free)


def gspm_create(device: int = 0, precision: int = GSPM_FP64, block_nodes: int = 0, profile: bool = False,
                stream=None, reorder: int = GSPM_REORDER_MORTON, allocator=None, deterministic: bool = False):
    """Returns an opaque context handle.  `stream` may be a torch.cuda.Stream
    (the library then runs on it) or a raw hipStream_t integer; `allocator` a
    (dev_alloc, dev_free) pair of C callbacks (see torch_allocator), which the
    caller keeps alive as long as the context."""
    opts = gspm_create_opts(device, precision, block_nodes, 1 if profile else 0, None, reorder)
    opts.deterministic = 1 if deterministic else 0
    if stream is not None:
        opts.stream = ctypes.c_void_p(int(getattr(stream, "cuda_stream", stream)))
    if allocator is not None:
        opts.dev_alloc, opts.dev_free = allocator
    h = ctypes.c_void_p()
    _check(None, load().gspm_create(ctypes.byref(h), ctypes.byref(opts)))
    return h


def gspm_destroy(ctx) -> None:
    if ctx is not None and ctx.value:
        load().gspm_destroy(ctx)


def gspm_upload_mesh(ctx, xyz, tets, tags, lo, hi, flags: int = GSPM_PERIODIC) -> None:
    xyz = _f64(xyz, (-1, 3))
    tets = np.ascontiguousarray(tets, dtype=np.int32).reshape(-1, 4)
    tags = np.ascontiguousarray(tags, dtype=np.uint8).reshape(-1)
    if tags.shape[0] != tets.shape[0]:
        raise ValueError("one tag per tetrahedron")
    _check(ctx, load().gspm_upload_mesh(ctx, xyz.shape[0], _dp(xyz), tets.shape[0], tets.ctypes.data,
                                        tags.ctypes.data, _dp(_f64(lo)), _dp(_f64(hi)), flags))


def make_params(params: dict, hext=(0.0, 0.0, 0.0), sigma_ext=(0.0,) * 6, precession: bool = True,
                cg_maxit: int = 10000, local_demag: bool = False) -> gspm_params:
    p = gspm_params()
    for k in ("Ms", "A", "K1", "lambda100", "lambda111", "c11", "c12", "c44", "alpha", "mu0", "gamma0"):
        setattr(p, k, float(params[k]))
    nd = np.asarray(params.get("Nd", np.eye(3) / 3.0), dtype=np.float64).reshape(9)
    for i in range(9):
        p.Nd[i] = nd[i]
    for i in range(3):
        p.hext[i] = float(hext[i])
    for i in range(6):
        p.sigma_ext[i] = float(sigma_ext[i])
    p.cg_tol = float(params.get("cg_tol", 1e-8))
    p.cg_maxit = int(params.get("cg_maxit", cg_maxit))
    p.precession = 1 if precession else 0
    p.local_demag = 1 if local_demag else 0
    rot = np.asarray(params.get("crystal_rot", np.eye(3)), dtype=np.float64).reshape(9)
    for i in range(9):
        p.crystal_rot[i] = rot[i]
    p.elastic_precond = int(params.get("elastic_precond", GSPM_PRECOND_NONE))
    p.gs_precond = int(params.get("gs_precond", GSPM_PRECOND_NONE))
    p.ms_tol = float(params.get("ms_tol", 0.0))
    return p


def gspm_set_params(ctx, params) -> None:
    if isinstance(params, dict):
        params = make_params(params)
    _check(ctx, load().gspm_set_params(ctx, ctypes.byref(params)))


def gspm_set_field(ctx, which: int, values) -> None:
    v = _f64(values, (-1,) if which == GSPM_FIELD_UD else (-1, 3))
    _check(ctx, load().gspm_set_field(ctx, which, _dp(v), v.shape[0]))


def gspm_get_field(ctx, which: int, n_nodes: int) -> np.ndarray:
    out = np.zeros(n_nodes if which == GSPM_FIELD_UD else (n_nodes, 3))
    _check(ctx, load().gspm_get_field(ctx, which, _dp(out), n_nodes))
    return out


def stats_dict(st: gspm_step_stats) -> dict:
    return dict(steps_done=st.steps_done, failed_step=st.failed_step, mech_iters=st.mech_iters,
                gs_iters=st.gs_iters, gs_iters_stage=list(st.gs_iters_stage), dm_avg=st.dm_avg,
                elapsed_ms=st.elapsed_ms, matvec_ms=st.matvec_ms, matvec_launches=st.matvec_launches,
                refinements=st.refinements, learned_starts=st.learned_starts, minres_starts=st.minres_starts,
                warm_coef=list(st.warm_coef), ms_iters=st.ms_iters, mech_refinements=st.mech_refinements,
                gs_matvec_ms=st.gs_matvec_ms, gs_matvec_launches=st.gs_matvec_launches,
                phase_ms=dict(zip(PHASES, st.phase_ms)), final_residual=dict(zip(RESIDUAL_SOLVES, st.final_residual)))


def gspm_step(ctx, dt: float, n_steps: int = 1) -> dict:
    """Runs n steps; returns the stats as a dict.  On failure the GspmError
    carries the stats in its `stats` attribute."""
    st = gspm_step_stats()
    status = load().gspm_step(ctx, dt, n_steps, ctypes.byref(st))
    if status != GSPM_OK:
        err = GspmError(status, gspm_last_error(ctx))
        err.stats = stats_dict(st)
        raise err
    return stats_dict(st)


def gspm_relax(ctx, dt: float, dm_tol: float, max_steps: int) -> dict:
    """Steps until <|dm|> < dm_tol; returns the summed stats.  On failure
    (GSPM_E_NOCONV after max_steps included) the GspmError carries them in
    its `stats` attribute."""
    st = gspm_step_stats()
    status = load().gspm_relax(ctx, dt, dm_tol, max_steps, ctypes.byref(st))
    if status != GSPM_OK:
        err = GspmError(status, gspm_last_error(ctx))
        err.stats = stats_dict(st)
        raise err
    return stats_dict(st)


def gspm_sweep(ctx, dt: float, dm_tol: float, max_steps: int, hext, sigma_ext=None,
               stop_on_reversal: bool = False, keep_going: bool = False) -> dict:
    """Relaxes at each applied field (n x 3) and stress (n x 6, or None);
    returns mbar (points done x 3), steps and converged (per point) and
    points_done.  keep_going sets GSPM_SWEEP_CONTINUE.  On failure the
    GspmError carries them in its `sweep` attribute."""
    h = _f64(hext, (-1, 3))
    n = h.shape[0]
    sg = None if sigma_ext is None else _f64(sigma_ext, (n, 6))
    mbar = np.zeros((n, 3))
    steps = np.zeros(n, dtype=np.int32)
    conv = np.zeros(n, dtype=np.int32)
    done = ctypes.c_int32(0)
    flags = (GSPM_SWEEP_STOP_ON_REVERSAL if stop_on_reversal else 0) | (GSPM_SWEEP_CONTINUE if keep_going else 0)
    i32p = ctypes.POINTER(ctypes.c_int32)
    status = load().gspm_sweep(ctx, dt, dm_tol, max_steps, n, _dp(h), None if sg is None else _dp(sg), flags,
                               _dp(mbar), steps.ctypes.data_as(i32p), conv.ctypes.data_as(i32p), ctypes.byref(done))
    k = done.value
    # a failing point has its steps filled but no mbar
    ns = k + 1 if status != GSPM_OK and k < n else k
    out = dict(mbar=mbar[:k].copy(), steps=steps[:ns].copy(), converged=conv[:ns].astype(bool), points_done=k)
    if status != GSPM_OK:
        err = GspmError(status, gspm_last_error(ctx))
        err.sweep = out
        raise err
    return out


ENERGY_KEYS = ("exchange", "anisotropy", "zeeman", "magnetoelastic", "stress", "demag_far", "total")


def gspm_energies(ctx) -> dict:
    out = np.zeros(7)
    _check(ctx, load().gspm_energies(ctx, _dp(out)))
    return dict(zip(ENERGY_KEYS, out.tolist()))


def gspm_demag_local_energy(ctx) -> float:
    out = np.zeros(1)
    _check(ctx, load().gspm_demag_local_energy(ctx, _dp(out)))
    return float(out[0])


def gspm_averages(ctx):
    mbar = np.zeros(3); ebar = np.zeros(6)
    _check(ctx, load().gspm_averages(ctx, _dp(mbar), _dp(ebar)))
    return mbar, ebar


def gspm_averages_noalloc(ctx, m_dev_ptr: int, out_dev_ptr: int) -> None:
    """Device pointers in, nothing allocated: m (n_nodes x 3 doubles, caller
    order) and out (9 doubles: mbar, ebar), both device addresses (for
    example torch tensors' data_ptr()).  Asynchronous on the context's
    stream."""
    _check(ctx, load().gspm_averages_noalloc(ctx, ctypes.c_void_p(m_dev_ptr), ctypes.c_void_p(out_dev_ptr)))


def gspm_apply(ctx, op: int, x, eps: float = 0.0) -> np.ndarray:
    x = _f64(x, (-1, 3)); y = np.zeros_like(x)
    _check(ctx, load().gspm_apply(ctx, op, eps, _dp(x), _dp(y), x.shape[0]))
    return y


def gspm_solve(ctx, op: int, b, x0=None, eps: float = 0.0, tol: float = 1e-8, maxit: int = 100000):
    b = _f64(b, (-1, 3))
    x = np.zeros_like(b) if x0 is None else _f64(x0, (-1, 3)).copy()
    it = ctypes.c_int32(0)
    _check(ctx, load().gspm_solve(ctx, op, eps, _dp(b), _dp(x), b.shape[0], tol, maxit, ctypes.byref(it)))
    return x, int(it.value)


def gspm_mesh_info(ctx) -> dict:
    a, b, c, d = (ctypes.c_int64() for _ in range(4))
    v = np.zeros(1)
    _check(ctx, load().gspm_mesh_info(ctx, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d),
                                      _dp(v)))
    return dict(n_unique=a.value, n_tets=b.value, n_blocks=c.value, n_elem_copies=d.value, volume=float(v[0]))


def gspm_time_operator(ctx, op: int, eps: float = 0.0, reps: int = 20) -> float:
    """Mean duration [ms] of one device-resident launch of operator `op`."""
    out = np.zeros(1)
    _check(ctx, load().gspm_time_operator(ctx, op, eps, reps, _dp(out)))
    return float(out[0])


def gspm_demag_factors(a: float, b: float, c: float) -> np.ndarray:
    out = np.zeros(3)
    _check(None, load().gspm_demag_factors(a, b, c, _dp(out)))
    return out


def _fp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _f32(a, n) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float32)
    if a.shape != (n,):
        raise ValueError(f"expected {n} parameters, got shape {a.shape}")
    return a


def gspm_set_profile(ctx, enable: bool) -> None:
    _check(ctx, load().gspm_set_profile(ctx, 1 if enable else 0))


def gspm_set_warm_start(ctx, mode: int) -> None:
    _check(ctx, load().gspm_set_warm_start(ctx, mode))


def gspm_set_gs_start(ctx, mode: int) -> None:
    _check(ctx, load().gspm_set_gs_start(ctx, mode))


def gspm_mpnn_set_params(ctx, params) -> None:
    p = _f32(params, GSPM_MPNN_PARAMS)
    _check(ctx, load().gspm_mpnn_set_params(ctx, _fp(p), p.size))


def gspm_mpnn_get_params(ctx) -> np.ndarray:
    out = np.zeros(GSPM_MPNN_PARAMS, dtype=np.float32)
    _check(ctx, load().gspm_mpnn_get_params(ctx, _fp(out), out.size))
    return out


def gspm_mpnn_forward(ctx, m_prev, m):
    """Network output (n_nodes x 3) and the increment scale s_m."""
    mp, mm = _f64(m_prev), _f64(m)
    n = mm.shape[0]
    y = np.zeros((n, 3))
    sm = np.zeros(1)
    _check(ctx, load().gspm_mpnn_forward(ctx, _dp(mp), _dp(mm), n, _dp(y), _dp(sm)))
    return y, float(sm[0])


def gspm_mpnn_train_step(ctx, m_prev, m, du, lr: float = 1e-3, update: bool = True, want_grad: bool = False):
    """One training step; returns (loss, gradient or None)."""
    mp, mm, dd = _f64(m_prev), _f64(m), _f64(du)
    n = mm.shape[0]
    loss = np.zeros(1)
    g = np.zeros(GSPM_MPNN_PARAMS, dtype=np.float32) if want_grad else None
    _check(ctx, load().gspm_mpnn_train_step(ctx, _dp(mp), _dp(mm), _dp(dd), n, lr, 1 if update else 0, _dp(loss),
                                            _fp(g) if g is not None else None))
    return float(loss[0]), g


def gspm_mpnn_warm_start(ctx, m_prev, u_prev=None):
    """The learned elastic start for the current state: (u0, (a, c))."""
    mp = _f64(m_prev)
    n = mp.shape[0]
    up = _f64(u_prev) if u_prev is not None else None
    u0 = np.zeros((n, 3))
    coef = np.zeros(2)
    _check(ctx, load().gspm_mpnn_warm_start(ctx, _dp(mp), _dp(up) if up is not None else None, n, _dp(u0),
                                            _dp(coef)))
    return u0, (float(coef[0]), float(coef[1]))


class Simulation:
    """Owns one context; thin convenience over the functions above."""

    def __init__(self, mesh, params: dict | None = None, hext=(0.0, 0.0, 0.0), sigma_ext=(0.0,) * 6,
                 precession: bool = True, local_demag: bool = False, **create_kw):
        self._allocator = create_kw.get("allocator")    # C callbacks must outlive the context
        self.ctx = gspm_create(**create_kw)
        self.n0 = int(np.asarray(mesh.xyz).shape[0])
        gspm_upload_mesh(self.ctx, mesh.xyz, mesh.tets, mesh.tags, mesh.lo, mesh.hi)
        if params is not None:
            self.set_params(params, hext, sigma_ext, precession, local_demag)

    def set_params(self, params: dict, hext=(0.0, 0.0, 0.0), sigma_ext=(0.0,) * 6, precession: bool = True,
                   local_demag: bool = False):
        gspm_set_params(self.ctx, make_params(params, hext, sigma_ext, precession, local_demag=local_demag))

    def set_m(self, m):
        gspm_set_field(self.ctx, GSPM_FIELD_M, m)

    def set_u(self, u):
        gspm_set_field(self.ctx, GSPM_FIELD_U, u)

    def get_m(self) -> np.ndarray:
        return gspm_get_field(self.ctx, GSPM_FIELD_M, self.n0)

    def get_u(self) -> np.ndarray:
        return gspm_get_field(self.ctx, GSPM_FIELD_U, self.n0)

    def set_ud(self, ud):
        gspm_set_field(self.ctx, GSPM_FIELD_UD, ud)

    def get_ud(self) -> np.ndarray:
        return gspm_get_field(self.ctx, GSPM_FIELD_UD, self.n0)

    def demag_local_energy(self) -> float:
        return gspm_demag_local_energy(self.ctx)

    def step(self, dt: float, n: int = 1) -> dict:
        return gspm_step(self.ctx, dt, n)

    def relax(self, dt: float, dm_tol: float, max_steps: int) -> dict:
        return gspm_relax(self.ctx, dt, dm_tol, max_steps)

    def sweep(self, dt: float, dm_tol: float, max_steps: int, hext, sigma_ext=None, stop_on_reversal=False,
              keep_going=False) -> dict:
        return gspm_sweep(self.ctx, dt, dm_tol, max_steps, hext, sigma_ext, stop_on_reversal, keep_going)

    def energies(self) -> dict:
        return gspm_energies(self.ctx)

    def averages(self):
        return gspm_averages(self.ctx)

    def apply(self, op: int, x, eps: float = 0.0) -> np.ndarray:
        return gspm_apply(self.ctx, op, x, eps)

    def solve(self, op: int, b, x0=None, eps: float = 0.0, tol: float = 1e-8, maxit: int = 100000):
        return gspm_solve(self.ctx, op, b, x0, eps, tol, maxit)

    def time_operator(self, op: int, eps: float = 0.0, reps: int = 20) -> float:
        return gspm_time_operator(self.ctx, op, eps, reps)

    def mesh_info(self) -> dict:
        return gspm_mesh_info(self.ctx)

    def set_profile(self, enable: bool):
        gspm_set_profile(self.ctx, enable)

    def set_warm_start(self, mode: int):
        gspm_set_warm_start(self.ctx, mode)

    def set_gs_start(self, mode: int):
        gspm_set_gs_start(self.ctx, mode)

    def mpnn_set_params(self, params):
        gspm_mpnn_set_params(self.ctx, params)

    def mpnn_get_params(self) -> np.ndarray:
        return gspm_mpnn_get_params(self.ctx)

    def mpnn_forward(self, m_prev, m):
        return gspm_mpnn_forward(self.ctx, m_prev, m)

    def mpnn_train_step(self, m_prev, m, du, lr: float = 1e-3, update: bool = True, want_grad: bool = False):
        return gspm_mpnn_train_step(self.ctx, m_prev, m, du, lr, update, want_grad)

    def mpnn_warm_start(self, m_prev, u_prev=None):
        return gspm_mpnn_warm_start(self.ctx, m_prev, u_prev)

    def close(self):
        gspm_destroy(getattr(self, "ctx", None))
        self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
