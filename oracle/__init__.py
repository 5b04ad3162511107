"""CPU FP64 oracle of the GSPM time step -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The product library (paper_2510_09812_amd) never
imports it and shares no code with it; the two meet only in the seeded inputs
of the `workloads` package.

The arithmetic lives in gspm_oracle.c (plain C, FP64, OpenMP loops); this
module only marshals arguments.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gspm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

OP_LAPLACE, OP_MASS, OP_GS, OP_ELASTIC, OP_LAPLACE_ALL, OP_MS = 0, 1, 2, 3, 4, 5
SOLVE_ELASTIC_JACOBI = 6
SOLVE_ELASTIC_GREEN = 7


_NATIVE_PATH = os.path.join(_HERE, "liboracle_native.so")


def build(native: bool = False) -> str:
    """Compile the oracle next to its source with plain gcc.  The default
    library (tests, smoke check) carries no target-specific flags, so it runs
    on any x86-64 host; native=True builds liboracle_native.so with
    -O3 -march=native for the CPU-baseline timing on the host that runs it."""
    path = _NATIVE_PATH if native else _LIB_PATH
    opt = ["-O3", "-march=native"] if native else ["-O2"]
    tmp = path + ".tmp"
    subprocess.check_call(["gcc"] + opt + ["-std=gnu11", "-fopenmp", "-fPIC", "-shared",
                           "-Wall", "-Wno-unused-function", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, path)
    return path


class _Params(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in
                ("Ms", "A", "K1", "lambda100", "lambda111", "c11", "c12", "c44", "alpha", "mu0", "gamma0")] + [
        ("Nd", ctypes.c_double * 9), ("hext", ctypes.c_double * 3), ("sigma_ext", ctypes.c_double * 6),
        ("cg_tol", ctypes.c_double), ("cg_maxit", ctypes.c_int32), ("precession", ctypes.c_int32),
        ("local_demag", ctypes.c_int32), ("crystal_rot", ctypes.c_double * 9), ("elastic_precond", ctypes.c_int32),
        ("gs_precond", ctypes.c_int32), ("ms_tol", ctypes.c_double)]


class _Stats(ctypes.Structure):
    _fields_ = [("steps_done", ctypes.c_int32), ("mech_iters", ctypes.c_int32),
                ("gs_iters", ctypes.c_int32 * 8), ("dm_avg", ctypes.c_double), ("ms_iters", ctypes.c_int32)]


_lib = None
_native = False


def select_native() -> str:
    """Use the -O3 -march=native build (compiled here, on this host) for every
    oracle created from now on in this process; only before the first load."""
    global _native
    if _lib is not None and not _native:
        raise RuntimeError("the portable oracle library is already loaded in this process")
    _native = True
    return build(native=True)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = _NATIVE_PATH if _native else _LIB_PATH
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
        build(native=_native)
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    lib.or_create.argtypes = [ctypes.POINTER(P), ctypes.c_int32, dp, ctypes.c_int32, P, P, dp, dp,
                              ctypes.c_int32, ctypes.c_char_p, ctypes.c_int32]
    lib.or_destroy.argtypes = [P]
    lib.or_n_unique.argtypes = [P]; lib.or_n_unique.restype = ctypes.c_int32
    lib.or_node_map.argtypes = [P, P]
    lib.or_geometry.argtypes = [P, dp, dp]
    lib.or_total_volume.argtypes = [P]; lib.or_total_volume.restype = ctypes.c_double
    lib.or_lumped_weights.argtypes = [P, dp]
    lib.or_pinned_node.argtypes = [P]; lib.or_pinned_node.restype = ctypes.c_int32
    lib.or_set_params.argtypes = [P, ctypes.POINTER(_Params)]
    lib.or_set_m.argtypes = [P, dp]; lib.or_set_u.argtypes = [P, dp]
    lib.or_get_m.argtypes = [P, dp]; lib.or_get_u.argtypes = [P, dp]
    lib.or_set_ud.argtypes = [P, dp]; lib.or_get_ud.argtypes = [P, dp]
    lib.or_demag_local_energy.argtypes = [P, dp]
    lib.or_ms_rhs_at.argtypes = [P, dp, dp]
    lib.or_ms_solve_at.argtypes = [P, dp, dp, ctypes.c_double, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    lib.or_ms_field.argtypes = [P, dp, dp]
    lib.or_ms_energy.argtypes = [P, dp, dp]
    lib.or_apply.argtypes = [P, ctypes.c_int32, ctypes.c_double, dp, dp]
    lib.or_solve.argtypes = [P, ctypes.c_int32, ctypes.c_double, dp, dp, ctypes.c_double, ctypes.c_int32,
                             ctypes.POINTER(ctypes.c_int32)]
    lib.or_step.argtypes = [P, ctypes.c_double, ctypes.c_int32, ctypes.POINTER(_Stats)]
    lib.or_energies.argtypes = [P, dp]
    lib.or_averages.argtypes = [P, dp, dp]
    lib.or_elastic_rhs.argtypes = [P, dp]
    lib.or_field_rhs.argtypes = [P, ctypes.c_double, dp, dp]
    lib.or_demag_factors.argtypes = [ctypes.c_double] * 3 + [dp]
    lib.or_h_local.argtypes = [ctypes.POINTER(_Params), dp, dp, dp, dp]
    lib.or_stiffness_voigt.argtypes = [ctypes.POINTER(_Params), dp]
    lib.or_spont_strain.argtypes = [ctypes.POINTER(_Params), dp, dp]
    lib.or_energy_density_local.argtypes = [ctypes.POINTER(_Params), dp, dp]
    lib.or_energy_density_local.restype = ctypes.c_double
    lib.or_last_error.argtypes = [P]; lib.or_last_error.restype = ctypes.c_char_p
    lib.or_num_threads.argtypes = []; lib.or_num_threads.restype = ctypes.c_int32
    lib.or_set_num_threads.argtypes = [ctypes.c_int32]
    lib.or_precond_apply.argtypes = [P, dp, dp]
    lib.or_precond_grid.argtypes = [P, P]
    lib.or_set_precond_omega.argtypes = [P, ctypes.c_double]
    _lib = lib
    return lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a, shape=None) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


class OracleError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"oracle error {code}: {msg}")
        self.code = code


def make_params(params: dict, hext=(0.0, 0.0, 0.0), sigma_ext=(0.0,) * 6, precession: bool = True,
                cg_maxit: int = 10000, local_demag: bool = False) -> _Params:
    """params may carry "crystal_rot" (3 x 3, v_sample = R v_crystal, App. D)
    "elastic_precond" (1: the Green's-operator preconditioned elastic
    solve) and "gs_precond" (2: Jacobi-preconditioned GS solves)."""
    p = _Params()
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
    p.elastic_precond = int(params.get("elastic_precond", 0))
    p.gs_precond = int(params.get("gs_precond", 0))
    p.ms_tol = float(params.get("ms_tol", 0.0))
    return p


def num_threads() -> int:
    return int(_load().or_num_threads())


def set_num_threads(k: int) -> None:
    _load().or_set_num_threads(int(k))


def demag_factors(a: float, b: float, c: float) -> np.ndarray:
    out = np.zeros(3)
    _load().or_demag_factors(a, b, c, _dp(out))
    return out


def h_local(params: dict, m, E6, mbar, hext=(0.0, 0.0, 0.0)) -> np.ndarray:
    p = make_params(params, hext)
    h = np.zeros(3)
    _load().or_h_local(ctypes.byref(p), _dp(_f64(m)), _dp(_f64(E6)), _dp(_f64(mbar)), _dp(h))
    return h


def stiffness_voigt(params: dict) -> np.ndarray:
    p = make_params(params)
    out = np.zeros(36)
    _load().or_stiffness_voigt(ctypes.byref(p), _dp(out))
    return out.reshape(6, 6)


def spont_strain(params: dict, m) -> np.ndarray:
    p = make_params(params)
    out = np.zeros(6)
    _load().or_spont_strain(ctypes.byref(p), _dp(_f64(m)), _dp(out))
    return out


def energy_density_local(params: dict, m, E6, hext=(0.0, 0.0, 0.0)) -> float:
    p = make_params(params, hext)
    return float(_load().or_energy_density_local(ctypes.byref(p), _dp(_f64(m)), _dp(_f64(E6))))


class Oracle:
    """One mesh plus state.  Field I/O is in the caller's node order (n0 x 3);
    operator and solver I/O is in the oracle's unique-node order (n x 3)."""

    def __init__(self, xyz, tets, tags, lo, hi, periodic: bool = True):
        lib = _load()
        self._lib = lib
        xyz = _f64(xyz, (-1, 3))
        self._tets = np.ascontiguousarray(tets, dtype=np.int32).reshape(-1, 4)
        self._tags = np.ascontiguousarray(tags, dtype=np.uint8)
        self.n0 = xyz.shape[0]
        self.ne = self._tets.shape[0]
        err = ctypes.create_string_buffer(256)
        h = ctypes.c_void_p()
        rc = lib.or_create(ctypes.byref(h), self.n0, _dp(xyz), self.ne, self._tets.ctypes.data,
                           self._tags.ctypes.data, _dp(_f64(lo)), _dp(_f64(hi)), 1 if periodic else 0, err, 256)
        if rc != 0:
            raise OracleError(rc, err.value.decode())
        self._h = h
        self.n = lib.or_n_unique(h)

    @classmethod
    def from_mesh(cls, mesh, periodic: bool = True) -> "Oracle":
        return cls(mesh.xyz, mesh.tets, mesh.tags, mesh.lo, mesh.hi, periodic)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.or_destroy(h)
            self._h = None

    def _check(self, rc):
        if rc != 0:
            raise OracleError(rc, self._lib.or_last_error(self._h).decode())

    # ---- mesh facts
    def node_map(self) -> np.ndarray:
        out = np.zeros(self.n0, dtype=np.int32)
        self._lib.or_node_map(self._h, out.ctypes.data)
        return out

    def geometry(self):
        vol = np.zeros(self.ne); grad = np.zeros((self.ne, 4, 3))
        self._lib.or_geometry(self._h, _dp(vol), _dp(grad))
        return vol, grad

    def total_volume(self) -> float:
        return float(self._lib.or_total_volume(self._h))

    def lumped_weights(self) -> np.ndarray:
        w = np.zeros(self.n)
        self._lib.or_lumped_weights(self._h, _dp(w))
        return w

    def pinned_node(self) -> int:
        return int(self._lib.or_pinned_node(self._h))

    # ---- state
    def set_params(self, params: dict, hext=(0.0, 0.0, 0.0), sigma_ext=(0.0,) * 6, precession=True,
                   local_demag=False):
        self._p = make_params(params, hext, sigma_ext, precession, local_demag=local_demag)
        self._check(self._lib.or_set_params(self._h, ctypes.byref(self._p)))

    def set_m(self, m):
        self._check(self._lib.or_set_m(self._h, _dp(_f64(m, (-1, 3)))))

    def set_u(self, u):
        self._check(self._lib.or_set_u(self._h, _dp(_f64(u, (-1, 3)))))

    def get_m(self) -> np.ndarray:
        out = np.zeros((self.n0, 3)); self._lib.or_get_m(self._h, _dp(out)); return out

    def get_u(self) -> np.ndarray:
        out = np.zeros((self.n0, 3)); self._lib.or_get_u(self._h, _dp(out)); return out

    def set_ud(self, ud):
        self._check(self._lib.or_set_ud(self._h, _dp(_f64(ud, (-1,)))))

    def get_ud(self) -> np.ndarray:
        out = np.zeros(self.n0); self._lib.or_get_ud(self._h, _dp(out)); return out

    def demag_local_energy(self) -> float:
        e = np.zeros(1); self._check(self._lib.or_demag_local_energy(self._h, _dp(e))); return float(e[0])

    # ---- local magnetostatics on explicit unique-order arrays (state untouched)
    def ms_rhs(self, m_unique) -> np.ndarray:
        b = np.zeros(self.n)
        self._check(self._lib.or_ms_rhs_at(self._h, _dp(_f64(m_unique, (self.n, 3))), _dp(b)))
        return b

    def ms_solve(self, m_unique, U0=None, tol: float = 1e-12, maxit: int = 100000):
        U = np.zeros(self.n) if U0 is None else _f64(U0, (self.n,)).copy()
        it = ctypes.c_int32(0)
        self._check(self._lib.or_ms_solve_at(self._h, _dp(_f64(m_unique, (self.n, 3))), _dp(U), tol, maxit,
                                             ctypes.byref(it)))
        return U, int(it.value)

    def ms_field(self, U) -> np.ndarray:
        hd = np.zeros((self.ne, 3))
        self._check(self._lib.or_ms_field(self._h, _dp(_f64(U, (self.n,))), _dp(hd)))
        return hd

    def ms_energy(self, U) -> float:
        e = np.zeros(1)
        self._check(self._lib.or_ms_energy(self._h, _dp(_f64(U, (self.n,))), _dp(e)))
        return float(e[0])

    def step(self, dt: float, n: int = 1) -> dict:
        st = _Stats()
        rc = self._lib.or_step(self._h, dt, n, ctypes.byref(st))
        stats = dict(steps_done=st.steps_done, mech_iters=st.mech_iters, gs_iters=list(st.gs_iters),
                     dm_avg=st.dm_avg, ms_iters=st.ms_iters)
        self._check(rc)
        return stats

    def relax(self, dt: float, dm_tol: float, max_steps: int):
        """Sec. 3.3: steps of dt until the step's mean per-node |m^n - m^{n-1}|
        over the magnetic nodes drops below dm_tol.  Returns (steps taken,
        converged)."""
        for k in range(1, max_steps + 1):
            if self.step(dt, 1)["dm_avg"] < dm_tol:
                return k, True
        return max_steps, False

    def sweep(self, params: dict, dt: float, dm_tol: float, max_steps: int, hext, sigma_ext=None,
              stop_on_reversal: bool = False, precession: bool = True, local_demag: bool = False,
              keep_going: bool = False):
        """Sec. 3.3 hysteresis protocol: for each applied field (and stress),
        relax and record the cell-averaged m; optionally stop after the first
        point whose mbar points against the first field.  A point that does
        not relax within max_steps ends the sweep, or with keep_going is
        recorded after max_steps and the sweep goes on.  Returns (mbar list,
        steps list), and with keep_going also the per-point converged list."""
        hext = np.asarray(hext, dtype=np.float64).reshape(-1, 3)
        first = hext[0]
        mbars, steps, conv = [], [], []
        for k in range(hext.shape[0]):
            sig = (0.0,) * 6 if sigma_ext is None else tuple(np.asarray(sigma_ext, dtype=np.float64).reshape(-1, 6)[k])
            self.set_params(params, hext=tuple(hext[k]), sigma_ext=sig, precession=precession, local_demag=local_demag)
            n, ok = self.relax(dt, dm_tol, max_steps)
            steps.append(n)
            conv.append(ok)
            if not ok and not keep_going:
                break
            mbar, _ = self.averages()
            mbars.append(mbar)
            if stop_on_reversal and float(np.dot(mbar, first)) <= 0.0:
                break
        return (mbars, steps, conv) if keep_going else (mbars, steps)

    def energies(self) -> dict:
        out = np.zeros(7)
        self._check(self._lib.or_energies(self._h, _dp(out)))
        return dict(zip(("exchange", "anisotropy", "zeeman", "magnetoelastic", "stress", "demag_far", "total"),
                        out.tolist()))

    def averages(self):
        mbar = np.zeros(3); ebar = np.zeros(6)
        self._check(self._lib.or_averages(self._h, _dp(mbar), _dp(ebar)))
        return mbar, ebar

    # ---- operators (unique-node order)
    def apply(self, which: int, x, eps: float = 0.0) -> np.ndarray:
        x = _f64(x, (self.n, 3)); y = np.zeros((self.n, 3))
        self._check(self._lib.or_apply(self._h, which, eps, _dp(x), _dp(y)))
        return y

    def solve(self, which: int, b, x0=None, eps: float = 0.0, tol: float = 1e-8, maxit: int = 100000):
        b = _f64(b, (self.n, 3))
        x = np.zeros((self.n, 3)) if x0 is None else _f64(x0, (self.n, 3)).copy()
        it = ctypes.c_int32(0)
        self._check(self._lib.or_solve(self._h, which, eps, _dp(b), _dp(x), tol, maxit, ctypes.byref(it)))
        return x, int(it.value)

    def precond_apply(self, r) -> np.ndarray:
        """z = B r for the elastic preconditioner (unique-node order)."""
        r = _f64(r, (self.n, 3)); z = np.zeros((self.n, 3))
        self._check(self._lib.or_precond_apply(self._h, _dp(r), _dp(z)))
        return z

    def precond_grid(self) -> tuple:
        g = np.zeros(3, dtype=np.int32)
        self._check(self._lib.or_precond_grid(self._h, g.ctypes.data))
        return tuple(int(v) for v in g)

    def set_precond_omega(self, omega: float) -> None:
        self._lib.or_set_precond_omega(self._h, float(omega))

    def elastic_rhs(self) -> np.ndarray:
        b = np.zeros((self.n, 3)); self._check(self._lib.or_elastic_rhs(self._h, _dp(b))); return b

    def field_rhs(self, c: float):
        b = np.zeros((self.n, 3)); ch = np.zeros((self.n, 3))
        self._check(self._lib.or_field_rhs(self._h, c, _dp(b), _dp(ch)))
        return b, ch

    # ---- helpers in the caller's order
    def to_user(self, v_unique: np.ndarray) -> np.ndarray:
        return np.asarray(v_unique)[self.node_map()]
