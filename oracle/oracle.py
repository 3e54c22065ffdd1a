"""ctypes front end of the FP64 CPU oracle (oracle/rfa_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the product package.  It shares
no code with the HIP library; both are driven by the seeded inputs of
paper_1907_05709_amd/workloads.py (which contains none of the method's
arithmetic).

Every function takes a workload Case (or its parts) and returns numpy FP64
arrays shaped like the grid, [nx, ny, nz] with z fastest.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rfa_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

DIAG_FIELDS = ("energy", "injected", "perfusion", "boundary", "residual",
               "mono", "tmin", "tmax")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-D_DEFAULT_SOURCE", "-Wall", "-Wextra",
                               "-Wno-unused-parameter", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Tissue(C.Structure):
    _fields_ = [("k", C.c_double), ("rho", C.c_double), ("c", C.c_double),
                ("h", C.c_double), ("q_met", C.c_double), ("t_fixed", C.c_double),
                ("fixed", C.c_int), ("tissue", C.c_int)]


class _Problem(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("labels", C.c_void_p), ("tab", C.POINTER(_Tissue)),
                ("n_classes", C.c_int), ("q", C.c_void_p), ("perf", C.c_void_p),
                ("t_blood", C.c_double), ("t_death", C.c_double),
                ("A", C.c_double), ("Ea", C.c_double), ("R", C.c_double),
                ("omega_cap", C.c_double), ("perf_decay", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=False)
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        L.oracle_source.restype = C.c_int
        L.oracle_run.restype = C.c_int
        L.oracle_adjoint.restype = C.c_int
        L.oracle_dt_max.restype = C.c_double
        L.oracle_damage_rate.restype = C.c_double
        L.oracle_damage_rate.argtypes = [C.c_double] * 4
        L.oracle_segment_density.restype = C.c_double
        L.oracle_segment_density.argtypes = [dp, dp, C.c_double, dp]
        L.oracle_tine_density_at.restype = C.c_double
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Problem:
    """Owns the ctypes problem struct and the arrays it points to."""

    def __init__(self, case, q: Optional[np.ndarray] = None,
                 perf: Optional[np.ndarray] = None):
        self.case = case
        nx, ny, nz = case.shape
        self.labels = np.ascontiguousarray(case.labels, dtype=np.uint8)
        tab = (_Tissue * len(case.tissue))()
        for i, t in enumerate(case.tissue):
            tab[i] = _Tissue(t.k, t.rho, t.c, t.h, t.q_met, t.t_fixed, t.fixed, t.tissue)
        self.tab = tab
        self.q = None if q is None else np.ascontiguousarray(q, dtype=np.float64)
        self.perf = None if perf is None else np.ascontiguousarray(perf, dtype=np.float64)
        dx, dy, dz = case.spacing
        self.s = _Problem(nx, ny, nz, dx, dy, dz, _ptr(self.labels),
                          C.cast(tab, C.POINTER(_Tissue)), len(case.tissue),
                          _ptr(self.q), _ptr(self.perf), case.t_blood, case.t_death,
                          case.arrhenius_a, case.arrhenius_ea, case.gas_r,
                          case.omega_cap, int(getattr(case, "perfusion_decay", False)))

    @property
    def ref(self):
        return C.byref(self.s)


def source(case, per_tine: bool = False):
    """RF power density q [W/m^3] of the case's needle (and, if per_tine,
    the per-watt tine shapes g_hat [n_tines, nx, ny, nz] and the
    unnormalised tine integrals)."""
    P = Problem(case)
    nd = case.needle
    q = np.zeros(case.shape)
    g = np.zeros((nd.n_tines,) + tuple(case.shape)) if per_tine else None
    un = np.zeros(nd.n_tines)
    offs = np.ascontiguousarray(nd.pt_offset, dtype=np.int32)
    pts = np.ascontiguousarray(nd.pts, dtype=np.float64)
    pw = np.ascontiguousarray(nd.power, dtype=np.float64)
    st = lib().oracle_source(P.ref, C.c_int(nd.n_tines), _ptr(offs), _ptr(pts), _ptr(pw),
                             C.c_double(nd.sigma), _ptr(q), _ptr(g), _ptr(un))
    if st != 0:
        raise ValueError("a tine has no weight on free voxels")
    return (q, g, un) if per_tine else q


def tine_density_at(case, tine: int, i: int, j: int, k: int) -> float:
    """Unnormalised density of one tine at one voxel (for sampled checks)."""
    P = Problem(case)
    nd = case.needle
    offs = np.ascontiguousarray(nd.pt_offset, dtype=np.int32)
    pts = np.ascontiguousarray(nd.pts, dtype=np.float64)
    return lib().oracle_tine_density_at(P.ref, _ptr(offs), _ptr(pts),
                                        C.c_double(nd.sigma), C.c_int(tine),
                                        C.c_int(i), C.c_int(j), C.c_int(k))


def segment_density(a, b, sigma: float, x) -> float:
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    return lib().oracle_segment_density(_dptr(a), _dptr(b), sigma, _dptr(x))


def damage_rate(case, t_c: float) -> float:
    return lib().oracle_damage_rate(case.arrhenius_a, case.arrhenius_ea, case.gas_r, t_c)


def initial_state(case):
    P = Problem(case)
    n = case.n_voxels
    T = np.zeros(n)
    om = np.zeros(n)
    tm = np.zeros(n)
    lib().oracle_init(P.ref, _ptr(T), _ptr(om), _ptr(tm))
    return T.reshape(case.shape), om.reshape(case.shape), tm.reshape(case.shape)


class State:
    """Temperature [degC], damage integral and running maximum temperature."""

    def __init__(self, T, omega, tmax):
        self.T, self.omega, self.tmax = T, omega, tmax

    def copy(self):
        return State(self.T.copy(), self.omega.copy(), self.tmax.copy())

    def masks(self, case):
        """bit0: latched T >= t_death, bit1: Omega >= 1 (tissue classes only)."""
        tis = np.array([t.tissue for t in case.tissue], dtype=bool)[case.labels]
        m = np.zeros(case.shape, dtype=np.uint8)
        m |= ((self.tmax >= case.t_death) & tis).astype(np.uint8)
        m |= (((self.omega >= 1.0) & tis).astype(np.uint8) << 1)
        return m


def run(case, n_steps: Optional[int] = None, dt: Optional[float] = None,
        q: Optional[np.ndarray] = None, perf: Optional[np.ndarray] = None,
        state: Optional[State] = None, diag: bool = False, trajectory: bool = False):
    """Run the explicit stepper.  Returns (State, diag[n_steps, 8] or None,
    trajectory[n_steps, nx, ny, nz] or None).  q defaults to the case's
    needle source; state defaults to the initial state."""
    n_steps = case.n_steps if n_steps is None else n_steps
    dt = case.dt if dt is None else dt
    if q is None:
        q = source(case)
    P = Problem(case, q=q, perf=perf)
    st = State(*initial_state(case)) if state is None else state.copy()
    T = np.ascontiguousarray(st.T, dtype=np.float64)
    om = np.ascontiguousarray(st.omega, dtype=np.float64)
    tm = np.ascontiguousarray(st.tmax, dtype=np.float64)
    dg = np.zeros((n_steps, len(DIAG_FIELDS))) if diag else None
    tr = np.zeros((n_steps,) + tuple(case.shape)) if trajectory else None
    rc = lib().oracle_run(P.ref, C.c_int(n_steps), C.c_double(dt), _ptr(T), _ptr(om),
                          _ptr(tm), _ptr(dg), _ptr(tr))
    if rc != 0:
        raise MemoryError("oracle_run failed")
    return State(T, om, tm), dg, tr


def dt_max(case, perf: Optional[np.ndarray] = None) -> float:
    P = Problem(case, perf=perf)
    return lib().oracle_dt_max(P.ref)


def step_linear(case, dt: float, x: np.ndarray, perf=None) -> np.ndarray:
    P = Problem(case, perf=perf)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.zeros_like(x)
    lib().oracle_step_linear(P.ref, C.c_double(dt), _ptr(x), _ptr(y))
    return y


def step_linear_transpose(case, dt: float, x: np.ndarray, perf=None) -> np.ndarray:
    P = Problem(case, perf=perf)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.zeros_like(x)
    lib().oracle_step_linear_transpose(P.ref, C.c_double(dt), _ptr(x), _ptr(y))
    return y


def adjoint(case, w: np.ndarray, n_steps: Optional[int] = None, dt: Optional[float] = None,
            q: Optional[np.ndarray] = None, perf: Optional[np.ndarray] = None,
            T0: Optional[np.ndarray] = None):
    """Discrete adjoint: returns (dL/dq [W/m^3]^-1, dL/dperf) per voxel for
    a loss with dL/dOmega^N = w, starting from T0 (default: initial state)."""
    n_steps = case.n_steps if n_steps is None else n_steps
    dt = case.dt if dt is None else dt
    if q is None:
        q = source(case)
    P = Problem(case, q=q, perf=perf)
    if T0 is None:
        T0 = initial_state(case)[0]
    T0 = np.ascontiguousarray(T0, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    dq = np.zeros(case.shape)
    dp = np.zeros(case.shape)
    rc = lib().oracle_adjoint(P.ref, C.c_int(n_steps), C.c_double(dt), _ptr(T0), _ptr(w),
                              _ptr(dq), _ptr(dp))
    if rc == -2:
        raise ValueError("no adjoint for damage-coupled perfusion")
    if rc != 0:
        raise MemoryError("oracle_adjoint failed")
    return dq, dp


def bspline_field(shape, ctrl: np.ndarray) -> np.ndarray:
    m = ctrl.shape[0]
    ctrl = np.ascontiguousarray(ctrl, dtype=np.float64)
    f = np.zeros(shape)
    lib().oracle_bspline_field(C.c_int(shape[0]), C.c_int(shape[1]), C.c_int(shape[2]),
                               C.c_int(m), _ptr(ctrl), _ptr(f))
    return f


def bspline_grad(f: np.ndarray, gf: np.ndarray, m: int) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.float64)
    gf = np.ascontiguousarray(gf, dtype=np.float64)
    g = np.zeros((m, m, m))
    lib().oracle_bspline_grad(C.c_int(f.shape[0]), C.c_int(f.shape[1]), C.c_int(f.shape[2]),
                              C.c_int(m), _ptr(f), _ptr(gf), _ptr(g))
    return g


def set_threads(n: int) -> None:
    """OpenMP threads of the oracle's parallel loops (the benchmark's
    single-core timing)."""
    lib().omp_set_num_threads(C.c_int(int(n)))
