"""Python binding of librfa.so (include/rfa.h): argument marshalling only.

Every function named rfa_* here calls the C entry point of the same name;
all computation runs in the library's HIP kernels.  If the library is not
built, loading fails loudly (there is no fallback implementation).

Bulk voxel arrays are numpy arrays (host) for grids created with
inputs_on_device=0, or torch tensors on the grid's device for grids created
with inputs_on_device=1; PyTorch only provides device memory and streams.

The `Grid` class is a convenience wrapper over the same calls.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "librfa.so")

RFA_OK, RFA_ERR_ARG, RFA_ERR_STATE, RFA_ERR_UNSTABLE, RFA_ERR_OOM, RFA_ERR_HIP, \
    RFA_ERR_NUMERIC = range(7)


class RfaError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"[{status}] {message}")
        self.status = status
        self.message = message


class rfa_tissue(C.Structure):
    _fields_ = [("k", C.c_double), ("rho", C.c_double), ("c", C.c_double),
                ("h_perf", C.c_double), ("q_met", C.c_double), ("t_fixed", C.c_double),
                ("fixed", C.c_int), ("tissue", C.c_int)]


class rfa_needle(C.Structure):
    _fields_ = [("n_tines", C.c_int), ("pt_offset", C.POINTER(C.c_int)),
                ("pts", C.POINTER(C.c_double)), ("power", C.POINTER(C.c_double)),
                ("sigma", C.c_double)]


class rfa_options(C.Structure):
    _fields_ = [("t_death", C.c_double), ("A", C.c_double), ("Ea", C.c_double),
                ("R", C.c_double), ("omega_cap", C.c_double), ("stream", C.c_void_p),
                ("inputs_on_device", C.c_int), ("depth", C.c_int), ("kernel", C.c_int),
                ("tile_y", C.c_int), ("tile_x", C.c_int), ("time_kernels", C.c_int),
                ("z_vec", C.c_int), ("store_policy", C.c_int)]


class rfa_diag(C.Structure):
    _fields_ = [("energy_J", C.c_double), ("injected_J", C.c_double),
                ("perfusion_J", C.c_double), ("boundary_J", C.c_double),
                ("residual_J", C.c_double), ("mono_violations", C.c_longlong),
                ("t_min_C", C.c_double), ("t_max_C", C.c_double), ("steps", C.c_longlong)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


# Entry points declared in include/rfa.h, with their argument types.
_SIGS = {
    "rfa_default_options": [C.POINTER(rfa_options)],
    "rfa_create_grid": [C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double,
                        C.POINTER(rfa_options), C.POINTER(C.c_void_p)],
    "rfa_set_tissue": [C.c_void_p, C.c_void_p, C.POINTER(rfa_tissue), C.c_int],
    "rfa_set_needle": [C.c_void_p, C.POINTER(rfa_needle)],
    "rfa_set_perfusion": [C.c_void_p, C.c_void_p],
    "rfa_set_perfusion_decay": [C.c_void_p, C.c_int],
    "rfa_step": [C.c_void_p, C.c_int, C.c_double, C.POINTER(rfa_diag)],
    "rfa_dt_max": [C.c_void_p, C.POINTER(C.c_double)],
    "rfa_damage": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
    "rfa_damage_noalloc": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
    "rfa_get_temperature": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
    "rfa_set_temperature": [C.c_void_p, C.c_void_p],
    "rfa_save_state": [C.c_void_p, C.c_void_p, C.POINTER(C.c_size_t)],
    "rfa_load_state": [C.c_void_p, C.c_void_p, C.c_size_t],
    "rfa_get_step_count": [C.c_void_p, C.POINTER(C.c_longlong)],
    "rfa_source_support": [C.c_void_p, C.POINTER(C.c_longlong)],
    "rfa_kernel_stats": [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_longlong),
                         C.POINTER(C.c_longlong)],
    "rfa_get_plan": [C.c_void_p] + [C.POINTER(C.c_int)] * 6,
    "rfa_tune": [C.c_void_p, C.c_double, C.c_int],
    "rfa_copy_bandwidth": [C.c_size_t, C.c_int, C.POINTER(C.c_double)],
    "rfa_mix_bandwidth": [C.c_longlong, C.c_int, C.POINTER(C.c_double)],
    "rfa_adjoint_kernel_stats": [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_longlong)],
    "rfa_warp": [C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.POINTER(C.c_double)],
    "rfa_warp2": [C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.c_double, C.c_void_p,
                  C.POINTER(C.c_double)],
    "rfa_set_perfusion_bspline": [C.c_void_p, C.c_int, C.c_void_p],
    "rfa_reset_state": [C.c_void_p],
    "rfa_set_tine_powers": [C.c_void_p, C.POINTER(C.c_double)],
    "rfa_forward_checkpointed": [C.c_void_p, C.c_int, C.c_double, C.c_int],
    "rfa_adjoint": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
    "rfa_batch_create": [C.c_int, C.POINTER(C.c_void_p), C.POINTER(C.c_double),
                         C.POINTER(C.c_void_p)],
    "rfa_batch_step": [C.c_void_p, C.c_int, C.c_void_p],
    "rfa_batch_set_plan": [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_longlong],
    "rfa_batch_get_plan": [C.c_void_p] + [C.POINTER(C.c_int)] * 6,
    "rfa_batch_tune": [C.c_void_p, C.c_int],
    "rfa_batch_last_time": [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_longlong)],
    "rfa_batch_destroy": [C.c_void_p],
    "rfa_destroy_grid": [C.c_void_p],
    "rfa_status_string": [C.c_int],
    "rfa_last_error": [],
}

_lib = None


def lib() -> C.CDLL:
    """Load librfa.so (built in-tree by paper_1907_05709_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m "
                               "paper_1907_05709_amd.build` (no CPU fallback exists)")
        # One HIP runtime per process: torch ships its own libamdhip64 (same
        # SONAME, requested under another file name), so load torch first and
        # let librfa bind to the runtime already in the process.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.rfa_destroy_grid.restype = None
        L.rfa_batch_destroy.restype = None
        L.rfa_status_string.restype = C.c_char_p
        L.rfa_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def exported_symbols() -> Sequence[str]:
    return tuple(_SIGS)


def _check(status: int):
    if status != RFA_OK:
        raise RfaError(status, lib().rfa_last_error().decode())


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


def _ptr(a, device: bool, dtype, writable=False):
    """Pointer to a bulk array: a contiguous torch tensor on the GPU when
    the grid takes device pointers, else a contiguous numpy array."""
    if a is None:
        return None
    if device:
        if not _is_torch(a) or not a.is_cuda:
            raise TypeError("grid expects device tensors (inputs_on_device=1)")
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        want = {np.uint8: "torch.uint8", np.float32: "torch.float32",
                np.float64: "torch.float64"}[dtype]
        if str(a.dtype) != want:
            raise TypeError(f"tensor dtype {a.dtype}, expected {want}")
        return C.c_void_p(a.data_ptr())
    if _is_torch(a):
        raise TypeError("grid expects host numpy arrays (inputs_on_device=0)")
    if a.dtype != dtype or not a.flags["C_CONTIGUOUS"] or (writable and not a.flags.writeable):
        raise ValueError(f"array must be C-contiguous {np.dtype(dtype).name}")
    return C.c_void_p(a.ctypes.data)


# ---- thin wrappers, same names as the C ABI --------------------------------
def rfa_default_options() -> rfa_options:
    o = rfa_options()
    _check(lib().rfa_default_options(C.byref(o)))
    return o


def rfa_create_grid(nx, ny, nz, dx, dy, dz, opt: Optional[rfa_options] = None) -> C.c_void_p:
    h = C.c_void_p()
    _check(lib().rfa_create_grid(nx, ny, nz, dx, dy, dz,
                                 C.byref(opt) if opt is not None else None, C.byref(h)))
    return h


def make_tissue_table(tissue) -> C.Array:
    tab = (rfa_tissue * len(tissue))()
    for i, t in enumerate(tissue):
        tab[i] = rfa_tissue(t.k, t.rho, t.c, t.h, t.q_met, t.t_fixed, int(t.fixed),
                            int(t.tissue))
    return tab


def rfa_set_tissue(g, labels_ptr, table, n_classes: int):
    _check(lib().rfa_set_tissue(g, labels_ptr, table, n_classes))


def make_needle(n_tines: int, pt_offset, pts, power, sigma: float):
    """Returns (struct, keepalive arrays)."""
    offs = np.ascontiguousarray(pt_offset, dtype=np.int32)
    p = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1)
    pw = np.ascontiguousarray(power, dtype=np.float64)
    nd = rfa_needle(n_tines, offs.ctypes.data_as(C.POINTER(C.c_int)),
                    p.ctypes.data_as(C.POINTER(C.c_double)),
                    pw.ctypes.data_as(C.POINTER(C.c_double)), float(sigma))
    return nd, (offs, p, pw)


def rfa_set_needle(g, needle: rfa_needle):
    _check(lib().rfa_set_needle(g, C.byref(needle)))


def rfa_set_perfusion(g, factor_ptr):
    _check(lib().rfa_set_perfusion(g, factor_ptr))


def rfa_set_perfusion_decay(g, enable: bool):
    _check(lib().rfa_set_perfusion_decay(g, int(bool(enable))))


def rfa_step(g, n_steps: int, dt: float, want_diag: bool = True):
    d = rfa_diag() if want_diag else None
    _check(lib().rfa_step(g, int(n_steps), float(dt), C.byref(d) if d is not None else None))
    return d


def rfa_dt_max(g) -> float:
    v = C.c_double()
    _check(lib().rfa_dt_max(g, C.byref(v)))
    return v.value


def rfa_damage(g, mask_ptr, omega_ptr, dead_ptr):
    _check(lib().rfa_damage(g, mask_ptr, omega_ptr, dead_ptr))


def rfa_get_temperature(g, t_ptr, hi_ptr, lo_ptr):
    _check(lib().rfa_get_temperature(g, t_ptr, hi_ptr, lo_ptr))


def rfa_set_temperature(g, t_ptr):
    _check(lib().rfa_set_temperature(g, t_ptr))


def rfa_save_state(g) -> bytes:
    n = C.c_size_t(0)
    _check(lib().rfa_save_state(g, None, C.byref(n)))
    buf = (C.c_ubyte * n.value)()
    _check(lib().rfa_save_state(g, buf, C.byref(n)))
    return bytes(buf)


def rfa_load_state(g, data: bytes):
    buf = (C.c_ubyte * len(data)).from_buffer_copy(data)
    _check(lib().rfa_load_state(g, buf, len(data)))


def rfa_get_step_count(g) -> int:
    v = C.c_longlong()
    _check(lib().rfa_get_step_count(g, C.byref(v)))
    return v.value


def rfa_kernel_stats(g):
    ms, n, vs = C.c_double(), C.c_longlong(), C.c_longlong()
    _check(lib().rfa_kernel_stats(g, C.byref(ms), C.byref(n), C.byref(vs)))
    return ms.value, n.value, vs.value


def rfa_get_plan(g):
    v = [C.c_int() for _ in range(6)]
    _check(lib().rfa_get_plan(g, *[C.byref(x) for x in v]))
    return dict(zip(("kernel", "depth", "tile_y", "tile_x", "workgroups", "z_vec"),
                    [x.value for x in v]))


def rfa_tune(g, dt: float, reps: int = 20):
    _check(lib().rfa_tune(g, float(dt), int(reps)))


def rfa_warp(g, v_ptr, beta: float, out_ptr, timed: bool = False):
    """Breathing-motion view of the temperature; returns the kernel time in
    ms when timed, else None."""
    ms = C.c_double(0.0)
    _check(lib().rfa_warp(g, v_ptr, float(beta), out_ptr, C.byref(ms) if timed else None))
    return ms.value if timed else None


def rfa_warp2(g, v1_ptr, beta1: float, v2_ptr, beta2: float, out_ptr, timed: bool = False):
    """Breathing view through beta1 v1 + beta2 v2; returns the kernel time
    in ms when timed, else None."""
    ms = C.c_double(0.0)
    _check(lib().rfa_warp2(g, v1_ptr, float(beta1), v2_ptr, float(beta2), out_ptr,
                           C.byref(ms) if timed else None))
    return ms.value if timed else None


def rfa_adjoint_kernel_stats(g):
    """(milliseconds, launches) of adjoint kernels timed since the last call."""
    ms, n = C.c_double(0.0), C.c_longlong(0)
    _check(lib().rfa_adjoint_kernel_stats(g, C.byref(ms), C.byref(n)))
    return ms.value, n.value


def rfa_copy_bandwidth(nbytes: int, reps: int = 20) -> float:
    v = C.c_double()
    _check(lib().rfa_copy_bandwidth(int(nbytes), int(reps), C.byref(v)))
    return v.value


def rfa_mix_bandwidth(n_voxels: int, reps: int = 10) -> float:
    """Streaming rate (GB/s) of the step's 25 B/voxel mix without the stencil."""
    v = C.c_double()
    _check(lib().rfa_mix_bandwidth(int(n_voxels), int(reps), C.byref(v)))
    return v.value


def rfa_set_perfusion_bspline(g, ctrl: np.ndarray):
    c = np.ascontiguousarray(ctrl, dtype=np.float32)
    m = c.shape[0]
    assert c.shape == (m, m, m)
    _check(lib().rfa_set_perfusion_bspline(g, m, C.c_void_p(c.ctypes.data)))


def rfa_reset_state(g):
    _check(lib().rfa_reset_state(g))


def rfa_set_tine_powers(g, power):
    p = np.ascontiguousarray(power, dtype=np.float64)
    _check(lib().rfa_set_tine_powers(g, p.ctypes.data_as(C.POINTER(C.c_double))))


def rfa_forward_checkpointed(g, n_steps: int, dt: float, ckpt_every: int):
    _check(lib().rfa_forward_checkpointed(g, int(n_steps), float(dt), int(ckpt_every)))


def rfa_adjoint(g, w_ptr, dL_dP: Optional[np.ndarray], dL_dctrl: Optional[np.ndarray],
                dperf_ptr):
    """dL_dP, dL_dctrl: host float64 arrays filled in place (or None);
    w_ptr / dperf_ptr: bulk pointers from _ptr()."""
    _check(lib().rfa_adjoint(g, w_ptr,
                             None if dL_dP is None else C.c_void_p(dL_dP.ctypes.data),
                             None if dL_dctrl is None else C.c_void_p(dL_dctrl.ctypes.data),
                             dperf_ptr))


def rfa_batch_create(handles, dts) -> C.c_void_p:
    n = len(handles)
    arr = (C.c_void_p * n)(*[h.value if isinstance(h, C.c_void_p) else h for h in handles])
    dt = (C.c_double * n)(*[float(d) for d in dts])
    b = C.c_void_p()
    _check(lib().rfa_batch_create(n, arr, dt, C.byref(b)))
    return b


def rfa_batch_step(b, n_steps: int, n_grids: int = 0, want_diag: bool = False):
    diags = (rfa_diag * n_grids)() if want_diag else None
    _check(lib().rfa_batch_step(b, int(n_steps), diags))
    return [d.as_dict() for d in diags] if want_diag else None


RFA_BATCH_TILES, RFA_BATCH_FLAT = 1, 2
_LAYOUTS = {0: 0, "tiles": RFA_BATCH_TILES, "flat": RFA_BATCH_FLAT,
            RFA_BATCH_TILES: RFA_BATCH_TILES, RFA_BATCH_FLAT: RFA_BATCH_FLAT}


def rfa_batch_set_plan(b, tile_y: int = 0, tile_x: int = 0, workgroups: int = 0,
                       group_voxels: int = -1, layout=0):
    """layout: 0 (keep), "tiles" or "flat" (or the RFA_BATCH_* values)."""
    if layout not in _LAYOUTS:
        raise RfaError(RFA_ERR_ARG, f"layout must be one of {sorted(map(str, _LAYOUTS))}")
    _check(lib().rfa_batch_set_plan(b, _LAYOUTS[layout], int(tile_y), int(tile_x),
                                    int(workgroups), int(group_voxels)))


def rfa_batch_get_plan(b) -> dict:
    v = [C.c_int() for _ in range(6)]
    _check(lib().rfa_batch_get_plan(b, *[C.byref(x) for x in v]))
    d = dict(zip(("layout", "tile_y", "tile_x", "items", "workgroups", "groups"),
                 [x.value for x in v]))
    d["layout"] = "flat" if d["layout"] == RFA_BATCH_FLAT else "tiles"
    return d


def rfa_batch_tune(b, reps: int = 20):
    _check(lib().rfa_batch_tune(b, int(reps)))


def rfa_batch_last_time(b):
    ms, vs = C.c_double(), C.c_longlong()
    _check(lib().rfa_batch_last_time(b, C.byref(ms), C.byref(vs)))
    return ms.value, vs.value


def rfa_batch_destroy(b):
    lib().rfa_batch_destroy(b)


def rfa_destroy_grid(g):
    lib().rfa_destroy_grid(g)


def rfa_status_string(s: int) -> str:
    return lib().rfa_status_string(s).decode()


def rfa_last_error() -> str:
    return lib().rfa_last_error().decode()


# ---- convenience wrapper -----------------------------------------------------
class Grid:
    """One simulation grid.  device=True: bulk arrays are torch CUDA tensors
    (inputs_on_device=1, kernels on torch's current stream); device=False:
    numpy arrays."""

    def __init__(self, shape, spacing, device: bool = False, depth: int = 0,
                 stream=None, kernel: int = 0, tile_y: int = 0, tile_x: int = 0,
                 time_kernels: int = 0, z_vec: int = 0, store_policy: int = 0, **damage):
        self.shape = tuple(int(s) for s in shape)
        self.spacing = tuple(float(s) for s in spacing)
        self.device = bool(device)
        opt = rfa_default_options()
        for k, v in damage.items():
            setattr(opt, k, v)
        opt.inputs_on_device = int(self.device)
        opt.depth = int(depth)
        opt.kernel = int(kernel)
        opt.tile_y = int(tile_y)
        opt.tile_x = int(tile_x)
        opt.time_kernels = int(time_kernels)
        opt.z_vec = int(z_vec)
        opt.store_policy = int(store_policy)
        if stream is not None:
            opt.stream = C.c_void_p(int(stream))
        elif self.device:
            import torch
            opt.stream = C.c_void_p(int(torch.cuda.current_stream().cuda_stream))
        self.opt = opt
        self.h = rfa_create_grid(*self.shape, *self.spacing, opt)
        self.n_classes = 0

    @property
    def n(self) -> int:
        return int(np.prod(self.shape))

    def close(self):
        if getattr(self, "h", None):
            rfa_destroy_grid(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- inputs
    def set_tissue(self, labels, tissue):
        self.n_classes = len(tissue)
        table = make_tissue_table(tissue)
        if self.device:
            rfa_set_tissue(self.h, _ptr(labels, True, np.uint8), table, len(tissue))
        else:
            lab = np.ascontiguousarray(labels, dtype=np.uint8)
            rfa_set_tissue(self.h, _ptr(lab, False, np.uint8), table, len(tissue))

    def set_needle(self, needle):
        if needle is None or needle.n_tines == 0:
            nd = rfa_needle(0, None, None, None, 1.0)
            rfa_set_needle(self.h, nd)
            return
        nd, keep = make_needle(needle.n_tines, needle.pt_offset, needle.pts, needle.power,
                               needle.sigma)
        rfa_set_needle(self.h, nd)
        del keep

    def set_perfusion(self, factor):
        if factor is None:
            rfa_set_perfusion(self.h, None)
        elif self.device:
            rfa_set_perfusion(self.h, _ptr(factor, True, np.float32))
        else:
            f = np.ascontiguousarray(factor, dtype=np.float32)
            rfa_set_perfusion(self.h, _ptr(f, False, np.float32))

    def load_case(self, case):
        """Tissue and needle of a workload Case (host arrays are moved to the
        device first for device grids)."""
        labels = case.labels
        if self.device:
            import torch
            labels = torch.from_numpy(np.ascontiguousarray(labels)).cuda()
        self.set_tissue(labels, case.tissue)
        self.set_needle(case.needle)
        if getattr(case, "perfusion_decay", False):
            self.set_perfusion_decay(True)

    def set_perfusion_decay(self, enable: bool = True):
        rfa_set_perfusion_decay(self.h, enable)

    # -- stepping
    def step(self, n_steps: int, dt: float, diag: bool = True):
        d = rfa_step(self.h, n_steps, dt, diag)
        return d.as_dict() if d is not None else None

    def dt_max(self) -> float:
        return rfa_dt_max(self.h)

    # -- outputs
    def _alloc(self, dtype):
        if self.device:
            import torch
            td = {np.uint8: torch.uint8, np.float32: torch.float32,
                  np.float64: torch.float64}[dtype]
            return torch.empty(self.shape, dtype=td, device="cuda")
        return np.empty(self.shape, dtype=dtype)

    def temperature(self):
        t = self._alloc(np.float64)
        rfa_get_temperature(self.h, _ptr(t, self.device, np.float64, True), None, None)
        return t

    def raw_state(self):
        hi, lo = self._alloc(np.float32), self._alloc(np.float32)
        rfa_get_temperature(self.h, None, _ptr(hi, self.device, np.float32, True),
                            _ptr(lo, self.device, np.float32, True))
        return hi, lo

    def set_temperature(self, t):
        if self.device:
            rfa_set_temperature(self.h, _ptr(t, True, np.float64))
        else:
            a = np.ascontiguousarray(t, dtype=np.float64)
            rfa_set_temperature(self.h, _ptr(a, False, np.float64))

    def warp(self, v, beta: float, out=None, timed: bool = False, v2=None, beta2: float = 0.0):
        """Temperature (degC, float) seen through the inverse breathing
        displacement beta * v (+ beta2 * v2 with a second field), each of
        shape (3, nx, ny, nz) in metres.  Returns out, or (out, kernel_ms)
        when timed."""
        fields = [v] if v2 is None else [v, v2]
        for f in fields:
            if tuple(f.shape) != (3,) + self.shape:
                raise ValueError(f"displacement fields must have shape {(3,) + self.shape}")
        if out is None:
            out = self._alloc(np.float32)
        if not self.device:
            fields = [np.ascontiguousarray(f, dtype=np.float32) for f in fields]
        ptrs = [_ptr(f, self.device, np.float32) for f in fields]
        optr = _ptr(out, self.device, np.float32, True)
        if v2 is None:
            ms = rfa_warp(self.h, ptrs[0], beta, optr, timed)
        else:
            ms = rfa_warp2(self.h, ptrs[0], beta, ptrs[1], beta2, optr, timed)
        return (out, ms) if timed else out

    def damage(self):
        mask, om = self._alloc(np.uint8), self._alloc(np.float32)
        dead = np.zeros(2 * max(self.n_classes, 1))
        rfa_damage(self.h, _ptr(mask, self.device, np.uint8, True),
                   _ptr(om, self.device, np.float32, True), C.c_void_p(dead.ctypes.data))
        return mask, om, dead.reshape(-1, 2)

    def omega(self):
        """The damage integral alone (rfa_damage with the other outputs NULL:
        for a device grid no synchronisation)."""
        om = self._alloc(np.float32)
        rfa_damage(self.h, None, _ptr(om, self.device, np.float32, True), None)
        return om

    def damage_noalloc(self, want_mask: bool = True, want_omega: bool = True,
                       want_dead: bool = True):
        """rfa_damage_noalloc: as damage(), through the allocation-free entry
        point (outputs not asked for are passed as NULL)."""
        mask = self._alloc(np.uint8) if want_mask else None
        om = self._alloc(np.float32) if want_omega else None
        dead = np.zeros(2 * max(self.n_classes, 1)) if want_dead else None
        _check(lib().rfa_damage_noalloc(
            self.h, None if mask is None else _ptr(mask, self.device, np.uint8, True),
            None if om is None else _ptr(om, self.device, np.float32, True),
            None if dead is None else C.c_void_p(dead.ctypes.data)))
        return mask, om, None if dead is None else dead.reshape(-1, 2)

    def save_state(self) -> bytes:
        return rfa_save_state(self.h)

    def load_state(self, data: bytes):
        rfa_load_state(self.h, data)

    def step_count(self) -> int:
        return rfa_get_step_count(self.h)

    def kernel_stats(self):
        """(kernel ms, launches, voxel-steps) since the last call."""
        return rfa_kernel_stats(self.h)

    # -- differentiation
    def set_perfusion_bspline(self, ctrl):
        rfa_set_perfusion_bspline(self.h, ctrl)

    def reset_state(self):
        rfa_reset_state(self.h)

    def set_tine_powers(self, power):
        rfa_set_tine_powers(self.h, power)

    def forward_checkpointed(self, n_steps: int, dt: float, ckpt_every: int):
        rfa_forward_checkpointed(self.h, n_steps, dt, ckpt_every)

    def adjoint(self, w_omega, n_tines: int = 0, m: int = 0, want_dperf: bool = False):
        """Returns (dL/dP [n_tines] or None, dL/dctrl [m,m,m] or None,
        dL/dperf per voxel or None) for dL/dOmega^N = w_omega."""
        dP = np.zeros(n_tines) if n_tines else None
        dc = np.zeros((m, m, m)) if m else None
        dperf = self._alloc(np.float32) if want_dperf else None
        if self.device:
            w = w_omega.contiguous().float()
            wp = _ptr(w, True, np.float32)
        else:
            w = np.ascontiguousarray(w_omega, dtype=np.float32)
            wp = _ptr(w, False, np.float32)
        rfa_adjoint(self.h, wp, dP, dc,
                    None if dperf is None else _ptr(dperf, self.device, np.float32, True))
        return dP, dc, dperf

    def adjoint_kernel_stats(self):
        return rfa_adjoint_kernel_stats(self.h)

    def plan(self) -> dict:
        return rfa_get_plan(self.h)

    def source_support(self) -> int:
        """rfa_source_support: voxels on which the step reads the source."""
        v = C.c_longlong()
        _check(lib().rfa_source_support(self.h, C.byref(v)))
        return int(v.value)

    def tune(self, dt: float, reps: int = 20) -> dict:
        rfa_tune(self.h, dt, reps)
        return self.plan()


class Batch:
    """Lockstep stepping of several Grid objects (each with its own dt) by
    one persistent launch per step, the step loop replayed from a hipGraph.
    The batch borrows the grids: close it before them."""

    def __init__(self, grids, dts):
        self.grids = list(grids)
        self.h = rfa_batch_create([g.h for g in self.grids], dts)

    def step(self, n_steps: int, diag: bool = False):
        return rfa_batch_step(self.h, n_steps, len(self.grids), diag)

    def last_time(self):
        """(device ms of the last step call, voxel-steps it advanced)."""
        return rfa_batch_last_time(self.h)

    def set_plan(self, tile_y: int = 0, tile_x: int = 0, workgroups: int = 0,
                 group_voxels: int = -1, layout=0):
        rfa_batch_set_plan(self.h, tile_y, tile_x, workgroups, group_voxels, layout)
        return self.plan()

    def plan(self) -> dict:
        return rfa_batch_get_plan(self.h)

    def tune(self, reps: int = 20) -> dict:
        """Time candidate launch shapes and keep the fastest (grids unchanged)."""
        rfa_batch_tune(self.h, reps)
        return self.plan()

    def close(self):
        if getattr(self, "h", None):
            rfa_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
