"""Thin ctypes binding of the C ABI declared in include/qhd.h.

Argument marshalling only: every step of the evolution and of the readouts
runs in the HIP kernels of libqhd.so.  There is no CPU fallback: if the
library is missing or cannot be loaded, every call raises.

The module-level functions carry the C names (qhd_plan_create, qhd_evolve,
...); ``Plan`` is a convenience wrapper that keeps the buffers alive.  Device
memory and streams come from PyTorch (ROCm build): pass ``torch`` tensors
that live on the GPU, or numpy arrays for host data.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqhd.so")

QHD_OK, QHD_EINVAL, QHD_EUNSUPPORTED, QHD_ENOMEM, QHD_EDEVICE, QHD_ESTATE, QHD_ENUMERIC = range(7)
STATUS_NAMES = {0: "QHD_OK", 1: "QHD_EINVAL", 2: "QHD_EUNSUPPORTED", 3: "QHD_ENOMEM",
                4: "QHD_EDEVICE", 5: "QHD_ESTATE", 6: "QHD_ENUMERIC"}
QHD_SCHED_NESTEROV, QHD_SCHED_CONST, QHD_SCHED_TABLE, QHD_SCHED_LINEAR = 0, 1, 2, 3
QHD_MODEL_QHD, QHD_MODEL_QAA = 0, 1
QHD_INIT_UNIFORM, QHD_INIT_USER = 0, 1
QHD_SCHEME_STRANG, QHD_SCHEME_LIE, QHD_SCHEME_YOSHIDA4, QHD_SCHEME_LEAPFROG = 0, 1, 2, 3
QHD_OPT_TIME_PASSES = 0x1
QHD_OPT_AUTOTUNE = 0x2
QHD_OPT_NO_GRAPH = 0x4
QHD_OPT_MFMA_DFT = 0x8
QHD_OPT_RESIDENT = 0x10


class QHDError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.message = message


class qhd_instance(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("n", ctypes.c_int32 * 3),
        ("lo", ctypes.c_double * 3),
        ("hi", ctypes.c_double * 3),
        ("dt", ctypes.c_double),
        ("nsteps", ctypes.c_int64),
        ("sched_kind", ctypes.c_int32),
        ("sched_p", ctypes.c_double * 2),
        ("sched_table", ctypes.POINTER(ctypes.c_double)),
        ("init_kind", ctypes.c_int32),
        ("success_radius", ctypes.c_double),
        ("scheme", ctypes.c_int32),
        ("model", ctypes.c_int32),
    ]


class qhd_plan_opts(ctypes.Structure):
    _fields_ = [
        ("flags", ctypes.c_uint32),
        ("norm_tolerance", ctypes.c_double),
        ("timing_stride", ctypes.c_int32),
        ("tune_cache", ctypes.c_char_p),
    ]


class qhd_observables(ctypes.Structure):
    _fields_ = [
        ("norm", ctypes.c_double),
        ("e_f", ctypes.c_double),
        ("success_mass", ctypes.c_double),
        ("f_min", ctypes.c_double),
        ("argmin_index", ctypes.c_int64),
        ("steps_done", ctypes.c_int64),
        ("t", ctypes.c_double),
    ]


class qhd_kernel_timing(ctypes.Structure):
    _fields_ = [
        ("name", ctypes.c_char * 48),
        ("launches", ctypes.c_int64),
        ("total_ms", ctypes.c_double),
        ("points", ctypes.c_double),
        ("bytes_per_point", ctypes.c_double),
    ]


QHD_SNO_BF16, QHD_SNO_FP32 = 0, 1


class qhd_sno_desc(ctypes.Structure):
    _fields_ = [
        ("grid", ctypes.c_int32),
        ("width", ctypes.c_int32),
        ("modes", ctypes.c_int32),
        ("layers", ctypes.c_int32),
        ("max_batch", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("train", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
    ]


class qhd_rqp_desc(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("r", ctypes.c_int32),
        ("dt", ctypes.c_double),
        ("nsteps", ctypes.c_int64),
        ("sched_kind", ctypes.c_int32),
        ("sched_p", ctypes.c_double * 2),
        ("sched_table", ctypes.POINTER(ctypes.c_double)),
        ("min_tol", ctypes.c_double),
    ]


class qhd_rqp_obs(ctypes.Structure):
    _fields_ = [
        ("norm", ctypes.c_double),
        ("e_f", ctypes.c_double),
        ("p_min", ctypes.c_double),
        ("f_min", ctypes.c_double),
        ("argmin_index", ctypes.c_int64),
        ("steps_done", ctypes.c_int64),
        ("t", ctypes.c_double),
    ]


class qhd_class_info(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("n", ctypes.c_int32 * 3),
        ("members", ctypes.c_int32),
        ("col_variant", ctypes.c_int32),
        ("grid_cap_row", ctypes.c_int32),
        ("grid_cap_col", ctypes.c_int32),
        ("tuned", ctypes.c_int32),
        ("mfma_dft", ctypes.c_int32),
        ("row_points_per_lane", ctypes.c_int32),
        ("resident", ctypes.c_int32),
    ]


class qhd_readout(ctypes.Structure):
    _fields_ = [
        ("norm", ctypes.c_double),
        ("e_f", ctypes.c_double),
        ("success_mass", ctypes.c_double),
        ("f_min", ctypes.c_double),
        ("argmin_index", ctypes.c_int64),
    ]


QHD_STATIC_MAX_LINES = 65536

_lib = None

# every entry point declared in include/qhd.h, include/qhd_sno.h and include/qhd_rqp.h,
# with its ctypes signature
_SIGNATURES = {
    "qhd_plan_create": (ctypes.c_int, [ctypes.POINTER(qhd_instance), ctypes.c_int32,
                                       ctypes.POINTER(qhd_plan_opts), ctypes.POINTER(ctypes.c_void_p)]),
    "qhd_set_potential": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32]),
    "qhd_set_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32]),
    "qhd_set_steps_done": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64]),
    "qhd_evolve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    "qhd_observe": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(qhd_observables),
                                   ctypes.c_void_p, ctypes.c_void_p]),
    "qhd_reset": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "qhd_readouts_static": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                           ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                           ctypes.c_double, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p]),
    "qhd_plan_points": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "qhd_kernel_timings": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(qhd_kernel_timing),
                                          ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "qhd_plan_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "qhd_spectrum": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                    ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_void_p]),
    "qhd_plan_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(qhd_class_info), ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "qhd_last_error": (ctypes.c_char_p, []),
    "qhd_version": (ctypes.c_char_p, []),
    "qhd_sno_create": (ctypes.c_int, [ctypes.POINTER(qhd_sno_desc), ctypes.POINTER(ctypes.c_void_p)]),
    "qhd_sno_param_count": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "qhd_sno_get_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "qhd_sno_set_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "qhd_sno_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                       ctypes.c_void_p]),
    "qhd_sno_backward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_double), ctypes.c_void_p, ctypes.c_void_p]),
    "qhd_sno_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_float, ctypes.c_void_p]),
    "qhd_sno_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "qhd_rqp_create": (ctypes.c_int, [ctypes.POINTER(qhd_rqp_desc), ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]),
    "qhd_rqp_set_objective": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "qhd_rqp_evolve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    "qhd_rqp_observe": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(qhd_rqp_obs),
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "qhd_rqp_reset": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "qhd_rqp_points": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "qhd_rqp_destroy": (ctypes.c_int, [ctypes.c_void_p]),
}


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libqhd.so (built by paper_2303_01471_amd/build.py).  Raises if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"HIP library not built: {path} is missing "
                               "(run __graft_entry__.build() or paper_2303_01471_amd/build.py)")
        lib = ctypes.CDLL(path)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(status: int):
    if status != QHD_OK:
        raise QHDError(status, load_library().qhd_last_error().decode())


# ------------------------------------------------------------------------------------
# C-named wrappers


def qhd_version() -> str:
    return load_library().qhd_version().decode()


def qhd_last_error() -> str:
    return load_library().qhd_last_error().decode()


def qhd_plan_create(instances: Sequence[qhd_instance], opts: Optional[qhd_plan_opts] = None) -> int:
    arr = (qhd_instance * len(instances))(*instances)
    out = ctypes.c_void_p()
    _check(load_library().qhd_plan_create(arr, len(instances),
                                          ctypes.byref(opts) if opts is not None else None,
                                          ctypes.byref(out)))
    return out.value


def qhd_set_potential(plan: int, i: int, ptr: int, on_device: bool):
    _check(load_library().qhd_set_potential(plan, i, ptr, 1 if on_device else 0))


def qhd_set_state(plan: int, i: int, ptr: int, on_device: bool):
    _check(load_library().qhd_set_state(plan, i, ptr, 1 if on_device else 0))


def qhd_set_steps_done(plan: int, i: int, j: int):
    _check(load_library().qhd_set_steps_done(plan, i, j))


def qhd_evolve(plan: int, max_steps: int, stream: int):
    _check(load_library().qhd_evolve(plan, max_steps, stream))


def qhd_reset(plan: int, stream: int):
    _check(load_library().qhd_reset(plan, stream))


def qhd_observe(plan: int, stream: int, out, rho_ptr: int, psi_ptr: int) -> int:
    """Returns the status (QHD_OK or QHD_ENUMERIC, the latter with `out` filled); raises otherwise."""
    st = load_library().qhd_observe(plan, stream, out, rho_ptr or None, psi_ptr or None)
    if st not in (QHD_OK, QHD_ENUMERIC):
        _check(st)
    return st


def qhd_readouts_static(shape: Sequence[int], count: int, psi_ptr: int, f_ptr: int, out_ptr: int,
                        box=None, radius: float = 0.1, stream: int = 0):
    """qhd_readouts_static on caller-owned device buffers; ``shape`` and ``box`` in array
    order ([y, x] or [z, y, x]); out_ptr receives ``count`` qhd_readout entries (device)."""
    nd = len(shape)
    box = box if box is not None else [(0.0, 1.0)] * nd
    n = (ctypes.c_int32 * 3)(*[int(shape[nd - 1 - a]) if a < nd else 1 for a in range(3)])
    lo = (ctypes.c_double * 3)(*[float(box[nd - 1 - a][0]) if a < nd else 0.0 for a in range(3)])
    hi = (ctypes.c_double * 3)(*[float(box[nd - 1 - a][1]) if a < nd else 1.0 for a in range(3)])
    _check(load_library().qhd_readouts_static(nd, n, lo, hi, float(radius), int(count), psi_ptr, f_ptr, out_ptr,
                                              stream))


def qhd_plan_points(plan: int) -> int:
    v = ctypes.c_int64()
    _check(load_library().qhd_plan_points(plan, ctypes.byref(v)))
    return v.value


def qhd_kernel_timings(plan: int, cap: int = 64):
    arr = (qhd_kernel_timing * cap)()
    n = ctypes.c_int32()
    _check(load_library().qhd_kernel_timings(plan, arr, cap, ctypes.byref(n)))
    return [arr[k] for k in range(min(n.value, cap))]


def qhd_plan_info(plan: int, cap: int = 16):
    arr = (qhd_class_info * cap)()
    n = ctypes.c_int32()
    g = ctypes.c_int32()
    _check(load_library().qhd_plan_info(plan, arr, cap, ctypes.byref(n), ctypes.byref(g)))
    return [arr[k] for k in range(min(n.value, cap))], g.value


def qhd_spectrum(plan: int, i: int, t: float, nev: int, krylov: int, psi_ptr: int = 0, stream: int = 0,
                 want_overlaps: bool = False, want_residuals: bool = True):
    """Returns (energies, overlaps or None, residuals or None) as numpy arrays."""
    e = np.zeros(nev)
    o = np.zeros(nev) if want_overlaps else None
    r = np.zeros(nev) if want_residuals else None
    _check(load_library().qhd_spectrum(plan, i, t, nev, krylov, psi_ptr or None, e.ctypes.data,
                                       o.ctypes.data if o is not None else None,
                                       r.ctypes.data if r is not None else None, stream))
    return e, o, r


def qhd_plan_destroy(plan: int):
    _check(load_library().qhd_plan_destroy(plan))


def qhd_sno_create(desc: qhd_sno_desc) -> int:
    out = ctypes.c_void_p()
    _check(load_library().qhd_sno_create(ctypes.byref(desc), ctypes.byref(out)))
    return out.value


def qhd_sno_param_count(sno: int) -> int:
    v = ctypes.c_int64()
    _check(load_library().qhd_sno_param_count(sno, ctypes.byref(v)))
    return v.value


def qhd_sno_get_params(sno: int, host_ptr: int):
    _check(load_library().qhd_sno_get_params(sno, host_ptr))


def qhd_sno_set_params(sno: int, host_ptr: int):
    _check(load_library().qhd_sno_set_params(sno, host_ptr))


def qhd_sno_forward(sno: int, f_ptr: int, batch: int, rho_ptr: int, stream: int):
    _check(load_library().qhd_sno_forward(sno, f_ptr, batch, rho_ptr, stream))


def qhd_sno_backward(sno: int, f_ptr: int, target_ptr: int, batch: int, grad_host_ptr: int,
                     stream: int) -> float:
    loss = ctypes.c_double()
    _check(load_library().qhd_sno_backward(sno, f_ptr, target_ptr, batch, ctypes.byref(loss),
                                           grad_host_ptr or None, stream))
    return loss.value


def qhd_sno_step(sno: int, lr: float, stream: int):
    _check(load_library().qhd_sno_step(sno, lr, stream))


def qhd_sno_destroy(sno: int):
    _check(load_library().qhd_sno_destroy(sno))


def qhd_rqp_create(desc: qhd_rqp_desc, batch: int) -> int:
    h = ctypes.c_void_p()
    _check(load_library().qhd_rqp_create(ctypes.byref(desc), batch, ctypes.byref(h)))
    return h.value


def qhd_rqp_set_objective(h: int, i: int, Q_ptr: int, b_ptr: int):
    _check(load_library().qhd_rqp_set_objective(h, i, Q_ptr, b_ptr))


def qhd_rqp_evolve(h: int, max_steps: int, stream: int):
    _check(load_library().qhd_rqp_evolve(h, max_steps, stream))


def qhd_rqp_observe(h: int, stream: int, out, marginals_ptr: int, prob_ptr: int, psi_ptr: int = 0) -> int:
    st = load_library().qhd_rqp_observe(h, stream, out, marginals_ptr or None, prob_ptr or None, psi_ptr or None)
    if st not in (QHD_OK, QHD_ENUMERIC):
        _check(st)
    return st


def qhd_rqp_reset(h: int, stream: int):
    _check(load_library().qhd_rqp_reset(h, stream))


def qhd_rqp_points(h: int) -> int:
    n = ctypes.c_int64()
    _check(load_library().qhd_rqp_points(h, ctypes.byref(n)))
    return n.value


def qhd_rqp_destroy(h: int):
    _check(load_library().qhd_rqp_destroy(h))


# ------------------------------------------------------------------------------------
# convenience layer


@dataclass
class InstanceSpec:
    """One QHD instance.  ``shape`` is in array order ([y, x] or [x]); ``box`` too."""
    shape: Sequence[int]
    nsteps: int
    dt: float
    box: Optional[Sequence[Sequence[float]]] = None
    sched: int = QHD_SCHED_NESTEROV
    sched_p: Sequence[float] = (1e-3, 0.0)
    table: Optional[np.ndarray] = None
    init: int = QHD_INIT_UNIFORM
    radius: float = 0.1
    scheme: int = QHD_SCHEME_STRANG
    model: int = QHD_MODEL_QHD

    def to_c(self, keep: list) -> qhd_instance:
        d = qhd_instance()
        nd = len(self.shape)
        box = self.box if self.box is not None else [(0.0, 1.0)] * nd
        d.ndim = nd
        for a in range(3):
            if a < nd:
                d.n[a] = int(self.shape[nd - 1 - a])
                d.lo[a] = float(box[nd - 1 - a][0])
                d.hi[a] = float(box[nd - 1 - a][1])
            else:
                d.n[a] = 1
                d.lo[a], d.hi[a] = 0.0, 1.0
        d.dt = float(self.dt)
        d.nsteps = int(self.nsteps)
        d.sched_kind = int(self.sched)
        d.sched_p[0] = float(self.sched_p[0])
        d.sched_p[1] = float(self.sched_p[1]) if len(self.sched_p) > 1 else 0.0
        if self.table is not None:
            tab = np.ascontiguousarray(self.table, dtype=np.float64).reshape(-1)
            keep.append(tab)
            d.sched_table = tab.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.init_kind = int(self.init)
        d.success_radius = float(self.radius)
        d.scheme = int(self.scheme)
        d.model = int(self.model)
        return d

    @property
    def points(self) -> int:
        return int(np.prod(self.shape))


def _stream_handle(stream) -> int:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class Plan:
    """A batch of QHD instances on the current GPU."""

    def __init__(self, specs: Sequence[InstanceSpec], flags: int = 0, norm_tolerance: float = 0.0,
                 timing_stride: int = 0, tune_cache: Optional[str] = None):
        self.specs = list(specs)
        keep: list = []
        cinst = [s.to_c(keep) for s in self.specs]
        opts = qhd_plan_opts(flags, norm_tolerance, timing_stride,
                             tune_cache.encode() if tune_cache else None)
        self.handle = qhd_plan_create(cinst, opts)
        self.points = qhd_plan_points(self.handle)
        self.offsets = np.concatenate([[0], np.cumsum([s.points for s in self.specs])]).astype(np.int64)

    # inputs -------------------------------------------------------------------------
    def set_potential(self, i: int, f):
        if hasattr(f, "data_ptr"):
            import torch
            assert f.dtype == torch.float64 and f.is_cuda and f.is_contiguous()
            assert f.numel() == self.specs[i].points
            qhd_set_potential(self.handle, i, f.data_ptr(), True)
        else:
            a = np.ascontiguousarray(f, dtype=np.float64)
            assert a.size == self.specs[i].points
            qhd_set_potential(self.handle, i, a.ctypes.data, False)

    def set_state(self, i: int, psi):
        if hasattr(psi, "data_ptr"):
            import torch
            assert psi.dtype == torch.complex64 and psi.is_cuda and psi.is_contiguous()
            assert psi.numel() == self.specs[i].points
            qhd_set_state(self.handle, i, psi.data_ptr(), True)
        else:
            a = np.ascontiguousarray(psi, dtype=np.complex64)
            assert a.size == self.specs[i].points
            qhd_set_state(self.handle, i, a.ctypes.data, False)

    def set_steps_done(self, i: int, j: int):
        qhd_set_steps_done(self.handle, i, j)

    # evolution ---------------------------------------------------------------------
    def evolve(self, max_steps: int = -1, stream=None):
        qhd_evolve(self.handle, int(max_steps), _stream_handle(stream))

    def reset(self, stream=None):
        qhd_reset(self.handle, _stream_handle(stream))

    def observe(self, stream=None, want_psi: bool = False, want_rho: bool = False):
        """Returns (list of dicts, psi tensor or None, rho tensor or None, status)."""
        import torch
        out = (qhd_observables * len(self.specs))()
        psi = torch.empty(self.points, dtype=torch.complex64, device="cuda") if want_psi else None
        rho = torch.empty(self.points, dtype=torch.float32, device="cuda") if want_rho else None
        st = qhd_observe(self.handle, _stream_handle(stream), out,
                         rho.data_ptr() if rho is not None else 0,
                         psi.data_ptr() if psi is not None else 0)
        res = [dict(norm=o.norm, e_f=o.e_f, success_mass=o.success_mass, f_min=o.f_min,
                    argmin_index=o.argmin_index, steps_done=o.steps_done, t=o.t) for o in out]
        return res, psi, rho, st

    def psi_of(self, psi_flat, i: int):
        a, b = int(self.offsets[i]), int(self.offsets[i + 1])
        return psi_flat[a:b].reshape(tuple(self.specs[i].shape))

    def spectrum(self, i: int, t: float, nev: int = 6, krylov: int = 200, psi=None, stream=None):
        """Lowest nev eigenvalues of H(t) of instance i (2-D), residual norms and, if a
        state psi (CUDA complex64, row-major) is given, the overlaps |<phi_n|psi>|^2."""
        if psi is not None:
            import torch
            assert psi.dtype == torch.complex64 and psi.is_cuda and psi.is_contiguous()
            assert psi.numel() == self.specs[i].points
        return qhd_spectrum(self.handle, i, float(t), nev, krylov, psi.data_ptr() if psi is not None else 0,
                            _stream_handle(stream), want_overlaps=psi is not None)

    def graph_info(self) -> dict:
        """Launch configuration chosen at plan creation (classes, graph chunk)."""
        cls, g = qhd_plan_info(self.handle)
        return dict(graph_steps=g, classes=[dict(ndim=c.ndim, n=tuple(c.n), members=c.members,
                                                 col_variant=c.col_variant, cap_row=c.grid_cap_row,
                                                 cap_col=c.grid_cap_col, tuned=bool(c.tuned),
                                                 mfma_dft=bool(c.mfma_dft),
                                                 row_points=c.row_points_per_lane,
                                                 resident=bool(c.resident)) for c in cls])

    def kernel_timings(self) -> List[dict]:
        return [dict(name=t.name.decode(), launches=t.launches, total_ms=t.total_ms, points=t.points,
                     bytes_per_point=t.bytes_per_point) for t in qhd_kernel_timings(self.handle)]

    def close(self):
        if getattr(self, "handle", None):
            qhd_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
