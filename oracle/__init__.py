"""FP64 CPU oracle for the QHD split-operator evolution (ctypes binding).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the HIP library (``paper_2303_01471_amd``); the two sides meet only through
the seeded input arrays of the top-level ``qhd_inputs`` module.

The arithmetic lives in ``qhd_oracle.c`` (plain C, FP64, OpenMP over lines);
this module only marshals numpy arrays.  Section/equation citations for every
step are in the C source.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qhd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

SCHED_NESTEROV, SCHED_CONST, SCHED_TABLE = 0, 1, 2
SCHEME_STRANG, SCHEME_LIE, SCHEME_YOSHIDA4 = 0, 1, 2

# planted mistakes (tests only); must match the MUT_* codes in qhd_oracle.c
MUTATIONS = {
    "drop_half_in_lambda": 1,
    "kinetic_sign": 2,
    "freq_no_wrap": 3,
    "swap_axis_length": 4,
    "left_end_coeff": 5,
    "no_ifft_scale": 6,
    "potential_sign": 7,
    "one_half_step": 8,
    "ef_unnormalised": 9,
    "success_wrap": 10,
    "twiddle_conj": 11,
}


def build(force: bool = True) -> str:
    """Compile qhd_oracle.c into liboracle.so (gcc, -O2, OpenMP, IEEE FP64)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp", "-fPIC", "-shared",
             "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Desc(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("n", ctypes.c_int32 * 3),
        ("lo", ctypes.c_double * 3),
        ("hi", ctypes.c_double * 3),
        ("dt", ctypes.c_double),
        ("sched", ctypes.c_int32),
        ("scheme", ctypes.c_int32),
        ("p", ctypes.c_double * 2),
        ("table", ctypes.POINTER(ctypes.c_double)),
        ("table_len", ctypes.c_int64),
        ("radius", ctypes.c_double),
        ("mutation", ctypes.c_int32),
        ("threads", ctypes.c_int32),
    ]


class _Obs(ctypes.Structure):
    _fields_ = [
        ("norm", ctypes.c_double),
        ("e_f", ctypes.c_double),
        ("success", ctypes.c_double),
        ("f_min", ctypes.c_double),
        ("argmin", ctypes.c_int64),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_fft.argtypes = [ctypes.POINTER(_Desc), dp, ctypes.c_int]
        lib.oracle_evolve.argtypes = [ctypes.POINTER(_Desc), dp, dp, ctypes.c_int64, ctypes.c_int64]
        lib.oracle_readout.argtypes = [ctypes.POINTER(_Desc), dp, dp, ctypes.POINTER(_Obs), dp]
        lib.oracle_uniform_state.argtypes = [ctypes.POINTER(_Desc), dp]
        lib.oracle_max_threads.argtypes = []
        for fn in (lib.oracle_fft, lib.oracle_evolve, lib.oracle_readout,
                   lib.oracle_uniform_state, lib.oracle_max_threads):
            fn.restype = ctypes.c_int
        _lib = lib
    return _lib


@dataclass
class Problem:
    """One QHD instance as the oracle sees it.

    ``shape`` is given in array order (slowest axis first, x last), matching a
    C-contiguous numpy array ``f[..., y, x]``; ``box`` lists (lo, hi) per array
    axis in the same order.
    """
    shape: Sequence[int]
    box: Optional[Sequence[Sequence[float]]] = None
    dt: float = 1e-3
    sched: int = SCHED_NESTEROV
    params: Sequence[float] = (1e-3, 0.0)
    table: Optional[np.ndarray] = None
    scheme: int = SCHEME_STRANG
    radius: float = 0.1
    mutation: int = 0
    threads: int = 0
    _keep: list = field(default_factory=list, repr=False)

    def desc(self) -> _Desc:
        d = _Desc()
        nd = len(self.shape)
        if nd < 1 or nd > 3:
            raise ValueError("ndim must be 1, 2 or 3")
        box = self.box if self.box is not None else [(0.0, 1.0)] * nd
        d.ndim = nd
        # oracle axis 0 = fastest = last numpy axis
        for a in range(3):
            if a < nd:
                d.n[a] = int(self.shape[nd - 1 - a])
                d.lo[a] = float(box[nd - 1 - a][0])
                d.hi[a] = float(box[nd - 1 - a][1])
            else:
                d.n[a] = 1
                d.lo[a] = 0.0
                d.hi[a] = 1.0
        d.dt = float(self.dt)
        d.sched = int(self.sched)
        d.scheme = int(self.scheme)
        d.p[0] = float(self.params[0])
        d.p[1] = float(self.params[1]) if len(self.params) > 1 else 0.0
        if self.table is not None:
            tab = np.ascontiguousarray(self.table, dtype=np.float64).reshape(-1)
            self._keep = [tab]
            d.table = tab.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            d.table_len = tab.size // 2
        else:
            d.table = ctypes.POINTER(ctypes.c_double)()
            d.table_len = 0
        d.radius = float(self.radius)
        d.mutation = int(self.mutation)
        d.threads = int(self.threads)
        return d


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _as_interleaved(psi: np.ndarray) -> np.ndarray:
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    return psi


def fft(psi: np.ndarray, sign: int = -1, box=None) -> np.ndarray:
    """Unnormalised DFT along every axis, X_k = sum_m x_m exp(sign 2 pi i m.k / N)."""
    out = _as_interleaved(psi).copy()
    prob = Problem(shape=out.shape, box=box)
    d = prob.desc()
    rc = _load().oracle_fft(ctypes.byref(d), _dp(out.view(np.float64)), int(sign))
    if rc != 0:
        raise ValueError("oracle_fft rejected its arguments")
    return out


def uniform_state(shape) -> np.ndarray:
    out = np.empty(tuple(shape), dtype=np.complex128)
    d = Problem(shape=shape).desc()
    if _load().oracle_uniform_state(ctypes.byref(d), _dp(out.view(np.float64))) != 0:
        raise ValueError("oracle_uniform_state rejected its arguments")
    return out


def evolve(prob: Problem, f: np.ndarray, psi: np.ndarray, j0: int = 0,
           nsteps: int = 1) -> np.ndarray:
    """Return psi advanced through global steps j0 .. j0+nsteps-1 (copy)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = _as_interleaved(psi).copy()
    if f.shape != tuple(prob.shape) or out.shape != tuple(prob.shape):
        raise ValueError("f / psi shape does not match the problem")
    d = prob.desc()
    rc = _load().oracle_evolve(ctypes.byref(d), _dp(f), _dp(out.view(np.float64)),
                               int(j0), int(nsteps))
    if rc != 0:
        raise ValueError("oracle_evolve rejected its arguments")
    return out


@dataclass
class Readout:
    norm: float
    e_f: float
    success: float
    f_min: float
    argmin: int
    rho: Optional[np.ndarray] = None


def readout(prob: Problem, f: np.ndarray, psi: np.ndarray, want_rho: bool = False) -> Readout:
    f = np.ascontiguousarray(f, dtype=np.float64)
    psi = _as_interleaved(psi)
    o = _Obs()
    rho = np.empty(prob.shape, dtype=np.float64) if want_rho else None
    d = prob.desc()
    rc = _load().oracle_readout(ctypes.byref(d), _dp(f), _dp(psi.view(np.float64)),
                                ctypes.byref(o),
                                _dp(rho) if rho is not None else ctypes.POINTER(ctypes.c_double)())
    if rc != 0:
        raise ValueError("oracle_readout rejected its arguments")
    return Readout(o.norm, o.e_f, o.success, o.f_min, int(o.argmin), rho)


def run(prob: Problem, f: np.ndarray, nsteps: int, psi0: Optional[np.ndarray] = None):
    """Uniform (or given) initial state -> nsteps steps -> (psi_T, readout)."""
    psi = uniform_state(prob.shape) if psi0 is None else np.asarray(psi0, dtype=np.complex128)
    psi = evolve(prob, f, psi, 0, nsteps)
    return psi, readout(prob, f, psi, want_rho=False)


def max_threads() -> int:
    return int(_load().oracle_max_threads())
