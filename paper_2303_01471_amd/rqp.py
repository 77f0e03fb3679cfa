"""Relaxed QHD for box-constrained quadratic programming (include/qhd_rqp.h): a thin
convenience wrapper over the C ABI in ``qhd``.  Every step runs in the HIP kernels
of libqhd.so; this module only marshals arguments and keeps buffers alive."""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np

from . import qhd as q


class RelaxedQP:
    """A batch of box-QP instances sharing the dimension d, the resolution r (r + 1
    lattice points per axis), dt, nsteps and the schedule."""

    def __init__(self, dim: int, r: int, batch: int, dt: float, nsteps: int,
                 sched: int = q.QHD_SCHED_NESTEROV, sched_p: Sequence[float] = (1e-3, 0.0),
                 table: Optional[np.ndarray] = None, min_tol: float = 1e-9):
        d = q.qhd_rqp_desc()
        d.dim, d.r, d.dt, d.nsteps = dim, r, float(dt), int(nsteps)
        d.sched_kind = int(sched)
        d.sched_p[0] = float(sched_p[0])
        d.sched_p[1] = float(sched_p[1]) if len(sched_p) > 1 else 0.0
        self._table = None
        if table is not None:
            self._table = np.ascontiguousarray(table, dtype=np.float64).reshape(-1)
            d.sched_table = self._table.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.min_tol = float(min_tol)
        self.dim, self.r, self.batch = dim, r, batch
        self.handle = q.qhd_rqp_create(d, batch)
        self.points = q.qhd_rqp_points(self.handle)

    def set_objective(self, i: int, Q, b):
        Qa = np.ascontiguousarray(Q, dtype=np.float64)
        ba = np.ascontiguousarray(b, dtype=np.float64)
        assert Qa.shape == (self.dim, self.dim) and ba.shape == (self.dim,)
        q.qhd_rqp_set_objective(self.handle, i, Qa.ctypes.data, ba.ctypes.data)

    def evolve(self, max_steps: int = -1, stream=None):
        q.qhd_rqp_evolve(self.handle, int(max_steps), q._stream_handle(stream))

    def reset(self, stream=None):
        q.qhd_rqp_reset(self.handle, q._stream_handle(stream))

    def observe(self, stream=None, want_marginals: bool = False, want_prob: bool = False, want_psi: bool = False):
        """Returns (list of dicts, marginals [batch, d, r+1] or None, prob [batch, (r+1)^d]
        or None, status), and with want_psi the state [batch, (r+1)^d] (complex64, the owed
        potential half step applied) as a fifth element; the tensors are on the GPU."""
        import torch
        out = (q.qhd_rqp_obs * self.batch)()
        marg = (torch.empty((self.batch, self.dim, self.r + 1), dtype=torch.float32, device="cuda")
                if want_marginals else None)
        prob = torch.empty((self.batch, self.points), dtype=torch.float32, device="cuda") if want_prob else None
        psi = torch.empty((self.batch, self.points), dtype=torch.complex64, device="cuda") if want_psi else None
        st = q.qhd_rqp_observe(self.handle, q._stream_handle(stream), out,
                               marg.data_ptr() if marg is not None else 0,
                               prob.data_ptr() if prob is not None else 0,
                               psi.data_ptr() if psi is not None else 0)
        res = [dict(norm=o.norm, e_f=o.e_f, p_min=o.p_min, f_min=o.f_min, argmin_index=o.argmin_index,
                    steps_done=o.steps_done, t=o.t) for o in out]
        if want_psi:
            return res, marg, prob, st, psi
        return res, marg, prob, st

    def close(self):
        if getattr(self, "handle", None):
            q.qhd_rqp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
