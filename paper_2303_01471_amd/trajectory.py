"""Trajectory observables of one 2-D QHD run at snapshot times.

At each snapshot time t_k the run is advanced to step round(t_k / dt) and read
out (qhd_observe: norm, E[f], success mass); optionally the lowest eigenpairs
of H(t_k) are computed (qhd_spectrum) together with the probability spectrum
|<n; t_k | psi_{t_k}>|^2, the quantities the paper follows along the QHD path
(App. D: low-lying levels and energy ratio E1/E0 of H(t), and the distribution of
the state over them).  The paper's snapshot times are 0.1, 0.5, 1, 2, 5 and 10.
"""
from __future__ import annotations

from typing import Dict, List, Sequence

import numpy as np

from . import qhd as q

PAPER_SNAPSHOTS = (0.1, 0.5, 1.0, 2.0, 5.0, 10.0)


def run(spec: q.InstanceSpec, f, times: Sequence[float] = PAPER_SNAPSHOTS, nev: int = 0, krylov: int = 200,
        stream=None) -> List[Dict]:
    """Evolve one instance to each snapshot time (ascending, within its nsteps*dt)
    and return per snapshot: t, steps, the readouts and, with nev > 0, the lowest
    nev levels of H(t), their residuals and the state's weights on them."""
    import torch
    out = []
    plan = q.Plan([spec])
    try:
        plan.set_potential(0, f)
        done = 0
        for t in times:
            j = int(round(t / spec.dt))
            if j < done or j > spec.nsteps:
                raise ValueError(f"snapshot t={t} is before the previous one or after the run's end")
            plan.evolve(j - done, stream)
            done = j
            res, psi, _, st = plan.observe(stream, want_psi=nev > 0)
            rec = dict(res[0])  # norm, e_f, success_mass, f_min, argmin_index, steps_done, t
            rec.update(steps=j, status=st)
            if nev > 0:
                torch.cuda.synchronize()
                e, ov, r = plan.spectrum(0, j * spec.dt, nev=nev, krylov=krylov, psi=psi, stream=stream)
                rec.update(energies=e, weights=ov, residuals=r, ratio_e1_e0=float(e[1] / e[0]) if e[0] != 0 else None)
            out.append(rec)
    finally:
        plan.close()
    return out
