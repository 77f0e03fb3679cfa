"""Shared helpers of the GPU tests: run a batch through the C ABI and the same
batch through the FP64 oracle."""
from __future__ import annotations

import math
import sys
from typing import List, Optional, Sequence

import numpy as np

import oracle
from paper_2303_01471_amd import qhd as q

PSI_TOL = 1e-4      # max |dpsi| against the FP64 oracle (FP32 state)
NORM_TOL = 1e-5     # |sum |psi|^2 - 1| per 10k steps


def stages_of(spec) -> int:
    """Symmetric steps per step of the spec's scheme: the fourth-order composition runs
    three, every other scheme one."""
    return 3 if getattr(spec, "scheme", 0) == q.QHD_SCHEME_YOSHIDA4 else 1


def spec_allowance(spec, nsteps: Optional[int] = None) -> float:
    """drift_allowance over the spec's symmetric steps."""
    n = spec.nsteps if nsteps is None else nsteps
    return drift_allowance(n * stages_of(spec))


def drift_allowance(nsteps: int) -> float:
    """|norm - 1| a run of nsteps steps may show under the bar of 1e-5 per 10^4 steps.

    From 10^4 steps on the bar is a rate: 1e-5 * nsteps / 1e4.  A shorter run is held
    to 1e-5 * sqrt(nsteps / 1e4): the FP32 rounding of the state is unbiased and its
    norm error walks like sqrt(steps), so a walk that meets the bar at 10^4 steps stays
    under this curve, while a systematic drift at the bar's rate r per step exceeds it
    once r * nsteps > 1e-5 sqrt(nsteps / 1e4), i.e. a short run catches any bias more
    than sqrt(1e4 / nsteps) times the bar's rate (the full-length tests hold the rate
    itself)."""
    x = max(int(nsteps), 1) / 1e4
    return NORM_TOL * max(x, math.sqrt(x))


def note(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def oracle_problem(spec: q.InstanceSpec) -> oracle.Problem:
    sched = {q.QHD_SCHED_NESTEROV: oracle.SCHED_NESTEROV, q.QHD_SCHED_CONST: oracle.SCHED_CONST,
             q.QHD_SCHED_TABLE: oracle.SCHED_TABLE}[spec.sched]
    scheme = {q.QHD_SCHEME_STRANG: oracle.SCHEME_STRANG, q.QHD_SCHEME_LIE: oracle.SCHEME_LIE,
              q.QHD_SCHEME_YOSHIDA4: oracle.SCHEME_YOSHIDA4}[spec.scheme]
    return oracle.Problem(shape=tuple(spec.shape), box=spec.box, dt=spec.dt, sched=sched,
                          params=tuple(spec.sched_p), table=spec.table, radius=spec.radius, scheme=scheme)


def run_gpu(specs: Sequence[q.InstanceSpec], fs: Sequence[np.ndarray], chunks: Optional[List[int]] = None,
            states: Optional[dict] = None, steps_done: Optional[dict] = None, flags: int = 0):
    import torch
    plan = q.Plan(specs, flags=flags)
    try:
        for i, f in enumerate(fs):
            plan.set_potential(i, f)
        for i, st in (states or {}).items():
            plan.set_state(i, st)
        for i, j in (steps_done or {}).items():
            plan.set_steps_done(i, j)
        if chunks:
            for c in chunks:
                plan.evolve(c)
        plan.evolve()
        res, psi, rho, st = plan.observe(want_psi=True, want_rho=True)
        torch.cuda.synchronize()
        psis = [plan.psi_of(psi, i).cpu().numpy() for i in range(len(specs))]
        rhos = [plan.psi_of(rho, i).cpu().numpy() for i in range(len(specs))]
        return res, psis, rhos, st
    finally:
        plan.close()


def run_oracle(spec: q.InstanceSpec, f: np.ndarray, psi0=None, j0: int = 0):
    if spec.model == q.QHD_MODEL_QAA:
        # split-step QAA reference (numpy FP64); readouts by the C oracle on the same mesh
        from oracle import qaa_reference as qa
        assert spec.sched == q.QHD_SCHED_LINEAR
        assert spec.scheme in (q.QHD_SCHEME_STRANG, q.QHD_SCHEME_LEAPFROG)
        psi = qa.uniform(spec.shape) if psi0 is None else np.asarray(psi0, np.complex128)
        step = qa.evolve_leapfrog if spec.scheme == q.QHD_SCHEME_LEAPFROG else qa.evolve
        psi = step(f, psi, spec.dt, spec.nsteps - j0, spec.sched_p[0], j0=j0)
        prob = oracle.Problem(shape=tuple(spec.shape), box=spec.box, dt=spec.dt, radius=spec.radius)
        return psi, oracle.readout(prob, f, psi)
    prob = oracle_problem(spec)
    psi = oracle.uniform_state(spec.shape) if psi0 is None else np.asarray(psi0, np.complex128)
    psi = oracle.evolve(prob, f, psi, j0, spec.nsteps - j0)
    return psi, oracle.readout(prob, f, psi)


def compare(spec, f, res_i, psi_i, ref_psi, ref_ro, label=""):
    err = float(np.max(np.abs(psi_i.astype(np.complex128) - ref_psi)))
    norm_drift = abs(res_i["norm"] - 1.0)
    d_ef = abs(res_i["e_f"] - ref_ro.e_f)
    d_p = abs(res_i["success_mass"] - ref_ro.success)
    note(f"  {label} shape={tuple(spec.shape)} steps={spec.nsteps}: max|dpsi|={err:.3e} "
         f"|norm-1|={norm_drift:.3e} (oracle {abs(ref_ro.norm - 1):.1e}) |dE[f]|={d_ef:.3e} "
         f"|dP|={d_p:.3e}")
    return err, norm_drift, d_ef, d_p
