"""Relaxed QHD for box-constrained QP on the GPU (include/qhd_rqp.h) against the
FP64 reference (oracle/rqp_reference.py): lattice densities and readouts for the
paper's 5-D, r = 8 setting and for lattice shapes that take the staged and the
direct axis passes at their limits (r + 1 = 2 with d = 8, r + 1 = 16), every schedule
kind, chunked runs, reset, the stationary kinetic ground state and norm drift."""
import numpy as np
import pytest

import qhd_inputs
from gpu_helpers import note
from paper_2303_01471_amd import qhd as q

pytestmark = pytest.mark.gpu

RHO_TOL = 1e-5   # |phi|^2 per lattice point (psi bar 1e-4 on amplitudes of O(0.1))
PSI_TOL = 1e-4   # phi per lattice point, element by element (the state bar of the QHD path)
OBS_TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    q.load_library()


def _ab(sched, p, table, dt):
    from oracle import rqp_reference as rq
    if sched == q.QHD_SCHED_NESTEROV:
        return lambda t: rq.nesterov_ab(t, p[0])
    if sched == q.QHD_SCHED_CONST:
        return lambda t: (p[0], p[1])
    if sched == q.QHD_SCHED_LINEAR:
        return lambda t: (1.0 - t / p[0], t / p[0])
    return lambda t: tuple(table[int(round(t / dt - 0.5))])


def _run(dim, r, probs, dt, nsteps, sched=q.QHD_SCHED_NESTEROV, p=(1e-3, 0.0), table=None, chunks=None):
    import torch
    from paper_2303_01471_amd.rqp import RelaxedQP
    h = RelaxedQP(dim, r, len(probs), dt, nsteps, sched, p, table)
    try:
        for i, (Q, b) in enumerate(probs):
            h.set_objective(i, Q, b)
        for c in chunks or []:
            h.evolve(c)
        h.evolve()
        res, marg, prob, st, psi = h.observe(want_marginals=True, want_prob=True, want_psi=True)
        torch.cuda.synchronize()
        return res, marg.cpu().numpy(), prob.cpu().numpy(), st, psi.cpu().numpy()
    finally:
        h.close()


def _check(dim, r, probs, dt, nsteps, label, **kw):
    from oracle import rqp_reference as rq
    res, marg, prob, st, psis = _run(dim, r, probs, dt, nsteps, **kw)
    assert st == q.QHD_OK
    ab = _ab(kw.get("sched", q.QHD_SCHED_NESTEROV), kw.get("p", (1e-3, 0.0)), kw.get("table"), dt)
    worst = 0.0
    for i, (Q, b) in enumerate(probs):
        f = rq.objective(Q, b, r)
        psi = rq.evolve(f, rq.initial_state(dim, r), r, dt, nsteps, ab)
        ro = rq.readout(f, psi)
        drho = float(np.max(np.abs(prob[i] - (np.abs(psi) ** 2).reshape(-1))))
        dpsi = float(np.max(np.abs(psis[i].astype(np.complex128) - psi.reshape(-1))))
        worst = max(worst, drho)
        note(f"  {label}[{i}] d={dim} r={r} steps={nsteps}: max|dpsi|={dpsi:.2e} max|drho|={drho:.2e} "
             f"|norm-1|={abs(res[i]['norm'] - 1):.2e} "
             f"|dE[f]|={abs(res[i]['e_f'] - ro['e_f']):.2e} p_min {res[i]['p_min']:.4f} (ref {ro['p_min']:.4f})")
        assert drho <= RHO_TOL and dpsi <= PSI_TOL
        assert abs(res[i]["norm"] - ro["norm"]) <= OBS_TOL and abs(res[i]["e_f"] - ro["e_f"]) <= OBS_TOL
        assert abs(res[i]["p_min"] - ro["p_min"]) <= OBS_TOL and abs(res[i]["f_min"] - ro["f_min"]) <= 1e-12
        assert np.unravel_index(res[i]["argmin_index"], f.shape) == np.unravel_index(np.argmin(f), f.shape)
        assert np.max(np.abs(marg[i] - ro["marginals"])) <= OBS_TOL
        assert res[i]["steps_done"] == nsteps and abs(res[i]["t"] - nsteps * dt) < 1e-12
    return worst


def test_paper_setting_5d_r8_against_reference():
    note("case: relaxed QHD, QP-5d recipe, r = 8 (9^5 lattice), 3 instances, 100 steps")
    _check(5, 8, qhd_inputs.qp_instances(3, 5), 1e-2, 100, "qp5d")


def test_bench_setting_full_length_amplitudes():
    """The relaxed-QP leg of the benchmark at its length: 5-D, r = 8, dt = 1e-2, 1000 steps
    (T = 10), the state compared element by element with the FP64 reference (Algorithm 2's
    relaxed QHD, App. F)."""
    note("case: relaxed QHD, QP-5d recipe, r = 8, 1 instance, 1000 steps")
    _check(5, 8, qhd_inputs.qp_instances(1, 5), 1e-2, 1000, "qp5d-full")


def test_lattice_shapes_at_the_staged_and_direct_limits():
    note("case: r + 1 = 2 with d = 8; r + 1 = 16 with d = 3; d = 1 and 2")
    _check(8, 1, qhd_inputs.qp_instances(2, 8, 7), 2e-2, 60, "np2")
    _check(3, 15, qhd_inputs.qp_instances(2, 3, 8), 5e-3, 60, "np16")
    _check(1, 12, qhd_inputs.qp_instances(3, 1, 9), 1e-2, 80, "d1")
    _check(2, 9, qhd_inputs.qp_instances(5, 2, 10), 1e-2, 80, "d2")


def test_every_schedule_kind():
    probs = qhd_inputs.qp_instances(2, 3, 11)
    _check(3, 8, probs, 1e-2, 50, "const", sched=q.QHD_SCHED_CONST, p=(0.5, 3.0))
    _check(3, 8, probs, 1e-2, 50, "linear", sched=q.QHD_SCHED_LINEAR, p=(0.5, 0.0))
    t = (np.arange(50) + 0.5) * 1e-2
    table = np.stack([0.2 + 0.1 * np.cos(t), 1.0 + t], axis=1)
    _check(3, 8, probs, 1e-2, 50, "table", sched=q.QHD_SCHED_TABLE, table=table)


def test_chunked_equals_one_shot_and_reset():
    from paper_2303_01471_amd.rqp import RelaxedQP
    probs = qhd_inputs.qp_instances(3, 4, 12)
    _, _, p1, _, s1 = _run(4, 8, probs, 1e-2, 70)
    _, _, p2, _, s2 = _run(4, 8, probs, 1e-2, 70, chunks=[1, 13, 30])
    assert np.array_equal(s1, s2)
    assert np.array_equal(p1, p2)
    h = RelaxedQP(4, 8, 3, 1e-2, 70)
    try:
        for i, (Q, b) in enumerate(probs):
            h.set_objective(i, Q, b)
        h.evolve(25)
        h.reset()
        h.evolve()
        _, _, p3, _ = h.observe(want_prob=True)
        assert np.array_equal(p1, p3.cpu().numpy())
    finally:
        h.close()


def test_kinetic_ground_state_is_stationary():
    # b = 0: the discrete Gaussian is an eigenvector of A'_d, so |phi|^2 does not move
    from oracle import rqp_reference as rq
    _, _, prob, _, _ = _run(5, 8, qhd_inputs.qp_instances(1, 5, 13), 1e-2, 200, sched=q.QHD_SCHED_CONST, p=(2.0, 0.0))
    want = (np.abs(rq.initial_state(5, 8)) ** 2).reshape(-1)
    assert np.max(np.abs(prob[0] - want)) < 1e-6


def test_norm_drift_over_two_thousand_steps():
    res, _, _, _, _ = _run(5, 8, qhd_inputs.qp_instances(8, 5, 14), 5e-3, 2000)
    drift = max(abs(r["norm"] - 1.0) for r in res)
    note(f"  relaxed QHD 9^5, 2000 steps: max |norm - 1| = {drift:.2e}")
    assert drift <= 1e-5


def test_fused_leading_axes_equal_one_pass_per_axis(monkeypatch):
    """The leading axes whose lattice fits one LDS run are applied in one pass; each axis
    rounds to FP32 on its LDS store as a separate pass does on its HBM store, so the
    states are bitwise equal (9^5: axes 1-4 fused; 16^3 and 2^8: every axis fused)."""
    cases = [(5, 8, qhd_inputs.qp_instances(4, 5, 15), 1e-2, 120),
             (3, 15, qhd_inputs.qp_instances(2, 3, 16), 5e-3, 60),
             (8, 1, qhd_inputs.qp_instances(2, 8, 17), 2e-2, 60),
             (2, 9, qhd_inputs.qp_instances(3, 2, 18), 1e-2, 50)]
    for dim, r, probs, dt, n in cases:
        monkeypatch.delenv("QHD_RQP_UNFUSED", raising=False)
        _, _, fused, _, fpsi = _run(dim, r, probs, dt, n, chunks=[7])
        monkeypatch.setenv("QHD_RQP_UNFUSED", "1")
        _, _, sep, _, spsi = _run(dim, r, probs, dt, n, chunks=[7])
        note(f"  d={dim} r={r}: fused vs per-axis max|drho| = {float(np.max(np.abs(fused - sep))):.2e}")
        assert np.array_equal(fused, sep) and np.array_equal(fpsi, spsi)
