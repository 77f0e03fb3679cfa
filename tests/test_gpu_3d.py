"""3-D parity of the HIP path with the FP64 oracle (two passes per step: the x-pass
and the (y, z)-plane pass; the plane pass takes its direct form, rows loaded and stored
as whole tiles, for 64- and 128-point y-lines and its staged form below)."""
import numpy as np
import pytest

import qhd_inputs
from gpu_helpers import PSI_TOL, compare, spec_allowance, note, run_gpu, run_oracle
from paper_2303_01471_amd import qhd as q

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    q.load_library()


def _f3(seed, shape, box=None):
    return qhd_inputs.evaluate(qhd_inputs.draw_landscape(seed, 3, 16, 4), shape, box)


def _check(specs, fs, res, psis, label):
    for i, (spec, f) in enumerate(zip(specs, fs)):
        ref, ro = run_oracle(spec, f)
        err, nd, d_ef, d_p = compare(spec, f, res[i], psis[i], ref, ro, f"{label}[{i}]")
        assert err <= PSI_TOL
        assert abs(res[i]["norm"] - ro.norm) <= spec_allowance(spec)
        assert d_ef <= 1e-3 and d_p <= 1e-4
        assert res[i]["argmin_index"] == ro.argmin


def test_3d_shapes_against_oracle():
    note("case: 3-D shapes")
    specs = [
        q.InstanceSpec(shape=(16, 16, 16), nsteps=200, dt=2e-3),
        q.InstanceSpec(shape=(32, 16, 64), nsteps=60, dt=2e-3,
                       box=[(0.0, 0.5), (-1.0, 1.0), (0.0, 1.5)], radius=0.3),
        q.InstanceSpec(shape=(64, 32, 16), nsteps=80, dt=2e-3, sched=q.QHD_SCHED_CONST, sched_p=(0.8, 3.0)),
        q.InstanceSpec(shape=(16, 16, 16), nsteps=150, dt=2e-3),
        # 128-point z-lines (16 points per lane) on a non-square tile grid, ragged length
        q.InstanceSpec(shape=(16, 32, 128), nsteps=45, dt=2e-3),
    ]
    fs = [_f3(10 + k, s.shape, s.box) for k, s in enumerate(specs)]
    res, psis, _, st = run_gpu(specs, fs)
    assert st == q.QHD_OK
    _check(specs, fs, res, psis, "3d")


def test_3d_direct_plane_shapes_against_oracle():
    """The direct plane pass at every y-line length it takes (64, 128) against z-lines of
    16 to 128 points (8 or 16 points per lane, one to sixteen tile rows of z), in one plan
    with a staged-form shape beside them; x short so that the oracle stays quick."""
    note("case: direct plane shapes")
    specs = [
        q.InstanceSpec(shape=(16, 64, 16), nsteps=50, dt=2e-3),
        q.InstanceSpec(shape=(128, 64, 16), nsteps=30, dt=2e-3, box=[(0.0, 2.0), (-0.5, 0.5), (0.0, 1.0)],
                       radius=0.25),
        q.InstanceSpec(shape=(32, 128, 16), nsteps=40, dt=2e-3, sched=q.QHD_SCHED_CONST, sched_p=(0.6, 2.0)),
        q.InstanceSpec(shape=(64, 128, 16), nsteps=35, dt=2e-3),
        q.InstanceSpec(shape=(64, 64, 32), nsteps=25, dt=2e-3),
        q.InstanceSpec(shape=(16, 32, 16), nsteps=40, dt=2e-3),
    ]
    fs = [_f3(40 + k, s.shape, s.box) for k, s in enumerate(specs)]
    res, psis, _, st = run_gpu(specs, fs)
    assert st == q.QHD_OK
    _check(specs, fs, res, psis, "3d-direct")


def test_3d_128_cubed_batch():
    """The 3-D workload shape: 128^3 instances, dt = 2e-3, 16 random cosine terms
    with k in [-4, 4]^3; a short run the oracle can follow."""
    note("case: 128^3 x 2")
    specs = [q.InstanceSpec(shape=(128, 128, 128), nsteps=60, dt=2e-3) for _ in range(2)]
    fs = [_f3(3030 + k, s.shape) for k, s in enumerate(specs)]
    res, psis, _, st = run_gpu(specs, fs)
    assert st == q.QHD_OK
    _check(specs, fs, res, psis, "c3")


def test_3d_chunked_is_bitwise_one_shot():
    note("case: 3-D chunked")
    specs = [q.InstanceSpec(shape=(32, 32, 32), nsteps=90, dt=2e-3)]
    fs = [_f3(5, (32, 32, 32))]
    _, p1, _, _ = run_gpu(specs, fs)
    _, p2, _, _ = run_gpu(specs, fs, chunks=[7, 40])
    assert np.array_equal(p1[0], p2[0])
