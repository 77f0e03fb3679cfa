"""Classes of narrow meshes, several instances each, against the FP64 oracle.

The row passes read the instance record once per wavefront: a wavefront's rows (64 P / n_x
of them, aligned) lie in one instance whenever they are at most 8, the smallest mesh size.
The column passes do the same per 8-line item, and the 512-point column pass loads the next
tile column while it transforms the current one.  These batches put those boundaries where
they are tightest: n_y = 8 under 64- and 512-point rows (a wavefront holds exactly one
instance's rows, or two rows), and one or two tile columns per instance under 64-, 256- and
512-point columns (neighbouring items and prefetches cross instances), with uneven step
counts so that members drop out of the launches at different sub-steps."""
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


def _check(specs, seed, label):
    fs = [qhd_inputs.landscape_grid(seed + k, s.shape) for k, s in enumerate(specs)]
    res, psis, _, st = run_gpu(specs, fs)
    assert st == q.QHD_OK
    for i, (spec, f) in enumerate(zip(specs, fs)):
        ref, ro = run_oracle(spec, f)
        err, nd, *_ = compare(spec, f, res[i], psis[i], ref, ro, f"{label}[{i}] {spec.shape}")
        assert err <= PSI_TOL and abs(res[i]["norm"] - ro.norm) <= spec_allowance(spec)


def test_qhd_narrow_mesh_classes():
    note("case: QHD classes of 64x8, 512x8, 8x64, 16x256, 16x512 meshes")
    shapes_steps = [((64, 8), (120, 97, 143)), ((512, 8), (60, 41)), ((8, 64), (110, 150, 75)),
                    ((16, 256), (50, 70, 35)), ((16, 512), (30, 45))]
    specs = [q.InstanceSpec(shape=sh, nsteps=n, dt=5e-3) for sh, ns in shapes_steps for n in ns]
    _check(specs, 500, "qhd-narrow")


def _qaa(shape, nsteps, dt, scheme):
    return q.InstanceSpec(shape=shape, nsteps=nsteps, dt=dt, model=q.QHD_MODEL_QAA, sched=q.QHD_SCHED_LINEAR,
                          sched_p=(nsteps * dt, 0.0), scheme=scheme)


@pytest.mark.parametrize("scheme", [q.QHD_SCHEME_STRANG, q.QHD_SCHEME_LEAPFROG], ids=["split", "leapfrog"])
def test_qaa_narrow_mesh_classes(scheme):
    note(f"case: QAA ({'leapfrog' if scheme == q.QHD_SCHEME_LEAPFROG else 'split step'}) classes of 64x8, 8x64")
    specs = [_qaa(sh, n, 5e-3, scheme) for sh, ns in (((64, 8), (140, 95, 120)), ((8, 64), (100, 130, 85)))
             for n in ns]
    # the leapfrog norm is not conserved exactly: it is compared with the reference's own
    _check(specs, 600, "qaa-narrow")
