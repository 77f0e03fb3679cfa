"""Mean norm change per line transform of the HIP passes.

The bar of 1e-5 per 10^4 steps leaves 2.5e-10 per line transform (four per 2-D step).
A transform whose products carry a systematic magnitude error (e.g. a twiddle rounded
to FP32, |w| != 1 by a fixed amount) drains or inflates the norm on every call, at
~5e-8 per transform, far above that; unbiased rounding averages out.

Each case evolves a batch of random unit-norm states with a = b = 0 (CONST schedule):
every step is then F_x V F_x^{-1} with V = 1 in the row pass and F_y^{-1} K F_y with
K = 1/(n_x n_y) in the column pass (App. C.2.1, eq. prod_qhd_fft), i.e. the identity up
to rounding, through the very kernels of the QHD evolution.  Over K steps the lines of
length n_x are transformed 2K times (the first step's F_x^{-1} is skipped on the clean
state, the readout's closes the last step) and those of length n_y 2K times; the mean
relative norm change over the batch, divided by the transforms, is the bias per
transform.  1024 or more lines of every length are transformed.
"""
import numpy as np
import pytest

from gpu_helpers import note, run_gpu
from paper_2303_01471_amd import qhd as q

pytestmark = pytest.mark.gpu

BIAS_TOL = 2.5e-10
STEPS = 40


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    q.load_library()


def _bias(shape, count, seed, flags=0):
    """(mean, standard error) of the relative norm change per line transform."""
    rng = np.random.default_rng(seed)
    specs, states = [], {}
    for i in range(count):
        psi = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
        psi = (psi / np.sqrt(np.sum(np.abs(psi) ** 2))).astype(np.complex64)
        states[i] = psi
        specs.append(q.InstanceSpec(shape=shape, nsteps=STEPS, dt=1e-3, sched=q.QHD_SCHED_CONST, sched_p=(0.0, 0.0),
                                    init=q.QHD_INIT_USER))
    norm0 = np.array([np.sum(np.abs(states[i].astype(np.complex128)) ** 2) for i in range(count)])
    fs = [np.zeros(shape) for _ in range(count)]
    res, psis, _, st = run_gpu(specs, fs, states=states, flags=flags)
    assert st == q.QHD_OK
    norm = np.array([r["norm"] for r in res])
    rel = norm / norm0 - 1.0
    transforms = 2 * len(shape) * STEPS  # 2K along every axis
    return float(np.mean(rel)) / transforms, float(np.std(rel)) / transforms / np.sqrt(count)


@pytest.mark.parametrize("n", [8, 16, 32, 64, 128, 256, 512, 1024])
def test_mean_norm_change_per_transform_square(n):
    """n x n meshes: rows and columns of n points, at least 1024 of each."""
    count = max(1, 1024 // n)
    bias, err = _bias((n, n), count, 500 + n)
    note(f"  {n}x{n} x {count}: mean relative norm change per transform {bias:+.3e} (+- {err:.1e})")
    assert abs(bias) <= BIAS_TOL


@pytest.mark.parametrize("nx,ny", [(512, 8), (8, 512), (1024, 16), (16, 1024), (128, 32), (32, 128)])
def test_mean_norm_change_per_transform_rectangular(nx, ny):
    """Unequal axes, so that the row and the column transforms differ in length."""
    count = max(1, 2048 // min(nx, ny))
    bias, err = _bias((ny, nx), count, 700 + nx + ny)
    note(f"  {ny}x{nx} (y, x) x {count}: mean relative norm change per transform {bias:+.3e} (+- {err:.1e})")
    assert abs(bias) <= BIAS_TOL


@pytest.mark.parametrize("shape", [(128, 128, 128), (32, 64, 16)])
def test_mean_norm_change_per_transform_3d(shape):
    """3-D meshes: the x-pass and the (y, z)-plane pass (2K transforms along each axis)."""
    count = 1 if shape[0] == 128 else 4
    bias, err = _bias(shape, count, 900 + shape[2])
    note(f"  {shape} x {count}: mean relative norm change per transform {bias:+.3e} (+- {err:.1e})")
    assert abs(bias) <= BIAS_TOL
