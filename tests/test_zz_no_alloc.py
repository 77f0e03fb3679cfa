"""qhd_readouts_static, the allocation-free readouts entry point, against the readouts
of qhd_observe on the very same states: two calls in a row through the C ABI, the
second with a smaller input (fewer and smaller instances), each compared with its own
plan's readouts.  x* and f(x*) must be equal; the FP64 sums agree to rounding (the two
sides add the same FP64 terms in different orders)."""
import ctypes

import numpy as np
import pytest

import qhd_inputs
from gpu_helpers import note
from paper_2303_01471_amd import qhd as q

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    q.load_library()


def _plan_and_static(shape, steps, seed, box=None, radius=0.1):
    import torch
    specs = [q.InstanceSpec(shape=shape, nsteps=n, dt=1e-3, box=box, radius=radius) for n in steps]
    fs = [qhd_inputs.landscape_grid(seed + k, shape, box=box) for k in range(len(specs))]
    plan = q.Plan(specs)
    try:
        for i, f in enumerate(fs):
            plan.set_potential(i, f)
        plan.evolve()
        res, psi, _, st = plan.observe(want_psi=True)
        assert st == q.QHD_OK
        stream = torch.cuda.current_stream()
        f_dev = torch.from_numpy(np.concatenate([f.reshape(-1) for f in fs])).cuda()
        out = torch.zeros(len(specs) * ctypes.sizeof(q.qhd_readout), dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        q.qhd_readouts_static(shape, len(specs), psi.data_ptr(), f_dev.data_ptr(), out.data_ptr(), box=box,
                              radius=radius, stream=stream.cuda_stream)
        torch.cuda.synchronize()
        raw = out.cpu().numpy().tobytes()
        got = (q.qhd_readout * len(specs)).from_buffer_copy(raw)
        return res, got
    finally:
        plan.close()


def _compare(res, got, label):
    for i, (r, g) in enumerate(zip(res, got)):
        note(f"  {label}[{i}]: norm {r['norm']:.15f} / {g.norm:.15f}, E[f] {r['e_f']:.12f} / {g.e_f:.12f}, "
             f"P {r['success_mass']:.12f} / {g.success_mass:.12f}, x* {r['argmin_index']} / {g.argmin_index}")
        assert g.argmin_index == r["argmin_index"] and g.f_min == r["f_min"]
        assert abs(g.norm - r["norm"]) <= 1e-13 * r["norm"]
        assert abs(g.e_f - r["e_f"]) <= 1e-12 * max(1.0, abs(r["e_f"]))
        assert abs(g.success_mass - r["success_mass"]) <= 1e-12


def test_static_readouts_match_observe_on_two_calls_in_a_row():
    note("case: static readouts, 5 x 256^2 then 3 x 64x128 (anisotropic box)")
    res1, got1 = _plan_and_static((256, 256), [300, 250, 200, 150, 100], 900)
    _compare(res1, got1, "first")
    box = [(0.0, 1.0), (-0.5, 1.5)]
    res2, got2 = _plan_and_static((64, 128), [200, 120, 80], 950, box=box, radius=0.3)
    _compare(res2, got2, "second")


def test_static_readouts_one_dimensional_and_three_dimensional():
    note("case: static readouts, 4 x 1-D 512 and 2 x 32^3")
    res, got = _plan_and_static((512,), [100, 90, 80, 70], 960)
    _compare(res, got, "1d")
    res, got = _plan_and_static((32, 32, 32), [40, 30], 970)
    _compare(res, got, "3d")


def test_static_readouts_reject_sizes_beyond_the_scratch():
    import torch
    dummy = torch.zeros(16, dtype=torch.float64, device="cuda")
    with pytest.raises(q.QHDError) as ei:
        q.qhd_readouts_static((1024, 1024), q.QHD_STATIC_MAX_LINES // 1024 + 1, dummy.data_ptr(), dummy.data_ptr(),
                              dummy.data_ptr())
    assert ei.value.status == q.QHD_EINVAL and "static scratch" in str(ei.value)
