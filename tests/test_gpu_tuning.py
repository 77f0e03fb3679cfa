"""Launch tuning and graph replay: both change how the passes are launched, never
what they compute.

* step-chunk graphs: bitwise identical to direct launches, over uneven evolve
  calls with readouts between them;
* column-pass variants chosen through the tuning cache (staged / tile-wave / split,
  grid sizes): each matches the FP64 oracle, and the split 512-point form is bitwise
  the staged one (same stages in the same precision, other lanes);
* the autotuner writes a cache entry that a later plan reads back."""
import os

import numpy as np
import pytest

import qhd_inputs
from gpu_helpers import PSI_TOL, compare, note, run_oracle
from paper_2303_01471_amd import qhd as q

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    q.load_library()


def _run(specs, fs, flags=0, chunks=(), tune_cache=None):
    import torch
    plan = q.Plan(specs, flags=flags, tune_cache=tune_cache)
    try:
        for i, f in enumerate(fs):
            plan.set_potential(i, f)
        seen = []
        for c in chunks:
            plan.evolve(c)
            res, psi, _, _ = plan.observe(want_psi=True)
            torch.cuda.synchronize()
            seen.append(psi.cpu().numpy().copy())
        plan.evolve()
        res, psi, _, st = plan.observe(want_psi=True)
        torch.cuda.synchronize()
        return res, [plan.psi_of(psi, i).cpu().numpy() for i in range(len(specs))], seen, plan.graph_info()
    finally:
        plan.close()


def test_graph_replay_is_bitwise_identical_to_direct_launches():
    note("case: graph replay vs direct launches, 2 x 128^2 + 1 x 64^2, 300 steps in uneven calls")
    specs = [q.InstanceSpec(shape=(128, 128), nsteps=300, dt=1e-3),
             q.InstanceSpec(shape=(64, 64), nsteps=300, dt=1e-3),
             q.InstanceSpec(shape=(128, 128), nsteps=300, dt=1e-3)]
    fs = [qhd_inputs.landscape_grid(s, sp.shape) for s, sp in zip((31, 32, 33), specs)]
    chunks = (100, 7, 64, 65)
    r_g, psi_g, seen_g, info_g = _run(specs, fs, chunks=chunks)
    r_d, psi_d, seen_d, info_d = _run(specs, fs, flags=q.QHD_OPT_NO_GRAPH, chunks=chunks)
    assert info_g["graph_steps"] == 64 and info_d["graph_steps"] == 0
    for a, b in zip(seen_g, seen_d):
        assert np.array_equal(a, b)
    for a, b in zip(psi_g, psi_d):
        assert np.array_equal(a, b)
    ref, ro = run_oracle(specs[0], fs[0])
    err, *_ = compare(specs[0], fs[0], r_g[0], psi_g[0], ref, ro, "graph")
    assert err <= PSI_TOL


def test_uneven_multiclass_graph_replay_is_bitwise_identical_to_direct_launches():
    """Uneven sizes and step counts in one plan (four shape classes on their own streams,
    members finishing at different steps, so the visited prefix of each class shrinks
    during the run): replays of the captured chunk, with direct chunks for the rest, give
    bitwise the states of direct launches, at every readout of a sequence of uneven calls."""
    note("case: uneven batch, graph replay vs direct launches")
    specs = [q.InstanceSpec(shape=(128, 128), nsteps=300, dt=1e-3),
             q.InstanceSpec(shape=(128, 128), nsteps=150, dt=1e-3),
             q.InstanceSpec(shape=(64, 64), nsteps=200, dt=1e-3),
             q.InstanceSpec(shape=(64, 64), nsteps=90, dt=1e-3),
             q.InstanceSpec(shape=(256, 256), nsteps=250, dt=1e-3),
             q.InstanceSpec(shape=(64, 32), nsteps=70, dt=1e-3),
             q.InstanceSpec(shape=(128, 128), nsteps=299, dt=1e-3)]
    fs = [qhd_inputs.landscape_grid(40 + k, sp.shape) for k, sp in enumerate(specs)]
    chunks = (100, 7, 64, 65)
    r_g, psi_g, seen_g, info_g = _run(specs, fs, chunks=chunks)
    r_d, psi_d, seen_d, info_d = _run(specs, fs, flags=q.QHD_OPT_NO_GRAPH, chunks=chunks)
    assert info_g["graph_steps"] == 64 and info_d["graph_steps"] == 0
    for a, b in zip(seen_g, seen_d):
        assert np.array_equal(a, b)
    for a, b in zip(psi_g, psi_d):
        assert np.array_equal(a, b)
    for a, b in zip(r_g, r_d):
        assert a == b
    for i in (0, 3, 4):
        ref, ro = run_oracle(specs[i], fs[i])
        err, *_ = compare(specs[i], fs[i], r_g[i], psi_g[i], ref, ro, f"uneven[{i}]")
        assert err <= PSI_TOL and r_g[i]["steps_done"] == specs[i].nsteps


@pytest.mark.parametrize("n,variant,cap_row,cap_col,row_pts", [(512, 2, 1024, 512, 8), (256, 1, 4096, 8192, 16),
                                                               (128, 1, 512, 1024, 8), (64, 2, 2048, 512, 8),
                                                               (512, 3, 2048, 4096, 16), (256, 3, 8192, 1024, 8),
                                                               (512, 4, 8192, 512, 16), (1024, 2, 1024, 256, 16)])
def test_cached_launch_choice_matches_oracle(tmp_path, n, variant, cap_row, cap_col, row_pts):
    import torch
    note(f"case: tuning-cache entry n={n} variant={variant} caps=({cap_row},{cap_col}) row points {row_pts}")
    nsteps = 300 if n >= 512 else 600
    specs = [q.InstanceSpec(shape=(n, n), nsteps=nsteps, dt=1e-3) for _ in range(3)]
    fs = [qhd_inputs.landscape_grid(70 + k, (n, n)) for k in range(3)]
    arch = torch.cuda.get_device_properties(0).gcnArchName.replace(" ", "_").replace(":", "_")
    cache = tmp_path / "tune.txt"
    cache.write_text(f"qhd-tune 1 {arch} {n} {n} 4 {variant} {cap_row} {cap_col} {row_pts}\n")
    res, psis, _, info = _run(specs, fs, tune_cache=str(cache))
    assert info["classes"][0]["col_variant"] == variant
    assert info["classes"][0]["row_points"] == row_pts
    assert info["classes"][0]["cap_row"] == cap_row and info["classes"][0]["cap_col"] == cap_col
    for i in (0, 2):
        ref, ro = run_oracle(specs[i], fs[i])
        err, *_ = compare(specs[i], fs[i], res[i], psis[i], ref, ro, f"variant{variant}")
        assert err <= PSI_TOL


def test_autotune_writes_cache_that_a_later_plan_reads(tmp_path):
    import torch
    cache = str(tmp_path / "tune.txt")
    specs = [q.InstanceSpec(shape=(256, 256), nsteps=50, dt=1e-3) for _ in range(16)]
    fs = [qhd_inputs.landscape_grid(90, (256, 256))] * 16
    r1, p1, _, info1 = _run(specs, fs, flags=q.QHD_OPT_AUTOTUNE, tune_cache=cache)
    text = open(cache).read()
    note("  cache: " + text.strip())
    assert text.startswith("qhd-tune 1 ") and info1["classes"][0]["tuned"]
    r2, p2, _, info2 = _run(specs, fs, tune_cache=cache)
    assert not info2["classes"][0]["tuned"]
    for k in ("col_variant", "cap_row", "cap_col", "row_points"):
        assert info1["classes"][0][k] == info2["classes"][0][k]
    # same launch choice => bitwise the same result; the uniform state was restored
    for a, b in zip(p1, p2):
        assert np.array_equal(a, b)
    assert abs(r1[0]["norm"] - 1.0) < 1e-5


def test_split_column_pass_is_bitwise_the_staged_form(tmp_path):
    """512-point columns: the split form (first forward and last inverse stage in the
    tile layout, straight from and to HBM) against the staged form, forced through the
    tuning cache, on uneven members (the visited prefix shrinks) and over several grid
    caps (items per block vary): bitwise equal states and readouts."""
    import torch
    note("case: split vs staged 512-point column pass")
    arch = torch.cuda.get_device_properties(0).gcnArchName.replace(" ", "_").replace(":", "_")
    specs = [q.InstanceSpec(shape=(512, 512), nsteps=n, dt=1e-3) for n in (120, 97, 64, 33)]
    fs = [qhd_inputs.landscape_grid(110 + k, (512, 512)) for k in range(4)]
    out = {}
    for variant, cap in ((1, 512), (4, 512), (4, 96)):
        cache = tmp_path / f"tune{variant}_{cap}.txt"
        cache.write_text(f"qhd-tune 1 {arch} 512 512 4 {variant} 8192 {cap} 8\n")
        res, psis, seen, info = _run(specs, fs, chunks=(40, 17), tune_cache=str(cache))
        assert info["classes"][0]["col_variant"] == variant
        out[(variant, cap)] = (res, psis, seen)
    ref = out[(1, 512)]
    for key in ((4, 512), (4, 96)):
        res, psis, seen = out[key]
        for a, b in zip(ref[2], seen):
            assert np.array_equal(a, b)
        for a, b in zip(ref[1], psis):
            assert np.array_equal(a, b)
        for a, b in zip(ref[0], res):
            assert a == b
