"""Host logic of the profile summaries (paper_2303_01471_amd/profiling.py): kernel-name
families and the counter-to-traffic mapping, on small synthetic counter databases of
the rocprofv3 layout."""
import sqlite3

from paper_2303_01471_amd import profiling


def test_families_of_the_pass_kernels():
    f = profiling.family_of
    assert f("void qhd::k_row_pass_2d<512, 16, 0, false>(qhd::InstDev const*)") == ("row_pass_2d/n512", 24.0)
    assert f("k_col_pass_2d<128, 8, 1, false>") == ("col_pass_2d_qaa/n128", 16.0)
    assert f("k_col_pass_tw<256, 8, true>") == ("col_pass_2d/n256", 16.0)
    assert f("k_lf_row_2d<64, 8>") == ("row_pass_2d_qaa_lf/n64", 20.0)
    assert f("k_argmin") is None
    assert f("k_col_pass_split<512, false>") == ("col_pass_2d/n512", 16.0)
    assert f("k_xpass_3d<128, false>") == ("xpass_3d/n128", 24.0)
    assert f("k_plane_direct_3d<128, 128, true>") == ("plane_3d/n128x128", 16.0)
    assert f("k_plane_3d<32, 16, false>") == ("plane_3d/n32x16", 16.0)
    assert f("k_mfma_pass_3d<0, 1>") == ("xpass_3d_mfma/n128", 24.0)
    assert f("k_mfma_pass_3d<1, 0>") == ("ypass_3d_mfma/n128", 16.0)
    assert f("k_mfma_pass_3d<2, 2>") == ("zpass_3d_mfma/n128", 16.0)
    assert profiling._short("void qhd::(anonymous namespace)::k_rqp_fused<9>(HIP_vector_type<float, 2u>*, "
                            "double const*)") == "k_rqp_fused<9>"


def _db(path, rows):
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (kernel_name text, counter_name text, value real, "
                "dispatch_id integer)")
    con.executemany("insert into counters_collection values (?, ?, ?, ?)", rows)
    con.commit()
    con.close()


def test_traffic_scales_by_the_copy_kernel_and_takes_the_main_instantiation(tmp_path):
    copy = "at::native::vectorized_elementwise_kernel<4, MulFunctor>"
    main, trial = "k_col_pass_2d<512, 8, 0, false>", "k_col_pass_2d<512, 16, 0, false>"
    pts = 1 << 20
    # the copy kernel moves 1 MiB each way; its FETCH_SIZE reads half of that (KiB units)
    fe = [(copy, "FETCH_SIZE", 512.0, 1)]
    wr = [(copy, "WRITE_SIZE", 1024.0, 1)]
    for d in range(10):  # 10 launches of the kernel the workload runs: 8 + 8 B per point
        fe.append((main, "FETCH_SIZE", pts * 8 / 1024 / 2, 100 + d))
        wr.append((main, "WRITE_SIZE", pts * 8 / 1024, 100 + d))
    fe.append((trial, "FETCH_SIZE", 1.0, 999))  # one autotuning trial of another variant
    wr.append((trial, "WRITE_SIZE", 0.0, 999))
    _db(tmp_path / "fe.db", fe)
    _db(tmp_path / "wr.db", wr)
    out = profiling.traffic(str(tmp_path / "fe.db"), str(tmp_path / "wr.db"), float(1 << 20),
                            {"col_pass_2d/n512": pts}, "h")
    assert abs(out["fetch_scale"] - 2.0) < 1e-12 and abs(out["write_scale"] - 1.0) < 1e-12
    k = out["kernels"]["col_pass_2d/n512"]
    assert k["kernel"] == main
    assert abs(k["hbm_bytes_per_point"] - 16.0) < 1e-9 and k["algorithmic_bytes_per_point"] == 16.0


def test_relaxed_qp_step_traffic_sums_the_step_kernels(tmp_path):
    """One fused pass (24 B/pt) and one axis pass (16 B/pt) per step, two steps."""
    copy = "at::native::vectorized_elementwise_kernel<4, MulFunctor>"
    pts = 1 << 16
    fe = [(copy, "FETCH_SIZE", 1024.0, 1)]
    wr = [(copy, "WRITE_SIZE", 1024.0, 1)]
    d = 10
    for step in range(2):
        fe.append(("k_rqp_fused<9>", "FETCH_SIZE", pts * 16 / 1024, d))
        wr.append(("k_rqp_fused<9>", "WRITE_SIZE", pts * 8 / 1024, d))
        fe.append(("k_rqp_axis_direct<9>", "FETCH_SIZE", pts * 8 / 1024, d + 1))
        wr.append(("k_rqp_axis_direct<9>", "WRITE_SIZE", pts * 8 / 1024, d + 1))
        fe.append(("k_rqp_matrix<9>", "FETCH_SIZE", 5.0, d + 2))  # not a pass over the lattice
        wr.append(("k_rqp_matrix<9>", "WRITE_SIZE", 1.0, d + 2))
        d += 3
    _db(tmp_path / "fe.db", fe)
    _db(tmp_path / "wr.db", wr)
    out = profiling.traffic(str(tmp_path / "fe.db"), str(tmp_path / "wr.db"), float(1 << 20),
                            {"rqp_step": pts, "rqp_bytes_per_point": 40.0}, "h")
    k = out["kernels"]["rqp_step"]
    assert k["steps"] == 2
    assert abs(k["fetch_bytes_per_point"] - 24.0) < 1e-9 and abs(k["write_bytes_per_point"] - 16.0) < 1e-9
    assert abs(k["hbm_bytes_per_point"] - 40.0) < 1e-9 and k["algorithmic_bytes_per_point"] == 40.0


def test_isolated_dispatches_are_those_that_overlap_no_other(tmp_path):
    con = sqlite3.connect(tmp_path / "k.db")
    con.execute('create table kernels (name text, start integer, "end" integer, duration integer, grid_x integer, '
                'grid_y integer, grid_z integer)')
    rows = [("a", 0, 10, 64), ("b", 5, 12, 8), ("a", 20, 30, 64), ("c", 30, 35, 8), ("a", 40, 50, 8), ("b", 45, 60, 8),
            ("c", 55, 58, 8), ("a", 70, 90, 64)]
    con.executemany("insert into kernels values (?, ?, ?, ?, ?, 1, 1)", [(n, s_, e, e - s_, g) for n, s_, e, g in rows])
    con.commit()
    con.close()
    st = {r["kernel"]: r for r in profiling.kernel_stats(str(tmp_path / "k.db"), isolated=True)}
    # alone: a at [20, 30) and [70, 90), c at [30, 35) (touching ends do not overlap)
    assert st["a"]["calls"] == 2 and st["a"]["mean_ns"] == 15
    assert st["c"]["calls"] == 1 and st["c"]["mean_ns"] == 5
    assert "b" not in st
    every = {r["kernel"]: r for r in profiling.kernel_stats(str(tmp_path / "k.db"))}
    assert every["a"]["calls"] == 4 and every["b"]["calls"] == 2
    big = {r["kernel"]: r for r in profiling.kernel_stats(str(tmp_path / "k.db"), largest_grid=True)}
    assert big["a"]["calls"] == 3 and big["a"]["mean_ns"] == 40 / 3  # the grid-64 dispatches
    assert big["c"]["calls"] == 2
