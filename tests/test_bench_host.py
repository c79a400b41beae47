"""Host logic of the benchmark's measurement (CPU): the zero-start block counts, the
algorithmic bytes it assigns to a traced smoother dispatch, the calibration of the HBM
counters by the copy probe, and the source digest that voids a stale measurement."""
import csv
import json
import math
import os

import pytest

import bench
import synth


def _column_colour(i, j):
    return (i % 2) + 2 * (j % 2)


def test_zero_start_block_counts_follow_from_the_stencil():
    """After a line sweep from zero, the columns of a colour read only the neighbouring
    columns swept before them (3 blocks each: the vertex below, level, above); counted
    here over the 8 neighbouring columns of a column of every colour."""
    counts = []
    for cc in range(4):
        i, j = cc & 1, cc >> 1
        earlier = sum(1 for dx in (-1, 0, 1) for dy in (-1, 0, 1)
                      if (dx or dy) and _column_colour(i + dx + 2, j + dy + 2) < cc)
        counts.append(3 * earlier)
    assert tuple(counts) == bench.ZERO_START_BLOCKS


def test_levels_halve_the_intervals():
    wl = synth.workload("qmc512_mixedres")
    lv = bench._levels(wl)
    assert lv[:4] == [(33, 33, 9), (17, 17, 5), (9, 9, 3), (5, 5, 2)]
    assert lv[-6:] == [(129, 129, 33), (65, 65, 17), (33, 33, 9), (17, 17, 5), (9, 9, 3),
                       (5, 5, 2)]


def _unique_sweep_key(sweep, nc, nz, cols):
    keys = [k for k, v in sweep.items() if (nc, nz) in v and k[2] == cols and len(v) == 1]
    assert keys, (nc, nz, cols)
    return keys[0]


@pytest.mark.parametrize("t,m,zc,tb,mb", [("float", "float", -1, 4, 4),
                                          ("double", "double", -1, 8, 8),
                                          ("float", "float", 2, 4, 4),
                                          ("float", "_Float16", 3, 4, 2)])
def test_dispatch_bytes_of_a_traced_line_sweep(t, m, zc, tb, mb):
    """A dispatch named as rocprofv3 prints it, on the 129x129x33 grid (the column colour
    the sweep form belongs to), 32 columns per workgroup, 3 active samples: per vertex of
    the colour's columns the blocks read (4 values each) plus 16 vector values."""
    wl = synth.workload("qmc512_mixedres")
    sweep, resid = bench._line_tables(wl)
    cc = max(zc, 0)
    nc, nz = (65 - (cc & 1)) * (65 - (cc >> 1)), 33
    bx, wx, cols = _unique_sweep_key(sweep, nc, nz, 32)
    assert (bx, wx) == (math.ceil(nc / 32), 256)
    name = f"void edf::k_line_sweep<{t}, {m}, true, {zc}, 32>(edf::Geom, {t} const*, int)"
    nb = 24 if zc < 0 else bench.ZERO_START_BLOCKS[zc]
    got = bench._dispatch_bytes(name, bx, wx, bx * wx, 3, sweep, resid)
    assert got == 3 * nc * nz * (4 * (nb + 1) * mb + 16 * tb)


def test_dispatch_bytes_ignore_other_kernels_and_ambiguous_grids():
    wl = synth.workload("qmc512_mixedres")
    sweep, resid = bench._line_tables(wl)
    assert bench._dispatch_bytes("void edf::k_jx<1>(edf::Geom)", 1, 256, 256, 1, sweep,
                                 resid) is None
    ambiguous = [k for k, v in sweep.items() if len(v) > 1 and k[1] == 256]
    if ambiguous:
        bx, wx, cols = ambiguous[0]
        name = f"void edf::k_line_sweep<float, float, true, -1, {cols}>(edf::Geom)"
        assert bench._dispatch_bytes(name, bx, wx, bx * wx, 1, sweep, resid) is None


def _write_run(d, dispatches, counters):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_kernel_trace.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp",
                    "Grid_Size_X", "Workgroup_Size_X", "Grid_Size_Y"])
        for row in dispatches:
            w.writerow(row)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Counter_Name", "Counter_Value"])
        for di, v in counters.items():
            w.writerow([di, "C", v])


def test_counter_summary_is_calibrated_by_the_isolated_copy_probe(tmp_path):
    """A sweep dispatch before the probe, the probe (a 1 GiB copy alone in 0.2 s of idle
    time either side; FETCH_SIZE counts it as 524,288 KiB, WRITE_SIZE as 1,048,576 KiB),
    then two sweep dispatches and another kernel: only the two count, scaled by 2 and 1."""
    wl = synth.workload("qmc512_mixedres")
    sweep, _ = bench._line_tables(wl)
    nc, nz = 65 * 65, 33
    bx, wx, cols = _unique_sweep_key(sweep, nc, nz, 32)
    name = "void edf::k_line_sweep<float, float, true, -1, 32>(edf::Geom, float const*)"
    s = 10 ** 9  # ns
    disp = [(1, name, 0, s // 10, bx * wx, wx, 8),
            (2, "__amd_rocclr_copyBuffer", 2 * s, 2 * s + s // 100, 4096, 256, 1),
            (3, name, 3 * s, 3 * s + s // 1000, bx * wx, wx, 8),
            (4, "void edf::k_restrict<float>(edf::Geom)", 3 * s + s // 500, 3 * s + s // 400,
             256, 256, 8),
            (5, name, 3 * s + s // 100, 3 * s + s // 90, bx * wx, wx, 16)]
    alg = [8 * nc * nz * 464, 16 * nc * nz * 464]
    fetch = {1: 7.0, 2: 524288.0, 3: 0.55 * alg[0] / 1024, 4: 3.0, 5: 0.5 * alg[1] / 1024}
    write = {1: 7.0, 2: 1048576.0, 3: 0.02 * alg[0] / 1024, 4: 3.0, 5: 0.01 * alg[1] / 1024}
    _write_run(str(tmp_path / "F"), disp, fetch)
    _write_run(str(tmp_path / "W"), disp, write)
    rec = bench.summarise_counters(str(tmp_path / "F"), str(tmp_path / "W"), wl, "mixed", 1,
                                   "cmd")
    assert rec["FETCH_SIZE"]["scale"] == pytest.approx(2.0)
    assert rec["WRITE_SIZE"]["scale"] == pytest.approx(1.0)
    a = rec["all"]
    assert a["dispatches"] == 2
    assert a["algorithmic_bytes_per_dispatch"] == pytest.approx(sum(alg) / 2)
    hbm = 2.0 * (0.55 * alg[0] + 0.5 * alg[1]) + (0.02 * alg[0] + 0.01 * alg[1])
    assert a["ratio"] == pytest.approx(hbm / sum(alg))
    # both launches exceed 256 MiB of algorithmic bytes
    assert rec["large"]["dispatches"] == 2


def test_counter_summary_needs_an_isolated_probe(tmp_path):
    wl = synth.workload("qmc512_mixedres")
    name = "void edf::k_line_sweep<float, float, true, -1, 32>(edf::Geom)"
    disp = [(1, name, 0, 100, 256, 256, 1),
            (2, "__amd_rocclr_copyBuffer", 200, 300, 4096, 256, 1),  # no idle time around it
            (3, name, 400, 500, 256, 256, 1)]
    _write_run(str(tmp_path / "F"), disp, {1: 1.0, 2: 1.0, 3: 1.0})
    _write_run(str(tmp_path / "W"), disp, {1: 1.0, 2: 1.0, 3: 1.0})
    with pytest.raises(SystemExit):
        bench.summarise_counters(str(tmp_path / "F"), str(tmp_path / "W"), wl, "mixed", 1, "c")


def _fake_root(tmp_path, body):
    csrc = tmp_path / "paper_1906_01632_amd" / "csrc"
    csrc.mkdir(parents=True, exist_ok=True)
    for name in bench.KERNEL_SOURCES[1]:
        (csrc / name).write_text(body)
    return str(tmp_path)


def test_digest_ignores_comments_and_spacing_but_not_code(tmp_path, monkeypatch):
    code = "int f(int a) {\n  return a + 1;  // one more\n}\n/* block */\n"
    monkeypatch.setattr(bench, "ROOT", _fake_root(tmp_path / "a", code))
    d0 = bench.kernel_digest(bench.KERNEL_SOURCES[1])
    monkeypatch.setattr(bench, "ROOT", _fake_root(tmp_path / "b", "int f(int a)   {\n"
                                                  "  // reworded\n  return a + 1;\n}\n"))
    assert bench.kernel_digest(bench.KERNEL_SOURCES[1]) == d0
    monkeypatch.setattr(bench, "ROOT", _fake_root(tmp_path / "c",
                                                  "int f(int a) { return a + 2; }"))
    assert bench.kernel_digest(bench.KERNEL_SOURCES[1]) != d0


def test_measured_traffic_is_void_once_the_smoother_changes(tmp_path, monkeypatch):
    root = _fake_root(tmp_path, "int g() { return 0; }")
    monkeypatch.setattr(bench, "ROOT", root)
    rec = {"smoother": 1, "workload": "qmc512_mixedres",
           "kernel_sources_sha256": bench.kernel_digest(bench.KERNEL_SOURCES[1]),
           "precisions": {"mixed": {"large": {"ratio": 1.05}}}}
    os.makedirs(os.path.join(root, "profiles"))
    with open(os.path.join(root, "profiles", "smoother_traffic.json"), "w") as f:
        json.dump(rec, f)
    assert bench.measured_traffic(1, "qmc512_mixedres", "mixed") == {"large": {"ratio": 1.05}}
    assert bench.measured_traffic(1, "mixed257", "mixed") is None
    (tmp_path / "paper_1906_01632_amd" / "csrc" / "line_kernels.hip").write_text(
        "int g() { return 1; }")
    assert bench.measured_traffic(1, "qmc512_mixedres", "mixed") is None


def test_committed_traffic_matches_the_committed_smoother():
    """The ratios in profiles/ were taken on the smoother code in the tree."""
    assert bench.measured_traffic(1, "qmc512_mixedres", "mixed") is not None
    assert bench.measured_traffic(1, "qmc512_mixedres", "f64") is not None


def test_trace_summary_selects_the_leg_and_counts_busy_time_once(tmp_path):
    """Two marked ranges of timed steps; the summary of the second counts only its
    kernels, overlapping kernels once in the busy time, and gives the matrix-free product
    (launched as tiles of 15 x 15 vertex columns times segments of 8 vertices, 256 threads
    each) its 80 B per vertex of the 129x129x33 group."""
    wl = synth.workload("qmc512_mixedres")
    d = tmp_path / "trace"
    d.mkdir()
    us = 1000  # ns
    jx_grid = 9 * 9 * 5 * 256
    kernels = [  # id, name, start, end, grid x, workgroup x, grid y
        (1, "void edf::k_bicg_p(unsigned long)", 10 * us, 20 * us, 256, 256, 4),
        (2, "void edf::k_bicg_p(unsigned long)", 110 * us, 130 * us, 256, 256, 4),
        (3, "void edf::k_jx<1>(edf::Geom, edf::Phys)", 120 * us, 160 * us, jx_grid, 256, 2),
        (4, "void edf::k_bicg_s(unsigned long)", 170 * us, 180 * us, 256, 256, 4),
        (5, "void edf::k_bicg_s(unsigned long)", 300 * us, 310 * us, 256, 256, 4)]
    with open(d / "t_kernel_trace.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp",
                    "Grid_Size_X", "Workgroup_Size_X", "Grid_Size_Y"])
        w.writerows(kernels)
    with open(d / "t_marker_api_trace.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Function", "Start_Timestamp", "End_Timestamp"])
        w.writerow(["timed steps", 0, 50 * us])
        w.writerow(["timed steps", 100 * us, 200 * us])
    out = bench.summarise_trace(str(d), 1, wl)
    assert "timed-steps range 1 of 2" in out
    # busy: [110, 160] and [170, 180] us = 60 us of a 100 us range
    assert "GPU busy 0.1 ms (60.0 %)" in out
    assert "| `k_bicg_p` | 1 |" in out and "| `k_bicg_s` | 1 |" in out
    row = [l for l in out.split("\n") if l.startswith("| k_jx (finest grids)")]
    assert len(row) == 1
    cells = [c.strip() for c in row[0].split("|")]
    assert cells[2] == "1" and float(cells[3]) == pytest.approx(40.0)
    assert float(cells[4]) == pytest.approx(bench.JX_BYTES * 129 * 129 * 33 * 2 / 1e6, rel=1e-3)


def test_mangled_fp16_instances_read_as_their_template_arguments():
    """rocprofv3 prints the _Float16 instances of the line kernels mangled."""
    assert bench._readable_name(
        "_ZN3edf12k_line_sweepIfDF16_Lb1ELin1ELi32EEEvNS_4GeomEiPKT0_PKT_S7_PS5_PKiSA_") == \
        "void edf::k_line_sweep<float, _Float16, true, -1, 32>()"
    assert bench._readable_name(
        "_ZN3edf12k_line_sweepIfDF16_Lb0ELi3ELi8EEEvNS_4GeomEiPKT0_PKT_S7_PS5_PKiSA_") == \
        "void edf::k_line_sweep<float, _Float16, false, 3, 8>()"
    assert bench._readable_name(
        "_ZN3edf13k_line_smoothIfDF16_Lb1ELi2EEEvNS_4GeomEiPKT0_PKT_S7_PS5_PKiSA_") == \
        "void edf::k_line_smooth<float, _Float16, true, 2>()"
    assert bench._readable_name(
        "_ZN3edf18k_line_residual_zsIfDF16_Lb0EEEvNS_4GeomEPKT0_PKT_S7_PS5_PKiSA_") == \
        "void edf::k_line_residual_zs<float, _Float16, false>()"
    plain = "void edf::k_line_sweep<float, float, true, -1, 32>(edf::Geom)"
    assert bench._readable_name(plain) == plain


def _table_runs(tmp_path, sweep_names):
    wl = synth.workload("qmc512_mixedres")
    sweep, _ = bench._line_tables(wl)
    nc, nz = 65 * 65, 33
    bx, wx, cols = _unique_sweep_key(sweep, nc, nz, 32)
    s = 10 ** 9
    jx_grid = 9 * 9 * 5 * 256
    disp = [(1, "__amd_rocclr_copyBuffer", s, s + s // 100, 4096, 256, 1)]
    fetch, write = {1: 524288.0}, {1: 1048576.0}
    t = 2 * s
    for n, name in enumerate(sweep_names):
        disp.append((2 + n, name, t, t + s // 1000, bx * wx, wx, 8))
        fetch[2 + n], write[2 + n] = 400000.0 * (n + 1), 10000.0
        t += s // 100
    disp.append((9, "void edf::k_jx<1>(edf::Geom, edf::Phys)", t, t + s // 2000, jx_grid, 256, 4))
    fetch[9], write[9] = 300000.0, 40000.0
    _write_run(str(tmp_path / "F"), disp, fetch)
    _write_run(str(tmp_path / "W"), disp, write)
    return wl, nc, nz


def test_counter_table_rows_and_the_matrix_free_product(tmp_path):
    f32 = "void edf::k_line_sweep<float, float, true, -1, 32>(edf::Geom)"
    wl, nc, nz = _table_runs(tmp_path, [f32, f32])
    out = bench.counter_table(str(tmp_path / "F"), str(tmp_path / "W"), wl)
    lines = out.split("\n")
    assert lines[0] == "fetch probe dispatches 1 KiB 524288.0"
    assert "probe scales: fetch 2.000, write 1.000" in lines
    row = [l for l in lines if l.startswith("| k_line_sweep |")][0].split("|")
    alg = 8 * nc * nz * (4 * 25 * 4 + 16 * 4)
    fetch = 2.0 * (400000.0 + 800000.0) * 1024 / 2
    write = 10000.0 * 1024
    assert int(row[2]) == 2
    assert float(row[3]) == pytest.approx(fetch / 1e6, abs=0.01)
    assert float(row[4]) == pytest.approx(write / 1e6, abs=0.01)
    assert float(row[5]) == pytest.approx(alg / 1e6, abs=0.01)
    assert float(row[6]) == pytest.approx((fetch + write) / alg, abs=1e-3)
    assert any(l.startswith("| k_line_sweep (>256MiB) | 2 |") for l in lines)
    jx = [l for l in lines if l.startswith("k_jx fetch grid 103680 (549153 vertices)")]
    assert len(jx) == 1
    assert f"algorithmic {bench.JX_BYTES * 549153 * 4 / 1e6:.1f} MB per dispatch" in jx[0]
    assert f"counted {2.0 * 300000.0 * 1024 / 1e6:.1f} MB" in jx[0]


def test_counter_table_by_matrix_type(tmp_path):
    f16 = "_ZN3edf12k_line_sweepIfDF16_Lb1ELin1ELi32EEEvNS_4GeomEiPKT0_PKT_S7_PS5_PKiSA_"
    f32 = "void edf::k_line_sweep<float, float, true, -1, 32>(edf::Geom)"
    wl, nc, nz = _table_runs(tmp_path, [f16, f32])
    out = bench.counter_table(str(tmp_path / "F"), str(tmp_path / "W"), wl, by_matrix=True)
    rows = {l.split("|")[1].strip(): l.split("|") for l in out.split("\n")
            if l.startswith("| k_")}
    assert set(rows) == {"k_line_sweep (FP16 matrix)", "k_line_sweep (FP32 matrix)", "k_jx"}
    for key, mb, counted in (("k_line_sweep (FP16 matrix)", 2, 400000.0),
                             ("k_line_sweep (FP32 matrix)", 4, 800000.0)):
        r = rows[key]
        alg = 8 * nc * nz * (4 * 25 * mb + 16 * 4)
        assert float(r[6]) == pytest.approx(alg / 1e6, abs=0.1)
        assert float(r[7]) == pytest.approx((2.0 * counted + 10000.0) * 1024 / alg, abs=1e-3)
    assert rows["k_jx"][7].strip() == "-"
