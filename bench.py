#!/usr/bin/env python3
"""Throughput of the batched Elder-box time step on one MI355X.

A step is one implicit-Euler time step (Newton + BiCGStab + multigrid V-cycles)
of every sample of the workload.  `value` is sample-timesteps per second over K
timed steps; the inputs (parameter fields, states, matrices) are resident in
HBM before timing starts.  Prints one JSON line on stdout; progress goes to stderr.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "qMC sample-timesteps/s + V-cycle HBM GB/s, mixed vs FP64 at 1e-6 rel L2"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def roctx_range():
    """(push, pop) of a named roctx range, recorded by `rocprofv3 --marker-trace` in the
    clock of its kernel trace; no-ops if the marker library is absent."""
    import ctypes
    for name in ("librocprofiler-sdk-roctx.so.1", "librocprofiler-sdk-roctx.so"):
        try:
            lib = ctypes.CDLL(name)
            lib.roctxRangePushA.argtypes = [ctypes.c_char_p]
            return (lambda: lib.roctxRangePushA(b"timed steps")), (lambda: lib.roctxRangePop())
        except (OSError, AttributeError):
            continue
    return (lambda: None), (lambda: None)


# the smoother kernels, their device helpers and the structures they take: the measured
# HBM traffic per launch is reported only while their code is unchanged
KERNEL_SOURCES = {0: ("mg_kernels.hip", "fv_common.h", "edf_internal.h"),
                  1: ("line_kernels.hip", "fv_common.h", "edf_internal.h")}


def kernel_digest(names):
    """sha256 of the code of the named sources: comments and blank space are left out, so
    that a change of wording does not void a measurement while any change of code does."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, "paper_1906_01632_amd", "csrc", name)) as f:
            src = f.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)   # block comments
        src = re.sub(r"//[^\n]*", " ", src)                # line comments
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()


def measured_traffic(smoother, wl_name, prec):
    """The committed rocprofv3 FETCH_SIZE / WRITE_SIZE measurement of the smoother for this
    workload and precision (ratios of HBM to algorithmic bytes per launch), or None when
    there is none or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "smoother_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
        digest = kernel_digest(KERNEL_SOURCES[smoother])
    except OSError:
        return None
    if rec.get("smoother") != smoother or rec.get("kernel_sources_sha256") != digest or \
            rec.get("workload") != wl_name:
        return None
    return rec.get("precisions", {}).get(prec)


# ---------------------------------------------------------------------------------------
# Summaries of rocprofv3 CSV output (host only; `--summarise-trace`, `--summarise-counters`)
# ---------------------------------------------------------------------------------------
LARGE_LAUNCH = 256 * 1024 * 1024   # working sets beyond the 256 MiB last-level cache
ZERO_START_BLOCKS = (0, 6, 18, 24)  # line sweep from zero: blocks read per column colour
JX_FLOPS = 967.0     # k_jx: FP64 operations per hexahedron of the compiled loop and the rows
                     # of its vertex (FMA = 2): one hexahedron per interior vertex
JX_BYTES = 80.0      # k_jx: u, x, y, d (16 B each) + phi and K (8 B each) per vertex


def _levels(wl):
    """(nx, ny, nz) of every level of every group of the workload."""
    out = []
    for q in wl.groups:
        for l in range(q.levels):
            f = 1 << l
            out.append(((q.nx - 1) // f + 1, (q.ny - 1) // f + 1, (q.nz - 1) // f + 1))
    return out


def _par(n, p):
    """indices of parity p among n."""
    return (n - p + 1) // 2


def _line_tables(wl):
    """(workgroups along x, threads per workgroup, columns per workgroup) -> {(columns, nz)}
    of the line-smoother launches of the workload's levels (k_line_sweep: 8, 16 or 32
    columns per 256-thread workgroup, the column-walk fallback k_line_smooth: 64 per 64),
    and padded colour-major size -> (level, per-colour-of-columns vertex counts) for the
    residual launches."""
    sweep, resid = {}, {}
    for nx, ny, nz in _levels(wl):
        for cc in range(4):
            nc = _par(nx, cc & 1) * _par(ny, cc >> 1)
            for cols in (8, 16, 32):
                sweep.setdefault((-(-nc // cols), 256, cols), set()).add((nc, nz))
            sweep.setdefault((-(-nc // 64), 64, 64), set()).add((nc, nz))
        # k_line_residual_zs runs in slab order: 8 slabs of every colour's 64-position
        # tiles, workgroups of 4 tiles, the grid a multiple of 8 workgroups
        T = [-(-(_par(nx, c & 1) * _par(ny, c >> 1 & 1) * _par(nz, c >> 2)) // 64) for c in range(8)]
        most = max(sum((x + 1) * t // 8 - x * t // 8 for t in T) for x in range(8))
        per_cc = [_par(nx, cc & 1) * _par(ny, cc >> 1) * nz for cc in range(4)]
        resid.setdefault(8 * -(-most // 4) * 256, set()).add(tuple(per_cc))
    return sweep, resid


def _jx_grids(wl):
    """grid x of the matrix-free product's launches on each group's finest grid (tiles of
    15 x 15 vertex columns times segments of 8 vertices, 256 threads each) -> vertices."""
    return {-(-q.nx // 15) * -(-q.ny // 15) * -(-q.nz // 8) * 256: q.nx * q.ny * q.nz
            for q in wl.groups}


def _dispatch_bytes(name, bx, wx, gx, rows, sweep, resid):
    """Algorithmic bytes of one smoother or residual dispatch (the library's count), or
    None for other kernels and ambiguous grids."""
    import re
    size = {"float": 4, "double": 8, "_Float16": 2}
    m = re.search(r"k_line_(sweep|smooth)<(float|double), (float|double|_Float16), (?:true|false), "
                  r"(-?\d+)(?:, (\d+))?>", name)
    if m:  # vectors in T (group 2), matrix in M (group 3)
        cols = int(m.group(5)) if m.group(5) else 64
        cand = sweep.get((bx, wx, cols), set())
        if len(cand) != 1:
            return None
        (nc, nz), = cand
        nb = 24 if int(m.group(4)) < 0 else ZERO_START_BLOCKS[int(m.group(4))]
        t, mt = size[m.group(2)], size[m.group(3)]
        return rows * nc * nz * (4 * (nb + 1) * mt + 16 * t)
    m = re.search(r"k_line_residual_zs<(float|double), (float|double|_Float16), (?:true|false)>", name)
    if m:
        cand = resid.get(gx, set())
        if len(cand) != 1:
            return None
        per_cc, = cand
        t, mt = size[m.group(1)], size[m.group(2)]
        unscale = 4 * t if mt == 2 else 0  # the FP16 matrix's residual reads D
        return rows * sum(n * (4 * (24 - ZERO_START_BLOCKS[cc]) * mt + 2 * t + unscale)
                          for cc, n in enumerate(per_cc))
    return None


def _csv(d, suffix):
    import glob
    f = glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)
    if not f:
        raise SystemExit(f"no *{suffix} under {d}")
    import csv
    with open(f[0]) as fh:
        return list(csv.DictReader(fh))


def _col(row, name):
    for c in row:
        if c.replace("-", "_").lower() == name.lower():
            return row[c]
    return None


def summarise_trace(d, leg, wl):
    """Markdown summary of a `rocprofv3 --kernel-trace --marker-trace` run of this script
    with --mark-timed-region: per-kernel totals inside the leg's "timed steps" range, the
    GPU busy share, algorithmic GB/s of the smoother (all launches and those beyond 256 MiB),
    of the residual and of the matrix-free product (with its FP64 TFLOP/s), and the
    histogram of active samples per launch."""
    import collections
    rows = _csv(d, "kernel_trace.csv")
    ranges = sorted((int(_col(r, "Start_Timestamp")), int(_col(r, "End_Timestamp")))
                    for r in _csv(d, "marker_api_trace.csv") if "timed steps" in str(r))
    t0, t1 = ranges[leg]
    sel = [r for r in rows if int(_col(r, "Start_Timestamp")) >= t0 and int(_col(r, "End_Timestamp")) <= t1]
    short = lambda n: n.split("(")[0].replace("void ", "").replace("edf::", "")
    out = [f"timed-steps range {leg} of {len(ranges)}"]
    tot = collections.defaultdict(lambda: [0, 0.0])
    iv = []
    for r in sel:
        s, e = int(_col(r, "Start_Timestamp")), int(_col(r, "End_Timestamp"))
        k = short(_readable_name(_col(r, "Kernel_Name")))
        tot[k][0] += 1
        tot[k][1] += (e - s) * 1e-3
        iv.append((s, e))
    iv.sort()
    busy, cs, ce = 0, None, None
    for s, e in iv:
        if ce is None or s > ce:
            if ce is not None:
                busy += ce - cs
            cs, ce = s, e
        else:
            ce = max(ce, e)
    if ce is not None:
        busy += ce - cs
    allms = sum(v[1] for v in tot.values()) * 1e-3
    out.append(f"timed region {(t1 - t0) * 1e-6:.1f} ms, GPU busy {busy * 1e-6:.1f} ms "
               f"({100 * busy / (t1 - t0):.1f} %), kernel time {allms:.1f} ms")
    out += ["", "| kernel | calls | avg us | total ms | % of kernel time |", "|---|---|---|---|---|"]
    for k, (n, us) in sorted(tot.items(), key=lambda kv: -kv[1][1])[:25]:
        out.append(f"| `{k}` | {n} | {us / n:.2f} | {us * 1e-3:.1f} | {100 * us * 1e-3 / allms:.1f} |")
    sweep, resid = _line_tables(wl)
    fin = _jx_grids(wl)
    agg = collections.defaultdict(lambda: [0, 0.0, 0.0, 0.0])
    hist = collections.defaultdict(collections.Counter)
    for r in sel:
        name = _readable_name(_col(r, "Kernel_Name"))
        k = short(name)
        dur = (int(_col(r, "End_Timestamp")) - int(_col(r, "Start_Timestamp"))) * 1e-9
        gx, gy = int(_col(r, "Grid_Size_X")), int(_col(r, "Grid_Size_Y"))
        wx = int(_col(r, "Workgroup_Size_X"))
        b = _dispatch_bytes(name, gx // wx, wx, gx, gy, sweep, resid)
        if b is not None:
            base = k.split("<")[0]
            for key in (base + " (all)",) + ((base + " (> 256 MiB)",) if b > LARGE_LAUNCH else ()):
                a = agg[key]; a[0] += 1; a[1] += dur; a[2] += b
        if k.startswith("k_jx") and gx in fin:
            a = agg["k_jx (finest grids)"]; a[0] += 1; a[1] += dur
            a[2] += JX_BYTES * fin[gx] * gy; a[3] += JX_FLOPS * fin[gx] * gy
        if k.startswith(("k_line_sweep", "k_jx", "k_line_residual_zs")):
            hist[(k.split("<")[0], gx)][gy] += 1
    out += ["", "| kernel | dispatches | avg us | MB per dispatch | GB/s (algorithmic) | frac of 8 TB/s | FP64 TFLOP/s |",
            "|---|---|---|---|---|---|---|"]
    for k, (n, sec, b, f) in sorted(agg.items()):
        tf = f"{f / sec / 1e12:.1f} ({f / sec / 78.6e12:.3f} of 78.6)" if f else "-"
        out.append(f"| {k} | {n} | {1e6 * sec / n:.1f} | {b / n / 1e6:.1f} | {b / sec / 1e9:.0f} | "
                   f"{b / sec / 8e12:.3f} | {tf} |")
    out += ["", "active samples per launch (grid rows), by kernel and grid x:"]
    edges = [1, 2, 4, 8, 16, 32, 64, 128, 256]
    for (name, x), c in sorted(hist.items(), key=lambda kv: -sum(kv[1].values()))[:10]:
        n = sum(c.values())
        parts = []
        for lo, hi in zip(edges, edges[1:] + [10 ** 9]):
            m = sum(v for rr, v in c.items() if lo <= rr < hi)
            parts.append(f"{lo}-{hi - 1 if hi < 10 ** 9 else 'up'}: {100 * m / n:.0f}%")
        out.append(f"- {name} grid x {x}: {n} dispatches; " + ", ".join(parts))
    return "\n".join(out)


def _readable_name(name):
    """rocprofv3 leaves the _Float16 instances of the line kernels mangled; their demangled
    form (as for the other instances), or the name unchanged."""
    import re
    flag = {"0": "false", "1": "true"}
    m = re.search(r"k_line_(sweep|smooth)IfDF16_Lb([01])ELi(n?\d+)E(?:Li(\d+)E)?E", name)
    if m:
        zc = m.group(3).replace("n", "-")
        cols = f", {m.group(4)}" if m.group(4) else ""
        return f"void edf::k_line_{m.group(1)}<float, _Float16, {flag[m.group(2)]}, {zc}{cols}>()"
    m = re.search(r"k_line_residual_zsIfDF16_Lb([01])EE", name)
    if m:
        return f"void edf::k_line_residual_zs<float, _Float16, {flag[m.group(1)]}>()"
    return name


def _probe(order, times):
    """The copy probe's dispatches: the last group of copy dispatches with 0.2 s or more
    of idle time before and after it (order: dispatch ids by start time)."""
    probe = []
    for n, di in enumerate(order):
        if "copyBuffer" not in times[di][2] or (n and times[di][0] - times[order[n - 1]][1] < 0.2e9):
            continue
        grp, m = [di], n + 1
        while m < len(order) and "copyBuffer" in times[order[m]][2] and \
                times[order[m]][0] - times[order[m - 1]][1] < 0.2e9:
            grp.append(order[m])
            m += 1
        if m == len(order) or times[order[m]][0] - times[order[m - 1]][1] >= 0.2e9:
            probe = grp
    return probe


def _load_counter_run(d):
    """(times, grids, per-dispatch counter totals) of one `rocprofv3 --pmc C --kernel-trace`
    run: times[id] = (start, end, readable name), grids[id] = (workgroups along x,
    workgroup size, grid x, grid y)."""
    times, grids = {}, {}
    for r in _csv(d, "kernel_trace.csv"):
        di = int(_col(r, "Dispatch_Id"))
        times[di] = (int(_col(r, "Start_Timestamp")), int(_col(r, "End_Timestamp")),
                     _readable_name(_col(r, "Kernel_Name")))
        gx, wx = int(_col(r, "Grid_Size_X")), int(_col(r, "Workgroup_Size_X"))
        grids[di] = (gx // wx, wx, gx, int(_col(r, "Grid_Size_Y")))
    per = {}
    for r in _csv(d, "counter_collection.csv"):
        di = int(_col(r, "Dispatch_Id"))
        per[di] = per.get(di, 0.0) + float(_col(r, "Counter_Value"))
    return times, grids, per


def _counter_run(d, regex, sweep, resid):
    """Counter totals of one `rocprofv3 --pmc C --kernel-trace` run of this script with
    --copy-probe: (KiB the probe's copy dispatches read or wrote, accumulators of the
    matching dispatches after it: all, and those beyond 256 MiB of algorithmic bytes)."""
    import re
    times, grids, per = _load_counter_run(d)
    order = sorted(times, key=lambda x: times[x][0])
    probe = _probe(order, times)
    if not probe:
        raise SystemExit(f"no isolated copy probe in {d}")
    acc = {"all": [0, 0.0, 0.0], "large": [0, 0.0, 0.0]}
    for di in order:
        if times[di][0] <= times[probe[-1]][0] or not re.search(regex, times[di][2]):
            continue
        bx, wx, gx, gy = grids[di]
        b = _dispatch_bytes(times[di][2], bx, wx, gx, gy, sweep, resid)
        if b is None:
            continue
        for k in ("all",) + (("large",) if b > LARGE_LAUNCH else ()):
            acc[k][0] += 1; acc[k][1] += per.get(di, 0.0); acc[k][2] += b
    return sum(per.get(di, 0.0) for di in probe), len(probe), acc


def summarise_counters(fetch_dir, write_dir, wl, precision, smoother, command):
    """The smoother's HBM traffic per launch over its algorithmic bytes, from a FETCH_SIZE
    and a WRITE_SIZE run, each scaled by what the same counter reads for the probe's 1 GiB
    device copy (1 GiB read, 1 GiB written)."""
    sweep, resid = _line_tables(wl)
    regex = r"k_line_sweep" if smoother else r"k_smooth<"
    rec = {"precision": precision, "command": command}
    runs = {}
    for cname, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        kib, n, acc = _counter_run(d, regex, sweep, resid)
        runs[cname] = (1024.0 * 1024.0 / kib, acc)
        rec[cname] = {"probe_kib": kib, "probe_dispatches": n, "scale": 1024.0 * 1024.0 / kib}
    for k in ("all", "large"):
        (fs, fa), (ws, wa) = runs["FETCH_SIZE"], runs["WRITE_SIZE"]
        if not fa[k][0] or not wa[k][0]:
            continue
        fetch = fs * fa[k][1] * 1024.0 / fa[k][0]
        write = ws * wa[k][1] * 1024.0 / wa[k][0]
        rec[k] = {"dispatches": fa[k][0], "algorithmic_bytes_per_dispatch": fa[k][2] / fa[k][0],
                  "hbm_fetch_bytes_per_dispatch": fetch, "hbm_write_bytes_per_dispatch": write,
                  "ratio": fs * fa[k][1] * 1024.0 / fa[k][2] + ws * wa[k][1] * 1024.0 / wa[k][2]}
    return rec


def counter_table(fetch_dir, write_dir, wl, by_matrix=False):
    """Markdown per-kernel HBM traffic of a FETCH_SIZE and a WRITE_SIZE run (each with
    --kernel-trace, of this script with --copy-probe): per kernel the dispatches after the
    probe, counted bytes (each counter scaled by what it reads for the probe's 1 GiB copy),
    the library's algorithmic bytes where it has them, their ratio and the counted GB/s
    over the fetch run's durations.  by_matrix: the line kernels split by the matrix type
    (FP16 / FP32) and a column of the share of kernel time; else launches beyond 256 MiB
    in rows of their own and the matrix-free product's bytes per finest grid."""
    import re
    sweep, resid = _line_tables(wl)
    short = lambda n: n.split("(")[0].replace("void ", "").replace("edf::", "")
    out, runs = [], {}
    for tag, d in (("fetch", fetch_dir), ("write", write_dir)):
        times, grids, per = _load_counter_run(d)
        order = sorted(times, key=lambda x: times[x][0])
        probe = _probe(order, times)
        if not probe:
            raise SystemExit(f"no isolated copy probe in {d}")
        kib = sum(per.get(x, 0.0) for x in probe)
        if not by_matrix:
            out.append(f"{tag} probe dispatches {len(probe)} KiB {kib}")
        scale = 1024.0 * 1024.0 / kib
        acc = {}
        for di in order:
            if times[di][0] <= times[probe[-1]][0]:
                continue
            name = times[di][2]
            bx, wx, gx, gy = grids[di]
            b = _dispatch_bytes(name, bx, wx, gx, gy, sweep, resid)
            base = re.sub(r"<.*", "", short(name))
            if by_matrix and base in ("k_line_sweep", "k_line_residual_zs"):
                keys = (base + (" (FP16 matrix)" if "_Float16" in name else " (FP32 matrix)"),)
            elif by_matrix:
                keys = (base,)
            else:
                keys = (base,) + ((base + " (>256MiB)",) if b and b > LARGE_LAUNCH else ())
            for k in keys:
                a = acc.setdefault(k, [0, 0.0, 0.0, 0.0])
                a[0] += 1
                a[1] += per.get(di, 0.0) * 1024 * scale
                a[2] += b or 0.0
                a[3] += (times[di][1] - times[di][0]) * 1e-9
        runs[tag] = (scale, acc, times, grids, per)
    (fs, fa, ft, fg, fp), (ws, wa, wt, wg, wp) = runs["fetch"], runs["write"]
    if by_matrix:
        tot = sum(v[3] for v in fa.values())
        out += ["| kernel | dispatches | % of kernel time | fetch MB/disp | write MB/disp | "
                "algorithmic MB/disp | (fetch+write)/alg | counted HBM GB/s |",
                "|---|---|---|---|---|---|---|---|"]
        for k in sorted(fa, key=lambda k: -fa[k][3])[:14]:
            n, fb, ab, t = fa[k]
            wb = wa.get(k, [1, 0.0])[1] / max(wa.get(k, [1])[0], 1) * n
            r = f"{(fb + wb) / ab:.3f}" if ab else "-"
            out.append(f"| {k} | {n} | {100 * t / tot:.1f} | {fb / n / 1e6:.1f} | {wb / n / 1e6:.1f} | "
                       f"{ab / n / 1e6:.1f} | {r} | {(fb + wb) / t / 1e9:.0f} |")
        return "\n".join(out)
    out += [f"probe scales: fetch {fs:.3f}, write {ws:.3f}",
            "| kernel | dispatches | fetch MB/disp | write MB/disp | algorithmic MB/disp | "
            "(fetch+write)/alg | HBM GB/s (counted, fetch run durations) |",
            "|---|---|---|---|---|---|---|"]
    for k in sorted(fa, key=lambda k: -fa[k][1])[:22]:
        n, f, b, t = fa[k]
        w = wa.get(k, [0, 0.0, 0.0, 0.0])[1]
        ratio = (f + w) / b if b else float("nan")
        out.append(f"| {k} | {n} | {f / n / 1e6:.2f} | {w / max(wa.get(k, [1])[0], 1) / 1e6:.2f} | "
                   f"{b / n / 1e6:.2f} | {ratio:.3f} | {(f + w) / t / 1e9 if t else 0:.0f} |")
    # the matrix-free product: JX_BYTES per vertex of its finest grid
    fin = _jx_grids(wl)
    for tag, (scale, _, times, grids, per) in (("fetch", runs["fetch"]), ("write", runs["write"])):
        tj = {}
        for di, (t0, t1, name) in times.items():
            if "k_jx" not in name or grids[di][2] not in fin:
                continue
            gx, gy = grids[di][2], grids[di][3]
            a = tj.setdefault(gx, [0, 0.0, 0.0, 0.0])
            a[0] += 1
            a[1] += per.get(di, 0.0) * 1024 * scale
            a[2] += JX_BYTES * fin[gx] * gy
            a[3] += (t1 - t0) * 1e-9
        for gx, (n, c, b, t) in sorted(tj.items()):
            out.append(f"k_jx {tag} grid {gx} ({fin[gx]} vertices): {n} dispatches, counted "
                       f"{c / n / 1e6:.1f} MB, algorithmic {b / n / 1e6:.1f} MB per dispatch, "
                       f"ratio {c / b:.2f}, {c / t / 1e9:.0f} GB/s")
    return "\n".join(out)


# quantity of interest of the gradient workload: salt mass in the bottom 50 m under
# the centre of the box, [200, 400] x [200, 400] x [100, 150] m (z = depth)
QOI_BOX = (200.0, 400.0, 200.0, 400.0, 100.0, 150.0)


def run_adjoint(args, wl, pb, prec):
    """One timed edf_adjoint call over args.steps steps: sample-timesteps/s of the
    gradient (forward steps with checkpoints plus the backward sweep)."""
    import numpy as np
    import torch
    pb.profile(True)
    t0 = time.perf_counter()
    pb.solve(wl.dt, args.steps, checkpoint_every=min(10, args.steps), stats=False)
    J, g = pb.adjoint(QOI_BOX)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = pb.profile(False)
    out = {"metric": "dJ/dxi sample-timesteps/s (forward with checkpoints every 10 steps + "
                     "discrete adjoint with recomputed segments)",
           "value": wl.n_samples * args.steps / el, "unit": "sample-timesteps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * el / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": {"f64": "f64", "mixed": "f64+f32", "mixed16": "f64+f32+f16"}[prec],
           "data": "synthetic (seeded lattice parameters; no dataset)",
           "config": {"workload": wl.name, "groups": [[q.nx, q.ny, q.nz, q.levels, q.samples]
                                                      for q in wl.groups],
                      "qoi_box": QOI_BOX, "dt_s": wl.dt, "precision": prec},
           "J_mean": float(np.mean(J)), "dJ_dxi_mean": np.mean(g, axis=0).tolist()}
    if prof["vcycles"]:
        vg = prof["vcycle_bytes"] / (prof["vcycle_ms"] * 1e-3) / 1e9
        out["vcycle"] = {"achieved": vg, "unit": "GB/s", "peak": HBM_PEAK_GBS,
                         "frac": vg / HBM_PEAK_GBS, "count": prof["vcycles"]}
    pb.destroy()
    print(json.dumps(out), flush=True)


FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector (and matrix) peak


def run_gpc(args, wl, pb, prec, degree=4, n_points=10**6, threshold=0.5):
    """The quadrature nodes' samples stepped wl.steps times (untimed), then the surrogate:
    projection of the full-grid c fields (HBM bound) and the exceedance probability
    from n_points surrogate samples per vertex (FP64 matrix cores), both timed by events
    around their kernels."""
    import numpy as np
    for k in range(wl.steps):
        t = time.perf_counter()
        pb.step(wl.dt)
        log(f"node samples, step {k + 1}: {time.perf_counter() - t:.2f} s")
    g = wl.groups[0]
    common = (g.nx, g.ny, g.nz)
    Nc, S = g.n_vertices, g.samples
    pts = np.random.default_rng(11).uniform(-1.0, 1.0, (n_points, wl.xi.shape[1]))
    proj_ms, ex_ms = [], []
    for r in range(1 + args.steps):  # the first of each is a warm-up
        out = pb.gpc_project(0, common, degree, wl.weights, coefficients=False)
        prob, ms = pb.gpc_exceed(pts, threshold, common)
        if r:
            proj_ms.append(out["kernel_ms"])
            ex_ms.append(ms)
    nc = out["n_coef"]
    pm, em = float(np.mean(proj_ms)), float(np.mean(ex_ms))
    proj_bytes = 8.0 * Nc * (S + nc)        # every sample field read, every coefficient written
    flops = 2.0 * nc * Nc * n_points        # one FMA per term, vertex and point (the basis
                                            # tables' time is counted, their flops are not)
    gbs, tfs = proj_bytes / (pm * 1e-3) / 1e9, flops / (em * 1e-3) / 1e12
    res = {"metric": "gPC surrogate: vertex-samples/s of the exceedance estimate",
           "value": Nc * n_points / (em * 1e-3), "unit": "vertex-samples/s", "n_gpus": 1,
           "steps": args.steps, "warmup": 1, "ms_per_step": pm + em, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (Gauss-Legendre nodes, seeded surrogate points; no dataset)",
           "config": {"workload": wl.name, "grid": list(common), "nodes": S, "degree": degree,
                      "n_coef": nc, "points": n_points, "threshold": threshold},
           "mean_range": [float(out["mean"].min()), float(out["mean"].max())],
           "max_var": float(out["var"].max()), "max_prob": float(prob.max()),
           "roofline": {"bound": "mfma", "kernel": "k_gpc_exceed (surrogate evaluation)",
                        "achieved": tfs, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": tfs / FP64_PEAK_TFLOPS, "traffic": None, "avg_launch_us": 1e3 * em,
                        "flops_per_launch": flops},
           "projection": {"bound": "hbm", "kernel": "k_gpc_project", "achieved": gbs,
                          "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                          "avg_launch_us": 1e3 * pm, "bytes_per_launch": proj_bytes}}
    pb.destroy()
    print(json.dumps(res), flush=True)


def _oracle_steps(job):
    """A worker of cpu_baseline: whole first steps of the given samples of one group with
    the oracle, until the budget is spent; returns (steps done, seconds)."""
    import synth
    from oracle import elder, newton
    field_model, shape, xis, dt, rtol, budget_s = job
    phys = synth.physics(field_model)
    box = elder.Box(*shape, phys)
    u0 = synth.initial_state(*shape, phys)
    done, t0 = 0, time.perf_counter()
    for xi in xis:
        newton.newton_solve(box, elder.coefficients(box, xi), u0, dt, rtol=rtol)
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    return done, time.perf_counter() - t0


def cpu_baseline(wl, phys, budget_s=20.0):
    """The oracle (plain FP64 NumPy/SciPy, unchanged) on a bounded sample of the
    workload: whole implicit-Euler steps of the samples of its smallest group, one sample
    per worker process at a time, one worker per host core (at most 16, the host share of
    one GPU), BLAS single-threaded in each."""
    import multiprocessing as mp
    g = min(wl.groups, key=lambda q: q.n_vertices)
    S0 = sum(q.samples for q in wl.groups[:wl.groups.index(g)])
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    workers = max(1, min(16, cores, g.samples))
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"  # inherited by the spawned workers
    xis = [list(wl.xi[S0 + i]) if wl.xi.shape[1] else [] for i in range(g.samples)]
    jobs = [(wl.field_model, (g.nx, g.ny, g.nz), xis[w::workers], wl.dt, wl.newton_rtol, budget_s)
            for w in range(workers)]
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(workers) as pool:  # fresh interpreters: no GPU state
        res = pool.map(_oracle_steps, jobs)
    wall = time.perf_counter() - t0
    done = sum(r[0] for r in res)
    busy = max(r[1] for r in res)
    return {"value": done / busy, "unit": "sample-timesteps/s", "cores": workers, "kind": "oracle",
            "dof_timesteps_per_s": done * 2 * g.n_vertices / busy,
            "sample": f"{done} sample(s) x 1 step (the first step) of the {g.nx}x{g.ny}x{g.nz} "
                      f"group on {workers} worker processes (one sample each at a time, SuperLU "
                      f"and NumPy single-threaded), {busy:.1f} s of solving ({wall:.1f} s with "
                      f"process start); host {cores} usable logical CPUs, "
                      f"{platform.processor() or platform.machine()}; the 65x65x17 and "
                      f"129x129x33 groups take minutes per oracle step and are not timed"}


PREC_NAMES = {"f64": "f64", "mixed": "f64+f32", "mixed16": "f64+f32+f16"}


def make_problem(args, wl, phys, groups, prec, log_tuning=True):
    """A problem of the workload with the benchmark's solver options, parameters set and
    the V-cycle bottom tuned (or fixed by --fuse-from)."""
    import numpy as np

    from paper_1906_01632_amd import PREC_F64, PREC_MIXED, PREC_MIXED_F16, Problem
    # the adjoint solves (transposed Jacobian, no Newton retry) get more Krylov iterations
    opts = dict(newton_rtol=wl.newton_rtol, lin_rtol=1e-6, lin_max_it=400 if args.adjoint else 100,
                newton_max_it=20,
                precision={"f64": PREC_F64, "mixed": PREC_MIXED, "mixed16": PREC_MIXED_F16}[prec],
                check_every=args.check_every, forcing=args.forcing,
                concurrent_groups=args.concurrent_groups,
                graph_vcycle=int(args.graph), substep_memory=int(args.substep_memory),
                smoother=int(args.smoother), matrix_free=int(args.matrix_free),
                predictor=int(args.predictor) if not args.adjoint else 0,
                nu_pre=args.nu[0], nu_post=args.nu[1], lag_preconditioner=args.lag_preconditioner)
    t = time.perf_counter()
    pb = Problem(phys, groups, opts)
    pb.set_parameters(wl.xi)
    fuse = args.fuse_from_fp64 if (prec == "f64" and args.fuse_from_fp64) else args.fuse_from
    if fuse:
        levels = [int(v) for v in fuse.split(",")]
        assert len(levels) == len(groups), "--fuse-from needs one level per group"
        for gi, lv in enumerate(levels):
            pb.set_tuning(gi, lv)
    elif not args.no_autotune:
        pb.autotune(wl.dt, cache=args.tuning_cache)
    tuning = [pb.tuning(g)[0] for g in range(len(groups))]
    if log_tuning:
        for gi in range(len(groups)):
            log(f"group {gi}: V-cycle ms per first fused level "
                f"{np.round(pb.tuning(gi)[1], 3).tolist()}; line-sweep columns per "
                f"workgroup by level {pb.line_tiles(gi)}")
    log(f"set-up {time.perf_counter() - t:.1f} s; fused V-cycle bottom from levels {tuning}")
    return pb, tuning


def run_steps(args, wl, pb, prec, region=(None, None)):
    """W warm-up steps, then K timed steps with the smoother and V-cycle event timing on;
    returns the leg's measurements."""
    import numpy as np
    import torch
    warm = []
    for w in range(args.warmup):
        t = time.perf_counter()
        warm.append(pb.step(wl.dt))
        log(f"[{prec}] warmup step {w + 1}: {time.perf_counter() - t:.2f} s")
    torch.cuda.synchronize()
    if not args.no_profile:
        pb.profile(True)
    if args.copy_probe:
        # idle gaps of 0.25 s on both sides set the probe's dispatches apart in a trace
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        time.sleep(0.25)
        b.copy_(a)
        torch.cuda.synchronize()
        time.sleep(0.25)
        del a, b
    if region[0]:
        region[0]()
    per_step = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        per_step.append(pb.step(wl.dt))
        if k < 10 or (k + 1) % 50 == 0 or k + 1 == args.steps:
            log(f"[{prec}] step {k + 1}: {time.perf_counter() - t0:.2f} s elapsed")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    if region[1]:
        region[1]()
    prof = pb.profile(False)
    S = wl.n_samples
    last = per_step[-1]
    # over all timed sample-steps: Newton and BiCGStab work, steps split into sub-steps,
    # failed attempts restarted with shorter sub-steps, samples failed, mass balance
    ran = [t for st in per_step for t in st if t["newton_its"] > 0]
    newton = sum(t["newton_its"] for t in ran)
    lin = sum(t["lin_its"] for t in ran)
    solver = {
        "sample_steps": len(ran),
        "newton_its_per_sample_step": newton / max(len(ran), 1),
        "bicgstab_its_per_newton": lin / max(newton, 1),
        "split_sample_steps": sum(t["substeps"] > 1 for t in ran),
        "substeps_per_sample_step": sum(t["substeps"] for t in ran) / max(len(ran), 1),
        "restarted_attempts": sum(t["retries"] for t in ran),
        "extrapolated_starts": sum(t["predicted"] for t in ran),
        "failed_samples": sum(t["status"] != 0 for t in last),
        "max_salt_balance_err": max((t["salt_balance_err"] for t in ran), default=0.0),
        "max_liquid_balance_err": max((t["liquid_balance_err"] for t in ran), default=0.0),
    }
    leg = {"value": S * args.steps / el, "el": el, "prof": prof, "solver": solver,
           # sub-steps of every sample in every step, warm-up included
           "substeps": np.array([[t["substeps"] for t in st] for st in warm + per_step])}
    if prof["vcycles"]:
        vg = prof["vcycle_bytes"] / (prof["vcycle_ms"] * 1e-3) / 1e9
        leg["vcycle"] = {"achieved": vg, "unit": "GB/s", "peak": HBM_PEAK_GBS,
                         "frac": vg / HBM_PEAK_GBS, "count": prof["vcycles"],
                         "avg_ms": prof["vcycle_ms"] / prof["vcycles"],
                         "bytes_per_vcycle": prof["vcycle_bytes"] / prof["vcycles"]}
        if prof["large_vcycles"]:
            # V-cycles whose algorithmic bytes exceed the 256 MiB last-level cache
            lg = prof["large_vcycle_bytes"] / (prof["large_vcycle_ms"] * 1e-3) / 1e9
            leg["vcycle"]["beyond_256MiB"] = {
                "achieved": lg, "frac": lg / HBM_PEAK_GBS, "count": prof["large_vcycles"],
                "share_of_vcycle_time": prof["large_vcycle_ms"] / prof["vcycle_ms"]}
    return leg


def roofline_of(leg, wl, prec, smoother):
    """The dominant kernel (the V-cycle smoother) from the leg's event timing.  The figure
    is that of the launches whose algorithmic bytes exceed the 256 MiB last-level cache
    (MALL), so that cache hits of small launches cannot pass for HBM bandwidth; the figure
    over every timed launch is reported beside it."""
    prof = leg["prof"]
    if not prof["launches"]:
        return None
    large = prof["large_launches"] > 0
    n, ms, b = ((prof["large_launches"], prof["large_ms"], prof["large_bytes"]) if large
                else (prof["launches"], prof["ms"], prof["bytes"]))
    gbs = b / (ms * 1e-3) / 1e9
    gbs_all = prof["bytes"] / (prof["ms"] * 1e-3) / 1e9
    tr = measured_traffic(smoother, wl.name, prec)
    traffic = ratio = None
    if tr and tr.get("large" if large else "all"):
        # HBM bytes per launch of this run's launch mix: the measured ratio of HBM to
        # algorithmic bytes (over the large launches) times this run's algorithmic bytes
        # per large launch
        ratio = tr["large" if large else "all"]["ratio"]
        traffic = ratio * (prof["large_all_bytes"] / prof["large_all_launches"] if large
                           else prof["all_bytes"] / prof["all_launches"])
    name = ("k_line_sweep (vertical-line block Gauss-Seidel, one column colour)" if smoother
            else "k_smooth (block Gauss-Seidel colour sweep)")
    return {"bound": "hbm", "kernel": name, "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS, "traffic": traffic, "traffic_over_algorithmic": ratio,
            "launches": "working set > 256 MiB" if large else "all",
            "launches_timed": n, "avg_launch_us": 1e3 * ms / n, "bytes_per_launch": b / n,
            "all_launches": {"achieved": gbs_all, "frac": gbs_all / HBM_PEAK_GBS,
                             "launches_timed": prof["launches"],
                             "launches_in_run": prof["all_launches"],
                             "avg_launch_us": 1e3 * prof["ms"] / prof["launches"],
                             "bytes_per_launch": prof["bytes"] / prof["launches"]}}


def compare_states(ref_states, ref_sub, pb, sub, S):
    """Relative L2 per field of pb's states against ref_states, over the samples that took
    the same sub-steps in every timed step (a different sub-step sequence is a different
    discrete trajectory)."""
    import numpy as np
    worst = {"p": 0.0, "c": 0.0}
    med = {"p": [], "c": []}
    compared = 0
    for s in range(S):
        if not np.array_equal(ref_sub[:, s], sub[:, s]) or ref_states[s] is None:
            continue
        u = pb.get_state(s)
        compared += 1
        for f, name in ((0, "p"), (1, "c")):
            a, b = u[..., f], ref_states[s][..., f]
            r = float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
            worst[name] = max(worst[name], r)
            med[name].append(r)
    return {"rel_l2_p_max": worst["p"], "rel_l2_c_max": worst["c"],
            "rel_l2_p_median": float(np.median(med["p"])) if med["p"] else None,
            "rel_l2_c_median": float(np.median(med["c"])) if med["c"] else None,
            "samples_compared": compared, "samples_other_substeps": S - compared,
            "within_1e-6": worst["p"] <= 1e-6 and worst["c"] <= 1e-6}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="qmc512_mixedres")
    ap.add_argument("--precision", choices=["f64", "mixed", "mixed16"], default=None,
                    help="V-cycle precision: FP64, FP32, or FP32 with the finest matrix in FP16 "
                         "(one leg); without it the qMC workload runs an FP64 leg and then the "
                         "FP32-V-cycle leg, compared field by field")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--graph", action="store_true",
                    help="capture each V-cycle launch configuration as a HIP graph and replay "
                         "it (implies --no-profile: the roofline times single launches)")
    ap.add_argument("--forcing", type=int, default=1, choices=[0, 1],
                    help="1: Eisenstat-Walker tolerances for the Newton systems")
    ap.add_argument("--smoother", type=int, default=1, choices=[0, 1],
                    help="0: point-block Gauss-Seidel in 8 colours; 1: vertical-line block "
                         "Gauss-Seidel (z-columns solved exactly, 4 column colours)")
    ap.add_argument("--matrix-free", type=int, default=1, choices=[0, 1],
                    help="1: matrix-free Jacobian products in BiCGStab (no exact stencil)")
    ap.add_argument("--substep-memory", type=int, default=1, choices=[0, 1],
                    help="1: a sample starts a step with the sub-step count that worked in its "
                         "previous step")
    ap.add_argument("--nu", type=int, nargs=2, default=[1, 1], metavar=("PRE", "POST"),
                    help="smoothing sweeps before and after the coarse correction")
    ap.add_argument("--check-every", type=int, default=1,
                    help="BiCGStab iterations between the host's checks of which samples are "
                         "still active (launches run over the samples active at the last check)")
    ap.add_argument("--lag-preconditioner", type=int, default=0, choices=[0, 1],
                    help="1: assemble the V-cycle's matrices only at the first Newton iteration "
                         "of each (sub-)step attempt")
    ap.add_argument("--predictor", type=int, default=1, choices=[0, 1],
                    help="1: Newton starts a step from the extrapolation 2 u^n - u^{n-1} where "
                         "its defect is smaller (same stopping test)")
    ap.add_argument("--concurrent-groups", type=int, default=2, choices=[0, 1, 2],
                    help="0: the grid groups one after the other; 1: at the same time, one host "
                         "thread and stream each (overlapping kernels lengthen the per-launch "
                         "durations the roofline is computed from); 2: one host thread each on a "
                         "shared stream, the V-cycles of the groups inside BiCGStab run together, "
                         "each level the groups share swept by one launch over all their samples")
    ap.add_argument("--adjoint", action="store_true",
                    help="time the gradient instead of plain steps: edf_solve with a checkpoint "
                         "every 10 steps over --steps steps, then edf_adjoint (segments "
                         "recomputed) of the salt mass in the lower-central box")
    ap.add_argument("--gpc", action="store_true",
                    help="time the polynomial chaos surrogate instead of plain steps: solve the "
                         "quadrature nodes' samples (untimed), then project them (degree 4) and "
                         "sample the surrogate's exceedance at 10^6 points (workload gpc125)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default fused-bottom levels instead of timing the choices")
    ap.add_argument("--fuse-from", default=None,
                    help="first fused V-cycle level per group, comma separated (instead of "
                         "autotuning; e.g. to repeat a run's launch configuration under a profiler)")
    ap.add_argument("--fuse-from-fp64", default=None,
                    help="as --fuse-from, for the FP64 leg of the two-leg default run")
    ap.add_argument("--tuning-cache", default=None,
                    help="JSON file of V-cycle tunings (fused bottom, line-sweep tile shapes) by "
                         "groups, precision, smoother and device: applied when it holds this "
                         "problem's key, else tuned and stored")
    ap.add_argument("--mark-timed-region", action="store_true",
                    help="mark the timed steps with a roctx range (rocprofv3 --marker-trace)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="copy 1 GiB device-to-device at the start of the timed region (a copy "
                         "of known size that calibrates the HBM byte counters)")
    ap.add_argument("--summarise-trace", metavar="DIR", default=None,
                    help="summarise the CSV of a rocprofv3 --kernel-trace --marker-trace run of "
                         "this script (with --mark-timed-region) and exit; no GPU is used")
    ap.add_argument("--leg", type=int, default=-1,
                    help="with --summarise-trace: which timed-steps range (in the default "
                         "two-leg run 0: the FP64 leg, 1: the mixed leg; -1: the last)")
    ap.add_argument("--summarise-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    default=None,
                    help="HBM traffic of the smoother from rocprofv3 --pmc FETCH_SIZE and "
                         "WRITE_SIZE runs (each with --kernel-trace) of this script with "
                         "--copy-probe; added to --summary-out under --precision; no GPU is used")
    ap.add_argument("--counters-table", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    default=None,
                    help="per-kernel HBM traffic (markdown) of the same two counter runs; "
                         "no GPU is used")
    ap.add_argument("--by-matrix", action="store_true",
                    help="with --counters-table: line kernels split by matrix type")
    ap.add_argument("--summary-out", default=None)
    ap.add_argument("--profile-command", default="",
                    help="with --summarise-counters: the command that made the counter runs")
    args = ap.parse_args()
    if args.summarise_trace or args.summarise_counters or args.counters_table:
        import synth
        wl = synth.workload(args.workload)
        if args.summarise_trace:
            print(summarise_trace(args.summarise_trace, args.leg, wl))
            return
        if args.counters_table:
            print(counter_table(*args.counters_table, wl, args.by_matrix))
            return
        prec = args.precision or "mixed"
        rec = summarise_counters(*args.summarise_counters, wl, prec, args.smoother,
                                 args.profile_command)
        digest = kernel_digest(KERNEL_SOURCES[args.smoother])
        full = {}
        if args.summary_out and os.path.exists(args.summary_out):
            with open(args.summary_out) as f:
                full = json.load(f)
        if (full.get("smoother"), full.get("workload"), full.get("kernel_sources_sha256")) != \
                (args.smoother, wl.name, digest):
            full = {"kernel": ("k_line_sweep<T, NT, ZC>, all instances" if args.smoother
                               else "k_smooth<T, NT, ZC>, all instances"),
                    "smoother": args.smoother, "workload": wl.name,
                    "kernel_sources": ["paper_1906_01632_amd/csrc/" + n
                                       for n in KERNEL_SOURCES[args.smoother]],
                    "kernel_sources_sha256": digest, "precisions": {}}
        full["precisions"][prec] = rec
        text = json.dumps(full, indent=1)
        if args.summary_out:
            with open(args.summary_out, "w") as f:
                f.write(text + "\n")
        print(text)
        return
    region = roctx_range() if args.mark_timed_region else (None, None)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): samples are independent, "
              "so N GPUs would each run their own share; no multi-GPU path is built.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    wl = synth.workload(args.workload)
    phys = synth.physics(wl.field_model)
    groups = [(g.nx, g.ny, g.nz, g.levels, g.samples) for g in wl.groups]
    if args.graph:
        args.no_profile = True
    two_legs = args.precision is None and wl.name == "qmc512_mixedres" and not (args.adjoint or args.gpc)
    prec = args.precision or ("mixed" if two_legs else wl.precision)
    S = wl.n_samples
    ref = None
    if two_legs:
        # the FP64 leg: the reference the mixed-precision states are compared with
        log(f"workload {wl.name}: groups {groups}, FP64 leg")
        pb, tuning64 = make_problem(args, wl, phys, groups, "f64")
        leg64 = run_steps(args, wl, pb, "f64", region)
        # the reference of the precision comparison: one more FP64 step from the states
        # reached, with every sample's sub-step history cleared (edf_set_state), so that the
        # mixed leg can take the same step from the same states
        end64 = [pb.get_state(s) for s in range(S)]
        for s in range(S):
            pb.set_state(s, end64[s])
        st64 = pb.step(wl.dt)
        ref = (end64, leg64["substeps"], [pb.get_state(s) for s in range(S)],
               np.array([[t["substeps"] for t in st64]]))
        pb.destroy()
        torch.cuda.synchronize()
    log(f"workload {wl.name}: groups {groups}, precision {prec}")
    pb, tuning = make_problem(args, wl, phys, groups, prec)
    if args.adjoint:
        for w in range(args.warmup):
            pb.step(wl.dt)
        return run_adjoint(args, wl, pb, prec)
    if args.gpc:
        return run_gpc(args, wl, pb, prec)
    tiles = [pb.line_tiles(g) for g in range(len(groups))]
    leg = run_steps(args, wl, pb, prec, region)
    el = leg["el"]
    dofs = sum(2 * g.n_vertices * g.samples for g in wl.groups)
    out = {
        "metric": METRIC,
        "value": leg["value"],
        "unit": "sample-timesteps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * el / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": PREC_NAMES[prec],
        "data": ("synthetic (Halton points and Gauss-Legendre nodes; no dataset)"
                 if wl.name in synth.E1_GRIDS else "synthetic (seeded lattice parameters; no dataset)"),
        "config": {"workload": wl.name, "groups": [list(g) for g in groups], "samples": S,
                   "dt_s": wl.dt, "precision": prec, "newton_rtol": wl.newton_rtol,
                   "lin_rtol": 1e-6, "lin_max_it": 100,
                   "forcing": "eisenstat-walker" if args.forcing else "fixed",
                   "smoother": ["point-block-gs-8-colour", "z-line-block-gs-4-colour"][args.smoother],
                   "matrix_free_jacobian": bool(args.matrix_free),
                   "substep_memory": bool(args.substep_memory),
                   "newton_predictor": bool(args.predictor),
                   "smoothing_sweeps": list(args.nu),
                   "bicgstab_check_every": args.check_every,
                   "lagged_preconditioner": bool(args.lag_preconditioner),
                   "fused_bottom_from_level": tuning,
                   "line_sweep_columns_per_workgroup": tiles,
                   "concurrent_groups": args.concurrent_groups,
                   "graph_vcycle": bool(args.graph)},
        "dof_timesteps_per_s": dofs * args.steps / el,
        "solver": leg["solver"],
    }
    if "vcycle" in leg:
        out["vcycle"] = leg["vcycle"]
    rl = roofline_of(leg, wl, prec, args.smoother)
    if rl:
        out["roofline"] = rl
    if two_legs:
        # context: the two trajectories after W + K steps (the fingering instability
        # amplifies the solvers' tolerance-level differences over the months)
        traj = compare_states(ref[0], ref[1], pb, leg["substeps"], S)
        # the comparison proper: one step of each precision from the same states
        for s in range(S):
            pb.set_state(s, ref[0][s])
        st = pb.step(wl.dt)
        out["mixed_vs_fp64"] = compare_states(ref[2], ref[3], pb,
                                              np.array([[t["substeps"] for t in st]]), S)
        out["mixed_vs_fp64"]["what"] = ("one step of each precision from the FP64 states after "
                                        f"{args.warmup + args.steps} steps, per sample and field")
        out["mixed_vs_fp64_trajectory"] = dict(traj, what=f"the two runs after {args.warmup + args.steps} "
                                               "steps each (context: trajectories of this unstable "
                                               "flow amplify tolerance-level differences)")
        out["fp64"] = {"value": leg64["value"], "ms_per_step": 1e3 * leg64["el"] / args.steps,
                       "dtype": "f64", "fused_bottom_from_level": tuning64,
                       "solver": leg64["solver"], "vcycle": leg64.get("vcycle"),
                       "roofline": roofline_of(leg64, wl, "f64", args.smoother)}
        out["mixed_over_fp64"] = leg["value"] / leg64["value"]
        log(f"mixed vs FP64, one step from shared states: {out['mixed_vs_fp64']}; trajectories: "
            f"{out['mixed_vs_fp64_trajectory']}; {out['mixed_over_fp64']:.3f} x the FP64 rate")
    if wl.name in synth.E1_GRIDS:
        # the box experiment's comparison after the last timed step: 200 Halton qMC samples
        # (group 0) against the degree-4 surrogate from the 125 quadrature nodes (group 1)
        from paper_1906_01632_amd.uq import qmc_vs_gpc
        g0 = wl.groups[0]
        res = qmc_vs_gpc(pb, 0, 1, wl.weights, (g0.nx, g0.ny, g0.nz), degree=4)
        out["e1_compare"] = dict(res["compare"], years=(args.warmup + args.steps) * wl.dt / synth.YEAR_S)
        log(f"qMC vs gPC: {out['e1_compare']}")
    if wl.mlmc_levels:
        # multilevel estimates after the last timed step on the coarsest grid: level 0
        # alone, levels 0-1, all levels (the differences are the level corrections)
        from paper_1906_01632_amd.uq import mlmc_weights
        g0 = wl.groups[0]
        common = (g0.nx, g0.ny, g0.nz)
        n = wl.mlmc_levels
        est = []
        for L in range(1, len(n) + 1):
            w = np.zeros(S)
            part = mlmc_weights(n[:L])
            w[:part.size] = part
            if L < len(n):  # the partners of level L stay out
                w[sum(n[:L]) + sum(n[1:L]):] = 0.0
            est.append(pb.moments(common, weights=w))
        ref0 = np.linalg.norm(est[0][0])
        out["mlmc"] = {"levels": list(n), "grids": [[g.nx, g.ny, g.nz] for g in wl.groups],
                       "correction_rel_l2": [float(np.linalg.norm(est[L][0] - est[L - 1][0]) / ref0)
                                             for L in range(1, len(n))],
                       "mean_range": [float(est[-1][0].min()), float(est[-1][0].max())],
                       "max_var": float(est[-1][1].max()),
                       "sample_dof_share": [g.samples * g.n_vertices / sum(q.samples * q.n_vertices
                                                                             for q in wl.groups)
                                            for g in wl.groups]}
        log(f"multilevel: {out['mlmc']}")
    pb.destroy()
    if not args.no_cpu_baseline:
        log("oracle timing on the host ...")
        out["cpu_baseline"] = cpu_baseline(wl, phys)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
