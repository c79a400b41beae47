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


def measured_traffic(smoother):
    """Ratio of measured HBM bytes to algorithmic bytes per smoother launch, from the
    committed rocprofv3 FETCH_SIZE / WRITE_SIZE measurement, or None when the kernel
    sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "smoother_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
        digest = kernel_digest(KERNEL_SOURCES[smoother])
    except OSError:
        return None
    if rec.get("smoother") != smoother or rec.get("kernel_sources_sha256") != digest:
        return None
    return rec


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


def cpu_baseline(wl, phys, budget_s=20.0):
    """The oracle (plain FP64 NumPy/SciPy, unchanged) on a bounded sample of the
    workload: whole implicit-Euler steps of the samples of its smallest group."""
    import numpy as np

    import synth
    from oracle import elder, newton
    g = min(wl.groups, key=lambda q: q.n_vertices)
    S0 = sum(q.samples for q in wl.groups[:wl.groups.index(g)])
    box = elder.Box(g.nx, g.ny, g.nz, phys)
    u0 = synth.initial_state(g.nx, g.ny, g.nz, phys)
    done, t0 = 0, time.perf_counter()
    while True:
        xi = wl.xi[S0 + done] if wl.xi.shape[1] else []
        newton.newton_solve(box, elder.coefficients(box, xi), u0, wl.dt, rtol=wl.newton_rtol)
        done += 1
        el = time.perf_counter() - t0
        if el > budget_s or done >= g.samples:
            break
    return {"value": done / el, "unit": "sample-timesteps/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} sample(s) x 1 step (the first step) of the {g.nx}x{g.ny}x{g.nz} "
                      f"group, {el:.1f} s; SuperLU and NumPy single-threaded; host "
                      f"{os.cpu_count()} logical CPUs, {platform.processor() or platform.machine()}"}


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
                check_every=1, forcing=args.forcing, concurrent_groups=int(args.concurrent_groups),
                graph_vcycle=int(args.graph), substep_memory=int(args.substep_memory),
                smoother=int(args.smoother), matrix_free=int(args.matrix_free))
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
        pb.autotune(wl.dt)
    tuning = [pb.tuning(g)[0] for g in range(len(groups))]
    if log_tuning:
        for gi in range(len(groups)):
            log(f"group {gi}: V-cycle ms per first fused level "
                f"{np.round(pb.tuning(gi)[1], 3).tolist()}")
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
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
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
    tr = measured_traffic(smoother)
    traffic = ratio = None
    if tr and tr.get("workload") == wl.name and tr.get("precision") == prec:
        # HBM bytes per launch of this run's launch mix: the measured ratio of HBM to
        # algorithmic bytes (over the large launches) times this run's algorithmic bytes
        # per large launch
        ratio = tr["ratio_large"] if large else tr["ratio"]
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
    ap.add_argument("--concurrent-groups", action="store_true",
                    help="advance the grid groups at the same time (one host thread and stream "
                         "each); more throughput, but overlapping kernels lengthen the per-launch "
                         "durations the roofline is computed from")
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
    ap.add_argument("--mark-timed-region", action="store_true",
                    help="mark the timed steps with a roctx range (rocprofv3 --marker-trace)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="copy 1 GiB device-to-device at the start of the timed region (a copy "
                         "of known size that calibrates the HBM byte counters)")
    args = ap.parse_args()
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
        leg64 = run_steps(args, wl, pb, "f64")
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
                   "fused_bottom_from_level": tuning,
                   "concurrent_groups": bool(args.concurrent_groups),
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
