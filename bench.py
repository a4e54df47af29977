"""Benchmark: batched cell-Sinkhorn inside domain decomposition on one MI355X.

Workload (default ms512): mu, nu = seeded 8-blob Gaussian mixtures (+1e-4 floor) on 512x512,
basic cells 4x4 (16,384 basic cells; 4,096 A / 4,225 B composite problems).  Untimed set-up:
multiscale domain decomposition from the 8x8 layer (2x2 block sums) up to 512x512, eps =
2h^2, h^2, h^2/2 per layer, then 2h^2 on the finest layer (8 half-iterations per stage).  Timed: K domain-decomposition
half-iterations (alternating A/B) at eps = h^2, Sinkhorn tolerance 1e-5 on the X-marginal
(App. A.2.1 batch rule), warm-started from the previous visit of the partition.  A step = one
half-iteration = BasicToComposite + cell Sinkhorn to tolerance + CompositeToBasic + balancing
+ truncation.  (--workload mix512: the same marginals from a Knothe-Rosenblatt start with the
single-scale eps schedule 64h^2 ... 2h^2.)

value  = algorithmic LSE bytes of the timed steps / wall time of the timed steps (GB/s);
         12 (|X_J| + W1 W2) bytes per cell per Sinkhorn iteration (read f, log nu_J, write g;
         read g, log nu_J, log mu, write f -- 4 bytes each at float32).
roofline: the Sinkhorn kernel does one multiply-add per LSE term (exponentials per input
         and output only): achieved = LSE terms / kernel time, peak = the FP32 vector rate
         157.3 TFLOP/s / 2 FLOP per term.
cpu_baseline: the oracle's dense float64 cell solver on a random sample of the composite cells
         of one more half-iteration of the same trajectory, from the same start and for the
         same number of iterations as the GPU (single thread and all host threads, medians of
         5 runs); the same solve gives the GPU result's error against the oracle.
time_to_tol: the replay protocol (8 consecutive states; zero, previous-iterate and learned
         starts, the same tolerance and stop rule).
f64, mix1024 / ms1024, full_solve: the same step in float64, the 1024^2 workload, and the whole
         multiscale solve down to eps = h^2/4 (the paper's schedule).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# LSE terms/s: one fused multiply-add per term at the FP32 vector peak (157.3 TFLOP/s)
TERM_PEAK = 157.3e12 / 2
# the same at the FP64 vector peak (78.6 TFLOP/s)
TERM_PEAK_F64 = 78.6e12 / 2
HBM_PEAK = 8.0e12


WORKLOAD_TEXT = {
    "mix512": "mix512: {N}x{N} 8-blob Gaussian mixtures + 1e-4 floor, s={s}, KR init, "
              "eps-scaling 64..2 untimed, timed DD iterations at eps=h^2",
    "mix256": "mix256: {N}x{N} 8-blob Gaussian mixtures + 1e-4 floor, s={s}, KR init, "
              "eps-scaling 64..2 untimed, timed DD iterations at eps=h^2",
    "mix1024": "mix1024: {N}x{N} 16-blob Gaussian mixtures + 1e-4 floor, s={s}, KR init, "
               "eps-scaling 64..2 untimed, timed DD iterations at eps=h^2",
    "ms512": "ms512: the mix512 marginals solved coarse to fine (untimed): layers 8^2 ... 256^2 "
             "of 2x2 block sums, eps = 2h^2, h^2, h^2/2 per layer (8 DD half-iterations each), "
             "then 512^2 at 2h^2 (8); timed DD half-iterations at eps=h^2, s={s}",
    "ms1024": "ms1024: the mix1024 marginals solved coarse to fine (untimed): layers 8^2 ... "
              "512^2, eps = 2h^2, h^2, h^2/2 per layer (8 DD half-iterations each), then 1024^2 "
              "at 2h^2 (8); timed DD half-iterations at eps=h^2, s={s}",
    "flow512": "flow512: {N}x{N}, mu 8-blob mixture, nu = mu rotated 30 deg, contracted 0.36, "
               "shifted (0.25, 0); s={s}; map init; eps=h^2; hybrid A, B, flow update",
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def setup(args, workload, prec_name):
    import torch

    import paper_2405_09400_amd as dd
    import synth

    w = synth.workload(workload, seed=args.seed)
    prec = dd.DD_PREC_F32 if prec_name == "f32" else dd.DD_PREC_F64
    t0 = time.perf_counter()
    levels = w.extra.get("levels", 0)
    ctx = dd.DomDec(w.mu, w.nu, w.s, w.init, prec=prec, levels=levels)
    log(f"[bench] init {workload} N={w.N} s={w.s} {prec_name} in {time.perf_counter() - t0:.2f}s")
    rule = dd.DD_STOP_CELL if args.stop_rule == "cell" else dd.DD_STOP_BATCH
    k = 0
    # coarser layers of a multiscale workload: their eps stages, then the refinement
    for layer in range(levels):
        for kappa in w.extra["layer_kappas"]:
            eps = kappa / ctx.N ** 2
            for _ in range(w.extra["layer_iters"]):
                st = ctx.iterate("AB"[k % 2], eps, tol=args.tol, stop_rule=rule,
                                 max_iter=args.max_iter, check_every=args.check_every)
                k += 1
        log(f"[bench] layer {ctx.N}x{ctx.N} done: last iters={st['sk']['iters_max']} "
            f"maxW={st['max_w1']}x{st['max_w2']}")
        ctx.refine()
    for kappa, its in zip(w.kappas[:-1], w.stage_iters[:-1]):
        eps = kappa / w.N ** 2
        for _ in range(its):
            st = ctx.iterate("AB"[k % 2], eps, tol=args.tol, stop_rule=rule, max_iter=args.max_iter,
                             check_every=args.check_every)
            k += 1
        log(f"[bench] stage kappa={kappa:g}: last iters={st['sk']['iters_max']} "
            f"maxW={st['max_w1']}x{st['max_w2']} entries={st['nu_entries']}")
    torch.cuda.synchronize()
    return w, ctx, rule, k


def run_steps(ctx, w, n, k0, args, rule, init=None, flows=None):
    """n DD half-iterations at the last eps of the schedule; on the flow workload a flow update
    follows every B half-iteration (the hybrid A, B, flow schedule), its stats in `flows`."""
    import paper_2405_09400_amd as dd
    eps = w.kappas[-1] / w.N ** 2
    flow_every = w.extra.get("flow_every", 0)
    out = []
    for i in range(n):
        part = "AB"[(k0 + i) % 2]
        t0 = time.perf_counter()
        st = ctx.iterate(part, eps, tol=args.tol, stop_rule=rule, max_iter=args.max_iter,
                         check_every=args.check_every,
                         init=dd.DD_INIT_PREV if init is None else init)
        st["wall_ms"] = (time.perf_counter() - t0) * 1e3  # iterate synchronises the stream
        out.append(st)
        if flow_every and part == "B":
            eg = None if args.flow_eps_gamma is None else args.flow_eps_gamma / w.N ** 2
            fs = ctx.flow_update(eps_gamma=eg)
            log(f"[bench] flow update: costs {fs['t_costs_ms']:.1f} ms, min-cost flow "
                f"{fs['t_mcf_ms']:.1f} ms, assembly {fs['t_assemble_ms']:.1f} ms, "
                f"moved mass {fs['moved_mass']:.3e}")
            if flows is not None:
                flows.append(fs)
    return out


def load_net(path):
    import paper_2405_09400_amd as dd
    if not path or not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        return dd.WarmStartNet(z["params"])


def time_to_tol(ctx, w, k0, args, rule):
    """Replay: from each of R consecutive states of the plain trajectory, solve the same
    half-iteration to the same tolerance with the zero start, the previous-iterate start and
    the learned start (time = start + Sinkhorn, device clock), then continue the trajectory
    with the previous-iterate step."""
    import paper_2405_09400_amd as dd
    net = load_net(args.net_weights)
    if net is not None:
        ctx.set_net(net)
    eps = w.kappas[-1] / w.N ** 2
    kinds = [("zero", dd.DD_INIT_ZERO)] + ([("learned_net", dd.DD_INIT_NET)] if net else []) + \
        [("prev_iterate", dd.DD_INIT_PREV)]
    rec = {name: {"ms": [], "iters": [], "f64_finish_iters": [], "sinkhorn_ms": [], "init_ms": []}
           for name, _ in kinds}
    for r in range(args.replay):
        log(f"[bench] replay state {r}")
        ctx.save()
        for j, (name, init) in enumerate(kinds):
            if j:
                ctx.restore()
            st = ctx.iterate("AB"[(k0 + r) % 2], eps, tol=args.tol, stop_rule=rule,
                             max_iter=args.max_iter, check_every=args.check_every, init=init)
            d = rec[name]
            d["sinkhorn_ms"].append(round(st["t_sinkhorn_ms"], 3))
            d["init_ms"].append(round(st["t_init_ms"], 3))
            d["ms"].append(round(st["t_sinkhorn_ms"] + st["t_init_ms"], 3))
            # float32 iterations (the stop of the float32 phase: at 0.85 tol, or handed over
            # when its error stalls) and the float64 finish that certifies the tolerance
            d["iters"].append(st["sk"]["iters_max"])
            d["f64_finish_iters"].append(st["sk"]["finish_iters_max"])
    out = {"tol": args.tol, "states": args.replay, "_steps": args.replay,
           "time": "start + Sinkhorn on the device clock; sums and medians over the states"}
    for name, _ in kinds:
        out[name] = rec[name]
        rec[name]["sum_ms"] = round(sum(rec[name]["ms"]), 3)
        rec[name]["median_ms"] = round(float(np.median(rec[name]["ms"])), 3)
    if not net:
        out["learned_net"] = None
    tot = {name: sum(rec[name]["ms"]) for name, _ in kinds}
    med = {name: float(np.median(rec[name]["ms"])) for name, _ in kinds}
    out["speedup_prev_vs_zero"] = tot["zero"] / tot["prev_iterate"]
    out["speedup_prev_vs_zero_median"] = med["zero"] / med["prev_iterate"]
    if net:
        out["speedup_net_vs_zero"] = tot["zero"] / tot["learned_net"]
        out["speedup_net_vs_prev"] = tot["prev_iterate"] / tot["learned_net"]
        out["speedup_net_vs_zero_median"] = med["zero"] / med["learned_net"]
        out["speedup_net_vs_prev_median"] = med["prev_iterate"] / med["learned_net"]
        ctx.set_net(None)
        net.close()
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cell_objective(od, xpix, ysup, plan, eps):
    """<c, pi> + eps sum pi (log(pi / (mu nu)) - 1) of one composite plan."""
    d = od.coords[xpix][:, None, :] - od.coords[ysup][None, :, :]
    c = (d ** 2).sum(axis=2)
    ref = od.mu[xpix][:, None] * od.nu[ysup][None, :]
    pos = plan > 0
    return float((c * plan).sum() + eps * (plan[pos] * (np.log(plan[pos] / ref[pos]) - 1.0)).sum())


def cpu_baseline(args, w, ctx, k, rule):
    """The oracle on the state the GPU is timed on, and the GPU's error against it.

    One more half-iteration of the benchmark's trajectory runs on the GPU (untimed, exactly as
    the timed ones).  The oracle takes the state just before it (basic-cell Y-marginals and the
    partition's X potentials, read through the C ABI) and solves a seeded random sample of the
    same composite cells for the same number of Sinkhorn iterations, with its dense float64
    cell solver: one warm-up, then the median of `runs` runs on one thread and on all host
    threads.  The same oracle solve gives the GPU result's error on the sampled cells (new
    basic-cell Y-marginals, both plan marginals, cell objective; relative, worst cell)."""
    import oracle

    import paper_2405_09400_amd as dd
    part = "AB"[k % 2]
    eps = w.kappas[-1] / w.N ** 2
    nu_before = ctx.nu_i_sparse()
    pre = ctx.extract_potentials(part, beta=False)
    st = ctx.iterate(part, eps, tol=args.tol, stop_rule=rule, max_iter=args.max_iter,
                     check_every=args.check_every, init=dd.DD_INIT_PREV)
    sk = st["sk"]
    n_its = sk["iters_max"]  # both phases
    nu_after = ctx.nu_i_sparse()
    post = ctx.extract_potentials(part)
    t0 = time.perf_counter()
    cells = oracle.basic_cell_pixels(w.N, w.s)
    xs = np.concatenate([np.full(len(i), cells[c][0], np.int64) for c, (i, _) in enumerate(nu_before)])
    od = oracle.DomDec(w.mu, w.nu, w.s, (xs, np.concatenate([i for i, _ in nu_before]),
                                         np.concatenate([v for _, v in nu_before])))
    log(f"[bench] oracle state built in {time.perf_counter() - t0:.1f}s")
    parts = od.parts[part]
    xside = pre["xside"]

    def alpha0(J, xpix):
        k1, k2 = np.divmod(xpix, w.N)
        xo = pre["xorig"][J]
        return pre["alpha"][J][(k1 - xo[0]) * xside + (k2 - xo[1])]

    def batch(sample):
        xo, yo, X, M, Y, V, R, A = [0], [0], [], [], [], [], [], []
        nbytes = 0.0
        for J in sample:
            basic = parts[J]
            xpix = np.concatenate([od.cells[i] for i in basic])
            ysup, nuJ = oracle.sparse_sum([od.nu_i[i] for i in basic])
            X.append(od.coords[xpix])
            M.append(od.mu[xpix])
            Y.append(od.coords[ysup])
            V.append(nuJ)
            R.append(od.nu[ysup])
            A.append(alpha0(J, xpix))
            xo.append(xo[-1] + len(xpix))
            yo.append(yo[-1] + len(ysup))
            W1, W2 = post["ydims"][J]
            nbytes += n_its * 12.0 * (xside * xside + int(W1) * int(W2))
        arrs = (np.array(xo), np.concatenate(X), np.concatenate(M), np.array(yo), np.concatenate(Y),
                np.concatenate(V), np.concatenate(R))
        return arrs, np.concatenate(A), nbytes

    def run(arrs, a0, nthreads):
        t1 = time.perf_counter()
        oracle.sinkhorn_cells(*arrs, eps, fixed_iters=n_its, alpha=a0, nthreads=nthreads)
        return time.perf_counter() - t1

    rng = np.random.default_rng(4096 + args.seed)
    order = rng.permutation(len(parts))
    # size the sample so that one single-thread run takes about cpu_seconds / 12
    n = 4
    arrs, a0, nbytes = batch(order[:n])
    t_one = run(arrs, a0, 1)
    n = int(min(len(parts), max(4, n * (args.cpu_seconds / 12.0) / max(t_one, 1e-3))))
    sample = sorted(order[:n].tolist())
    arrs, a0, nbytes = batch(sample)
    nthreads = os.cpu_count() or 1
    runs = max(args.cpu_runs, 1)
    res = {}
    for name, th in (("single", 1), ("all", nthreads)):
        run(arrs, a0, th)  # warm-up
        ts = [run(arrs, a0, th) for _ in range(runs)]
        res[name] = float(np.median(ts))
    # the GPU's error on the sampled cells against the oracle's solve of the same problems
    for J in sample:
        od.alpha[part][J] = alpha0(J, np.concatenate([od.cells[i] for i in parts[J]]))
    od.iterate(part, eps, fixed_iters=n_its, cells=sample)
    worst = {"basic_nu_i": 0.0, "x_marginal": 0.0, "y_marginal": 0.0, "objective": 0.0}
    for J, cs in zip(sample, od.last[part]):
        for i in parts[J]:
            a = np.zeros(w.N * w.N)
            b = np.zeros(w.N * w.N)
            a[nu_after[i][0]] = nu_after[i][1]
            b[od.nu_i[i][0]] = od.nu_i[i][1]
            worst["basic_nu_i"] = max(worst["basic_nu_i"], float(np.abs(a - b).sum() / od.m[i]))
        P_or = oracle.cell_plan(od.coords[cs.xpix], od.mu[cs.xpix], cs.alpha, od.coords[cs.ysup],
                                od.nu[cs.ysup], cs.beta, eps)
        k1, k2 = np.divmod(cs.xpix, w.N)
        xo = pre["xorig"][J]
        a_g = post["alpha"][J][(k1 - xo[0]) * xside + (k2 - xo[1])]
        y1, y2 = np.divmod(cs.ysup, w.N)
        W2 = post["ydims"][J][1]
        b_g = post["beta"][post["ybase"][J] + (y1 - post["yorig"][J][0]) * W2 +
                           (y2 - post["yorig"][J][1])]
        P_g = oracle.cell_plan(od.coords[cs.xpix], od.mu[cs.xpix], a_g, od.coords[cs.ysup],
                               od.nu[cs.ysup], b_g, eps)
        m = P_or.sum()
        worst["x_marginal"] = max(worst["x_marginal"], float(np.abs(P_g.sum(1) - P_or.sum(1)).sum() / m))
        worst["y_marginal"] = max(worst["y_marginal"], float(np.abs(P_g.sum(0) - P_or.sum(0)).sum() / m))
        e_or = _cell_objective(od, cs.xpix, cs.ysup, P_or, eps)
        e_g = _cell_objective(od, cs.xpix, cs.ysup, P_g, eps)
        worst["objective"] = max(worst["objective"], abs(e_g - e_or) / abs(e_or))
    return {"value": nbytes / res["all"] / 1e9, "unit": "GB/s", "cores": nthreads, "kind": "oracle",
            "single_thread_value": nbytes / res["single"] / 1e9,
            "cpu_model": cpu_model(),
            "statistic": f"median of {runs} runs after one warm-up, single thread and {nthreads} threads",
            "sample": f"{len(sample)} random composite cells of the half-iteration after the timed "
                      f"ones (partition {part}, kappa=1), solved from the GPU's start of that "
                      f"half-iteration for its {n_its} Sinkhorn iterations by the dense float64 "
                      f"oracle ({res['single']:.2f} s single thread, {res['all']:.2f} s all "
                      f"threads per run)",
            "gpu_vs_oracle": {"cells": len(sample), "iterations": n_its,
                              "worst_relative": worst}}


# ---- HBM traffic of the dominant kernel (rocprofv3 counters) ------------------------------
#
# `traffic` in the roofline line is read from a committed counter summary: FETCH_SIZE and
# WRITE_SIZE (KiB per dispatch, one rocprofv3 --pmc run each) averaged over the dispatches of
# the timed steps, each scaled by what the same counter reads for a plain copy of known size
# (--copy-calibration).  The summary records the SHA-256 of the kernel's source; when the
# source has changed since, traffic is null.

KERNEL_SOURCE = os.path.join(ROOT, "paper_2405_09400_amd", "csrc", "fastcell.hip")
DEFAULT_CLASSES = (32, 2048)


def _classes_suffix(classes):
    """'' for the library's default cell classes, '_c<side>_<entries>' for another pair."""
    return "" if tuple(classes) == DEFAULT_CLASSES else f"_c{classes[0]}_{classes[1]}"


def traffic_summary_path(workload, classes=DEFAULT_CLASSES):
    return os.path.join(ROOT, "profiles",
                        f"fast_kernel_{workload}{_classes_suffix(classes)}_traffic.md")


def trace_summary_path(workload, classes=DEFAULT_CLASSES):
    return os.path.join(ROOT, "profiles", f"fast_kernel_{workload}{_classes_suffix(classes)}.md")


def summary_classes(args):
    """The cell classes a profile summary is written for (--classes, else the default)."""
    if not args.classes:
        return DEFAULT_CLASSES
    ws, be = (int(v) for v in args.classes.split(","))
    return (ws, be)


WORKLOAD_TITLE = {"ms512": "ms512 (512² coarse to fine, s = 4, timed at κ = 1, tol 1e-5, batch rule)",
                  "mix512": "mix512 (512², s = 4, κ = 1, tol 1e-5, batch rule)"}
COPY_MIB = 256


def source_sha256(path=KERNEL_SOURCE):
    import hashlib
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def copy_calibration():
    """A plain device copy of COPY_MIB MiB, three times (the counters' reference)."""
    import torch
    n = COPY_MIB * 2 ** 20 // 4
    src = torch.ones(n, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_mib": COPY_MIB, "copies": 3}), flush=True)


def _pmc_rows(d):
    import csv
    import glob
    out = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        out += list(csv.DictReader(open(f)))
    return out


def _per_dispatch(rows, name_part):
    got = {}
    for r in rows:
        if name_part in r["Kernel_Name"]:
            key = int(r["Dispatch_Id"])
            got[key] = got.get(key, 0.0) + float(r["Counter_Value"])
    return [got[k] for k in sorted(got)]


def traffic_summary(args):
    """Write the traffic summary from the four counter runs (directories given on the command
    line): FETCH_SIZE and WRITE_SIZE of the benchmark and of the copy calibration, for each of
    the kernels named by --traffic-kernel."""
    fb, wb, fc, wc = args.traffic_from
    last = args.traffic_last
    ref_kib = COPY_MIB * 1024.0
    f_copy = _per_dispatch(_pmc_rows(fc), "copyBuffer")
    w_copy = _per_dispatch(_pmc_rows(wc), "copyBuffer")
    ff = ref_kib / (sum(f_copy) / len(f_copy))
    wf = ref_kib / (sum(w_copy) / len(w_copy))
    f_rows, w_rows = _pmc_rows(fb), _pmc_rows(wb)
    cls = summary_classes(args)
    cmd_b = ("rocprofv3 --pmc {c} --kernel-trace -d <out> -o run --output-format csv -- "
             f"python3 bench.py --workload {args.workload} --steps 3 --warmup 1 --no-compare "
             f"--no-cpu-baseline --no-extra --classes {cls[0]},{cls[1]}")
    cmd_c = ("rocprofv3 --pmc {c} --kernel-trace -d <out> -o run --output-format csv -- "
             "python3 bench.py --copy-calibration")
    kinds = " ".join(f"'{k}'" for k in args.traffic_kernel)
    lines = [f"# HBM traffic of the register-blocked kernels, {WORKLOAD_TITLE[args.workload]}, "
             f"cell classes {cls[0]},{cls[1]}", "",
             "Commands (from the repository root on the MI355X machine, after `cd /tmp && export "
             "TMPDIR=/tmp`; one counter per run):", "", "```",
             cmd_b.format(c="FETCH_SIZE"), cmd_b.format(c="WRITE_SIZE"),
             cmd_c.format(c="FETCH_SIZE"), cmd_c.format(c="WRITE_SIZE"), "```", "",
             f"Summarised by `python bench.py --workload {args.workload} --classes {cls[0]},{cls[1]} "
             f"--traffic-from <four output dirs> --traffic-kernel {kinds} --traffic-last {last}`.",
             "",
             f"Copy of 256 MiB: FETCH_SIZE reads {sum(f_copy) / len(f_copy):.0f} KiB (scale "
             f"{ff:.3f}), WRITE_SIZE {sum(w_copy) / len(w_copy):.0f} KiB (scale {wf:.3f}).", "",
             "| kernel | FETCH_SIZE KiB per dispatch | WRITE_SIZE KiB per dispatch | HBM bytes per "
             "launch (scaled) |", "|---|---:|---:|---:|"]
    recs = []
    for kern in args.traffic_kernel:
        fk = _per_dispatch(f_rows, kern)[-last:]
        wk = _per_dispatch(w_rows, kern)[-last:]
        fkib, wkib = sum(fk) / len(fk), sum(wk) / len(wk)
        rec = {"kernel": kern, "source_sha256": source_sha256(), "classes": list(cls),
               "dispatches": len(fk),
               "fetch_kib_per_dispatch": fkib, "write_kib_per_dispatch": wkib,
               "fetch_factor": ff, "write_factor": wf,
               "bytes_per_launch": (fkib * ff + wkib * wf) * 1024.0}
        recs.append(rec)
        lines.append(f"| `{kern}` | {fkib:.1f} | {wkib:.1f} | {rec['bytes_per_launch']:.4g} |")
    lines += ["", f"Averaged over the last {last} dispatches of each kernel (the launches of the "
              "timed steps, the ones after the stop, which exit at once, included).", ""]
    lines += ["traffic-json: " + json.dumps(r) for r in recs]
    with open(args.traffic_out or traffic_summary_path(args.workload, cls), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def trace_summary(args):
    """Write the kernel-time summary of a rocprofv3 --kernel-trace --stats run (directory on
    the command line): per-kernel totals, and the average duration of the dispatches of the
    timed steps of the two register-blocked kernels (the last --traffic-last of each)."""
    import csv
    import glob
    d = args.trace_from
    stats = list(csv.DictReader(open(glob.glob(os.path.join(d, "**", "*kernel_stats.csv"),
                                               recursive=True)[0])))
    trace = list(csv.DictReader(open(glob.glob(os.path.join(d, "**", "*kernel_trace.csv"),
                                               recursive=True)[0])))
    tot = sum(float(r["TotalDurationNs"]) for r in stats)
    cls = summary_classes(args)
    cmd = ("rocprofv3 --kernel-trace --stats -d <out> -o run --output-format csv -- "
           f"python3 bench.py --workload {args.workload} --steps 3 --warmup 1 --no-compare "
           f"--no-cpu-baseline --no-extra --classes {cls[0]},{cls[1]}")
    lines = [f"# Cell Sinkhorn kernels, {WORKLOAD_TITLE[args.workload]}, cell classes "
             f"{cls[0]},{cls[1]}", "",
             "Command (from the repository root on the MI355X machine, after `cd /tmp && export "
             "TMPDIR=/tmp`):", "", "```", cmd, "```", "",
             f"Summarised by `python bench.py --workload {args.workload} --classes "
             f"{cls[0]},{cls[1]} --trace-from <out> --trace-json <its JSON line> --traffic-last "
             f"{args.traffic_last}`.  Kernel "
             f"source SHA-256 (fastcell.hip): "
             f"`{source_sha256()}`.", "",
             "Device: one MI355X (gfx950).  Per-kernel totals over the whole run (set-up "
             "stages included):", "",
             "| kernel | calls | total ms | average us | % |", "|---|---:|---:|---:|---:|"]
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:12]:
        name = r["Name"].replace("dd::(anonymous namespace)::", "").split("(")[0]
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | "
                     f"{100 * float(r['TotalDurationNs']) / tot:.1f} |")
    for k in ("fast_kernel<4, 16, false, 2>", "fast_kernel<8, 8, false, 2>",
              "fast_kernel<1, 4, true, 2>"):
        rows = sorted((r for r in trace if k in r["Kernel_Name"]),
                      key=lambda r: int(r["Start_Timestamp"]))[-args.traffic_last:]
        durs = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in rows]
        if durs:
            lines += ["", f"Timed steps: the last {len(durs)} dispatches of `{k}` (the "
                      f"launches after the stop, which exit at once, included): average "
                      f"{sum(durs) / len(durs):.1f} us, min {min(durs):.1f} us, max "
                      f"{max(durs):.1f} us."]
    if args.trace_json:
        with open(args.trace_json) as f:
            r = json.load(f)["roofline"]
        lines += ["", f"The JSON line of the same run: dominant kernel `{r['kernel']}`, "
                  f"{r['launches']} launches in the timed steps, "
                  f"{1e3 * r['kernel_ms_per_launch']:.1f} us per launch on its HIP events."]
    with open(args.trace_out or trace_summary_path(args.workload, cls), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def traffic_bytes(kernel_name, workload, classes):
    """HBM bytes per launch of `kernel_name` from the committed summary of the workload, or
    None when there is none, it covers another kernel or other cell classes, or the kernel's
    source has changed since."""
    path = traffic_summary_path(workload, tuple(classes[0])) if len(classes) == 1 else None
    if not path or not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("traffic-json: "):
            rec = json.loads(line[len("traffic-json: "):])
            if (rec["kernel"] in kernel_name and rec["source_sha256"] == source_sha256() and
                    [list(c) for c in classes] == [rec.get("classes")]):
                return rec["bytes_per_launch"]
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="ms512")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--tol", type=float, default=1e-5)
    ap.add_argument("--max-iter", type=int, default=20000)
    ap.add_argument("--stop-rule", choices=["batch", "cell"], default="batch")
    ap.add_argument("--check-every", type=int, default=8,
                    help="batch rule: iterations between stop tests (register-blocked path)")
    ap.add_argument("--prec", choices=["f32", "f64"], default="f32")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-runs", type=int, default=5)
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the float64 and 1024^2 records of the mix512 line")
    ap.add_argument("--extra-steps", type=int, default=4)
    ap.add_argument("--no-global", action="store_true",
                    help="skip the global Sinkhorn comparison record")
    ap.add_argument("--global-max-iter", type=int, default=4000)
    ap.add_argument("--flow-eps-gamma", type=float, default=None,
                    help="flow workload: glued edge candidates at this eps_gamma (units of h^2); "
                         "default: product candidates")
    ap.add_argument("--paper-table", action="store_true",
                    help="only run the whole float64 multiscale solve at 64^2 ... 1024^2 "
                         "(Table 1's DomDecGPU setting) and print one JSON line")
    ap.add_argument("--no-flow", action="store_true",
                    help="skip the flow workload record (hybrid A, B, flow schedule at 512^2)")
    ap.add_argument("--no-clusters", action="store_true",
                    help="skip the clustering study (time against K-means clusters at 1024^2)")
    ap.add_argument("--classes", default=None, metavar="WS,BE",
                    help="force the register-blocked path's cell classes (one-wave side limit, "
                         "eight-wave entry threshold) instead of the library's tuner")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--replay", type=int, default=8)
    ap.add_argument("--net-weights", default=os.path.join(ROOT, "paper_2405_09400_amd", "weights",
                                                          "warmstart_s4_k1.npz"))
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run the plain copy that calibrates the traffic counters")
    ap.add_argument("--traffic-from", nargs=4, metavar="DIR",
                    help="write the traffic summary from four rocprofv3 --pmc output "
                         "directories: FETCH_SIZE and WRITE_SIZE of the benchmark, then of the copy")
    ap.add_argument("--traffic-kernel", nargs="+",
                    default=["fast_kernel<1, 4, true, 2>", "fast_kernel<4, 16, false, 2>",
                             "fast_kernel<8, 8, false, 2>"])
    ap.add_argument("--traffic-last", type=int, default=139)
    ap.add_argument("--traffic-out", default=None)
    ap.add_argument("--trace-from", metavar="DIR",
                    help="write the kernel-time summary of a rocprofv3 kernel-trace run")
    ap.add_argument("--trace-out", default=None)
    ap.add_argument("--trace-json", default=None,
                    help="with --trace-from: the JSON line the profiled run printed, whose "
                         "per-launch time of the dominant kernel is quoted beside the trace's")
    args = ap.parse_args()
    if args.traffic_from:
        traffic_summary(args)
        return
    if args.trace_from:
        trace_summary(args)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding of the method is not built (this benchmark runs one GPU).", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2405_09400_amd as dd
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.paper_table:
        paper_table(args)
        return
    dd.lib()
    if args.classes:
        ws, be = (int(x) for x in args.classes.split(","))
        dd.set_classes(ws, be)

    line = measure(args, args.workload, args.prec, args.steps, args.warmup,
                   replay=0 if args.no_compare else args.replay, cpu=not args.no_cpu_baseline)
    larger = {"mix512": "mix1024", "ms512": "ms1024"}
    if not args.no_extra and args.workload in larger:
        # the same step in the paper's arithmetic (float64 throughout), and the 1024^2 workload
        sub = measure(args, args.workload, "f64", args.extra_steps, 1, replay=0, cpu=False)
        line["f64"] = {key: sub[key] for key in ("value", "unit", "ms_per_step", "ms_per_step_median",
                                                 "dtype", "roofline")}
        line["f64"]["detail"] = {key: sub["detail"][key] for key in
                                 ("sinkhorn_iters", "sinkhorn_ms_per_step", "x_marginal_l1",
                                  "y_marginal_l1", "primal", "dual", "pd_gap")}
        sub = measure(args, larger[args.workload], args.prec, args.extra_steps, 1, replay=0,
                      cpu=False)
        rec = {key: sub[key] for key in ("value", "unit", "ms_per_step", "ms_per_step_median",
                                         "dtype", "roofline")}
        rec["config"] = sub["config"]
        rec["value_frac_of_hbm_peak"] = sub["value"] * 1e9 / HBM_PEAK
        rec["detail"] = {key: sub["detail"][key] for key in
                         ("sinkhorn_iters", "sinkhorn_ms_per_step", "max_box", "x_marginal_l1",
                          "y_marginal_l1", "primal", "pd_gap")}
        line["size1024"] = rec
        if not args.no_clusters:
            line["clusters"] = clusters_record(args, larger[args.workload])
        if not args.no_flow:
            line["flow"] = flow_record(args)
        if args.workload.startswith("ms"):
            # the whole multiscale solve at the paper's arithmetic and stopping tolerance, and
            # the global Sinkhorn on the same problem
            line["full_solve"] = full_solve(args, args.workload, "f64", 1e-4)
            # the megapixel solve (Table 1's 1024^2 column)
            line["full_solve_1024"] = full_solve(args, larger[args.workload], "f64", 1e-4)
            if not args.no_global:
                g = global_record(args, args.workload)
                fs = line["full_solve"]
                g["dd_full_solve_speedup"] = g["wall_s"] / fs["wall_s"]
                g["dual_rel_diff_vs_dd_primal"] = abs(g["dual"] - fs["primal"]) / abs(fs["primal"])
                line["global"] = g
    print(json.dumps(line), flush=True)


def flow_record(args, steps=6, warmup=2):
    """The flow workload (Sec. 5.1: 512^2, s = 2, 65,536 basic cells, nu = a rotated, contracted,
    shifted mu, map start, eps = h^2) on the hybrid schedule A, B, flow update: the warm-up's
    A, B and first flow update (its min-cost flow from scratch), then `steps` half-iterations
    with a flow update after every B (each from the previous optimal basis)."""
    sub = measure(args, "flow512", args.prec, steps, warmup, replay=0, cpu=False)
    rec = {key: sub[key] for key in ("value", "unit", "ms_per_step", "ms_per_step_median", "dtype")}
    rec["config"] = sub["config"]
    rec["detail"] = {key: sub["detail"][key] for key in
                     ("step_ms", "sinkhorn_iters", "sinkhorn_ms_per_step", "flow", "primal",
                      "x_marginal_l1", "y_marginal_l1")}
    return rec


def clusters_record(args, workload, ks=(1, 2, 4, 8), steps=4):
    """Batching and clustering (App. A.1, App. A.2.1 Fig. "clustering": the time of the last
    multiscale layer against the number of K-means clusters, N = 1024, s = 4).  From the
    workload's untimed set-up, one saved state; for each k the state is restored and `steps`
    half-iterations at the timed eps run with the partition split into k clusters solved one
    after another (each batch with its own stopping test).  Reports the wall time per
    half-iteration and the composite work arrays' size (7 float64 per composite entry of the
    largest batch) against one batch."""
    import torch

    w, ctx, rule, k0 = setup(args, workload, args.prec)
    ctx.save()
    out = []
    for k in ks:
        ctx.restore()
        ctx.set_clusters(k)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sts = run_steps(ctx, w, steps, k0, args, rule)
        wall = (time.perf_counter() - t0) * 1e3 / steps
        peak = max(st["peak_comp_entries"] for st in sts)
        total = max(st["comp_entries"] for st in sts)
        out.append({"clusters": k, "batches": [st["batches"] for st in sts],
                    "ms_per_step": wall,
                    "sinkhorn_iters": [st["sk"]["iters_max"] for st in sts],
                    "peak_comp_entries": peak, "comp_entries": total,
                    "work_bytes": 56 * peak, "work_frac_of_one_batch": peak / total})
        log(f"[bench] clusters {k}: {wall:.2f} ms/step, batches {out[-1]['batches']}, composite "
            f"work {56 * peak / 2**20:.1f} MiB ({peak / total:.2f} of one batch)")
    ctx.close()
    return {"workload": workload, "dtype": args.prec, "steps": steps,
            "heuristic_clusters": max(1, w.N // 256), "runs": out}


def full_solve(args, workload, prec_name, tol, N=None, seed=None):
    """The whole multiscale solve, timed end to end: set-up, every layer's eps stages and
    refinements, and on the finest layer eps = 2h^2, h^2, h^2/2, h^2/4 (the paper's schedule,
    App. A.2.1), each stage `layer_iters` half-iterations; then the relative primal-dual gap
    and the marginal errors of the result (evaluated after the clock stops)."""
    import torch

    import paper_2405_09400_amd as dd
    import synth
    w = synth.workload(workload, seed=args.seed if seed is None else seed, N=N)
    L = w.extra["levels"]
    prec = dd.DD_PREC_F32 if prec_name == "f32" else dd.DD_PREC_F64
    rule = dd.DD_STOP_BATCH
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx = dd.DomDec(w.mu, w.nu, w.s, w.init, prec=prec, levels=L)
    k, sk_ms, box_ms, its = 0, 0.0, 0.0, 0
    for layer in range(L + 1):
        kappas = w.extra["layer_kappas"] if layer < L else [2.0, 1.0, 0.5, 0.25]
        for kappa in kappas:
            for _ in range(w.extra["layer_iters"]):
                st = ctx.iterate("AB"[k % 2], kappa / ctx.N ** 2, tol=tol, stop_rule=rule,
                                 max_iter=args.max_iter, check_every=args.check_every)
                k += 1
                sk_ms += st["t_sinkhorn_ms"]
                box_ms += st["t_b2c_ms"] + st["t_c2b_ms"]
                its += st["sk"]["iters_max"]
        if layer < L:
            ctx.refine()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev = ctx.evaluate()
    ctx.close()
    log(f"[bench] full multiscale solve {workload} {prec_name} tol {tol}: {wall:.2f} s, relative "
        f"PD gap {ev['pd_gap'] / ev['primal']:.3e}")
    return {"workload": workload, "grid": w.N, "seed": w.seed, "dtype": prec_name, "tol": tol,
            "wall_s": wall,
            "sinkhorn_s": sk_ms / 1e3, "bbox_and_balance_s": box_ms / 1e3, "half_iterations": k,
            "sinkhorn_iterations": its, "layers": [w.N >> (L - l) for l in range(L + 1)],
            "relative_pd_gap": ev["pd_gap"] / ev["primal"], "primal": ev["primal"],
            "dual": ev["dual"], "x_marginal_l1": ev["x_marginal_l1"],
            "y_marginal_l1": ev["y_marginal_l1"],
            "schedule": "eps = 2h^2, h^2, h^2/2 per layer, finest 2h^2, h^2, h^2/2, h^2/4, "
                        f"{w.extra['layer_iters']} half-iterations per stage"}


def paper_table(args, sizes=(64, 128, 256, 512, 1024), seeds=3):
    """The whole multiscale solve in float64 at tolerance 1e-4 (Table 1's DomDecGPU setting:
    s = 4, eps down to h^2/4 on the finest layer) at every grid size, `seeds` seeded mixture
    pairs per size (one at 1024^2); one JSON line."""
    rows = []
    for N in sizes:
        name = {512: "ms512", 1024: "ms1024"}.get(N, "ms256")
        recs = [full_solve(args, name, "f64", 1e-4, N=N, seed=sd)
                for sd in range(seeds if N < 1024 else 1)]
        rows.append({"grid": N, "seeds": [r["seed"] for r in recs],
                     "wall_s": [r["wall_s"] for r in recs],
                     "sinkhorn_s": [r["sinkhorn_s"] for r in recs],
                     "bbox_and_balance_s": [r["bbox_and_balance_s"] for r in recs],
                     "relative_pd_gap": [r["relative_pd_gap"] for r in recs],
                     "x_marginal_l1": [r["x_marginal_l1"] for r in recs],
                     "y_marginal_l1": [r["y_marginal_l1"] for r in recs]})
    print(json.dumps({"paper_table": rows, "dtype": "f64", "tol": 1e-4,
                      "data": "synthetic seeded Gaussian mixtures (8 blobs, 16 at 1024^2)"}),
          flush=True)


def global_record(args, workload):
    """global_sinkhorn on the whole grid of the workload's marginals, with eps-scaling from
    eps = 1 (the squared diameter scale) halving down to h^2/4, tolerance 1e-4 at every stage
    (the paper's), warm-started across stages: the global GPU Sinkhorn of the paper's
    comparison (Table 1), on the same GPU as the domain decomposition."""
    import torch

    import paper_2405_09400_amd as dd
    import synth
    w = synth.workload(workload, seed=args.seed)
    N = w.N
    dev = torch.device("cuda", torch.cuda.current_device())
    mu = torch.tensor(w.mu, dtype=torch.float64, device=dev)
    nu = torch.tensor(w.nu, dtype=torch.float64, device=dev)
    a = torch.zeros((N, N), dtype=torch.float64, device=dev)
    b = torch.zeros_like(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its, terms, dev_ms, status = 0, 0.0, 0.0, 0
    k = int(round(math.log2(N * N)))
    stages = []
    for e in range(k, -3, -1):
        kappa = 2.0 ** e
        status, st = dd.global_sinkhorn(mu, nu, kappa / N ** 2, a, b, tol=1e-4,
                                        max_iter=args.global_max_iter, raise_on_error=False)
        its += st["iters"]
        terms += st["lse_terms"]
        dev_ms += st["time_ms"]
        stages.append(st["iters"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    D = float((a * mu).sum() + (b * nu).sum())
    log(f"[bench] global Sinkhorn {N}x{N}: {wall:.1f} s, {its} iterations, err {st['err']:.2e}")
    return {"solver": "global_sinkhorn (float64, whole grid, no domain decomposition)",
            "grid": N, "tol": 1e-4, "wall_s": wall, "device_s": dev_ms / 1e3, "iterations": its,
            "iterations_per_stage": stages, "final_err": st["err"],
            "converged": bool(st["converged"]), "dual": D,
            "lse_tterm_s": terms / (dev_ms * 1e-3) / 1e12,
            "schedule": "eps = 2^k h^2 from 1 down to h^2/4, warm-started, tol 1e-4 per stage, "
                        f"at most {args.global_max_iter} iterations per stage"}


def measure(args, workload, prec, steps, warmup, replay=0, cpu=False):
    """Set-up (untimed), warm-up, `steps` timed half-iterations, then optionally the replay
    protocol and the oracle leg; returns the JSON record."""
    import torch

    import paper_2405_09400_amd as dd
    w, ctx, rule, k = setup(args, workload, prec)
    log(f"[bench] warmup {warmup} steps")
    warm_flows = []
    run_steps(ctx, w, warmup, k, args, rule, flows=warm_flows)
    k += warmup
    torch.cuda.synchronize()
    log(f"[bench] timing {steps} steps ({workload}, {prec})")
    t0 = time.perf_counter()
    flows = []
    stats = run_steps(ctx, w, steps, k, args, rule, flows=flows)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    k += steps
    if flows and "AB"[(k - 1) % 2] == "B":
        # the plan after a flow update has no composite potentials yet: evaluate after one
        # more (untimed) half-iteration
        run_steps(ctx, w, 1, k, args, rule)
        k += 1
    ev = ctx.evaluate()

    alg_bytes = sum(s["sk"]["alg_bytes"] for s in stats)
    terms = sum(s["sk"]["lse_terms"] for s in stats)
    sk_ms = sum(s["t_sinkhorn_ms"] for s in stats)
    sk_iters = [s["sk"]["iters_max"] for s in stats]
    launches = sum((s["sk"]["iters_max"] + 1) if rule == dd.DD_STOP_BATCH else 1 for s in stats)
    achieved = terms / (sk_ms * 1e-3)
    peak = TERM_PEAK if prec == "f32" else TERM_PEAK_F64
    # the dominant kernel: the register-blocked class with the most device time (HIP events on
    # the stream it is launched on, summed over the launches of the timed steps that iterated)
    roof_kernel, k_launch, k_ms, k_terms = "sinkhorn (all kernels of the solve)", launches, sk_ms, terms
    if all(s["sk"]["path"] == 1 for s in stats) and rule == dd.DD_STOP_BATCH:
        per = [(sum(s["sk"]["kernel_ms"][c] for s in stats), c) for c in (0, 1, 2)]
        ms_c, c = max(per)
        if ms_c > 0:
            names = ("fast_kernel<1, 4, true, 2> (box side <= 32: one wave per cell)",
                     "fast_kernel<4, 16, false, 2> (up to 2048 box entries: four waves per cell)",
                     "fast_kernel<8, 8, false, 2> (larger boxes: eight waves per cell)")
            roof_kernel = names[c]
            k_launch = sum(s["sk"]["kernel_launches"][c] for s in stats)
            k_ms = ms_c
            k_terms = sum(s["sk"]["kernel_terms"][c] for s in stats)
    k_achieved = k_terms / (k_ms * 1e-3)
    run_classes = sorted({(s["sk"]["wave_side"], s["sk"]["big_entries"]) for s in stats})
    traffic = traffic_bytes(roof_kernel, workload, run_classes) \
        if roof_kernel.startswith("fast_kernel") else None
    step_ms = [s["wall_ms"] for s in stats]
    log(f"[bench] steps: sinkhorn iters {sk_iters}, sinkhorn {sk_ms / len(stats):.3f} ms/step, "
        f"wall {wall * 1e3 / len(stats):.3f} ms/step")

    compare = None
    if replay:
        a = argparse.Namespace(**vars(args))
        a.replay = replay
        compare = time_to_tol(ctx, w, k, a, rule)
        k += compare.pop("_steps")

    cpu_rec = None
    if cpu:
        cpu_rec = cpu_baseline(args, w, ctx, k, rule)
        k += 1

    traffic_gb_s = (traffic / (k_ms / max(k_launch, 1) * 1e-3) / 1e9) if traffic is not None else None
    out = {
        "metric": "cell-Sinkhorn LSE GB/s + time-to-marginal-err 1e-5 at 512^2, warm-start vs plain",
        "value": alg_bytes / wall / 1e9,
        "unit": "GB/s",
        "value_kind": "algorithmic bytes (12 (|X_J| + W1 W2) per cell-iteration) / wall time of "
                      "the timed steps",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": wall * 1e3 / steps,
        "ms_per_step_median": float(np.median(step_ms)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic",
        "config": {
            "workload": WORKLOAD_TEXT.get(workload, workload).format(N=w.N, s=w.s),
            "tol": args.tol, "stop_rule": args.stop_rule, "check_every": args.check_every,
            "seed": args.seed,
            "cells_per_step": stats[0]["sk"]["ncells"],
        },
        "roofline": {
            "bound": "alu", "kernel": roof_kernel,
            "achieved": k_achieved / 1e12, "peak": peak / 1e12, "unit": "Tterm/s",
            "frac": k_achieved / peak, "traffic": traffic,
            "traffic_unit": "HBM bytes per launch",
            "traffic_gb_s": traffic_gb_s,
            "traffic_frac_of_hbm_peak": traffic_gb_s * 1e9 / HBM_PEAK if traffic_gb_s else None,
            "launches": k_launch, "kernel_ms_per_launch": k_ms / max(k_launch, 1),
            "terms_per_launch": k_terms / max(k_launch, 1),
            "all_sinkhorn_kernels_tterm_s": achieved / 1e12,
        },
        "cpu_baseline": cpu_rec,
        "error_vs_oracle": cpu_rec["gpu_vs_oracle"] if cpu_rec else None,
        # the register-blocked path's cell classes in the timed steps (the tuner's pick:
        # boxes with long side <= wave_side one wave, more than big_entries entries eight)
        "tuner": {"classes": sorted({(s["sk"]["wave_side"], s["sk"]["big_entries"])
                                     for s in stats}),
                  "candidates": [[32, 2048], [32, 1024], [32, 4096], [24, 2048], [24, 1024],
                                 [24, 4096]],
                  # host waits for the device per timed half-iteration (1: the composite
                  # boxes predicted by the previous iteration and the whole solve enqueued;
                  # more when the enqueued rounds were not enough and the solve was resumed)
                  "host_waits": [s["host_waits"] for s in stats],
                  "resumed": [s["spec_resumed"] for s in stats]},
        "time_to_tol": compare,
        "detail": {
            "step_ms": [round(t, 3) for t in step_ms],
            "sinkhorn_iters": sk_iters,
            "cell_split": [{"n_big": s["sk"]["n_big"], "n_giant": s["sk"]["n_giant"],
                            "lds_kb": s["sk"]["lds_kb"],
                            "tile_small": s["sk"]["tile_small"], "tile_big": s["sk"]["tile_big"]}
                           for s in stats[:2]],
            "finish_f64_iters": [s["sk"]["finish_iters_max"] for s in stats],
            "class_kernel_ms_per_step": [sum(s["sk"]["kernel_ms"][c] for s in stats) / len(stats)
                                         for c in (0, 1, 2)],
            "class_tterm_s": [sum(s["sk"]["kernel_terms"][c] for s in stats) /
                              max(sum(s["sk"]["kernel_ms"][c] for s in stats), 1e-9) / 1e9
                              for c in (0, 1, 2)],
            "main_ms_per_step": sum(s["sk"]["main_ms"] for s in stats) / len(stats),
            "sinkhorn_ms_per_step": sk_ms / len(stats),
            "b2c_ms_per_step": sum(s["t_b2c_ms"] for s in stats) / len(stats),
            "c2b_ms_per_step": sum(s["t_c2b_ms"] for s in stats) / len(stats),
            "device_ms_per_step": sum(s["t_total_ms"] for s in stats) / len(stats),
            "lse_terms_per_step": terms / len(stats),
            "max_box": [max(s["max_w1"] for s in stats), max(s["max_w2"] for s in stats)],
            "nu_entries": stats[-1]["nu_entries"],
            "x_marginal_l1": ev["x_marginal_l1"], "y_marginal_l1": ev["y_marginal_l1"],
            "primal": ev["primal"], "dual": ev["dual"], "pd_gap": ev["pd_gap"],
        },
    }
    if flows:
        out["detail"]["flow"] = {
            "updates": len(flows), "nodes": flows[0]["n_nodes"], "arcs": flows[0]["n_arcs"],
            "costs_ms": sum(f["t_costs_ms"] for f in flows) / len(flows),
            "mcf_ms": sum(f["t_mcf_ms"] for f in flows) / len(flows),
            "mcf_ms_each": [round(f["t_mcf_ms"], 2) for f in flows],
            "assemble_ms": sum(f["t_assemble_ms"] for f in flows) / len(flows),
            "value": [f["value"] for f in flows], "moved_mass": [f["moved_mass"] for f in flows],
            # the first update of the run (in the warm-up) solves its min-cost flow from scratch;
            # later ones start from the previous optimal basis
            "first_update_mcf_ms": warm_flows[0]["t_mcf_ms"] if warm_flows else None,
            # one cycle of the hybrid schedule: A, B, flow update
            "cycle_ms": wall * 1e3 / len(flows),
            "mcf_share_of_cycle": (sum(f["t_mcf_ms"] for f in flows) / (wall * 1e3)),
        }
    ctx.close()
    return out


if __name__ == "__main__":
    main()
