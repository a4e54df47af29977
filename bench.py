"""Benchmark: batched cell-Sinkhorn inside domain decomposition on one MI355X.

Workload (mix512): mu, nu = seeded 8-blob Gaussian mixtures (+1e-4 floor) on 512x512,
basic cells 4x4 (16,384 basic cells; 4,096 A / 4,225 B composite problems), initial
coupling = Knothe-Rosenblatt.  Untimed set-up: eps-scaling kappa = eps/h^2 = 64, 32, ..., 2
with 4 DD iterations per stage.  Timed: K domain-decomposition iterations (alternating A/B)
at kappa = 1 (eps = h^2), Sinkhorn tolerance 1e-5 on the X-marginal (App. A.2.1 rule),
warm-started from the previous visit of the partition.  A step = one DD iteration =
BasicToComposite + cell Sinkhorn to tolerance + CompositeToBasic + balancing + truncation.

value  = algorithmic LSE bytes of the timed steps / wall time of the timed steps (GB/s);
         12 (|X_J| + W1 W2) bytes per cell per Sinkhorn iteration (read f, log nu_J, write g;
         read g, log nu_J, log mu, write f -- 4 bytes each at float32).
roofline: the Sinkhorn kernel does one multiply-add per LSE term (exponentials per input
         and output only): achieved = LSE terms / kernel time, peak = the FP32 vector rate
         157.3 TFLOP/s / 2 FLOP per term.
cpu_baseline: the oracle's dense float64 cell solver on a bounded sample of the same
         workload's cell problems, on the host's cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# LSE terms/s: one fused multiply-add per term at the FP32 vector peak (157.3 TFLOP/s)
TERM_PEAK = 157.3e12 / 2
HBM_PEAK = 8.0e12


WORKLOAD_TEXT = {
    "mix512": "mix512: {N}x{N} 8-blob Gaussian mixtures + 1e-4 floor, s={s}, KR init, "
              "eps-scaling 64..2 untimed, timed DD iterations at eps=h^2",
    "mix256": "mix256: {N}x{N} 8-blob Gaussian mixtures + 1e-4 floor, s={s}, KR init, "
              "eps-scaling 64..2 untimed, timed DD iterations at eps=h^2",
    "mix1024": "mix1024: {N}x{N} 16-blob Gaussian mixtures + 1e-4 floor, s={s}, KR init, "
               "eps-scaling 64..2 untimed, timed DD iterations at eps=h^2",
    "flow512": "flow512: {N}x{N}, mu 8-blob mixture, nu = mu rotated 30 deg, contracted 0.36, "
               "shifted (0.25, 0); s={s}; map init; eps=h^2; hybrid A, B, flow update",
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def setup(args):
    import torch

    import paper_2405_09400_amd as dd
    import synth

    w = synth.workload(args.workload, seed=args.seed)
    prec = dd.DD_PREC_F32 if args.prec == "f32" else dd.DD_PREC_F64
    t0 = time.perf_counter()
    ctx = dd.DomDec(w.mu, w.nu, w.s, w.init, prec=prec)
    log(f"[bench] init {args.workload} N={w.N} s={w.s} in {time.perf_counter() - t0:.2f}s")
    rule = dd.DD_STOP_CELL if args.stop_rule == "cell" else dd.DD_STOP_BATCH
    k = 0
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
        st = ctx.iterate(part, eps, tol=args.tol, stop_rule=rule, max_iter=args.max_iter,
                         check_every=args.check_every,
                         init=dd.DD_INIT_PREV if init is None else init)
        out.append(st)
        if flow_every and part == "B":
            fs = ctx.flow_update()
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
    rec = {name: {"ms": [], "iters": [], "sinkhorn_ms": [], "init_ms": []} for name, _ in kinds}
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
            d["iters"].append(st["sk"]["iters_max"])
    out = {"tol": args.tol, "states": args.replay, "_steps": args.replay}
    for name, _ in kinds:
        out[name] = rec[name]
    if not net:
        out["learned_net"] = None
    tot = {name: sum(rec[name]["ms"]) for name, _ in kinds}
    out["speedup_prev_vs_zero"] = tot["zero"] / tot["prev_iterate"]
    if net:
        out["speedup_net_vs_zero"] = tot["zero"] / tot["learned_net"]
        out["speedup_net_vs_prev"] = tot["prev_iterate"] / tot["learned_net"]
        ctx.set_net(None)
        net.close()
    return out


def cpu_baseline(args, w):
    """Oracle dense cell Sinkhorn on a bounded sample: the first composite cells of partition A
    on the workload's initial coupling at kappa = 1, a fixed number of iterations."""
    import oracle

    t0 = time.perf_counter()
    od = oracle.DomDec(w.mu, w.nu, w.s, w.init)
    log(f"[bench] oracle state built in {time.perf_counter() - t0:.1f}s")
    eps = w.kappas[-1] / w.N ** 2
    parts = od.parts["A"]
    iters = 10
    nthreads = os.cpu_count() or 1
    done_cells, t_used, bytes_alg = 0, 0.0, 0.0
    chunk = 64
    while t_used < args.cpu_seconds:
        start = done_cells % len(parts)
        cells = parts[start:start + chunk]
        xo, yo, X, M, Y, V = [0], [0], [], [], [], []
        for basic in cells:
            xpix = np.concatenate([od.cells[i] for i in basic])
            ysup, nuJ = oracle.sparse_sum([od.nu_i[i] for i in basic])
            X.append(od.coords[xpix])
            M.append(od.mu[xpix])
            Y.append(od.coords[ysup])
            V.append(nuJ)
            xo.append(xo[-1] + len(xpix))
            yo.append(yo[-1] + len(ysup))
            k1, k2 = ysup // w.N, ysup % w.N
            W1 = int(k1.max() - k1.min() + 1)
            W2 = int(k2.max() - k2.min() + 1)
            bytes_alg += iters * 12.0 * (len(xpix) + W1 * W2)
        Vc = np.concatenate(V)
        t1 = time.perf_counter()
        oracle.sinkhorn_cells(np.array(xo), np.concatenate(X), np.concatenate(M), np.array(yo),
                              np.concatenate(Y), Vc, Vc, eps, fixed_iters=iters, nthreads=nthreads)
        t_used += time.perf_counter() - t1
        done_cells += len(cells)
    return {"value": bytes_alg / t_used / 1e9, "unit": "GB/s", "cores": nthreads, "kind": "oracle",
            "sample": f"{done_cells} cell solves (partition A cells in order, repeated) on the initial "
                      f"coupling at kappa=1, {iters} dense float64 Sinkhorn iterations each "
                      f"({t_used:.1f}s of solver time)"}


# ---- HBM traffic of the dominant kernel (rocprofv3 counters) ------------------------------
#
# `traffic` in the roofline line is read from a committed counter summary: FETCH_SIZE and
# WRITE_SIZE (KiB per dispatch, one rocprofv3 --pmc run each) averaged over the dispatches of
# the timed steps, each scaled by what the same counter reads for a plain copy of known size
# (--copy-calibration).  The summary records the SHA-256 of the kernel's source; when the
# source has changed since, traffic is null.

KERNEL_SOURCE = os.path.join(ROOT, "paper_2405_09400_amd", "csrc", "fastcell.hip")
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "fast_kernel_mix512_traffic.md")
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
    cmd_b = ("rocprofv3 --pmc {c} --kernel-trace -d <out> -o run --output-format csv -- "
             "python3 bench.py --steps 3 --warmup 1 --no-compare --no-cpu-baseline")
    cmd_c = ("rocprofv3 --pmc {c} --kernel-trace -d <out> -o run --output-format csv -- "
             "python3 bench.py --copy-calibration")
    kinds = " ".join(f"'{k}'" for k in args.traffic_kernel)
    lines = ["# HBM traffic of the register-blocked kernels, mix512 (512², s = 4, κ = 1, tol 1e-5, "
             "batch rule)", "",
             "Commands (from the repository root on the MI355X machine, after `cd /tmp && export "
             "TMPDIR=/tmp`; one counter per run):", "", "```",
             cmd_b.format(c="FETCH_SIZE"), cmd_b.format(c="WRITE_SIZE"),
             cmd_c.format(c="FETCH_SIZE"), cmd_c.format(c="WRITE_SIZE"), "```", "",
             f"Summarised by `python bench.py --traffic-from <four output dirs> --traffic-kernel "
             f"{kinds} --traffic-last {last}`.", "",
             f"Copy of 256 MiB: FETCH_SIZE reads {sum(f_copy) / len(f_copy):.0f} KiB (scale "
             f"{ff:.3f}), WRITE_SIZE {sum(w_copy) / len(w_copy):.0f} KiB (scale {wf:.3f}).", "",
             "| kernel | FETCH_SIZE KiB per dispatch | WRITE_SIZE KiB per dispatch | HBM bytes per "
             "launch (scaled) |", "|---|---:|---:|---:|"]
    recs = []
    for kern in args.traffic_kernel:
        fk = _per_dispatch(f_rows, kern)[-last:]
        wk = _per_dispatch(w_rows, kern)[-last:]
        fkib, wkib = sum(fk) / len(fk), sum(wk) / len(wk)
        rec = {"kernel": kern, "source_sha256": source_sha256(), "dispatches": len(fk),
               "fetch_kib_per_dispatch": fkib, "write_kib_per_dispatch": wkib,
               "fetch_factor": ff, "write_factor": wf,
               "bytes_per_launch": (fkib * ff + wkib * wf) * 1024.0}
        recs.append(rec)
        lines.append(f"| `{kern}` | {fkib:.1f} | {wkib:.1f} | {rec['bytes_per_launch']:.4g} |")
    lines += ["", f"Averaged over the last {last} dispatches of each kernel (the launches of the "
              "timed steps, the ones after the stop, which exit at once, included).", ""]
    lines += ["traffic-json: " + json.dumps(r) for r in recs]
    with open(args.traffic_out, "w") as f:
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
    cmd = ("rocprofv3 --kernel-trace --stats -d <out> -o run --output-format csv -- "
           "python3 bench.py --steps 3 --warmup 1 --no-compare --no-cpu-baseline")
    lines = ["# Cell Sinkhorn kernels, mix512 (512², s = 4, κ = 1, tol 1e-5, batch rule)", "",
             "Command (from the repository root on the MI355X machine, after `cd /tmp && export "
             "TMPDIR=/tmp`):", "", "```", cmd, "```", "",
             f"Summarised by `python bench.py --trace-from <out> --traffic-last "
             f"{args.traffic_last}`.  Kernel source SHA-256 (fastcell.hip): "
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
    with open(args.trace_out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def traffic_bytes(kernel_name):
    """HBM bytes per launch of `kernel_name` from the committed summary, or None when there is
    none, it covers another kernel, or the kernel's source has changed since."""
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    for line in open(TRAFFIC_SUMMARY):
        if line.startswith("traffic-json: "):
            rec = json.loads(line[len("traffic-json: "):])
            if rec["kernel"] in kernel_name and rec["source_sha256"] == source_sha256():
                return rec["bytes_per_launch"]
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="mix512")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--tol", type=float, default=1e-5)
    ap.add_argument("--max-iter", type=int, default=20000)
    ap.add_argument("--stop-rule", choices=["batch", "cell"], default="batch")
    ap.add_argument("--check-every", type=int, default=8,
                    help="batch rule: iterations between stop tests (register-blocked path)")
    ap.add_argument("--prec", choices=["f32", "f64"], default="f32")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--replay", type=int, default=4)
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
    ap.add_argument("--traffic-out", default=TRAFFIC_SUMMARY)
    ap.add_argument("--trace-from", metavar="DIR",
                    help="write the kernel-time summary of a rocprofv3 kernel-trace run")
    ap.add_argument("--trace-out", default=os.path.join(ROOT, "profiles", "fast_kernel_mix512.md"))
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
    dd.lib()

    w, ctx, rule, k = setup(args)
    log(f"[bench] warmup {args.warmup} steps")
    run_steps(ctx, w, args.warmup, k, args, rule)
    k += args.warmup
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} steps")
    t0 = time.perf_counter()
    flows = []
    stats = run_steps(ctx, w, args.steps, k, args, rule, flows=flows)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    k += args.steps
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
    traffic = traffic_bytes(roof_kernel) if roof_kernel.startswith("fast_kernel") else None
    log(f"[bench] steps: sinkhorn iters {sk_iters}, sinkhorn {sk_ms / len(stats):.3f} ms/step, "
        f"wall {wall * 1e3 / len(stats):.3f} ms/step")

    compare = None
    if not args.no_compare:
        compare = time_to_tol(ctx, w, k, args, rule)
        k += compare.pop("_steps")

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args, w)

    out = {
        "metric": "cell-Sinkhorn LSE GB/s + time-to-marginal-err 1e-5 at 512^2, warm-start vs plain",
        "value": alg_bytes / wall / 1e9,
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.prec == "f32" else "f64",
        "data": "synthetic",
        "config": {
            "workload": WORKLOAD_TEXT.get(args.workload, args.workload).format(N=w.N, s=w.s),
            "tol": args.tol, "stop_rule": args.stop_rule, "check_every": args.check_every,
            "seed": args.seed,
            "cells_per_step": stats[0]["sk"]["ncells"],
        },
        "roofline": {
            "bound": "alu", "kernel": roof_kernel,
            "achieved": k_achieved / 1e12, "peak": TERM_PEAK / 1e12, "unit": "Tterm/s",
            "frac": k_achieved / TERM_PEAK, "traffic": traffic,
            "traffic_unit": "HBM bytes per launch",
            "traffic_gb_s": (traffic / (k_ms / max(k_launch, 1) * 1e-3) / 1e9
                             if traffic is not None else None),
            "launches": k_launch, "kernel_ms_per_launch": k_ms / max(k_launch, 1),
            "terms_per_launch": k_terms / max(k_launch, 1),
            "all_sinkhorn_kernels_tterm_s": achieved / 1e12,
        },
        "cpu_baseline": cpu,
        "time_to_tol": compare,
        "detail": {
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
            "assemble_ms": sum(f["t_assemble_ms"] for f in flows) / len(flows),
            "value": [f["value"] for f in flows], "moved_mass": [f["moved_mass"] for f in flows],
        }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
