"""Benchmark: exact hypothesis evaluation on one MI355X.

A step is one batched exact evaluation of the whole hypothesis set of the
workload (host plan compile + every kernel, coverage counts left on the
device), with the knowledge base resident in HBM.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--config c2]
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

METRIC = "exact hypotheses/sec + achieved HBM GB/s; screened vs plain exhaustive"
HBM_PEAK_GBS = 8000.0
KIND_NAMES = {0: "k_threshold", 1: "k_region", 2: "k_role", 3: "k_tbuild", 4: "k_group", 5: "k_fill_rows",
              6: "k_dp_emit", 7: "k_group_short"}
# the dominant kernel's source: its counters are void once these change
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2412_00802_amd", "csrc", f)
                  for f in ("group_kernels.h", "hth_internal.h", "exec.hip")]
# the kernels that write every role node's row (or add a root's coverage) and
# read each (role, direction) CSR: the roofline's kernel family, against the
# byte model's role-pass bytes
ROLE_PASS_KINDS = (2, 4, 5, 7)          # k_role (+ heavy rows), k_group, k_fill_rows, k_group_short
ROLE_PASS_KERNELS = ("k_role", "k_role_heavy", "k_role_heavy_fix", "k_group", "k_group_short", "k_fill_rows")
TRAFFIC_DIR = os.path.join(ROOT, "profiles")          # traffic_<workload>.json: the counters of a workload
COPY_BYTES = 256 << 20      # elementwise pass used to calibrate the byte counters


def source_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def traffic_file(workload: str) -> str:
    return os.path.join(TRAFFIC_DIR, f"traffic_{workload}.json")


def recorded_traffic(kernels, workload: str):
    """HBM bytes per step of the kernels named in `kernels` (summed over their
    launches) from the committed counter summary of `workload`, or None when
    the kernel sources changed since the counters were taken."""
    try:
        rec = json.load(open(traffic_file(workload)))
    except (OSError, ValueError):
        return None
    if rec.get("source_sha") != source_sha():
        return None
    steps = rec.get("steps", 3)
    tot = 0.0
    for k in kernels:
        e = rec.get("kernels", {}).get(k)
        if e is not None:
            tot += e["hbm_bytes_per_launch"] * e["launches"] / steps
    return tot


def kernel_name(name: str) -> str:
    """A rocprofv3 kernel name without its arguments (anonymous namespaces dropped)."""
    return name.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "")[:60]


def summarize(kt_dir: str, fetch_dir: str, write_dir: str, command: str, out_md: str,
              sha: str = None, title: str = "c3 workload (4M individuals, 65,536 hypotheses, batched)",
              workload: str = "c3", tcc_dir: str = None) -> None:
    """Turn rocprofv3 outputs (kernel trace stats, FETCH_SIZE, WRITE_SIZE passes,
    each run with --calibrate-copy) into the committed summary and traffic file.
    sha: the kernel source hash of the profiled build (default: the current one)."""
    sha = sha or source_sha()
    import csv
    import glob

    def counters(d, name):
        per = {}
        for f in glob.glob(os.path.join(d, "*counter_collection.csv")):
            for r in csv.DictReader(open(f)):
                if r["Counter_Name"] != name:
                    continue
                k = r["Kernel_Name"].split("(")[0].replace("void ", "")
                e = per.setdefault(k, {"calls": set(), "kib": 0.0})
                e["calls"].add(r["Dispatch_Id"])
                e["kib"] += float(r["Counter_Value"])
        return {k: (len(v["calls"]), v["kib"] / len(v["calls"])) for k, v in per.items()}

    fetch, write = counters(fetch_dir, "FETCH_SIZE"), counters(write_dir, "WRITE_SIZE")
    copy = [k for k in fetch if "elementwise" in k.lower()]
    ck = max(copy, key=lambda k: fetch[k][1])
    # the copy reads and writes COPY_BYTES: bytes per counted KiB
    f_fac = COPY_BYTES / (fetch[ck][1] * 1024)
    w_fac = COPY_BYTES / (write[ck][1] * 1024)
    stats = []
    for f in glob.glob(os.path.join(kt_dir, "*kernel_stats.csv")):
        stats += list(csv.DictReader(open(f)))
    lines = [f"# rocprofv3 summary: {title}", "",
             "Command (kernel trace):", "", "    " + command.format(opts="--kernel-trace --stats --output-format csv"), "",
             "Counter passes (one counter per run):", "",
             "    " + command.format(opts="--pmc FETCH_SIZE --output-format csv"),
             "    " + command.format(opts="--pmc WRITE_SIZE --output-format csv"), "",
             f"Kernel source sha256[:16] of csrc/group_kernels.h + csrc/hth_internal.h + csrc/exec.hip: {sha}", "",
             "## Kernel time (kernel trace)", "",
             "| kernel | calls | avg us | total % |", "|---|---|---|---|"]
    for r in sorted(stats, key=lambda r: -float(r["Percentage"]))[:12]:
        lines.append(f"| {kernel_name(r['Name'])} | {r['Calls']} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
    lines += ["", "## Bytes (FETCH_SIZE / WRITE_SIZE, KiB per dispatch)", "",
              f"Calibration: `{ck[:50]}` (one elementwise pass over {COPY_BYTES >> 20} MiB written just before, into another buffer) reads "
              f"{fetch[ck][1]:.0f} KiB and writes {write[ck][1]:.0f} KiB per dispatch: "
              f"{f_fac:.3f} fetched bytes and {w_fac:.3f} written bytes per counted KiB-byte.", "",
              "| kernel | fetch KiB | write KiB | HBM bytes per launch (scaled) |", "|---|---|---|---|"]
    out = {"source_sha": sha, "fetch_factor": f_fac, "write_factor": w_fac, "steps": 3, "kernels": {}}
    agg = {}
    for k in sorted(fetch, key=lambda k: -fetch[k][1]):
        if k not in write:
            continue
        hb = fetch[k][1] * 1024 * f_fac + write[k][1] * 1024 * w_fac
        lines.append(f"| {k[:60]} | {fetch[k][1]:.0f} | {write[k][1]:.0f} | {hb / 1e6:.1f} MB |")
        # per launch over every instantiation of the kernel, weighted by launches
        base = k.split("<")[0].split("::")[-1]
        a = agg.setdefault(base, [0, 0.0, []])
        a[0] += fetch[k][0]
        a[1] += hb * fetch[k][0]
        a[2].append(k)
    for base, (n, tot, names) in agg.items():
        out["kernels"][base] = {"names": names, "launches": n, "hbm_bytes_per_launch": tot / n}
    lines += ["", "HBM bytes per launch over all instantiations (launch-weighted): " +
              ", ".join(f"{b} {v['hbm_bytes_per_launch'] / 1e6:.1f} MB" for b, v in
                        sorted(out["kernels"].items(), key=lambda kv: -kv[1]["hbm_bytes_per_launch"])[:6])]
    if tcc_dir:
        hit, miss = counters(tcc_dir, "TCC_HIT_sum"), counters(tcc_dir, "TCC_MISS_sum")
        lines += ["", "## L2 (TCC_HIT_sum / TCC_MISS_sum per dispatch)", "",
                  "    " + command.format(opts="--pmc TCC_HIT_sum TCC_MISS_sum --output-format csv"), "",
                  "| kernel | hits | misses | miss rate |", "|---|---|---|---|"]
        for k in sorted(miss, key=lambda k: -miss[k][1])[:10]:
            h, m = hit.get(k, (0, 0.0))[1], miss[k][1]
            lines.append(f"| {k[:60]} | {h:.3g} | {m:.3g} | {m / max(h + m, 1e-9):.2f} |")
    open(out_md, "w").write("\n".join(lines) + "\n")
    json.dump(out, open(traffic_file(workload), "w"), indent=1)


def summarize_trace(kt_dir: str, command: str, out_md: str, title: str, by_grid: str = None) -> None:
    """Kernel-time table of one rocprofv3 --kernel-trace --stats run; with
    by_grid, also the dispatches of the kernels whose names hold that text,
    grouped by grid (workgroups in x and y)."""
    import csv
    import glob
    stats = []
    for f in glob.glob(os.path.join(kt_dir, "*kernel_stats.csv")):
        stats += list(csv.DictReader(open(f)))
    lines = [f"# rocprofv3 summary: {title}", "", "Command:", "",
             "    " + command.format(opts="--kernel-trace --stats --output-format csv"), "",
             "| kernel | calls | avg us | total ms | total % |", "|---|---|---|---|---|"]
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:16]:
        lines.append(f"| {kernel_name(r['Name'])} | {r['Calls']} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['TotalDurationNs']) / 1e6:.1f} | "
                     f"{float(r['Percentage']):.1f} |")
    if by_grid:
        groups = {}
        for f in glob.glob(os.path.join(kt_dir, "*kernel_trace.csv")):
            for r in csv.DictReader(open(f)):
                if by_grid not in r["Kernel_Name"]:
                    continue
                key = (kernel_name(r["Kernel_Name"]), int(r["Grid_Size_X"]) // int(r["Workgroup_Size_X"]),
                       int(r["Grid_Size_Y"]))
                groups.setdefault(key, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
        tile = "; one 128 x 128 output tile each" if "gemm" in by_grid else ""
        lines += ["", f"Dispatches of `{by_grid}` by grid (workgroups in x, y{tile}):", "",
                  "| kernel | grid x, y | calls | avg us | total ms |", "|---|---|---|---|---|"]
        for (name, gx, gy), v in sorted(groups.items(), key=lambda kv: -sum(kv[1])):
            lines.append(f"| {name} | {gx}, {gy} | {len(v)} | {sum(v) / len(v):.1f} | {sum(v) / 1e3:.2f} |")
    open(out_md, "w").write("\n".join(lines) + "\n")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def describe(name, cfg, kb) -> str:
    hyps = (f"{cfg.n_hyps} hypotheses with node counts geometric on 1..31, 30% of child subtrees "
            f"drawn from a shared pool" if name == "c3" else
            f"{cfg.n_hyps} random hypotheses of depth <= {cfg.hyp_depth}")
    return (f"{name}: {cfg.n_individuals:,} individuals, {cfg.n_concepts} concepts (tree depth "
            f"{cfg.tree_depth}), {cfg.n_roles} roles / {kb.n_edges:,} assertions (Zipf s={cfg.zipf_s}, "
            f"cap {cfg.degree_cap}), {cfg.n_data} float32 properties ({int(cfg.missing * 100)}% missing), "
            f"{cfg.n_pos:,}+{cfg.n_neg:,} examples; {hyps}; batched exact evaluation")


def make_workload_hypotheses(name, cfg, kb):
    from paper_2412_00802_amd import synth
    if name == "c3":
        return synth.make_sized_hypotheses(cfg, kb)
    return synth.make_hypotheses(cfg, kb)


def cpu_info() -> dict:
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "model": model}


def cpu_baseline(kb, hyps, got, budget_s: float, runs: int):
    """The C++ oracle (one byte per membership, recursive, OpenMP over
    hypotheses) on a bounded sample: `runs` timed runs on all the cores this
    process may use and `runs` on one thread.  The sample is sized from a
    first probe so that all runs together take about budget_s seconds."""
    from oracle.cpp_oracle import CppOracle, batch_tokens
    info = cpu_info()
    threads = info["affinity"]
    t = time.perf_counter()
    o = CppOracle(kb)
    load_s = time.perf_counter() - t
    # probe: a few hypotheses on all threads
    probe = min(len(hyps), max(8, threads))
    toks, offs = batch_tokens(hyps[:probe])
    t = time.perf_counter()
    o.coverages_tokens(toks, offs, threads)
    per_hyp_1t = (time.perf_counter() - t) * threads / probe       # thread-seconds per hypothesis
    # all-core runs get ~2/3 of the budget, one-thread runs ~1/3
    n_all = int(min(len(hyps), max(threads, budget_s * 2 / 3 / runs / per_hyp_1t * threads)))
    n_one = int(min(n_all, max(2, budget_s / 3 / runs / per_hyp_1t)))
    toks, offs = batch_tokens(hyps[:n_all])
    rates_all, rates_one, want = [], [], None
    for _ in range(runs):
        t = time.perf_counter()
        want = o.coverages_tokens(toks, offs, threads)
        rates_all.append(n_all / (time.perf_counter() - t))
    t1, o1 = batch_tokens(hyps[:n_one])
    for _ in range(runs):
        t = time.perf_counter()
        o.coverages_tokens(t1, o1, 1)
        rates_one.append(n_one / (time.perf_counter() - t))
    o.close()
    parity = {"checked": n_all, "equal": int((got[:n_all] == want).all(axis=1).sum()), "against": "oracle/cpp"}
    rec = {"value": round(float(np.median(rates_all)), 2), "unit": "hypotheses/s", "cores": threads,
           "kind": "oracle",
           "sample": f"first {n_all} hypotheses of the batch (one thread: first {n_one}); oracle/cpp, one byte "
                     f"per membership, OpenMP over hypotheses; KB in RAM (conversion {load_s:.1f}s excluded); "
                     f"{runs} runs each, median",
           "all_cores": {"threads": threads, "runs": [round(r, 2) for r in rates_all],
                         "mean": round(float(np.mean(rates_all)), 2), "median": round(float(np.median(rates_all)), 2)},
           "one_thread": {"runs": [round(r, 3) for r in rates_one], "mean": round(float(np.mean(rates_one)), 3),
                          "median": round(float(np.median(rates_one)), 3)},
           "cpu": info}
    return rec, parity


def kernel_table(entries, steps):
    out = {}
    for k, e in enumerate(entries):
        if e["launches"]:
            out[KIND_NAMES.get(k, str(k))] = {
                "launches_per_step": e["launches"] / steps, "ms_per_step": round(e["ms"] / steps, 4),
                "model_GBps": round(e["bytes"] / (e["ms"] * 1e-3) / 1e9, 1) if e["ms"] else None}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c3")
    ap.add_argument("--host-plans", action="store_true",
                    help="time the host-compiled batch (hth_eval_batch) as the step instead of device plans")
    ap.add_argument("--other-steps", type=int, default=3, help="steps of the other plan path (0: skip)")
    ap.add_argument("--graph", type=int, default=10, metavar="REPLAYS",
                    help="replays of the step's plan launch captured in a HIP graph (0: skip)")
    ap.add_argument("--plain", type=int, default=256, help="hypotheses timed one at a time (0 = skip)")
    ap.add_argument("--cache-rows", type=int, default=32768,
                    help="rows of the cross-batch subexpression cache leg: the batch in four chunks, "
                         "with and without the cache (0: skip)")
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of the CPU-baseline runs (0: skip)")
    ap.add_argument("--cpu-runs", type=int, default=5)
    ap.add_argument("--c5", type=int, default=1, help="screened-search leg on the c3 KB (c3 only)")
    ap.add_argument("--c5-pairs", type=int, default=200_000)
    ap.add_argument("--c5-mode", default="logdelta", help="the screener of the c5 leg (see screened.py)")
    ap.add_argument("--c5-draws", type=int, default=3, help="candidate sets of the c5 leg")
    ap.add_argument("--c4-rounds", type=int, default=3, help="refinement-trace rounds at c4 (0: skip)")
    ap.add_argument("--time-budget", type=float, default=420.0,
                    help="seconds after which the optional legs are skipped")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--autotune", action="store_true", help="pick the schedule with the autotuner first")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain device copy of 256 MiB (byte-counter calibration)")
    ap.add_argument("--summarize", nargs=3, metavar=("KT_DIR", "FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--summary-out", default=os.path.join(ROOT, "profiles", "k_group_c3.md"))
    ap.add_argument("--summary-sha", default=None, help="kernel source hash of the profiled build")
    ap.add_argument("--summary-tcc", default=None, help="rocprofv3 output of the L2 hit/miss pass")
    ap.add_argument("--summarize-trace", default=None, metavar="KT_DIR",
                    help="write only the kernel-time table of a kernel-trace run")
    ap.add_argument("--summary-title", default="")
    ap.add_argument("--summary-by-grid", default=None, help="group these kernels' dispatches by grid")
    ap.add_argument("--summary-command", default="rocprofv3 {opts} -d OUT -o run -- python3 bench.py "
                    "--steps 2 --warmup 1 --plain 0 --cpu-budget 0 --c5 0 --c4-rounds 0 --graph 0 "
                    "--other-steps 0 --cache-rows 0 --no-profile --calibrate-copy")
    args = ap.parse_args()
    if args.summarize_trace:
        summarize_trace(args.summarize_trace, args.summary_command, args.summary_out, args.summary_title,
                        args.summary_by_grid)
        return
    if args.summarize:
        summarize(*args.summarize, args.summary_command, args.summary_out, args.summary_sha,
                  title=args.summary_title or f"{args.config} workload, batched", workload=args.config,
                  tcc_dir=args.summary_tcc)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU path is a "
              "design note, not implemented", file=sys.stderr)
        sys.exit(2)

    t_start = time.perf_counter()
    import torch
    from paper_2412_00802_amd import bytes_model, hthedl, synth

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    cfg = synth.CONFIGS[args.config]
    t = time.perf_counter()
    kb = synth.make_kb(cfg)
    hyps = make_workload_hypotheses(args.config, cfg, kb)
    log(f"[bench] generated {args.config} in {time.perf_counter() - t:.1f}s: {kb.n_edges:,} assertions")
    nodes, offs, ch = hthedl.encode_batch(hyps)
    t = time.perf_counter()
    eng = hthedl.Engine(kb, max_nodes=64, max_hyps=1)
    eng.ensure_workspace(hthedl.hth_batch_workspace_bytes(eng.handle, nodes, offs, ch))
    d_nodes, d_offs, d_ch = eng.upload_batch(encoded=(nodes, offs, ch))
    n_nodes = int(nodes.shape[0])
    eng.ensure_plan_scratch(n_nodes)
    torch.cuda.synchronize()
    log(f"[bench] uploaded + kb_create in {time.perf_counter() - t:.1f}s")
    H = len(hyps)
    stream = torch.cuda.current_stream()
    counts = torch.empty((H, 2), dtype=torch.int32, device="cuda")
    other = torch.empty((H, 2), dtype=torch.int32, device="cuda")

    def host_step(out):
        hthedl.hth_eval_batch(eng.handle, nodes, offs, ch, eng.ws, eng.ws_bytes, out, stream)

    def device_plan():
        plan, nb = hthedl.hth_dplan_create(eng.handle, d_nodes, n_nodes, d_offs, H, d_ch, int(d_ch.shape[0]),
                                           eng.dp_scratch, eng.dp_scratch_bytes, stream)
        eng.ensure_workspace(nb)
        return plan

    def device_step(out):
        # the node arrays are in HBM: the plan is generated there (count pass,
        # the summary read back, the emit pass) and run
        plan = device_plan()
        try:
            hthedl.hth_dplan_launch(plan, eng.ws, eng.ws_bytes, out, stream)
        finally:
            hthedl.hth_dplan_destroy(plan)

    step, other_step = (host_step, device_step) if args.host_plans else (device_step, host_step)
    schedule = None
    if args.autotune:
        from paper_2412_00802_amd import autotune
        schedule = autotune.autotune(eng, hyps, reps=1, cache=None, log=log)
        eng.ensure_workspace(hthedl.hth_batch_workspace_bytes(eng.handle, nodes, offs, ch))
        log(f"[bench] schedule {schedule}")
    if args.calibrate_copy:
        # the byte-counter calibration: one elementwise kernel reading a buffer
        # that was written first (so its pages are resident) and writing another
        src = torch.ones(COPY_BYTES // 4, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        dst = torch.add(src, 1)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        step(counts)
    torch.cuda.synchronize()
    if not args.no_profile:
        hthedl.hth_profile_begin(eng.handle)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(counts)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    entries = hthedl.hth_profile_end(eng.handle) if not args.no_profile else None
    got = counts.cpu().numpy().view(np.uint32).copy()
    value = H * args.steps / dt
    ms_step = dt / args.steps * 1e3
    log(f"[bench] batched ({'host' if args.host_plans else 'device'} plans): {value:,.0f} hyp/s "
        f"({ms_step:.3f} ms/step)")

    # the byte model of this batch: the roofline of the whole step
    t = time.perf_counter()
    shape = bytes_model.KBShape(kb)
    model = bytes_model.batch_model(hyps, shape)
    log(f"[bench] byte model in {time.perf_counter() - t:.1f}s: {bytes_model.summary(model)}")
    step_roofline = {"bound": "hbm", "model_bytes": model["total"], "achieved": round(model["total"] / dt * args.steps / 1e9, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(model["total"] / (dt / args.steps) / 1e9 / HBM_PEAK_GBS, 4),
                     "model_GB": bytes_model.summary(model)}

    roofline, kernels = None, {}
    if entries is not None:
        kernels = kernel_table(entries, args.steps)
        # the role passes: every role node's row written once (or a root's
        # coverage added without one) and each (role, direction) CSR read once
        # per level sweep -- the byte model's role-pass bytes -- over the
        # summed event time of the kernels that do it
        ms = sum(entries[k]["ms"] for k in ROLE_PASS_KINDS) / args.steps
        launches = sum(entries[k]["launches"] for k in ROLE_PASS_KINDS) / args.steps
        ach = model["role_pass"] / (ms * 1e-3) / 1e9
        traffic = recorded_traffic(ROLE_PASS_KERNELS, args.config) if not args.autotune else None
        roofline = {"kernel": "role passes (" + " + ".join(KIND_NAMES[k] for k in ROLE_PASS_KINDS) + ")",
                    "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(ach / HBM_PEAK_GBS, 4),
                    "traffic": traffic, "traffic_unit": "HBM bytes per step (counters, all launches of the family)",
                    "model_bytes_per_step": model["role_pass"], "ms_per_step": round(ms, 4),
                    "launches_per_step": launches, "avg_launch_ms": round(ms / max(launches, 1), 4),
                    "bytes_note": "byte model role-pass bytes: each (role, direction) CSR once per level sweep "
                                  "+ one row write per role node with a row (a node that is only a hypothesis's "
                                  "root gets its coverage fused, no row); reads of children are in step_roofline"}
        log(f"[bench] kernels: {json.dumps(kernels)}")

    elapsed = lambda: time.perf_counter() - t_start  # noqa: E731
    extra = {}
    # the other plan path, same batch: counts must agree
    if args.other_steps:
        other_step(other)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.other_steps):
            other_step(other)
        torch.cuda.synchronize()
        odt = time.perf_counter() - t0
        ogot = other.cpu().numpy().view(np.uint32)
        extra["host_plans" if not args.host_plans else "device_plans"] = {
            "value": round(H * args.other_steps / odt, 1), "unit": "hypotheses/s",
            "ms_per_step": round(odt / args.other_steps * 1e3, 3), "equal": bool((ogot == got).all())}
        log(f"[bench] other path: {extra}")

    # one device plan launched eagerly, then captured in a HIP graph and replayed
    if args.graph:
        plan = device_plan()
        try:
            gc = torch.empty((H, 2), dtype=torch.int32, device="cuda")
            hthedl.hth_dplan_launch(plan, eng.ws, eng.ws_bytes, gc, stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.graph):
                hthedl.hth_dplan_launch(plan, eng.ws, eng.ws_bytes, gc, stream)
            torch.cuda.synchronize()
            eager = (time.perf_counter() - t0) / args.graph
            g = torch.cuda.CUDAGraph()
            side = torch.cuda.Stream()
            side.wait_stream(stream)
            with torch.cuda.stream(side):
                g.capture_begin()
                hthedl.hth_dplan_launch(plan, eng.ws, eng.ws_bytes, gc, side)
                g.capture_end()
            stream.wait_stream(side)
            torch.cuda.synchronize()
            ok = True
            t_rep = 0.0
            for _ in range(args.graph):
                gc.fill_(-1)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                g.replay()
                torch.cuda.synchronize()
                t_rep += time.perf_counter() - t0
                ok &= bool((gc.cpu().numpy().view(np.uint32) == got).all())
            extra["graph"] = {"replays": args.graph, "replay_ms": round(t_rep / args.graph * 1e3, 3),
                              "eager_launch_ms": round(eager * 1e3, 3),
                              "replay_hyp_per_s": round(H / (t_rep / args.graph), 1),
                              "every_replay_equal": ok,
                              "note": "the same device plan launched eagerly and replayed from one capture; "
                                      "plan generation (count pass, readback) is outside both"}
            del g
        finally:
            hthedl.hth_dplan_destroy(plan)
        log(f"[bench] graph: {extra['graph']}")

    if args.cache_rows:
        extra["cache"] = cache_leg(eng, nodes, offs, ch, H, got, args.cache_rows, stream, log)

    if args.plain:
        P = min(args.plain, H)
        pc = torch.empty((P, 2), dtype=torch.int32, device="cuda")
        enc = [hthedl.encode_one(h) for h in hyps[:P]]
        eng.reserve(max(e[0].shape[0] for e in enc), 1)
        for i in range(min(8, P)):
            hthedl.hth_eval_one(eng.handle, enc[i][0], enc[i][1], eng.ws, eng.ws_bytes, None, pc[i], stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(P):
            hthedl.hth_eval_one(eng.handle, enc[i][0], enc[i][1], eng.ws, eng.ws_bytes, None, pc[i], stream)
        torch.cuda.synchronize()
        pdt = time.perf_counter() - t0
        pgot = pc.cpu().numpy().view(np.uint32)
        pm = sum(bytes_model.plain_model(h, shape) for h in hyps[:P])
        extra["plain"] = {"value": round(P / pdt, 1), "unit": "hypotheses/s", "hyps": P,
                          "equal_to_batched": bool((pgot == got[:P]).all()),
                          "model_frac": round(pm / pdt / 1e9 / HBM_PEAK_GBS, 4)}
        log(f"[bench] plain: {extra['plain']}")

    cpu, parity = None, None
    if args.cpu_budget > 0:
        cpu, parity = cpu_baseline(kb, hyps, got, args.cpu_budget, args.cpu_runs)
        log(f"[bench] oracle/cpp: {cpu}; parity {parity}")

    if args.c5 and args.config == "c3" and elapsed() < args.time_budget:
        from paper_2412_00802_amd import screened
        t = time.perf_counter()
        c5 = screened.run(kb, eng, pairs=args.c5_pairs, modes=(args.c5_mode,), sweep=(), name="c3",
                          draws=args.c5_draws)
        scr = c5["screener"][args.c5_mode]
        extra["c5"] = {"screened_hyp_per_s": scr["screened_hyp_per_s"],
                       "exhaustive_hyp_per_s": c5["exhaustive_hyp_per_s"], "speedup": scr["speedup"],
                       "recall_at_100": scr["recall_at_100"], "exact_budget": scr["exact_budget"],
                       "candidates": c5["candidates"], "stages_s": scr["stages_synchronised"],
                       "screened_seconds": scr["screened_seconds"], "exhaustive_seconds": c5["exhaustive_seconds"],
                       "train_seconds": scr["train_seconds"], "training_pairs": c5["training_pairs"],
                       "random_recall_at_100": c5["random_recall_at_100"], "screener": args.c5_mode,
                       "draws": c5["draws"], "recall_at_100_per_draw": c5["recall_at_100_per_draw"][args.c5_mode],
                       "recall_at_100_mean": c5["recall_at_100_mean"][args.c5_mode],
                       "recall_at_100_min": c5["recall_at_100_min"][args.c5_mode],
                       "leg_seconds": round(time.perf_counter() - t, 1)}
        log(f"[bench] c5: {extra['c5']}")

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "hypotheses/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": describe(args.config, cfg, kb), "n_hyps": H,
                   "n_individuals": cfg.n_individuals, "n_assertions": kb.n_edges,
                   "mode": "batched, plans generated on the device" if not args.host_plans else
                           "batched, plans compiled on the host",
                   "schedule": schedule or hthedl.hth_kb_get_tuning(eng.handle)},
        "roofline": roofline, "step_roofline": step_roofline, "cpu_baseline": cpu,
        "parity_sample": parity, "kernels": kernels,
    }
    out.update(extra)

    if args.c4_rounds and elapsed() < args.time_budget:
        del eng, d_nodes, d_offs, d_ch, counts, other
        kb = None
        torch.cuda.empty_cache()
        out["c4"] = c4_leg(args.c4_rounds, log)
    print(json.dumps(out), flush=True)


def cache_leg(eng, nodes, offs, ch, H, got, n_rows, stream, log) -> dict:
    """The batch in four consecutive chunks (host-compiled plans), first without
    and then with the cross-batch subexpression cache: later chunks read the
    role restrictions they share with earlier ones from the cache's rows."""
    import torch
    from paper_2412_00802_amd import hthedl
    q = (H + 3) // 4
    chunks = [hthedl.slice_encoded((nodes, offs, ch), a, min(H, a + q)) for a in range(0, H, q)]
    for c in chunks:
        eng.ensure_workspace(hthedl.hth_batch_workspace_bytes(eng.handle, *c))
    out = torch.empty((H, 2), dtype=torch.int32, device="cuda")

    def run(cache):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i, c in enumerate(chunks):
            o = out[i * q:i * q + int(c[1].shape[0]) - 1]
            if cache is None:
                hthedl.hth_eval_batch(eng.handle, *c, eng.ws, eng.ws_bytes, o, stream)
            else:
                hthedl.hth_eval_batch_cached(eng.handle, cache, *c, eng.ws, eng.ws_bytes, o, stream)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    run(None)
    t_plain = run(None)
    rows = torch.empty((n_rows, eng.S), dtype=torch.int64, device="cuda")
    cache = hthedl.hth_cache_create(eng.handle, rows, n_rows)
    try:
        t_cached = run(cache)
        equal = bool((out.cpu().numpy().view(np.uint32) == got).all())
        st = hthedl.hth_cache_stats(cache)
    finally:
        hthedl.hth_cache_destroy(cache)
    del rows
    rec = {"chunks": len(chunks), "rows": n_rows, "row_bytes": eng.S * 8,
           "ms_without": round(t_plain * 1e3, 3), "ms_with": round(t_cached * 1e3, 3),
           "hyp_per_s_with": round(H / t_cached, 1), "equal": equal,
           "hits": st["hits"], "misses": st["misses"], "evictions": st["evictions"],
           "note": "four chunks of the batch in order, host-compiled plans, each chunk reading the role "
                   "restrictions earlier chunks left in the cache"}
    log(f"[bench] cache: {rec}")
    return rec


def c4_leg(rounds: int, log) -> dict:
    """A few rounds of the c4 refinement trace (32M individuals, 16,384
    candidates per round, added conjuncts drawn on the device): device and
    end-to-end hypotheses/s per round."""
    from paper_2412_00802_amd import hthedl, synth, trace
    t = time.perf_counter()
    cfg = synth.CONFIGS["c4"]
    kb = synth.make_kb(cfg)
    gen_s = time.perf_counter() - t
    t = time.perf_counter()
    eng = hthedl.Engine(kb, max_nodes=64, max_hyps=1)
    up_s = time.perf_counter() - t
    cache = trace.SetCache(eng, 4096)
    rng = np.random.default_rng(synth.BASE_SEED + 40)
    recs = []
    for rec, _, _ in trace.run_trace_device(cfg, kb, eng, rounds, 16384, 256, 16384, cache, rng,
                                            synth.BASE_SEED + 41):
        log(f"[bench] c4 round {rec['round']}: {rec}")
        recs.append(rec)
    cache.close()
    later = recs[1:] or recs
    dev = sum(r["device_ms"] + r["set_fill_ms"] for r in later) / 1e3
    e2e = sum(r["end_to_end_s"] for r in later)
    n = sum(r["candidates"] for r in later)
    return {"workload": f"c4: {kb.n:,} individuals, {kb.n_edges:,} assertions, {kb.n_data} properties; "
                        f"{rounds} trace rounds x 16,384 candidates, beam 256, added conjuncts drawn on the device",
            "device_hyp_per_s": round(n / dev, 1), "end_to_end_hyp_per_s": round(n / e2e, 1),
            "rounds_counted": len(later), "kb_generate_s": round(gen_s, 1), "kb_upload_s": round(up_s, 1),
            "rounds": recs}


if __name__ == "__main__":
    main()
