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
              6: "k_dp_emit"}
# the dominant kernel's source: its counters are void once these change
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2412_00802_amd", "csrc", f)
                  for f in ("group_kernels.h", "hth_internal.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_c2.json")   # counters of the c2 workload
COPY_BYTES = 256 << 20      # elementwise pass used to calibrate the byte counters


def source_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def recorded_traffic(kernel: str, traffic_file: str = TRAFFIC_FILE):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when the kernel source changed since the counters were taken."""
    try:
        rec = json.load(open(traffic_file))
    except (OSError, ValueError):
        return None
    if rec.get("source_sha") != source_sha():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k["hbm_bytes_per_launch"]


def kernel_name(name: str) -> str:
    """A rocprofv3 kernel name without its arguments (anonymous namespaces dropped)."""
    return name.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "")[:60]


def summarize(kt_dir: str, fetch_dir: str, write_dir: str, command: str, out_md: str,
              sha: str = None, title: str = "c2 workload (1M individuals, 4096 hypotheses, batched)",
              traffic_file: str = TRAFFIC_FILE, tcc_dir: str = None) -> None:
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
             f"Kernel source sha256[:16] of csrc/group_kernels.h + csrc/hth_internal.h: {sha}", "",
             "## Kernel time (kernel trace)", "",
             "| kernel | calls | avg us | total % |", "|---|---|---|---|"]
    for r in sorted(stats, key=lambda r: -float(r["Percentage"]))[:12]:
        lines.append(f"| {kernel_name(r['Name'])} | {r['Calls']} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
    lines += ["", "## Bytes (FETCH_SIZE / WRITE_SIZE, KiB per dispatch)", "",
              f"Calibration: `{ck[:50]}` (one elementwise pass over {COPY_BYTES >> 20} MiB of untouched memory) reads "
              f"{fetch[ck][1]:.0f} KiB and writes {write[ck][1]:.0f} KiB per dispatch: "
              f"{f_fac:.3f} fetched bytes and {w_fac:.3f} written bytes per counted KiB-byte.", "",
              "| kernel | fetch KiB | write KiB | HBM bytes per launch (scaled) |", "|---|---|---|---|"]
    out = {"source_sha": sha, "fetch_factor": f_fac, "write_factor": w_fac, "kernels": {}}
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
    json.dump(out, open(traffic_file, "w"), indent=1)


def summarize_trace(kt_dir: str, command: str, out_md: str, title: str) -> None:
    """Kernel-time table of one rocprofv3 --kernel-trace --stats run."""
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


def cpu_baseline(kb, hyps, sample: int, budget_s: float):
    from oracle import Oracle
    o = Oracle(kb)
    for r in range(kb.n_roles):          # the KB resident in RAM before timing
        o.assertions(r)
    t0 = time.perf_counter()
    out = []
    for h in hyps[:sample]:
        out.append(o.coverage(h))
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return np.asarray(out, dtype=np.uint32).reshape(-1, 2), dt


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--plain", type=int, default=512, help="hypotheses timed one at a time (0 = skip)")
    ap.add_argument("--cpu-sample", type=int, default=512)
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--device-plans", type=int, default=5, metavar="STEPS",
                    help="also time STEPS evaluations of the batch with plans generated on the device (0: skip)")
    ap.add_argument("--device-chunk", type=int, default=0,
                    help="hypotheses per device plan (0: the whole batch in one plan)")
    ap.add_argument("--autotune", action="store_true", help="pick the schedule with the autotuner first")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain device copy of 256 MiB (byte-counter calibration)")
    ap.add_argument("--summarize", nargs=3, metavar=("KT_DIR", "FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--summary-out", default=os.path.join(ROOT, "profiles", "k_group_c2.md"))
    ap.add_argument("--summary-sha", default=None, help="kernel source hash of the profiled build")
    ap.add_argument("--summary-tcc", default=None, help="rocprofv3 output of the L2 hit/miss pass")
    ap.add_argument("--summarize-trace", default=None, metavar="KT_DIR",
                    help="write only the kernel-time table of a kernel-trace run")
    ap.add_argument("--summary-title", default="")
    ap.add_argument("--summary-command", default="rocprofv3 {opts} -d OUT -o run -- python3 bench.py "
                    "--steps 2 --warmup 1 --plain 0 --cpu-sample 0 --no-profile --calibrate-copy")
    args = ap.parse_args()
    if args.summarize_trace:
        summarize_trace(args.summarize_trace, args.summary_command, args.summary_out, args.summary_title)
        return
    if args.summarize:
        summarize(*args.summarize, args.summary_command, args.summary_out, args.summary_sha,
                  tcc_dir=args.summary_tcc)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU path is a "
              "design note, not part of this build", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2412_00802_amd import hthedl, synth

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
    torch.cuda.synchronize()
    log(f"[bench] uploaded + kb_create in {time.perf_counter() - t:.1f}s; workspace {eng.ws_bytes / 2**30:.2f} GiB")
    H = len(hyps)
    counts = torch.empty((H, 2), dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()

    def step():
        hthedl.hth_eval_batch(eng.handle, nodes, offs, ch, eng.ws, eng.ws_bytes, counts, stream)

    schedule = None
    if args.autotune:
        from paper_2412_00802_amd import autotune
        schedule = autotune.autotune(eng, hyps, reps=1, cache=None, log=log)
        eng.ensure_workspace(hthedl.hth_batch_workspace_bytes(eng.handle, nodes, offs, ch))
        log(f"[bench] schedule {schedule}")
    if args.calibrate_copy:
        # one elementwise kernel over memory nothing has touched: reads and
        # writes COPY_BYTES each (the byte-counter calibration)
        src = torch.empty(COPY_BYTES // 4, dtype=torch.int32, device="cuda")
        dst = torch.add(src, 1)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if not args.no_profile:
        hthedl.hth_profile_begin(eng.handle)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    entries = None
    if not args.no_profile:
        entries = hthedl.hth_profile_end(eng.handle)
    got = counts.cpu().numpy().view(np.uint32).copy()
    value = H * args.steps / dt
    log(f"[bench] batched: {value:,.0f} hyp/s ({dt / args.steps * 1e3:.3f} ms/step)")

    roofline = None
    kernels = {}
    if entries is not None:
        for k, e in enumerate(entries):
            if e["launches"]:
                kernels[KIND_NAMES.get(k, str(k))] = {
                    "launches_per_step": e["launches"] / args.steps,
                    "ms_per_step": e["ms"] / args.steps,
                    "GBps": e["bytes"] / (e["ms"] * 1e-3) / 1e9 if e["ms"] else None}
        dom = max(range(len(entries)), key=lambda k: entries[k]["ms"])
        e = entries[dom]
        ach = e["bytes"] / (e["ms"] * 1e-3) / 1e9
        roofline = {"kernel": KIND_NAMES.get(dom), "bound": "hbm", "achieved": round(ach, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                    "traffic": recorded_traffic(KIND_NAMES.get(dom)) if args.config == "c2" and not args.autotune
                    else None,
                    "algorithmic_bytes_per_launch": e["bytes"] / e["launches"],
                    "avg_launch_ms": e["ms"] / e["launches"]}
        log(f"[bench] kernels: {json.dumps(kernels)}")

    plain = None
    if args.plain:
        P = min(args.plain, H)
        pc = torch.empty((P, 2), dtype=torch.int32, device="cuda")
        sub = hyps[:P]
        enc = [hthedl.encode_one(h) for h in sub]
        for i in range(min(8, P)):
            hthedl.hth_eval_one(eng.handle, enc[i][0], enc[i][1], eng.ws, eng.ws_bytes, None, pc[i], stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(P):
            hthedl.hth_eval_one(eng.handle, enc[i][0], enc[i][1], eng.ws, eng.ws_bytes, None, pc[i], stream)
        torch.cuda.synchronize()
        pdt = time.perf_counter() - t0
        pgot = pc.cpu().numpy().view(np.uint32)
        plain = {"value": round(P / pdt, 1), "unit": "hypotheses/s", "hyps": P,
                 "equal_to_batched": bool((pgot == got[:P]).all())}
        log(f"[bench] plain: {P / pdt:,.0f} hyp/s")

    dplans = None
    if args.device_plans:
        # the batch's node arrays already in device memory; a step generates
        # the plan there (count pass + summary readback, emit pass) and runs it
        d_nodes, d_offs, d_ch = eng.upload_batch(encoded=(nodes, offs, ch))
        n_nodes = int(nodes.shape[0])
        dc = torch.empty((H, 2), dtype=torch.int32, device="cuda")

        eng.ensure_plan_scratch(n_nodes)
        dchunk = args.device_chunk or H

        def dstep():
            for a in range(0, H, dchunk):
                b = min(H, a + dchunk)
                plan, nb = hthedl.hth_dplan_create(eng.handle, d_nodes, n_nodes, d_offs[a:], b - a, d_ch,
                                                   int(d_ch.shape[0]), eng.dp_scratch, eng.dp_scratch_bytes, stream)
                eng.ensure_workspace(nb)
                hthedl.hth_dplan_launch(plan, eng.ws, eng.ws_bytes, dc[a:b], stream)
                hthedl.hth_dplan_destroy(plan)

        dstep()
        torch.cuda.synchronize()
        hthedl.hth_profile_begin(eng.handle)
        t0 = time.perf_counter()
        for _ in range(args.device_plans):
            dstep()
        torch.cuda.synchronize()
        ddt = time.perf_counter() - t0
        dent = hthedl.hth_profile_end(eng.handle)
        dgot = dc.cpu().numpy().view(np.uint32)
        dplans = {"value": round(H * args.device_plans / ddt, 1), "unit": "hypotheses/s", "hyps_per_plan": dchunk,
                  "ms_per_step": round(ddt / args.device_plans * 1e3, 3),
                  "equal_to_batched": bool((dgot == got).all()),
                  "kernels_ms_per_step": {KIND_NAMES.get(k, str(k)): round(e["ms"] / args.device_plans, 3)
                                          for k, e in enumerate(dent) if e["launches"]}}
        log(f"[bench] device plans: {dplans}")

    cpu = None
    parity = None
    if args.cpu_sample:
        want, cdt = cpu_baseline(kb, hyps, args.cpu_sample, args.cpu_budget)
        n = want.shape[0]
        parity = {"checked": n, "equal": int((got[:n] == want).all(axis=1).sum())}
        cpu = {"value": round(n / cdt, 3), "unit": "hypotheses/s", "cores": 1, "kind": "oracle",
               "sample": f"first {n} of the {H} {args.config} hypotheses, numpy set-based oracle, "
                         f"one thread, KB in RAM, {cdt:.1f}s"}
        log(f"[bench] oracle: {n / cdt:.2f} hyp/s; parity {parity}")

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "hypotheses/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": describe(args.config, cfg, kb), "n_hyps": H,
                   "n_individuals": cfg.n_individuals, "n_assertions": kb.n_edges,
                   "mode": "batched",
                   "schedule": schedule or hthedl.hth_kb_get_tuning(eng.handle)},
        "roofline": roofline, "cpu_baseline": cpu, "plain": plain, "device_plans": dplans,
        "parity_sample": parity,
        "kernels": kernels,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
