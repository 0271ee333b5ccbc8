"""Per-operation microbenchmarks in the shapes of the paper's operation tables.

    python -m paper_2412_00802_amd.microbench [--quick]

M1 (Table 2's shape): a conjunction of five atomic concepts at N from 10k to
32M individuals.  M2 (Table 4 and the cardinality table's shapes): one role
with either a single subject of degree E ("single subject") or E subjects of
degree 1 ("unique subject"), E up to 10M, evaluated as an existential and as
an at-least-2 restriction.  M3 (Table 8's shape): one numeric concrete role
with the same two layouts and every value 1.0, under MIN at 0.5 (every
subject decided by its first value) and at 2.0 (every value read).  M4
(Table 8's string rows): one string concrete role in the same two layouts,
every value the same 8-byte word of a 1,000-word dictionary, under EQUAL and
CONTAIN with a query that matches and one that does not.  Each operation is compiled once (hth_plan_create),
uploaded once and launched repeatedly; the time is the device time per launch
(HIP events on the launch stream).  Prints one JSON line per case.
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

from . import hthedl, synth


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_kb(n: int, n_concepts: int, rows: np.ndarray, targets: np.ndarray, seed: int,
            miss_targets: bool = False) -> synth.KB:
    """A KB with random concept rows (density 1/2) and one role whose subject
    rows are given (sorted subjects, one target list per row, concatenated).
    With miss_targets, one more concept holds every individual that is not a
    target, so a restriction on it has to read every assertion."""
    rng = np.random.default_rng(seed)
    w = (n + 63) // 64
    bits = rng.integers(0, 1 << 63, size=(n_concepts, w), dtype=np.int64).view(np.uint64)
    if miss_targets:
        hit = synth.ids_to_bits(np.unique(targets), n)
        bits = np.concatenate([bits, ~hit[None, :]])
        n_concepts += 1
    tail = np.uint64((1 << (n & 63)) - 1) if n & 63 else np.uint64(0xFFFFFFFFFFFFFFFF)
    bits[:, -1] &= tail
    deg = np.zeros(n, dtype=np.int64)
    np.add.at(deg, rows, 1)
    offs = np.zeros((1, n + 1), dtype=np.int64)
    np.cumsum(deg, out=offs[0, 1:])
    ex = rng.choice(n, size=min(n, 2000), replace=False)
    pos = synth.ids_to_bits(ex[: len(ex) // 2], n)
    neg = synth.ids_to_bits(ex[len(ex) // 2:], n)
    return synth.KB(n, bits, offs, targets.astype(np.int32), np.zeros((0, n), np.float32), pos, neg,
                    np.full(n_concepts, -1, np.int32), np.zeros(n_concepts, np.int32), np.zeros((0, 9), np.float32))


def time_op(eng, h, reps: int) -> float:
    """Device ms per launch of the compiled operation."""
    import torch
    nodes, offs, ch = hthedl.encode_batch([h])
    plan, nb = hthedl.hth_plan_create(eng.handle, nodes, offs, ch)
    try:
        ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=eng.device)
        counts = torch.empty((1, 2), dtype=torch.int32, device=eng.device)
        hthedl.hth_plan_upload(plan, ws, nb)
        for _ in range(3):
            hthedl.hth_plan_launch(plan, ws, nb, counts)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            hthedl.hth_plan_launch(plan, ws, nb, counts)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps
    finally:
        hthedl.hth_plan_destroy(plan)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true", help="smaller sizes")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--markdown", default=None, help="also write the results as a markdown table here")
    args = ap.parse_args()
    results = []

    def emit(rec):
        results.append(rec)
        print(json.dumps(rec), flush=True)

    sizes = [10_000, 100_000, 1_000_000, 10_000_000, 32_000_000]
    edges = [10_000, 100_000, 1_000_000, 10_000_000]
    if args.quick:
        sizes, edges = sizes[:3], edges[:2]
    rng = np.random.default_rng(synth.BASE_SEED + 70)
    # M1: A1 and ... and A5
    for n in sizes:
        kb = make_kb(n, 5, np.zeros(0, np.int64), np.zeros(0, np.int32), seed=1)
        eng = hthedl.Engine(kb, max_nodes=16, max_hyps=1)
        ms = time_op(eng, ("and",) + tuple(("atom", i) for i in range(5)), args.reps)
        w8 = 8 * ((n + 63) // 64)
        emit({"case": "M1 five-concept conjunction", "individuals": n, "us_per_op": round(ms * 1e3, 2),
              "GBps": round(7 * w8 / (ms * 1e-3) / 1e9, 1)})
        eng.close()
    # M2: single subject and unique subject
    for e in edges:
        n = max(1_000_000, 2 * e)
        for shape in ("single subject", "unique subject"):
            if shape == "single subject":
                rows = np.zeros(e, dtype=np.int64)
                tg = np.sort(rng.choice(n, size=e, replace=False))
            else:
                rows = np.sort(rng.choice(n, size=e, replace=False))
                tg = rng.integers(0, n, size=e)
            kb = make_kb(n, 1, rows, tg, seed=2, miss_targets=True)
            eng = hthedl.Engine(kb, max_nodes=16, max_hyps=1)
            w8 = 8 * ((n + 63) // 64)
            for op, h in (("exists, decided early", ("exists", 0, 0, ("atom", 0))),
                          ("exists, every assertion read", ("exists", 0, 0, ("atom", 1))),
                          ("at least 2, every assertion read", ("atleast", 2, 0, 0, ("atom", 1)))):
                ms = time_op(eng, h, args.reps)
                byts = 4.0 * e + 4.0 * (n + 1) + 2 * w8
                emit({"case": f"M2 {shape}, {op}", "assertions": e, "individuals": n,
                      "us_per_op": round(ms * 1e3, 2), "GBps": round(byts / (ms * 1e-3) / 1e9, 1)})
            eng.close()
    # M3: numeric concrete role, single subject and unique subject, values 1.0
    for e in edges:
        n = max(1_000_000, 2 * e)
        for shape in ("single subject", "unique subject"):
            deg = np.zeros(n, dtype=np.int64)
            if shape == "single subject":
                deg[0] = e
            else:
                deg[np.sort(rng.choice(n, size=e, replace=False))] = 1
            offs = np.zeros((1, n + 1), dtype=np.int64)
            np.cumsum(deg, out=offs[0, 1:])
            kb = synth.with_numeric_roles(make_kb(n, 1, np.zeros(0, np.int64), np.zeros(0, np.int32), seed=3),
                                          offs, np.ones(e, dtype=np.float32))
            eng = hthedl.Engine(kb, max_nodes=16, max_hyps=1)
            w8 = 8 * ((n + 63) // 64)
            for op, h in (("MIN 0.5, decided by the first value", ("nge", 0, 0.5)),
                          ("MIN 2.0, every value read", ("nge", 0, 2.0))):
                ms = time_op(eng, h, args.reps)
                byts = 4.0 * e + 4.0 * (n + 1) + 2 * w8
                emit({"case": f"M3 numeric {shape}, {op}", "assertions": e, "individuals": n,
                      "us_per_op": round(ms * 1e3, 2), "GBps": round(byts / (ms * 1e-3) / 1e9, 1)})
            eng.close()
    # M4: string concrete role, single subject and unique subject, one repeated value
    words = [b"w%07d" % i for i in range(1000)]
    for e in edges:
        n = max(1_000_000, 2 * e)
        for shape in ("single subject", "unique subject"):
            deg = np.zeros(n, dtype=np.int64)
            if shape == "single subject":
                deg[0] = e
            else:
                deg[np.sort(rng.choice(n, size=e, replace=False))] = 1
            offs = np.zeros((1, n + 1), dtype=np.int64)
            np.cumsum(deg, out=offs[0, 1:])
            kb = synth.with_string_roles(make_kb(n, 1, np.zeros(0, np.int64), np.zeros(0, np.int32), seed=4),
                                         offs, np.full(e, 7, dtype=np.int32), words)
            eng = hthedl.Engine(kb, max_nodes=16, max_hyps=1)
            w8 = 8 * ((n + 63) // 64)
            for op, h in (("EQUAL, matching", ("sequal", 0, words[7])),
                          ("EQUAL, no match", ("sequal", 0, words[8])),
                          ("CONTAIN, matching", ("scontains", 0, b"0007")),
                          ("CONTAIN, no match", ("scontains", 0, b"0008"))):
                ms = time_op(eng, eng.intern(h), args.reps)
                byts = 4.0 * e + 4.0 * (n + 1) + 2 * w8
                emit({"case": f"M4 string {shape}, {op}", "assertions": e, "individuals": n,
                      "us_per_op": round(ms * 1e3, 2), "GBps": round(byts / (ms * 1e-3) / 1e9, 1)})
            eng.close()
    if args.markdown:
        cmd = "python -m paper_2412_00802_amd.microbench " + " ".join(sys.argv[1:])
        lines = ["# Per-operation microbenchmarks (M1: five-concept conjunction; M2: one role, M3: one "
                 "numeric and M4: one string concrete role, single subject / unique subject)", "", "Command:", "",
                 "    " + cmd, "",
                 "Device time per launch of a compiled one-hypothesis plan (all of its kernels: count "
                 "clearing, the operation, coverage), HIP events around back-to-back launches.  GB/s "
                 "counts algorithmic bytes: M1 the five rows read, the example rows and the output; M2 "
                 "the assertions' targets (4 B each), the row offsets (4 B per individual) and two bit "
                 "rows; M3 and M4 the values or string ids (4 B each), the 32-bit row offsets (4 B per "
                 "individual) and two bit rows.", "",
                 "| case | individuals | assertions | us per op | GB/s |", "|---|---|---|---|---|"]
        for r in results:
            lines.append(f"| {r['case']} | {r['individuals']:,} | {r.get('assertions', '')} | "
                         f"{r['us_per_op']} | {r['GBps']} |")
        open(args.markdown, "w").write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
