"""Refinement trace (the c4 workload): rounds of one-step refinements of the
previous round's best hypotheses by exact F1, every candidate evaluated
exactly on the GPU.

The subtrees of the round's parents stay on the device as instance sets in
the set table (HTH_SET leaves), so a candidate re-evaluates only the path its
refinement changed: an added conjunct reads the parent's set, a specialised
filler re-runs the role restrictions above it and reads every unchanged
sibling from the table.  The table has two halves; the sets of the next
round's parents are written into the half the current round does not read.

    python -m paper_2412_00802_amd.trace [--small] [--rounds R] [--no-cache]

Prints one JSON line with per-round device and end-to-end times.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import sys
import time
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import hthedl, search, synth

ROLE_OPS = ("exists", "forall", "atleast", "atmost", "exactly")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def round0(cfg, kb, count: int) -> List[tuple]:
    """Refinements of top: every atom, every exists r.top (both directions),
    every decile threshold, topped up with random depth-2 hypotheses."""
    out = [("atom", a) for a in range(kb.n_concepts)]
    out += [("exists", r, inv, ("top",)) for r in range(kb.n_roles) for inv in (0, 1)]
    dec = np.asarray(kb.deciles, dtype=np.float32)
    out += [(op, p, float(dec[p, k])) for p in range(kb.n_data) for k in range(9) for op in ("dge", "dle")]
    seen = set(out)
    if len(out) < count:
        for h in synth.make_hypotheses(cfg, kb, count=2 * count, depth=2, stream=5):
            if h not in seen:
                seen.add(h)
                out.append(h)
                if len(out) >= count:
                    break
    return out[:count]


def subtrees(h, out: Dict[tuple, None]) -> None:
    """Distinct compound and data subtrees of h, parents before children."""
    if h[0] in ("atom", "top", "bot", "set"):
        return
    out.setdefault(h, None)
    if h[0] == "not":
        subtrees(h[1], out)
    elif h[0] in ("and", "or"):
        for c in h[1:]:
            subtrees(c, out)
    elif h[0] in ROLE_OPS:
        subtrees(h[-1], out)


class SetCache:
    """Two halves of `cap` rows each; slot maps a subtree to its row."""

    def __init__(self, eng, cap: int):
        torch = eng.torch
        self.eng, self.cap = eng, cap
        self.table = torch.zeros((2 * cap, eng.S), dtype=torch.int64, device=eng.device)
        hthedl.hth_kb_set_sets(eng.handle, self.table, 2 * cap)
        self.half = 0
        self.slot: Dict[tuple, int] = {}

    def close(self) -> None:
        """Unregister the table (the library must not read it once it is freed)."""
        if self.table is not None and self.eng.handle is not None:
            hthedl.hth_kb_set_sets(self.eng.handle, None, 0)
        self.table = None
        self.slot = {}

    def substitute(self, h, parent=None):
        """h with every cached subtree replaced by its set leaf.  When h adds
        conjuncts to an and-parent, the parent's conjuncts become one leaf."""
        if parent is not None and parent in self.slot and h[0] == "and" and parent[0] == "and" \
                and len(h) > len(parent) and h[:len(parent)] == parent:
            return ("and", ("set", self.slot[parent])) + tuple(self._sub(c) for c in h[len(parent):])
        return self._sub(h)

    def _sub(self, h):
        s = self.slot.get(h)
        if s is not None:
            return ("set", s)
        op = h[0]
        if op == "not":
            return ("not", self._sub(h[1]))
        if op in ("and", "or"):
            return (op,) + tuple(self._sub(c) for c in h[1:])
        if op in ROLE_OPS:
            return h[:-1] + (self._sub(h[-1]),)
        return h

    def refill(self, parents: Sequence[tuple], chunk: int, every_parent: bool = False) -> float:
        """Write the sets of the parents' subtrees (parents first, up to cap)
        into the other half, each computed from the current half; returns the
        device time in ms.  every_parent: atomic parents get rows too."""
        torch = self.eng.torch
        want: Dict[tuple, None] = {}
        for p in parents:
            if every_parent or p[0] not in ("atom", "top", "bot"):
                want.setdefault(p, None)
        for p in parents:
            subtrees(p, want)
        keys = list(want)[: self.cap]
        base = (1 - self.half) * self.cap
        exprs = [self._sub(k) for k in keys]
        cnt = torch.empty((max(1, len(keys)), 2), dtype=torch.int32, device=self.eng.device)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for a in range(0, len(keys), chunk):
            b = min(len(keys), a + chunk)
            nodes, offs, ch = hthedl.encode_batch(exprs[a:b])
            self.eng.ensure_workspace(hthedl.hth_batch_workspace_bytes(self.eng.handle, nodes, offs, ch))
            hthedl.hth_eval_batch_sets(self.eng.handle, nodes, offs, ch, self.eng.ws, self.eng.ws_bytes,
                                       self.table[base + a:base + b], cnt[a:b])
        e1.record()
        torch.cuda.synchronize()
        self.half = 1 - self.half
        self.slot = {k: base + i for i, k in enumerate(keys)}
        return e0.elapsed_time(e1)


def run_trace(cfg, kb, eng, rounds: int, per_round: int, beam: int, chunk: int, cache: Optional[SetCache],
              rng):
    """Yields one record per round (timings, sizes, best F1) with the round's
    candidates (full form) and their exact counts."""
    torch = eng.torch
    ref = search.Refiner(kb, rng)
    t_ref = time.perf_counter()
    cands = round0(cfg, kb, per_round)
    parent_of = [None] * len(cands)
    refine_s = time.perf_counter() - t_ref
    for r in range(rounds):
        t0 = time.perf_counter()
        exprs = cands if cache is None else [cache.substitute(c, p) for c, p in zip(cands, parent_of)]
        n_in = sum(synth.hyp_size(c) for c in cands)
        n_ex = sum(synth.hyp_size(c) for c in exprs)
        enc = hthedl.encode_batch(exprs)
        out = torch.empty((len(cands), 2), dtype=torch.int32, device=eng.device)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        eng.eval_batch(None, counts=out, chunk=chunk, encoded=enc)
        e1.record()
        counts = out.cpu().numpy().view(np.uint32).copy()
        dev_ms = e0.elapsed_time(e1)
        top = search.top_indices(counts, eng.n_pos, beam)
        parents = [cands[i] for i in top]
        fill_ms = cache.refill(parents, chunk) if cache is not None else 0.0
        t_eval = time.perf_counter() - t0
        best = counts[top[0]]
        # end to end: the host refinement that built this round's candidates,
        # then substitution, encoding, evaluation, selection and the set fill
        rec = {"round": r, "candidates": len(cands), "device_ms": round(dev_ms, 3),
               "set_fill_ms": round(fill_ms, 3), "refine_s": round(refine_s, 3),
               "end_to_end_s": round(refine_s + t_eval, 3),
               "nodes": n_in, "nodes_after_sets": n_ex, "best_f1": round(float(search.f1_float(best[None], eng.n_pos)[0]), 5),
               "best": [int(best[0]), int(best[1])]}
        yield rec, cands, counts
        # next round: one-step refinements of the parents
        t_ref = time.perf_counter()
        per_parent = max(1, per_round // max(1, len(parents)))
        nxt, pof, seen = [], [], set()
        for p in parents:
            for c in ref.refine(p, per_parent):
                if c not in seen:
                    seen.add(c)
                    nxt.append(c)
                    pof.append(p)
        tries = 0
        while len(nxt) < per_round and tries < 16 * per_round:
            tries += 1
            p = parents[int(rng.integers(0, len(parents)))]
            base = p[1:] if p[0] == "and" else (p,)
            c = ("and",) + tuple(base) + (ref.conjunct(),)
            if c not in seen:
                seen.add(c)
                nxt.append(c)
                pof.append(p)
        cands, parent_of = nxt[:per_round], pof[:per_round]
        refine_s = time.perf_counter() - t_ref


def run_trace_device(cfg, kb, eng, rounds: int, per_round: int, beam: int, chunk: int, cache: SetCache, rng,
                     seed: int, decode: bool = False):
    """The trace with each round's added conjuncts made on the device: the
    host writes only the local specialisations of the parents (tree positions
    changed); hth_draw_conjuncts and hth_conjoin fill the rest of the round
    from the parents' set-table rows.  Both halves are planned on the device
    (hth_dplan_*).  Only the selected candidates' specs come back to the host
    (to name the next parents).  Yields one record per round, as run_trace does (the round's
    candidates in full form only with decode, which reads every spec back)."""
    torch = eng.torch
    ref = search.Refiner(kb, rng)
    t_ref = time.perf_counter()
    host = round0(cfg, kb, per_round)
    host_parent = [None] * len(host)
    parents: List[tuple] = []
    refine_s = time.perf_counter() - t_ref
    for r in range(rounds):
        t0 = time.perf_counter()
        exprs = [cache.substitute(c, p) for c, p in zip(host, host_parent)]
        n_dev = per_round - len(host) if parents else 0
        out = torch.empty((len(host) + n_dev, 2), dtype=torch.int32, device=eng.device)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        # two plans, both generated on the device: the host's candidates
        # (uploaded) and the device's (written there)
        if host:
            eng.eval_batch_device(encoded=hthedl.encode_batch(exprs), counts=out[:len(host)])
        if n_dev:
            per = -(-n_dev // len(parents))
            rows = np.array([cache.slot[p] for p in parents], dtype=np.uint32)
            d_specs, batch = eng.conjunct_candidates(rows, per, seed + r, kb.deciles, count=n_dev)
            eng.eval_batch_device(device_batch=batch, counts=out[len(host):])
        e1.record()
        counts = out.cpu().numpy().view(np.uint32).copy()
        dev_ms = e0.elapsed_time(e1)
        top = search.top_indices(counts, eng.n_pos, beam)
        specs = d_specs.cpu().numpy().view(hthedl.CONJ_DTYPE) if n_dev else None
        by_row = {cache.slot[p]: p for p in parents}

        def full(i):
            if i < len(host):
                return host[i]
            sp = specs[i - len(host)]
            p = by_row[int(sp["parent"])]
            return ("and",) + (p[1:] if p[0] == "and" else (p,)) + (hthedl.conjunct_tuple(sp),)

        cands = [full(i) for i in range(len(host) + n_dev)] if decode else None
        nxt, seen = [], set()
        for i in top:
            c = full(i)
            if c not in seen:                   # device draws may repeat
                seen.add(c)
                nxt.append(c)
        parents = nxt
        fill_ms = cache.refill(parents, chunk, every_parent=True)
        t_eval = time.perf_counter() - t0
        best = counts[top[0]]
        rec = {"round": r, "candidates": len(host) + n_dev, "on_device": n_dev, "device_ms": round(dev_ms, 3),
               "set_fill_ms": round(fill_ms, 3), "refine_s": round(refine_s, 3),
               "end_to_end_s": round(refine_s + t_eval, 3),
               "best_f1": round(float(search.f1_float(best[None], eng.n_pos)[0]), 5),
               "best": [int(best[0]), int(best[1])]}
        yield rec, cands, counts
        # the host's share of the next round: local specialisations only
        t_ref = time.perf_counter()
        per_parent = max(1, per_round // max(1, len(parents)))
        host, host_parent, seen = [], [], set()
        for p in parents:
            for c in ref.refine(p, per_parent, conjuncts=False):
                if c not in seen:
                    seen.add(c)
                    host.append(c)
                    host_parent.append(p)
        host, host_parent = host[:per_round], host_parent[:per_round]
        refine_s = time.perf_counter() - t_ref


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--small", action="store_true", help="a reduced KB with the same pipeline")
    ap.add_argument("--rounds", type=int, default=16)
    ap.add_argument("--per-round", type=int, default=16384)
    ap.add_argument("--beam", type=int, default=256)
    ap.add_argument("--chunk", type=int, default=16384, help="candidates compiled together (a round by default)")
    ap.add_argument("--cache-rows", type=int, default=4096)
    ap.add_argument("--no-cache", action="store_true")
    ap.add_argument("--compare", action="store_true", help="also run the trace without the set table and "
                    "check that every round's counts are identical")
    ap.add_argument("--device-candidates", action="store_true",
                    help="make each round's added conjuncts on the device (hth_draw_conjuncts, device plans)")
    args = ap.parse_args()
    import torch

    cfg = synth.CONFIGS["c4"]
    if args.small:
        cfg = dataclasses.replace(cfg, name="c4-small", n_individuals=400_000, total_edges=6_000_000,
                                  n_data=16, n_pos=20_000, n_neg=20_000, degree_cap=4096)
    t = time.perf_counter()
    kb = synth.make_kb(cfg, log=lambda m: log(f"[trace] generated {m} ({time.perf_counter() - t:.1f}s)"))
    log(f"[trace] KB {cfg.name}: N={kb.n:,}, {kb.n_edges:,} assertions, {kb.n_data} properties "
        f"({time.perf_counter() - t:.1f}s)")
    t = time.perf_counter()
    eng = hthedl.Engine(kb, max_nodes=64, max_hyps=1)
    log(f"[trace] uploaded + kb_create in {time.perf_counter() - t:.1f}s")
    runs = [("cached", not args.no_cache)] + ([("plain", False)] if args.compare else [])
    if args.device_candidates:
        runs = [("device candidates", True)]
    result = {"workload": f"{cfg.name}: {kb.n:,} individuals, {kb.n_concepts} concepts, {kb.n_roles} roles / "
                          f"{kb.n_edges:,} assertions (Zipf s={cfg.zipf_s}, cap {cfg.degree_cap}), {kb.n_data} "
                          f"float32 properties; {args.rounds} rounds x {args.per_round} candidates, beam "
                          f"{args.beam}", "runs": {}}
    ref_counts = []
    for name, use_cache in runs:
        cache = SetCache(eng, args.cache_rows) if use_cache else None
        rng = np.random.default_rng(synth.BASE_SEED + 40)
        recs = []
        gen = (run_trace_device(cfg, kb, eng, args.rounds, args.per_round, args.beam, args.chunk, cache, rng,
                                synth.BASE_SEED + 41) if args.device_candidates else
               run_trace(cfg, kb, eng, args.rounds, args.per_round, args.beam, args.chunk, cache, rng))
        for i, (rec, cands, counts) in enumerate(gen):
            log(f"[trace] {name} round {rec['round']}: {rec['candidates']} candidates, device "
                f"{rec['device_ms']:.1f} ms (+{rec['set_fill_ms']:.1f} ms set fill), end-to-end "
                f"{rec['end_to_end_s']:.2f}s, nodes {rec.get('nodes')} -> {rec.get('nodes_after_sets')}, "
                f"on the device {rec.get('on_device', 0)}, best F1 {rec['best_f1']}")
            recs.append(rec)
            if name == "cached":
                ref_counts.append(counts)
            elif name == "plain":
                assert np.array_equal(ref_counts[i], counts), f"round {i}: set-table counts differ"
        if cache is not None:
            cache.close()
        dev = sum(r["device_ms"] + r["set_fill_ms"] for r in recs) / 1e3
        e2e = sum(r["end_to_end_s"] for r in recs)
        n = sum(r["candidates"] for r in recs)
        result["runs"][name] = {"set_table": use_cache, "device_hyp_per_s": round(n / dev, 1),
                                "end_to_end_hyp_per_s": round(n / e2e, 1), "rounds": recs}
    if args.compare:
        result["compare"] = "identical counts in every round"
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
