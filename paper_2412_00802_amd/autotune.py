"""Schedule autotuner for the batched executor.

The schedule (shared-pass width, XCD placement, T-row budget, load unroll,
sharing threshold) changes speed only, never results.  The autotuner times a
small grid of candidates derived from the knowledge base's shape on a sample
batch, checks that every candidate returns identical coverage, keeps the
fastest and caches it per (arch, N, roles, assertions, degree signature).
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import hthedl

CACHE = os.environ.get("HTHEDL_TUNING_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "hthedl_tuning.json"))


def signature(eng) -> str:
    import torch
    arch = torch.cuda.get_device_properties(eng.device).gcnArchName.split(":")[0]
    R = int(eng.desc.n_roles)
    deg = [hthedl.hth_kb_max_degree(eng.handle, r, d) for r in range(R) for d in (0, 1)]
    dsig = int(np.log2(1 + max(deg))) if deg else 0
    return f"{arch}/N{eng.n}/R{R}/E{int(eng.desc.n_edges)}/D{dsig}"


def candidates(n_individuals: int) -> List[Dict[str, int]]:
    """Each T width (8..64 bits) with: XCD-local passes and a budget of one
    group per XCD, 64 MiB and the 1 GiB default, both unrolls; chip-wide passes
    with one and four groups per launch; one run sharing passes from a single
    node up; the region kernel at one and four words per lane; and the push
    threshold of single existential restrictions at 0 (never) and 8%.  Widths
    whose T rows exceed 1 GiB per group are left out."""
    out = []
    for k, w in ((8, 1), (16, 2), (32, 4), (64, 8)):
        t_mb = max(1, -(-(n_individuals * w) // (1 << 20)))
        if t_mb > 1024:
            continue
        for budget in sorted({max(64, 8 * t_mb), 64, 1024}):
            for unroll in (8, 16):
                out.append(dict(group_min=2, group_k=k, xcd_local=1, t_budget_mb=max(budget, t_mb),
                                unroll=unroll))
        for budget in sorted({t_mb, 4 * t_mb}):
            out.append(dict(group_min=2, group_k=k, xcd_local=0, t_budget_mb=budget, unroll=16))
    widest = max((c["group_k"] for c in out), default=8)
    out.append(dict(group_min=1, group_k=widest, xcd_local=1, t_budget_mb=1024, unroll=16))
    # words per lane of the region kernel (the others keep the default, 2)
    out += [dict(group_min=2, group_k=widest, xcd_local=1, t_budget_mb=1024, unroll=16, region_reg=r) for r in (1, 4)]
    # the push/pull density switch of single existential restrictions (default 2%)
    out += [dict(group_min=2, group_k=widest, xcd_local=1, t_budget_mb=1024, unroll=16, push_pct=p) for p in (0, 8)]
    for c in out:
        c.setdefault("region_reg", 2)
        c.setdefault("push_pct", 2)
    return out


def autotune(eng, sample: Sequence[tuple], grid: Optional[List[Dict[str, int]]] = None, reps: int = 3,
             cache: Optional[str] = CACHE, log=None) -> Dict[str, int]:
    """Time each schedule on `sample` (batched evaluation), pick the fastest,
    apply it to eng and cache it.  Raises if two schedules disagree."""
    import torch
    grid = candidates(eng.n) if grid is None else grid
    nodes, offs, ch = hthedl.encode_batch(sample)
    eng.ensure_workspace(max(hthedl.hth_batch_workspace_bytes(eng.handle, nodes, offs, ch), 1))
    counts = torch.empty((len(sample), 2), dtype=torch.int32, device=eng.device)
    ref = None
    results = []
    for cand in grid:
        hthedl.hth_kb_set_tuning(eng.handle, **cand)
        eng.ensure_workspace(hthedl.hth_batch_workspace_bytes(eng.handle, nodes, offs, ch))
        hthedl.hth_eval_batch(eng.handle, nodes, offs, ch, eng.ws, eng.ws_bytes, counts)
        torch.cuda.synchronize()
        got = counts.cpu().numpy().copy()
        if ref is None:
            ref = got
        elif not np.array_equal(ref, got):
            raise RuntimeError(f"schedule {cand} changed the coverage counts")
        t0 = time.perf_counter()
        for _ in range(reps):
            hthedl.hth_eval_batch(eng.handle, nodes, offs, ch, eng.ws, eng.ws_bytes, counts)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        results.append((dt, cand))
        if log:
            log(f"[autotune] {cand} -> {dt * 1e3:.2f} ms")
    best = min(results, key=lambda r: r[0])[1]
    hthedl.hth_kb_set_tuning(eng.handle, **best)
    if cache:
        try:
            os.makedirs(os.path.dirname(cache), exist_ok=True)
            data = json.load(open(cache)) if os.path.exists(cache) else {}
            data[signature(eng)] = {"schedule": best,
                                    "timings_ms": [[round(d * 1e3, 3), c] for d, c in results]}
            json.dump(data, open(cache, "w"), indent=1)
        except OSError:
            pass
    return best


def apply_cached(eng, cache: str = CACHE) -> Optional[Dict[str, int]]:
    """Apply a cached schedule for this KB shape, if one exists."""
    try:
        data = json.load(open(cache))
    except (OSError, ValueError):
        return None
    rec = data.get(signature(eng))
    if not rec:
        return None
    hthedl.hth_kb_set_tuning(eng.handle, **rec["schedule"])
    return rec["schedule"]
