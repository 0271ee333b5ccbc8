"""Screened search (the c5 workload): train the screener on engine-evaluated
refinements, then rank a large candidate set with it and evaluate exactly only
the top fraction plus a uniform audit sample.  The exact engine supplies every
training label and judges the screener: recall of the exhaustive top-k.

    python -m paper_2412_00802_amd.screened [--small]

Prints one JSON line: screened vs exhaustive hypotheses/s, top-100 recall,
training time and loss, and the same recall for random selection and for the
parents' F1 at the same exact budget.
"""
from __future__ import annotations

import argparse
import json
import sys
import time
from typing import List

import numpy as np

from . import hthedl, search, synth
from .screener import D_IN, FeatureBatch, Screener, init_params


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def coverage_targets(counts: np.ndarray, n_pos: int, n_neg: int, base: np.ndarray = None) -> np.ndarray:
    """Training targets: covered fractions of the examples, or with base (the
    parents' coverage) the shares of the parent's coverage each child keeps
    (0 where the parent covers nothing)."""
    c = counts.astype(np.float64)
    if base is None:
        return np.stack([c[:, 0] / max(1, n_pos), c[:, 1] / max(1, n_neg)], 1).astype(np.float32)
    b = np.asarray(base, dtype=np.float64)
    return np.where(b > 0, c / np.maximum(b, 1), 0.0).astype(np.float32)


def removal_targets(counts: np.ndarray, base: np.ndarray) -> np.ndarray:
    """log(1 + positives and negatives a refinement removes from its parent)."""
    d = np.maximum(np.asarray(base, dtype=np.float64) - counts.astype(np.float64), 0.0)
    return np.log1p(d).astype(np.float32)


def gather_training_pairs(eng, kb, n_pairs, per_round, beam, rng, chunk, late_beam: int = 0):
    """Refinement rounds from top; every candidate is evaluated exactly.
    Returns the candidates, their counts, their parents' counts, the parents
    (distinct, in round order) and each candidate's parent index."""
    hyps: List[tuple] = []
    counts, pcounts, pidx = [], [], []
    parents: List[tuple] = []
    ev = lambda hs: eng.eval_batch(hs, chunk=chunk)  # noqa: E731
    rounds = (n_pairs + per_round - 1) // per_round
    for r, cands, cnt, plist, pi, pc in search.refinement_rounds(
            kb, ev, eng.n_pos, rounds, per_round, beam, rng, start_counts=[eng.n_pos, eng.n_neg],
            with_parents=True, late_beam=late_beam):
        hyps.extend(cands)
        counts.append(cnt)
        pcounts.append(pc)
        pidx.append(np.asarray(pi) + len(parents))
        parents.extend(plist)
        log(f"[screen] training round {r}: {len(hyps)} pairs, best F1 "
            f"{search.f1_float(cnt, eng.n_pos).max():.4f}")
    return (hyps[:n_pairs], np.concatenate(counts)[:n_pairs], np.concatenate(pcounts)[:n_pairs], parents,
            np.concatenate(pidx)[:n_pairs])


def train(scr: Screener, fb: FeatureBatch, y_dev, n: int, epochs: int, batch: int, rng,
          parents: FeatureBatch = None, parent_index=None, context: int = 0) -> List[float]:
    """Epochs of minibatch AdamW over rows [0, n); with parents, the features
    are relative to each row's parent (hth_densify_delta; with context, the
    parent's own features too)."""
    torch = scr.t
    losses = []
    nb = n // batch
    for ep in range(epochs):
        scr.loss.zero_()
        for bi in rng.permutation(nb):
            r0 = int(bi) * batch
            fb.densify(r0, batch, scr.x, parents, parent_index, context)
            scr.train_step(batch, y_dev[r0:r0 + batch])
        losses.append(scr.loss.item() / (2 * nb * batch))
        log(f"[screen] epoch {ep}: loss {losses[-1]:.5f}")
    torch.cuda.synchronize()
    return losses


def score(scr: Screener, fb: FeatureBatch, n: int, n_pos: int, n_neg: int, out, base=None,
          parents: FeatureBatch = None, parent_index=None, kind: int = 0, context: int = 0) -> None:
    """Predicted F1 of candidates [0, n); base (device uint32 [n][2]): the
    parents' coverage (kept shares, kind 0, or removed counts, kind 1);
    parents: features relative to the parents."""
    B = scr.batch
    for r0 in range(0, n, B):
        m = min(B, n - r0)
        fb.densify(r0, m, scr.x, parents, parent_index, context)
        z = scr.logits(m)
        hthedl.hth_head_score(z, m, float(n_pos), float(n_neg), out[r0:r0 + m],
                              base=None if base is None else base[r0:r0 + m], kind=kind)


def run(kb, eng, pairs: int = 200_000, candidates_beam: int = 4096, refinements: int = 256, epochs: int = 10,
        top: float = 0.02, audit: float = 0.005, k: int = 100, lr: float = 5e-4, per_round: int = 16384,
        chunk: int = 65536, modes=("logdelta", "delta", "relative", "absolute"), sweep=(0.02, 0.05, 0.1),
        name: str = "c3", draws: int = 1, late_beam: int = 0, weight_decay: float = 1e-4) -> dict:
    """The screened search on one resident KB: training pairs from the exact
    engine, screeners trained on the GPU, candidates, the exhaustive exact
    evaluation (the judge) and each screener's pipeline.  With draws > 1 the
    candidates are drawn again from the same parents that many times (the
    screeners are not retrained) and each draw's recall is reported.  Returns
    the record."""
    import torch
    rng = np.random.default_rng(synth.BASE_SEED + 50)

    # 1. training pairs from the engine
    t = time.perf_counter()
    hyps, counts, pcounts, tparents, tpidx = gather_training_pairs(eng, kb, pairs, per_round, 256, rng, chunk,
                                                                   late_beam)
    t_pairs = time.perf_counter() - t
    order = rng.permutation(len(hyps))
    hyps = [hyps[i] for i in order]
    counts, pcounts, tpidx = counts[order], pcounts[order], tpidx[order]
    n_val = len(hyps) // 10
    n_tr = len(hyps) - n_val
    fb = FeatureBatch(*hthedl.encode_batch(hyps))
    tpfb = FeatureBatch(*hthedl.encode_batch(tparents))
    tpi = torch.from_numpy(tpidx.astype(np.int32)).cuda()

    # 2. training: "logdelta" predicts log(1 + removed positives / negatives)
    # from features relative to the parent, with the squared error ("logctx":
    # the same with the parent's own features beside them); "delta"
    # the shares of the parent's coverage a refinement keeps, from the same
    # features; "relative" those shares from the candidate's own features;
    # "absolute" the covered fractions of the examples
    models = {}
    for mode in modes:
        if mode in LOG_MODES:
            y = torch.from_numpy(removal_targets(counts, pcounts)).cuda()
        else:
            y = torch.from_numpy(coverage_targets(counts, eng.n_pos, eng.n_neg,
                                                  None if mode == "absolute" else pcounts)).cuda()
        scr = Screener(init_params(seed=11), batch=8192, lr=lr, weight_decay=weight_decay,
                       loss="mse" if mode in LOG_MODES else "bce")
        t = time.perf_counter()
        losses = train(scr, fb, y, n_tr, epochs, 1024, rng,
                       *((tpfb, tpi) if mode in REL_MODES else (None, None)), context=int(mode == "logctx"))
        models[mode] = (scr, losses, time.perf_counter() - t)
    best = search.top_indices(counts, eng.n_pos, candidates_beam)
    parents = [hyps[i] for i in best]
    out = None
    recalls = {m: [] for m in models}
    for d in range(draws):
        rec = _draw(kb, eng, models, parents, counts[best], rng, refinements, top, audit, k, chunk,
                    sweep if d == 0 else (), log_tag=f"draw {d}")
        for m in models:
            recalls[m].append(rec["screener"][m][f"recall_at_{k}"])
        if out is None:
            out = rec
    out.update({"workload": f"screened search on the {name} KB ({kb.n:,} individuals)",
                "training_pairs": len(hyps), "pairs_seconds": round(t_pairs, 2), "draws": draws,
                f"recall_at_{k}_per_draw": recalls,
                f"recall_at_{k}_mean": {m: round(float(np.mean(v)), 4) for m, v in recalls.items()},
                f"recall_at_{k}_min": {m: round(float(np.min(v)), 4) for m, v in recalls.items()}})
    return out


LOG_MODES = ("logdelta", "logctx")            # targets: log(1 + removed counts)
REL_MODES = ("delta", "logdelta", "logctx")   # features relative to the parent


def _draw(kb, eng, models, parents, pcounts, rng, refinements, top, audit, k, chunk, sweep, log_tag=""):
    """One set of candidates (every parent refined), the exhaustive exact
    evaluation of all of them, and each screener's pipeline on them."""
    import torch

    # 3. candidates: the best `candidates_beam` evaluated so far, each refined
    ref = search.Refiner(kb, rng)
    cands, parent_of = [], []
    seen = set()
    t = time.perf_counter()
    for pi, p in enumerate(parents):
        for c in ref.refine(p, refinements):
            if c not in seen:
                seen.add(c)
                cands.append(c)
                parent_of.append(pi)
    t_cands = time.perf_counter() - t
    parent_of = np.asarray(parent_of)
    n = len(cands)
    log(f"[screen] {n:,} candidates from {len(parents)} parents ({t_cands:.1f}s)")
    cenc = hthedl.encode_batch(cands, child_offsets=True)
    cfb = FeatureBatch(*cenc[:3])
    cbase = torch.from_numpy(pcounts[parent_of].astype(np.uint32).view(np.int32)).cuda()
    cpfb = FeatureBatch(*hthedl.encode_batch(parents))
    cpi = torch.from_numpy(parent_of.astype(np.int32)).cuda()
    n_sel = int(round(top * n))
    n_aud = int(round(audit * n))
    aud = rng.choice(n, size=n_aud, replace=False)           # drawn on the host: an input
    scores = torch.empty(n, dtype=torch.float32, device="cuda")
    sel = torch.empty(n_sel, dtype=torch.int32, device="cuda")
    work = torch.empty(65538, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()

    # 4. exhaustive exact evaluation of every candidate (the judge)
    t0 = time.perf_counter()
    allc = torch.empty((n, 2), dtype=torch.int32, device="cuda")
    eng.eval_batch(None, counts=allc, chunk=chunk, encoded=cenc[:3])
    all_np = allc.cpu().numpy().view(np.uint32)
    exact_top = search.top_indices(all_np, eng.n_pos, k)
    torch.cuda.synchronize()
    t_exh = time.perf_counter() - t0
    f_np = search.f1_float(all_np, eng.n_pos)

    def screened(scr, mode, m_sel, sel_t, stages=None):
        """features + scores + top-k + exact evaluation of the selection; with
        `stages` (a dict) each stage is synchronised and timed on its own."""
        mark = time.perf_counter()

        def stage(key):
            nonlocal mark
            if stages is not None:
                torch.cuda.synchronize()
                now = time.perf_counter()
                stages[key] = round(now - mark, 5)
                mark = now

        rel = mode in REL_MODES
        cfb.recompute()
        if rel:
            cpfb.recompute()
        stage("features_s")
        score(scr, cfb, n, eng.n_pos, eng.n_neg, scores, base=None if mode == "absolute" else cbase,
              parents=cpfb if rel else None, parent_index=cpi if rel else None,
              kind=1 if mode in LOG_MODES else 0, context=int(mode == "logctx"))
        stage("mlp_s")
        hthedl.hth_topk(scores, n, m_sel, sel_t, work)
        chosen = np.union1d(sel_t.cpu().numpy().astype(np.int64), aud)
        stage("topk_s")
        sub = hthedl.gather_encoded(cenc, chosen)
        sc = torch.empty((chosen.size, 2), dtype=torch.int32, device="cuda")
        eng.eval_batch(None, counts=sc, chunk=chunk, encoded=sub)
        sc_np = sc.cpu().numpy().view(np.uint32)
        got = chosen[search.top_indices(sc_np, eng.n_pos, k)]
        stage("exact_s")
        return chosen, sc_np, got

    # 5. screened: features + scores + top-k + exact evaluation of the selection
    res = {}
    for mode, (scr, losses, t_train) in models.items():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        chosen, sc_np, screened_top = screened(scr, mode, n_sel, sel)
        torch.cuda.synchronize()
        t_screen = time.perf_counter() - t0
        assert np.array_equal(all_np[chosen], sc_np), "screened and exhaustive exact counts differ"
        stages = {}
        screened(scr, mode, n_sel, sel, stages)          # the same pipeline again, stage by stage
        s_np = scores.cpu().numpy()
        rank_corr = float(np.corrcoef(np.argsort(np.argsort(s_np)), np.argsort(np.argsort(f_np)))[0, 1])
        res[mode] = {"screened_hyp_per_s": round(n / t_screen, 1), "speedup": round(t_exh / t_screen, 3),
                     f"recall_at_{k}": search.recall_at(screened_top, exact_top),
                     "score_rank_correlation": round(rank_corr, 4), "exact_budget": int(chosen.size),
                     "screened_seconds": round(t_screen, 4), "stages_synchronised": stages,
                     "train_seconds": round(t_train, 2),
                     "train_loss_first_last": [round(losses[0], 5), round(losses[-1], 5)]}
        log(f"[screen] {log_tag} {mode}: recall@{k} {res[mode][f'recall_at_{k}']:.2f}, "
            f"{res[mode]['speedup']}x the exhaustive rate; stages {stages}")
    # recall and speed of the first log-removal screener at other exact budgets
    budget_sweep = []
    swept = next((m for m in models if m in LOG_MODES), None)
    if swept:
        scr_d = models[swept][0]
        for frac in sweep:
            m_sel = int(round(frac * n))
            sel_m = torch.empty(m_sel, dtype=torch.int32, device="cuda")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            chosen, _, got = screened(scr_d, swept, m_sel, sel_m)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            budget_sweep.append({"top_fraction": frac, "exact_budget": int(chosen.size),
                                 f"recall_at_{k}": search.recall_at(got, exact_top),
                                 "speedup": round(t_exh / dt, 3)})
            log(f"[screen] {swept} at top {frac}: recall {budget_sweep[-1][f'recall_at_{k}']:.2f}, "
                f"{budget_sweep[-1]['speedup']}x")
    # ties at the k-th exact F1 make part of the exact top-k a matter of the index tie-break
    kth = np.sort(f_np)[::-1][k - 1] if n >= k else 0.0
    ties = int(np.sum(np.isclose(f_np, kth, rtol=0, atol=1e-12)))
    first = next(iter(res.values()))
    budget = first["exact_budget"]
    rand = rng.choice(n, size=budget, replace=False)
    rand_top = rand[search.top_indices(all_np[rand], eng.n_pos, k)]
    pf1 = search.f1_float(pcounts, eng.n_pos)[parent_of]
    heur = np.argsort(-pf1, kind="stable")[:budget]
    heur_top = heur[search.top_indices(all_np[heur], eng.n_pos, k)]
    return {
        "candidates": n, "top_fraction": top, "audit_fraction": audit,
        "exhaustive_hyp_per_s": round(n / t_exh, 1), "exhaustive_seconds": round(t_exh, 4),
        "screener": res, "budget_sweep": budget_sweep, "budget_sweep_screener": swept,
        "candidates_tied_at_kth_f1": ties,
        f"random_recall_at_{k}": search.recall_at(rand_top, exact_top),
        f"parent_f1_recall_at_{k}": search.recall_at(heur_top, exact_top),
        "candidates_seconds": round(t_cands, 2),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--small", action="store_true", help="a reduced run of the same pipeline")
    ap.add_argument("--pairs", type=int, default=200_000)
    ap.add_argument("--candidates-beam", type=int, default=4096)
    ap.add_argument("--refinements", type=int, default=256)
    ap.add_argument("--epochs", type=int, default=10)
    ap.add_argument("--top", type=float, default=0.02)
    ap.add_argument("--audit", type=float, default=0.005)
    ap.add_argument("--k", type=int, default=100)
    ap.add_argument("--lr", type=float, default=5e-4)
    ap.add_argument("--modes", default="logdelta,delta,relative,absolute")
    ap.add_argument("--sweep", default="0.02,0.05,0.1",
                    help="top fractions at which the first log-removal screener's recall and speed are also "
                         "reported")
    ap.add_argument("--draws", type=int, default=1, help="candidate sets drawn from the same parents")
    ap.add_argument("--weight-decay", type=float, default=1e-4)
    ap.add_argument("--late-beam", type=int, default=0,
                    help="beam of the training rounds' second half (0: the same 256 throughout)")
    args = ap.parse_args()

    cfg = synth.CONFIGS["c3"]
    per_round = 16384
    if args.small:
        cfg = synth.small_config(n=200_000, n_concepts=256, depth=5, n_roles=12, s=1.6, cap=1024,
                                 n_data=8, missing=0.1, n_pos=10_000, n_neg=10_000, seed_index=3,
                                 total_edges=2_000_000)
        cfg = synth.KBConfig(**{**cfg.__dict__, "examples": "planted"})
        args.pairs, args.candidates_beam, args.refinements = 40_000, 512, 128
        per_round = 8192
    t = time.perf_counter()
    kb = synth.make_kb(cfg)
    log(f"[screen] KB {cfg.name}: N={kb.n:,}, {kb.n_edges:,} assertions ({time.perf_counter() - t:.1f}s)")
    eng = hthedl.Engine(kb, max_nodes=64, max_hyps=1)
    out = run(kb, eng, args.pairs, args.candidates_beam, args.refinements, args.epochs, args.top, args.audit,
              args.k, args.lr, per_round, modes=[m for m in args.modes.split(",") if m],
              sweep=[float(v) for v in args.sweep.split(",") if v], name=cfg.name, draws=args.draws,
              late_beam=args.late_beam, weight_decay=args.weight_decay)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
