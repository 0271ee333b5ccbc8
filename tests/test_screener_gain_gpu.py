"""What the learned screener gains: trained on engine-labelled refinements of a
planted-target KB, it ranks a fresh candidate set, and its top share holds far
more of the exact top-k than a random share of the same size (the exact engine,
run on every candidate, is the judge)."""
import sys

import numpy as np
import pytest

from paper_2412_00802_amd import hthedl, search, synth
from paper_2412_00802_amd.screened import gather_training_pairs, removal_targets, score, train
from paper_2412_00802_amd.screener import FeatureBatch, Screener, init_params

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_screener_beats_random_selection():
    import torch
    assert torch.cuda.is_available()
    cfg = synth.small_config(n=100_000, n_concepts=96, depth=4, n_roles=6, s=1.6, cap=256, n_data=4,
                             missing=0.1, n_pos=5000, n_neg=5000, seed_index=1900, total_edges=600_000)
    cfg = synth.KBConfig(**{**cfg.__dict__, "examples": "planted"})
    kb = synth.make_kb(cfg)
    eng = hthedl.Engine(kb, max_nodes=64, max_hyps=1)
    rng = np.random.default_rng(19)
    hyps, counts, pcounts, tparents, tpidx = gather_training_pairs(eng, kb, 16384, 4096, 64, rng, 8192)
    order = rng.permutation(len(hyps))
    hyps = [hyps[i] for i in order]
    counts, pcounts, tpidx = counts[order], pcounts[order], tpidx[order]
    fb = FeatureBatch(*hthedl.encode_batch(hyps))
    tpfb = FeatureBatch(*hthedl.encode_batch(tparents))
    tpi = torch.from_numpy(tpidx.astype(np.int32)).cuda()
    # the screener predicts log(1 + positives and negatives a refinement removes
    # from its exactly evaluated parent), from features relative to the parent
    y = torch.from_numpy(removal_targets(counts, pcounts)).cuda()
    scr = Screener(init_params(seed=11), batch=4096, lr=5e-4, loss="mse")
    losses = train(scr, fb, y, len(hyps), 16, 512, rng, tpfb, tpi)
    say(f"[gain] {len(hyps)} pairs, loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert losses[-1] < losses[0]
    # fresh candidates: refinements of the best 128 hypotheses seen
    top = search.top_indices(counts, eng.n_pos, 128)
    ref = search.Refiner(kb, rng)
    cands, base, pidx, seen = [], [], [], set(hyps)
    for j, i in enumerate(top):
        for c in ref.refine(hyps[i], 96):
            if c not in seen:
                seen.add(c)
                cands.append(c)
                base.append(counts[i])
                pidx.append(j)
    n = len(cands)
    cfb = FeatureBatch(*hthedl.encode_batch(cands))
    pfb = FeatureBatch(*hthedl.encode_batch([hyps[i] for i in top]))
    scores = torch.empty(n, dtype=torch.float32, device="cuda")
    base = torch.from_numpy(np.asarray(base, dtype=np.uint32).view(np.int32)).cuda()
    score(scr, cfb, n, eng.n_pos, eng.n_neg, scores, base=base, parents=pfb,
          parent_index=torch.from_numpy(np.asarray(pidx, dtype=np.int32)).cuda(), kind=1)
    exact = eng.eval_batch(cands, chunk=8192)
    k, budget = 50, n // 20
    want = search.top_indices(exact, eng.n_pos, k)
    pick = np.argsort(-scores.cpu().numpy(), kind="stable")[:budget]
    got = pick[search.top_indices(exact[pick], eng.n_pos, k)]
    recall = search.recall_at(got, want)
    rand = []
    for s in range(5):
        rp = np.random.default_rng(100 + s).choice(n, size=budget, replace=False)
        rand.append(search.recall_at(rp[search.top_indices(exact[rp], eng.n_pos, k)], want))
    say(f"[gain] {n} candidates, exact budget {budget}: screener recall@{k} {recall:.2f}, "
        f"random {np.mean(rand):.2f}")
    assert recall >= np.mean(rand) + 0.2
