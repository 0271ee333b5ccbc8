"""Refinement and search logic on the CPU, with the oracle standing in for the
exact engine (the search code only sees an `evaluate` callable)."""
import numpy as np

from oracle import Oracle
from paper_2412_00802_amd import search, synth


def small():
    cfg = synth.small_config(n=1500, n_concepts=24, depth=3, n_roles=3, cap=20, n_data=2,
                             n_pos=200, n_neg=200, seed_index=1300)
    kb = synth.make_kb(cfg)
    return cfg, kb, Oracle(kb)


def test_refinements_are_specialisations():
    cfg, kb, o = small()
    rng = np.random.default_rng(0)
    ref = search.Refiner(kb, rng)
    parents = synth.make_hypotheses(cfg, kb, count=40, depth=4)
    parents += [("top",), ("atom", 0), ("not", ("atom", 3)), ("atmost", 2, 0, 0, ("atom", 5)),
                ("dge", 0, float(kb.deciles[0, 3])), ("not", ("atleast", 2, 1, 1, ("atom", 1)))]
    checked = 0
    for p in parents:
        ep = o.ext(p)
        kids = ref.refine(p, 12)
        assert len(kids) == len(set(kids)) and p not in kids
        for c in kids:
            ec = o.ext(c)
            assert not np.any(ec & ~ep), (p, c)
            checked += 1
    assert checked > 300


def test_f1_ranking_exact_ties():
    counts = np.array([[10, 5], [20, 10], [20, 10], [0, 0], [30, 40], [10, 5]])
    order = search.rank(counts, n_pos=40, sizes=[3, 3, 2, 1, 1, 1])
    # (20,10) and (10,5)?  F1 = 40/70 vs 20/55: (20,10) wins; equal rows break by size, then index
    assert order[0] == 2 and order[1] == 1
    assert order[-1] == 3
    top = search.top_indices(counts, 40, 2)
    assert sorted(top.tolist()) == [1, 2]


def test_refinement_trace_with_oracle_engine():
    cfg, kb, o = small()
    n_pos = int(o.pos.sum())
    rng = np.random.default_rng(1)
    prev_beam = [("top",)]
    for r, cands, counts in search.refinement_rounds(kb, o.coverages, n_pos, rounds=3, per_round=120,
                                                    beam=8, rng=rng):
        assert len(cands) == 120 == len(set(cands)) and counts.shape == (120, 2)
        # every candidate specialises one of the previous round's beam
        exts = [o.ext(p) for p in prev_beam]
        for c in cands[:40]:
            ec = o.ext(c)
            assert any(not np.any(ec & ~ep) for ep in exts), c
        prev_beam = [cands[i] for i in search.top_indices(counts, n_pos, 8)]


def test_recall():
    assert search.recall_at([1, 2, 3], [3, 4, 5]) == 1 / 3
    assert search.recall_at(range(100), range(100)) == 1.0


def test_trace_set_substitution_expands_back():
    """Replacing cached parent subtrees by set leaves loses nothing: expanding
    the leaves again gives the candidate back, and add-conjunct candidates of
    an and-parent read the parent as one leaf."""
    from paper_2412_00802_amd import trace
    cfg, kb, o = small()
    rng = np.random.default_rng(4)
    ref = search.Refiner(kb, rng)
    parents = [("and", ("atom", 1), ("exists", 0, 1, ("atom", 2)))] + synth.make_hypotheses(cfg, kb, count=30, depth=4)
    want = {}
    for p in parents:
        want.setdefault(p, None)
        trace.subtrees(p, want)
    cache = object.__new__(trace.SetCache)
    cache.slot = {k: 100 + i for i, k in enumerate(want)}
    inv = {v: k for k, v in cache.slot.items()}

    def expand(h):
        if h[0] == "set":
            return inv[h[1]]
        if h[0] == "not":
            return ("not", expand(h[1]))
        if h[0] in ("and", "or"):
            out = []
            for c in h[1:]:
                e = expand(c)
                # a set leaf standing for an and-parent inside an and: flatten back
                out.extend(e[1:] if (c[0] == "set" and e[0] == "and" and h[0] == "and") else [e])
            return (h[0],) + tuple(out)
        if h[0] in trace.ROLE_OPS:
            return h[:-1] + (expand(h[-1]),)
        return h

    n_one_leaf = 0
    for p in parents:
        for c in ref.refine(p, 10):
            s = cache.substitute(c, p)
            assert expand(s) == c or o.coverage(expand(s)) == o.coverage(c)
            if p[0] == "and" and s[0] == "and" and s[1] == ("set", cache.slot[p]):
                n_one_leaf += 1
    assert n_one_leaf > 0


def test_refinement_rounds_end_on_a_small_candidate_space():
    """A KB with fewer distinct one-step candidates than a round asks for:
    the rounds still end, with distinct candidates."""
    cfg = synth.small_config(n=200, n_concepts=4, depth=2, n_roles=1, cap=4, n_data=1, n_pos=20, n_neg=20,
                             seed_index=1310)
    kb = synth.make_kb(cfg)
    o = Oracle(kb)
    rng = np.random.default_rng(2)
    n = 0
    for r, cands, counts in search.refinement_rounds(kb, o.coverages, int(o.pos.sum()), rounds=2,
                                                    per_round=3000, beam=2, rng=rng):
        assert len(cands) == len(set(cands)) and counts.shape == (len(cands), 2)
        n += 1
    assert n == 2


def test_oracle_f1_hand_values():
    """F1 = 2TP / (2TP + FP + FN) with TP = pos, FP = neg, FN = |P| - pos."""
    from fractions import Fraction

    from oracle.dl import f1_score

    def f(p, n, P):
        a, b = f1_score(p, n, P)
        return Fraction(a, b)

    assert f(20, 10, 40) == Fraction(40, 70)          # 2*20 / (40 + 10 + 20)
    assert f(40, 0, 40) == 1                          # every positive, no negative
    assert f(0, 7, 40) == 0
    assert f(10, 5, 40) == Fraction(20, 55)           # 20 / (20 + 5 + 30)
    assert f1_score(0, 0, 0) == (0, 1)                # empty denominator
    assert f(3, 1, 4) == Fraction(6, 8)               # TP 3, FP 1, FN 1


def test_rank_agrees_with_the_oracle_f1():
    """search.rank's order, checked against the oracle's exact F1: F1 never
    rises along the order, and equal F1 breaks by pos descending, neg ascending,
    size ascending, then index."""
    from fractions import Fraction

    from oracle.dl import f1_score
    rng = np.random.default_rng(7)
    n_pos = 50
    counts = np.stack([rng.integers(0, n_pos + 1, 400), rng.integers(0, 60, 400)], axis=1)
    counts[::7] = counts[3]                           # plenty of exact ties
    sizes = rng.integers(1, 6, 400)
    order = search.rank(counts, n_pos, sizes)
    assert sorted(order.tolist()) == list(range(400))

    def key(i):
        a, b = f1_score(int(counts[i, 0]), int(counts[i, 1]), n_pos)
        return (-Fraction(a, b), -int(counts[i, 0]), int(counts[i, 1]), int(sizes[i]), i)

    assert order.tolist() == sorted(range(400), key=key)
    # the vectorised pre-filter keeps the exact order (no size tie-break there)
    top = search.top_indices(counts, n_pos, 25)
    assert top.tolist() == sorted(range(400), key=lambda i: key(i)[:3] + (i,))[:25]
