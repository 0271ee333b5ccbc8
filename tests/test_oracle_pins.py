"""Pins of the CPU oracle against formulations that share nothing with it.

* brute-force first-order evaluation on tiny KBs (random and exhaustive);
* the dense adjacency closed form cnt = A 1_C;
* an SQLite translation of each hypothesis;
* coverage as |ext(H) & P| on explicit sets (Algorithm 15).
"""
import itertools
import random

import numpy as np
import pytest

from oracle import Oracle
from paper_2412_00802_amd import synth
from tests.pin_semantics import SqlKB, bits_to_set, brute_ext, dense_counts, kb_sets

VALUES = [-1.5, -0.0, 0.0, 0.25, 0.25, 2.0, float("nan")]


def random_kb(rnd: random.Random, n, n_concepts=3, n_roles=2, n_data=2, p_edge=None):
    concepts = [[x for x in range(n) if rnd.random() < rnd.choice([0.2, 0.5, 0.8])]
                for _ in range(n_concepts)]
    roles = []
    for _ in range(n_roles):
        p = p_edge if p_edge is not None else rnd.choice([0.1, 0.3, 0.6])
        roles.append([(a, b) for a in range(n) for b in range(n) if rnd.random() < p])
    data = np.array([[rnd.choice(VALUES) for _ in range(n)] for _ in range(n_data)],
                    dtype=np.float32)
    pos = [x for x in range(n) if rnd.random() < 0.3]
    neg = [x for x in range(n) if x not in pos and rnd.random() < 0.4]
    return synth.kb_from_edges(n, concepts, roles, data, pos, neg)


def random_hyp(rnd: random.Random, depth, n_concepts, n_roles, n_data):
    if depth <= 1 or rnd.random() < 0.25:
        u = rnd.random()
        if u < 0.55:
            return ("atom", rnd.randrange(n_concepts))
        if u < 0.8 and n_data:
            t = rnd.choice([-2.0, -1.5, -0.0, 0.0, 0.25, 1.0, 2.0, 3.0])
            return (rnd.choice(["dge", "dle"]), rnd.randrange(n_data), t)
        return (rnd.choice(["top", "bot"]),)
    op = rnd.choice(["and", "or", "not", "exists", "forall", "atleast", "atmost", "exactly"])
    sub = lambda: random_hyp(rnd, depth - 1, n_concepts, n_roles, n_data)  # noqa: E731
    if op in ("and", "or"):
        return (op,) + tuple(sub() for _ in range(rnd.choice([0, 1, 2, 3])))
    if op == "not":
        return ("not", sub())
    r, inv = rnd.randrange(n_roles), rnd.randrange(2)
    if op in ("exists", "forall"):
        return (op, r, inv, sub())
    return (op, rnd.randrange(0, 5), r, inv, sub())


def test_brute_force_random_tiny():
    rnd = random.Random(7)
    checked = 0
    for trial in range(60):
        n = rnd.randint(1, 9)
        kb = random_kb(rnd, n)
        o = Oracle(kb)
        sets = kb_sets(kb)
        for _ in range(40):
            h = random_hyp(rnd, 4, 3, 2, 2)
            got = set(np.flatnonzero(o.ext(h)).tolist())
            assert got == brute_ext(sets, n, h), (trial, h)
            pos, neg = o.coverage(h)
            pset = bits_to_set(kb.pos_bits, n)
            nset = bits_to_set(kb.neg_bits, n)
            assert (pos, neg) == (len(got & pset), len(got & nset))
            checked += 1
    assert checked == 2400


def _exhaustive_hyps():
    fillers = [("atom", 0), ("not", ("atom", 0)), ("top",), ("bot",)]
    hs = [("top",), ("bot",), ("atom", 0), ("not", ("atom", 0))]
    for inv in (0, 1):
        for c in fillers:
            hs.append(("exists", 0, inv, c))
            hs.append(("forall", 0, inv, c))
            for k in range(4):
                for op in ("atleast", "atmost", "exactly"):
                    hs.append((op, k, 0, inv, c))
    return hs


def test_exhaustive_three_individuals():
    """Every relation on 3 individuals (2^9) x every concept extension (2^3)."""
    n = 3
    pairs = [(a, b) for a in range(n) for b in range(n)]
    hs = _exhaustive_hyps()
    for rel_mask in range(1 << 9):
        rel = [pairs[i] for i in range(9) if (rel_mask >> i) & 1]
        for cmask in range(8):
            conc = [x for x in range(n) if (cmask >> x) & 1]
            kb = synth.kb_from_edges(n, [conc], [rel])
            o = Oracle(kb)
            sets = kb_sets(kb)
            for h in hs:
                got = set(np.flatnonzero(o.ext(h)).tolist())
                assert got == brute_ext(sets, n, h), (rel, conc, h)


def test_dense_adjacency_closed_form():
    rnd = random.Random(11)
    for n in (1, 17, 64, 65, 130):
        kb = random_kb(rnd, n, n_concepts=4, n_roles=3, p_edge=0.08)
        o = Oracle(kb)
        for a in range(4):
            c = o.member(a)
            for r in range(3):
                for inv in (0, 1):
                    np.testing.assert_array_equal(o.count(r, inv, c), dense_counts(kb, r, inv, c))
                    cnt = dense_counts(kb, r, inv, c)
                    cnt_not = dense_counts(kb, r, inv, ~c)
                    np.testing.assert_array_equal(o.ext(("exists", r, inv, ("atom", a))), cnt >= 1)
                    np.testing.assert_array_equal(o.ext(("forall", r, inv, ("atom", a))), cnt_not == 0)
                    for k in range(4):
                        np.testing.assert_array_equal(
                            o.ext(("atleast", k, r, inv, ("atom", a))), cnt >= k)
                        np.testing.assert_array_equal(
                            o.ext(("atmost", k, r, inv, ("atom", a))), cnt <= k)
                        np.testing.assert_array_equal(
                            o.ext(("exactly", k, r, inv, ("atom", a))), cnt == k)


def test_sqlite_translation():
    rnd = random.Random(3)
    for trial in range(6):
        n = rnd.randint(20, 60)
        kb = random_kb(rnd, n, n_concepts=4, n_roles=3, p_edge=rnd.choice([0.03, 0.1]))
        o = Oracle(kb)
        sq = SqlKB(kb)
        for _ in range(40):
            h = random_hyp(rnd, 4, 4, 3, 2)
            got = set(np.flatnonzero(o.ext(h)).tolist())
            assert got == sq.ext(h), (trial, h)


def test_sqlite_on_generated_workload():
    """The generator's own hypothesis shapes on a small generated KB."""
    cfg = synth.small_config(n=120, n_concepts=10, n_roles=3, cap=8, n_hyps=80, seed_index=5)
    kb = synth.make_kb(cfg)
    hyps = synth.make_hypotheses(cfg, kb)
    o = Oracle(kb)
    sq = SqlKB(kb)
    for h in hyps:
        assert set(np.flatnonzero(o.ext(h)).tolist()) == sq.ext(h), h


@pytest.mark.parametrize("n", [1, 63, 64, 65, 200])
def test_ext_bits_padding(n):
    rnd = random.Random(n)
    kb = random_kb(rnd, n)
    o = Oracle(kb)
    for h in [("top",), ("not", ("atom", 0)), ("forall", 0, 1, ("bot",))]:
        words = o.ext_bits(h)
        assert words.shape[0] == (n + 63) // 64
        assert bits_to_set(words, 10 ** 9) == set(np.flatnonzero(o.ext(h)).tolist())
        r = n & 63
        if r:
            assert int(words[-1]) >> r == 0
