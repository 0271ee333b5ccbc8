"""Pins of the oracle's string concrete roles (EQUAL and CONTAIN, Section
3.2.3, Algorithms 11-14) against brute force over explicit string tables, the
identity CONTAIN(s) = union of EQUAL(t) over the strings t holding s, and
planted mistakes."""
import random

import numpy as np
import pytest

from oracle import Oracle
from paper_2412_00802_amd import synth

WORDS = [b"", b"a", b"ab", b"abc", b"ba", b"cab", b"abab", b"c"]


def table_kb(n, tables, strings):
    """KB with string roles given as {subject: [string ids]} per role."""
    kb = synth.kb_from_edges(n, [[0]], [[]], pos=list(range(0, n, 2)), neg=list(range(1, n, 2)))
    offs = np.zeros((len(tables), n + 1), np.int64)
    ids, base = [], 0
    for r, tab in enumerate(tables):
        offs[r, 0] = base
        for x in range(n):
            vs = tab.get(x, [])
            ids.extend(vs)
            base += len(vs)
            offs[r, x + 1] = base
    return synth.with_string_roles(kb, offs, np.asarray(ids, np.int32), strings)


def brute(tab, strings, n, kind, q):
    out = set()
    for x in range(n):
        for i in tab.get(x, []):
            s = strings[i]
            if (kind == "sequal" and s == q) or (kind == "scontains" and s.find(q) >= 0):
                out.add(x)
                break
    return out


def random_tables(rnd, n, k=2):
    return [{x: [rnd.randrange(len(WORDS)) for _ in range(rnd.randint(0, 3))] for x in range(n)
             if rnd.random() < 0.7} for _ in range(k)]


@pytest.mark.parametrize("seed", range(6))
def test_strings_against_brute_force(seed):
    rnd = random.Random(seed)
    n = rnd.randint(1, 12)
    tables = random_tables(rnd, n)
    o = Oracle(table_kb(n, tables, WORDS))
    for r, tab in enumerate(tables):
        for kind in ("sequal", "scontains"):
            for q in WORDS + [b"zz", b"abcabc", b"b"]:
                got = set(np.flatnonzero(o.ext((kind, r, q))).tolist())
                assert got == brute(tab, WORDS, n, kind, q), (r, kind, q)


def test_contain_is_the_union_of_equals():
    n = 3000
    kb = synth.kb_from_edges(n, [[0]], [[]])
    offs, ids, strings = synth.string_roles(n, 2, seed=4, n_strings=300)
    o = Oracle(synth.with_string_roles(kb, offs, ids, strings))
    has = np.diff(offs, axis=1) > 0
    for r in range(2):
        for q in (b"a", b"ab", b"fed", b"cc", b"abcdefabcdef"):
            union = np.zeros(n, bool)
            for t in strings:
                if q in t:
                    union |= o.ext(("sequal", r, t))
            assert np.array_equal(o.ext(("scontains", r, q)), union)
        assert np.array_equal(o.ext(("scontains", r, b"")), has[r])
        assert not o.ext(("sequal", r, b"not-a-word")).any()
        for t in strings[:20]:
            assert not (o.ext(("sequal", r, t)) & ~o.ext(("scontains", r, t))).any()


class PrefixContain(Oracle):
    def ext(self, h):
        if h[0] == "scontains":
            q = bytes(h[2])
            return self.str_some(h[1], lambda v: v.startswith(q))
        return super().ext(h)


class EqualIsContain(Oracle):
    def ext(self, h):
        if h[0] == "sequal":
            q = bytes(h[2])
            return self.str_some(h[1], lambda v: q in v)
        return super().ext(h)


class EveryStringMustMatch(Oracle):
    def str_some(self, p, test):
        subj, vals = self.str_values(p)
        out = np.diff(self._soff[p]) > 0
        for x, v in zip(subj.tolist(), vals):
            if not test(v):
                out[x] = False
        return out


@pytest.mark.parametrize("mutant", [PrefixContain, EqualIsContain, EveryStringMustMatch])
def test_pins_reject_planted_mistakes(mutant):
    caught = False
    for seed in range(40):
        rnd = random.Random(seed)
        n = rnd.randint(2, 10)
        tables = random_tables(rnd, n, k=1)
        o = mutant(table_kb(n, tables, WORDS))
        for kind in ("sequal", "scontains"):
            for q in WORDS:
                if set(np.flatnonzero(o.ext((kind, 0, q))).tolist()) != brute(tables[0], WORDS, n, kind, q):
                    caught = True
        if caught:
            break
    assert caught


def test_string_hypotheses_evaluate():
    n = 500
    kb = synth.kb_from_edges(n, [[0, 1, 2], list(range(0, n, 3))], [[(i, (i * 7) % n) for i in range(n)]])
    offs, ids, strings = synth.string_roles(n, 2, seed=9, n_strings=100)
    kb = synth.with_string_roles(kb, offs, ids, strings)
    hs = synth.make_string_hypotheses(kb, 50, seed=1)
    assert Oracle(kb).coverages(hs).shape == (50, 2)
