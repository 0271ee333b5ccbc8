"""Pins of the oracle's numeric EXACT and multi-valued numeric concrete roles
(Section 3.2.3, Algorithms 9/10) against brute force over explicit
(subject, value) lists, the single-valued case, and order identities."""
import random

import numpy as np
import pytest

from oracle import Oracle
from paper_2412_00802_amd import synth

VALUES = [-2.0, -0.5, -0.0, 0.0, 0.5, 0.5, 1.0, float("inf"), float("-inf")]


def table_kb(n, tables, data=None):
    """KB with numeric roles given as {subject: [values]} per role."""
    kb = synth.kb_from_edges(n, [[0]], [[]], data, pos=list(range(0, n, 2)), neg=list(range(1, n, 2)))
    offs = np.zeros((len(tables), n + 1), np.int64)
    vals, base = [], 0
    for r, tab in enumerate(tables):
        offs[r, 0] = base
        for x in range(n):
            vs = tab.get(x, [])
            vals.extend(vs)
            base += len(vs)
            offs[r, x + 1] = base
    return synth.with_numeric_roles(kb, offs, np.asarray(vals, np.float32))


def brute(tab, n, cmp, t):
    """Written from the definition, one subject and one value at a time."""
    t = np.float32(t)
    out = set()
    for x in range(n):
        for v in tab.get(x, []):
            v = np.float32(v)
            if (cmp == "ge" and v >= t) or (cmp == "le" and v <= t) or (cmp == "eq" and v == t):
                out.add(x)
                break
    return out


@pytest.mark.parametrize("seed", range(6))
def test_numeric_roles_against_brute_force(seed):
    rnd = random.Random(seed)
    n = rnd.randint(1, 12)
    tables = [{x: [rnd.choice(VALUES) for _ in range(rnd.randint(0, 4))] for x in range(n) if rnd.random() < 0.7}
              for _ in range(2)]
    o = Oracle(table_kb(n, tables))
    for r, tab in enumerate(tables):
        for cmp in ("ge", "le", "eq"):
            for t in VALUES + [0.25, -1.0]:
                got = set(np.flatnonzero(o.ext(("n" + cmp, r, t))).tolist())
                assert got == brute(tab, n, cmp, t), (r, cmp, t)


def test_hand_example():
    # subject 0: {1, 3}; subject 1: {2}; subject 2: none; subject 3: {-1, 5}
    o = Oracle(table_kb(4, [{0: [1, 3], 1: [2], 3: [-1, 5]}]))
    assert np.flatnonzero(o.ext(("nge", 0, 3.0))).tolist() == [0, 3]
    assert np.flatnonzero(o.ext(("nle", 0, 1.0))).tolist() == [0, 3]
    assert np.flatnonzero(o.ext(("neq", 0, 2.0))).tolist() == [1]
    assert np.flatnonzero(o.ext(("neq", 0, 4.0))).tolist() == []
    assert np.flatnonzero(o.ext(("not", ("nge", 0, float("-inf"))))).tolist() == [2]


def test_single_values_match_the_data_column():
    """A role with at most one value per individual is the column with NaN
    where the value is absent: MIN / MAX / EXACT agree with >= / <= / ==."""
    rng = np.random.default_rng(3)
    n = 300
    col = np.round(rng.standard_normal(n) * 4).astype(np.float32)
    col[rng.random(n) < 0.2] = np.nan
    tab = {x: [float(col[x])] for x in range(n) if not np.isnan(col[x])}
    o = Oracle(table_kb(n, [tab], data=col[None, :]))
    for t in (-3.0, -0.0, 0.0, 1.0, 2.5, float("inf")):
        assert np.array_equal(o.ext(("nge", 0, t)), o.ext(("dge", 0, t)))
        assert np.array_equal(o.ext(("nle", 0, t)), o.ext(("dle", 0, t)))
        assert np.array_equal(o.ext(("neq", 0, t)), o.ext(("deq", 0, t)))
        # single-valued EXACT is MIN and MAX at once; NaN passes none of them
        assert np.array_equal(o.ext(("deq", 0, t)), o.ext(("dge", 0, t)) & o.ext(("dle", 0, t)))
    assert not o.ext(("deq", 0, float("nan"))).any()


def test_multi_value_identities():
    n = 2000
    kb = synth.kb_from_edges(n, [[0]], [[]])
    offs, vals = synth.numeric_roles(n, 3, seed=5, cap=16)
    o = Oracle(synth.with_numeric_roles(kb, offs, vals))
    has = np.diff(offs, axis=1) > 0
    for r in range(3):
        for t in (-1.0, 0.0, 0.0625, 1.5):
            ge, le, eq = (o.ext((c, r, t)) for c in ("nge", "nle", "neq"))
            assert not (eq & ~(ge & le)).any()            # EXACT within MIN and MAX
            assert np.array_equal(ge | le, has[r])        # every value is >= t or <= t
            assert not ((ge | le) & ~has[r]).any()
        assert np.array_equal(o.ext(("nge", r, float("-inf"))), has[r])
        a, b = o.ext(("nge", r, -0.5)), o.ext(("nge", r, 0.5))
        assert not (b & ~a).any()                         # MIN is antitone in t
        # with many values per subject, EXACT is strictly inside MIN and MAX somewhere
    assert any((o.ext(("nge", r, 0.0)) & o.ext(("nle", r, 0.0)) & ~o.ext(("neq", r, 0.0))).any()
               for r in range(3))


def test_numeric_hypotheses_evaluate():
    n = 500
    kb = synth.kb_from_edges(n, [[0, 1, 2], list(range(0, n, 3))], [[(i, (i * 7) % n) for i in range(n)]])
    offs, vals = synth.numeric_roles(n, 2, seed=9)
    kb = synth.with_numeric_roles(kb, offs, vals)
    hs = synth.make_numeric_hypotheses(kb, 50, seed=1)
    cov = Oracle(kb).coverages(hs)
    assert cov.shape == (50, 2)


class StrictMin(Oracle):
    def num_some(self, p, cmp, t):
        if cmp == "ge":
            subj, val = self.num_values(p)
            out = np.zeros(self.n, dtype=bool)
            out[subj[val > np.float32(t)]] = True
            return out
        return super().num_some(p, cmp, t)


class EveryValueMustPass(Oracle):
    """A universal reading of the concrete restriction."""
    def num_some(self, p, cmp, t):
        subj, val = self.num_values(p)
        bad = ~(val >= np.float32(t)) if cmp == "ge" else ~(val <= np.float32(t)) if cmp == "le" else val != t
        out = np.diff(self._noff[p]) > 0
        out[subj[bad]] = False
        return out


class ExactIsMinAndMax(Oracle):
    def num_some(self, p, cmp, t):
        if cmp == "eq":
            return super().num_some(p, "ge", t) & super().num_some(p, "le", t)
        return super().num_some(p, cmp, t)


@pytest.mark.parametrize("mutant", [StrictMin, EveryValueMustPass, ExactIsMinAndMax])
def test_pins_reject_planted_mistakes(mutant):
    """Each plausible mistake in the numeric concrete-role code fails the
    brute-force pin on some small table."""
    caught = False
    for seed in range(40):
        rnd = random.Random(seed)
        n = rnd.randint(2, 10)
        tab = {x: [rnd.choice(VALUES) for _ in range(rnd.randint(0, 4))] for x in range(n)}
        o = mutant(table_kb(n, [tab]))
        for cmp in ("ge", "le", "eq"):
            for t in VALUES:
                if set(np.flatnonzero(o.ext(("n" + cmp, 0, t))).tolist()) != brute(tab, n, cmp, t):
                    caught = True
        if caught:
            break
    assert caught
