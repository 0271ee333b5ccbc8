"""The pins catch plausible mistakes: each mutant plants one in a copy of the
oracle (on the CPU) and the brute-force pin must reject it."""
import random

import numpy as np
import pytest

from oracle import Oracle
from tests.pin_semantics import bits_to_set, brute_ext, kb_sets
from tests.test_oracle_pins import random_hyp, random_kb


class InverseIgnored(Oracle):
    def count(self, r, inv, c):
        return super().count(r, 0, c)


class ForwardTransposed(Oracle):
    def count(self, r, inv, c):
        return super().count(r, 1 - inv, c)


class PaperAtMost(Oracle):
    """At-most with the extra cnt > 0 guard of the printed filter."""
    def ext(self, h):
        if h[0] == "atmost":
            _, k, r, inv, c = h
            cnt = self.count(r, inv, self.ext(c))
            return (cnt <= k) & (cnt > 0)
        return super().ext(h)


class ForallNeedsSuccessor(Oracle):
    def ext(self, h):
        if h[0] == "forall":
            _, r, inv, c = h
            has = self.count(r, inv, np.ones(self.n, dtype=bool)) > 0
            return super().ext(h) & has
        return super().ext(h)


class ExistsOffByOne(Oracle):
    def ext(self, h):
        if h[0] == "exists":
            _, r, inv, c = h
            return self.count(r, inv, self.ext(c)) >= 2
        return super().ext(h)


class StrictThreshold(Oracle):
    def data_ge(self, p, t):
        return self._data[p] > np.float32(t)


class EmptyAndIsBottom(Oracle):
    def ext(self, h):
        if h == ("and",):
            return np.zeros(self.n, dtype=bool)
        return super().ext(h)


class ExactlyAsAtLeast(Oracle):
    def ext(self, h):
        if h[0] == "exactly":
            return super().ext(("atleast",) + tuple(h[1:]))
        return super().ext(h)


class MissingIsZero(Oracle):
    def data_le(self, p, t):
        col = np.nan_to_num(self._data[p], nan=0.0)
        return col <= np.float32(t)


class CoverageSwapped(Oracle):
    def coverage(self, h):
        p, q = super().coverage(h)
        return q, p


MUTANTS = [InverseIgnored, ForwardTransposed, PaperAtMost, ForallNeedsSuccessor,
           ExistsOffByOne, StrictThreshold, EmptyAndIsBottom, ExactlyAsAtLeast,
           MissingIsZero, CoverageSwapped]


@pytest.mark.parametrize("mutant", MUTANTS, ids=lambda m: m.__name__)
def test_pin_rejects_mutant(mutant):
    rnd = random.Random(1234)
    for trial in range(400):
        n = rnd.randint(1, 8)
        kb = random_kb(rnd, n)
        o = mutant(kb)
        sets = kb_sets(kb)
        pset, nset = bits_to_set(kb.pos_bits, n), bits_to_set(kb.neg_bits, n)
        for _ in range(20):
            h = random_hyp(rnd, 3, 3, 2, 2)
            want = brute_ext(sets, n, h)
            if set(np.flatnonzero(o.ext(h)).tolist()) != want:
                return
            if o.coverage(h) != (len(want & pset), len(want & nset)):
                return
    pytest.fail(f"{mutant.__name__} survived the brute-force pin")
