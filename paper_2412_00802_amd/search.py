"""Refinement search around the exact engine (host-side orchestration).

The paper evaluates hypotheses for an ILP learner but defines no learner.  The
refinement trace and the screened search of this project need one: a
refinement operator (one-step specialisations), F1 scoring compared exactly,
beam selection, and the screened search that ranks candidates with the learned
screener before exact evaluation.

Readings (the paper is silent on all of them):
* F1 = 2 TP / (2 TP + FP + FN) with TP = pos, FP = neg, FN = |P| - pos; 0 when
  the denominator is 0.  Comparisons cross-multiply in integers.  Ties break by
  pos descending, then neg ascending, then node count ascending, then the
  candidate's index.
* Every refinement is a specialisation: ext(child) is a subset of ext(parent).
  Positions under an odd number of {not, at-most filler} have negative
  polarity; nothing is refined inside an exactly-n filler.
"""
from __future__ import annotations

import functools
from typing import Callable, List, Sequence, Tuple

import numpy as np

from .synth import hyp_size

ROLE_OPS = ("exists", "forall", "atleast", "atmost", "exactly")


# ---------------------------------------------------------------------------
# scoring
# ---------------------------------------------------------------------------


def f1_key(pos: int, neg: int, n_pos: int) -> Tuple[int, int]:
    """F1 as an exact fraction (numerator, denominator)."""
    den = pos + neg + n_pos                  # = 2 TP + FP + FN
    return (2 * pos, den) if den else (0, 1)


def rank(counts: np.ndarray, n_pos: int, sizes: Sequence[int] = None) -> np.ndarray:
    """Indices sorted best-first by exact F1 with the stated tie-breaks."""
    counts = np.asarray(counts, dtype=np.int64)

    def cmp(i, j):
        a_num, a_den = f1_key(counts[i, 0], counts[i, 1], n_pos)
        b_num, b_den = f1_key(counts[j, 0], counts[j, 1], n_pos)
        lhs, rhs = a_num * b_den, b_num * a_den
        if lhs != rhs:
            return -1 if lhs > rhs else 1
        if counts[i, 0] != counts[j, 0]:
            return -1 if counts[i, 0] > counts[j, 0] else 1
        if counts[i, 1] != counts[j, 1]:
            return -1 if counts[i, 1] < counts[j, 1] else 1
        if sizes is not None and sizes[i] != sizes[j]:
            return -1 if sizes[i] < sizes[j] else 1
        return -1 if i < j else (1 if i > j else 0)

    return np.array(sorted(range(counts.shape[0]), key=functools.cmp_to_key(cmp)), dtype=np.int64)


def f1_float(counts: np.ndarray, n_pos: int) -> np.ndarray:
    c = np.asarray(counts, dtype=np.float64)
    den = c[:, 0] + c[:, 1] + n_pos
    return np.where(den > 0, 2 * c[:, 0] / np.maximum(den, 1), 0.0)


def top_indices(counts: np.ndarray, n_pos: int, k: int) -> np.ndarray:
    """The k best by exact F1 (vectorised pre-filter, exact rank on the short list)."""
    f = f1_float(counts, n_pos)
    k = min(k, counts.shape[0])
    if k == 0:
        return np.zeros(0, dtype=np.int64)
    # candidates whose float F1 reaches the k-th value (ties kept), then exact ranking
    kth = np.partition(f, counts.shape[0] - k)[counts.shape[0] - k]
    short = np.flatnonzero(f >= kth - 1e-12)
    order = rank(counts[short], n_pos)
    return short[order[:k]]


# ---------------------------------------------------------------------------
# refinement operator
# ---------------------------------------------------------------------------


class Refiner:
    """One-step specialisations of a hypothesis.

    kb supplies concept_parent (to find tree children), n_concepts, n_roles,
    n_data and deciles."""

    def __init__(self, kb, rng: np.random.Generator):
        self.rng = rng
        self.nc, self.nr, self.nd = kb.n_concepts, kb.n_roles, kb.n_data
        self.dec = np.asarray(kb.deciles, dtype=np.float32)
        parent = np.asarray(kb.concept_parent)
        self.children = [[] for _ in range(self.nc)]
        for c, p in enumerate(parent.tolist()):
            if p >= 0:
                self.children[p].append(c)

    # a random conjunct X (the added conjunct of H -> H and X)
    def conjunct(self):
        u = self.rng.random()
        if u < 0.5:
            return ("atom", int(self.rng.integers(0, self.nc)))
        if u < 0.8 and self.nr:
            return ("exists", int(self.rng.integers(0, self.nr)), int(self.rng.integers(0, 2)),
                    ("atom", int(self.rng.integers(0, self.nc))))
        if self.nd:
            p, k = int(self.rng.integers(0, self.nd)), int(self.rng.integers(0, 9))
            return ("dge" if self.rng.random() < 0.5 else "dle", p, float(self.dec[p, k]))
        return ("atom", int(self.rng.integers(0, self.nc)))

    def _decile_index(self, p, t):
        hits = np.flatnonzero(self.dec[p] == np.float32(t))
        return int(hits[0]) if hits.size else -1

    def positions(self, h, pol=1, path=()):
        """(path, node, polarity) of every refinable position."""
        yield path, h, pol
        op = h[0]
        if op == "not":
            yield from self.positions(h[1], -pol, path + (1,))
        elif op in ("and", "or"):
            for i, c in enumerate(h[1:], start=1):
                yield from self.positions(c, pol, path + (i,))
        elif op in ("exists", "forall", "atleast"):
            yield from self.positions(h[-1], pol, path + (len(h) - 1,))
        elif op == "atmost":
            yield from self.positions(h[-1], -pol, path + (len(h) - 1,))

    @staticmethod
    def replace(h, path, new):
        if not path:
            return new
        i = path[0]
        return h[:i] + (Refiner.replace(h[i], path[1:], new),) + h[i + 1:]

    def local(self, node, pol):
        """Specialisations (pol > 0) or generalisations (pol < 0) of one node."""
        op = node[0]
        out = []
        if op == "atom":
            a = node[1]
            if pol > 0:
                out += [("atom", c) for c in self.children[a]]
                out.append(("and", node, ("atom", int(self.rng.integers(0, self.nc)))))
            else:
                out.append(("or", node, ("atom", int(self.rng.integers(0, self.nc)))))
        elif op == "atleast" and pol > 0:
            out.append(("atleast", node[1] + 1) + node[2:])
        elif op == "atmost" and pol > 0 and node[1] >= 1:
            out.append(("atmost", node[1] - 1) + node[2:])
        elif op == "atleast" and pol < 0 and node[1] >= 2:
            out.append(("atleast", node[1] - 1) + node[2:])
        elif op == "atmost" and pol < 0:
            out.append(("atmost", node[1] + 1) + node[2:])
        elif op in ("dge", "dle"):
            k = self._decile_index(node[1], node[2])
            if k >= 0:
                tighter = k + 1 if (op == "dge") == (pol > 0) else k - 1
                if 0 <= tighter < 9:
                    out.append((op, node[1], float(self.dec[node[1], tighter])))
        return out

    def refine(self, h, count: int, conjuncts: bool = True) -> List[tuple]:
        """Up to `count` distinct one-step specialisations of h: up to half of
        them local (a position of h specialised), the rest added conjuncts
        (none with conjuncts=False)."""
        seen, out = {h}, []
        locs = []
        for path, node, pol in self.positions(h):
            for r in self.local(node, pol):
                locs.append(self.replace(h, path, r))
        self.rng.shuffle(locs)
        for c in locs[: count // 2]:
            if c not in seen:
                seen.add(c)
                out.append(c)
        tries = 0
        while conjuncts and len(out) < count and tries < 8 * count:
            tries += 1
            base = h[1:] if h[0] == "and" else (h,)
            c = ("and",) + tuple(base) + (self.conjunct(),)
            if c not in seen:
                seen.add(c)
                out.append(c)
        return out


def refinement_rounds(kb, evaluate: Callable[[Sequence[tuple]], np.ndarray], n_pos: int,
                      rounds: int, per_round: int, beam: int, rng: np.random.Generator,
                      start: Sequence[tuple] = (("top",),), start_counts=None, with_parents: bool = False,
                      late_beam: int = 0):
    """A refinement trace: each round refines the previous round's top `beam`
    hypotheses into `per_round` candidates and evaluates them exactly (from
    round rounds // 2 on, the top `late_beam` when it is set).
    Yields (round, candidates, counts), and with with_parents also the round's
    parents, each candidate's parent index among them and its parent's
    coverage (start_counts for the first round's parents)."""
    ref = Refiner(kb, rng)
    parents = list(start)
    pcounts = (np.zeros((len(parents), 2), dtype=np.int64) if start_counts is None
               else np.asarray(start_counts, dtype=np.int64).reshape(len(parents), 2))
    for r in range(rounds):
        per_parent = max(1, per_round // max(1, len(parents)))
        cands = []
        pidx = []
        seen = set()
        for pi, p in enumerate(parents):
            for c in ref.refine(p, per_parent):
                if c not in seen:
                    seen.add(c)
                    cands.append(c)
                    pidx.append(pi)
        # top up with added conjuncts (two at once once single ones run out);
        # a small KB may have fewer distinct candidates than asked for
        tries = 0
        while len(cands) < per_round and tries < 16 * per_round:
            tries += 1
            extra = (ref.conjunct(),) if tries < 2 * per_round else (ref.conjunct(), ref.conjunct())
            pi = int(rng.integers(0, len(parents)))
            c = ("and", parents[pi]) + extra
            if c not in seen:
                seen.add(c)
                cands.append(c)
                pidx.append(pi)
        cands = cands[:per_round]
        pidx = np.asarray(pidx[:per_round], dtype=np.int64)
        counts = evaluate(cands)
        if with_parents:
            yield r, cands, counts, list(parents), pidx, pcounts[pidx]
        else:
            yield r, cands, counts
        top = top_indices(counts, n_pos, late_beam if late_beam and r + 1 >= rounds // 2 else beam)
        parents = [cands[i] for i in top]
        pcounts = np.asarray(counts, dtype=np.int64)[top]


def recall_at(screened_top: Sequence[int], exhaustive_top: Sequence[int]) -> float:
    a, b = set(int(i) for i in screened_top), set(int(i) for i in exhaustive_top)
    return len(a & b) / max(1, len(b))


def sizes(hyps) -> List[int]:
    return [hyp_size(h) for h in hyps]
