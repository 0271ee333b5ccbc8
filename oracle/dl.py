"""Plain CPU oracle for exact ALCQI(D) hypothesis evaluation.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  The library's compute
path never calls it, and it shares no code with the HIP path: it reads the
seeded input arrays and nothing else.

What it computes is the plain set semantics of the description-logic
constructs that HT-HEDL (Algahtani, "HT-HEDL: High-Throughput Hypothesis
Evaluation in Description Logic") evaluates, under the closed-world and
unique-name assumptions of its knowledge representation (Section 3.1).  Every
sub-result is a full membership vector over all N individuals; a hypothesis is
evaluated recursively, with no plan, no sharing and no reordering.

Readings of the paper taken here (each also listed in the design notes):

* at-most n is the textbook one, {x : cnt(x) <= n}, so individuals with no
  matching successor belong to it (the paper's filter in Algorithm 7 adds a
  cnt > 0 guard; that variant equals (<= n r.C) and (exists r.C));
* a role is a set of assertions, so counting assertions (Algorithms 7/8) and
  counting distinct successors agree;
* empty conjunction = top, empty disjunction = bottom; >= 0 r.C = top;
* a numeric restriction holds when the individual has a value and the float32
  comparison holds (existential concrete-role semantics of Section 3.2.3);
  a missing value (NaN) satisfies neither >= t nor <= t nor == t;
* a multi-valued numeric concrete role (Section 3.1: a subject may hold many
  assertions of one concrete role) gives x to its restriction when some value
  of x passes the comparison (MIN >=, MAX <=, EXACT ==, Algorithms 9/10); an
  individual without values of that role passes none;
* string concrete roles work the same way over strings: EQUAL holds when some
  value of x is the query string, CONTAIN when some value has the pattern as
  a substring (Algorithms 11-14; the empty pattern is a substring of every
  string); a query string absent from the knowledge base's strings matches
  nothing (the short-circuit of Algorithms 11/12);
* the inverse role swaps the subject and object of every assertion
  (end of Section 3.2.2).

Parity status: every function here is pinned by the CPU test suite against
brute-force first-order evaluation on tiny knowledge bases, a dense-adjacency
closed form, an SQLite translation and algebraic invariants.
"""
from __future__ import annotations

from typing import Dict, Iterable, List, Sequence, Tuple

import numpy as np


class Oracle:
    """Set-based evaluator over one knowledge base.

    ``kb`` needs the attributes ``n``, ``concept_bits`` (uint64 [C][W]),
    ``role_offsets`` (int64 [R][N+1], absolute), ``role_targets`` (int32 [E]),
    ``data`` (float32 [D][N]), ``pos_bits`` and ``neg_bits`` (uint64 [W]);
    optionally ``num_offsets`` (int64 [P][N+1], absolute) and ``num_values``
    (float32 [V]) for multi-valued numeric concrete roles, and ``str_offsets``
    (int64 [Q][N+1]), ``str_ids`` (int32 [V']) and ``strings`` (list of bytes:
    the distinct strings, indexed by id) for string concrete roles.
    """

    def __init__(self, kb):
        self.n = int(kb.n)
        self._cbits = np.asarray(kb.concept_bits, dtype=np.uint64)
        self._off = np.asarray(kb.role_offsets, dtype=np.int64)
        self._tg = np.asarray(kb.role_targets, dtype=np.int64)
        self._data = np.asarray(kb.data, dtype=np.float32)
        no = getattr(kb, "num_offsets", None)
        self._noff = np.zeros((0, self.n + 1), np.int64) if no is None else np.asarray(no, dtype=np.int64)
        nv = getattr(kb, "num_values", None)
        self._nval = np.zeros(0, np.float32) if nv is None else np.asarray(nv, dtype=np.float32)
        so = getattr(kb, "str_offsets", None)
        self._soff = np.zeros((0, self.n + 1), np.int64) if so is None else np.asarray(so, dtype=np.int64)
        si = getattr(kb, "str_ids", None)
        self._sids = np.zeros(0, np.int64) if si is None else np.asarray(si, dtype=np.int64)
        self._strings = list(getattr(kb, "strings", None) or [])
        self.pos = self._unpack(np.asarray(kb.pos_bits, dtype=np.uint64))
        self.neg = self._unpack(np.asarray(kb.neg_bits, dtype=np.uint64))
        self._edges: Dict[int, Tuple[np.ndarray, np.ndarray]] = {}
        self._atoms: Dict[int, np.ndarray] = {}

    # -- input decoding -----------------------------------------------------

    def _unpack(self, words: np.ndarray) -> np.ndarray:
        """Bit row -> bool [N] (individual i = bit i%64 of word i//64)."""
        b = np.unpackbits(words.view(np.uint8), bitorder="little")
        return b[: self.n].astype(bool)

    def member(self, a: int) -> np.ndarray:
        """Membership of atomic concept a: one row of the transposed concepts
        matrix (Section 3.1)."""
        m = self._atoms.get(a)
        if m is None:
            m = self._unpack(self._cbits[a])
            if len(self._atoms) < 4096:
                self._atoms[a] = m
        return m

    def assertions(self, r: int) -> Tuple[np.ndarray, np.ndarray]:
        """All (subject, object) assertions of role r, from its CSR rows."""
        e = self._edges.get(r)
        if e is None:
            off = self._off[r]
            lo, hi = int(off[0]), int(off[-1])
            subj = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(off))
            obj = self._tg[lo:hi]
            e = (subj, obj)
            self._edges[r] = e
        return e

    # -- role restrictions (Section 3.2.2, Algorithms 3-8) ----------------

    def count(self, r: int, inv: int, c: np.ndarray) -> np.ndarray:
        """cnt(x) = number of assertions (x, y) of the role (or of its inverse,
        subject and object swapped) whose object y is in c."""
        subj, obj = self.assertions(r)
        if inv:
            subj, obj = obj, subj
        return np.bincount(subj[c[obj]], minlength=self.n)

    # -- concrete roles (Section 3.2.3, Algorithms 9/10) -------------------

    def data_ge(self, p: int, t: float) -> np.ndarray:
        return self._data[p] >= np.float32(t)

    def data_le(self, p: int, t: float) -> np.ndarray:
        return self._data[p] <= np.float32(t)

    def data_eq(self, p: int, t: float) -> np.ndarray:
        return self._data[p] == np.float32(t)

    def num_values(self, p: int) -> Tuple[np.ndarray, np.ndarray]:
        """(subject, value) of every assertion of numeric concrete role p."""
        off = self._noff[p]
        subj = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(off))
        return subj, self._nval[int(off[0]):int(off[-1])]

    def num_some(self, p: int, cmp: str, t: float) -> np.ndarray:
        """{x : some value v of x in role p with v cmp t}, cmp in ge / le / eq."""
        subj, val = self.num_values(p)
        t = np.float32(t)
        ok = val >= t if cmp == "ge" else val <= t if cmp == "le" else val == t
        out = np.zeros(self.n, dtype=bool)
        out[subj[ok]] = True
        return out

    def str_values(self, p: int) -> Tuple[np.ndarray, List[bytes]]:
        """(subject, string) of every assertion of string concrete role p."""
        off = self._soff[p]
        subj = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(off))
        ids = self._sids[int(off[0]):int(off[-1])]
        return subj, [self._strings[i] for i in ids]

    def str_some(self, p: int, test) -> np.ndarray:
        """{x : some string value s of x in role p with test(s)}."""
        subj, vals = self.str_values(p)
        out = np.zeros(self.n, dtype=bool)
        for x, v in zip(subj.tolist(), vals):
            if test(v):
                out[x] = True
        return out

    # -- recursive evaluation ---------------------------------------------

    def ext(self, h) -> np.ndarray:
        """Instance set of hypothesis h as bool [N]."""
        op = h[0]
        n = self.n
        if op == "top":
            return np.ones(n, dtype=bool)
        if op == "bot":
            return np.zeros(n, dtype=bool)
        if op == "atom":
            return self.member(h[1]).copy()
        if op == "not":                                   # complement in the domain (CWA)
            return ~self.ext(h[1])
        if op == "and":                                   # Algorithms 1/2, n-ary
            out = np.ones(n, dtype=bool)
            for c in h[1:]:
                out &= self.ext(c)
            return out
        if op == "or":
            out = np.zeros(n, dtype=bool)
            for c in h[1:]:
                out |= self.ext(c)
            return out
        if op == "exists":                                # Algorithms 3/4
            _, r, inv, c = h
            return self.count(r, inv, self.ext(c)) >= 1
        if op == "forall":                                # Algorithms 5/6: no successor outside C
            _, r, inv, c = h
            return self.count(r, inv, ~self.ext(c)) == 0
        if op in ("atleast", "atmost", "exactly"):        # Algorithms 7/8
            _, k, r, inv, c = h
            cnt = self.count(r, inv, self.ext(c))
            if op == "atleast":
                return cnt >= k
            if op == "atmost":
                return cnt <= k
            return cnt == k
        if op == "dge":
            return self.data_ge(h[1], h[2])
        if op == "dle":
            return self.data_le(h[1], h[2])
        if op == "deq":
            return self.data_eq(h[1], h[2])
        if op in ("nge", "nle", "neq"):
            return self.num_some(h[1], op[1:], h[2])
        if op == "sequal":                                # Algorithms 11/12
            q = bytes(h[2])
            return self.str_some(h[1], lambda v: v == q)
        if op == "scontains":                             # Algorithms 13/14
            q = bytes(h[2])
            return self.str_some(h[1], lambda v: q in v)
        raise ValueError(f"unknown construct {op!r}")

    def coverage(self, h) -> Tuple[int, int]:
        """(covered positives, covered negatives) -- Algorithm 15."""
        e = self.ext(h)
        return int(np.count_nonzero(e & self.pos)), int(np.count_nonzero(e & self.neg))

    def coverages(self, hyps: Iterable) -> np.ndarray:
        """uint32 [H][2] coverage of every hypothesis."""
        out = [self.coverage(h) for h in hyps]
        return np.asarray(out, dtype=np.uint32).reshape(-1, 2)

    def ext_bits(self, h) -> np.ndarray:
        """Instance set packed as uint64 words (LSB first, zero padding)."""
        e = self.ext(h)
        w = (self.n + 63) // 64
        buf = np.zeros(w * 64, dtype=bool)
        buf[: self.n] = e
        return np.packbits(buf, bitorder="little").view(np.uint64).copy()


def f1_score(pos: int, neg: int, n_pos: int) -> Tuple[int, int]:
    """F1 = 2TP / (2TP + FP + FN) as an exact fraction (numerator, denominator),
    with TP = pos, FP = neg, FN = n_pos - pos; 0/1 when the denominator is 0."""
    num = 2 * pos
    den = 2 * pos + neg + (n_pos - pos)
    return (0, 1) if den == 0 else (num, den)
