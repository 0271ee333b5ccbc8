"""Algebraic invariants of the semantics, checked on the oracle (property tests)."""
import numpy as np
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from oracle import Oracle
from paper_2412_00802_amd import synth

_KBS = {}


def _kb(seed):
    if seed not in _KBS:
        cfg = synth.small_config(n=150 + 37 * seed, n_concepts=12, n_roles=3, cap=10,
                                 seed_index=200 + seed)
        kb = synth.make_kb(cfg)
        _KBS[seed] = (kb, Oracle(kb))
    return _KBS[seed]


def _leaf():
    return st.one_of(
        st.builds(lambda a: ("atom", a), st.integers(0, 11)),
        st.builds(lambda p, k, g: (g, p, float(_kb(0)[0].deciles[p, k])),
                  st.integers(0, 1), st.integers(0, 8), st.sampled_from(["dge", "dle"])),
        st.just(("top",)), st.just(("bot",)))


def _concept(depth=3):
    if depth <= 1:
        return _leaf()
    sub = _concept(depth - 1)
    role = st.tuples(st.integers(0, 2), st.integers(0, 1))
    return st.one_of(
        _leaf(),
        st.builds(lambda c: ("not", c), sub),
        st.builds(lambda a, b: ("and", a, b), sub, sub),
        st.builds(lambda a, b: ("or", a, b), sub, sub),
        st.builds(lambda ri, c: ("exists", ri[0], ri[1], c), role, sub),
        st.builds(lambda ri, c: ("forall", ri[0], ri[1], c), role, sub),
        st.builds(lambda k, ri, c: ("atleast", k, ri[0], ri[1], c), st.integers(0, 4), role, sub),
        st.builds(lambda k, ri, c: ("atmost", k, ri[0], ri[1], c), st.integers(0, 4), role, sub))


SETTINGS = settings(max_examples=150, deadline=None, suppress_health_check=list(HealthCheck))
seeds = st.integers(0, 2)
roles = st.integers(0, 2)
invs = st.integers(0, 1)


def eq(o, a, b):
    np.testing.assert_array_equal(o.ext(a), o.ext(b))


def sub(o, a, b):
    ea, eb = o.ext(a), o.ext(b)
    assert not np.any(ea & ~eb), (a, b)


@SETTINGS
@given(seeds, _concept(), roles, invs)
def test_forall_is_not_exists_not(seed, c, r, inv):
    _, o = _kb(seed)
    eq(o, ("forall", r, inv, c), ("not", ("exists", r, inv, ("not", c))))


@SETTINGS
@given(seeds, _concept(), roles, invs, st.integers(0, 4))
def test_counting_identities(seed, c, r, inv, k):
    _, o = _kb(seed)
    eq(o, ("atleast", 1, r, inv, c), ("exists", r, inv, c))
    eq(o, ("atmost", k, r, inv, c), ("not", ("atleast", k + 1, r, inv, c)))
    eq(o, ("exactly", k, r, inv, c), ("and", ("atleast", k, r, inv, c), ("atmost", k, r, inv, c)))
    eq(o, ("atleast", 0, r, inv, c), ("top",))
    eq(o, ("atmost", 0, r, inv, c), ("not", ("exists", r, inv, c)))
    sub(o, ("atleast", k + 1, r, inv, c), ("atleast", k, r, inv, c))   # antitone in n
    sub(o, ("atmost", k, r, inv, c), ("atmost", k + 1, r, inv, c))


@SETTINGS
@given(seeds, _concept(), _concept(), roles, invs)
def test_boolean_and_distribution(seed, c, d, r, inv):
    _, o = _kb(seed)
    eq(o, ("not", ("and", c, d)), ("or", ("not", c), ("not", d)))
    eq(o, ("not", ("or", c, d)), ("and", ("not", c), ("not", d)))
    eq(o, ("not", ("not", c)), c)
    eq(o, ("or", c, ("not", c)), ("top",))
    eq(o, ("and", c, ("not", c)), ("bot",))
    eq(o, ("exists", r, inv, ("or", c, d)), ("or", ("exists", r, inv, c), ("exists", r, inv, d)))
    eq(o, ("forall", r, inv, ("and", c, d)), ("and", ("forall", r, inv, c), ("forall", r, inv, d)))
    eq(o, ("exists", r, inv, ("bot",)), ("bot",))
    eq(o, ("forall", r, inv, ("top",)), ("top",))
    # monotone in the filler
    sub(o, ("exists", r, inv, ("and", c, d)), ("exists", r, inv, c))
    sub(o, ("forall", r, inv, ("and", c, d)), ("forall", r, inv, c))
    sub(o, ("atmost", 1, r, inv, ("or", c, d)), ("atmost", 1, r, inv, c))


@SETTINGS
@given(seeds, _concept(), roles)
def test_inverse_role_symmetry(seed, c, r):
    _, o = _kb(seed)
    sub(o, c, ("forall", r, 0, ("exists", r, 1, c)))
    sub(o, ("exists", r, 0, ("forall", r, 1, c)), c)
    sub(o, c, ("forall", r, 1, ("exists", r, 0, c)))


@settings(max_examples=60, deadline=None, suppress_health_check=list(HealthCheck))
@given(seeds, st.integers(0, 11), st.integers(0, 11), roles)
def test_edge_count_identity(seed, a, b, r):
    """sum_n |ext(>=n r.B) & A| = #(r & A x B) = sum_n |ext(>=n r^-.A) & B|."""
    kb, o = _kb(seed)
    ma, mb = o.member(a), o.member(b)
    maxdeg = int(np.max(np.diff(kb.role_offsets[r]))) + int(kb.n)
    fwd = inv = 0
    n = 1
    while True:
        f = o.ext(("atleast", n, r, 0, ("atom", b))) & ma
        g = o.ext(("atleast", n, r, 1, ("atom", a))) & mb
        if not f.any() and not g.any():
            break
        fwd += int(f.sum())
        inv += int(g.sum())
        n += 1
        assert n < maxdeg
    off = kb.role_offsets[r]
    subj = np.repeat(np.arange(kb.n), np.diff(off))
    obj = kb.role_targets[off[0]:off[-1]]
    direct = int(np.sum(ma[subj] & mb[obj]))
    assert fwd == direct == inv


def test_subsumption_monotonicity():
    """A' child of A in the concept tree: ext(A') within ext(A), and every
    positive-polarity context preserves it, negative flips it."""
    kb, o = _kb(1)
    for child in np.flatnonzero(kb.concept_parent >= 0)[:6]:
        par = int(kb.concept_parent[child])
        c, p = ("atom", int(child)), ("atom", par)
        sub(o, c, p)
        for r in range(3):
            for inv in (0, 1):
                sub(o, ("exists", r, inv, c), ("exists", r, inv, p))
                sub(o, ("forall", r, inv, c), ("forall", r, inv, p))
                sub(o, ("atleast", 2, r, inv, c), ("atleast", 2, r, inv, p))
                sub(o, ("atmost", 1, r, inv, p), ("atmost", 1, r, inv, c))
                sub(o, ("not", p), ("not", c))


def test_data_threshold_properties():
    kb, o = _kb(2)
    col = kb.data[0]
    has = ~np.isnan(col)
    np.testing.assert_array_equal(o.ext(("dge", 0, float("-inf"))), has)
    np.testing.assert_array_equal(o.ext(("dle", 0, float("inf"))), has)
    prev = None
    for t in list(kb.deciles[0]) + [10.0]:
        cur = o.ext(("dge", 0, float(t)))
        if prev is not None:
            assert not np.any(cur & ~prev)
        prev = cur
        both = o.ext(("and", ("dge", 0, float(t)), ("dle", 0, float(t))))
        np.testing.assert_array_equal(both, has & (col == np.float32(t)))
    eq(o, ("or", ("dge", 0, 0.0), ("dle", 0, 0.0)), ("dge", 0, float("-inf")))


def test_coverage_identities():
    kb, o = _kb(0)
    npos, nneg = int(o.pos.sum()), int(o.neg.sum())
    assert o.coverage(("top",)) == (npos, nneg)
    assert o.coverage(("bot",)) == (0, 0)
    for h in synth.make_hypotheses(synth.small_config(n=150, n_concepts=12, n_roles=3,
                                                      seed_index=200), kb, count=40):
        p, q = o.coverage(h)
        pn, qn = o.coverage(("not", h))
        assert p + pn == npos and q + qn == nneg
        assert 0 <= p <= npos and 0 <= q <= nneg
