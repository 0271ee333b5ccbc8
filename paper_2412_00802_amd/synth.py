"""Seeded synthetic inputs: knowledge bases, example sets and hypotheses.

This module only draws random inputs.  It evaluates no description-logic
construct: it never computes the instance set of a concept expression.  Both
the HIP path and the CPU oracle receive exactly the arrays produced here.

Shapes follow the paper's workloads (all synthetic, Section 6) and the five
workload descriptions of this project:

* concept memberships are a random subsumption tree materialised as bit rows
  (the transposed concepts matrix of Section 3.1, one bit per individual);
* object roles are sets of (subject, object) assertions with Zipf-distributed
  out-degrees, stored as one CSR per role (offsets int64 [R][N+1], absolute
  into one int32 target array; targets strictly increasing inside a row, so a
  role is a set of assertions, never a multiset);
* numeric concrete roles are single-valued float32 columns, NaN = no value;
* positive and negative examples are two bit rows.

Bit layout everywhere: individual i is bit (i & 63) of uint64 word (i >> 6),
least significant bit first; bits past N are zero.

Hypotheses are nested tuples::

    ('top',) ('bot',) ('atom', a) ('not', C) ('and', C1, ...) ('or', C1, ...)
    ('exists', r, inv, C) ('forall', r, inv, C)
    ('atleast', n, r, inv, C) ('atmost', n, r, inv, C) ('exactly', n, r, inv, C)
    ('dge', p, t) ('dle', p, t)          # t is exactly representable in float32

``inv`` = 1 selects the inverse role r^-.
"""
from __future__ import annotations

import concurrent.futures as _cf
import dataclasses
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np

BASE_SEED = 241200802

# ---------------------------------------------------------------------------
# workload descriptions
# ---------------------------------------------------------------------------


@dataclasses.dataclass(frozen=True)
class KBConfig:
    name: str
    n_individuals: int
    n_concepts: int
    tree_depth: int
    n_roles: int
    zipf_s: float
    degree_cap: int
    n_data: int
    missing: float
    n_pos: int
    n_neg: int
    n_hyps: int
    hyp_depth: int
    # expected total edge count; None = every individual is a subject of every role
    total_edges: Optional[int] = None
    root_density: float = 0.3
    seed_index: int = 0
    examples: str = "uniform"      # "uniform" | "planted"

    @property
    def words(self) -> int:
        return (self.n_individuals + 63) // 64


CONFIGS = {
    # tiny plain one-at-a-time workload
    "c1": KBConfig("c1", 10_000, 64, 4, 8, 2.0, 64, 4, 0.20, 1_000, 1_000, 256, 4,
                   seed_index=1),
    # mid KB, plain vs batched
    "c2": KBConfig("c2", 1_000_000, 512, 6, 32, 1.8, 1024, 16, 0.10, 50_000, 50_000,
                   4096, 5, seed_index=2),
    # uneven batch (sparse roles: ~40M edges over 48 roles)
    "c3": KBConfig("c3", 4_000_000, 1024, 6, 48, 1.6, 8192, 32, 0.10, 200_000, 200_000,
                   65_536, 5, total_edges=40_000_000, seed_index=3, examples="planted"),
    # refinement trace at large scale (16 rounds x 16,384 candidates)
    "c4": KBConfig("c4", 32_000_000, 1024, 6, 64, 1.5, 65_536, 128, 0.10, 1_000_000, 1_000_000,
                   16_384, 2, total_edges=500_000_000, seed_index=4, examples="planted"),
}


def small_config(n=300, n_concepts=12, depth=3, n_roles=3, s=1.5, cap=12, n_data=2,
                 missing=0.2, n_pos=40, n_neg=40, n_hyps=64, hyp_depth=4, seed_index=100,
                 total_edges=None) -> KBConfig:
    """A small workload of the same shape, for tests."""
    return KBConfig(f"small{seed_index}", n, n_concepts, depth, n_roles, s, cap, n_data,
                    missing, n_pos, n_neg, n_hyps, hyp_depth, total_edges=total_edges,
                    seed_index=seed_index)


# ---------------------------------------------------------------------------
# knowledge base container
# ---------------------------------------------------------------------------


@dataclasses.dataclass
class KB:
    n: int                       # individuals
    concept_bits: np.ndarray     # uint64 [C][W]
    role_offsets: np.ndarray     # int64 [R][N+1], absolute into role_targets
    role_targets: np.ndarray     # int32 [E]
    data: np.ndarray             # float32 [D][N], NaN = missing
    pos_bits: np.ndarray         # uint64 [W]
    neg_bits: np.ndarray         # uint64 [W]
    concept_parent: np.ndarray   # int32 [C], -1 for roots
    concept_level: np.ndarray    # int32 [C]
    deciles: np.ndarray          # float32 [D][9]
    # multi-valued numeric concrete roles (optional)
    num_offsets: Optional[np.ndarray] = None   # int64 [P][N+1], absolute into num_values
    num_values: Optional[np.ndarray] = None    # float32 [V]
    # string concrete roles (optional): values are ids into `strings`
    str_offsets: Optional[np.ndarray] = None   # int64 [Q][N+1], absolute into str_ids
    str_ids: Optional[np.ndarray] = None       # int32 [V']
    strings: Optional[List[bytes]] = None      # the distinct strings

    @property
    def words(self) -> int:
        return (self.n + 63) // 64

    @property
    def n_concepts(self) -> int:
        return int(self.concept_bits.shape[0])

    @property
    def n_roles(self) -> int:
        return int(self.role_offsets.shape[0])

    @property
    def n_data(self) -> int:
        return int(self.data.shape[0])

    @property
    def n_edges(self) -> int:
        return int(self.role_targets.shape[0])


# ---------------------------------------------------------------------------
# helpers
# ---------------------------------------------------------------------------


def pack_bits(mask: np.ndarray) -> np.ndarray:
    """bool [N] -> uint64 [ceil(N/64)], LSB-first."""
    n = mask.shape[0]
    w = (n + 63) // 64
    buf = np.zeros(w * 64, dtype=bool)
    buf[:n] = mask
    return np.packbits(buf, bitorder="little").view(np.uint64).copy()


def ids_to_bits(ids: np.ndarray, n: int) -> np.ndarray:
    m = np.zeros(n, dtype=bool)
    m[ids] = True
    return pack_bits(m)


def _tail_mask(n: int) -> np.uint64:
    r = n & 63
    return np.uint64((1 << r) - 1) if r else np.uint64(0xFFFFFFFFFFFFFFFF)


def zipf_table(s: float, cap: int) -> np.ndarray:
    """CDF of the Zipf(s) law truncated to 1..cap (renormalised)."""
    d = np.arange(1, cap + 1, dtype=np.float64)
    p = d ** (-s)
    c = np.cumsum(p)
    return c / c[-1]


def zipf_mean(s: float, cap: int) -> float:
    d = np.arange(1, cap + 1, dtype=np.float64)
    p = d ** (-s)
    return float((d * p).sum() / p.sum())


def _streams(cfg: KBConfig, k: int = 6) -> List[np.random.SeedSequence]:
    return np.random.SeedSequence(BASE_SEED + cfg.seed_index).spawn(k)


# ---------------------------------------------------------------------------
# concepts: random subsumption tree
# ---------------------------------------------------------------------------


def _gen_concepts(cfg: KBConfig, ss: np.random.SeedSequence, workers: int = 1):
    """Levels of equal size; a root-level concept holds each individual with
    probability root_density, a deeper concept keeps each member of a uniform
    parent on the level above with probability 1/2.  The tree comes from one
    stream, each concept's row from a stream of its own (rows of one level are
    drawn in parallel)."""
    tree_ss, row_ss = ss.spawn(2)
    rng = np.random.default_rng(tree_ss)
    n, c, depth = cfg.n_individuals, cfg.n_concepts, cfg.tree_depth
    w = cfg.words
    sizes = [c // depth] * depth
    for i in range(c % depth):
        sizes[i] += 1
    bits = np.zeros((c, w), dtype=np.uint64)
    parent = np.full(c, -1, dtype=np.int32)
    level = np.zeros(c, dtype=np.int32)
    tail = _tail_mask(n)
    streams = row_ss.spawn(c)
    start = 0
    prev = None
    for lv, sz in enumerate(sizes):
        ids = np.arange(start, start + sz)
        level[ids] = lv
        if lv:
            parent[ids] = prev[rng.integers(0, len(prev), size=sz)]

        def row(cid):
            r = np.random.default_rng(streams[cid])
            if parent[cid] < 0:
                out = pack_bits(r.random(n, dtype=np.float32) < cfg.root_density)
            else:
                out = bits[parent[cid]] & r.bit_generator.random_raw(w).astype(np.uint64)
            out[-1] &= tail
            bits[cid] = out

        with _cf.ThreadPoolExecutor(max_workers=workers) as ex:
            list(ex.map(row, ids.tolist()))
        prev = ids
        start += sz
    return bits, parent, level


# ---------------------------------------------------------------------------
# roles: Zipf out-degrees, uniform targets without replacement
# ---------------------------------------------------------------------------


def _subject_probability(cfg: KBConfig) -> float:
    if cfg.total_edges is None:
        return 1.0
    mean = zipf_mean(cfg.zipf_s, cfg.degree_cap)
    p = cfg.total_edges / (cfg.n_roles * cfg.n_individuals * mean)
    return float(min(1.0, p))


def _gen_role(n: int, cdf: np.ndarray, p_subj: float, ss: np.random.SeedSequence):
    """Return (degrees int64 [N], sorted targets int32 [E]) for one role."""
    rng = np.random.default_rng(ss)
    u = rng.random(n)
    deg = np.searchsorted(cdf, u, side="right").astype(np.int64) + 1
    np.minimum(deg, len(cdf), out=deg)
    if p_subj < 1.0:
        subj = rng.random(n) < p_subj
        deg[~subj] = 0
    off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(deg, out=off[1:])
    e = int(off[-1])
    tg = np.empty(e, dtype=np.int32)
    order = np.argsort(deg, kind="stable")
    sdeg = deg[order]
    bounds = np.flatnonzero(np.diff(sdeg)) + 1
    starts = np.concatenate(([0], bounds))
    ends = np.concatenate((bounds, [n]))
    for a, b in zip(starts, ends):
        dv = int(sdeg[a])
        if dv == 0:
            continue
        rows = order[a:b]
        if dv * dv > n // 5:
            # heavy rows: exact sampling without replacement row by row
            for x in rows:
                t = np.sort(rng.choice(n, size=dv, replace=False)).astype(np.int32)
                tg[off[x]:off[x] + dv] = t
            continue
        m = rng.integers(0, n, size=(rows.shape[0], dv), dtype=np.int32)
        m.sort(axis=1)
        if dv > 1:
            bad = np.flatnonzero((m[:, 1:] == m[:, :-1]).any(axis=1))
            while bad.size:
                r2 = rng.integers(0, n, size=(bad.shape[0], dv), dtype=np.int32)
                r2.sort(axis=1)
                m[bad] = r2
                still = (r2[:, 1:] == r2[:, :-1]).any(axis=1)
                bad = bad[still]
        pos = off[rows][:, None] + np.arange(dv, dtype=np.int64)[None, :]
        tg[pos] = m
    return deg, tg


def _gen_roles(cfg: KBConfig, ss: np.random.SeedSequence, workers: int):
    n, r = cfg.n_individuals, cfg.n_roles
    cdf = zipf_table(cfg.zipf_s, cfg.degree_cap)
    p = _subject_probability(cfg)
    subs = ss.spawn(r)
    with _cf.ThreadPoolExecutor(max_workers=workers) as ex:
        res = list(ex.map(lambda i: _gen_role(n, cdf, p, subs[i]), range(r)))
    counts = np.array([int(d.sum()) for d, _ in res], dtype=np.int64)
    base = np.zeros(r + 1, dtype=np.int64)
    np.cumsum(counts, out=base[1:])
    offsets = np.empty((r, n + 1), dtype=np.int64)
    targets = np.empty(int(base[-1]), dtype=np.int32)
    for i, (deg, tg) in enumerate(res):
        offsets[i, 0] = base[i]
        np.cumsum(deg, out=offsets[i, 1:])
        offsets[i, 1:] += base[i]
        targets[base[i]:base[i + 1]] = tg
    return offsets, targets


# ---------------------------------------------------------------------------
# data properties and examples
# ---------------------------------------------------------------------------


def _gen_data(cfg: KBConfig, ss: np.random.SeedSequence, workers: int = 1):
    """float32 N(0,1) columns, a Bernoulli(missing) share set to NaN, one
    stream per property (columns drawn in parallel); deciles as the order
    statistics t_k = v_((k (m-1)) // 10) of the m defined values."""
    n, d = cfg.n_individuals, cfg.n_data
    cols = np.empty((d, n), dtype=np.float32)
    dec = np.zeros((d, 9), dtype=np.float32)
    streams = ss.spawn(d)

    def column(j):
        rng = np.random.default_rng(streams[j])
        col = rng.standard_normal(n, dtype=np.float32)
        col[rng.random(n, dtype=np.float32) < cfg.missing] = np.nan
        cols[j] = col
        vals = col[~np.isnan(col)]
        m = vals.shape[0]
        if m:
            kth = [(k * (m - 1)) // 10 for k in range(1, 10)]
            dec[j] = np.partition(vals, kth)[kth]

    with _cf.ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(column, range(d)))
    return cols, dec


def _gen_examples_uniform(cfg: KBConfig, ss: np.random.SeedSequence):
    rng = np.random.default_rng(ss)
    idx = rng.choice(cfg.n_individuals, size=cfg.n_pos + cfg.n_neg, replace=False)
    return (ids_to_bits(idx[:cfg.n_pos], cfg.n_individuals),
            ids_to_bits(idx[cfg.n_pos:], cfg.n_individuals))


def _gen_examples_planted(cfg: KBConfig, ss: np.random.SeedSequence, concept_bits,
                          concept_level):
    """Positives mostly drawn from the members of one root concept (a planted
    target read straight from the input rows), negatives mostly from the
    non-members, with 5% of each swapped for the other side (label noise)."""
    rng = np.random.default_rng(ss)
    n = cfg.n_individuals
    roots = np.flatnonzero(concept_level == 0)
    a = int(roots[rng.integers(0, roots.shape[0])])
    member = np.unpackbits(concept_bits[a].view(np.uint8), bitorder="little")[:n].astype(bool)
    ins = np.flatnonzero(member)
    outs = np.flatnonzero(~member)
    npn, nnn = int(round(cfg.n_pos * 0.05)), int(round(cfg.n_neg * 0.05))
    pa = rng.choice(ins, size=cfg.n_pos - npn, replace=False)
    na = rng.choice(outs, size=cfg.n_neg - nnn, replace=False)
    rest_out = np.setdiff1d(outs, na, assume_unique=True)
    rest_in = np.setdiff1d(ins, pa, assume_unique=True)
    pb = rng.choice(rest_out, size=npn, replace=False)
    nb = rng.choice(rest_in, size=nnn, replace=False)
    return (ids_to_bits(np.concatenate([pa, pb]), n), ids_to_bits(np.concatenate([na, nb]), n))


def make_kb(cfg: KBConfig, workers: Optional[int] = None, log=None) -> KB:
    """Build the seeded knowledge base of a workload (log: optional progress
    callback, called after each stage)."""
    if workers is None:
        workers = max(1, min(16, os.cpu_count() or 1))
    say = log or (lambda *_: None)
    s_con, s_role, s_data, s_ex, _s_hyp, _s_trace = _streams(cfg)
    bits, parent, level = _gen_concepts(cfg, s_con, workers)
    say(f"concepts: {cfg.n_concepts} rows")
    offsets, targets = _gen_roles(cfg, s_role, workers)
    say(f"roles: {targets.shape[0]:,} assertions")
    cols, dec = _gen_data(cfg, s_data, workers)
    say(f"data: {cfg.n_data} columns")
    if cfg.examples == "planted":
        pos, neg = _gen_examples_planted(cfg, s_ex, bits, level)
    else:
        pos, neg = _gen_examples_uniform(cfg, s_ex)
    return KB(cfg.n_individuals, bits, offsets, targets, cols, pos, neg, parent, level, dec)


# ---------------------------------------------------------------------------
# random hypotheses
# ---------------------------------------------------------------------------

_OPS = ("and", "or", "not", "exists", "forall", "atleast", "atmost")


class _HypGen:
    def __init__(self, rng: np.random.Generator, n_concepts, n_roles, n_data, deciles,
                 p_leaf=0.3, ops: Sequence[str] = _OPS, max_n: int = 4, p_inv=0.5):
        self.rng = rng
        self.nc, self.nr, self.nd = n_concepts, n_roles, n_data
        self.dec = deciles
        self.p_leaf = p_leaf
        self.ops = tuple(ops)
        self.max_n = max_n
        self.p_inv = p_inv

    def leaf(self):
        u = self.rng.random()
        if u < 0.75 or self.nd == 0:
            if u >= 0.95 and self.nd == 0:
                return ("top",)
            return ("atom", int(self.rng.integers(0, self.nc)))
        if u < 0.95:
            p = int(self.rng.integers(0, self.nd))
            k = int(self.rng.integers(0, 9))
            t = float(self.dec[p, k])
            return ("dge" if self.rng.random() < 0.5 else "dle", p, t)
        return ("top",)

    def tree(self, depth: int, root: bool = False):
        if depth <= 1 or (not root and self.rng.random() < self.p_leaf):
            return self.leaf()
        op = self.ops[int(self.rng.integers(0, len(self.ops)))]
        if op in ("and", "or"):
            k = 2 + int(self.rng.integers(0, 2))
            return (op,) + tuple(self.tree(depth - 1) for _ in range(k))
        if op == "not":
            return ("not", self.tree(depth - 1))
        r = int(self.rng.integers(0, self.nr))
        inv = int(self.rng.random() < self.p_inv)
        if op in ("exists", "forall"):
            return (op, r, inv, self.tree(depth - 1))
        n = 1 + int(self.rng.integers(0, self.max_n))
        return (op, n, r, inv, self.tree(depth - 1))


def make_hypotheses(cfg: KBConfig, kb: KB, count: Optional[int] = None,
                    depth: Optional[int] = None, stream: int = 4, **kw) -> List[tuple]:
    """Random hypotheses of syntax-tree depth <= depth (leaf depth = 1).

    The root is always an operator; every other position is a leaf with
    probability 0.3.  Leaves: atom 0.75, data threshold 0.2 (>= or <= at one of
    the nine property deciles), top 0.05.  Operators uniform over
    and/or/not/exists/forall/atleast/atmost, and/or of arity 2 or 3, role
    uniform, inverse with probability 0.5, n uniform on 1..4.
    """
    ss = _streams(cfg)[stream]
    rng = np.random.default_rng(ss)
    g = _HypGen(rng, kb.n_concepts, kb.n_roles, kb.n_data, kb.deciles, **kw)
    count = cfg.n_hyps if count is None else count
    depth = cfg.hyp_depth if depth is None else depth
    return [g.tree(depth, root=True) for _ in range(count)]


class _SizedGen(_HypGen):
    """Trees of an exact node count; children are drawn from a pool of earlier
    subtrees of the same size with probability p_share."""

    def __init__(self, *a, p_share=0.3, pool_size=4096, **kw):
        super().__init__(*a, **kw)
        self.p_share = p_share
        self.pool_size = pool_size
        self.pool = {}          # size -> list of subtrees (ring buffers)
        self.pool_n = 0

    def _remember(self, t, k):
        lst = self.pool.setdefault(k, [])
        if self.pool_n < self.pool_size:
            lst.append(t)
            self.pool_n += 1
        elif lst:
            lst[int(self.rng.integers(0, len(lst)))] = t

    def child(self, k):
        lst = self.pool.get(k)
        if lst and self.rng.random() < self.p_share:
            return lst[int(self.rng.integers(0, len(lst)))]
        return self.sized(k)

    def sized(self, k):
        if k == 1:
            t = self.leaf()
        elif k == 2:
            t = self._unary(self.child(1))
        else:
            op = self.ops[int(self.rng.integers(0, len(self.ops)))]
            if op in ("and", "or"):
                a = min(k - 1, 2 + int(self.rng.integers(0, 2)))
                cuts = np.sort(self.rng.choice(np.arange(1, k - 1), size=a - 1, replace=False))
                parts = np.diff(np.concatenate(([0], cuts, [k - 1]))).tolist()
                t = (op,) + tuple(self.child(int(p)) for p in parts)
            else:
                t = self._unary(self.child(k - 1), op)
        self._remember(t, k)
        return t

    def _unary(self, c, op=None):
        if op is None or op in ("and", "or"):
            op = ("not", "exists", "forall", "atleast", "atmost")[int(self.rng.integers(0, 5))]
        if op == "not":
            return ("not", c)
        r = int(self.rng.integers(0, self.nr))
        inv = int(self.rng.random() < self.p_inv)
        if op in ("exists", "forall"):
            return (op, r, inv, c)
        return (op, 1 + int(self.rng.integers(0, self.max_n)), r, inv, c)


def make_sized_hypotheses(cfg: KBConfig, kb: KB, count: Optional[int] = None, p_geo: float = 0.15,
                          max_nodes: int = 31, p_share: float = 0.3, stream: int = 4) -> List[tuple]:
    """The uneven-batch workload: node counts geometric(p_geo) truncated to
    1..max_nodes by rejection, trees grown to exactly that many nodes, each
    child subtree drawn from a pool of 4,096 earlier subtrees of the same size
    with probability p_share (shared subexpressions across the batch)."""
    ss = _streams(cfg)[stream]
    rng = np.random.default_rng(ss)
    g = _SizedGen(rng, kb.n_concepts, kb.n_roles, kb.n_data, kb.deciles, p_share=p_share)
    count = cfg.n_hyps if count is None else count
    out = []
    while len(out) < count:
        k = int(rng.geometric(p_geo))
        if k > max_nodes:
            continue
        out.append(g.sized(k))
    return out


def hyp_depth(h) -> int:
    op = h[0]
    if op in ("top", "bot", "atom", "dge", "dle"):
        return 1
    if op == "not":
        return 1 + hyp_depth(h[1])
    if op in ("and", "or"):
        return 1 + max((hyp_depth(c) for c in h[1:]), default=0)
    return 1 + hyp_depth(h[-1])


def hyp_size(h) -> int:
    op = h[0]
    if op in ("top", "bot", "atom", "dge", "dle", "set"):
        return 1
    if op == "not":
        return 1 + hyp_size(h[1])
    if op in ("and", "or"):
        return 1 + sum(hyp_size(c) for c in h[1:])
    return 1 + hyp_size(h[-1])


def numeric_roles(n: int, n_roles: int, seed: int, p_subj: float = 0.5, zipf_s: float = 1.6,
                  cap: int = 64, step: float = 1.0 / 16) -> Tuple[np.ndarray, np.ndarray]:
    """Multi-valued numeric concrete roles: each individual is a subject of a
    role with probability p_subj, with a Zipf(zipf_s) number of values capped
    at cap; values ~ N(0, 1) rounded to multiples of `step` (so that equal
    values, and EXACT matches, occur).  -> (offsets int64 [R][N+1], values
    float32 [V]), roles stored one after the other."""
    rng = np.random.default_rng(seed)
    pmf = 1.0 / np.arange(1, cap + 1, dtype=np.float64) ** zipf_s
    pmf /= pmf.sum()
    offs = np.zeros((n_roles, n + 1), dtype=np.int64)
    vals = []
    base = 0
    for r in range(n_roles):
        subj = rng.random(n) < p_subj
        deg = np.where(subj, rng.choice(np.arange(1, cap + 1), size=n, p=pmf), 0).astype(np.int64)
        offs[r, 0] = base
        offs[r, 1:] = base + np.cumsum(deg)
        v = np.round(rng.standard_normal(int(deg.sum())) / step) * step
        vals.append(v.astype(np.float32))
        base += int(deg.sum())
    return offs, (np.concatenate(vals) if vals else np.zeros(0, np.float32))


def with_numeric_roles(kb: KB, offsets: np.ndarray, values: np.ndarray) -> KB:
    """The same KB with multi-valued numeric concrete roles attached."""
    import dataclasses
    return dataclasses.replace(kb, num_offsets=np.asarray(offsets, dtype=np.int64),
                               num_values=np.asarray(values, dtype=np.float32))


def string_roles(n: int, n_roles: int, seed: int, n_strings: int = 2000, p_subj: float = 0.4,
                 zipf_s: float = 1.8, cap: int = 16, alphabet: bytes = b"abcdef",
                 max_len: int = 12) -> Tuple[np.ndarray, np.ndarray, List[bytes]]:
    """String concrete roles over a dictionary of n_strings distinct random
    words (lengths 1..max_len over a small alphabet, so that substrings
    recur): each individual is a subject with probability p_subj, with a
    Zipf number of values capped at cap, each a uniform dictionary id.
    -> (offsets int64 [R][N+1], ids int32 [V], strings)."""
    rng = np.random.default_rng(seed)
    seen = set()
    strings: List[bytes] = []
    while len(strings) < n_strings:
        k = int(rng.integers(1, max_len + 1))
        w = bytes(alphabet[int(i)] for i in rng.integers(0, len(alphabet), size=k))
        if w not in seen:
            seen.add(w)
            strings.append(w)
    pmf = 1.0 / np.arange(1, cap + 1, dtype=np.float64) ** zipf_s
    pmf /= pmf.sum()
    offs = np.zeros((n_roles, n + 1), dtype=np.int64)
    ids = []
    base = 0
    for r in range(n_roles):
        subj = rng.random(n) < p_subj
        deg = np.where(subj, rng.choice(np.arange(1, cap + 1), size=n, p=pmf), 0).astype(np.int64)
        offs[r, 0] = base
        offs[r, 1:] = base + np.cumsum(deg)
        ids.append(rng.integers(0, n_strings, size=int(deg.sum())).astype(np.int32))
        base += int(deg.sum())
    return offs, (np.concatenate(ids) if ids else np.zeros(0, np.int32)), strings


def with_string_roles(kb: KB, offsets: np.ndarray, ids: np.ndarray, strings: List[bytes]) -> KB:
    """The same KB with string concrete roles attached."""
    import dataclasses
    return dataclasses.replace(kb, str_offsets=np.asarray(offsets, dtype=np.int64),
                               str_ids=np.asarray(ids, dtype=np.int32), strings=list(strings))


def make_string_hypotheses(kb: KB, count: int, seed: int) -> List[tuple]:
    """EQUAL at dictionary strings and at absent ones; CONTAIN at short
    patterns (often substrings), the empty pattern and absent ones; alone and
    inside negations, conjunctions and role restrictions."""
    rng = np.random.default_rng(seed)
    Q = kb.str_offsets.shape[0]
    out: List[tuple] = []
    for _ in range(count):
        p = int(rng.integers(0, Q))
        u = rng.random()
        if u < 0.35:
            leaf = ("sequal", p, kb.strings[int(rng.integers(0, len(kb.strings)))])
        elif u < 0.4:
            leaf = ("sequal", p, b"zz" + bytes([97 + int(rng.integers(0, 6))]))
        elif u < 0.9:
            s = kb.strings[int(rng.integers(0, len(kb.strings)))]
            a = int(rng.integers(0, len(s)))
            leaf = ("scontains", p, s[a:a + int(rng.integers(1, 4))])
        elif u < 0.95:
            leaf = ("scontains", p, b"")
        else:
            leaf = ("scontains", p, b"fedcbafedcbafedcba")
        k = int(rng.integers(0, 4))
        if k == 0:
            out.append(leaf)
        elif k == 1:
            out.append(("not", leaf))
        elif k == 2:
            out.append(("and", leaf, ("atom", int(rng.integers(0, kb.n_concepts)))))
        else:
            out.append(("exists", int(rng.integers(0, kb.n_roles)), int(rng.integers(0, 2)), leaf)
                       if kb.n_roles else leaf)
    return out


def make_numeric_hypotheses(kb: KB, count: int, seed: int) -> List[tuple]:
    """Hypotheses over the numeric concrete roles: MIN / MAX / EXACT at
    values drawn from each role (ties and exact matches exercised), alone and
    inside conjunctions, negations and role restrictions."""
    rng = np.random.default_rng(seed)
    P = kb.num_offsets.shape[0]
    out: List[tuple] = []
    for _ in range(count):
        p = int(rng.integers(0, P))
        lo, hi = int(kb.num_offsets[p, 0]), int(kb.num_offsets[p, -1])
        t = float(kb.num_values[int(rng.integers(lo, hi))]) if hi > lo else float(rng.standard_normal())
        leaf = (["nge", "nle", "neq"][int(rng.integers(0, 3))], p, t)
        k = int(rng.integers(0, 5))
        if k == 0:
            out.append(leaf)
        elif k == 1:
            out.append(("not", leaf))
        elif k == 2:
            out.append(("and", leaf, ("atom", int(rng.integers(0, kb.n_concepts)))))
        elif k == 3 and kb.n_roles:
            out.append(("exists", int(rng.integers(0, kb.n_roles)), int(rng.integers(0, 2)), leaf))
        else:
            q = int(rng.integers(0, P))
            out.append(("or", leaf, ("neq", q, 0.0)))
    return out


def kb_from_edges(n: int, concept_sets: Sequence[Sequence[int]],
                  role_edges: Sequence[Sequence[Tuple[int, int]]],
                  data: Optional[np.ndarray] = None,
                  pos: Sequence[int] = (), neg: Sequence[int] = ()) -> KB:
    """Build a KB from explicit sets (hand-made test fixtures)."""
    w = (n + 63) // 64
    cb = np.zeros((len(concept_sets), w), dtype=np.uint64)
    for i, s in enumerate(concept_sets):
        cb[i] = ids_to_bits(np.asarray(sorted(set(s)), dtype=np.int64), n)
    r = len(role_edges)
    offsets = np.zeros((r, n + 1), dtype=np.int64)
    tgs = []
    base = 0
    for i, edges in enumerate(role_edges):
        es = sorted(set((int(a), int(b)) for a, b in edges))
        deg = np.zeros(n, dtype=np.int64)
        for a, _ in es:
            deg[a] += 1
        offsets[i, 0] = base
        offsets[i, 1:] = base + np.cumsum(deg)
        tgs.extend(b for _, b in es)
        base += len(es)
    targets = np.asarray(tgs, dtype=np.int32)
    if data is None:
        data = np.zeros((0, n), dtype=np.float32)
    data = np.asarray(data, dtype=np.float32)
    dec = np.zeros((data.shape[0], 9), dtype=np.float32)
    for j in range(data.shape[0]):
        vals = np.sort(data[j][~np.isnan(data[j])])
        if vals.shape[0]:
            for k in range(1, 10):
                dec[j, k - 1] = vals[(k * (vals.shape[0] - 1)) // 10]
    return KB(n, cb, offsets, targets, data,
              ids_to_bits(np.asarray(list(pos), dtype=np.int64), n),
              ids_to_bits(np.asarray(list(neg), dtype=np.int64), n),
              np.full(len(concept_sets), -1, dtype=np.int32),
              np.zeros(len(concept_sets), dtype=np.int32), dec)
