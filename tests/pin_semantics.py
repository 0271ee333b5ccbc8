"""Independent formulations of the semantics, used only to pin the oracle.

Three evaluators that share nothing with ``oracle.dl``:

* ``brute_ext``: first-order quantifiers over explicit Python sets,
  one individual at a time (only for tiny KBs);
* ``dense_counts``: the successor count as a dense adjacency matrix product,
  cnt = A_r @ 1_C (forward) or A_r^T @ 1_C (inverse);
* ``sql_ext``: the hypothesis compiled to SQL and run by SQLite (the
  relational evaluation of hypotheses mentioned in the paper's related work).
"""
from __future__ import annotations

import sqlite3
import struct

import numpy as np


def kb_sets(kb):
    """Decode a KB into Python sets: concepts, assertion sets, values."""
    n = kb.n
    concepts = []
    for row in kb.concept_bits:
        ids = set()
        for w, word in enumerate(row.tolist()):
            for b in range(64):
                if (word >> b) & 1:
                    ids.add(w * 64 + b)
        concepts.append(ids)
    roles = []
    for r in range(kb.role_offsets.shape[0]):
        off = kb.role_offsets[r]
        pairs = set()
        for x in range(n):
            for e in range(int(off[x]), int(off[x + 1])):
                pairs.add((x, int(kb.role_targets[e])))
        roles.append(pairs)
    values = []
    for p in range(kb.data.shape[0]):
        values.append({x: float(v) for x, v in enumerate(kb.data[p].tolist()) if v == v})
    return concepts, roles, values


def bits_to_set(words, n):
    out = set()
    for w, word in enumerate(np.asarray(words).tolist()):
        for b in range(64):
            if (word >> b) & 1 and w * 64 + b < n:
                out.add(w * 64 + b)
    return out


def _f32(t):
    return struct.unpack("f", struct.pack("f", t))[0]


def brute_ext(sets, n, h):
    """First-order evaluation: x is an instance iff the formula holds at x."""
    concepts, roles, values = sets
    dom = range(n)
    op = h[0]
    if op == "top":
        return set(dom)
    if op == "bot":
        return set()
    if op == "atom":
        return set(concepts[h[1]])
    if op == "not":
        inner = brute_ext(sets, n, h[1])
        return {x for x in dom if x not in inner}
    if op == "and":
        parts = [brute_ext(sets, n, c) for c in h[1:]]
        return {x for x in dom if all(x in p for p in parts)}
    if op == "or":
        parts = [brute_ext(sets, n, c) for c in h[1:]]
        return {x for x in dom if any(x in p for p in parts)}
    if op in ("exists", "forall", "atleast", "atmost", "exactly"):
        if op in ("exists", "forall"):
            _, r, inv, c = h
            k = None
        else:
            _, k, r, inv, c = h
        filler = brute_ext(sets, n, c)
        rel = roles[r]

        def succ(x):
            if inv:
                return [y for y in dom if (y, x) in rel]
            return [y for y in dom if (x, y) in rel]

        out = set()
        for x in dom:
            s = succ(x)
            m = sum(1 for y in s if y in filler)
            if op == "exists":
                ok = any(y in filler for y in s)
            elif op == "forall":
                ok = all(y in filler for y in s)
            elif op == "atleast":
                ok = m >= k
            elif op == "atmost":
                ok = m <= k
            else:
                ok = m == k
            if ok:
                out.add(x)
        return out
    if op in ("dge", "dle"):
        _, p, t = h
        t = _f32(t)
        vals = values[p]
        if op == "dge":
            return {x for x, v in vals.items() if v >= t}
        return {x for x, v in vals.items() if v <= t}
    raise ValueError(op)


def dense_adjacency(kb, r):
    n = kb.n
    a = np.zeros((n, n), dtype=np.int64)
    off = kb.role_offsets[r]
    for x in range(n):
        for e in range(int(off[x]), int(off[x + 1])):
            a[x, int(kb.role_targets[e])] = 1
    return a


def dense_counts(kb, r, inv, member):
    a = dense_adjacency(kb, r)
    if inv:
        a = a.T
    return a @ member.astype(np.int64)


class SqlKB:
    """The KB as four relations: ind(x), mem(c, x), edge(r, s, o), val(p, x, v)."""

    def __init__(self, kb):
        self.n = kb.n
        db = sqlite3.connect(":memory:")
        db.execute("CREATE TABLE ind(x INTEGER PRIMARY KEY)")
        db.execute("CREATE TABLE mem(c INTEGER, x INTEGER)")
        db.execute("CREATE TABLE edge(r INTEGER, s INTEGER, o INTEGER)")
        db.execute("CREATE TABLE val(p INTEGER, x INTEGER, v REAL)")
        db.executemany("INSERT INTO ind VALUES (?)", [(x,) for x in range(kb.n)])
        concepts, roles, values = kb_sets(kb)
        db.executemany("INSERT INTO mem VALUES (?, ?)",
                       [(c, x) for c, s in enumerate(concepts) for x in s])
        db.executemany("INSERT INTO edge VALUES (?, ?, ?)",
                       [(r, s, o) for r, rel in enumerate(roles) for s, o in rel])
        db.executemany("INSERT INTO val VALUES (?, ?, ?)",
                       [(p, x, v) for p, vals in enumerate(values) for x, v in vals.items()])
        db.execute("CREATE INDEX ie ON edge(r, s, o)")
        db.execute("CREATE INDEX ie2 ON edge(r, o, s)")
        self.db = db

    def query(self, h) -> str:
        op = h[0]
        if op == "top":
            return "SELECT x FROM ind"
        if op == "bot":
            return "SELECT x FROM ind WHERE 0"
        if op == "atom":
            return f"SELECT x FROM mem WHERE c = {int(h[1])}"
        if op == "not":
            return f"SELECT x FROM ind EXCEPT SELECT * FROM ({self.query(h[1])})"
        if op in ("and", "or"):
            if len(h) == 1:
                return self.query(("top",) if op == "and" else ("bot",))
            glue = " INTERSECT " if op == "and" else " UNION "
            return glue.join(f"SELECT * FROM ({self.query(c)})" for c in h[1:])
        if op in ("dge", "dle"):
            _, p, t = h
            cmp = ">=" if op == "dge" else "<="
            return f"SELECT x FROM val WHERE p = {int(p)} AND v {cmp} {repr(_f32(t))}"
        if op in ("exists", "forall"):
            _, r, inv, c = h
        else:
            _, k, r, inv, c = h
        me, other = ("o", "s") if inv else ("s", "o")
        sub = self.query(c)
        if op == "exists":
            return (f"SELECT DISTINCT {me} FROM edge WHERE r = {int(r)} "
                    f"AND {other} IN ({sub})")
        if op == "forall":
            return (f"SELECT x FROM ind WHERE NOT EXISTS (SELECT 1 FROM edge e WHERE "
                    f"e.r = {int(r)} AND e.{me} = ind.x AND e.{other} NOT IN ({sub}))")
        cmp = {"atleast": ">=", "atmost": "<=", "exactly": "="}[op]
        return (f"SELECT x FROM ind WHERE (SELECT COUNT(DISTINCT e.{other}) FROM edge e "
                f"WHERE e.r = {int(r)} AND e.{me} = ind.x AND e.{other} IN ({sub})) "
                f"{cmp} {int(k)}")

    def ext(self, h):
        return {row[0] for row in self.db.execute(self.query(h))}
