"""Algorithmic (compulsory) HBM bytes of a batch of hypotheses: the byte model
the roofline fraction is taken against.

The model counts what an ideal evaluation of the batch must move between HBM
and the chip, over the batch's shared-subexpression DAG (equal subexpressions
are one node; ⊓/⊔ flattened, deduplicated and sorted, ¬¬C = C, ⊤/⊥ absorbed).
Role nodes are placed on role-nesting levels (a role node whose filler holds
no role node is on level 0, otherwise one above the highest role node in its
filler); a level's role nodes run in one sweep, the root regions in a last
sweep.  Per sweep, every array it references is read once:

==================================  ==========================================
term                                bytes
==================================  ==========================================
atomic concept A                    W8, once per (A, sweep)
data property p (all thresholds)    4 N, once per (p, sweep)
CSR of (role r, direction)          4 E_r + min(8 rows_nonempty, 4 (N + 1)),
                                    once per (r, direction, sweep)
role node output                    W8 written + W8 read, per distinct role
                                    node (0 when it is only ever a root: the
                                    coverage is fused into it)
compound filler of a role node      W8 written + W8 read, per distinct filler
                                    (¬ of a leaf or of a role node is a fused
                                    negation, not a compound filler)
coverage                            2 W8 (P and Ng) + 8 B per hypothesis
⊓ / ⊔ / ¬ / ⊤ / ⊥ inside a region   0 (fused)
==================================  ==========================================

with W8 = 8 ceil(N / 64) bytes, one bit per individual.  The fraction of the
roofline is model bytes / time / peak bandwidth; bytes a kernel moves beyond
the model (re-reads, intermediate tables) show up as traffic amplification
in the counters, not here.
"""
from __future__ import annotations

from typing import Dict, Sequence, Tuple

import numpy as np

ROLE_OPS = ("exists", "forall", "atleast", "atmost", "exactly")
LEAF_OPS = ("top", "bot", "atom", "dge", "dle", "deq")


class KBShape:
    """The knowledge-base sizes the model needs: N, and per role the assertion
    count and the non-empty rows of each direction."""

    def __init__(self, kb):
        self.n = int(kb.n)
        self.w8 = 8 * ((self.n + 63) // 64)
        off = np.asarray(kb.role_offsets, dtype=np.int64)
        tg = np.asarray(kb.role_targets)
        self.edges, self.rows = [], []
        for r in range(off.shape[0]):
            lo, hi = int(off[r, 0]), int(off[r, -1])
            fwd_rows = int(np.count_nonzero(np.diff(off[r])))
            inv_rows = int(np.unique(tg[lo:hi]).size) if hi > lo else 0
            self.edges.append(hi - lo)
            self.rows.append((fwd_rows, inv_rows))

    def csr_bytes(self, r: int, inv: int) -> float:
        return 4.0 * self.edges[r] + min(8.0 * self.rows[r][inv], 4.0 * (self.n + 1))


class _Dag:
    """Hash-consed canonical nodes: id -> (op, args, child ids)."""

    def __init__(self):
        self.ids: Dict[tuple, int] = {}
        self.nodes = []

    def intern(self, key: tuple) -> int:
        i = self.ids.get(key)
        if i is None:
            i = len(self.nodes)
            self.ids[key] = i
            self.nodes.append(key)
        return i

    def canon(self, h) -> int:
        op = h[0]
        if op in ("top", "bot"):
            return self.intern((op,))
        if op == "atom":
            return self.intern(("atom", int(h[1])))
        if op in ("dge", "dle", "deq"):
            return self.intern((op, int(h[1]), float(np.float32(h[2]))))
        if op == "not":
            c = self.canon(h[1])
            cn = self.nodes[c]
            if cn[0] == "not":
                return cn[1]
            if cn[0] == "top":
                return self.intern(("bot",))
            if cn[0] == "bot":
                return self.intern(("top",))
            return self.intern(("not", c))
        if op in ("and", "or"):
            unit, zero = ("top", "bot") if op == "and" else ("bot", "top")
            kids = set()
            for c in h[1:]:
                ci = self.canon(c)
                cn = self.nodes[ci]
                if cn[0] == op:
                    kids.update(cn[1])
                elif cn[0] == unit:
                    continue
                elif cn[0] == zero:
                    return self.intern((zero,))
                else:
                    kids.add(ci)
            if not kids:
                return self.intern((unit,))
            if len(kids) == 1:
                return next(iter(kids))
            return self.intern((op, tuple(sorted(kids))))
        if op in ("exists", "forall"):
            _, r, inv, c = h
            return self.intern((op, int(r), int(inv), 0, self.canon(c)))
        if op in ("atleast", "atmost", "exactly"):
            _, n, r, inv, c = h
            if op == "atleast" and int(n) == 0:
                return self.intern(("top",))
            return self.intern((op, int(r), int(inv), int(n), self.canon(c)))
        raise ValueError(f"construct {op!r} is outside the byte model")


def batch_model(hyps: Sequence, shape: KBShape) -> Dict[str, float]:
    """Model bytes of evaluating `hyps` as one batch, with the breakdown."""
    dag = _Dag()
    roots = [dag.canon(h) for h in hyps]
    nodes = dag.nodes
    level = [-1] * len(nodes)          # highest role level inside the node's subtree
    for i, nd in enumerate(nodes):     # children are interned before parents
        op = nd[0]
        if op in ROLE_OPS:
            level[i] = 1 + level[nd[4]]
        elif op == "not":
            level[i] = level[nd[1]]
        elif op in ("and", "or"):
            level[i] = max(level[c] for c in nd[1])
    w8, n = shape.w8, shape.n
    atoms, props, csr = set(), set(), set()     # (id, sweep)
    fillers = set()

    def region(i: int, sweep) -> None:
        """Leaves a region reads, up to role nodes (their outputs are counted
        with the role nodes)."""
        nd = nodes[i]
        op = nd[0]
        if op == "atom":
            atoms.add((nd[1], sweep))
        elif op in ("dge", "dle", "deq"):
            props.add((nd[1], sweep))
        elif op == "not":
            region(nd[1], sweep)
        elif op in ("and", "or"):
            for c in nd[1]:
                region(c, sweep)

    role_read = set()
    root_only = set(roots)
    for i, nd in enumerate(nodes):
        if nd[0] in ROLE_OPS:
            _, r, inv, _, c = nd
            L = level[i]
            csr.add(((r, inv), L))
            region(c, L)
            cn = nodes[c]
            f = cn[1] if cn[0] == "not" else c
            if nodes[f][0] not in LEAF_OPS and nodes[f][0] not in ROLE_OPS:
                fillers.add(f)              # a compound filler is materialised
            # role nodes referenced from this filler are read by a consumer
            stack = [c]
            while stack:
                j = stack.pop()
                m = nodes[j]
                if m[0] in ROLE_OPS:
                    role_read.add(j)
                elif m[0] == "not":
                    stack.append(m[1])
                elif m[0] in ("and", "or"):
                    stack.extend(m[1])
    for i in set(roots):
        region(i, "root")
        stack = [i] if nodes[i][0] not in ROLE_OPS else []
        while stack:
            j = stack.pop()
            m = nodes[j]
            if m[0] in ROLE_OPS:
                role_read.add(j)
            elif m[0] == "not":
                stack.append(m[1])
            elif m[0] in ("and", "or"):
                stack.extend(m[1])
    role_nodes = [i for i, nd in enumerate(nodes) if nd[0] in ROLE_OPS]
    # a role node only ever used as a whole hypothesis writes no row: its
    # coverage is fused into it
    n_role_rows = sum(1 for i in role_nodes if i in role_read or i not in root_only)
    out = {
        "atoms": float(len(atoms) * w8),
        "data": len(props) * 4.0 * n,
        "csr": sum(shape.csr_bytes(r, inv) for (r, inv), _ in csr),
        "role_outputs": n_role_rows * 2.0 * w8,
        "fillers": len(fillers) * 2.0 * w8,
        "coverage": 2.0 * w8 + 8.0 * len(hyps),
    }
    out["total"] = float(sum(out.values()))
    out["distinct_role_nodes"] = len(role_nodes)
    out["distinct_fillers"] = len(fillers)
    out["levels"] = 1 + max([level[i] for i in role_nodes], default=-1)
    out["csr_sweeps"] = len(csr)
    # the shared role passes' share: each (role, direction, sweep) CSR once and
    # every role node's output row written once
    out["role_pass"] = out["csr"] + n_role_rows * w8
    return out


def plain_model(h, shape: KBShape) -> float:
    """Model bytes of one hypothesis evaluated alone (the unit is the hypothesis)."""
    return batch_model([h], shape)["total"]


def summary(m: Dict[str, float]) -> Dict[str, float]:
    return {k: (round(v / 1e9, 4) if isinstance(v, float) else v) for k, v in m.items()}


def per_hypothesis(m: Dict[str, float], n_hyps: int) -> Tuple[float, float]:
    return m["total"] / max(n_hyps, 1), m["role_pass"] / max(n_hyps, 1)
