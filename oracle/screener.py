"""CPU references for the learned screener -- test infrastructure only.

The screener is this project's extension (the paper has no learner): a bf16
MLP over hashed subtree features that ranks refinement candidates.  These
references define what its kernels compute:

* ``subtree_features``: the hashed subtree features of a hypothesis given as a
  nested tuple, node by node in postfix order; ``dense_features`` and
  ``delta_features`` (a refinement's counts minus its parent's);
* ``bf16``: float32 -> bfloat16 round-to-nearest-even, returned as float64;
* ``forward`` / ``backward``: the MLP 4096 -> 1024 -> 256 -> 2 with ReLU and
  either BCE-with-logits (targets are fractions) or the squared error
  (targets are log(1 + removed counts)), in float64, exact (``rounding=False``,
  pinned by finite differences in the tests) or with the bf16 roundings the
  kernels apply to their stored operands and activations;
* ``adamw``: one AdamW step with decoupled weight decay;
* ``predicted_f1``: the screening score from the two outputs.

Parity status: the MLP gradients are pinned by central finite differences;
the feature hash and the optimiser step follow their written definitions.
"""
from __future__ import annotations

import struct
from typing import Dict, List, Tuple

import numpy as np

FNV_OFFSET = 0xCBF29CE484222325
FNV_PRIME = 0x100000001B3
MASK64 = (1 << 64) - 1
FEATURE_DIM = 4096

_OPS = {"top": 0, "bot": 1, "atom": 2, "not": 3, "and": 4, "or": 5, "exists": 6, "forall": 7,
        "atleast": 8, "atmost": 9, "exactly": 10, "dge": 11, "dle": 12,
        "deq": 14, "nge": 15, "nle": 16, "neq": 17}


def _fnv(h: int, data: bytes) -> int:
    for byte in data:
        h ^= byte
        h = (h * FNV_PRIME) & MASK64
    return h


def _splitmix(x: int) -> int:
    z = (x + 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def _header(op: str, inv: int = 0, arity: int = 0, arg: int = 0, q: int = 0) -> bytes:
    return struct.pack("<BBHII", _OPS[op], inv, arity, arg, q)


def _f32_bits(t: float) -> int:
    return struct.unpack("<I", struct.pack("<f", t))[0]


def subtree_features(h) -> List[Tuple[int, int]]:
    """(hash, feature index) of every node of h in postfix order (children
    left to right before the node), the order of the library's node arrays."""
    out: List[Tuple[int, int]] = []

    def visit(t) -> int:
        op = t[0]
        if op in ("top", "bot"):
            v = _fnv(FNV_OFFSET, _header(op))
        elif op == "atom":
            v = _fnv(FNV_OFFSET, _header(op, arg=t[1]))
        elif op in ("dge", "dle", "deq", "nge", "nle", "neq"):
            v = _fnv(FNV_OFFSET, _header(op, arg=t[1], q=_f32_bits(t[2])))
        elif op == "not":
            c = visit(t[1])
            v = _fnv(_fnv(FNV_OFFSET, _header(op)), struct.pack("<Q", c))
        elif op in ("and", "or"):
            cs = [visit(c) for c in t[1:]]
            s = sum(_splitmix(c) for c in cs) & MASK64
            v = _fnv(_fnv(FNV_OFFSET, _header(op, arity=len(cs))), struct.pack("<Q", s))
        else:
            if op in ("exists", "forall"):
                _, r, inv, c = t
                q = 0
            else:
                _, q, r, inv, c = t
            ch = visit(c)
            v = _fnv(_fnv(FNV_OFFSET, _header(op, inv=inv, arg=r, q=q)), struct.pack("<Q", ch))
        out.append((v, v % FEATURE_DIM))
        return v

    visit(h)
    return out


def dense_features(hyps) -> np.ndarray:
    """[H][4096] counts of subtrees per feature index."""
    x = np.zeros((len(hyps), FEATURE_DIM), dtype=np.float64)
    for i, h in enumerate(hyps):
        for _, f in subtree_features(h):
            x[i, f] += 1
    return x


def delta_features(children, parents, parent_index, context: bool = False) -> np.ndarray:
    """[H][4096] subtree counts of each child minus those of its parent; with
    context, plus the parent's own counts at index f XOR 2048."""
    par = dense_features(parents)[np.asarray(parent_index)]
    x = dense_features(children) - par
    if context:
        x += par[:, np.arange(FEATURE_DIM) ^ (FEATURE_DIM // 2)]
    return x


def bf16(x) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest, ties to even); float64 result."""
    a = np.asarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    r = np.where(np.isnan(a), u, r).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def _r(x, rounding: bool):
    return bf16(x) if rounding else np.asarray(x, dtype=np.float64)


def forward(p: Dict[str, np.ndarray], x: np.ndarray, y: np.ndarray = None, rounding: bool = False,
            loss: str = "bce"):
    """Activations, and when y is given the summed loss: BCE-with-logits
    (loss="bce") or the squared error (z - y)^2 / 2 (loss="mse")."""
    w1, w2 = _r(p["w1"], rounding), _r(p["w2"], rounding)
    h1 = _r(np.maximum(x @ w1 + p["b1"], 0.0), rounding)
    h2 = _r(np.maximum(h1 @ w2 + p["b2"], 0.0), rounding)
    z = h2 @ p["w3"] + p["b3"]
    acts = {"x": x, "h1": h1, "h2": h2, "z": z}
    if y is None:
        return acts, None
    if loss == "mse":
        return acts, float(np.sum(0.5 * (z - y) ** 2))
    return acts, float(np.sum(np.maximum(z, 0) - z * y + np.log1p(np.exp(-np.abs(z)))))


def backward(p, acts, y, scale: float, rounding: bool = False, loss: str = "bce"):
    """Gradients of scale * loss."""
    x, h1, h2, z = acts["x"], acts["h1"], acts["h2"], acts["z"]
    dz = ((z - y) if loss == "mse" else (1.0 / (1.0 + np.exp(-z)) - y)) * scale
    g = {"w3": h2.T @ dz, "b3": dz.sum(0)}
    dh2 = _r((dz @ p["w3"].T) * (h2 > 0), rounding)
    g["w2"] = h1.T @ dh2
    g["b2"] = dh2.sum(0)
    dh1 = _r((dh2 @ _r(p["w2"], rounding).T) * (h1 > 0), rounding)
    g["w1"] = x.T @ dh1
    g["b1"] = dh1.sum(0)
    return g


def adamw(p, g, m, v, lr, b1, b2, eps, wd, step):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    p = p * (1 - lr * wd) - lr * mh / (np.sqrt(vh) + eps)
    return p, m, v


def predicted_f1(z: np.ndarray, n_pos: int, n_neg: int, base: np.ndarray = None,
                 kind: str = "share") -> np.ndarray:
    """F1 of the predicted coverage (p, q), F1 = 2p / (2p + q + (|P| - p)), with
    (P_b, N_b) = base[b] (a parent's coverage) or (|P|, |Ng|):
    kind "share": p = sigmoid(z0) P_b, q = sigmoid(z1) N_b;
    kind "log_removed": p = P_b - (e^z0 - 1), q = N_b - (e^z1 - 1), with z
    taken as at least 0 and p, q clamped to [0, base]."""
    bp = np.full(z.shape[0], float(n_pos)) if base is None else np.asarray(base, dtype=np.float64)[:, 0]
    bn = np.full(z.shape[0], float(n_neg)) if base is None else np.asarray(base, dtype=np.float64)[:, 1]
    if kind == "log_removed":
        p = np.clip(bp - np.expm1(np.maximum(z[:, 0], 0.0)), 0.0, bp)
        q = np.clip(bn - np.expm1(np.maximum(z[:, 1], 0.0)), 0.0, bn)
    else:
        p = bp / (1.0 + np.exp(-z[:, 0]))
        q = bn / (1.0 + np.exp(-z[:, 1]))
    den = p + q + n_pos
    return np.where(den > 0, 2 * p / np.maximum(den, 1e-30), 0.0)
