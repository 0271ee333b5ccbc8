"""A CPU reference of the device's conjunct draws and candidate layout
(hth_draw_conjuncts, hth_conjoin), written from the definitions in
include/hthedl.h; it shares no code with the library."""
import numpy as np

from paper_2412_00802_amd.hthedl import CJ_ATOM, CJ_EQ, CJ_EXISTS, CJ_GE, CJ_LE, CONJ_DTYPE, NODE_DTYPE, OPS

M64 = (1 << 64) - 1


def splitmix64(seed: int, i: int) -> int:
    """Value i of the SplitMix64 sequence started at seed (Steele, Lea and
    Flood, OOPSLA 2014): the state advances by the golden-ratio increment and
    each output is the state through the generator's mixing function."""
    z = (seed + (i + 1) * 0x9E3779B97F4A7C15) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def draw(seed, parent_rows, per_parent, n_concepts, n_roles, n_data, deciles) -> np.ndarray:
    n = len(parent_rows) * per_parent
    out = np.zeros(n, dtype=CONJ_DTYPE)
    dec = np.asarray(deciles, dtype=np.float32)
    for i in range(n):
        u0, u1, u2, u3 = (splitmix64(seed, 4 * i + k) for k in range(4))
        k = u0 % 10
        kind = CJ_ATOM if k < 5 else CJ_EXISTS if k < 8 else (CJ_LE if u3 & 1 else CJ_GE)
        if (kind == CJ_EXISTS and not n_roles) or (kind in (CJ_GE, CJ_LE) and not n_data):
            kind = CJ_ATOM
        rec = out[i]
        rec["parent"] = parent_rows[i // per_parent]
        rec["kind"] = kind
        if kind == CJ_ATOM:
            rec["a"] = u1 % n_concepts
        elif kind == CJ_EXISTS:
            rec["b"] = u1 % n_roles
            rec["inv"] = (u1 >> 32) & 1
            rec["a"] = u2 % n_concepts
        else:
            rec["a"] = u1 % n_data
            rec["b"] = int(np.float32(dec[rec["a"], u2 % 9]).view(np.uint32))
    return out


def conjoin(specs: np.ndarray, node_base: int = 0, child_base: int = 0):
    """-> (nodes [4n], offsets [n+1], children [2n]) as hth_conjoin writes them
    at the given bases."""
    n = specs.shape[0]
    nodes = np.zeros(4 * n, dtype=NODE_DTYPE)
    kids = np.zeros(2 * n, dtype=np.uint32)
    leaf_op = {CJ_GE: OPS["dge"], CJ_LE: OPS["dle"], CJ_EQ: OPS["deq"]}
    for i, c in enumerate(specs):
        nodes[4 * i] = (OPS["set"], 0, 0, c["parent"], 0, 0)
        x = 1
        if c["kind"] == CJ_ATOM:
            nodes[4 * i + 1] = (OPS["atom"], 0, 0, c["a"], 0, 0)
        elif c["kind"] == CJ_EXISTS:
            nodes[4 * i + 1] = (OPS["atom"], 0, 0, c["a"], 0, 0)
            nodes[4 * i + 2] = (OPS["exists"], c["inv"], 0, c["b"], 1, 0)
            x = 2
        elif c["kind"] in leaf_op:
            nodes[4 * i + 1] = (leaf_op[int(c["kind"])], 0, 0, c["a"], 0, c["b"])
        else:
            nodes[4 * i + 1] = (0xFF, 0, 0, 0, 0, 0)
        if x == 1:
            nodes[4 * i + 2] = (OPS["top"], 0, 0, 0, 0, 0)
        nodes[4 * i + 3] = (OPS["and"], 0, 2, 0, child_base + 2 * i, 0)
        kids[2 * i + 1] = x
    return nodes, (node_base + 4 * np.arange(n + 1)).astype(np.uint32), kids
