"""The byte model of the roofline on hand-computed cases: which arrays a sweep
reads, what a role node and a compound filler cost, and what sharing saves."""
import numpy as np
import pytest

from paper_2412_00802_amd import bytes_model as bm
from paper_2412_00802_amd import synth


@pytest.fixture(scope="module")
def shape():
    # 130 individuals (3 words: W8 = 24 B); role 0: 4 assertions from 2
    # subjects to 3 objects; role 1: 1 assertion
    roles = [[(0, 5), (0, 7), (3, 5), (3, 9)], [(2, 2)]]
    data = np.zeros((2, 130), dtype=np.float32)
    kb = synth.kb_from_edges(130, [[1, 2], [3], [4]], roles, data, [1], [2])
    return bm.KBShape(kb)


def csr(shape, r, inv):
    return shape.csr_bytes(r, inv)


def test_kb_shape(shape):
    assert shape.w8 == 24
    assert shape.edges == [4, 1]
    assert shape.rows == [(2, 3), (1, 1)]
    assert csr(shape, 0, 0) == 4 * 4 + 8 * 2 and csr(shape, 0, 1) == 4 * 4 + 8 * 3


def test_single_constructs(shape):
    cov = 2 * 24 + 8
    assert bm.batch_model([("atom", 0)], shape)["total"] == 24 + cov
    assert bm.batch_model([("top",)], shape)["total"] == cov
    assert bm.batch_model([("dge", 1, 0.5)], shape)["total"] == 4 * 130 + cov
    # a root role node: its CSR and its filler's leaf; the output is fused into coverage
    assert bm.batch_model([("exists", 0, 1, ("atom", 2))], shape)["total"] == csr(shape, 0, 1) + 24 + cov
    # a compound filler is written and read once; its leaves are read in the role's sweep
    m = bm.batch_model([("forall", 0, 0, ("or", ("atom", 0), ("atom", 1)))], shape)
    assert m["total"] == csr(shape, 0, 0) + 2 * 24 + 2 * 24 + cov
    # a negated leaf is a fused negation, not a compound filler
    m = bm.batch_model([("exists", 1, 0, ("not", ("atom", 0)))], shape)
    assert m["fillers"] == 0 and m["total"] == csr(shape, 1, 0) + 24 + cov


def test_nesting_and_sharing(shape):
    cov1 = 2 * 24 + 8
    inner = ("exists", 1, 0, ("atom", 0))
    # two levels: the inner role node's row is written and read once
    m = bm.batch_model([("atleast", 2, 0, 0, inner)], shape)
    assert m["levels"] == 2
    assert m["total"] == csr(shape, 1, 0) + 24 + 2 * 24 + csr(shape, 0, 0) + cov1
    # shared between two hypotheses: one role node, one CSR sweep
    m2 = bm.batch_model([inner, ("and", inner, ("atom", 1))], shape)
    assert m2["distinct_role_nodes"] == 1 and m2["csr_sweeps"] == 1
    # atom 0 in the role's sweep, atom 1 in the root sweep; the row is read by the second root
    assert m2["total"] == csr(shape, 1, 0) + 24 + 24 + 2 * 24 + 2 * 24 + 2 * 8
    # the same atom in two sweeps is read twice
    m3 = bm.batch_model([("and", inner, ("atom", 0))], shape)
    assert m3["atoms"] == 2 * 24


def test_canonical_forms_share(shape):
    a, b, c = ("atom", 0), ("atom", 1), ("atom", 2)
    h1 = ("exists", 0, 0, ("and", a, ("and", b, c)))
    h2 = ("exists", 0, 0, ("and", ("and", c, b), a, ("top",)))
    h3 = ("exists", 0, 0, ("not", ("not", ("and", b, a, c, a))))
    m = bm.batch_model([h1, h2, h3], shape)
    assert m["distinct_role_nodes"] == 1 and m["distinct_fillers"] == 1
    assert bm.batch_model([("atleast", 0, 0, 0, a)], shape)["total"] == 2 * 24 + 8   # >= 0 is top
