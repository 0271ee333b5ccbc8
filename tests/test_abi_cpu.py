"""The C-ABI library loads and exports what include/hthedl.h declares; host-side
argument checks and the hypothesis encoding work without a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2412_00802_amd import hthedl, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "hthedl.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hth_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    L = hthedl.lib()
    names = declared_functions()
    assert len(names) >= 11
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(hthedl.EXPORTED)


def test_status_strings():
    for code, name in hthedl.STATUS.items():
        assert hthedl.hth_status_str(code) == name


def _desc(n=100, stride=None, n_concepts=0):
    d = hthedl.KBDesc()
    d.n_individuals = n
    d.stride_words = stride if stride is not None else hthedl.stride_for(n)
    d.n_concepts = n_concepts
    d.concept_bits = 0x1000 if n_concepts else None
    d.n_roles = 0
    d.pos_bits = 0x2000
    d.neg_bits = 0x3000
    return d


def test_derived_bytes_host_checks():
    assert hthedl.hth_kb_derived_bytes(_desc()) > 0
    with pytest.raises(hthedl.HthError) as e:
        hthedl.hth_kb_derived_bytes(_desc(stride=3))
    assert e.value.status == -1 and "stride" in str(e.value)
    with pytest.raises(hthedl.HthError) as e:
        hthedl.hth_kb_derived_bytes(_desc(n=0))
    assert e.value.status == -2
    d = _desc()
    d.pos_bits = None
    with pytest.raises(hthedl.HthError):
        hthedl.hth_kb_derived_bytes(d)


def test_derived_bytes_scale_with_kb():
    d = _desc(n=1000)
    d.n_roles = 4
    d.n_edges = 5000
    d.role_offsets = 0x4000
    d.role_targets = 0x5000
    b = hthedl.hth_kb_derived_bytes(d)
    # two 32-bit offset arrays + inverse targets + scan cursor at least
    assert b >= 3 * 4 * 1001 * 4 + 5000 * 4


def test_null_handle_rejected():
    with pytest.raises(hthedl.HthError):
        hthedl.hth_workspace_bytes(None, 10, 1)
    assert "NULL" in hthedl.hth_last_error()


def test_encoding_is_postfix():
    h = ("and", ("atom", 3), ("exists", 2, 1, ("not", ("atom", 1))),
         ("atleast", 3, 0, 0, ("dge", 1, 0.5)), ("or",))
    nodes, ch = hthedl.encode_one(h)
    assert nodes.dtype.itemsize == 16
    root = nodes[-1]
    assert root["op"] == hthedl.OPS["and"] and root["arity"] == 4
    kids = ch[root["child"]:root["child"] + root["arity"]]
    assert all(k < len(nodes) - 1 for k in kids)
    for i, nd in enumerate(nodes):
        if nd["op"] in (3, 6, 7, 8, 9, 10):
            assert nd["child"] < i
    dge = [nd for nd in nodes if nd["op"] == hthedl.OPS["dge"]][0]
    assert np.array([dge["q"]], dtype=np.uint32).view(np.float32)[0] == np.float32(0.5)
    al = [nd for nd in nodes if nd["op"] == hthedl.OPS["atleast"]][0]
    assert al["q"] == 3 and al["arg"] == 0


def test_batch_encoding_offsets():
    cfg = synth.CONFIGS["c1"]
    kb = synth.make_kb(cfg)
    hs = synth.make_hypotheses(cfg, kb, count=20)
    nodes, offs, ch = hthedl.encode_batch(hs)
    assert offs[0] == 0 and offs[-1] == len(nodes) and len(offs) == 21
    assert [offs[i + 1] - offs[i] for i in range(20)] == [synth.hyp_size(h) for h in hs]


def test_noalloc_scratch_size_matches_header():
    """The binding's scratch size is the header's HTH_NOALLOC_SCRATCH_BYTES."""
    text = open(os.path.join(ROOT, "include", "hthedl.h")).read()
    m = re.search(r"#define\s+HTH_NOALLOC_SCRATCH_BYTES\s+\((\d+)u\s*<<\s*(\d+)\)", text)
    assert m, "HTH_NOALLOC_SCRATCH_BYTES not found"
    assert int(m.group(1)) << int(m.group(2)) == hthedl.NOALLOC_SCRATCH_BYTES
