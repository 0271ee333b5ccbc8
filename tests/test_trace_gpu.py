"""The refinement trace on the GPU: every round's counts equal the oracle's,
with and without the set table of cached parent subtrees."""
import dataclasses
import sys

import numpy as np
import pytest

from oracle import Oracle
from paper_2412_00802_amd import hthedl, synth, trace

pytestmark = pytest.mark.gpu


def test_trace_rounds_match_oracle():
    import torch
    assert torch.cuda.is_available()
    cfg = dataclasses.replace(synth.CONFIGS["c4"], name="c4-test", n_individuals=20_000, n_concepts=48,
                              n_roles=4, total_edges=120_000, degree_cap=512, n_data=3, n_pos=1500,
                              n_neg=1500)
    kb = synth.make_kb(cfg)
    o = Oracle(kb)
    eng = hthedl.Engine(kb)
    got = {}
    for name, cap in (("cached", 64), ("plain", 0)):
        cache = trace.SetCache(eng, cap) if cap else None
        rng = np.random.default_rng(3)
        got[name] = []
        for rec, cands, counts in trace.run_trace(cfg, kb, eng, rounds=4, per_round=384, beam=12, chunk=160,
                                                  cache=cache, rng=rng):
            print(f"[trace] {name} round {rec['round']}: nodes {rec['nodes']} -> {rec['nodes_after_sets']}",
                  file=sys.stderr, flush=True)
            if name == "cached":
                assert np.array_equal(counts, o.coverages(cands)), rec["round"]
                if rec["round"]:
                    assert rec["nodes_after_sets"] < rec["nodes"]
            got[name].append(counts)
        if cache is not None:
            cache.close()
    for a, b in zip(got["cached"], got["plain"]):
        assert np.array_equal(a, b)


def test_trace_with_device_candidates():
    """Rounds whose added conjuncts are drawn, written and planned on the
    device: every candidate of every round (host local specialisations and
    device conjuncts, decoded from their specs) covers what the oracle says."""
    import torch
    assert torch.cuda.is_available()
    cfg = dataclasses.replace(synth.CONFIGS["c4"], name="c4-test", n_individuals=20_000, n_concepts=48,
                              n_roles=4, total_edges=120_000, degree_cap=512, n_data=3, n_pos=1500,
                              n_neg=1500)
    kb = synth.make_kb(cfg)
    o = Oracle(kb)
    eng = hthedl.Engine(kb)
    cache = trace.SetCache(eng, 64)
    rng = np.random.default_rng(4)
    on_device = 0
    for rec, cands, counts in trace.run_trace_device(cfg, kb, eng, rounds=4, per_round=384, beam=12, chunk=160,
                                                     cache=cache, rng=rng, seed=99, decode=True):
        print(f"[trace] device candidates round {rec['round']}: {rec['on_device']} on the device",
              file=sys.stderr, flush=True)
        assert len(cands) == counts.shape[0] == 384
        assert np.array_equal(counts, o.coverages(cands)), rec["round"]
        on_device += rec["on_device"]
    assert on_device > 384
    cache.close()
