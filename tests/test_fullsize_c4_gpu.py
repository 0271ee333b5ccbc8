"""Parity at the refinement trace's full size: 32M individuals, 1,024
concepts, 64 roles (about 495M assertions, Zipf s = 1.5, cap 65,536; the
inverse built by the library), 128 properties, 1M + 1M examples.  Two rounds
of 16,384 candidates run as the benchmark runs them (the parents' subtrees in
the set table, the added conjuncts drawn, written and planned on the device);
sampled candidates of both rounds cover what the oracle says, bit for bit."""
import gc
import sys

import numpy as np
import pytest

from oracle import Oracle
from paper_2412_00802_amd import hthedl, synth, trace

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_c4_trace_rounds_against_oracle():
    import torch
    assert torch.cuda.is_available(), "the gpu tests need an MI355X"
    cfg = synth.CONFIGS["c4"]
    kb = synth.make_kb(cfg)
    assert kb.n == 32_000_000
    say(f"[c4] {kb.n_edges:,} assertions")
    eng = hthedl.Engine(kb, max_nodes=64, max_hyps=1)
    cache = trace.SetCache(eng, 4096)
    rng = np.random.default_rng(synth.BASE_SEED + 40)
    o = Oracle(kb)
    pick = np.random.default_rng(2412)
    checked = 0
    for rec, cands, counts in trace.run_trace_device(cfg, kb, eng, 2, 16384, 256, 16384, cache, rng,
                                                     synth.BASE_SEED + 41, decode=True):
        assert len(cands) == counts.shape[0] == 16384
        say(f"[c4] round {rec['round']}: {rec['on_device']} candidates on the device, "
            f"{rec['device_ms']} ms; checking 64 against the oracle")
        idx = np.sort(pick.choice(len(cands), size=64, replace=False))
        if rec["on_device"]:          # at least half of the sample among the device-written candidates
            host = len(cands) - rec["on_device"]
            idx = np.union1d(idx, host + np.sort(pick.choice(rec["on_device"], size=32, replace=False)))
        want = o.coverages([cands[i] for i in idx])
        bad = np.flatnonzero((counts[idx] != want).any(axis=1))
        assert bad.size == 0, (rec["round"], idx[bad[:5]], counts[idx[bad[0]]], want[bad[0]])
        checked += idx.size
    assert checked >= 128
    cache.close()
    eng.close()
    del eng, cache
    gc.collect()
    torch.cuda.empty_cache()
