"""The cross-batch subexpression cache (hth_cache_*): batches that share role
restrictions with earlier batches read them from the cache's rows, and every
batch's coverage equals the oracle's -- with rows to spare, with a cache too
small for one batch (least-recently-used eviction), and across rows that a
batch both reads and must not evict."""
import sys

import numpy as np
import pytest

from oracle import Oracle
from paper_2412_00802_amd import hthedl, synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def setup():
    import torch
    assert torch.cuda.is_available(), "the gpu tests need an MI355X"
    cfg = synth.small_config(n=30_011, n_concepts=40, n_roles=4, s=1.5, cap=300, n_data=3, n_pos=3000,
                             n_neg=2500, seed_index=3100)
    kb = synth.make_kb(cfg)
    hyps = synth.make_sized_hypotheses(cfg, kb, count=1600)
    return torch, cfg, kb, hyps, Oracle(kb).coverages(hyps)


def _run(torch, eng, cache, batch):
    nodes, offs, ch = hthedl.encode_batch(batch)
    eng.ensure_workspace(hthedl.hth_batch_workspace_bytes(eng.handle, nodes, offs, ch))
    out = torch.empty((len(batch), 2), dtype=torch.int32, device="cuda")
    hthedl.hth_eval_batch_cached(eng.handle, cache, nodes, offs, ch, eng.ws, eng.ws_bytes, out)
    return out.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("n_rows", [4096, 97])
def test_cached_batches_equal_the_oracle(setup, n_rows):
    torch, cfg, kb, hyps, want = setup
    eng = hthedl.Engine(kb, max_hyps=len(hyps))
    rows = torch.empty((n_rows, eng.S), dtype=torch.int64, device="cuda")
    cache = hthedl.hth_cache_create(eng.handle, rows, n_rows)
    try:
        # four batches of 400 sized hypotheses (their subtrees come from one
        # shared pool), then the first batch again, then everything at once
        parts = [(a, a + 400) for a in range(0, 1600, 400)] + [(0, 400), (0, 1600)]
        for a, b in parts:
            got = _run(torch, eng, cache, hyps[a:b])
            st = hthedl.hth_cache_stats(cache)
            say(f"[cache] rows {n_rows}, batch [{a}, {b}): {st}")
            bad = np.flatnonzero((got != want[a:b]).any(axis=1))
            assert bad.size == 0, (n_rows, a, b, a + bad[0], hyps[a + bad[0]], got[bad[0]], want[a + bad[0]])
        st = hthedl.hth_cache_stats(cache)
        assert st["hits"] > 0 and st["batches"] == len(parts)
        assert st["entries"] <= n_rows and st["admitted"] - st["evictions"] == st["entries"]
        if n_rows < 400:
            assert st["evictions"] > 0
        # a batch repeated right after itself reads every role restriction from the cache
        if n_rows >= 4096:
            before = hthedl.hth_cache_stats(cache)
            got = _run(torch, eng, cache, hyps[:400])
            after = hthedl.hth_cache_stats(cache)
            assert np.array_equal(got, want[:400])
            assert after["misses"] == before["misses"] and after["hits"] > before["hits"]
    finally:
        hthedl.hth_cache_destroy(cache)
    # the kb works as before without the cache
    assert np.array_equal(eng.eval_batch(hyps[:200]), want[:200])
    eng.close()


def test_cache_rejects_set_leaves_and_a_replaced_table(setup):
    torch, cfg, kb, hyps, want = setup
    eng = hthedl.Engine(kb, max_hyps=64)
    rows = torch.empty((64, eng.S), dtype=torch.int64, device="cuda")
    cache = hthedl.hth_cache_create(eng.handle, rows, 64)
    try:
        with pytest.raises(hthedl.HthError) as e:
            _run(torch, eng, cache, [("and", ("set", 0), ("atom", 1))])
        assert e.value.status == -7
        other = torch.zeros((2, eng.S), dtype=torch.int64, device="cuda")
        hthedl.hth_kb_set_sets(eng.handle, other, 2)
        with pytest.raises(hthedl.HthError) as e:
            _run(torch, eng, cache, hyps[:8])
        assert e.value.status == -6
    finally:
        hthedl.hth_cache_destroy(cache)
    eng.close()
