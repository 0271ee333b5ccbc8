"""hth_eval_one_noalloc (a fixed device scratch instead of a caller
workspace) gives exactly what hth_eval_one gives, call after call on one GPU,
and rejects a plan larger than its scratch before launching anything."""
import sys

import numpy as np
import pytest

from oracle import Oracle
from paper_2412_00802_amd import hthedl, synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available(), "the gpu tests need an MI355X"
    hthedl.lib()
    return torch


def _both(torch, eng, h):
    """(counts, instance words) from hth_eval_one_noalloc and from hth_eval_one
    on the same stream."""
    nodes, ch = hthedl.encode_one(eng.intern(h))
    eng.reserve(nodes.shape[0], 1)
    st = torch.cuda.current_stream()
    c_na = torch.full((2,), -1, dtype=torch.int32, device="cuda")
    i_na = torch.full((eng.S,), -1, dtype=torch.int64, device="cuda")
    hthedl.hth_eval_one_noalloc(eng.handle, nodes, ch, i_na, c_na, st)
    c_ws = torch.full((2,), -1, dtype=torch.int32, device="cuda")
    i_ws = torch.full((eng.S,), -1, dtype=torch.int64, device="cuda")
    hthedl.hth_eval_one(eng.handle, nodes, ch, eng.ws, eng.ws_bytes, i_ws, c_ws, st)
    torch.cuda.synchronize()
    return ((c_na.cpu().numpy().view(np.uint32), i_na.cpu().numpy().view(np.uint64)),
            (c_ws.cpu().numpy().view(np.uint32), i_ws.cpu().numpy().view(np.uint64)))


def _kb(n, seed, cap=3000):
    cfg = synth.small_config(n=n, n_concepts=24, n_roles=4, s=1.1, cap=cap, n_pos=n // 7, n_neg=n // 9,
                             n_hyps=40, hyp_depth=5, seed_index=seed)
    return cfg, synth.make_kb(cfg)


def test_noalloc_equals_workspace_path_two_calls(torch):
    """A large hypothesis, then a smaller one, then many more on the same KB;
    then a smaller KB: every call equals hth_eval_one and the oracle."""
    cfg, kb = _kb(200_003, 971)          # ragged tail; heavy rows (cap 3000 > 2048)
    eng = hthedl.Engine(kb, max_nodes=256, max_hyps=1)
    o = Oracle(kb)
    big = ("and", ("exists", 0, 0, ("or", ("atom", 3), ("atleast", 2, 1, 1, ("atom", 5)))),
           ("forall", 2, 1, ("not", ("exists", 3, 0, ("atom", 7)))),
           ("atmost", 3, 0, 0, ("and", ("atom", 1), ("dge", 0, float(kb.deciles[0][4])))),
           ("not", ("exists", 1, 1, ("forall", 0, 0, ("atom", 9)))))
    small = ("exists", 2, 0, ("atom", 11))
    say(f"[noalloc] N={kb.n}: big ({synth.hyp_size(big)} nodes), then small ({synth.hyp_size(small)} nodes)")
    for h in (big, small):
        (c_na, i_na), (c_ws, i_ws) = _both(torch, eng, h)
        np.testing.assert_array_equal(c_na, c_ws)
        np.testing.assert_array_equal(i_na, i_ws)
        np.testing.assert_array_equal(c_na, np.asarray(o.coverage(h), np.uint32))
        np.testing.assert_array_equal(i_na[: kb.words], o.ext_bits(h))
        assert not i_na[kb.words:].any()
    hyps = synth.make_hypotheses(cfg, kb)
    hyps = sorted(hyps, key=synth.hyp_size, reverse=True)       # each call smaller than the last
    want = o.coverages(hyps)
    for i, h in enumerate(hyps):
        (c_na, _), (c_ws, _) = _both(torch, eng, h)
        assert (c_na == c_ws).all() and (c_na == want[i]).all(), (i, h, c_na, c_ws, want[i])
    eng.close()
    # a second, smaller knowledge base on the same GPU: the same scratch, smaller rows
    cfg2, kb2 = _kb(4_097, 972, cap=64)
    eng2 = hthedl.Engine(kb2, max_nodes=256, max_hyps=1)
    o2 = Oracle(kb2)
    for h in synth.make_hypotheses(cfg2, kb2)[:16]:
        (c_na, i_na), (c_ws, i_ws) = _both(torch, eng2, h)
        np.testing.assert_array_equal(c_na, c_ws)
        np.testing.assert_array_equal(i_na, i_ws)
        np.testing.assert_array_equal(c_na, np.asarray(o2.coverage(h), np.uint32))
    eng2.close()


def test_noalloc_rejects_plans_beyond_its_scratch(torch):
    """300 distinct role restrictions over 2M individuals need about 75 MB of
    bit rows: HTH_E_NOMEM before any launch, outputs untouched; a small
    hypothesis on the same KB still runs."""
    n = 2_000_000
    cfg = synth.small_config(n=n, n_concepts=64, n_roles=4, s=1.5, cap=32, n_pos=1000, n_neg=1000,
                             n_hyps=4, seed_index=973, total_edges=2_000_000)
    kb = synth.make_kb(cfg)
    eng = hthedl.Engine(kb, max_nodes=64, max_hyps=1)
    wide = ("and",) + tuple(("exists", r % 4, (r // 4) % 2, ("atom", r // 8)) for r in range(300))
    nodes, ch = hthedl.encode_one(wide)
    c = torch.full((2,), 7, dtype=torch.int32, device="cuda")
    with pytest.raises(hthedl.HthError) as e:
        hthedl.hth_eval_one_noalloc(eng.handle, nodes, ch, None, c, torch.cuda.current_stream())
    assert e.value.status == -3                                  # HTH_E_NOMEM
    assert "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert (c.cpu().numpy() == 7).all()
    h = ("exists", 1, 1, ("atom", 2))
    (c_na, i_na), (c_ws, i_ws) = _both(torch, eng, h)
    np.testing.assert_array_equal(c_na, c_ws)
    np.testing.assert_array_equal(i_na, i_ws)
    np.testing.assert_array_equal(c_na, np.asarray(Oracle(kb).coverage(h), np.uint32))
    eng.close()
