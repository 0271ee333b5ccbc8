"""Parity at the uneven-batch workload's full size: 4M individuals, 1,024
concepts, 48 roles (39.7M assertions, Zipf s = 1.6, cap 8,192), 32 properties,
65,536 sized hypotheses with shared subtrees.  The whole batch is evaluated in
the configuration the benchmark times (plans generated on the device, one
plan for the batch) and with host-compiled plans; the two agree on every
hypothesis, and sampled hypotheses' counts and instance rows equal the
oracle's bit for bit."""
import sys

import numpy as np
import pytest

from oracle import Oracle
from oracle.cpp_oracle import CppOracle, batch_tokens
from paper_2412_00802_amd import hthedl, synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_c3_full_batch_against_oracle():
    import torch
    assert torch.cuda.is_available(), "the gpu tests need an MI355X"
    cfg = synth.CONFIGS["c3"]
    kb = synth.make_kb(cfg)
    hyps = synth.make_sized_hypotheses(cfg, kb)
    H = len(hyps)
    assert H == 65_536 and kb.n == 4_000_000
    say(f"[c3] {kb.n_edges:,} assertions, {H} hypotheses")
    enc = hthedl.encode_batch(hyps)
    eng = hthedl.Engine(kb, max_nodes=64, max_hyps=1)
    # hash-consing on the device, with the batch's 256 blocks of hypotheses
    # spread over every XCD: one role node per distinct role subexpression and
    # one row per distinct threshold, exactly
    from tests.test_devplan_gpu import _distinct
    n_roles, n_thr, depth = _distinct(hyps)
    d_nodes, d_offs, d_ch = eng.upload_batch(encoded=enc)
    eng.ensure_plan_scratch(int(enc[0].shape[0]))
    plan, _ = hthedl.hth_dplan_create(eng.handle, d_nodes, int(enc[0].shape[0]), d_offs, H, d_ch,
                                      int(d_ch.shape[0]), eng.dp_scratch, eng.dp_scratch_bytes)
    try:
        info = hthedl.hth_dplan_stats(plan)
    finally:
        hthedl.hth_dplan_destroy(plan)
    say(f"[c3] device plan {info}; distinct role subexpressions {n_roles}, thresholds {n_thr}, depth {depth}")
    assert info["role_nodes"] == n_roles and info["thresholds"] == n_thr and info["levels"] == depth
    # the benchmark's step: one device-generated plan for the whole batch
    dev = eng.eval_batch_device(device_batch=(d_nodes, d_offs, d_ch))
    # host-compiled plan, instance rows written for every hypothesis
    nodes, offs, ch = enc
    eng.ensure_workspace(hthedl.hth_batch_workspace_bytes(eng.handle, nodes, offs, ch))
    sets = torch.empty((H, eng.S), dtype=torch.int64, device="cuda")
    cnt = torch.empty((H, 2), dtype=torch.int32, device="cuda")
    hthedl.hth_eval_batch_sets(eng.handle, nodes, offs, ch, eng.ws, eng.ws_bytes, sets, cnt)
    host = cnt.cpu().numpy().view(np.uint32)
    bad = np.flatnonzero((dev != host).any(axis=1))
    assert bad.size == 0, f"device and host plans differ at {bad[:5]}"
    rng = np.random.default_rng(2412)
    sample = np.sort(rng.choice(H, size=256, replace=False))
    o = Oracle(kb)
    want = o.coverages([hyps[i] for i in sample])
    bad = np.flatnonzero((dev[sample] != want).any(axis=1))
    assert bad.size == 0, f"oracle mismatch at {sample[bad[:5]]}: got {dev[sample[bad[0]]]} want {want[bad[0]]}"
    say("[c3] 256 sampled hypotheses equal the oracle")
    rows = sample[:16]
    got_rows = sets[torch.from_numpy(rows).cuda()].cpu().numpy().view(np.uint64)
    for j, i in enumerate(rows):
        np.testing.assert_array_equal(got_rows[j, : kb.words], o.ext_bits(hyps[i]), err_msg=f"instance row {i}")
        assert not got_rows[j, kb.words:].any()
    say("[c3] 16 instance rows equal the oracle's")
    # a wider sample through the C++ oracle (pinned to the numpy oracle)
    wide = np.sort(rng.choice(H, size=2048, replace=False))
    co = CppOracle(kb)
    toks, toffs = batch_tokens([hyps[i] for i in wide])
    want_c = co.coverages_tokens(toks, toffs, 16)
    co.close()
    bad = np.flatnonzero((dev[wide] != want_c).any(axis=1))
    assert bad.size == 0, f"C++ oracle mismatch at {wide[bad[:5]]}"
    say("[c3] 2,048 sampled hypotheses equal the C++ oracle")
    del sets
    eng.close()
