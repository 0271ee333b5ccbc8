"""GPU parity of plans generated on the device (hth_dplan_*): the node arrays
sit in device memory, the library's count and emit kernels build the plan,
and the coverage equals the oracle's (and the host-compiled batch's) bit for
bit.  Errors are found by the count pass, before any evaluation kernel runs."""
import sys

import numpy as np
import pytest

from oracle import Oracle
from paper_2412_00802_amd import hthedl, synth
from tests.test_parity_gpu import heavy_kb, heavy_zoo

pytestmark = pytest.mark.gpu

OPS = hthedl.OPS


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "the gpu tests need an MI355X"
    hthedl.lib()
    return torch


def check_device(kb, hyps, label, chunk=None, eng=None, host=True):
    say(f"[devplan] {label}: N={kb.n} hyps={len(hyps)}")
    eng = eng or hthedl.Engine(kb, max_hyps=max(1, len(hyps)))
    want = Oracle(kb).coverages(hyps)
    got = eng.eval_batch_device(hyps, chunk=chunk)
    bad = np.flatnonzero((got != want).any(axis=1))
    assert bad.size == 0, f"device plan mismatch at {bad[:5]}: {hyps[bad[0]]} got {got[bad[0]]} want {want[bad[0]]}"
    if host:
        assert np.array_equal(eng.eval_batch(hyps), want)
    return eng


@pytest.mark.parametrize("n", [1, 63, 64, 65, 4097])
def test_tail_sizes(n):
    cfg = synth.small_config(n=n, n_concepts=10, n_roles=3, cap=min(16, max(1, n)),
                             n_pos=max(1, n // 5), n_neg=n // 5, n_hyps=48, seed_index=300 + n % 97)
    kb = synth.make_kb(cfg)
    check_device(kb, synth.make_hypotheses(cfg, kb), f"tail n={n}")


@pytest.mark.parametrize("seed", range(4))
def test_small_workloads(seed):
    """Random hypotheses over every construct (thresholds included), 600 per
    batch: several blocks of the one-thread-per-hypothesis passes."""
    cfg = synth.small_config(n=3000 + 517 * seed, n_concepts=24, n_roles=4, s=1.2 + 0.3 * seed,
                             cap=[8, 64, 300, 1000][seed], n_data=3, n_pos=400, n_neg=300, n_hyps=600,
                             hyp_depth=5, seed_index=400 + seed)
    kb = synth.make_kb(cfg)
    check_device(kb, synth.make_hypotheses(cfg, kb), f"small seed={seed}")


@pytest.mark.parametrize("heavy_min", [None, 1024])
def test_heavy_rows(monkeypatch, heavy_min):
    """Heavy rows at several levels: the per-level heavy-block ranges come
    from the device scan over the role tasks in task order."""
    if heavy_min is not None:
        monkeypatch.setenv("HTHEDL_HEAVY_MIN", str(heavy_min))
    kb = heavy_kb()
    hs = heavy_zoo()
    hs += [("exists", 0, 0, ("atleast", 2049, 0, 0, ("not", ("atom", 2)))),
           ("atmost", 3000, 1, 1, ("exists", 0, 1, ("and", ("atom", 0), ("atom", 1)))),
           ("and", ("forall", 1, 1, ("exists", 0, 0, ("top",))), ("atleast", 1025, 0, 0, ("atom", 0)))]
    check_device(kb, hs, f"heavy rows, threshold {heavy_min}", chunk=150)


def test_set_table_leaves():
    import torch
    cfg = synth.small_config(n=20000, n_concepts=24, n_roles=4, s=1.5, cap=100, n_data=3,
                             n_pos=2000, n_neg=2000, seed_index=1600)
    kb = synth.make_kb(cfg)
    o = Oracle(kb)
    subs = synth.make_hypotheses(cfg, kb, count=20, depth=3)
    eng = hthedl.Engine(kb)
    table = torch.zeros((len(subs), eng.S), dtype=torch.int64, device="cuda")
    nodes, offs, ch = hthedl.encode_batch(subs)
    eng.ensure_workspace(hthedl.hth_batch_workspace_bytes(eng.handle, nodes, offs, ch))
    cnt = torch.empty((len(subs), 2), dtype=torch.int32, device="cuda")
    hthedl.hth_eval_batch_sets(eng.handle, nodes, offs, ch, eng.ws, eng.ws_bytes, table, cnt)
    hthedl.hth_kb_set_sets(eng.handle, table, len(subs))
    rng = np.random.default_rng(3)
    hyps, full = [], []
    for i, s in enumerate(subs):
        a = ("atom", int(rng.integers(0, 24)))
        e = ("exists", int(rng.integers(0, 4)), int(rng.integers(0, 2)), ("set", i))
        hyps += [("and", ("set", i), a), ("or", ("not", ("set", i)), e), e]
        full += [("and", s, a), ("or", ("not", s), ("exists", e[1], e[2], s)), ("exists", e[1], e[2], s)]
    got = eng.eval_batch_device(hyps)
    assert np.array_equal(got, o.coverages(full))
    hthedl.hth_kb_set_sets(eng.handle, None, 0)


def _node(op, inv=0, arity=0, arg=0, child=0, q=0):
    return (OPS[op], inv, arity, arg, child, q)


def _batch(hyp_nodes, hyp_children):
    """Hand-built hypotheses: lists of node tuples (local child indices; and/or
    `child` relative to the hypothesis's own children list)."""
    nodes, children, offs = [], [], [0]
    for nd, ch in zip(hyp_nodes, hyp_children):
        base = len(children)
        for t in nd:
            t = list(t)
            if t[0] in (OPS["and"], OPS["or"]):
                t[4] += base
            nodes.append(tuple(t))
        children.extend(ch)
        offs.append(len(nodes))
    return (np.array(nodes, dtype=hthedl.NODE_DTYPE), np.array(offs, dtype=np.uint32),
            np.array(children, dtype=np.uint32))


def test_shared_nodes_within_a_hypothesis():
    """The node format allows a DAG inside a hypothesis: a node referenced
    twice is evaluated once and read from both places; a shared compound
    filler is written into each referencing region's program."""
    cfg = synth.small_config(n=5000, n_concepts=8, n_roles=2, cap=20, n_data=1, n_pos=900, n_neg=900,
                             seed_index=1900)
    kb = synth.make_kb(cfg)
    t = float(kb.deciles[0, 4])
    tb = int(np.float32(t).view(np.uint32))
    a0, ex = ("atom", 0), ("exists", 1, 0, ("atom", 0))
    conj = ("and", ex, ex)
    hyp_nodes = [
        # 0 A0, 1 exists r1.A0, 2 and(1, 1), 3 not 1, 4 or(2, 3, 0)
        [_node("atom", arg=0), _node("exists", arg=1, child=0), _node("and", arity=2, child=0),
         _node("not", child=1), _node("or", arity=3, child=2)],
        # 0 A0, 1 exists, 2 and(1,1), 3 atleast 2 r0^- .(2), 4 forall r1.(2), 5 and(3, 4, 2), 6 dge
        [_node("atom", arg=0), _node("exists", arg=1, child=0), _node("and", arity=2, child=0),
         _node("atleast", inv=1, arg=0, child=2, q=2), _node("forall", arg=1, child=2),
         _node("dge", arg=0, q=tb), _node("and", arity=4, child=2)],
        # unreachable nodes before the root are evaluated too and change nothing
        [_node("atom", arg=3), _node("atmost", arg=1, child=0, q=1), _node("atom", arg=5)],
    ]
    hyp_children = [[1, 1, 2, 3, 0], [1, 1, 3, 4, 2, 5]]
    hyp_children.append([])
    trees = [("or", conj, ("not", ex), a0),
             ("and", ("atleast", 2, 0, 1, conj), ("forall", 1, 0, conj), conj, ("dge", 0, t)),
             ("atom", 5)]
    enc = _batch(hyp_nodes, hyp_children)
    eng = hthedl.Engine(kb)
    got = eng.eval_batch_device(encoded=enc)
    assert np.array_equal(got, Oracle(kb).coverages(trees))
    assert np.array_equal(eng.eval_batch(None, encoded=enc), got)


def _balanced(k, rng, op="and"):
    if k == 0:
        return ("atom", int(rng.integers(0, 16)))
    other = "or" if op == "and" else "and"
    return (op, _balanced(k - 1, rng, other), _balanced(k - 1, rng, other))


def test_deep_regions_and_nested_roles():
    """Region programs that need 2..16 stack entries (the register kernel up to
    six, the LDS kernel above), role restrictions nested 64 deep, and the
    limits beyond (17 entries, 65 levels, 33 nested operators) rejected."""
    cfg = synth.small_config(n=3000, n_concepts=16, n_roles=2, cap=8, n_data=1, n_pos=500, n_neg=500,
                             seed_index=2000)
    kb = synth.make_kb(cfg)
    rng = np.random.default_rng(20)
    hyps = [_balanced(k, rng, op) for k in (1, 2, 5, 6, 7, 9) for op in ("and", "or")]
    nest = ("atom", 1)
    for i in range(64):
        nest = ("exists", i % 2, (i // 2) % 2, ("or", nest, ("atom", i % 16)) if i % 3 == 0 else nest)
    hyps.append(nest)
    hyps.append(("exists", 0, 0, _balanced(8, rng)))      # a deep filler region
    eng = hthedl.Engine(kb, max_nodes=1 << 17)
    for reg in (2, 0):
        hthedl.hth_kb_set_tuning(eng.handle, region_reg=reg)
        check_device(kb, hyps, f"deep regions, region_reg {reg}", eng=eng, host=False)
    deep16 = _balanced(15, rng)
    assert np.array_equal(eng.eval_batch_device([deep16]), Oracle(kb).coverages([deep16]))
    for bad in (_balanced(16, rng), ("exists", 0, 0, nest)):
        with pytest.raises(hthedl.HthError) as e:
            eng.eval_batch_device([("atom", 0), bad])
        assert e.value.status == -7 and "hypothesis 1" in str(e.value), str(e.value)
    chain = ("and", ("atom", 0), ("atom", 1))
    for _ in range(33):
        chain = ("not", chain)
    with pytest.raises(hthedl.HthError) as e:
        eng.eval_batch_device([chain])
    assert e.value.status == -7
    chain32 = ("and", ("atom", 0), ("atom", 1))
    for _ in range(31):
        chain32 = ("not", chain32)
    assert np.array_equal(eng.eval_batch_device([chain32]), Oracle(kb).coverages([chain32]))


def test_errors(gpu):
    """Each invalid node is reported with its hypothesis and node by the count
    pass; nothing is evaluated (the counts keep their sentinel)."""
    torch = gpu
    cfg = synth.small_config(n=2000, n_concepts=6, n_roles=2, cap=8, n_data=2, seed_index=2100)
    kb = synth.make_kb(cfg)
    eng = hthedl.Engine(kb)
    good = [_node("atom", arg=1)]
    nan = int(np.float32(np.nan).view(np.uint32))
    cases = [
        ([_node("atom", arg=6)], [], -2, "concept"),
        ([_node("atom", arg=0), _node("not", child=1)], [], -5, "child"),
        ([_node("atom", arg=0), _node("exists", arg=2, child=0)], [], -2, "role"),
        ([_node("atom", arg=0), _node("exists", inv=2, arg=0, child=0)], [], -1, "inv"),
        ([_node("atom", arg=0), _node("atleast", arg=0, child=0, q=1 << 31)], [], -2, "n >"),
        ([_node("dge", arg=2, q=0)], [], -2, "property"),
        ([_node("dle", arg=0, q=nan)], [], -1, "NaN"),
        ([_node("nge", arg=0, q=0)], [], -7, "concrete"),
        ([_node("set", arg=0)], [], -2, "set row"),
        ([(99, 0, 0, 0, 0, 0)], [], -1, "unknown op"),
        ([_node("atom", arg=0), _node("and", arity=3, child=0)], [0, 0], -2, "children range"),
        ([_node("atom", arg=0), _node("or", arity=2, child=0)], [0, 1], -5, "child"),
    ]
    counts = torch.full((2, 2), -7, dtype=torch.int32, device="cuda")
    for nodes, ch, status, word in cases:
        enc = _batch([good, nodes], [[], ch])
        d = eng.upload_batch(encoded=enc)
        with pytest.raises(hthedl.HthError) as e:
            eng.eval_batch_device(device_batch=d, counts=counts)
        assert e.value.status == status, (nodes, str(e.value))
        assert "hypothesis 1 node" in str(e.value) and word in str(e.value), str(e.value)
    assert (counts.cpu().numpy() == -7).all()
    # offsets: empty hypothesis, decreasing, past the node array
    d_nodes, _, d_ch = eng.upload_batch(encoded=_batch([good, good], [[], []]))
    for offs, status in (([0, 1, 1], -5), ([0, 2, 1], -1), ([0, 1, 3], -1)):
        d_offs = torch.tensor(offs, dtype=torch.int32, device="cuda")
        with pytest.raises(hthedl.HthError) as e:
            eng.eval_batch_device(device_batch=(d_nodes, d_offs, d_ch), counts=counts)
        assert e.value.status == status, (offs, str(e.value))
    eng.ensure_plan_scratch(2)
    with pytest.raises(hthedl.HthError) as e:
        hthedl.hth_dplan_create(eng.handle, d_nodes, 2, d_offs, 0, None, 0, eng.dp_scratch, eng.dp_scratch_bytes)
    assert e.value.status == -2
    need = hthedl.hth_dplan_scratch_bytes(eng.handle, 2)
    assert need <= eng.dp_scratch_bytes
    for scratch, nbytes, status in ((eng.dp_scratch, need - 1, -3), (eng.dp_scratch[8:], need, -1)):
        with pytest.raises(hthedl.HthError) as e:
            hthedl.hth_dplan_create(eng.handle, d_nodes, 2, d_offs, 1, None, 0, scratch, nbytes)
        assert e.value.status == status


def test_chunks_relaunch_and_workspace(gpu):
    """Chunks of one uploaded batch (the offsets pointer advanced), a plan
    launched twice, and the workspace checks."""
    torch = gpu
    cfg = synth.small_config(n=8000, n_concepts=16, n_roles=3, cap=64, n_data=2, n_pos=1000, n_neg=1000,
                             n_hyps=300, hyp_depth=5, seed_index=2200)
    kb = synth.make_kb(cfg)
    hyps = synth.make_hypotheses(cfg, kb)
    want = Oracle(kb).coverages(hyps)
    eng = hthedl.Engine(kb, max_hyps=len(hyps))
    d = eng.upload_batch(hyps)
    for chunk in (1, 37, 300):
        assert np.array_equal(eng.eval_batch_device(device_batch=d, chunk=chunk), want), chunk
    d_nodes, d_offs, d_ch = d
    n_nodes = d_nodes.shape[0] // 16
    eng.ensure_plan_scratch(n_nodes)
    plan, nb = hthedl.hth_dplan_create(eng.handle, d_nodes, n_nodes, d_offs[100:], 50, d_ch, d_ch.shape[0],
                                       eng.dp_scratch, eng.dp_scratch_bytes)
    try:
        ws = torch.empty(nb + 512, dtype=torch.uint8, device="cuda")
        out = torch.empty((50, 2), dtype=torch.int32, device="cuda")
        for _ in range(2):
            out.fill_(-1)
            hthedl.hth_dplan_launch(plan, ws, nb, out)
            assert np.array_equal(out.cpu().numpy().view(np.uint32), want[100:150])
        with pytest.raises(hthedl.HthError) as e:
            hthedl.hth_dplan_launch(plan, ws, nb - 1, out)
        assert e.value.status == -3
        with pytest.raises(hthedl.HthError) as e:
            hthedl.hth_dplan_launch(plan, ws[8:], nb, out)
        assert e.value.status == -1
    finally:
        hthedl.hth_dplan_destroy(plan)


@pytest.mark.parametrize("tuning", [dict(group_min=0), dict(group_k=8), dict(group_min=1, xcd_local=0),
                                    dict(t_segment_kb=16), dict(t_compact=0, unroll=8)])
def test_schedules(tuning):
    """Device plans under other schedules: every role node alone, narrow
    shared passes, single-node passes, chip-wide passes, passes cut by T row,
    full-width T rows.  The count pass's bucket counts decide the shared
    passes; the emit pass fills their members in any order."""
    cfg = synth.small_config(n=30000, n_concepts=32, n_roles=3, s=1.4, cap=400, n_data=2, n_pos=3000,
                             n_neg=3000, n_hyps=700, hyp_depth=5, seed_index=2300)
    kb = synth.make_kb(cfg)
    hyps = synth.make_hypotheses(cfg, kb)
    eng = hthedl.Engine(kb, max_hyps=len(hyps))
    hthedl.hth_kb_set_tuning(eng.handle, **tuning)
    check_device(kb, hyps, f"schedule {tuning}", eng=eng)


def test_plans_keep_their_schedule(gpu):
    """A compiled plan (hth_plan_*) and a device plan (hth_dplan_*) run with
    the schedule they were laid out for, whatever hth_kb_set_tuning did since:
    passes cut by T row need a partial-count area that only a plan created
    with the cut has."""
    torch = gpu
    cfg = synth.small_config(n=30000, n_concepts=32, n_roles=3, s=1.4, cap=400, n_data=2, n_pos=3000,
                             n_neg=3000, n_hyps=300, hyp_depth=4, seed_index=2400)
    kb = synth.make_kb(cfg)
    hyps = synth.make_hypotheses(cfg, kb)
    want = Oracle(kb).coverages(hyps)
    eng = hthedl.Engine(kb, max_hyps=len(hyps))
    nodes, offs, ch = hthedl.encode_batch(hyps)
    d_nodes, d_offs, d_ch = eng.upload_batch(encoded=(nodes, offs, ch))
    out = torch.empty((len(hyps), 2), dtype=torch.int32, device="cuda")
    for at_create, at_launch in ((dict(t_segment_kb=0, region_reg=2), dict(t_segment_kb=64, region_reg=0)),
                                 (dict(t_segment_kb=64, region_reg=0), dict(t_segment_kb=0, region_reg=4))):
        hthedl.hth_kb_set_tuning(eng.handle, **at_create)
        plan, nb = hthedl.hth_plan_create(eng.handle, nodes, offs, ch)
        eng.ensure_plan_scratch(nodes.shape[0])
        dplan, dnb = hthedl.hth_dplan_create(eng.handle, d_nodes, nodes.shape[0], d_offs, len(hyps), d_ch,
                                             d_ch.shape[0], eng.dp_scratch, eng.dp_scratch_bytes)
        hthedl.hth_kb_set_tuning(eng.handle, **at_launch)
        try:
            ws = torch.empty(max(nb, dnb), dtype=torch.uint8, device="cuda")
            hthedl.hth_plan_upload(plan, ws, nb)
            out.fill_(-1)
            hthedl.hth_plan_launch(plan, ws, nb, out)
            assert np.array_equal(out.cpu().numpy().view(np.uint32), want), at_create
            out.fill_(-1)
            hthedl.hth_dplan_launch(dplan, ws, dnb, out)
            assert np.array_equal(out.cpu().numpy().view(np.uint32), want), at_create
        finally:
            hthedl.hth_plan_destroy(plan)
            hthedl.hth_dplan_destroy(dplan)


def test_shared_thresholds():
    """Identical threshold leaves across the batch share one task and row
    (hash-consed by the count pass); the same value under another comparison,
    -0.0 against +0.0, infinities and 40 thresholds on one property (two
    column passes) stay distinct where they must."""
    cfg = synth.small_config(n=9000, n_concepts=8, n_roles=2, cap=20, n_data=3, n_pos=1500, n_neg=1500,
                             seed_index=2500)
    kb = synth.make_kb(cfg)
    rng = np.random.default_rng(25)
    vals = [float(v) for v in kb.deciles[1]] + [0.0, -0.0, float("inf"), float("-inf")]
    vals += [float(v) for v in np.float32(rng.normal(size=30))]
    leaves = [(op, p, t) for p in (0, 1) for t in vals for op in ("dge", "dle", "deq")]
    hyps = []
    for _ in range(900):
        a, b = leaves[int(rng.integers(len(leaves)))], leaves[int(rng.integers(len(leaves)))]
        k = int(rng.integers(3))
        hyps.append(a if k == 0 else ("and", a, b) if k == 1 else ("exists", 0, 1, ("or", a, ("not", b))))
    check_device(kb, hyps, "shared thresholds", chunk=400)


def test_device_candidates(gpu):
    """Added-conjunct candidates drawn and written on the device equal the CPU
    reference's specs and node arrays bit for bit, and their device plans
    cover what the oracle gives for parent and conjunct."""
    import torch
    from tests import conjunct_ref
    cfg = synth.small_config(n=20000, n_concepts=24, n_roles=4, s=1.5, cap=100, n_data=3,
                             n_pos=2000, n_neg=2000, seed_index=2600)
    kb = synth.make_kb(cfg)
    o = Oracle(kb)
    parents = synth.make_hypotheses(cfg, kb, count=7, depth=3)
    eng = hthedl.Engine(kb)
    table = torch.zeros((len(parents), eng.S), dtype=torch.int64, device="cuda")
    nodes, offs, ch = hthedl.encode_batch(parents)
    eng.ensure_workspace(hthedl.hth_batch_workspace_bytes(eng.handle, nodes, offs, ch))
    cnt = torch.empty((len(parents), 2), dtype=torch.int32, device="cuda")
    hthedl.hth_eval_batch_sets(eng.handle, nodes, offs, ch, eng.ws, eng.ws_bytes, table, cnt)
    hthedl.hth_kb_set_sets(eng.handle, table, len(parents))
    rows = np.array([3, 0, 5, 1, 2, 6, 4], dtype=np.uint32)
    for seed, per in ((2412, 41), (7, 1), (1 << 63, 300)):
        d_specs, batch = eng.conjunct_candidates(rows, per, seed, kb.deciles)
        specs = d_specs.cpu().numpy().view(hthedl.CONJ_DTYPE)
        want = conjunct_ref.draw(seed, rows, per, kb.n_concepts, kb.n_roles, kb.n_data, kb.deciles)
        assert np.array_equal(specs, want), seed
        wn, wo, wc = conjunct_ref.conjoin(want)
        got_nodes = batch[0].cpu().numpy().view(hthedl.NODE_DTYPE)
        assert np.array_equal(got_nodes, wn) and np.array_equal(batch[1].cpu().numpy().view(np.uint32), wo)
        assert np.array_equal(batch[2].cpu().numpy().view(np.uint32), wc)
        full = [("and", parents[int(c["parent"])], hthedl.conjunct_tuple(c)) for c in specs]
        got = eng.eval_batch_device(device_batch=batch)
        assert np.array_equal(got, o.coverages(full)), seed
        assert np.array_equal(eng.eval_batch(None, encoded=(wn, wo, wc)), got)
    # host hypotheses in front of the candidates, one plan for both
    front = synth.make_hypotheses(cfg, kb, count=50, depth=3)
    enc = hthedl.encode_batch(front)
    d_specs, batch = eng.conjunct_candidates(rows, 9, 5, kb.deciles, before=enc, count=60)
    specs = d_specs.cpu().numpy().view(hthedl.CONJ_DTYPE)
    assert specs.shape[0] == 63 and np.array_equal(specs, conjunct_ref.draw(5, rows, 9, kb.n_concepts, kb.n_roles,
                                                                             kb.n_data, kb.deciles))
    wn, wo, wc = conjunct_ref.conjoin(specs[:60], enc[0].shape[0], enc[2].shape[0])
    assert np.array_equal(batch[0].cpu().numpy().view(hthedl.NODE_DTYPE), np.concatenate([enc[0], wn]))
    assert np.array_equal(batch[1].cpu().numpy().view(np.uint32), np.concatenate([enc[1][:-1], wo]))
    assert np.array_equal(batch[2].cpu().numpy().view(np.uint32), np.concatenate([enc[2], wc]))
    both = front + [("and", parents[int(c["parent"])], hthedl.conjunct_tuple(c)) for c in specs[:60]]
    assert np.array_equal(eng.eval_batch_device(device_batch=batch), o.coverages(both))
    # a kind outside the family is rejected by the plan's count pass
    bad = want.copy()
    bad["kind"][5] = 9
    d_bad = torch.from_numpy(bad.view(np.uint8)).cuda()
    n = bad.shape[0]
    bn = torch.empty(16 * 4 * n, dtype=torch.uint8, device="cuda")
    bo = torch.empty(n + 1, dtype=torch.int32, device="cuda")
    bc = torch.empty(2 * n, dtype=torch.int32, device="cuda")
    hthedl.hth_conjoin(d_bad, n, bn, bo, bc)
    with pytest.raises(hthedl.HthError) as e:
        eng.eval_batch_device(device_batch=(bn, bo, bc))
    assert e.value.status == -1 and "hypothesis 5 node 1" in str(e.value)
    hthedl.hth_kb_set_sets(eng.handle, None, 0)
    # a KB without properties draws no thresholds
    cfg0 = synth.small_config(n=3000, n_concepts=9, n_roles=2, n_data=0, n_pos=300, n_neg=300, seed_index=2601)
    kb0 = synth.make_kb(cfg0)
    eng0 = hthedl.Engine(kb0)
    t0 = torch.full((2, eng0.S), -1, dtype=torch.int64, device="cuda")   # both parents: every individual
    hthedl.hth_kb_set_sets(eng0.handle, t0, 2)
    d0, b0 = eng0.conjunct_candidates(np.array([1, 0], np.uint32), 60, 31, None)
    s0 = d0.cpu().numpy().view(hthedl.CONJ_DTYPE)
    assert np.array_equal(s0, conjunct_ref.draw(31, [1, 0], 60, kb0.n_concepts, kb0.n_roles, 0, kb0.deciles))
    full0 = [("and", ("top",), hthedl.conjunct_tuple(c)) for c in s0]
    assert np.array_equal(eng0.eval_batch_device(device_batch=b0), Oracle(kb0).coverages(full0))
    hthedl.hth_kb_set_sets(eng0.handle, None, 0)


def test_hash_consing_shares_equal_subexpressions():
    """A batch repeated twenty times plans exactly the passes of the batch
    alone: every copy of a subexpression finds the first one's representative."""
    cfg = synth.small_config(n=30000, n_concepts=32, n_roles=3, s=1.4, cap=400, n_data=2, n_pos=3000,
                             n_neg=3000, n_hyps=60, hyp_depth=5, seed_index=2700)
    kb = synth.make_kb(cfg)
    hyps = synth.make_hypotheses(cfg, kb)
    eng = hthedl.Engine(kb, max_hyps=20 * len(hyps))
    launches = {}
    for reps in (1, 20):
        batch = hyps * reps
        eng.eval_batch_device(batch)
        hthedl.hth_profile_begin(eng.handle)
        got = eng.eval_batch_device(batch)
        prof = hthedl.hth_profile_end(eng.handle)
        launches[reps] = [prof[k]["launches"] for k in (0, 2, 3, 4)]   # thresholds, roles, T builds, passes
        assert np.array_equal(got, np.tile(Oracle(kb).coverages(hyps), (reps, 1)))
    say(f"[devplan] launches alone / repeated: {launches}")
    assert launches[1] == launches[20]


ROLE_OPS = ("exists", "forall", "atleast", "atmost", "exactly")


def _distinct(hyps):
    """Distinct role subexpressions and thresholds of a batch, with the deepest
    role nesting (equality of the tuple forms: what hash-consing must find)."""
    roles, thr = set(), set()

    def walk(h):
        if h[0] in ROLE_OPS:
            roles.add(h)
            return walk(h[-1]) + 1
        if h[0] in ("dge", "dle", "deq"):
            thr.add((h[0], h[1], np.float32(h[2]).view(np.uint32).item()))
        if h[0] == "not":
            return walk(h[1])
        if h[0] in ("and", "or"):
            return max([walk(c) for c in h[1:]] + [0])
        return 0

    depth = max(walk(h) for h in hyps)
    return len(roles), len(thr), depth


def test_hash_consing_finds_every_shared_subtree(gpu):
    """Sized hypotheses whose subtrees come from a shared pool (the uneven
    batch's generator): the device plan holds exactly one role node per
    distinct role subexpression and one task per distinct threshold, and its
    levels are the deepest role nesting."""
    cfg = synth.small_config(n=20000, n_concepts=48, n_roles=4, s=1.5, cap=200, n_data=4, n_pos=2000,
                             n_neg=2000, seed_index=2800)
    kb = synth.make_kb(cfg)
    hyps = synth.make_sized_hypotheses(cfg, kb, count=3000)
    n_roles, n_thr, depth = _distinct(hyps)
    eng = hthedl.Engine(kb, max_hyps=len(hyps))
    nodes, offs, ch = hthedl.encode_batch(hyps)
    d_nodes, d_offs, d_ch = eng.upload_batch(encoded=(nodes, offs, ch))
    eng.ensure_plan_scratch(nodes.shape[0])
    plan, nb = hthedl.hth_dplan_create(eng.handle, d_nodes, nodes.shape[0], d_offs, len(hyps), d_ch, d_ch.shape[0],
                                       eng.dp_scratch, eng.dp_scratch_bytes)
    try:
        info = hthedl.hth_dplan_stats(plan)
    finally:
        hthedl.hth_dplan_destroy(plan)
    say(f"[devplan] pool batch: {info}; distinct role subexpressions {n_roles}, thresholds {n_thr}, depth {depth}")
    assert info["role_nodes"] == n_roles and info["thresholds"] == n_thr and info["levels"] == depth
    got = eng.eval_batch_device(encoded=(nodes, offs, ch))
    assert np.array_equal(got, Oracle(kb).coverages(hyps))
