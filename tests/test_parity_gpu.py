"""GPU parity: coverage and instance sets from the HIP path equal the oracle's,
bit for bit, through the C ABI (plain one-at-a-time and batched)."""
import sys

import numpy as np
import pytest

from oracle import Oracle
from paper_2412_00802_amd import hthedl, synth
from tests.test_golden import load_c1_counts

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "the gpu tests need an MI355X"
    hthedl.lib()
    return torch


def check(kb, hyps, plain=True, batch=True, label=""):
    say(f"[parity] {label}: N={kb.n} hyps={len(hyps)}")
    eng = hthedl.Engine(kb, max_hyps=max(1, len(hyps)))
    want = Oracle(kb).coverages(hyps)
    if batch:
        got = eng.eval_batch(hyps)
        bad = np.flatnonzero((got != want).any(axis=1))
        assert bad.size == 0, f"batch mismatch at {bad[:5]}: {hyps[bad[0]]} got {got[bad[0]]} want {want[bad[0]]}"
    if plain:
        got = eng.eval_plain(hyps)
        bad = np.flatnonzero((got != want).any(axis=1))
        assert bad.size == 0, f"plain mismatch at {bad[:5]}: {hyps[bad[0]]} got {got[bad[0]]} want {want[bad[0]]}"
    return eng


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 127, 4095, 4097, 20011])
def test_tail_sizes(n):
    cfg = synth.small_config(n=n, n_concepts=10, n_roles=3, cap=min(16, max(1, n)),
                             n_pos=max(1, n // 5), n_neg=n // 5, n_hyps=48, seed_index=300 + n % 97)
    kb = synth.make_kb(cfg)
    check(kb, synth.make_hypotheses(cfg, kb), label=f"tail n={n}")


@pytest.mark.parametrize("seed", range(4))
def test_small_workloads(seed):
    cfg = synth.small_config(n=3000 + 517 * seed, n_concepts=24, n_roles=4, s=1.2 + 0.3 * seed,
                             cap=[8, 64, 300, 1000][seed], n_pos=400, n_neg=300, n_hyps=96,
                             hyp_depth=5, seed_index=400 + seed)
    kb = synth.make_kb(cfg)
    check(kb, synth.make_hypotheses(cfg, kb), label=f"small seed={seed}")


def test_c1_full_against_golden():
    cfg = synth.CONFIGS["c1"]
    kb = synth.make_kb(cfg)
    hyps = synth.make_hypotheses(cfg, kb)
    want = load_c1_counts()
    eng = hthedl.Engine(kb, max_hyps=len(hyps))
    np.testing.assert_array_equal(eng.eval_batch(hyps), want)
    np.testing.assert_array_equal(eng.eval_plain(hyps), want)


def test_instance_bits():
    cfg = synth.small_config(n=5000, n_concepts=16, n_roles=3, cap=40, n_hyps=40, seed_index=501)
    kb = synth.make_kb(cfg)
    hyps = synth.make_hypotheses(cfg, kb)
    o = Oracle(kb)
    eng = hthedl.Engine(kb)
    for h in hyps + [("not", ("top",)), ("forall", 0, 1, ("bot",)), ("atom", 3)]:
        (p, q), bits = eng.eval_one(h, instances=True)
        np.testing.assert_array_equal(bits, o.ext_bits(h))
        assert (p, q) == o.coverage(h)


def skew_kb(n=6000, e=5000, seed=0):
    """The paper's two restriction datasets: role 0 'single subject' (every
    assertion has the same subject), role 1 'unique subject' (all subjects
    distinct), role 2 empty, role 3 with self-loops."""
    rnd = np.random.default_rng(seed)
    single = [(17, int(t)) for t in rnd.choice(n, size=e, replace=False)]
    subj = rnd.choice(n, size=e, replace=False)
    unique = [(int(s), int(t)) for s, t in zip(subj, rnd.integers(0, n, size=e))]
    loops = [(x, x) for x in range(0, n, 3)] + [(x, (x + 1) % n) for x in range(0, n, 5)]
    concepts = [list(rnd.choice(n, size=n // 2, replace=False)),
                list(rnd.choice(n, size=n // 50, replace=False)),
                list(range(n))]
    data = rnd.standard_normal((1, n)).astype(np.float32)
    data[0, ::7] = np.nan
    data[0, 5] = -0.0
    data[0, 6] = 0.0
    return synth.kb_from_edges(n, concepts, [single, unique, [], loops], data,
                               pos=list(range(0, n, 2)), neg=list(range(1, n, 3)))


def role_zoo(n_roles, n_concepts):
    fillers = [("atom", 0), ("atom", 1), ("not", ("atom", 1)), ("top",), ("bot",),
               ("and", ("atom", 0), ("dge", 0, 0.0)), ("or", ("atom", 1), ("dle", 0, -0.0))]
    hs = []
    for r in range(n_roles):
        for inv in (0, 1):
            for c in fillers:
                hs.append(("exists", r, inv, c))
                hs.append(("forall", r, inv, c))
                for k in (0, 1, 2, 3, 7, 1000, 4999, 5000, 5001, 2 ** 31 - 1):
                    hs.append(("atleast", k, r, inv, c))
                    hs.append(("atmost", k, r, inv, c))
                hs.append(("exactly", 1, r, inv, c))
                hs.append(("exactly", 0, r, inv, c))
    return hs


def test_skewed_and_degenerate_roles():
    kb = skew_kb()
    hs = role_zoo(4, 3)
    hs += [("and",), ("or",), ("dge", 0, float("inf")), ("dge", 0, float("-inf")),
           ("dle", 0, float("inf")), ("dle", 0, -0.0), ("dge", 0, 0.0),
           ("exists", 0, 0, ("exists", 0, 1, ("atom", 0))),
           ("forall", 1, 1, ("atmost", 0, 0, 0, ("atom", 1))),
           ("not", ("and", ("top",), ("not", ("bot",))))]
    check(kb, hs, label="skew")


def test_shared_subexpressions_batch():
    """Heavy sharing inside one batch: every hypothesis reuses the same role nodes."""
    cfg = synth.small_config(n=8000, n_concepts=12, n_roles=2, cap=50, seed_index=610)
    kb = synth.make_kb(cfg)
    base = [("exists", 0, 0, ("atom", a)) for a in range(6)] + [("atmost", 2, 1, 1, ("atom", 7))]
    hs = []
    for i in range(120):
        a, b = base[i % len(base)], base[(i * 5 + 1) % len(base)]
        hs.append(("and", a, ("not", b)) if i % 3 else ("or", a, ("forall", 1, 0, b)))
    hs += hs[:10]   # duplicate hypotheses
    check(kb, hs, plain=False, label="shared")


def _sentinel(torch, k):
    return torch.full((k, 2), 12345, dtype=torch.int32, device="cuda")


def test_errors_leave_outputs_untouched(gpu):
    torch = gpu
    cfg = synth.small_config(n=500, seed_index=700)
    kb = synth.make_kb(cfg)
    eng = hthedl.Engine(kb)
    bad = [
        (("atom", 10 ** 6), hthedl.STATUS[-2]),
        (("exists", 99, 0, ("atom", 0)), hthedl.STATUS[-2]),
        (("dge", 0, float("nan")), hthedl.STATUS[-1]),
        (("dge", 55, 0.0), hthedl.STATUS[-2]),
    ]
    for h, status in bad:
        out = _sentinel(torch, 1)
        with pytest.raises(hthedl.HthError) as e:
            eng.eval_one(h, counts=out[0])
        assert status in str(e.value)
        assert out.cpu().numpy().tolist() == [[12345, 12345]]
    # child after parent: not postfix
    nodes = np.array([(3, 0, 0, 0, 1, 0), (2, 0, 0, 0, 0, 0)], dtype=hthedl.NODE_DTYPE)
    out = _sentinel(torch, 1)
    with pytest.raises(hthedl.HthError) as e:
        hthedl.hth_eval_one(eng.handle, nodes, np.zeros(0, np.uint32), eng.ws, eng.ws_bytes,
                            None, out[0])
    assert "HTH_E_PLAN" in str(e.value)
    # workspace too small
    nodes, ch = hthedl.encode_one(("exists", 0, 0, ("and", ("atom", 1), ("atom", 2))))
    with pytest.raises(hthedl.HthError) as e:
        hthedl.hth_eval_one(eng.handle, nodes, ch, eng.ws, 256, None, out[0])
    assert "HTH_E_NOMEM" in str(e.value)
    assert out.cpu().numpy().tolist() == [[12345, 12345]]


def test_kb_validation(gpu):
    kb = synth.kb_from_edges(100, [[1, 2, 3]], [[(0, 5), (0, 9), (4, 2)]])
    hthedl.Engine(kb)   # valid
    bad = synth.kb_from_edges(100, [[1, 2, 3]], [[(0, 5), (0, 9), (4, 2)]])
    bad.role_targets = bad.role_targets.copy()
    bad.role_targets[1] = 5          # duplicate target in row 0
    with pytest.raises(hthedl.HthError) as e:
        hthedl.Engine(bad)
    assert "strictly increasing" in str(e.value)
    bad.role_targets[1] = 100        # out of range
    with pytest.raises(hthedl.HthError) as e:
        hthedl.Engine(bad)
    assert "outside" in str(e.value)
    pad = synth.kb_from_edges(100, [[1, 2, 3]], [[(0, 5)]])
    pad.concept_bits = pad.concept_bits.copy()
    pad.concept_bits[0, 1] |= np.uint64(1) << np.uint64(40)   # individual 104 >= N
    with pytest.raises(hthedl.HthError) as e:
        hthedl.Engine(pad)
    assert "padding" in str(e.value)


def test_bit_rows_must_be_16_byte_aligned(gpu):
    """Example rows and the set table are read with 16-byte loads: a buffer
    8 bytes off is refused (HTH_E_INVALID) and the previous rows stay."""
    torch = gpu
    kb = synth.kb_from_edges(100, [[1, 2, 3]], [[(0, 5), (0, 9), (4, 2)]])
    eng = hthedl.Engine(kb)
    want = eng.eval_batch([("atom", 0), ("exists", 0, 0, ("atom", 0))])
    buf = torch.zeros(eng.S + 2, dtype=torch.int64, device="cuda")
    off = buf[1:1 + eng.S]
    with pytest.raises(hthedl.HthError) as e:
        hthedl.hth_kb_set_examples(eng.handle, off, off)
    assert "16-byte" in str(e.value)
    with pytest.raises(hthedl.HthError) as e:
        hthedl.hth_kb_set_sets(eng.handle, off, 1)
    assert "16-byte" in str(e.value)
    assert np.array_equal(eng.eval_batch([("atom", 0), ("exists", 0, 0, ("atom", 0))]), want)


def test_kb_validation_heavy_rows(gpu):
    """Rows above the heavy-row threshold are checked chunk by chunk at load:
    an unsorted pair, a duplicate across a chunk boundary and a target out of
    range are each found; a valid heavy row loads."""
    n = 20000
    row = np.arange(0, 3 * 4096 + 10) + 50                # subject 7, degree 12298: 4 chunks
    edges = [(7, int(t)) for t in row] + [(8, 1), (8, 3)]
    good = synth.kb_from_edges(n, [[1, 2, 3]], [edges])
    hthedl.Engine(good).close()
    off0 = int(good.role_offsets[0, 7])
    for pos, val, msg in ((100, 50 + 99, "strictly increasing"),      # equals its predecessor
                          (4096, 50 + 4095, "strictly increasing"),   # first of chunk 1 = last of chunk 0
                          (8191, 50 + 8193, "strictly increasing"),   # last of chunk 1 above its successor
                          (5000, n, "outside"),
                          (12297, -1, "outside")):
        bad = synth.kb_from_edges(n, [[1, 2, 3]], [edges])
        bad.role_targets = bad.role_targets.copy()
        bad.role_targets[off0 + pos] = val
        with pytest.raises(hthedl.HthError) as e:
            hthedl.Engine(bad)
        assert msg in str(e.value), (pos, val)


def test_max_degrees_and_inverse(gpu):
    cfg = synth.small_config(n=7000, n_roles=3, cap=200, seed_index=800)
    kb = synth.make_kb(cfg)
    eng = hthedl.Engine(kb)
    for r in range(3):
        off = kb.role_offsets[r]
        tg = kb.role_targets[off[0]:off[-1]]
        assert hthedl.hth_kb_max_degree(eng.handle, r, 0) == int(np.diff(off).max())
        assert hthedl.hth_kb_max_degree(eng.handle, r, 1) == int(np.bincount(tg, minlength=kb.n).max())


def _distinct_role_nodes(m, n_concepts, role, inv, seed):
    rnd = np.random.default_rng(seed)
    hs, seen = [], set()
    ops = ["exists", "forall", "atleast", "atmost", "exactly"]
    while len(hs) < m:
        op = ops[int(rnd.integers(0, 5))]
        a, b = int(rnd.integers(0, n_concepts)), int(rnd.integers(0, n_concepts))
        c = ("atom", a) if rnd.random() < 0.5 else ("or", ("atom", a), ("not", ("atom", b)))
        h = (op, role, inv, c) if op in ("exists", "forall") else (op, int(rnd.integers(0, 4)), role, inv, c)
        if h not in seen:
            seen.add(h)
            hs.append(h)
    return hs


@pytest.mark.parametrize("m", [4, 8, 9, 16, 17, 32, 33, 64, 65, 130])
def test_group_widths(m):
    """A (role, direction, level) bucket of m role nodes: shared passes of every
    T width and split groups, next to the single-node path."""
    cfg = synth.small_config(n=9000, n_concepts=40, n_roles=2, s=1.3, cap=400, n_pos=900,
                             n_neg=800, seed_index=950)
    kb = synth.make_kb(cfg)
    hs = _distinct_role_nodes(m, 40, 1, m % 2, seed=m)
    hs += [("and", h, ("atom", i % 40)) for i, h in enumerate(hs[: m // 2])]
    check(kb, hs, label=f"group m={m}")


@pytest.mark.parametrize("seg_kb", [0, 16, 40, 64, 128, 100000])
def test_segmented_shared_passes(seg_kb):
    """Shared passes cut into 2..4 passes over T-row ranges (partial counts
    carried between them) give the oracle's counts for every T width, full and
    compact T rows, dense and sparse directions, and nested role nodes; sizes
    whose cut would need more than four passes run as one pass."""
    cfg = synth.small_config(n=30011, n_concepts=40, n_roles=4, s=1.4, cap=600, n_pos=3000, n_neg=2500,
                             n_hyps=200, hyp_depth=5, seed_index=1700)
    kb = synth.make_kb(cfg)
    hs = synth.make_hypotheses(cfg, kb)
    for m, role, inv in ((70, 0, 0), (40, 1, 1), (20, 2, 0), (9, 3, 1)):
        hs += _distinct_role_nodes(m, 40, role, inv, seed=m + seg_kb)
    hs += [("exists", 0, 0, ("atleast", 2, 1, 1, ("atom", i))) for i in range(12)]
    want = Oracle(kb).coverages(hs)
    eng = hthedl.Engine(kb)
    hthedl.hth_kb_set_tuning(eng.handle, t_segment_kb=seg_kb)
    for compact in (1, 0):
        hthedl.hth_kb_set_tuning(eng.handle, t_compact=compact)
        got = eng.eval_batch(hs)
        bad = np.flatnonzero((got != want).any(axis=1))
        assert bad.size == 0, f"t_segment_kb={seg_kb} compact={compact}: {hs[bad[0]]} {got[bad[0]]} {want[bad[0]]}"


@pytest.mark.parametrize("push_pct", [0, 3, 100])
def test_pushed_restrictions(push_pct):
    """Single existential restrictions (and their negations, via forall and
    at-most-0) over sparse atomic concepts, evaluated from the concept's
    members over the opposite direction: the counts equal the oracle's at every
    push threshold, in both directions, next to nodes that cannot be pushed
    (computed children, at-least-2, a direction with heavy rows)."""
    cfg = synth.small_config(n=40013, n_concepts=48, n_roles=3, s=1.6, cap=300, n_pos=4000, n_neg=3500,
                             n_hyps=120, hyp_depth=4, seed_index=1800)
    kb = synth.make_kb(cfg)
    rnd = np.random.default_rng(18)
    hs = synth.make_hypotheses(cfg, kb)
    for a in range(48):
        r, inv = a % 3, (a // 3) % 2
        hs += [("exists", r, inv, ("atom", a)), ("forall", r, inv, ("not", ("atom", a))),
               ("atmost", 0, r, inv, ("atom", a)), ("atleast", 2, r, inv, ("atom", a)),
               ("and", ("atom", int(rnd.integers(0, 48))), ("exists", r, 1 - inv, ("atom", a)))]
    hs += [("exists", 0, 0, ("exists", 1, 1, ("atom", 7))), ("not", ("exists", 2, 1, ("atom", 40)))]
    want = Oracle(kb).coverages(hs)
    eng = hthedl.Engine(kb, max_hyps=len(hs))
    hthedl.hth_kb_set_tuning(eng.handle, push_pct=push_pct)
    got = eng.eval_plain(hs)
    bad = np.flatnonzero((got != want).any(axis=1))
    assert bad.size == 0, f"plain, push {push_pct}%: {hs[bad[0]]} {got[bad[0]]} {want[bad[0]]}"
    hthedl.hth_kb_set_tuning(eng.handle, group_min=0)
    got = eng.eval_batch(hs)
    bad = np.flatnonzero((got != want).any(axis=1))
    assert bad.size == 0, f"batch, push {push_pct}%: {hs[bad[0]]} {got[bad[0]]} {want[bad[0]]}"
    o = Oracle(kb)
    for h in (("exists", 1, 0, ("atom", 45)), ("forall", 2, 1, ("not", ("atom", 46)))):
        (p, q), bits = eng.eval_one(h, instances=True)
        np.testing.assert_array_equal(bits, o.ext_bits(h))


def test_pushed_restrictions_skip_heavy_directions(monkeypatch):
    """No push over a direction with heavy rows: counted per subject there."""
    kb = heavy_kb()
    hs = [("exists", r, inv, ("atom", 1)) for r in (0, 1) for inv in (0, 1)]
    hs += [("forall", r, inv, ("not", ("atom", 1))) for r in (0, 1) for inv in (0, 1)]
    eng = hthedl.Engine(kb)
    hthedl.hth_kb_set_tuning(eng.handle, push_pct=100)
    assert np.array_equal(eng.eval_plain(hs), Oracle(kb).coverages(hs))


@pytest.mark.parametrize("n,edges", [(5000, 300), (70000, 4000), (130001, 60000)])
def test_sparse_roles(n, edges):
    """Most 64-subject words have no assertion: the passes visit the non-empty
    words only and the others hold the zero-count result (all ones for
    forall / at-most / exactly-0, zeros otherwise)."""
    cfg = synth.small_config(n=n, n_concepts=20, n_roles=3, s=1.4, cap=300, n_pos=n // 10,
                             n_neg=n // 10, n_hyps=80, hyp_depth=4, total_edges=edges,
                             seed_index=1400 + n % 89)
    kb = synth.make_kb(cfg)
    hs = synth.make_hypotheses(cfg, kb)
    hs += _distinct_role_nodes(70, 20, 0, 1, seed=n)
    hs += [("forall", 2, 0, ("atom", 1)), ("atmost", 0, 1, 1, ("atom", 2)), ("exactly", 0, 0, 0, ("atom", 3)),
           ("not", ("exists", 1, 0, ("top",)))]
    eng = check(kb, hs, label=f"sparse n={n}")
    o = Oracle(kb)
    for h in hs[-4:]:
        (_, bits) = eng.eval_one(h, instances=True)
        np.testing.assert_array_equal(bits, o.ext_bits(h))


def test_every_schedule_gives_identical_counts():
    """The autotuner's schedules change speed only: each one reproduces the
    oracle's coverage (and the autotuner itself checks them against each other)."""
    from paper_2412_00802_amd import autotune
    cfg = synth.small_config(n=30000, n_concepts=30, n_roles=4, s=1.5, cap=200, n_pos=3000, n_neg=3000,
                             n_hyps=300, hyp_depth=5, seed_index=1500)
    kb = synth.make_kb(cfg)
    hs = synth.make_hypotheses(cfg, kb) + synth.make_sized_hypotheses(cfg, kb, count=300)
    want = Oracle(kb).coverages(hs)
    eng = hthedl.Engine(kb)
    grid = autotune.candidates(kb.n) + [dict(group_min=0, group_k=64, xcd_local=1, t_budget_mb=64, unroll=8),
                                        dict(region_reg=1), dict(region_reg=4), dict(region_reg=0)]
    for cand in grid:
        hthedl.hth_kb_set_tuning(eng.handle, **cand)
        got = eng.eval_batch(hs)
        assert np.array_equal(got, want), cand
    best = autotune.autotune(eng, hs, grid=grid[:4], reps=1, cache=None)
    got = hthedl.hth_kb_get_tuning(eng.handle)
    assert {k: got[k] for k in best} == best
    with pytest.raises(hthedl.HthError):
        hthedl.hth_kb_set_tuning(eng.handle, group_k=65)


def _subtrees(h, out):
    """Distinct compound or data subtrees of h (atoms, top and bottom excluded)."""
    if h[0] in ("atom", "top", "bot"):
        return
    out.setdefault(h, len(out))
    if h[0] == "not":
        _subtrees(h[1], out)
    elif h[0] in ("and", "or"):
        for c in h[1:]:
            _subtrees(c, out)
    elif h[0] in ("exists", "forall", "atleast", "atmost", "exactly"):
        _subtrees(h[-1], out)


def _substitute(h, slot):
    if h in slot:
        return ("set", slot[h])
    if h[0] == "not":
        return ("not", _substitute(h[1], slot))
    if h[0] in ("and", "or"):
        return (h[0],) + tuple(_substitute(c, slot) for c in h[1:])
    if h[0] in ("exists", "forall", "atleast", "atmost", "exactly"):
        return h[:-1] + (_substitute(h[-1], slot),)
    return h


def test_set_table_leaves():
    """Instance sets written by hth_eval_batch_sets equal the oracle's, and
    hypotheses whose subtrees are replaced by set-table leaves cover exactly
    what the full hypotheses cover (plain and batched)."""
    import torch
    from paper_2412_00802_amd import search
    cfg = synth.small_config(n=20000, n_concepts=24, n_roles=4, s=1.5, cap=100, n_data=3,
                             n_pos=2000, n_neg=2000, seed_index=1600)
    kb = synth.make_kb(cfg)
    o = Oracle(kb)
    parents = synth.make_hypotheses(cfg, kb, count=40, depth=4)
    slot: dict = {}
    for p in parents:
        _subtrees(p, slot)
    subs = sorted(slot, key=slot.get)
    say(f"[parity] set table: {len(subs)} subtrees of {len(parents)} parents")
    eng = hthedl.Engine(kb)
    base = 5                                   # rows before `base` stay unused
    table = torch.full((base + len(subs), eng.S), -1, dtype=torch.int64, device="cuda")
    nodes, offs, ch = hthedl.encode_batch(subs)
    eng.ensure_workspace(hthedl.hth_batch_workspace_bytes(eng.handle, nodes, offs, ch))
    cnt = torch.empty((len(subs), 2), dtype=torch.int32, device="cuda")
    hthedl.hth_eval_batch_sets(eng.handle, nodes, offs, ch, eng.ws, eng.ws_bytes, table[base:], cnt)
    rows = table.cpu().numpy().view(np.uint64)
    assert np.array_equal(cnt.cpu().numpy().view(np.uint32), o.coverages(subs))
    for i, s in enumerate(subs):
        assert np.array_equal(rows[base + i, :eng.W], o.ext_bits(s)), s
        assert not rows[base + i, eng.W:].any()
    hthedl.hth_kb_set_sets(eng.handle, table, table.shape[0])
    slot = {s: base + i for i, s in enumerate(subs)}
    ref = search.Refiner(kb, np.random.default_rng(5))
    full = []
    for p in parents:
        full.extend(ref.refine(p, 12))
    cached = [_substitute(c, slot) for c in full]
    assert sum(c != f for c, f in zip(cached, full)) > len(full) // 2
    want = o.coverages(full)
    assert np.array_equal(eng.eval_batch(cached), want)
    assert np.array_equal(eng.eval_plain(cached[:60]), want[:60])
    # a refinement of every parent with the parent itself as one set leaf
    adds = [("and", ("set", slot[p]), ref.conjunct()) for p in parents if p in slot]
    want = o.coverages([("and", p, a[2]) for p, a in zip([p for p in parents if p in slot], adds)])
    assert np.array_equal(eng.eval_batch(adds), want)
    with pytest.raises(hthedl.HthError) as e:
        eng.eval_one(("set", table.shape[0]))
    assert e.value.status == -2
    hthedl.hth_kb_set_sets(eng.handle, None, 0)
    with pytest.raises(hthedl.HthError) as e:
        eng.eval_batch([("set", 0)])
    assert e.value.status == -2


def test_deep_regions_both_region_kernels():
    """Balanced and/or trees whose value stacks need 2..10 entries: the
    register-stack region kernel (up to six) and the LDS-stack kernel (deeper
    programs, or all programs when switched off) agree with the oracle."""
    cfg = synth.small_config(n=5000, n_concepts=64, n_roles=3, n_data=2, n_pos=800, n_neg=800,
                             seed_index=1700)
    kb = synth.make_kb(cfg)
    rng = np.random.default_rng(17)

    def tree(h, op="and"):
        if h == 0:
            u = rng.random()
            if u < 0.7:
                a = ("atom", int(rng.integers(0, 64)))
                return ("not", a) if rng.random() < 0.3 else a
            if u < 0.85:
                return ("exists", int(rng.integers(0, 3)), int(rng.integers(0, 2)), ("atom", int(rng.integers(0, 64))))
            return ("dge", 0, float(kb.deciles[0, int(rng.integers(0, 9))]))
        other = "or" if op == "and" else "and"
        return (op, tree(h - 1, other), tree(h - 1, other))

    hyps = [tree(h, op) for h in range(1, 11) for op in ("and", "or") for _ in range(3)]
    want = Oracle(kb).coverages(hyps)
    eng = hthedl.Engine(kb, max_nodes=4096)
    for reg in (1, 2, 4, 0):
        hthedl.hth_kb_set_tuning(eng.handle, region_reg=reg)
        assert np.array_equal(eng.eval_batch(hyps), want), reg
        assert np.array_equal(eng.eval_plain(hyps), want), reg


def test_compact_transposed_rows_on_sparse_roles():
    """Role directions whose objects are few: shared passes over T rows kept
    for the objects only (indexed by rank) equal the oracle, the full-row
    passes and the single-node passes, in both directions and every T width."""
    cfg = synth.small_config(n=70000, n_concepts=40, n_roles=3, s=1.4, cap=400, n_data=2, n_pos=5000,
                             n_neg=5000, seed_index=1800, total_edges=9000)
    kb = synth.make_kb(cfg)
    rng = np.random.default_rng(18)
    hyps = []
    for _ in range(700):
        r, inv = int(rng.integers(0, 3)), int(rng.integers(0, 2))
        c = ("atom", int(rng.integers(0, 40)))
        if rng.random() < 0.3:
            c = ("or", c, ("dle", 1, float(kb.deciles[1, int(rng.integers(0, 9))])))
        op = rng.choice(["exists", "forall", "atleast", "atmost"])
        hyps.append((op, r, inv, c) if op in ("exists", "forall") else (op, int(rng.integers(1, 4)), r, inv, c))
    want = Oracle(kb).coverages(hyps)
    eng = hthedl.Engine(kb)
    say(f"[parity] compact T: objects per direction {[hthedl.hth_kb_max_degree(eng.handle, r, 0) for r in range(3)]}")
    for k in (8, 16, 32, 64):
        for compact in (1, 0):
            hthedl.hth_kb_set_tuning(eng.handle, group_min=1, group_k=k, t_compact=compact)
            assert np.array_equal(eng.eval_batch(hyps), want), (k, compact)
    hthedl.hth_kb_set_tuning(eng.handle, group_min=0)
    assert np.array_equal(eng.eval_batch(hyps), want)


def test_plan_reuse_and_graph_replay():
    """A compiled plan launched repeatedly, and captured in a HIP graph and
    replayed with eager work in between, gives the oracle's counts every time
    (the counts are cleared by a kernel, not a memset)."""
    import torch
    cfg = synth.small_config(n=20000, n_concepts=30, n_roles=4, s=1.5, cap=200, n_pos=2500, n_neg=2500,
                             n_hyps=200, hyp_depth=5, seed_index=2000)
    kb = synth.make_kb(cfg)
    hyps = synth.make_hypotheses(cfg, kb)
    want = Oracle(kb).coverages(hyps)
    eng = hthedl.Engine(kb)
    nodes, offs, ch = hthedl.encode_batch(hyps)
    plan, nb = hthedl.hth_plan_create(eng.handle, nodes, offs, ch)
    try:
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
        hthedl.hth_plan_upload(plan, ws, nb)
        counts = torch.full((len(hyps), 2), -1, dtype=torch.int32, device="cuda")
        for _ in range(3):
            hthedl.hth_plan_launch(plan, ws, nb, counts)
            assert np.array_equal(counts.cpu().numpy().view(np.uint32), want)
        with pytest.raises(hthedl.HthError):
            hthedl.hth_plan_launch(plan, ws, nb - 256, counts)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            hthedl.hth_plan_launch(plan, ws, nb, counts, stream=torch.cuda.current_stream())
        other = hyps[:25]
        for rep in range(4):
            counts.fill_(-1)
            assert np.array_equal(eng.eval_batch(other), want[:25])      # eager work between replays
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert np.array_equal(counts.cpu().numpy().view(np.uint32), want), rep
        del g
    finally:
        hthedl.hth_plan_destroy(plan)


@pytest.mark.parametrize("region_reg", [1, 2, 0])
def test_grids_beyond_one_dispatch(region_reg):
    """70,000 root regions over 4M individuals need more work-items than one
    dispatch holds (about 17M blocks of 256 lanes at one word per lane): the
    launches are split, and the counts equal those of small batches and the
    oracle's."""
    cfg = synth.small_config(n=4_000_000, n_concepts=64, depth=4, n_roles=2, n_data=2, n_pos=100_000,
                             n_neg=100_000, seed_index=2100, total_edges=40_000)
    kb = synth.make_kb(cfg)
    rng = np.random.default_rng(21)
    ops = ("and", "or")
    hyps = []
    seen = set()
    while len(hyps) < 70_000:
        leaves = tuple(("not", ("atom", int(v))) if rng.random() < 0.5 else ("atom", int(v))
                       for v in rng.integers(0, 64, 3))
        h = (ops[int(rng.integers(0, 2))],) + leaves
        if h not in seen:
            seen.add(h)
            hyps.append(h)
    eng = hthedl.Engine(kb)
    hthedl.hth_kb_set_tuning(eng.handle, region_reg=region_reg)
    say(f"[parity] {len(hyps)} regions over N={kb.n}, region_reg={region_reg}")
    whole = eng.eval_batch(hyps)
    parts = eng.eval_batch(hyps, chunk=4096)
    assert np.array_equal(whole, parts)
    pick = rng.choice(len(hyps), size=40, replace=False)
    assert np.array_equal(whole[pick], Oracle(kb).coverages([hyps[i] for i in pick]))


def heavy_kb(n=60000, seed=7):
    """Roles whose rows straddle the heavy-row threshold: role 0 has subjects
    of degree 1025 .. 30000 (some sharing a word with light subjects, some in
    adjacent words) over light rows of degree 0..40; role 1 has a few objects
    with thousands of subjects (heavy rows of the inverse direction)."""
    rnd = np.random.default_rng(seed)
    edges0 = set()
    heavy = {64 * 3 + 5: 1025, 64 * 3 + 6: 2048, 64 * 3 + 63: 2049, 64 * 4: 4096, 64 * 9 + 31: 4097,
             64 * 200 + 1: 9000, n - 1: 30000, 64 * 500 + 2: 12288}
    for s, d in heavy.items():
        for t in rnd.choice(n, size=d, replace=False):
            edges0.add((s, int(t)))
    for s in range(0, n, 3):
        if s not in heavy:
            for t in rnd.choice(n, size=int(rnd.integers(0, 41)), replace=False):
                edges0.add((s, int(t)))
    edges1 = set()
    for obj, d in ((11, 5000), (12, 1500), (64 * 7, 20000)):
        for s in rnd.choice(n, size=d, replace=False):
            edges1.add((int(s), obj))
    for s in rnd.choice(n, size=20000):
        edges1.add((int(s), int(rnd.integers(0, n))))
    hit = np.zeros(n, bool)
    for s, t in edges0:
        if s in heavy:
            hit[t] = True
    concepts = [list(rnd.choice(n, size=n // 2, replace=False)),
                list(rnd.choice(n, size=n // 100, replace=False)),
                list(np.flatnonzero(~hit))]
    return synth.kb_from_edges(n, concepts, [sorted(edges0), sorted(edges1)], None,
                               pos=list(range(0, n, 2)), neg=list(range(1, n, 3)))


def heavy_zoo():
    fillers = [("atom", 0), ("atom", 1), ("atom", 2), ("not", ("atom", 2)), ("top",),
               ("atleast", 2, 1, 1, ("atom", 0))]
    hs = []
    for r in (0, 1):
        for inv in (0, 1):
            for c in fillers:
                hs.append(("exists", r, inv, c))
                hs.append(("forall", r, inv, c))
                for k in (0, 1, 2, 512, 1024, 1025, 2048, 2049, 4096, 4097, 8999, 9000, 30000, 30001):
                    hs.append(("atleast", k, r, inv, c))
                    hs.append(("atmost", k, r, inv, c))
                hs.append(("exactly", 1025, r, inv, c))
                hs.append(("exactly", 2 * 1500 // 3, r, inv, c))
    hs.append(("and", ("exists", 0, 0, ("atom", 2)), ("atleast", 5000, 1, 1, ("top",))))
    return hs


@pytest.mark.parametrize("heavy_min", [None, 1024, 100000])
def test_heavy_rows(monkeypatch, heavy_min):
    """Rows above the heavy-row threshold are counted chunk by chunk on many
    blocks; the counts equal the oracle's at every threshold (100000: no row
    is heavy), in the plain path, the batch with shared passes, and the batch
    with every role node on its own."""
    if heavy_min is not None:
        monkeypatch.setenv("HTHEDL_HEAVY_MIN", str(heavy_min))
    kb = heavy_kb()
    hs = heavy_zoo()
    eng = check(kb, hs, label=f"heavy rows, threshold {heavy_min}")
    hthedl.hth_kb_set_tuning(eng.handle, group_min=0)
    want = Oracle(kb).coverages(hs)
    assert np.array_equal(eng.eval_batch(hs), want)
    o = Oracle(kb)
    for h in (("exists", 0, 0, ("atom", 2)), ("atleast", 2049, 0, 0, ("top",)), ("forall", 1, 1, ("atom", 0))):
        (p, q), bits = eng.eval_one(h, instances=True)
        np.testing.assert_array_equal(bits, o.ext_bits(h))


def numeric_kb(n=50000, seed=21):
    """Concepts and roles from the small generator plus three numeric concrete
    roles: Zipf value counts, values on a 1/16 grid (exact matches and ties),
    and two subjects above the heavy-row threshold (1,500 and 9,000 values)."""
    cfg = synth.small_config(n=n, n_concepts=24, n_roles=3, cap=40, n_pos=n // 10, n_neg=n // 12,
                             seed_index=seed)
    kb = synth.make_kb(cfg)
    offs, vals = synth.numeric_roles(n, 3, seed=seed, cap=48)
    # splice two long rows into role 1: subjects 777 and n - 1
    rows = [list(vals[offs[1, x]:offs[1, x + 1]]) for x in range(n)]
    rng = np.random.default_rng(seed)
    rows[777] = list(np.round(rng.standard_normal(1500) * 16) / 16)
    rows[n - 1] = list(np.round(rng.standard_normal(9000) * 16) / 16) + [7.5]
    base = offs[1, 0]
    new1 = np.zeros(n + 1, np.int64)
    new1[0] = base
    new1[1:] = base + np.cumsum([len(r) for r in rows])
    v1 = np.asarray([v for r in rows for v in r], np.float32)
    shift = new1[-1] - offs[1, -1]
    offs = offs.copy()
    offs[1] = new1
    offs[2] += shift
    vals = np.concatenate([vals[: offs[0, -1]], v1, vals[offs[2, 0] - shift:]]).astype(np.float32)
    return synth.with_numeric_roles(kb, offs, vals), cfg


@pytest.mark.parametrize("heavy_min", [None, 1024])
def test_numeric_concrete_roles(monkeypatch, heavy_min):
    """MIN / MAX / EXACT over multi-valued numeric concrete roles, alone and
    nested, equal the oracle in the plain path and the batch, with heavy rows
    counted chunk by chunk (threshold 1,024) or in the wave walk (2,048 for
    the 1,500-value row)."""
    if heavy_min is not None:
        monkeypatch.setenv("HTHEDL_HEAVY_MIN", str(heavy_min))
    kb, cfg = numeric_kb()
    hs = synth.make_numeric_hypotheses(kb, 300, seed=5)
    for p in range(3):
        for t in (float("-inf"), -0.0, 0.0, 0.0625, 7.5, 1e30, float("inf")):
            hs += [("nge", p, t), ("nle", p, t), ("neq", p, t)]
    hs += [("not", ("neq", 1, 7.5)), ("exists", 0, 1, ("nge", 1, 3.0)),
           ("and", ("nle", 0, -1.0), ("nge", 2, 1.0), ("atom", 3)), ("forall", 2, 0, ("nle", 1, 0.5))]
    eng = check(kb, hs, label=f"numeric roles, heavy {heavy_min}")
    o = Oracle(kb)
    for h in (("nge", 1, 2.0), ("neq", 1, 7.5), ("nle", 2, -2.0)):
        (p, q), bits = eng.eval_one(h, instances=True)
        np.testing.assert_array_equal(bits, o.ext_bits(h))


def test_data_exact():
    """EXACT on single-valued columns: NaN never equal, +0 == -0, ties at deciles."""
    cfg = synth.small_config(n=20011, n_concepts=16, n_roles=2, cap=20, n_data=3, n_hyps=10, seed_index=2100)
    kb = synth.make_kb(cfg)
    hs = []
    for p in range(3):
        for t in list(kb.deciles[p]) + [0.0, -0.0, 1e9, float("-inf")]:
            hs += [("deq", p, float(t)), ("not", ("deq", p, float(t))),
                   ("and", ("deq", p, float(t)), ("dge", p, float(t)))]
    check(kb, hs, label="data exact")


def test_numeric_registration_errors(gpu):
    torch = gpu
    kb, _ = numeric_kb(n=3000)
    eng = hthedl.Engine(kb)
    P = kb.num_offsets.shape[0]
    good_off = torch.from_numpy(kb.num_offsets.copy()).cuda()
    V = int(kb.num_values.shape[0])
    nb = hthedl.hth_numeric_derived_bytes(eng.handle, P, V)
    der = torch.empty(nb, dtype=torch.uint8, device="cuda")
    bad_vals = kb.num_values.copy()
    bad_vals[5] = np.nan
    with pytest.raises(hthedl.HthError, match="NaN"):
        hthedl.hth_kb_set_numeric(eng.handle, P, good_off, torch.from_numpy(bad_vals).cuda(), V, der, nb)
    off = kb.num_offsets.copy()
    off[1, 10], off[1, 11] = off[1, 11] + 1, off[1, 10]       # a row that runs backwards
    with pytest.raises(hthedl.HthError, match="monotone"):
        hthedl.hth_kb_set_numeric(eng.handle, P, torch.from_numpy(off).cuda(),
                                  torch.from_numpy(kb.num_values).cuda(), V, der, nb)
    off = kb.num_offsets.copy()
    off[2] += 1                                               # role 2 does not start where role 1 ends
    with pytest.raises(hthedl.HthError):
        hthedl.hth_kb_set_numeric(eng.handle, P, torch.from_numpy(off).cuda(),
                                  torch.from_numpy(kb.num_values).cuda(), V, der, nb)
    with pytest.raises(hthedl.HthError, match="NOMEM|smaller"):
        hthedl.hth_kb_set_numeric(eng.handle, P, good_off, torch.from_numpy(kb.num_values).cuda(), V, der, 256)
    # the failed calls left the earlier registration in place
    assert eng.eval_plain([("nge", 1, 0.0)]).tolist() == [list(Oracle(kb).coverage(("nge", 1, 0.0)))]
    with pytest.raises(hthedl.HthError, match="numeric concrete role id"):
        eng.eval_plain([("nge", 3, 0.0)])
    hthedl.hth_kb_set_numeric(eng.handle, 0, None, None, 0, None, 0)
    with pytest.raises(hthedl.HthError):
        eng.eval_plain([("nge", 0, 0.0)])


def string_kb(n=40000, seed=31):
    """String concrete roles over a 3,000-word dictionary, with one subject of
    role 1 holding 3,000 values and one holding 1,500 (heavy at 1,024)."""
    cfg = synth.small_config(n=n, n_concepts=20, n_roles=2, cap=30, n_pos=n // 10, n_neg=n // 12,
                             seed_index=seed)
    kb = synth.make_kb(cfg)
    offs, ids, strings = synth.string_roles(n, 2, seed=seed, n_strings=3000)
    rng = np.random.default_rng(seed)
    rows = [list(ids[offs[1, x]:offs[1, x + 1]]) for x in range(n)]
    rows[123] = list(rng.integers(0, 3000, size=1500))
    rows[n - 2] = list(rng.integers(0, 3000, size=3000))
    base = offs[1, 0]
    new1 = np.zeros(n + 1, np.int64)
    new1[0] = base
    new1[1:] = base + np.cumsum([len(r) for r in rows])
    offs = offs.copy()
    offs[1] = new1
    ids = np.concatenate([ids[: offs[0, -1]], np.asarray([v for r in rows for v in r], np.int32)]).astype(np.int32)
    return synth.with_string_roles(kb, offs, ids, strings)


@pytest.mark.parametrize("heavy_min", [None, 1024])
def test_string_concrete_roles(monkeypatch, heavy_min):
    """EQUAL and CONTAIN over string concrete roles equal the oracle (plain,
    batch, instance bits), with absent strings, the empty pattern, patterns
    longer than any string and heavy rows."""
    if heavy_min is not None:
        monkeypatch.setenv("HTHEDL_HEAVY_MIN", str(heavy_min))
    kb = string_kb()
    hs = synth.make_string_hypotheses(kb, 300, seed=7)
    hs += [("sequal", 0, kb.strings[0]), ("sequal", 1, b"not-a-word"), ("scontains", 1, b""),
           ("scontains", 0, b"abcdefabcdefabcdef"), ("scontains", 1, kb.strings[5]),
           ("not", ("scontains", 0, b"a")), ("forall", 1, 0, ("scontains", 1, b"ab")),
           ("and", ("scontains", 0, b"fe"), ("sequal", 1, kb.strings[9]))]
    eng = check(kb, hs, label=f"string roles, heavy {heavy_min}")
    o = Oracle(kb)
    for h in (("scontains", 1, b"cd"), ("sequal", 1, kb.strings[3])):
        (p, q), bits = eng.eval_one(h, instances=True)
        np.testing.assert_array_equal(bits, o.ext_bits(h))


def test_string_registration_errors(gpu):
    torch = gpu
    kb = string_kb(n=4000)
    eng = hthedl.Engine(kb)
    Q, V = kb.str_offsets.shape[0], int(kb.str_ids.shape[0])
    nb = hthedl.hth_string_derived_bytes(eng.handle, Q, V)
    der = torch.empty(nb, dtype=torch.uint8, device="cuda")
    off = torch.from_numpy(kb.str_offsets.copy()).cuda()
    bad = kb.str_ids.copy()
    bad[7] = 3000                                             # one past the dictionary
    with pytest.raises(hthedl.HthError, match="out of range"):
        hthedl.hth_kb_set_strings(eng.handle, Q, off, torch.from_numpy(bad).cuda(), V, 3000,
                                  eng.dict_offsets, eng.dict_chars, der, nb)
    doff = eng.dict_offsets.clone()
    doff[10] = doff[9] - 1                                    # a dictionary entry that runs backwards
    with pytest.raises(hthedl.HthError, match="non-decreasing"):
        hthedl.hth_kb_set_strings(eng.handle, Q, off, eng.str_ids, V, 3000, doff, eng.dict_chars, der, nb)
    pat = torch.tensor([0, 3, 2], dtype=torch.int64, device="cuda")
    with pytest.raises(hthedl.HthError, match="non-decreasing"):
        hthedl.hth_kb_set_patterns(eng.handle, 2, pat, eng.dict_chars)
    # the registration in place still answers
    h = ("scontains", 0, b"ab")
    assert eng.eval_plain([h]).tolist() == [list(Oracle(kb).coverage(h))]
    with pytest.raises(hthedl.HthError, match="string concrete role id"):
        eng.eval_plain([("sequal", 2, kb.strings[0])])


def test_value_roles_in_compiled_plans():
    """Numeric and string restrictions in a compiled plan (their tasks, heavy
    rows and CONTAIN id sets in the plan's workspace), launched twice."""
    import torch
    kb = string_kb(n=30000)
    offs, vals = synth.numeric_roles(kb.n, 2, seed=12)
    kb = synth.with_numeric_roles(kb, offs, vals)
    hs = synth.make_string_hypotheses(kb, 60, seed=3) + synth.make_numeric_hypotheses(kb, 60, seed=4)
    want = Oracle(kb).coverages(hs)
    eng = hthedl.Engine(kb)
    nodes, offs_, ch = hthedl.encode_batch([eng.intern(h) for h in hs])
    plan, nb = hthedl.hth_plan_create(eng.handle, nodes, offs_, ch)
    try:
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
        hthedl.hth_plan_upload(plan, ws, nb)
        for _ in range(2):
            counts = torch.full((len(hs), 2), 7, dtype=torch.int32, device="cuda")
            hthedl.hth_plan_launch(plan, ws, nb, counts)
            torch.cuda.synchronize()
            assert np.array_equal(counts.cpu().numpy().view(np.uint32), want)
    finally:
        hthedl.hth_plan_destroy(plan)


@pytest.mark.parametrize("n", [200_003, 65_536])
def test_short_row_passes(n):
    """Shared passes that walk one subject per lane (directions whose rows are
    all short, like the inverse of a role with sparse subjects and uniform
    objects): equal to the oracle and to the sliced passes, at every T width,
    compact or full T rows, with the short-row limit below, at and above the
    longest row, through host-compiled and device-generated plans."""
    cfg = synth.small_config(n=n, n_concepts=40, n_roles=3, s=1.6, cap=300, n_data=2, n_pos=n // 10,
                             n_neg=n // 12, seed_index=2600 + n % 7, total_edges=n // 2)
    kb = synth.make_kb(cfg)
    rng = np.random.default_rng(26)
    hyps = []
    for _ in range(900):
        r, inv = int(rng.integers(0, 3)), int(rng.integers(0, 2))
        c = ("atom", int(rng.integers(0, 40)))
        if rng.random() < 0.4:
            r2 = int(rng.integers(0, 3))
            c = ("exists", r2, 1 - inv, c) if rng.random() < 0.5 else ("or", c, ("atleast", 2, r2, inv, c))
        op = rng.choice(["exists", "forall", "atleast", "atmost", "exactly"])
        hyps.append((op, r, inv, c) if op in ("exists", "forall") else (op, int(rng.integers(0, 5)), r, inv, c))
    want = Oracle(kb).coverages(hyps)
    eng = hthedl.Engine(kb, max_hyps=len(hyps))
    longest = [hthedl.hth_kb_max_degree(eng.handle, r, 1) for r in range(3)]
    say(f"[parity] short rows n={n}: longest inverse rows {longest}, forward "
        f"{[hthedl.hth_kb_max_degree(eng.handle, r, 0) for r in range(3)]}")
    assert max(longest) <= 12
    for limit in (0, min(longest) - 1, 12, 64):
        for k, compact in ((8, 1), (64, 1), (32, 0)):
            hthedl.hth_kb_set_tuning(eng.handle, group_min=1, group_k=k, t_compact=compact, short_rows=max(0, limit))
            got = eng.eval_batch(hyps)
            bad = np.flatnonzero((got != want).any(axis=1))
            assert bad.size == 0, (limit, k, compact, hyps[bad[0]], got[bad[0]], want[bad[0]])
            got = eng.eval_batch_device(hyps)
            bad = np.flatnonzero((got != want).any(axis=1))
            assert bad.size == 0, ("device", limit, k, compact, hyps[bad[0]], got[bad[0]], want[bad[0]])


def test_tbuild_dense_and_sparse_compact_objects():
    """Compact T rows where a 64-word wave of the T build holds more object
    rows than it stages in LDS (forward directions whose objects are about 40%
    of the individuals: the wave stores its rows directly) and fewer (inverse
    directions, 10%: the rows go out as one run from LDS), at every T width,
    through host-compiled and device-generated plans, against the oracle."""
    n = 131_101
    cfg = synth.small_config(n=n, n_concepts=24, n_roles=3, s=1.5, cap=40, n_data=1, n_pos=n // 10,
                             n_neg=n // 12, seed_index=2800, total_edges=3 * n // 2)
    kb = synth.make_kb(cfg)
    off, tg = np.asarray(kb.role_offsets), np.asarray(kb.role_targets)
    for r in range(3):
        obj = np.zeros(n, bool)
        obj[tg[int(off[r, 0]):int(off[r, -1])]] = True
        per_wave = np.add.reduceat(obj.astype(np.int64), np.arange(0, n, 4096))
        assert 2 * int(obj.sum()) <= n and per_wave.max() > 1024   # compact, some waves beyond the stage
    rng = np.random.default_rng(28)
    hyps = []
    for _ in range(700):
        r, inv = int(rng.integers(0, 3)), int(rng.integers(0, 2))
        c = ("atom", int(rng.integers(0, 24)))
        if rng.random() < 0.3:
            c = ("or", c, ("exists", int(rng.integers(0, 3)), 1 - inv, ("atom", int(rng.integers(0, 24)))))
        op = rng.choice(["exists", "forall", "atleast", "atmost", "exactly"])
        hyps.append((op, r, inv, c) if op in ("exists", "forall") else (op, int(rng.integers(0, 6)), r, inv, c))
    want = Oracle(kb).coverages(hyps)
    eng = hthedl.Engine(kb, max_hyps=len(hyps))
    for k in (64, 32, 16, 8):
        hthedl.hth_kb_set_tuning(eng.handle, group_min=1, group_k=k, t_compact=1)
        got = eng.eval_batch(hyps)
        bad = np.flatnonzero((got != want).any(axis=1))
        assert bad.size == 0, ("host", k, hyps[bad[0]], got[bad[0]], want[bad[0]])
        got = eng.eval_batch_device(hyps)
        bad = np.flatnonzero((got != want).any(axis=1))
        assert bad.size == 0, ("device", k, hyps[bad[0]], got[bad[0]], want[bad[0]])


def test_short_row_passes_with_saturating_counts():
    """Short-row passes over directions whose longest rows hold 8 to 12
    assertions (every direction of this KB is within the short-row limit):
    the counters keep their saturation plane, and counts from 6 to beyond 8
    decide the members.  Host-compiled and device-generated plans, every T
    width, against the oracle."""
    n = 90_001
    cfg = synth.small_config(n=n, n_concepts=20, n_roles=2, s=1.2, cap=12, n_data=1, n_pos=n // 10,
                             n_neg=n // 12, seed_index=2901, total_edges=5 * n)
    kb = synth.make_kb(cfg)
    rng = np.random.default_rng(29)
    hyps = []
    for _ in range(600):
        r, inv = int(rng.integers(0, 2)), int(rng.integers(0, 2))
        c = ("atom", int(rng.integers(0, 20)))
        if rng.random() < 0.3:
            c = ("not", c)
        op = rng.choice(["exists", "forall", "atleast", "atmost", "exactly"])
        hyps.append((op, r, inv, c) if op in ("exists", "forall") else (op, int(rng.integers(1, 9)), r, inv, c))
    want = Oracle(kb).coverages(hyps)
    eng = hthedl.Engine(kb, max_hyps=len(hyps))
    longest = [hthedl.hth_kb_max_degree(eng.handle, r, d) for r in range(2) for d in range(2)]
    say(f"[parity] saturating short rows: longest rows {longest}")
    assert max(longest) >= 8 and max(longest) <= 12
    for k in (64, 8):
        hthedl.hth_kb_set_tuning(eng.handle, group_min=1, group_k=k, short_rows=12)
        got = eng.eval_batch(hyps)
        bad = np.flatnonzero((got != want).any(axis=1))
        assert bad.size == 0, ("host", k, hyps[bad[0]], got[bad[0]], want[bad[0]])
        got = eng.eval_batch_device(hyps)
        bad = np.flatnonzero((got != want).any(axis=1))
        assert bad.size == 0, ("device", k, hyps[bad[0]], got[bad[0]], want[bad[0]])


@pytest.mark.parametrize("short_rows", [0, 12])
def test_role_roots_with_fused_coverage(short_rows):
    """Hypotheses that are a single role restriction: where such a node is the
    root of one hypothesis and read by no other node, its shared pass adds its
    coverage directly (no row, no root region).  Covered: universal and
    at-most roots (they hold every individual of the words without
    assertions), roots repeated in the batch, roots that other hypotheses also
    read, both directions of roles with sparse subjects, host-compiled and
    device-generated plans; all against the oracle."""
    n = 150_011
    cfg = synth.small_config(n=n, n_concepts=32, n_roles=3, s=1.6, cap=500, n_data=2, n_pos=n // 9,
                             n_neg=n // 11, seed_index=2700, total_edges=n // 3)
    kb = synth.make_kb(cfg)
    rng = np.random.default_rng(27)
    hyps = []
    for _ in range(1200):
        r, inv = int(rng.integers(0, 3)), int(rng.integers(0, 2))
        c = ("atom", int(rng.integers(0, 32)))
        if rng.random() < 0.3:
            c = ("and", c, ("exists", int(rng.integers(0, 3)), 1 - inv, ("atom", int(rng.integers(0, 32)))))
        op = rng.choice(["exists", "forall", "atleast", "atmost"])
        hyps.append((op, r, inv, c) if op in ("exists", "forall") else (op, int(rng.integers(0, 4)), r, inv, c))
    hyps += hyps[:40]                                             # roots repeated
    hyps += [("and", h, ("atom", 1)) for h in hyps[40:80]]        # roots read by other hypotheses
    hyps += [("not", h) for h in hyps[80:100]]
    want = Oracle(kb).coverages(hyps)
    eng = hthedl.Engine(kb, max_hyps=len(hyps))
    for k in (64, 16):
        hthedl.hth_kb_set_tuning(eng.handle, group_min=2, group_k=k, short_rows=short_rows)
        got = eng.eval_batch(hyps)
        bad = np.flatnonzero((got != want).any(axis=1))
        assert bad.size == 0, ("host", k, hyps[bad[0]], got[bad[0]], want[bad[0]])
        got = eng.eval_batch_device(hyps)
        bad = np.flatnonzero((got != want).any(axis=1))
        assert bad.size == 0, ("device", k, hyps[bad[0]], got[bad[0]], want[bad[0]])
