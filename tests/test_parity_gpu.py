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
