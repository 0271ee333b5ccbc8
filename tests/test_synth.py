"""The seeded generators: determinism and the statistics each workload asks for."""
import numpy as np
import pytest

from paper_2412_00802_amd import synth


@pytest.fixture(scope="module")
def c1():
    return synth.make_kb(synth.CONFIGS["c1"])


def test_deterministic(c1):
    kb2 = synth.make_kb(synth.CONFIGS["c1"], workers=1)
    for f in ("concept_bits", "role_offsets", "role_targets", "pos_bits", "neg_bits"):
        np.testing.assert_array_equal(getattr(c1, f), getattr(kb2, f))
    np.testing.assert_array_equal(np.isnan(c1.data), np.isnan(kb2.data))
    np.testing.assert_array_equal(np.nan_to_num(c1.data), np.nan_to_num(kb2.data))
    h1 = synth.make_hypotheses(synth.CONFIGS["c1"], c1)
    h2 = synth.make_hypotheses(synth.CONFIGS["c1"], kb2)
    assert h1 == h2


def test_csr_is_a_set_of_assertions(c1):
    n = c1.n
    for r in range(c1.n_roles):
        off = c1.role_offsets[r]
        assert np.all(np.diff(off) >= 0)
        if r:
            assert off[0] == c1.role_offsets[r - 1][-1]
        t = c1.role_targets[off[0]:off[-1]].astype(np.int64)
        assert t.min() >= 0 and t.max() < n
        subj = np.repeat(np.arange(n), np.diff(off))
        key = subj * n + t
        assert np.all(np.diff(key) > 0)     # strictly increasing: sorted, no duplicates
    assert c1.role_offsets[-1][-1] == c1.n_edges


def test_degree_law(c1):
    cfg = synth.CONFIGS["c1"]
    deg = np.diff(c1.role_offsets, axis=1)
    assert deg.min() >= 1 and deg.max() <= cfg.degree_cap
    mean = synth.zipf_mean(cfg.zipf_s, cfg.degree_cap)
    assert abs(deg.mean() - mean) / mean < 0.02
    assert abs(synth.zipf_mean(1.8, 1024) - 8.29) < 0.01     # the mid workload's "mean ~8"


def test_concept_tree(c1):
    n = c1.n
    cfg = synth.CONFIGS["c1"]
    assert c1.n_concepts == cfg.n_concepts
    for c in range(c1.n_concepts):
        p = int(c1.concept_parent[c])
        if p >= 0:
            assert np.all((c1.concept_bits[c] & ~c1.concept_bits[p]) == 0)
            assert c1.concept_level[c] == c1.concept_level[p] + 1
    pad = np.uint64(~np.uint64((1 << (n & 63)) - 1)) if n & 63 else np.uint64(0)
    assert np.all((c1.concept_bits[:, -1] & pad) == 0)
    roots = np.flatnonzero(c1.concept_level == 0)
    dens = np.mean([np.unpackbits(c1.concept_bits[a].view(np.uint8)).sum() / n for a in roots])
    assert abs(dens - 0.3) < 0.02


def test_data_and_examples(c1):
    cfg = synth.CONFIGS["c1"]
    miss = np.isnan(c1.data).mean()
    assert abs(miss - cfg.missing) < 0.02
    for p in range(c1.n_data):
        vals = set(c1.data[p][~np.isnan(c1.data[p])].tolist())
        assert all(float(t) in vals for t in c1.deciles[p])
        assert np.all(np.diff(c1.deciles[p]) >= 0)
    pos = np.unpackbits(c1.pos_bits.view(np.uint8)).sum()
    neg = np.unpackbits(c1.neg_bits.view(np.uint8)).sum()
    assert (pos, neg) == (cfg.n_pos, cfg.n_neg)
    assert np.all((c1.pos_bits & c1.neg_bits) == 0)


def test_hypothesis_shapes(c1):
    cfg = synth.CONFIGS["c1"]
    hs = synth.make_hypotheses(cfg, c1)
    assert len(hs) == cfg.n_hyps
    assert max(synth.hyp_depth(h) for h in hs) <= cfg.hyp_depth
    assert all(h[0] not in ("atom", "top", "dge", "dle") for h in hs)


def test_sparse_subjects():
    cfg = synth.small_config(n=20000, n_roles=2, s=1.6, cap=64, total_edges=4000,
                             seed_index=9)
    kb = synth.make_kb(cfg)
    assert abs(kb.n_edges - 4000) / 4000 < 0.15
    assert np.mean(np.diff(kb.role_offsets, axis=1) > 0) < 0.1
