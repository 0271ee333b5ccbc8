"""The C++ oracle (oracle/cpp, the timed CPU baseline) against the pinned
Python oracle and brute force: instance sets and coverage bit for bit on the
whole c1 workload and on random tiny knowledge bases, with every construct,
empty conjunctions, n = 0, NaN values and signed zeros; one thread and many
agree; malformed streams are refused."""
import random

import numpy as np
import pytest

from oracle import Oracle
from oracle.cpp_oracle import CppOracle, batch_tokens, max_threads
from paper_2412_00802_amd import synth
from tests.pin_semantics import brute_ext, kb_sets
from tests.test_golden import load_c1_counts
from tests.test_oracle_pins import random_hyp, random_kb


def test_c1_workload_equals_python_oracle_and_golden():
    cfg = synth.CONFIGS["c1"]
    kb = synth.make_kb(cfg)
    hyps = synth.make_hypotheses(cfg, kb)
    got = CppOracle(kb).coverages(hyps)
    np.testing.assert_array_equal(got, Oracle(kb).coverages(hyps))
    np.testing.assert_array_equal(got, load_c1_counts())


def test_random_tiny_kbs_against_brute_force():
    rnd = random.Random(17)
    checked = 0
    for trial in range(50):
        n = rnd.randint(1, 9)
        kb = random_kb(rnd, n)
        sets = kb_sets(kb)
        c = CppOracle(kb)
        for _ in range(30):
            h = random_hyp(rnd, rnd.randint(1, 4), 3, 2, 2)
            want = brute_ext(sets, n, h)
            got = set(np.flatnonzero(c.ext(h)).tolist())
            assert got == want, (trial, h)
            checked += 1
    assert checked == 1500


@pytest.mark.parametrize("seed", range(3))
def test_small_workloads_equal_python_oracle(seed):
    cfg = synth.small_config(n=700 + 331 * seed, n_concepts=16, n_roles=3, s=1.3, cap=40,
                             n_pos=120, n_neg=150, n_hyps=120, hyp_depth=5, seed_index=1500 + seed)
    kb = synth.make_kb(cfg)
    hyps = synth.make_hypotheses(cfg, kb)
    o, c = Oracle(kb), CppOracle(kb)
    for h in hyps[:40]:
        np.testing.assert_array_equal(c.ext(h), o.ext(h), err_msg=str(h))
    want = o.coverages(hyps)
    np.testing.assert_array_equal(c.coverages(hyps, threads=1), want)
    np.testing.assert_array_equal(c.coverages(hyps, threads=max(2, max_threads())), want)


def test_edge_constructs():
    rnd = random.Random(3)
    kb = random_kb(rnd, 8)
    o, c = Oracle(kb), CppOracle(kb)
    hyps = [("and",), ("or",), ("top",), ("bot",), ("atleast", 0, 0, 0, ("atom", 1)),
            ("atmost", 0, 1, 1, ("atom", 0)), ("exactly", 0, 0, 1, ("top",)),
            ("forall", 0, 0, ("bot",)), ("exists", 1, 1, ("top",)),
            ("dge", 0, -0.0), ("dle", 1, 0.0), ("dge", 0, float("-inf")), ("dle", 1, float("inf")),
            ("not", ("not", ("atom", 2))), ("atleast", 2 ** 31 - 1, 0, 0, ("top",))]
    for h in hyps:
        np.testing.assert_array_equal(c.ext(h), o.ext(h), err_msg=str(h))


def test_malformed_streams_are_refused():
    kb = random_kb(random.Random(5), 6)
    c = CppOracle(kb)
    with pytest.raises(ValueError):
        c.ext(("atom", 7))                     # concept out of range
    with pytest.raises(ValueError):
        c.ext(("exists", 5, 0, ("top",)))      # role out of range
    toks, offs = batch_tokens([("and", ("atom", 0), ("atom", 1))])
    with pytest.raises(ValueError):            # stream cut short
        c.coverages_tokens(toks[:-1].copy(), np.array([0, toks.size - 1], dtype=np.int64))
