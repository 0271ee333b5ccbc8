"""The stored tiny-workload coverage still follows from the seeded inputs."""
import os

import numpy as np

from oracle import Oracle
from paper_2412_00802_amd import synth

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_c1_counts():
    return np.loadtxt(os.path.join(HERE, "c1_counts.txt"), dtype=np.uint32, comments="#")


def test_c1_golden_matches_oracle():
    cfg = synth.CONFIGS["c1"]
    kb = synth.make_kb(cfg)
    hyps = synth.make_hypotheses(cfg, kb)
    want = load_c1_counts()
    assert want.shape == (cfg.n_hyps, 2)
    np.testing.assert_array_equal(Oracle(kb).coverages(hyps), want)
    # the counts are not degenerate: many distinct values, some zero, some full
    assert len({tuple(r) for r in want.tolist()}) > 100
