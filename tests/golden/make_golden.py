"""Writes the stored expected values under tests/golden/ (calls only the oracle).

c1_counts.txt: (pos, neg) coverage of the 256 seeded hypotheses of the tiny
plain workload (10,000 individuals), one line per hypothesis, computed by the
CPU oracle (Algorithm 15 over the set semantics of Section 3.2).

Run:  python tests/golden/make_golden.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import Oracle                      # noqa: E402
from paper_2412_00802_amd import synth         # noqa: E402


def main():
    cfg = synth.CONFIGS["c1"]
    kb = synth.make_kb(cfg)
    hyps = synth.make_hypotheses(cfg, kb)
    counts = Oracle(kb).coverages(hyps)
    with open(os.path.join(HERE, "c1_counts.txt"), "w") as f:
        f.write("# (pos, neg) per hypothesis of the seeded tiny workload; written by make_golden.py\n")
        for p, q in counts.tolist():
            f.write(f"{p} {q}\n")


if __name__ == "__main__":
    main()
