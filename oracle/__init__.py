"""CPU oracle -- test infrastructure only (see ``oracle.dl``).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The library never does.
"""
from .dl import Oracle, f1_score  # noqa: F401
