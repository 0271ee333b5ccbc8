"""MI355X-native exact evaluation of ALCQI(D) concept hypotheses over a knowledge base.

The compute path is the HIP library ``libhthedl.so`` (built from ``csrc/``);
``hthedl`` is its thin ctypes binding and ``synth`` draws seeded inputs.
Importing the package loads nothing: the library is opened on first use.
"""
