"""The CPU reference of the device's conjunct draws, pinned: its generator
reproduces SplitMix64's published reference outputs, and its draws cover
every kind in the stated proportions and ranges."""
import numpy as np

from paper_2412_00802_amd.hthedl import CJ_ATOM, CJ_EXISTS, CJ_GE, CJ_LE
from tests import conjunct_ref


def test_splitmix64_reference_outputs():
    # the generator's reference outputs for seeds 0 and 1234567
    assert conjunct_ref.splitmix64(0, 0) == 0xE220A8397B1DCDAF
    assert [conjunct_ref.splitmix64(1234567, i) for i in range(3)] == [
        6457827717110365317, 3203168211198807973, 9817491932198370423]


def test_draws_follow_the_stated_distribution():
    dec = np.sort(np.random.default_rng(0).normal(size=(3, 9)).astype(np.float32), axis=1)
    specs = conjunct_ref.draw(99, np.arange(40, dtype=np.uint32), 250, 17, 5, 3, dec)
    kinds = np.bincount(specs["kind"], minlength=4) / specs.shape[0]
    np.testing.assert_allclose(kinds, [0.5, 0.3, 0.1, 0.1], atol=0.02)
    assert (specs["parent"] == np.repeat(np.arange(40), 250)).all()
    atom = specs["kind"] == CJ_ATOM
    ex = specs["kind"] == CJ_EXISTS
    thr = (specs["kind"] == CJ_GE) | (specs["kind"] == CJ_LE)
    assert specs["a"][atom | ex].max() == 16 and specs["b"][ex].max() == 4
    assert set(specs["inv"][ex]) == {0, 1}
    t = specs["b"][thr].view(np.float32)
    assert all(t[j] in dec[specs["a"][thr][j]] for j in range(t.size))
    # no properties and no roles: every draw is an atom
    only = conjunct_ref.draw(5, np.arange(3, dtype=np.uint32), 50, 4, 0, 0, np.zeros((0, 9), np.float32))
    assert (only["kind"] == CJ_ATOM).all()


def test_bindings_refuse_short_buffers():
    """The bindings check tensor sizes before the library writes into them."""
    import pytest
    import torch
    from paper_2412_00802_amd import hthedl
    n = 10
    specs = torch.zeros(16 * n, dtype=torch.uint8)
    for nodes, offs, ch in ((torch.zeros(16 * n, dtype=torch.uint8), torch.zeros(n + 1, dtype=torch.int32),
                             torch.zeros(2 * n, dtype=torch.int32)),
                            (torch.zeros(64 * n, dtype=torch.uint8), torch.zeros(n, dtype=torch.int32),
                             torch.zeros(2 * n, dtype=torch.int32)),
                            (torch.zeros(64 * n, dtype=torch.uint8), torch.zeros(n + 1, dtype=torch.int32),
                             torch.zeros(n, dtype=torch.int32))):
        with pytest.raises(ValueError):
            hthedl.hth_conjoin(specs, n, nodes, offs, ch)
    with pytest.raises(ValueError):
        hthedl.hth_draw_conjuncts(None, 1, torch.zeros(2, dtype=torch.int32), 2, 10, None,
                                  torch.zeros(16 * 19, dtype=torch.uint8))
