"""Pins of the screener references (no GPU): finite-difference gradients of
the MLP, bf16 rounding against exact cases, and properties of the subtree hash."""
import numpy as np
import pytest

from oracle import screener as S


def small_params(rng, d_in=24, h1=16, h2=8, scale=0.4):
    return {"w1": rng.standard_normal((d_in, h1)) * scale, "b1": rng.standard_normal(h1) * 0.1,
            "w2": rng.standard_normal((h1, h2)) * scale, "b2": rng.standard_normal(h2) * 0.1,
            "w3": rng.standard_normal((h2, 2)) * scale, "b3": rng.standard_normal(2) * 0.1}


@pytest.mark.parametrize("loss", ["bce", "mse"])
def test_gradients_match_central_differences(loss):
    rng = np.random.default_rng(0)
    p = small_params(rng)
    x = rng.integers(0, 3, size=(7, 24)).astype(np.float64)
    y = rng.random((7, 2)) * (5 if loss == "mse" else 1)
    scale = 1.0 / 14
    acts, _ = S.forward(p, x, y, loss=loss)
    g = S.backward(p, acts, y, scale, loss=loss)
    eps = 1e-6
    for name in ("w1", "b1", "w2", "b2", "w3", "b3"):
        flat = p[name].reshape(-1)
        idx = rng.choice(flat.size, size=min(12, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + eps
            lp = S.forward(p, x, y, loss=loss)[1] * scale
            flat[i] = old - eps
            lm = S.forward(p, x, y, loss=loss)[1] * scale
            flat[i] = old
            num = (lp - lm) / (2 * eps)
            ana = g[name].reshape(-1)[i]
            assert abs(num - ana) <= 1e-6 + 1e-4 * abs(num), (name, i, num, ana)


def test_bf16_rounding_exact_cases():
    vals = np.array([1.0, 1.00390625, 1.005859375, 1.0078125, -2.5, 3.0e-39, 65504.0], dtype=np.float32)
    r = S.bf16(vals)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: rounds to even (1.0)
    assert r[0] == 1.0 and r[1] == 1.0
    assert r[2] == 1.0078125            # above the tie: rounds up
    assert r[3] == 1.0078125 and r[4] == -2.5
    assert r[6] == 65536.0              # 65504 rounds to 2^16 in bf16
    assert np.isnan(S.bf16(np.array([np.nan], dtype=np.float32)))[0]
    # every result has a zero low half
    u = r.astype(np.float32).view(np.uint32)
    assert np.all((u & 0xFFFF) == 0)


def test_subtree_hash_properties():
    a, b = ("atom", 3), ("exists", 1, 0, ("atom", 4))
    f1 = S.subtree_features(("and", a, b))
    f2 = S.subtree_features(("and", b, a))
    assert f1[-1] == f2[-1]                                   # and/or: order independent
    assert S.subtree_features(("exists", 1, 0, a))[-1] != S.subtree_features(("exists", 1, 1, a))[-1]
    assert S.subtree_features(("atleast", 2, 1, 0, a))[-1] != S.subtree_features(("atleast", 3, 1, 0, a))[-1]
    assert S.subtree_features(("dge", 0, 0.5))[-1] != S.subtree_features(("dle", 0, 0.5))[-1]
    assert len(S.subtree_features(("or", a, ("not", b)))) == 5
    x = S.dense_features([("and", a, b), ("atom", 3)])
    assert x.sum(axis=1).tolist() == [4.0, 1.0]
    # the atom's own feature is shared between the two hypotheses
    fa = S.subtree_features(a)[0][1]
    assert x[0, fa] >= 1 and x[1, fa] == 1


def test_adamw_reference_first_step():
    p, g = np.array([1.0, -2.0]), np.array([0.5, -0.25])
    q, m, v = S.adamw(p, g, np.zeros(2), np.zeros(2), lr=0.1, b1=0.9, b2=0.999, eps=0.0, wd=0.0, step=1)
    # first bias-corrected step moves each weight by lr * sign(g)
    np.testing.assert_allclose(q, p - 0.1 * np.sign(g))


def test_predicted_f1_closed_forms():
    """z = 0 keeps half of the base coverage; very large logits keep all of it;
    a base equal to (|P|, |Ng|) is the same as no base."""
    n_pos, n_neg = 100, 300
    base = np.array([[40, 10], [100, 300], [0, 0]])
    f = S.predicted_f1(np.zeros((3, 2)), n_pos, n_neg, base)
    want = [2 * 20 / (20 + 5 + 100), 2 * 50 / (50 + 150 + 100), 0.0]
    np.testing.assert_allclose(f, want, rtol=1e-12)
    f = S.predicted_f1(np.full((3, 2), 60.0), n_pos, n_neg, base)
    np.testing.assert_allclose(f, [2 * 40 / (40 + 10 + 100), 2 * 100 / (100 + 300 + 100), 0.0], rtol=1e-12)
    z = np.random.default_rng(3).standard_normal((5, 2))
    np.testing.assert_allclose(S.predicted_f1(z, n_pos, n_neg, np.tile([n_pos, n_neg], (5, 1))),
                               S.predicted_f1(z, n_pos, n_neg), rtol=1e-12)


def test_delta_features_cancel_unchanged_subtrees():
    """A child that adds one conjunct X to an and-parent differs from its parent
    by X's subtrees plus the new root, minus the old root."""
    parent = ("and", ("atom", 1), ("exists", 0, 1, ("atom", 2)))
    x = ("dge", 3, 0.25)
    child = ("and", ("atom", 1), ("exists", 0, 1, ("atom", 2)), x)
    d = S.delta_features([child], [parent], [0])[0]
    want = np.zeros(S.FEATURE_DIM)
    for _, f in S.subtree_features(x):
        want[f] += 1
    want[S.subtree_features(child)[-1][1]] += 1
    want[S.subtree_features(parent)[-1][1]] -= 1
    np.testing.assert_array_equal(d, want)
    assert not S.delta_features([parent], [parent], [0]).any()


def test_delta_features_with_parent_context():
    """The context variant adds the parent's own subtree counts once, each at
    its feature index with the top bit (2048) flipped, and nothing else."""
    parent = ("and", ("atom", 1), ("exists", 0, 1, ("atom", 2)))
    child = ("and", ("atom", 1), ("exists", 0, 1, ("atom", 2)), ("atom", 7))
    d0 = S.delta_features([child], [parent], [0])[0]
    d1 = S.delta_features([child], [parent], [0], context=True)[0]
    want = np.zeros(S.FEATURE_DIM)
    for _, f in S.subtree_features(parent):
        want[f ^ 2048] += 1
    np.testing.assert_array_equal(d1 - d0, want)
    assert (d1 - d0).sum() == len(S.subtree_features(parent)) == 4


def test_predicted_f1_from_log_removed_counts():
    """z = log(1 + removed): z = 0 keeps the base; z = log(1 + r) removes r
    (exactly, up to rounding); removals beyond the base clamp to 0."""
    n_pos, n_neg = 100, 300
    base = np.array([[40, 10], [40, 10], [40, 10]])
    z = np.array([[0.0, 0.0], [np.log1p(5.0), np.log1p(4.0)], [20.0, 20.0]])
    f = S.predicted_f1(z, n_pos, n_neg, base, kind="log_removed")
    np.testing.assert_allclose(f, [2 * 40 / (40 + 10 + 100), 2 * 35 / (35 + 6 + 100), 0.0], rtol=1e-12)
    assert S.predicted_f1(np.array([[-3.0, -1.0]]), n_pos, n_neg, base[:1], kind="log_removed")[0] == f[0]


def test_fnv1a64_published_vectors():
    """The subtree hash's byte hash is FNV-1a 64 (xor, then multiply), pinned to
    the published test vectors of Fowler, Noll and Vo; FNV-1 (multiply, then
    xor) gives other values and would fail."""
    assert S._fnv(S.FNV_OFFSET, b"") == 0xCBF29CE484222325
    assert S._fnv(S.FNV_OFFSET, b"a") == 0xAF63DC4C8601EC8C
    assert S._fnv(S.FNV_OFFSET, b"foobar") == 0x85944171F73967E8
    # the FNV-1 vectors of the same inputs differ from what _fnv returns
    assert S._fnv(S.FNV_OFFSET, b"a") != 0xAF63BD4C8601B7BE
    assert S._fnv(S.FNV_OFFSET, b"foobar") != 0x340D8765A4DDA9C2
    # byte order: a header is hashed as its little-endian bytes
    h = S._header("atom", arg=0x01020304)
    assert h[4:8] == b"\x04\x03\x02\x01"


def test_splitmix64_published_outputs():
    """_splitmix(x) is the output of a SplitMix64 generator whose state was x
    (Steele, Lea and Flood): state + golden gamma, then the two multiply-xorshift
    rounds.  Outputs k = 0, 1, 2, ... of seed s are _splitmix(s + k * gamma);
    seed 1234567 gives the published reference sequence, seed 0 its first value."""
    gamma = 0x9E3779B97F4A7C15
    seq = [S._splitmix((1234567 + k * gamma) & S.MASK64) for k in range(5)]
    assert seq == [6457827717110365317, 3203168211198807973, 9817491932198370423,
                   4593380528125082431, 16408922859458223821]
    assert S._splitmix(0) == 0xE220A8397B1DCDAF
