"""GPU parity of the screener kernels against the CPU references: MFMA GEMM,
feature hashing and densify, output layer and loss, AdamW, top-k, and a whole
training step."""
import sys

import numpy as np
import pytest

from oracle import screener as S
from paper_2412_00802_amd import hthedl, synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "the gpu tests need an MI355X"
    hthedl.lib()
    return t


def bf16_dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda().to(torch.bfloat16)


def f64(torch, t):
    return t.float().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("ta,tb", [(0, 0), (0, 1), (1, 0)])
@pytest.mark.parametrize("M,N,K", [(8, 8, 8), (128, 128, 32), (200, 136, 72), (256, 1024, 4096),
                                   (1024, 256, 1024), (40, 264, 1000)])
def test_gemm_matches_reference(torch, ta, tb, M, N, K):
    say(f"[gemm] ta={ta} tb={tb} M={M} N={N} K={K}")
    rng = np.random.default_rng(M * 7 + N * 3 + K + ta * 11 + tb * 13)
    a = rng.standard_normal((M, K)).astype(np.float32)
    b = rng.standard_normal((K, N)).astype(np.float32)
    A = bf16_dev(torch, a.T.copy() if ta else a)
    B = bf16_dev(torch, b.T.copy() if tb else b)
    lda = M if ta else K
    ldb = K if tb else N
    c = torch.empty((M, N), dtype=torch.float32, device="cuda")
    hthedl.hth_gemm_bf16(ta, tb, M, N, K, A, lda, B, ldb, c32=c, ldc=N)
    want = S.bf16(a) @ S.bf16(b)
    got = c.cpu().numpy()
    np.testing.assert_allclose(got, want, rtol=1e-4, atol=1e-4 * np.sqrt(K))


def test_gemm_epilogues(torch):
    rng = np.random.default_rng(5)
    M, N, K = 192, 160, 96
    a, b = rng.standard_normal((M, K)).astype(np.float32), rng.standard_normal((K, N)).astype(np.float32)
    bias = rng.standard_normal(N).astype(np.float32)
    mask = (rng.random((M, N)) < 0.5).astype(np.float32) * rng.standard_normal((M, N)).astype(np.float32)
    A, B, Mk = bf16_dev(torch, a), bf16_dev(torch, b), bf16_dev(torch, mask)
    c32 = torch.empty((M, N), dtype=torch.float32, device="cuda")
    cbf = torch.empty((M, N), dtype=torch.bfloat16, device="cuda")
    hthedl.hth_gemm_bf16(0, 0, M, N, K, A, K, B, N, bias=torch.from_numpy(bias).cuda(), relu=1,
                         c32=c32, ldc=N, cbf=cbf, ldcb=N)
    want = np.maximum(S.bf16(a) @ S.bf16(b) + bias, 0)
    np.testing.assert_allclose(c32.cpu().numpy(), want, rtol=1e-4, atol=1e-3)
    np.testing.assert_array_equal(f64(torch, cbf), S.bf16(c32.cpu().numpy()))
    hthedl.hth_gemm_bf16(0, 0, M, N, K, A, K, B, N, mask=Mk, ldm=N, c32=c32, ldc=N)
    want = (S.bf16(a) @ S.bf16(b)) * (S.bf16(mask) > 0)
    np.testing.assert_allclose(c32.cpu().numpy(), want, rtol=1e-4, atol=1e-3)


def test_gemm_nt_epilogue_and_transpose(torch):
    """The forward layers' layout (B as [N][K] from hth_transpose_bf16): bias,
    ReLU and the bf16 output, on ragged sizes with K not a multiple of the
    64-wide k-tile; the transpose is exact."""
    rng = np.random.default_rng(6)
    M, N, K = 333, 200, 1000
    a, b = rng.standard_normal((M, K)).astype(np.float32), rng.standard_normal((K, N)).astype(np.float32)
    bias = rng.standard_normal(N).astype(np.float32)
    A, B = bf16_dev(torch, a), bf16_dev(torch, b)
    Bt = torch.empty((N, K), dtype=torch.bfloat16, device="cuda")
    hthedl.hth_transpose_bf16(B, K, N, Bt)
    np.testing.assert_array_equal(f64(torch, Bt), S.bf16(b).T)
    c32 = torch.empty((M, N), dtype=torch.float32, device="cuda")
    cbf = torch.empty((M, N), dtype=torch.bfloat16, device="cuda")
    hthedl.hth_gemm_bf16(0, 1, M, N, K, A, K, Bt, K, bias=torch.from_numpy(bias).cuda(), relu=1,
                         c32=c32, ldc=N, cbf=cbf, ldcb=N)
    want = np.maximum(S.bf16(a) @ S.bf16(b) + bias, 0)
    np.testing.assert_allclose(c32.cpu().numpy(), want, rtol=1e-4, atol=1e-4 * np.sqrt(K))
    np.testing.assert_array_equal(f64(torch, cbf), S.bf16(c32.cpu().numpy()))


def _feature_batch(torch, hyps):
    from paper_2412_00802_amd.screener import FeatureBatch
    nodes, offs, ch = hthedl.encode_batch(hyps)
    return FeatureBatch(nodes, offs, ch), nodes


def test_features_and_densify(torch):
    cfg = synth.small_config(n=500, n_concepts=40, n_roles=5, n_data=3, seed_index=1200)
    kb = synth.make_kb(cfg)
    hyps = synth.make_hypotheses(cfg, kb, count=200, depth=5)
    hyps += synth.make_sized_hypotheses(cfg, kb, count=200)
    hyps += [("and",), ("or", ("atom", 1)), ("exactly", 3, 2, 1, ("dle", 1, -0.5)), ("top",)]
    # EXACT on columns and numeric concrete roles hash like the other value leaves
    hyps += [("deq", 2, 0.25), ("nge", 0, -1.5), ("and", ("nle", 1, 2.0), ("neq", 0, 0.0)),
             ("exists", 1, 0, ("nge", 3, 1.0))]
    fb, nodes = _feature_batch(torch, hyps)
    torch.cuda.synchronize()
    assert int(fb.bad.item()) == 0
    got_hash = fb.hash.cpu().numpy().view(np.uint64)
    got_feat = fb.feat.cpu().numpy().view(np.uint16)
    want = [v for h in hyps for v in S.subtree_features(h)]
    assert len(want) == nodes.shape[0]
    np.testing.assert_array_equal(got_hash, np.array([w[0] for w in want], dtype=np.uint64))
    np.testing.assert_array_equal(got_feat, np.array([w[1] for w in want], dtype=np.uint16))
    x = torch.empty((len(hyps), S.FEATURE_DIM), dtype=torch.bfloat16, device="cuda")
    fb.densify(0, len(hyps), x)
    np.testing.assert_array_equal(f64(torch, x), S.dense_features(hyps))
    # relative to parents: refinements of the first 30 hypotheses, minus their parents' features
    from paper_2412_00802_amd import search
    ref = search.Refiner(kb, np.random.default_rng(2))
    parents = hyps[:30]
    kids, pidx = [], []
    for i, p in enumerate(parents):
        for c in ref.refine(p, 5):
            kids.append(c)
            pidx.append(i)
    kfb, _ = _feature_batch(torch, kids)
    pfb, _ = _feature_batch(torch, parents)
    P = torch.from_numpy(np.asarray(pidx, dtype=np.int32)).cuda()
    xd = torch.empty((len(kids), S.FEATURE_DIM), dtype=torch.bfloat16, device="cuda")
    kfb.densify(3, len(kids) - 3, xd, parents=pfb, parent_index=P)
    np.testing.assert_array_equal(f64(torch, xd)[:len(kids) - 3], S.delta_features(kids, parents, pidx)[3:])
    kfb.densify(3, len(kids) - 3, xd, parents=pfb, parent_index=P, context=1)
    np.testing.assert_array_equal(f64(torch, xd)[:len(kids) - 3],
                                  S.delta_features(kids, parents, pidx, context=True)[3:])


def test_features_flag_malformed_children(torch):
    from paper_2412_00802_amd.screener import FeatureBatch
    nodes = np.array([(3, 0, 0, 0, 0, 0)], dtype=hthedl.NODE_DTYPE)     # NOT whose child is itself
    fb = FeatureBatch(nodes, np.array([0, 1], np.uint32), np.zeros(0, np.uint32))
    torch.cuda.synchronize()
    assert int(fb.bad.item()) == 1


def test_head_loss_and_backward(torch):
    rng = np.random.default_rng(9)
    Bn, Kd = 300, 256
    h = np.maximum(rng.standard_normal((Bn, Kd)), 0).astype(np.float32)
    w = rng.standard_normal((Kd, 2)).astype(np.float32) * 0.1
    b = rng.standard_normal(2).astype(np.float32)
    y = rng.random((Bn, 2)).astype(np.float32)
    H = bf16_dev(torch, h)
    W, Bb, Y = (torch.from_numpy(v).cuda() for v in (w, b, y))
    z = torch.empty((Bn, 2), dtype=torch.float32, device="cuda")
    dz = torch.empty_like(z)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    scale = 1.0 / (2 * Bn)
    hthedl.hth_head_forward(H, Bn, Kd, W, Bb, z, Y, dz, scale, loss)
    hr = S.bf16(h)
    zr = hr @ w + b
    np.testing.assert_allclose(z.cpu().numpy(), zr, rtol=1e-4, atol=1e-4)
    lr = np.sum(np.maximum(zr, 0) - zr * y + np.log1p(np.exp(-np.abs(zr))))
    assert abs(loss.item() - lr) <= 1e-4 * abs(lr)
    dzr = (1 / (1 + np.exp(-zr)) - y) * scale
    np.testing.assert_allclose(dz.cpu().numpy(), dzr, rtol=1e-4, atol=1e-7)
    dw = torch.empty((Kd, 2), dtype=torch.float32, device="cuda")
    dh = torch.empty((Bn, Kd), dtype=torch.bfloat16, device="cuda")
    hthedl.hth_head_backward(H, Bn, Kd, W, dz, dw, dh)
    dzg = dz.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(dw.cpu().numpy(), hr.T @ dzg, rtol=1e-4, atol=1e-8)
    np.testing.assert_allclose(f64(torch, dh), S.bf16((dzg @ w.T) * (hr > 0)), rtol=1e-2, atol=1e-9)
    # the squared-error head (regression of log(1 + removed count))
    yl = (rng.random((Bn, 2)) * 8).astype(np.float32)
    Yl = torch.from_numpy(yl).cuda()
    loss.zero_()
    hthedl.hth_head_forward(H, Bn, Kd, W, Bb, z, Yl, dz, scale, loss, loss_kind=1)
    lr = 0.5 * np.sum((zr - yl) ** 2)
    assert abs(loss.item() - lr) <= 1e-4 * abs(lr)
    np.testing.assert_allclose(dz.cpu().numpy(), (zr - yl) * scale, rtol=1e-4, atol=1e-7)
    with pytest.raises(hthedl.HthError):
        hthedl.hth_head_forward(H, Bn, Kd, W, Bb, z, Yl, dz, scale, loss, loss_kind=2)


def test_adamw_matches_reference(torch):
    rng = np.random.default_rng(3)
    n = 5000
    p, g = rng.standard_normal(n).astype(np.float32), rng.standard_normal(n).astype(np.float32)
    P, G = torch.from_numpy(p.copy()).cuda(), torch.from_numpy(g).cuda()
    Mm, V = torch.zeros_like(P), torch.zeros_like(P)
    pb = torch.empty(n, dtype=torch.bfloat16, device="cuda")
    rp, rm, rv = p.astype(np.float64), np.zeros(n), np.zeros(n)
    for step in (1, 2, 3):
        hthedl.hth_adamw(P, G, Mm, V, pb, n, 1e-2, 0.9, 0.999, 1e-8, 0.01, step)
        rp, rm, rv = S.adamw(rp, g.astype(np.float64), rm, rv, 1e-2, 0.9, 0.999, 1e-8, 0.01, step)
    np.testing.assert_allclose(P.cpu().numpy(), rp, rtol=1e-5, atol=1e-6)
    np.testing.assert_array_equal(f64(torch, pb), S.bf16(P.cpu().numpy()))


@pytest.mark.parametrize("M,N", [(1024, 1024), (1000, 130), (7, 2), (1, 65), (0, 3)])
def test_colsum_matches_reference(torch, M, N):
    """Column sums (bias gradients) of bf16 and fp32 matrices, against fp64
    sums of the same values, with ragged column tiles and row counts that
    are not a multiple of the four waves; two calls give identical bits."""
    rng = np.random.default_rng(M * 31 + N)
    a = rng.standard_normal((M, N)).astype(np.float32)
    for is_bf16 in (1, 0):
        d = torch.from_numpy(a).cuda()
        if is_bf16:
            d = d.to(torch.bfloat16)
        ref = d.float().cpu().numpy().astype(np.float64).sum(axis=0)
        out = torch.full((N,), 7.0, dtype=torch.float32, device="cuda")
        hthedl.hth_colsum(d, is_bf16, M, N, out)
        got = out.cpu().numpy()
        np.testing.assert_allclose(got, ref, rtol=1e-5, atol=1e-4 * max(1.0, np.sqrt(M)))
        again = torch.empty_like(out)
        hthedl.hth_colsum(d, is_bf16, M, N, again)
        np.testing.assert_array_equal(again.cpu().numpy(), got)


@pytest.mark.parametrize("n,k", [(1, 1), (1000, 10), (100003, 2000), (50000, 50000)])
def test_topk(torch, n, k):
    rng = np.random.default_rng(n + k)
    s = rng.standard_normal(n).astype(np.float32)
    s[rng.integers(0, n, size=n // 10)] = 0.5          # many ties
    s[rng.integers(0, n, size=max(1, n // 100))] = np.nan
    D = torch.from_numpy(s).cuda()
    idx = torch.empty(k, dtype=torch.int32, device="cuda")
    work = torch.empty(65538, dtype=torch.int32, device="cuda")
    hthedl.hth_topk(D, n, k, idx, work)
    got = idx.cpu().numpy()
    assert len(set(got.tolist())) == k and got.min() >= 0 and got.max() < n
    key = np.where(np.isnan(s), -np.inf, s)
    np.testing.assert_array_equal(np.sort(key[got]), np.sort(key)[n - k:])


def _gemm_bound(a, b, k):
    """Element-wise bound of an fp32-accumulated product a @ b against its exact
    value: 8 * 2^-24 * sqrt(K) * (|a| @ |b|) (rounding of each partial sum,
    random-walk growth over the reduction length K)."""
    return 8 * 2.0 ** -24 * np.sqrt(k) * (np.abs(a) @ np.abs(b))


def _close(name, got, want, bound, rtol=1e-3):
    """|got - want| <= rtol |want| + bound, element by element."""
    err = np.abs(got - want)
    lim = rtol * np.abs(want) + bound
    bad = np.argwhere(err > lim)
    say(f"[train] {name}: max |err| {err.max():.3e}, worst err/limit {np.max(err / np.maximum(lim, 1e-300)):.3f}")
    assert bad.size == 0, (name, bad[:4].tolist(), got[tuple(bad[0])], want[tuple(bad[0])])


def _half_ulp(name, got_bf16, pre):
    """A stored bf16 value is the exact value rounded to nearest: within half a
    bf16 unit in the last place (2^-8 relative) of the exact fp64 value, plus
    the fp32 accumulation bound carried in `pre[1]`."""
    exact, bound = pre
    _close(name, got_bf16, exact, bound + 1e-30, rtol=2.0 ** -8)


def test_training_step_matches_reference(torch):
    """One training step, element by element.  Each stored tensor of the step
    (h1, h2, z, dz, dh2, dh1) and each gradient is compared with the float64
    product of the operands the GPU itself stored for that step, so both sides
    see identical bf16 roundings: gradients within rel 1e-3 plus the fp32
    accumulation bound of their reduction length, bf16 activations within half
    a bf16 ulp of the exact value.  The whole step is then also compared with
    the independent float64 reference (relative norm, a summary)."""
    from paper_2412_00802_amd.screener import Screener, init_params
    rng = np.random.default_rng(11)
    B = 256
    params = init_params(seed=3)
    params["b1"] = rng.standard_normal(1024).astype(np.float32) * 0.05
    params["b2"] = rng.standard_normal(256).astype(np.float32) * 0.05
    x = (rng.random((B, 4096)) < 0.004).astype(np.float32) * rng.integers(1, 3, size=(B, 4096))
    y = rng.random((B, 2)).astype(np.float32)
    scr = Screener(params, batch=B, lr=1e-3)
    scr.x.copy_(bf16_dev(torch, x))
    Y = torch.from_numpy(y).cuda()
    scr.train_step(B, Y)
    torch.cuda.synchronize()
    scale = 1.0 / (2 * B)
    d = lambda t: t.detach().float().cpu().numpy().astype(np.float64)   # noqa: E731
    xg, h1, h2, z, dz, dh2, dh1 = (d(t) for t in (scr.x, scr.h1, scr.h2, scr.z, scr.dz, scr.dh2, scr.dh1))
    g = {k: d(v) for k, v in scr.g.items()}
    w1b, w2b = S.bf16(params["w1"]), S.bf16(params["w2"])
    w3, b1, b2, b3 = (params[k].astype(np.float64) for k in ("w3", "b1", "b2", "b3"))
    np.testing.assert_array_equal(xg, x)                       # small integers: exact in bf16
    # forward, each layer from the GPU's own stored input
    _half_ulp("h1", h1, (np.maximum(xg @ w1b + b1, 0.0), _gemm_bound(xg, w1b, 4096)))
    _half_ulp("h2", h2, (np.maximum(h1 @ w2b + b2, 0.0), _gemm_bound(h1, w2b, 1024)))
    _close("z", z, h2 @ w3 + b3, _gemm_bound(h2, w3, 256), rtol=1e-5)
    _close("dz", dz, (1.0 / (1.0 + np.exp(-z)) - y) * scale, 1e-9, rtol=1e-5)
    # backward
    _close("g.w3", g["w3"], h2.T @ dz, _gemm_bound(h2.T, dz, B))
    _close("g.b3", g["b3"], dz.sum(0), _gemm_bound(np.ones((1, B)), dz, B)[0])
    _half_ulp("dh2", dh2, ((dz @ w3.T) * (h2 > 0), _gemm_bound(dz, w3.T, 2)))
    _close("g.w2", g["w2"], h1.T @ dh2, _gemm_bound(h1.T, dh2, B))
    _close("g.b2", g["b2"], dh2.sum(0), _gemm_bound(np.ones((1, B)), dh2, B)[0])
    _half_ulp("dh1", dh1, ((dh2 @ w2b.T) * (h1 > 0), _gemm_bound(dh2, w2b.T, 256)))
    _close("g.w1", g["w1"], xg.T @ dh1, _gemm_bound(xg.T, dh1, B))
    _close("g.b1", g["b1"], dh1.sum(0), _gemm_bound(np.ones((1, B)), dh1, B)[0])
    # summary against the independent float64 reference of the whole step
    p64 = {k: v.astype(np.float64) for k, v in params.items()}
    acts, loss = S.forward(p64, x.astype(np.float64), y.astype(np.float64), rounding=True)
    gr = S.backward(p64, acts, y.astype(np.float64), scale, rounding=True)
    assert abs(scr.loss.item() - loss) <= 2e-3 * abs(loss)
    for k in ("w3", "b3", "w2", "b2", "w1", "b1"):
        rel = np.linalg.norm(g[k] - gr[k]) / max(np.linalg.norm(gr[k]), 1e-30)
        say(f"[train] grad {k}: relative error against the whole-step reference {rel:.2e}")
        assert rel < 2e-2, (k, rel)


def test_training_lowers_loss(torch):
    """A learnable target: the covered fractions are functions of a few features."""
    from paper_2412_00802_amd.screener import Screener, init_params
    rng = np.random.default_rng(12)
    B = 512
    x = (rng.random((B, 4096)) < 0.003).astype(np.float32)
    u = x[:, :64].sum(1) + 2 * x[:, 64:128].sum(1)
    y = np.stack([1 / (1 + np.exp(-(u - 0.5))), 1 / (1 + np.exp(u - 0.5))], 1).astype(np.float32)
    scr = Screener(init_params(seed=4), batch=B, lr=2e-3)
    scr.x.copy_(bf16_dev(torch, x))
    Y = torch.from_numpy(y).cuda()
    losses = []
    for _ in range(60):
        scr.loss.zero_()
        scr.train_step(B, Y)
        losses.append(scr.loss.item() / (2 * B))
    # BCE against soft targets is bounded below by the targets' entropy
    ent = -np.mean(y * np.log(y) + (1 - y) * np.log(1 - y))
    say(f"[train] loss {losses[0]:.4f} -> {losses[-1]:.4f} (entropy floor {ent:.4f})")
    assert losses[-1] - ent < 0.3 * (losses[0] - ent)


def test_head_score_with_and_without_base(torch):
    rng = np.random.default_rng(21)
    n, n_pos, n_neg = 3000, 5000, 7000
    z = rng.standard_normal((n, 2)).astype(np.float32) * 3
    base = np.stack([rng.integers(0, n_pos + 1, n), rng.integers(0, n_neg + 1, n)], 1).astype(np.uint32)
    Z = torch.from_numpy(z).cuda()
    B = torch.from_numpy(base.view(np.int32)).cuda()
    out = torch.empty(n, dtype=torch.float32, device="cuda")
    hthedl.hth_head_score(Z, n, float(n_pos), float(n_neg), out)
    np.testing.assert_allclose(out.cpu().numpy(), S.predicted_f1(z.astype(np.float64), n_pos, n_neg),
                               rtol=2e-5, atol=1e-7)
    hthedl.hth_head_score(Z, n, float(n_pos), float(n_neg), out, base=B)
    np.testing.assert_allclose(out.cpu().numpy(), S.predicted_f1(z.astype(np.float64), n_pos, n_neg, base),
                               rtol=2e-5, atol=1e-7)
    zl = (rng.random((n, 2)) * 10 - 1).astype(np.float32)       # log(1 + removed), some below 0
    hthedl.hth_head_score(torch.from_numpy(zl).cuda(), n, float(n_pos), float(n_neg), out, base=B, kind=1)
    np.testing.assert_allclose(out.cpu().numpy(),
                               S.predicted_f1(zl.astype(np.float64), n_pos, n_neg, base, kind="log_removed"),
                               rtol=1e-4, atol=1e-6)
    with pytest.raises(hthedl.HthError):
        hthedl.hth_head_score(Z, n, float(n_pos), float(n_neg), out, kind=1)
