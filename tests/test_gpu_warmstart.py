"""The learned warm start's BF16 MFMA kernels against the CPU reference of the network.

Both sides round every operand of a matrix product to BF16 at the same places; the library
accumulates in FP32, the reference in FP64, so the remaining differences come from the
accumulation order and from the rare intermediate whose BF16 rounding the two sides take
differently (an FP32 value within ~1e-7 of a BF16 rounding boundary).  Error model: one such
flip moves one operand of a product by a BF16 unit (2^-8 relative) and the product by about
2^-8 / 256 of its scale, so outputs and gradients are held to 1e-3 of the largest entry of
their block.  Sizes span several 64 x 64 tiles with ragged edges (m, n not multiples of 64).
"""
import numpy as np
import pytest

from oracle import warmstart_ref as R
from paper_2603_07156_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ib():
    from paper_2603_07156_amd import ibsn
    return ibsn


@pytest.fixture(scope="module")
def ctx(ib):
    return ib.Context(0)


def batch(B, m, n, seed):
    feats = []
    rng = np.random.default_rng(seed)
    for b in range(B):
        inst = W.uniform_points(n, seed + b, m=m)
        x = np.random.default_rng(seed + b).random((m, 2))
        y = np.random.default_rng(seed + b + 1000).random((n, 2))
        C = ((x[:, None] - y[None]) ** 2).sum(-1)
        C /= C.max()
        a = rng.uniform(0.5, 1.5, m)
        a /= a.sum()
        feats.append(R.features(x, y, a, inst.b, C))
    fs = np.concatenate([f[0] for f in feats]).astype(np.float32)
    fte = np.concatenate([f[1] for f in feats]).astype(np.float32)
    fth = np.concatenate([f[2] for f in feats]).astype(np.float32)
    t = rng.standard_normal(B * n).astype(np.float32)
    return fs, fte, fth, t


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def random_params(ws, seed):
    """Every parameter random (the library starts Wc, ws and the biases at zero, which
    would leave most of the network out of the outputs and gradients): matrices with the
    He scale, biases and the linear path with std 0.1.  Returns the FP64 copy."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, r, c in R.SHAPES:
        sd = np.sqrt(2.0 / r) if (r > 1 and name != "ws") else 0.1
        p[name] = rng.standard_normal((r, c)) * sd
    flat = R.pack(p).astype(np.float32)
    ws.set_params(flat)
    return flat.astype(np.float64)


def test_forward_matches_reference(ib, ctx):
    B, m, n = 2, 70, 90
    ws = ib.WarmStart(ctx, seed=5)
    flat = random_params(ws, 5)
    fs, fte, fth, _ = batch(B, m, n, 11)
    out = ws.forward(B, m, n, dev(fs), dev(fte), dev(fth)).cpu().numpy().astype(np.float64)
    ref, _ = R.forward(flat, fs, fte, fth, B, m, n, bf16=True)
    scale = np.abs(ref).max()
    assert scale > 0
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-3 * scale)
    # the reference without BF16 rounding differs by more on the typical entry: the rounding
    # points are what is held (the largest differences come from the rare flips above)
    plain, _ = R.forward(flat, fs, fte, fth, B, m, n, bf16=False)
    assert np.median(np.abs(plain - ref)) > 10 * np.median(np.abs(out - ref))
    ws.free()


def test_gradient_matches_reference(ib, ctx):
    B, m, n = 3, 100, 77
    ws = ib.WarmStart(ctx, seed=6)
    flat = random_params(ws, 6)
    fs, fte, fth, t = batch(B, m, n, 21)
    loss, grad = ws.train_step(B, m, n, dev(fs), dev(fte), dev(fth), dev(t), 0.0, want_grad=True)
    L, g, _ = R.loss_and_grad(flat, fs, fte, fth, t, B, m, n, bf16=True)
    assert abs(loss - L) <= 1e-3 * abs(L)
    off = 0
    for name, r, c in R.SHAPES:
        blk, ref = grad[off:off + r * c].astype(np.float64), g[off:off + r * c]
        off += r * c
        if name == "bo":   # zero by construction (centred outputs): FP32 sums of +-terms
            assert abs(blk[0]) <= 1e-6 * np.abs(g).max()
            continue
        # The encoder's gradients pass through the pooled gradient dCTX, broadcast to every
        # point of an instance: one BF16 rounding flip in dCTX (the two sides accumulate in
        # FP32 and FP64) moves a whole instance's contribution to a column by 2^-8, about
        # 2^-8 / B of the largest entry.  The head's gradients see no such broadcast.
        enc = name in ("W1", "b1", "W2", "b2", "W3", "b3")
        tol = (1.5 * 2.0 ** -8 / B if enc else 1e-3) * np.abs(ref).max()
        np.testing.assert_allclose(blk, ref, rtol=0, atol=tol + 1e-30, err_msg=name)
    # lr = 0 leaves the parameters as they were
    np.testing.assert_array_equal(ws.params(), flat.astype(np.float32))
    ws.free()


def test_training_reduces_loss_and_adam_step(ib, ctx):
    """Adam steps on a fixed batch lower the loss; the first step moves each parameter by
    lr sign(g) (Adam's first step with bias correction), up to eps."""
    B, m, n = 2, 64, 64
    ws = ib.WarmStart(ctx, seed=7)
    flat0 = random_params(ws, 7)
    fs, fte, fth, t = batch(B, m, n, 31)
    _, g = ws.train_step(B, m, n, dev(fs), dev(fte), dev(fth), dev(t), 0.0, want_grad=True)
    lr = 1e-3
    l0, _ = ws.train_step(B, m, n, dev(fs), dev(fte), dev(fth), dev(t), lr)
    step = ws.params().astype(np.float64) - flat0
    big = np.abs(g) > 1e-4 * np.abs(g).max()
    np.testing.assert_allclose(step[big], -lr * np.sign(g[big]), rtol=1e-3, atol=1e-9)
    losses = [l0]
    for _ in range(30):
        losses.append(ws.train_step(B, m, n, dev(fs), dev(fte), dev(fth), dev(t), lr)[0])
    assert losses[-1] < 0.7 * losses[0], losses
    ws.free()


def test_features_and_predict(ib, ctx):
    m, n = 300, 257
    inst = W.uniform_points(n, 4, m=m)
    x = np.random.default_rng(4).random((m, 2))
    y = np.random.default_rng(1004).random((n, 2))
    C = ((x[:, None] - y[None]) ** 2).sum(-1)
    C /= C.max()
    pr = ib.Problem(dev(C), dev(inst.a), dev(inst.b), 1e-6)
    ws = ib.WarmStart(ctx, seed=8)
    fs, fte, fth, scale = ws.features(pr, dev(x), dev(y))
    rfs, rfte, rfth, rscale = R.features(x, y, inst.a, inst.b, C)
    assert abs(scale - rscale) <= 1e-12 * rscale
    for gpu, ref in ((fs, rfs), (fte, rfte), (fth[:, :4], rfth[:, :4])):
        np.testing.assert_allclose(gpu.cpu().numpy(), ref.astype(np.float32), rtol=2e-7,
                                   atol=1e-7)
    # the potentials: FP32 box coordinates and logs (one rounding each, ~6e-8 relative) over
    # 9 (m + n) terms of size ~|log d| / m whose weighted sum cancels to ~1e-3 before the
    # division by s (~0.02): about 1e-5 of the largest feature, held to 1e-4
    gp = fth[:, 4:].cpu().numpy().astype(np.float64)
    rp = rfth[:, 4:]
    np.testing.assert_allclose(gp, rp, rtol=0, atol=1e-4 * np.abs(rp).max())
    gam = ws.predict(m, n, fs, fte, fth, scale).cpu().numpy()
    o = ws.forward(1, m, n, fs, fte, fth).cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(gam, scale * (o - o.mean()), rtol=1e-12, atol=1e-18)
    assert abs(gam.sum()) <= 1e-12 * np.abs(gam).sum()
    ws.free()


def test_initial_output_is_zero(ib, ctx):
    """A new model starts with zero biases, linear path and context map: every output is
    exactly 0, and the parameters other than those are He-scaled."""
    ws = ib.WarmStart(ctx, seed=9)
    fs, fte, fth, _ = batch(1, 64, 80, 41)
    out = ws.forward(1, 64, 80, dev(fs), dev(fte), dev(fth)).cpu().numpy()
    assert np.all(out == 0.0)
    p = R.unpack(ws.params().astype(np.float64))
    for name, r, c in R.SHAPES:
        if r == 1 or name in ("ws", "Wc"):
            assert np.all(p[name] == 0.0), name
        else:
            assert abs(p[name].std() / np.sqrt(2.0 / r) - 1.0) < 0.1, name
    ws.free()
