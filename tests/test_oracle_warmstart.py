"""Pins of the warm-start network's CPU reference (oracle/warmstart_ref.py).

The reference is the definition the BF16 MFMA kernels are held to.  Here it is checked
against things it does not compute itself: its backward pass against central finite
differences of its own loss (plain FP64 network), the invariance of the loss under a shift
of the outputs (the dual is defined up to a constant), and its BF16 rounding against
PyTorch's conversion to bfloat16.
"""
import numpy as np
import pytest

from oracle import warmstart_ref as R

torch = pytest.importorskip("torch")


def tiny(seed=0, B=2, m=5, n=6):
    rng = np.random.default_rng(seed)
    flat = np.zeros(R.param_count())
    p = R.unpack(flat)
    for name, r, c in R.SHAPES:
        p[name] = rng.standard_normal((r, c)) * (np.sqrt(2.0 / r) if r > 1 else 0.1)
    flat = R.pack(p)
    fs = rng.standard_normal((B * m, 4))
    fte = rng.standard_normal((B * n, 4))
    fth = rng.standard_normal((B * n, 4))
    t = rng.standard_normal(B * n)
    return flat, fs, fte, fth, t, B, m, n


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-30, 30, 10000),
                        [0.0, -0.0, 1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -2.5, 3.4e38]])
    x32 = x.astype(np.float32)
    ref = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(R.bf16_round(x32), ref)
    # ties go to even: 1 + 2^-8 is halfway between 1 and 1 + 2^-7
    assert R.bf16_round(np.float32(1.0 + 2.0 ** -8)) == 1.0


def test_gradient_against_finite_differences():
    flat, fs, fte, fth, t, B, m, n = tiny()
    L, g, _ = R.loss_and_grad(flat, fs, fte, fth, t, B, m, n, bf16=False)
    rng = np.random.default_rng(1)
    offs, off = {}, 0
    for name, r, c in R.SHAPES:
        offs[name] = (off, r * c)
        off += r * c
    idx = []
    for name, (o, cnt) in offs.items():
        idx += list(o + rng.choice(cnt, min(cnt, 6), replace=False))
    h = 1e-6
    for i in idx:
        fp, fm = flat.copy(), flat.copy()
        fp[i] += h
        fm[i] -= h
        Lp = R.loss(R.forward(fp, fs, fte, fth, B, m, n, False)[0], t, B, n)
        Lm = R.loss(R.forward(fm, fs, fte, fth, B, m, n, False)[0], t, B, n)
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * (abs(fd) + abs(g[i])) + 1e-9, (i, fd, g[i])


def test_loss_ignores_output_shift():
    """The outputs are centred per instance: the output bias bo changes nothing, so its
    gradient is zero, and the loss is the same after any shift of bo."""
    flat, fs, fte, fth, t, B, m, n = tiny(seed=2)
    L, g, _ = R.loss_and_grad(flat, fs, fte, fth, t, B, m, n, bf16=False)
    assert abs(g[-1]) <= 1e-14
    f2 = flat.copy()
    f2[-1] += 3.0
    assert abs(R.loss(R.forward(f2, fs, fte, fth, B, m, n, False)[0], t, B, n) - L) <= 1e-13


def test_pooling_is_a_mean_over_each_instance():
    """Permuting the points inside an instance leaves its outputs permuted the same way
    (targets) or unchanged (sources): the network is a function of the point sets."""
    flat, fs, fte, fth, t, B, m, n = tiny(seed=4)
    O, _ = R.forward(flat, fs, fte, fth, B, m, n, False)
    ps, pt = np.random.default_rng(0).permutation(m), np.random.default_rng(1).permutation(n)
    fs2 = fs.reshape(B, m, 4)[:, ps].reshape(-1, 4)
    fte2 = fte.reshape(B, n, 4)[:, pt].reshape(-1, 4)
    fth2 = fth.reshape(B, n, 4)[:, pt].reshape(-1, 4)
    O2, _ = R.forward(flat, fs2, fte2, fth2, B, m, n, False)
    np.testing.assert_allclose(O2.reshape(B, n), O.reshape(B, n)[:, pt], rtol=1e-12, atol=1e-12)
