"""Pins of the warm-start network's CPU reference (oracle/warmstart_ref.py).

The reference is the definition the BF16 MFMA kernels are held to.  Here it is checked
against things it does not compute itself: its backward pass against central finite
differences of its own loss (plain FP64 network), the invariance of the loss under a shift
of the outputs (the dual is defined up to a constant), its BF16 rounding against PyTorch's
conversion to bfloat16, and its features against closed forms: the Laplacian of the
smoothed potentials (finite differences against the analytic density), their mirror
symmetry, the scale as a brute-force nearest-neighbour distance, and invariance under a
shift and a uniform scaling of the points.
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
    fth = rng.standard_normal((B * n, R.NFH))
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
        # central differences carry about eps |L| / h of rounding (2e-10 |L| here)
        assert abs(fd - g[i]) <= 1e-6 * (abs(fd) + abs(g[i])) + 1e-9 * (1 + abs(L)), \
            (i, fd, g[i])


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
    fth2 = fth.reshape(B, n, R.NFH)[:, pt].reshape(-1, R.NFH)
    O2, _ = R.forward(flat, fs2, fte2, fth2, B, m, n, False)
    np.testing.assert_allclose(O2.reshape(B, n), O.reshape(B, n)[:, pt], rtol=1e-12, atol=1e-12)


def _green_at(R_, xs, ys, a, b, hi, q):
    """The potential features at an arbitrary point q (one extra target of weight 0)."""
    yy = np.vstack([ys, q[None]])
    bb = np.concatenate([b, [0.0]])
    return R_.green_potentials(xs, yy, a, bb, hi)[-1]


def test_green_potentials_laplacian():
    """Laplacian of log(r^2 + e^2)/2 in the plane is 2 e^2 / (r^2 + e^2)^2: the five-point
    finite-difference Laplacian of G_k at a probe point equals that density summed over the
    nine images of every point, sources with +a_i and targets with -b_l."""
    rng = np.random.default_rng(5)
    m, n = 7, 5
    xs, ys = rng.random((m, 2)), rng.random((n, 2))
    a = rng.uniform(0.5, 1.5, m); a /= a.sum()
    b = rng.uniform(0.5, 1.5, n); b /= b.sum()
    hi = np.array([1.0, 1.0])
    q = np.array([0.37, 0.61])
    h = 1e-4   # truncation ~(h / r)^2 with r the distance to the nearest point; rounding ~1e-16 / h^2
    lap = (_green_at(R, xs, ys, a, b, hi, q + [h, 0]) + _green_at(R, xs, ys, a, b, hi, q - [h, 0])
           + _green_at(R, xs, ys, a, b, hi, q + [0, h]) + _green_at(R, xs, ys, a, b, hi, q - [0, h])
           - 4 * _green_at(R, xs, ys, a, b, hi, q)) / h ** 2
    for k, e in enumerate(R.GREEN_EPS):
        dens = 0.0
        for P, w, sgn in ((xs, a, 1.0), (ys, b, -1.0)):
            for i in range(len(P)):
                for px in (-P[i, 0], P[i, 0], 2.0 - P[i, 0]):
                    for py in (-P[i, 1], P[i, 1], 2.0 - P[i, 1]):
                        r2 = (px - q[0]) ** 2 + (py - q[1]) ** 2
                        dens += sgn * w[i] * 2 * e * e / (r2 + e * e) ** 2
        assert abs(lap[k] - dens) <= 1e-4 * abs(dens), (k, lap[k], dens)


def test_green_potentials_mirror_symmetry():
    """With the reflections across both sides of the box, mirroring every point about the
    box centre line x1 = h1/2 mirrors the potentials (a missing image breaks this)."""
    rng = np.random.default_rng(6)
    xs, ys = rng.random((9, 2)) * [0.8, 1.0], rng.random((6, 2)) * [0.8, 1.0]
    hi = np.array([0.8, 1.0])
    a, b = np.full(9, 1 / 9), np.full(6, 1 / 6)
    G = R.green_potentials(xs, ys, a, b, hi)
    mx = lambda P: np.column_stack([hi[0] - P[:, 0], P[:, 1]])
    Gm = R.green_potentials(mx(xs), mx(ys), a, b, hi)
    np.testing.assert_allclose(Gm, G, rtol=0, atol=1e-12)


def test_features_scale_and_invariance():
    """scale = u s with u the cost of a unit box distance squared and s^2 the mean squared
    distance from a target to its nearest source in box units (brute force from the
    points); features are unchanged by a shift and a uniform scaling of all points (the
    cost scaled to match), and the scale follows the cost."""
    rng = np.random.default_rng(7)
    m, n = 40, 30
    x, y = rng.random((m, 2)) * [2.0, 1.5], rng.random((n, 2)) * [2.0, 1.5]
    a, b = np.full(m, 1 / m), np.full(n, 1 / n)
    C = 0.7 * ((x[:, None] - y[None]) ** 2).sum(-1)
    fs, fte, fth, scale = R.features(x, y, a, b, C)
    P = np.vstack([x, y])
    L = (P.max(0) - P.min(0)).max()
    nn2 = ((x[:, None] - y[None]) ** 2).sum(-1).min(0) / L ** 2
    u = 0.7 * L ** 2
    assert abs(scale - u * np.sqrt(nn2.mean())) <= 1e-12 * scale
    assert fth.shape == (n, R.NFH)
    np.testing.assert_allclose(fth[:, 4:].mean(0), 0.0, atol=1e-12)
    c, t = 3.5, np.array([-1.0, 4.0])
    fs2, fte2, fth2, scale2 = R.features(c * x + t, c * y + t, a, b, c * c * C)
    for u1, u2 in ((fs, fs2), (fte, fte2), (fth, fth2)):
        np.testing.assert_allclose(u2, u1, rtol=1e-9, atol=1e-9)
    assert abs(scale2 - c * c * scale) <= 1e-12 * scale2
