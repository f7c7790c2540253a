"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle (oracle/ibsn_oracle.c) against something other than
itself: exact LP optima (brute force, the Hungarian method, HiGHS), closed forms,
the paper's theorems and identities, finite differences, and an independent
log-domain Sinkhorn for the entropic problem.  None of these runs on a GPU.
"""
import itertools

import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment, linprog

import oracle as orc
from paper_2603_07156_amd import workloads as W


def dense_center(C, r, s, k, eta):
    """X^k_ij = exp(r_i + s_j - k C_ij / eta) written out as a matrix."""
    return np.exp(r[:, None] + s[None, :] - k * C / eta)


def state_after(inst, k, gamma_seed=1):
    """An outer state (r, s, k) and a dual gamma reached by running k exact-ish outer
    iterations of the oracle, for tests that need k > 0."""
    opt = orc.default_options(max_outer=k, gap_tol=0.0, marg_tol=0.0)
    res = orc.solve(inst.C, inst.a, inst.b, inst.eta, options=opt)
    return res["r"], res["s"], res["k"], res["gamma"]


# ---------------------------------------------------------------------------
# end results: exact LP optima
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,seed", [(4, 0), (5, 1), (6, 2), (7, 3)])
def test_p1_bruteforce_permutations(n, seed):
    """Uniform weights: the LP optimum is attained at a permutation matrix / n
    (Birkhoff), so f* = min over all n! permutations (eq. (1))."""
    inst = W.uniform_points(n, seed)
    fstar = min(inst.C[np.arange(n), list(p)].sum() for p in itertools.permutations(range(n))) / n
    opt = orc.default_options(max_outer=20000, gap_tol=1e-12, marg_tol=0.0)
    res = orc.solve(inst.C, inst.a, inst.b, inst.eta, options=opt, want_plan=True)
    rep = res["report"]
    assert res["status"] == 0
    assert rep["dual"] <= fstar * (1 + 1e-13)
    assert abs(rep["primal"] - fstar) <= 1e-10 * fstar
    # the rounded plan is feasible and its cost is the reported primal
    X = res["plan"]
    assert np.allclose(X.sum(1), inst.a, atol=1e-15 * n, rtol=0)
    assert np.allclose(X.sum(0), inst.b, atol=1e-15 * n, rtol=0)
    assert abs((inst.C * X).sum() - rep["primal"]) <= 1e-15


def test_p1_hungarian_n64():
    """Uniform weights at n=64: f* from the Hungarian method; the certified relative gap
    1e-8 must bracket it."""
    inst = W.uniform_points(64, 0)
    r, c = linear_sum_assignment(inst.C)
    fstar = inst.C[r, c].sum() / 64
    opt = orc.default_options(max_outer=20000, gap_tol=1e-8, marg_tol=0.0)
    res = orc.solve(inst.C, inst.a, inst.b, inst.eta, options=opt)
    rep = res["report"]
    assert res["status"] == 0
    assert rep["rel_gap"] <= 1e-8
    assert rep["dual"] <= fstar * (1 + 1e-14) and rep["primal"] >= fstar * (1 - 1e-14)
    assert (rep["primal"] - fstar) / fstar <= 1e-8


@pytest.mark.parametrize("m,n,seed", [(12, 16, 100), (24, 20, 101)])
def test_p2_highs_general_weights(m, n, seed):
    """Non-uniform weights and m != n: f* from HiGHS on the dense LP (eq. (1))."""
    inst = W.gmm_points(n, seed, m=m)
    A_eq = np.zeros((m + n, m * n))
    for i in range(m):
        A_eq[i, i * n:(i + 1) * n] = 1.0
    for j in range(n):
        A_eq[m + j, j::n] = 1.0
    lp = linprog(inst.C.ravel(), A_eq=A_eq, b_eq=np.concatenate([inst.a, inst.b]),
                 bounds=(0, None), method="highs")
    fstar = lp.fun
    opt = orc.default_options(max_outer=20000, gap_tol=1e-10, marg_tol=0.0)
    res = orc.solve(inst.C, inst.a, inst.b, inst.eta, options=opt)
    rep = res["report"]
    assert res["status"] == 0
    assert abs(rep["primal"] - fstar) <= 1e-8 * fstar
    assert rep["dual"] <= fstar * (1 + 1e-8)


# ---------------------------------------------------------------------------
# eval pass: definitions, derivatives, invariances
# ---------------------------------------------------------------------------
def test_eval_matches_explicit_center():
    """The implicit centre log X^k = r + s - kC/eta reproduces eq. (5)-(8) computed
    from an explicitly stored X^k (small sizes, no overflow), at k = 0 and k = 3."""
    inst = W.gmm_points(12, 7, m=9)
    eta = 0.1
    for k in (0, 3):
        if k == 0:
            r, s, kk, gamma = np.log(inst.a), np.log(inst.b), 0, W.random_dual(12, 3, 0.05)
        else:
            inst2 = W.Instance(inst.C, inst.a, inst.b, eta, "x")
            r, s, kk, gamma = state_after(inst2, k)
        Xk = dense_center(inst.C, r, s, kk, eta)
        Kmat = Xk * np.exp((gamma[None, :] - inst.C) / eta)
        P = Kmat / Kmat.sum(1, keepdims=True)                       # eq. (7)
        L = -inst.b @ gamma + eta * inst.a @ np.log(Kmat.sum(1))    # eq. (6)
        ev = orc.eval_pass(inst.C, inst.a, inst.b, eta, gamma, r=r, s=s, k=kk, want_plan=True)
        np.testing.assert_allclose(ev.plan, inst.a[:, None] * P, rtol=1e-12, atol=1e-300)
        np.testing.assert_allclose(ev.g, P.T @ inst.a - inst.b, rtol=0, atol=1e-14)   # eq. (8)
        assert abs(ev.L - L) <= 1e-12 * (abs(L) + eta * np.abs(inst.a @ r) + 1)


def test_p5_finite_difference_gradient_and_hessian():
    """g = grad L (eq. (8)) and H (eq. (8)) = Jacobian of g, by central differences;
    the Hessian is probed through the HVP with rho = 0 (P_rho = P, Algorithm 1)."""
    inst = W.gmm_points(10, 5, m=8)
    eta = 0.05
    gamma = W.random_dual(10, 9, 0.02)
    r, s = np.log(inst.a), np.log(inst.b)
    ev = orc.eval_pass(inst.C, inst.a, inst.b, eta, gamma, r=r, s=s)
    h = 1e-6
    gfd = np.empty(10)
    Hfd = np.empty((10, 10))
    for j in range(10):
        e = np.zeros(10)
        e[j] = h
        Lp = orc.eval_pass(inst.C, inst.a, inst.b, eta, gamma + e, r=r, s=s)
        Lm = orc.eval_pass(inst.C, inst.a, inst.b, eta, gamma - e, r=r, s=s)
        gfd[j] = (Lp.L - Lm.L) / (2 * h)
        Hfd[:, j] = (Lp.g - Lm.g) / (2 * h)
    np.testing.assert_allclose(ev.g, gfd, rtol=0, atol=1e-6 * np.abs(ev.g).max() + 1e-9)
    csr = orc.sparsify(inst.C, inst.a, eta, gamma, ev.M, ev.S, 0.0, s=s)
    H = np.stack([orc.hvp(csr, inst.a, eta, 0.0, np.eye(10)[j]) for j in range(10)], 1)
    np.testing.assert_allclose(H, Hfd, rtol=0, atol=1e-6 * np.abs(H).max())


def test_p12_shift_invariance():
    """L(gamma + c 1) = L(gamma) and P is unchanged (1^T a = 1^T b = 1, eq. (6)-(7))."""
    inst = W.uniform_points(40, 3)
    gamma = W.random_dual(40, 1, 0.01)
    e0 = orc.eval_pass(inst.C, inst.a, inst.b, inst.eta, gamma, want_plan=True)
    e1 = orc.eval_pass(inst.C, inst.a, inst.b, inst.eta, gamma + 0.0137, want_plan=True)
    assert abs(e0.L - e1.L) <= 1e-13 * (abs(e0.L) + 1)
    np.testing.assert_allclose(e0.plan, e1.plan, rtol=1e-11, atol=1e-300)


def test_p13_semi_dual_equals_two_dual_plus_constant():
    """L^k(gamma) = Z^k(gamma, zeta(gamma)) + eta sum a log a - eta, with zeta from eq. (5)
    and Z^k from eq. (4) evaluated on an explicit X^k (proof of Lemma 3.1)."""
    inst = W.gmm_points(14, 11, m=10)
    eta = 0.1
    inst2 = W.Instance(inst.C, inst.a, inst.b, eta, "x")
    r, s, k, gamma = state_after(inst2, 2)
    gamma = gamma + W.random_dual(14, 4, 0.01)
    Xk = dense_center(inst.C, r, s, k, eta)
    zeta = eta * np.log(inst.a) - eta * np.log((Xk * np.exp((gamma[None] - inst.C) / eta)).sum(1))
    Z = (-inst.a @ zeta - inst.b @ gamma
         + eta * (Xk * np.exp((zeta[:, None] + gamma[None] - inst.C) / eta)).sum())
    ev = orc.eval_pass(inst.C, inst.a, inst.b, eta, gamma, r=r, s=s, k=k)
    const = eta * inst.a @ np.log(inst.a) - eta
    assert abs(ev.L - (Z + const)) <= 1e-12 * (abs(ev.L) + 1)


def test_p17_sinkhorn_step_is_two_dual_alternation():
    """The warm-up step gamma_j += eta log(b_j / c_j) equals minimising Z^k (eq. (4))
    over gamma with zeta = zeta(gamma) fixed (closed form from dZ/dgamma = 0)."""
    inst = W.gmm_points(16, 2, m=12)
    eta = 0.1
    gamma = W.random_dual(16, 5, 0.05)
    r, s = np.log(inst.a), np.log(inst.b)
    ev = orc.eval_pass(inst.C, inst.a, inst.b, eta, gamma, r=r, s=s)
    step = gamma + eta * (np.log(inst.b) - np.log(ev.c))
    Xk = dense_center(inst.C, r, s, 0, eta)
    zeta = eta * np.log(inst.a) - eta * np.log((Xk * np.exp((gamma[None] - inst.C) / eta)).sum(1))
    alt = eta * np.log(inst.b) - eta * np.log((Xk * np.exp((zeta[:, None] - inst.C) / eta)).sum(0))
    np.testing.assert_allclose(step, alt, rtol=0, atol=1e-13)


# ---------------------------------------------------------------------------
# Algorithm 1: sparsification; Theorems 3.2-3.4 and the E_P lemma
# ---------------------------------------------------------------------------
def _hrho_dense(csr, a, eta):
    n = csr.n
    return np.stack([orc.hvp(csr, a, eta, 0.0, np.eye(n)[j]) for j in range(n)], 1)


@pytest.fixture(scope="module")
def sparse_case():
    inst = W.gmm_points(24, 21, m=20)
    eta = 0.02
    gamma = W.random_dual(24, 2, 0.02)
    s = np.log(inst.b)
    ev = orc.eval_pass(inst.C, inst.a, inst.b, eta, gamma, s=s, want_plan=True)
    P = ev.plan / inst.a[:, None]
    return inst, eta, gamma, s, ev, P


def test_p6_rho_zero_keeps_P(sparse_case):
    inst, eta, gamma, s, ev, P = sparse_case
    csr = orc.sparsify(inst.C, inst.a, eta, gamma, ev.M, ev.S, 0.0, s=s)
    assert csr.nnz == P.size
    expect = P / P.sum(1, keepdims=True)        # kept sum kappa_i = whole row
    expect[csr.istar] = P[csr.istar]            # row i* copied unchanged
    np.testing.assert_allclose(csr.dense(), expect, rtol=1e-14, atol=0)
    np.testing.assert_allclose(csr.d, csr.dense().T @ inst.a, rtol=1e-14)


@pytest.mark.parametrize("rho", [0.0, 1e-4, 1e-3, 1e-2, 5e-2])
def test_p7_p8_p9_p10_theorems(sparse_case, rho):
    inst, eta, gamma, s, ev, P = sparse_case
    m, n = P.shape
    csr = orc.sparsify(inst.C, inst.a, eta, gamma, ev.M, ev.S, rho, s=s)
    Pr = csr.dense()
    istar = csr.istar
    assert istar == int(np.argmax(inst.a))
    # Algorithm 1 step 3, element by element
    for i in range(m):
        if i == istar:
            np.testing.assert_allclose(Pr[i], P[i], rtol=1e-14, atol=0)
        else:
            keep = P[i] >= rho
            np.testing.assert_allclose(Pr[i], np.where(keep, P[i], 0) / P[i][keep].sum(),
                                       rtol=1e-13, atol=0)
    Hr = _hrho_dense(csr, inst.a, eta)
    # Theorem 3.2: symmetric PSD with H_rho 1 = 0
    np.testing.assert_allclose(Hr, Hr.T, atol=1e-13 * np.abs(Hr).max())
    np.testing.assert_allclose(Hr @ np.ones(n), 0, atol=1e-12 * np.abs(Hr).max())
    lam = np.linalg.eigvalsh(0.5 * (Hr + Hr.T))
    assert lam.min() >= -1e-12 * lam.max()
    # Theorem 3.3 on the complement of span{1}
    Q = np.linalg.qr(np.concatenate([np.ones((n, 1)), np.eye(n)[:, : n - 1]], 1))[0][:, 1:]
    lam_perp = np.linalg.eigvalsh(Q.T @ Hr @ Q)
    p = P[istar].min()
    assert lam_perp.min() >= n * inst.a[istar] * p ** 2 / eta * (1 - 1e-10)
    assert lam.max() <= 1 / (2 * eta) * (1 + 1e-12)
    # Theorem 3.4
    csr0 = orc.sparsify(inst.C, inst.a, eta, gamma, ev.M, ev.S, 0.0, s=s)
    H = _hrho_dense(csr0, inst.a, eta)
    assert np.linalg.norm(H - Hr, 2) <= 6 * m * n * inst.a.max() * rho / eta + 1e-12
    # lemma (bound for E_P): per-row identity ||P_i - P_rho,i||_1 = 2 r_i, r_i = dropped mass
    for i in range(m):
        if i == istar:
            continue
        r_i = P[i][P[i] < rho].sum()
        assert abs(np.abs(P[i] - Pr[i]).sum() - 2 * r_i) <= 1e-14
    EP = P - Pr
    assert np.abs(EP).sum(1).max() <= 2 * n * rho + 1e-14
    assert np.abs(EP).sum(0).max() <= 2 * m * n * rho + 1e-14


def test_p11_cg_direction_in_complement(sparse_case):
    """Lemma 4.1: the Newton direction satisfies 1^T Delta = 0 (CG from 0 on 1-perp)."""
    inst, eta, gamma, s, ev, P = sparse_case
    gn = np.linalg.norm(ev.g)
    csr = orc.sparsify(inst.C, inst.a, eta, gamma, ev.M, ev.S, eta * gn / P.size, s=s)
    x, it = orc.cg(csr, inst.a, eta, gn, -ev.g, 1e-14, 200)
    assert abs(x.sum()) <= 1e-12 * np.abs(x).max()
    A = _hrho_dense(csr, inst.a, eta) + gn * np.eye(P.shape[1])
    np.testing.assert_allclose(A @ x, -ev.g, atol=1e-12)


# ---------------------------------------------------------------------------
# Armijo trial: exact algebra of the difference form
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("split", [True, False])
def test_trial_difference_form_matches_two_evals(split):
    """The trial's dL is L(w + tau) - L(w) for the step tau = t Delta / eta (two-level
    potentials; split=False: the grid step tau = grid(t Delta / eta)): compare with two
    separate evaluations, and with the directional derivative for a tiny step (where a
    difference of two rounded objectives would be pure noise)."""
    inst = W.gmm_points(30, 4, m=26)
    eta = 0.05
    gamma = W.random_dual(30, 6, 0.02)
    s = np.log(inst.b)
    r = np.log(inst.a)
    ev = orc.eval_pass(inst.C, inst.a, inst.b, eta, gamma, r=r, s=s, split=split)
    q = ev.q

    def step(t):
        return t * Delta / eta if split else q * np.rint(t * Delta / eta / q)

    Delta = W.random_dual(30, 8, 0.01)
    for t in (1.0, 0.8, 0.3, 1e-3):
        dL, Mn, Sn, cn, gn = orc.trial_pass(inst.C, inst.a, inst.b, eta, gamma, ev.M, Delta, t,
                                            s=s, q=q, split=split)
        tau = step(t)
        # the point with potentials w + tau: gamma + eta tau (exact in split form up to the
        # rounding of gamma + eta tau; exactly on the grid otherwise)
        gamma2 = gamma + eta * tau if split else eta * ((ev.w + tau) - s)
        ev2 = orc.eval_pass(inst.C, inst.a, inst.b, eta, gamma2, r=r, s=s, q=q, split=split)
        if not split:
            np.testing.assert_array_equal(ev2.w, ev.w + tau)
        Lw = -inst.b @ gamma + eta * inst.a @ (r + ev.lse)
        Lw2 = -inst.b @ gamma2 + eta * inst.a @ (r + ev2.lse)
        assert abs(dL - (Lw2 - Lw)) <= 1e-13 * (abs(Lw) + 1)
        np.testing.assert_allclose(cn, ev2.c, rtol=1e-12)
        np.testing.assert_allclose(Mn + np.log(Sn), ev2.lse, rtol=0, atol=1e-12)
    # tiny step (second-order term ~1e-19): dL recovers g^T (eta tau)
    t = 1e-8
    tau = step(t)
    dL, *_ = orc.trial_pass(inst.C, inst.a, inst.b, eta, gamma, ev.M, Delta, t, s=s, q=q,
                            split=split)
    slope = ev.g @ (eta * tau)
    assert abs(dL - slope) <= 1e-6 * abs(slope)


def test_p18_newton_step_decreases_objective(sparse_case):
    """Lemma (Armijo) (i): the shifted Newton direction is a descent direction, and the
    full step satisfies the Armijo inequality near the optimum (Thm 4.2)."""
    inst, eta, gamma, s, ev, P = sparse_case
    gn = np.linalg.norm(ev.g)
    csr = orc.sparsify(inst.C, inst.a, eta, gamma, ev.M, ev.S, eta * gn / P.size, s=s)
    x, _ = orc.cg(csr, inst.a, eta, gn, -ev.g, min(0.1, gn) * gn, 1000)
    gd = ev.g @ x
    assert gd < 0
    dL, *_ = orc.trial_pass(inst.C, inst.a, inst.b, eta, gamma, ev.M, x, 1.0, s=s)
    ok = dL <= 1e-4 * gd
    if not ok:  # backtracking must terminate (Lemma, part (ii))
        t = 1.0
        for _ in range(60):
            t *= 0.8
            dL, *_ = orc.trial_pass(inst.C, inst.a, inst.b, eta, gamma, ev.M, x, t, s=s)
            if dL <= 1e-4 * t * gd:
                ok = True
                break
    assert ok


# ---------------------------------------------------------------------------
# Algorithm 3 rounding, D_phi, certificate
# ---------------------------------------------------------------------------
def test_p3_p4_rounding_and_weak_duality():
    inst = W.gmm_points(18, 12, m=15)
    eta = 0.05
    for seed in range(4):
        gamma = W.random_dual(18, seed, 0.05)
        s = np.log(inst.b)
        ev = orc.eval_pass(inst.C, inst.a, inst.b, eta, gamma, s=s, want_plan=True)
        st = orc.stop_pass(inst.C, inst.a, inst.b, eta, gamma, ev.M, ev.S, s=s, want_xhat=True)
        Xh = st["xhat"]
        assert Xh.min() >= 0
        np.testing.assert_allclose(Xh.sum(1), inst.a, atol=1e-15 * 18, rtol=0)
        np.testing.assert_allclose(Xh.sum(0), inst.b, atol=1e-15 * 18, rtol=0)
        assert abs((inst.C * Xh).sum() - st["primal"]) <= 1e-15
        # weak duality (c-transform duals are feasible)
        assert st["primal"] - st["dual"] >= -1e-14
        zc = (inst.C - gamma[None]).min(1)
        assert abs(st["dual_gamma"] - (inst.a @ zc + inst.b @ gamma)) <= 1e-15
        # D_phi >= 0 and equals its definition on the dense matrices
        X = ev.plan
        mask = Xh > 0
        D = (Xh[mask] * np.log(Xh[mask] / X[mask])).sum() - Xh.sum() + X.sum()
        assert st["dphi"] >= 0
        assert abs(st["dphi"] - D) <= 1e-13


def test_p14_p22_constant_cost():
    """Constant C: g = 0 at gamma = 0, the plan is a b^T, D_phi(X, X) = 0 and the
    solve stops at once with the exact optimum."""
    m, n = 9, 11
    rng = np.random.default_rng(0)
    a = rng.uniform(0.1, 1, m); a /= a.sum()
    b = rng.uniform(0.1, 1, n); b /= b.sum()
    C = np.full((m, n), 0.5)
    ev = orc.eval_pass(C, a, b, 0.01, np.zeros(n), want_plan=True)
    # w = log b on the grid (spacing ~2^-44 here) perturbs P by ~1e-14 relative
    np.testing.assert_allclose(ev.g, 0, atol=1e-14)
    np.testing.assert_allclose(ev.plan, np.outer(a, b), rtol=1e-13)
    st = orc.stop_pass(C, a, b, 0.01, np.zeros(n), ev.M, ev.S)
    assert abs(st["dphi"]) <= 1e-15
    res = orc.solve(C, a, b, 0.01, want_plan=True)
    assert res["status"] == 0 and res["report"]["outer"] == 1
    np.testing.assert_allclose(res["plan"], np.outer(a, b), rtol=1e-13)
    assert abs(res["report"]["primal"] - 0.5) <= 1e-15


# ---------------------------------------------------------------------------
# outer loop: exact proximal steps are entropic OT with eps = eta / k
# ---------------------------------------------------------------------------
def log_sinkhorn(C, a, b, eps, iters=20000):
    """Independent log-domain Sinkhorn for min <C,X> + eps KL(X, a b^T)."""
    f = np.zeros(len(a))
    g = np.zeros(len(b))
    la, lb = np.log(a), np.log(b)

    def lse(Mx, axis):
        mx = Mx.max(axis, keepdims=True)
        return (mx + np.log(np.exp(Mx - mx).sum(axis, keepdims=True))).squeeze(axis)

    for _ in range(iters):
        f = -eps * lse((g[None] - C) / eps + lb[None], 1)
        g = -eps * lse((f[:, None] - C) / eps + la[:, None], 0)
    return np.exp((f[:, None] + g[None] - C) / eps + la[:, None] + lb[None])


def test_p15_outer_iterates_are_entropic_ot():
    inst = W.gmm_points(10, 31, m=8)
    eta = 0.2
    opt = orc.default_options(max_outer=3, gap_tol=0.0, marg_tol=0.0, mu0=1e-14,
                              mu_floor=1e-15, max_newton=200)
    res = orc.solve(inst.C, inst.a, inst.b, eta, options=opt)
    r, s, k = res["r"], res["s"], res["k"]
    assert k == 3
    Xk = dense_center(inst.C, r, s, k, eta)
    Xe = log_sinkhorn(inst.C, inst.a, inst.b, eta / k)
    np.testing.assert_allclose(Xk, Xe, rtol=0, atol=1e-10)


def test_p19_sparsified_and_exact_hessian_same_optimum():
    """Table 1: IBSN and IBN (rho = 0) reach the same objective."""
    inst = W.uniform_points(48, 5)
    o1 = orc.default_options(max_outer=20000, gap_tol=1e-9, marg_tol=0.0)
    o2 = orc.default_options(max_outer=20000, gap_tol=1e-9, marg_tol=0.0, rho_mode=1)
    r1 = orc.solve(inst.C, inst.a, inst.b, inst.eta, options=o1)["report"]
    r2 = orc.solve(inst.C, inst.a, inst.b, inst.eta, options=o2)["report"]
    assert abs(r1["primal"] - r2["primal"]) <= 2e-9 * r1["primal"]


def test_resume_matches_uninterrupted():
    """The outer state (k, r, s, gamma) is the whole solver state: stopping after j outer
    iterations and resuming gives the uninterrupted run bit for bit."""
    inst = W.uniform_points(20, 8)
    o_all = orc.default_options(max_outer=12, gap_tol=0.0, marg_tol=0.0)
    full = orc.solve(inst.C, inst.a, inst.b, inst.eta, options=o_all)
    o5 = orc.default_options(max_outer=5, gap_tol=0.0, marg_tol=0.0)
    part = orc.solve(inst.C, inst.a, inst.b, inst.eta, options=o5)
    o7 = orc.default_options(max_outer=7, gap_tol=0.0, marg_tol=0.0)
    rest = orc.solve(inst.C, inst.a, inst.b, inst.eta, options=o7, gamma0=part["gamma"],
                     state=(part["r"], part["s"], part["k"]))
    assert rest["k"] == full["k"] == 12
    np.testing.assert_array_equal(rest["gamma"], full["gamma"])
    np.testing.assert_array_equal(rest["s"], full["s"])


def test_p16_eibsn_single_subproblem_is_entropic_ot():
    # (E)IBSN (appendix C.4): prox centre 1 1^T and one subproblem solved to a small gradient;
    # its plan diag(a) P(gamma) is the entropic OT plan at epsilon = eta, here computed
    # independently by log-domain Sinkhorn
    inst = W.gmm_points(12, 41, m=9)
    eta = 0.15
    opt = orc.default_options(eot=1, eot_tol=1e-13, max_newton=200)
    res = orc.solve(inst.C, inst.a, inst.b, eta, options=opt)
    rep = res["report"]
    assert res["status"] == 0 and rep["outer"] == 1 and rep["grad_norm"] < 1e-13
    m, n = inst.C.shape
    ev = orc.eval_pass(inst.C, inst.a, inst.b, eta, res["gamma"], r=np.zeros(m), s=np.zeros(n),
                       k=0, want_plan=True)
    Xe = log_sinkhorn(inst.C, inst.a, inst.b, eta)
    np.testing.assert_allclose(ev.plan, Xe, rtol=0, atol=1e-12)
    # rows are exact by construction; columns to the gradient tolerance
    np.testing.assert_allclose(ev.plan.sum(1), inst.a, rtol=0, atol=1e-15)
    np.testing.assert_allclose(ev.plan.sum(0), inst.b, rtol=0, atol=1e-13)


def test_tiny_eta_log_domain_sinkhorn_reaches_optimum():
    """At eta = 1e-6 (sigma = 1e6 on a cost normalised to max 1) whole columns of the first
    subproblem's kernel fall below the FP64 range, so c_j = 0 and log c_j = -inf: the
    Sinkhorn step takes log c_j in the log domain instead, and the solve reaches the exact
    assignment optimum (Birkhoff: f* = min over permutations / n)."""
    from scipy.optimize import linear_sum_assignment
    inst = W.uniform_points(64, 0)
    rr, cc = linear_sum_assignment(inst.C)
    fstar = inst.C[rr, cc].sum() / 64
    opt = orc.default_options(max_outer=50, gap_tol=1e-10, marg_tol=0.0, sinkhorn_maxit=200)
    res = orc.solve(inst.C, inst.a, inst.b, 1e-6, options=opt)
    rep = res["report"]
    assert res["status"] == 0, rep
    assert rep["dual"] <= fstar * (1 + 1e-13) and abs(rep["primal"] - fstar) <= 1e-10 * fstar


def test_log_domain_column_sums_against_long_double():
    """The Sinkhorn step's log c_j (log_colsums in the oracle): where every entry of a column
    underflows, log c_j = LSE_i (log a_i + theta_ij - lse_i) evaluated in long double from the
    explicit kernel; the step is gamma + eta (log b - log c), centred."""
    inst = W.uniform_points(40, 3, m=35)
    eta = 1e-6
    gamma = np.zeros(40)
    s = np.log(inst.b)
    ev = orc.eval_pass(inst.C, inst.a, inst.b, eta, gamma, s=s)
    assert ev.c.min() == 0.0   # columns underflow in FP64
    out = orc.sinkhorn_step(inst.C, inst.a, inst.b, eta, gamma, ev.M, ev.S, ev.c, s, q=ev.q)
    LD = np.longdouble
    th = (ev.w.astype(LD) + ev.wl.astype(LD))[None, :] - LD(1 / eta) * inst.C.astype(LD)
    lse = th.max(1) + np.log(np.exp(th - th.max(1)[:, None]).sum(1))
    v = np.log(inst.a.astype(LD))[:, None] + th - lse[:, None]
    lc = v.max(0) + np.log(np.exp(v - v.max(0)[None, :]).sum(0))
    step = eta * (np.log(inst.b.astype(LD)) - lc)
    expect = gamma.astype(LD) + step
    expect -= expect.mean()
    np.testing.assert_allclose(out, np.asarray(expect, np.float64), rtol=0,
                               atol=1e-9 * float(np.abs(expect).max()))
    assert abs(out.sum()) <= 1e-12 * np.abs(out).max()
