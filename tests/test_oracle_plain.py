"""Pins of the oracle's plain passes (no potential grid), and of the grid scheme against them.

The plain passes (orc_plain_eval, orc_plain_sparsify, orc_plain_stop, orc_round) take the
subproblem's quantities straight from their definitions: eq. (7) for P, eqs. (5), (6) and (8)
for the row normalisers, the objective and the gradient, Algorithm 1, Algorithm 3 and the
relative KKT residual of appendix C.1.  They are checked here against references computed
independently in numpy: the prox centre X^k written out explicitly and evaluated in long
double (64-bit significand), Algorithm 3 and appendix C.1 transcribed into array code, and
exactly rounded sums (math.fsum).  The tolerances follow from the FP64 rounding of each side
(u = 2^-53), worked out in `entry_bound`.
"""
import math

import numpy as np
import pytest

import oracle as orc
from paper_2603_07156_amd import workloads as W

U = 2.0 ** -53
LD = np.longdouble


def state_after(inst, k):
    """(r, s, k, gamma) after k outer iterations of the oracle's solver."""
    if k == 0:
        return np.log(inst.a), np.log(inst.b), 0, W.random_dual(inst.n, 5, 0.02)
    opt = orc.default_options(max_outer=k, gap_tol=0.0, marg_tol=0.0)
    res = orc.solve(inst.C, inst.a, inst.b, inst.eta, options=opt)
    return res["r"], res["s"], res["k"], res["gamma"] + W.random_dual(inst.n, 3, 1e-5)


def explicit_center_ld(C, a, b, eta, r, s, k, gamma):
    """Eq. (7) with X^k = exp(r_i + s_j - k C_ij / eta) as an explicit matrix, all in long
    double: P, the full row normaliser log sum_j X^k_ij exp((gamma_j - C_ij)/eta), and L^k
    (eq. (6))."""
    Cl = C.astype(LD)
    eta_l = LD(eta)
    logXk = r.astype(LD)[:, None] + s.astype(LD)[None, :] - LD(k) * Cl / eta_l
    th = logXk + (gamma.astype(LD)[None, :] - Cl) / eta_l
    M = th.max(1)
    E = np.exp(th - M[:, None])
    S = E.sum(1)
    P = E / S[:, None]
    lse_full = M + np.log(S)
    L = -(b.astype(LD) * gamma.astype(LD)).sum() + eta_l * (a.astype(LD) * lse_full).sum()
    return P, lse_full, L


def entry_bound(C, s, gamma, eta, k, q=0.0):
    """Bound on |x_ij - exact| for x_ij = theta_ij - M_i formed in FP64 from (s, gamma):
    w = s + gamma/eta (two roundings), sigma = (k+1)/eta (one rounding, times C),
    theta = fma(-sigma, C, w) (one rounding at |theta|), and for the grid scheme the grid
    rounding of w (q/2).  The row maximum carries the same error again, and P = exp(x)/S
    doubles it once more through the normaliser, so P's relative error is below
    4 * entry_bound + 1e-14."""
    sigma = (k + 1) / eta
    w = s + gamma / eta
    big = sigma * np.abs(C).max() + np.abs(w).max()
    return q / 2 + U * (2 * big + 2 * np.abs(w).max() + np.abs(gamma).max() / eta + 64)


CASES = [(0.1, 0), (1e-2, 0), (1e-2, 99), (1e-2, 1999)]


@pytest.fixture(scope="module", params=CASES, ids=lambda c: f"eta{c[0]:g}-k{c[1]}")
def case(request):
    eta, k = request.param
    inst = W.uniform_points(30, 3, m=26)
    inst = W.Instance(inst.C, inst.a, inst.b, eta, "uniform points")
    r, s, kk, gamma = state_after(inst, k)
    return inst, r, s, kk, gamma


def test_plain_eval_matches_explicit_center_long_double(case):
    """At k = 0 (sigma = 10, 100) and at sigma = 10^4 and 2*10^5: the plain eval's plan,
    row normalisers, column sums, gradient and objective against eq. (5)-(8) evaluated from
    the explicit X^k in long double."""
    inst, r, s, k, gamma = case
    P, lse_full, L = explicit_center_ld(inst.C, inst.a, inst.b, inst.eta, r, s, k, gamma)
    pe = orc.plain_eval(inst.C, inst.a, inst.b, inst.eta, gamma, r=r, s=s, k=k, want_plan=True)
    tol = 4 * entry_bound(inst.C, s, gamma, inst.eta, k) + 1e-14
    Pd = np.asarray(P, dtype=np.float64)
    X = inst.a[:, None] * Pd
    np.testing.assert_allclose(pe.plan, X, rtol=tol, atol=1e-300)
    # the oracle's lse leaves out r_i (it cancels in P); the paper's normaliser includes it
    np.testing.assert_allclose(pe.lse + r, np.asarray(lse_full, dtype=np.float64), rtol=0,
                               atol=2 * entry_bound(inst.C, s, gamma, inst.eta, k)
                               + 4 * U * np.abs(np.asarray(lse_full, dtype=np.float64)).max())
    c = np.asarray((inst.a.astype(LD)[:, None] * P).sum(0), dtype=np.float64)
    np.testing.assert_allclose(pe.c, c, rtol=tol)
    np.testing.assert_allclose(pe.g, c - inst.b, rtol=0, atol=tol * c.max())       # eq. (8)
    scale = abs(inst.b @ gamma) + inst.eta * np.abs(inst.a * (r + pe.lse)).sum()
    assert abs(pe.L - float(L)) <= inst.eta * 4 * entry_bound(inst.C, s, gamma, inst.eta, k) \
        + 8 * U * scale


def test_grid_eval_within_its_bound_of_plain(case):
    """The grid scheme (orc_eval on w = grid(s + gamma/eta)) deviates from the plain
    definition only by the grid rounding of w and the FP64 roundings: P within
    4 (q/2 + ...) relative, the same bound the GPU passes are held to."""
    inst, r, s, k, gamma = case
    ge = orc.eval_pass(inst.C, inst.a, inst.b, inst.eta, gamma, r=r, s=s, k=k, want_plan=True)
    pe = orc.plain_eval(inst.C, inst.a, inst.b, inst.eta, gamma, r=r, s=s, k=k, want_plan=True)
    tol = 4 * (entry_bound(inst.C, s, gamma, inst.eta, k, q=ge.q)
               + entry_bound(inst.C, s, gamma, inst.eta, k)) + 1e-14
    np.testing.assert_allclose(ge.plan, pe.plan, rtol=tol, atol=1e-300)
    np.testing.assert_allclose(ge.c, pe.c, rtol=tol)
    if k == 0 and inst.eta >= 1e-2:
        assert tol < 1e-12   # at the first centre the grid is finer than the parity bar


def test_plain_gradient_is_derivative_of_plain_objective():
    """g = grad L^k (eq. (8)) by central differences of the plain objective."""
    inst = W.gmm_points(10, 5, m=8)
    eta = 0.05
    gamma = W.random_dual(10, 9, 0.02)
    r, s = np.log(inst.a), np.log(inst.b)
    pe = orc.plain_eval(inst.C, inst.a, inst.b, eta, gamma, r=r, s=s)
    h = 1e-6
    gfd = np.empty(10)
    for j in range(10):
        e = np.zeros(10)
        e[j] = h
        Lp = orc.plain_eval(inst.C, inst.a, inst.b, eta, gamma + e, r=r, s=s).L
        Lm = orc.plain_eval(inst.C, inst.a, inst.b, eta, gamma - e, r=r, s=s).L
        gfd[j] = (Lp - Lm) / (2 * h)
    np.testing.assert_allclose(pe.g, gfd, rtol=0, atol=1e-6 * np.abs(pe.g).max() + 1e-9)


# ---------------------------------------------------------------------------
# Algorithm 1 on the plain P
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("rho", [0.0, 1e-4, 1e-2])
def test_plain_sparsify_is_algorithm1_on_the_plan(rho):
    """Algorithm 1 transcribed in numpy on the plain plan: the kept pattern (P_ij >= rho,
    row i* whole), the row renormalisation and d = P_rho^T a, entry by entry."""
    inst = W.gmm_points(40, 11, m=33)
    gamma = W.random_dual(40, 2, 0.02)
    s = np.log(inst.b)
    pe = orc.plain_eval(inst.C, inst.a, inst.b, inst.eta, gamma, s=s, want_plan=True)
    P = pe.plan / inst.a[:, None]
    istar = int(np.argmax(inst.a))
    keep = P >= rho
    keep[istar] = True
    Pr = np.where(keep, P, 0.0)
    rows = np.arange(P.shape[0]) != istar
    Pr[rows] /= Pr[rows].sum(1, keepdims=True)
    csr = orc.plain_sparsify(inst.C, inst.a, inst.eta, gamma, rho, s)
    D = csr.dense()
    np.testing.assert_array_equal(D != 0, keep & (P > 0))
    np.testing.assert_allclose(D, Pr, rtol=1e-13, atol=0)
    np.testing.assert_allclose(csr.d, Pr.T @ inst.a, rtol=1e-13)
    assert csr.istar == istar


# ---------------------------------------------------------------------------
# Algorithm 3 (rounding) and appendix C.1
# ---------------------------------------------------------------------------
def alg3_numpy(X, a, b):
    """Algorithm 3 as printed: z from the rows of X, y from the columns of X (step 7),
    F = diag(z) X diag(y), e_r, e_c, Xhat = F + e_r e_c^T / ||e_r||_1."""
    z = np.minimum(a / X.sum(1), 1.0)
    y = np.minimum(b / X.sum(0), 1.0)
    F = z[:, None] * X * y[None, :]
    er = a - F.sum(1)
    ec = b - F.sum(0)
    l1 = np.abs(er).sum()
    Xh = F + np.outer(er, ec) / l1 if l1 > 0 else F
    return Xh, z, y, er, ec


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_round_is_algorithm3(seed):
    """orc_round on a nonnegative matrix whose row and column sums both exceed the
    marginals in places: every vector of Algorithm 3 and the output against the numpy
    transcription; the output is feasible.  The matrix is chosen so that y computed from
    the columns of F instead of X (the other reading of step 7) differs by far more than
    the tolerance."""
    rng = np.random.default_rng(seed)
    m, n = 17, 23
    X = rng.random((m, n)) * 2.0 / (m * n) * rng.uniform(0.3, 3.0, (m, 1))
    a = rng.uniform(0.1, 1, m)
    a /= a.sum()
    b = rng.uniform(0.1, 1, n)
    b /= b.sum()
    xh, z, y, er, ec = orc.round_plan(X, a, b)
    Xh, z0, y0, er0, ec0 = alg3_numpy(X, a, b)
    np.testing.assert_allclose(z, z0, rtol=1e-15)
    np.testing.assert_allclose(y, y0, rtol=1e-15)
    # e_r and e_c are differences a - F1, b - F^T 1: they carry the marginals' rounding
    np.testing.assert_allclose(er, np.maximum(er0, 0), rtol=0, atol=8 * U * a.max())
    np.testing.assert_allclose(ec, np.maximum(ec0, 0), rtol=0, atol=8 * U * b.max())
    np.testing.assert_allclose(xh, Xh, rtol=1e-12, atol=8 * U * a.max() * b.max())
    np.testing.assert_allclose(xh.sum(1), a, rtol=0, atol=1e-16)
    np.testing.assert_allclose(xh.sum(0), b, rtol=0, atol=1e-16)
    assert xh.min() >= 0
    F = z[:, None] * X
    y_alt = np.minimum(b / F.sum(0), 1.0)
    assert np.abs(y_alt - y).max() > 1e-3


def kkt_numpy(X, C, a, b, gamma):
    """Appendix C.1: Delta_kkt = max(Delta_p, Delta_d, Delta_c) for (X, gamma, zeta) with
    zeta the c-transform of gamma, U = C - zeta 1^T - 1 gamma^T."""
    zeta = (C - gamma[None, :]).min(1)
    Umat = (C - gamma[None, :]) - zeta[:, None]   # >= 0 exactly: zeta is the row minimum
    nC = np.linalg.norm(C)
    dp = max(np.linalg.norm(X.sum(1) - a) / (1 + np.linalg.norm(a)),
             np.linalg.norm(X.sum(0) - b) / (1 + np.linalg.norm(b)),
             np.linalg.norm(np.minimum(X, 0)) / (1 + np.linalg.norm(X)))
    dd = np.linalg.norm(np.minimum(Umat, 0)) / (1 + nC)
    dc = abs((X * Umat).sum()) / (1 + nC)
    return max(dp, dd, dc), dd, zeta


@pytest.mark.parametrize("k", [0, 40])
def test_plain_stop_against_numpy(k):
    """orc_plain_stop: Algorithm 3's vectors and Xhat on the plain plan, D_phi(Xhat, X)
    (eq. (3)), <C, Xhat>, <C, X>, the c-transform dual bounds and Delta_kkt (appendix
    C.1), each against numpy on the dense plan, the sums exactly rounded (math.fsum)."""
    inst = W.gmm_points(36, 21, m=29)
    r, s, kk, gamma = state_after(inst, k)
    pe = orc.plain_eval(inst.C, inst.a, inst.b, inst.eta, gamma, r=r, s=s, k=kk, want_plan=True)
    X = pe.plan
    st = orc.plain_stop(inst.C, inst.a, inst.b, inst.eta, gamma, s, k=kk, want_xhat=True,
                        want_steps=True)
    Xh, z, y, er, ec = alg3_numpy(X, inst.a, inst.b)
    np.testing.assert_allclose(st["z"], z, rtol=1e-15)
    np.testing.assert_allclose(st["y"], y, rtol=1e-15)
    # e_r, e_c are differences of nearly equal numbers: compare at the marginals' scale
    np.testing.assert_allclose(st["er"], np.maximum(er, 0), rtol=0, atol=8 * U * inst.a.max())
    np.testing.assert_allclose(st["ec"], np.maximum(ec, 0), rtol=0, atol=8 * U * inst.b.max())
    # step 11 on the oracle's own e_r, e_c (which carry the marginals' rounding): every
    # entry to a few units of its own size
    F = st["z"][:, None] * X * st["y"][None, :]
    Xh_own = F + np.outer(st["er"], st["ec"]) / st["er"].sum()
    np.testing.assert_allclose(st["xhat"], Xh_own, rtol=1e-14, atol=0)
    np.testing.assert_allclose(st["xhat"], Xh, rtol=1e-12, atol=16 * U * inst.a.max())
    xh = st["xhat"]
    # log X in the log domain (X underflows where Xhat's rank-one term is not 0):
    # log X_ij = log a_i + theta_ij - lse_i, theta from eq. (7) with the implicit centre
    sigma = (kk + 1) / inst.eta
    theta = (s + gamma / inst.eta)[None, :] - sigma * inst.C
    logX = np.log(inst.a)[:, None] + theta - pe.lse[:, None]
    terms = np.where(xh > 0, xh * (np.log(np.where(xh > 0, xh, 1)) - logX) - xh + X, X)
    dphi = math.fsum(terms.ravel())
    eb = entry_bound(inst.C, s, gamma, inst.eta, kk)
    assert abs(st["dphi"] - dphi) <= 1e-12 * abs(dphi) + 8 * eb * xh.sum() + 1e-17
    assert st["dphi"] >= -1e-18                                      # P22
    assert abs(st["primal"] - math.fsum((inst.C * xh).ravel())) <= 1e-15 * st["primal"]
    assert abs(st["cx"] - math.fsum((inst.C * X).ravel())) <= 1e-15 * st["cx"]
    kkt, dd, zeta = kkt_numpy(X, inst.C, inst.a, inst.b, gamma)
    assert dd == 0.0                                                  # P21: Delta_d = 0
    assert abs(st["kkt"] - kkt) <= 1e-12 * kkt
    dual_g = math.fsum(np.concatenate([inst.a * zeta, inst.b * gamma]))
    assert abs(st["dual_gamma"] - dual_g) <= 1e-14 * abs(dual_g) + 1e-17
    psi = ((s + gamma / inst.eta) - np.log(inst.b)) / sigma
    zp = (inst.C - psi[None, :]).min(1)
    dual_p = math.fsum(np.concatenate([inst.a * zp, inst.b * psi]))
    assert abs(st["dual_psi"] - dual_p) <= 1e-13 * abs(dual_p) + 1e-17
    assert st["dual"] == max(st["dual_gamma"], st["dual_psi"])
    assert st["primal"] - st["dual"] >= -1e-14                      # P4, weak duality


def test_stop_sums_exactly_rounded_at_many_entries():
    """The stop pass sums each row, then the rows.  On 600 x 700 entries the sums of
    <C, Xhat>, <C, X> and D_phi stay within a few units of the exactly rounded sums."""
    inst = W.uniform_points(700, 2, m=600)
    gamma = W.random_dual(700, 4, 0.01)
    s = np.log(inst.b)
    st = orc.plain_stop(inst.C, inst.a, inst.b, inst.eta, gamma, s, want_xhat=True)
    pe = orc.plain_eval(inst.C, inst.a, inst.b, inst.eta, gamma, s=s, want_plan=True)
    xh, X = st["xhat"], pe.plan
    for key, exact in (("primal", math.fsum((inst.C * xh).ravel())),
                       ("cx", math.fsum((inst.C * X).ravel()))):
        assert abs(st[key] - exact) <= 64 * U * exact, key


# ---------------------------------------------------------------------------
# Armijo trial of the grid scheme, both branches, against long double
# ---------------------------------------------------------------------------
def lse_ld(C, w, sigma):
    th = w.astype(LD)[None, :] - LD(sigma) * C.astype(LD)
    M = th.max(1)
    return M + np.log(np.exp(th - M[:, None]).sum(1))


@pytest.mark.parametrize("split", [True, False])
@pytest.mark.parametrize("t,scale", [(1.0, 0.01), (1.0, 30.0), (0.5, 80.0)])
def test_trial_branches_against_long_double(t, scale, split):
    """orc_trial's dL = L(w + tau) - L(w), in its small-step form (max tau <= 500,
    expm1/log1p) and its shifted form (max tau > 500), against two evaluations of the
    objective in long double.  Two-level potentials (split): w + wl carried in long double,
    tau = t Delta / eta; grid form: tau on the grid.  The row state it returns gives the
    trial point's normalisers."""
    inst = W.gmm_points(30, 4, m=26)
    eta = 0.05
    gamma = W.random_dual(30, 6, 0.02)
    s, r = np.log(inst.b), np.log(inst.a)
    ev = orc.eval_pass(inst.C, inst.a, inst.b, eta, gamma, r=r, s=s, split=split)
    q = ev.q
    Delta = W.random_dual(30, 8, 1.0) * scale
    dL, Mn, Sn, cn, gn = orc.trial_pass(inst.C, inst.a, inst.b, eta, gamma, ev.M, Delta, t,
                                        s=s, q=q, split=split)
    tau = t * Delta / eta if split else q * np.rint(t * Delta / eta / q)
    big = tau.max() > 500
    assert big == (scale > 10)
    sigma = 1.0 / eta
    w0 = ev.w.astype(LD) + (ev.wl.astype(LD) if split else LD(0))
    l0 = lse_ld(inst.C, w0, sigma)
    l1 = lse_ld(inst.C, w0 + tau.astype(LD), sigma)
    dL_ld = -LD(eta) * (inst.b.astype(LD) * tau.astype(LD)).sum() \
        + LD(eta) * (inst.a.astype(LD) * (l1 - l0)).sum()
    scale_L = eta * (np.abs(inst.b @ tau) + np.abs(inst.a @ np.asarray(l1 - l0, np.float64)))
    assert abs(dL - float(dL_ld)) <= 1e-13 * scale_L + 1e-18
    np.testing.assert_allclose(Mn + np.log(Sn), np.asarray(l1, np.float64), rtol=1e-14,
                               atol=1e-12)
