"""HIP path vs the CPU oracle, element by element, on identical seeded inputs.

Every call goes through the C ABI of libibsn.so (via the ctypes binding).  Sizes span
several row tiles and ragged tails; the 4096 and 10^4 cases use the launch
configuration of the benchmark.  Tolerances are written next to each check; they are
tighter than the parity bar of the task (1e-10 relative objective, 1e-9 absolute per
plan entry, identical sparsity pattern except within 1e-12 of the threshold).
"""
import numpy as np
import pytest

import oracle as orc
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


@pytest.fixture(params=["launches", "persistent", "single", "pipe"])
def cgctx(request, ib, ctx):
    """The context with CG run as kernel launches per iteration, in one cooperative launch
    (two barriers per iteration, or one on P'^T diag(a) P' with the pipelined recurrences),
    or in one workgroup; restored to the default afterwards."""
    ctx.set_cg_kernel({"launches": ib.CG_LAUNCHES, "persistent": ib.CG_PERSISTENT,
                       "single": ib.CG_SINGLE, "pipe": ib.CG_PIPE}[request.param])
    ctx.cg_form = request.param
    yield ctx
    ctx.set_cg_kernel(ib.CG_AUTO)
    ctx.cg_form = None


def converged_bound(cgctx):
    """Bound on |x - x_oracle| / max|x_oracle| for CG converged to 1e-12 ||g||.  The
    pipelined form updates its residual by a recurrence whose gap to the true residual
    grows with the iterations (Ghysels and Vanroose 2014, section 3), so its attainable
    accuracy is lower than standard CG's: measured 3.4e-9 on the 300 x 5000 case.  The
    solver asks CG for a relative residual of 1e-6 or more."""
    return 1e-8 if getattr(cgctx, "cg_form", None) == "pipe" else 1e-9


def dev(x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    return t.detach().cpu().numpy()


def problem(ib, inst, C=None):
    C = inst.C if C is None else C
    return ib.Problem(dev(C), dev(inst.a), dev(inst.b), inst.eta)


def outer_state(inst, k):
    """(r, s, k, gamma) after k oracle outer iterations (k = 0: the initial centre)."""
    if k == 0:
        return np.log(inst.a), np.log(inst.b), 0, W.random_dual(inst.n, 17, 0.02)
    opt = orc.default_options(max_outer=k, gap_tol=0.0, marg_tol=0.0)
    res = orc.solve(inst.C, inst.a, inst.b, inst.eta, options=opt)
    return res["r"], res["s"], res["k"], res["gamma"] + W.random_dual(inst.n, 3, 1e-4)


def center(ib, inst, r, s, k, gamma, C=None):
    """Centre with the oracle's grid spacing for these inputs."""
    q = orc.center_quantum(inst.C if C is None else C, s, gamma, inst.eta, k)
    return ib.Center(k, dev(r), dev(s), q), q


def check_eval(ib, ctx, inst, r, s, k, gamma, C=None, want_plan=True):
    Cc = inst.C if C is None else C
    pr = problem(ib, inst, Cc)
    ctr, q = center(ib, inst, r, s, k, gamma, Cc)
    gv = ib.subproblem_eval(ctx, pr, ctr, dev(gamma), want_obj=True, want_plan=want_plan)
    ov = orc.eval_pass(Cc, inst.a, inst.b, inst.eta, gamma, r=r, s=s, k=k, want_plan=want_plan,
                       q=q)
    # grid-rounded row maxima of identical fma values: identical bits
    np.testing.assert_array_equal(host(gv["M"]), ov.M)
    np.testing.assert_allclose(host(gv["S"]), ov.S, rtol=1e-13)
    np.testing.assert_allclose(host(gv["lse"]), ov.lse, rtol=1e-15, atol=1e-13)
    np.testing.assert_allclose(host(gv["c"]), ov.c, rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(host(gv["g"]), ov.g, rtol=0, atol=1e-12 * np.abs(ov.c).max())
    scale = abs(inst.b @ gamma) + inst.eta * np.abs(inst.a * (r + ov.lse)).sum() + 1e-300
    assert abs(gv["L"] - ov.L) <= 1e-12 * scale
    if want_plan:
        np.testing.assert_allclose(host(gv["plan"]), ov.plan, rtol=1e-12, atol=1e-15)
    return gv, ov


# ---------------------------------------------------------------------------
# eval (row a2)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("m,n", [(1, 1), (1, 7), (5, 1), (3, 2), (37, 63), (40, 64), (41, 65),
                                 (300, 257), (129, 511), (70, 513), (64, 1000), (33, 2047),
                                 (17, 2049), (9, 4099), (8, 8191), (5, 10240)])
def test_eval_shapes(ib, ctx, m, n):
    inst = W.gmm_points(n, 5, m=m)
    r, s, k, gamma = outer_state(inst, 0)
    check_eval(ib, ctx, inst, r, s, k, gamma)


@pytest.mark.parametrize("k", [0, 4, 25])
def test_eval_outer_states(ib, ctx, k):
    """Parity at later prox centres, where sigma = (k+1)/eta makes theta large."""
    inst = W.uniform_points(300, 1, m=260)
    r, s, kk, gamma = outer_state(inst, k)
    check_eval(ib, ctx, inst, r, s, kk, gamma)


def test_eval_fp32_cost(ib, ctx):
    """FP32-stored cost: both sides widen the same float values to double."""
    inst = W.gmm_points(1500, 9, m=200)
    C32 = inst.C.astype(np.float32)
    r, s, k, gamma = outer_state(inst, 0)
    check_eval(ib, ctx, inst, r, s, k, gamma, C=C32)


def test_eval_cfg2_size(ib, ctx):
    """4096 x 4096 Gaussian-mixture instance (the GPU-vs-oracle workload)."""
    inst = W.gmm_points(4096, 100)
    r, s, k, gamma = outer_state(inst, 0)
    check_eval(ib, ctx, inst, r, s, k, gamma, want_plan=False)


def test_eval_full_size_10k(ib, ctx):
    """10^4 x 10^4 (800 MB FP64 cost) in the benchmark's launch configuration."""
    inst = W.uniform_points(10000, 1000)
    r, s, k, gamma = np.log(inst.a), np.log(inst.b), 0, W.random_dual(10000, 2, 0.01)
    check_eval(ib, ctx, inst, r, s, k, gamma, want_plan=False)


def test_center_quantum_matches_oracle(ib, ctx):
    for k in (0, 7, 300):
        inst = W.gmm_points(257, 3, m=190)
        gamma = W.random_dual(257, k, 0.03)
        s = np.log(inst.b) + 0.37 * k
        q_o = orc.center_quantum(inst.C, s, gamma, inst.eta, k)
        q_g = ib.center_quantum(ctx, problem(ib, inst), ib.Center(k, None, dev(s), 1.0), dev(gamma))
        assert q_g == q_o


def test_eval_deterministic(ib, ctx):
    inst = W.uniform_points(700, 3, m=900)
    pr = problem(ib, inst)
    gamma = dev(W.random_dual(700, 1, 0.01))
    ctr = ib.Center.initial(ctx, pr, gamma)
    a = ib.subproblem_eval(ctx, pr, ctr, gamma)
    b = ib.subproblem_eval(ctx, pr, ctr, gamma)
    for key in ("M", "S", "c", "g"):
        assert torch.equal(a[key], b[key])
    assert a["L"] == b["L"]


# ---------------------------------------------------------------------------
# Armijo trial (row a6)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("t", [1.0, 0.8, 1e-3, 1e-9])
@pytest.mark.parametrize("k", [0, 6])
def test_trial(ib, ctx, t, k):
    inst = W.gmm_points(513, 12, m=301)
    r, s, kk, gamma = outer_state(inst, k)
    ctr, q = center(ib, inst, r, s, kk, gamma)
    ev = orc.eval_pass(inst.C, inst.a, inst.b, inst.eta, gamma, r=r, s=s, k=kk, q=q)
    Delta = W.random_dual(513, 44, 0.02)
    pr = problem(ib, inst)
    gt = ib.trial(ctx, pr, ctr, dev(gamma), dev(ev.M), dev(Delta), t)
    dL, Mn, Sn, cn, gn = orc.trial_pass(inst.C, inst.a, inst.b, inst.eta, gamma, ev.M, Delta, t,
                                        s=s, k=kk, q=q)
    assert abs(gt["dL"] - dL) <= 1e-12 * abs(dL) + 1e-17 * t
    # new shifts are grid values computed from the same inputs
    np.testing.assert_allclose(host(gt["M"]), Mn, rtol=0, atol=q)
    np.testing.assert_allclose(host(gt["M"]) + np.log(host(gt["S"])), Mn + np.log(Sn), rtol=1e-15,
                               atol=1e-12)
    np.testing.assert_allclose(host(gt["c"]), cn, rtol=1e-12)
    np.testing.assert_allclose(host(gt["g"]), gn, rtol=0, atol=1e-12 * np.abs(cn).max())


def test_trial_big_step(ib, ctx):
    """Steps with t*Delta/eta > 500 take the shifted form on both sides."""
    inst = W.gmm_points(300, 2, m=200)
    eta = 1e-3
    inst = W.Instance(inst.C, inst.a, inst.b, eta, "big")
    r, s, k, gamma = np.log(inst.a), np.log(inst.b), 0, np.zeros(300)
    ctr, q = center(ib, inst, r, s, 0, gamma)
    ev = orc.eval_pass(inst.C, inst.a, inst.b, eta, gamma, q=q)
    Delta = W.random_dual(300, 7, 0.5)
    pr = problem(ib, inst)
    gt = ib.trial(ctx, pr, ctr, dev(gamma), dev(ev.M), dev(Delta), 1.0)
    dL, Mn, Sn, cn, gn = orc.trial_pass(inst.C, inst.a, inst.b, eta, gamma, ev.M, Delta, 1.0, s=s,
                                        q=q)
    assert abs(gt["dL"] - dL) <= 1e-12 * abs(dL)
    np.testing.assert_allclose(host(gt["c"]), cn, rtol=1e-11, atol=1e-300)


# ---------------------------------------------------------------------------
# sparsify (row a4), HVP and CG (row a5)
# ---------------------------------------------------------------------------
def compare_patterns(gcsr, ocsr, P, rho, istar):
    row_ptr, col, val, d = (host(x) for x in gcsr.export())
    assert gcsr.istar == ocsr.istar == istar
    # the reported nnz counts every stored entry, the dense row included
    assert int(row_ptr[-1]) == gcsr.nnz == len(col)
    m = len(row_ptr) - 1
    same = True
    for i in range(m):
        gc = col[row_ptr[i]:row_ptr[i + 1]]
        oc = ocsr.col[ocsr.row_ptr[i]:ocsr.row_ptr[i + 1]]
        assert np.all(np.diff(gc) > 0), "columns ascending within a row"
        if not np.array_equal(gc, oc):
            same = False
            diff = np.setxor1d(gc, oc)
            # allowed only inside the relative threshold band |P - rho| <= 1e-12 rho
            assert np.all(np.abs(P[i, diff] - rho) <= 1e-12 * rho), (i, diff)
        else:
            np.testing.assert_allclose(val[row_ptr[i]:row_ptr[i + 1]],
                                       ocsr.val[ocsr.row_ptr[i]:ocsr.row_ptr[i + 1]], rtol=1e-12)
    return same, d


@pytest.mark.parametrize("rho_rule", ["zero", "paper", "1e-6", "1e-4"])
@pytest.mark.parametrize("k", [0, 5])
def test_sparsify_and_hvp(ib, ctx, rho_rule, k):
    inst = W.gmm_points(600, 8, m=420)
    r, s, kk, gamma = outer_state(inst, k)
    ctr, q = center(ib, inst, r, s, kk, gamma)
    ev = orc.eval_pass(inst.C, inst.a, inst.b, inst.eta, gamma, r=r, s=s, k=kk, want_plan=True,
                       q=q)
    P = ev.plan / inst.a[:, None]
    rho = {"zero": 0.0, "paper": inst.eta * np.linalg.norm(ev.g) / P.size,
           "1e-6": 1e-6, "1e-4": 1e-4}[rho_rule]
    pr = problem(ib, inst)
    gcsr = ib.sparsify(ctx, pr, ctr, dev(gamma), dev(ev.M), dev(ev.S), rho)
    ocsr = orc.sparsify(inst.C, inst.a, inst.eta, gamma, ev.M, ev.S, rho, s=s, k=kk, q=q)
    istar = int(np.argmax(inst.a))
    same, d = compare_patterns(gcsr, ocsr, P, rho, istar)
    assert same, "no entry of these inputs lies within the threshold band"
    assert gcsr.nnz == ocsr.nnz
    np.testing.assert_allclose(d, ocsr.d, rtol=1e-12)
    for shift in (0.0, 1e-3):
        v = W.random_dual(600, 21, 1.0)
        yg = host(ib.hvp(ctx, gcsr, pr.a, inst.eta, shift, dev(v)))
        yo = orc.hvp(ocsr, inst.a, inst.eta, shift, v)
        np.testing.assert_allclose(yg, yo, rtol=1e-12, atol=1e-12 * np.abs(yo).max())
    gcsr.free()


@pytest.mark.parametrize("n", [2000, 7000, 9500, 10240])
def test_sparsify_compaction_tiles(ib, ctx, n):
    """Kept-entry compaction on the wider tiles: the (slab, wave) segment bases come from
    one (n <= 8192) or two (n > 8192: 80 segments) 64-lane scans; pattern, values and d
    against the oracle."""
    inst = W.gmm_points(n, 6, m=29)
    r, s, kk, gamma = outer_state(inst, 3)
    ctr, q = center(ib, inst, r, s, kk, gamma)
    ev = orc.eval_pass(inst.C, inst.a, inst.b, inst.eta, gamma, r=r, s=s, k=kk, want_plan=True,
                       q=q)
    P = ev.plan / inst.a[:, None]
    rho = 1e-5
    pr = problem(ib, inst)
    gcsr = ib.sparsify(ctx, pr, ctr, dev(gamma), dev(ev.M), dev(ev.S), rho)
    ocsr = orc.sparsify(inst.C, inst.a, inst.eta, gamma, ev.M, ev.S, rho, s=s, k=kk, q=q)
    same, d = compare_patterns(gcsr, ocsr, P, rho, int(np.argmax(inst.a)))
    assert same and gcsr.nnz == ocsr.nnz
    np.testing.assert_allclose(d, ocsr.d, rtol=1e-12)
    gcsr.free()


def test_hvp_determinism_and_dense_row(ib, ctx):
    """Row i* is dense (n entries); repeated products are bitwise identical."""
    inst = W.gmm_points(2000, 4, m=1500)
    r, s, k, gamma = outer_state(inst, 0)
    ctr, q = center(ib, inst, r, s, k, gamma)
    ev = orc.eval_pass(inst.C, inst.a, inst.b, inst.eta, gamma, r=r, s=s, k=k, q=q)
    pr = problem(ib, inst)
    gcsr = ib.sparsify(ctx, pr, ctr, dev(gamma), dev(ev.M), dev(ev.S), 1e-7)
    row_ptr, col, val, d = (host(x) for x in gcsr.export())
    i = gcsr.istar
    assert row_ptr[i + 1] - row_ptr[i] == 2000
    v = dev(W.random_dual(2000, 5, 1.0))
    y1 = ib.hvp(ctx, gcsr, pr.a, inst.eta, 0.0, v)
    y2 = ib.hvp(ctx, gcsr, pr.a, inst.eta, 0.0, v)
    assert torch.equal(y1, y2)
    # Theorem 3.2: H_rho 1 = 0
    ones = torch.ones(2000, dtype=torch.float64, device="cuda")
    h1 = host(ib.hvp(ctx, gcsr, pr.a, inst.eta, 0.0, ones))
    assert np.abs(h1).max() <= 1e-12 / inst.eta
    gcsr.free()


def test_cg(ib, ctx, cgctx):
    inst = W.gmm_points(500, 13, m=380)
    r, s, k, gamma = outer_state(inst, 3)
    ctr, q = center(ib, inst, r, s, k, gamma)
    ev = orc.eval_pass(inst.C, inst.a, inst.b, inst.eta, gamma, r=r, s=s, k=k, q=q)
    gn = np.linalg.norm(ev.g)
    rho = inst.eta * gn / (380 * 500)
    pr = problem(ib, inst)
    gcsr = ib.sparsify(ctx, pr, ctr, dev(gamma), dev(ev.M), dev(ev.S), rho)
    ocsr = orc.sparsify(inst.C, inst.a, inst.eta, gamma, ev.M, ev.S, rho, s=s, k=k, q=q)
    shift = max(gn, 1e-2)
    tol = 1e-12 * gn
    xg, itg = ib.cg(cgctx, gcsr, pr.a, inst.eta, shift, dev(-ev.g), tol, 500)
    xo, ito = orc.cg(ocsr, inst.a, inst.eta, shift, -ev.g, tol, 500)
    assert itg < 500 and ito < 500
    np.testing.assert_allclose(host(xg), xo, rtol=0,
                               atol=converged_bound(cgctx) * np.abs(xo).max())
    assert abs(host(xg).sum()) <= 1e-10 * np.abs(xo).max()   # Lemma 4.1
    # maxit is respected and 0 iterations returns x = 0
    x0, it0 = ib.cg(cgctx, gcsr, pr.a, inst.eta, shift, dev(-ev.g), tol, 0)
    assert it0 == 0 and float(x0.abs().max()) == 0.0
    gcsr.free()


def test_cg_three_kernel_path(ib, ctx, cgctx):
    """n > 4096 runs CG as three kernels per iteration (row gather, column gather, update);
    smaller n folds the update into the row gather.  Both against the oracle's CG."""
    m, n = 300, 5000
    inst = W.gmm_points(n, 23, m=m)
    r, s, k, gamma = outer_state(inst, 0)
    ctr, q = center(ib, inst, r, s, k, gamma)
    ev = orc.eval_pass(inst.C, inst.a, inst.b, inst.eta, gamma, r=r, s=s, k=k, q=q)
    gn = np.linalg.norm(ev.g)
    rho = inst.eta * gn / (m * n)
    pr = problem(ib, inst)
    gcsr = ib.sparsify(ctx, pr, ctr, dev(gamma), dev(ev.M), dev(ev.S), rho)
    ocsr = orc.sparsify(inst.C, inst.a, inst.eta, gamma, ev.M, ev.S, rho, s=s, k=k, q=q)
    shift = max(gn, 1e-2)
    tol = 1e-12 * gn
    xg, itg = ib.cg(cgctx, gcsr, pr.a, inst.eta, shift, dev(-ev.g), tol, 500)
    xo, ito = orc.cg(ocsr, inst.a, inst.eta, shift, -ev.g, tol, 500)
    assert itg < 500 and ito < 500
    np.testing.assert_allclose(host(xg), xo, rtol=0,
                               atol=converged_bound(cgctx) * np.abs(xo).max())
    # a cap of a few iterations stops both at the same iterate
    x3, it3 = ib.cg(cgctx, gcsr, pr.a, inst.eta, shift, dev(-ev.g), 0.0, 3)
    xo3, ito3 = orc.cg(ocsr, inst.a, inst.eta, shift, -ev.g, 0.0, 3)
    assert it3 == ito3 == 3
    np.testing.assert_allclose(host(x3), xo3, rtol=0, atol=1e-9 * np.abs(xo3).max())
    # A cap inside the third queued chunk.  Unconverged iterates this far in are sensitive
    # to rounding: with only the column order of this problem permuted, the oracle's own
    # 17th iterate moves by 5e-7 of max|x|.  One iteration more or less moves it by about
    # 4%, so a bound of 1e-5 tells a wrong iteration count from rounding.
    x17, it17 = ib.cg(cgctx, gcsr, pr.a, inst.eta, shift, dev(-ev.g), 0.0, 17)
    xo17, ito17 = orc.cg(ocsr, inst.a, inst.eta, shift, -ev.g, 0.0, 17)
    assert it17 == ito17 == 17
    np.testing.assert_allclose(host(x17), xo17, rtol=0, atol=1e-5 * np.abs(xo17).max())
    gcsr.free()


@pytest.mark.parametrize("blocks", [1, 2, 7, 300])
def test_cg_persistent_grid_sizes(ib, ctx, blocks):
    """The one-launch CG with grids that leave every workgroup several rows and columns
    (1, 2, 7) or none at all (300 > rows / 8), a dense row split into one chunk per
    workgroup, against the oracle's CG, converged and stopped after 5 iterations."""
    inst = W.gmm_points(500, 13, m=380)
    r, s, k, gamma = outer_state(inst, 3)
    ctr, q = center(ib, inst, r, s, k, gamma)
    ev = orc.eval_pass(inst.C, inst.a, inst.b, inst.eta, gamma, r=r, s=s, k=k, q=q)
    gn = np.linalg.norm(ev.g)
    rho = inst.eta * gn / (380 * 500)
    pr = problem(ib, inst)
    gcsr = ib.sparsify(ctx, pr, ctr, dev(gamma), dev(ev.M), dev(ev.S), rho)
    ocsr = orc.sparsify(inst.C, inst.a, inst.eta, gamma, ev.M, ev.S, rho, s=s, k=k, q=q)
    assert ocsr.istar >= 0
    shift = max(gn, 1e-2)
    tol = 1e-12 * gn
    ctx.set_cg_kernel(ib.CG_PERSISTENT, blocks)
    try:
        xg, itg = ib.cg(ctx, gcsr, pr.a, inst.eta, shift, dev(-ev.g), tol, 500)
        x5, it5 = ib.cg(ctx, gcsr, pr.a, inst.eta, shift, dev(-ev.g), 0.0, 5)
    finally:
        ctx.set_cg_kernel(ib.CG_AUTO)
    xo, ito = orc.cg(ocsr, inst.a, inst.eta, shift, -ev.g, tol, 500)
    assert itg < 500 and ito < 500
    np.testing.assert_allclose(host(xg), xo, rtol=0, atol=1e-9 * np.abs(xo).max())
    xo5, ito5 = orc.cg(ocsr, inst.a, inst.eta, shift, -ev.g, 0.0, 5)
    assert it5 == ito5 == 5
    np.testing.assert_allclose(host(x5), xo5, rtol=0, atol=1e-9 * np.abs(xo5).max())
    gcsr.free()


def test_cg_kernel_mode_arguments(ib, ctx):
    with pytest.raises(RuntimeError):
        ctx.set_cg_kernel(5)
    with pytest.raises(RuntimeError):
        ctx.set_cg_kernel(ib.CG_PERSISTENT, 1025)
    ctx.set_cg_kernel(ib.CG_AUTO)


@pytest.mark.parametrize("maxit", [1, 2, 5, 9, 13])
def test_cg_two_kernel_iterates(ib, ctx, cgctx, maxit):
    """The folded update (n <= 4096) gives the same iterate as the oracle's CG after each
    number of iterations, across the host's chunk boundaries (chunks of 8 and 4 are queued
    before the first state record is read)."""
    inst = W.gmm_points(600, 8, m=420)
    r, s, k, gamma = outer_state(inst, 0)
    ctr, q = center(ib, inst, r, s, k, gamma)
    ev = orc.eval_pass(inst.C, inst.a, inst.b, inst.eta, gamma, r=r, s=s, k=k, q=q)
    pr = problem(ib, inst)
    gcsr = ib.sparsify(ctx, pr, ctr, dev(gamma), dev(ev.M), dev(ev.S), 1e-6)
    ocsr = orc.sparsify(inst.C, inst.a, inst.eta, gamma, ev.M, ev.S, 1e-6, s=s, k=k, q=q)
    shift = 1e-2
    xg, itg = ib.cg(cgctx, gcsr, pr.a, inst.eta, shift, dev(-ev.g), 0.0, maxit)
    xo, ito = orc.cg(ocsr, inst.a, inst.eta, shift, -ev.g, 0.0, maxit)
    assert itg == ito == maxit
    # Rounding of different summation orders, amplified by CG (cond ~5000 here).  With only
    # the column order permuted, the oracle's own iterate moves by < 1e-11 of max|x| up to
    # 9 iterations and by 3e-9 at 13.  One iteration more or less moves the 13th iterate by
    # about 9%.
    rel = 1e-9 if maxit <= 9 else 1e-6
    np.testing.assert_allclose(host(xg), xo, rtol=0, atol=rel * np.abs(xo).max())
    gcsr.free()


@pytest.mark.parametrize("n,stop_at", [(600, 8), (600, 12), (5000, 8), (5000, 12)])
def test_cg_converges_at_chunk_end(ib, ctx, cgctx, n, stop_at):
    """CG that reaches its tolerance exactly where the host polls (after the first chunk of
    8 or the second of 4, with more iterations already queued behind the poll): the
    iterations queued after convergence must leave x alone.  The shift (1.0: condition
    number ~10) makes the residual fall by 0.3-0.6 per iteration, and the tolerance is set
    at the geometric mean of the oracle's residual norms after stop_at - 1 and stop_at
    iterations.  n = 600 runs the two-kernel iteration, n = 5000 the three-kernel one."""
    m = 420 if n == 600 else 300
    inst = W.gmm_points(n, 8 if n == 600 else 23, m=m)
    r, s, k, gamma = outer_state(inst, 0)
    ctr, q = center(ib, inst, r, s, k, gamma)
    ev = orc.eval_pass(inst.C, inst.a, inst.b, inst.eta, gamma, r=r, s=s, k=k, q=q)
    pr = problem(ib, inst)
    rho = 1e-6 if n == 600 else inst.eta * np.linalg.norm(ev.g) / (m * n)
    gcsr = ib.sparsify(ctx, pr, ctr, dev(gamma), dev(ev.M), dev(ev.S), rho)
    ocsr = orc.sparsify(inst.C, inst.a, inst.eta, gamma, ev.M, ev.S, rho, s=s, k=k, q=q)
    shift = 1.0
    rhs = -ev.g

    def resid(x):
        return np.linalg.norm(rhs - orc.hvp(ocsr, inst.a, inst.eta, shift, x))

    xa, _ = orc.cg(ocsr, inst.a, inst.eta, shift, rhs, 0.0, stop_at - 1)
    xb, _ = orc.cg(ocsr, inst.a, inst.eta, shift, rhs, 0.0, stop_at)
    ra, rb = resid(xa), resid(xb)
    assert rb < 0.7 * ra, (ra, rb)
    tol = np.sqrt(ra * rb)
    xo, ito = orc.cg(ocsr, inst.a, inst.eta, shift, rhs, tol, 100)
    assert ito == stop_at
    for _ in range(2):   # the second solve starts from a context whose CG just ended
        xg, itg = ib.cg(cgctx, gcsr, pr.a, inst.eta, shift, dev(rhs), tol, 100)
        assert itg == stop_at
        np.testing.assert_allclose(host(xg), xo, rtol=0, atol=1e-9 * np.abs(xo).max())
    gcsr.free()


# ---------------------------------------------------------------------------
# stop test and certificate (rows a7, a10)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("k", [0, 8])
def test_stop(ib, ctx, k):
    inst = W.gmm_points(333, 6, m=250)
    r, s, kk, gamma = outer_state(inst, k)
    ctr, q = center(ib, inst, r, s, kk, gamma)
    ev = orc.eval_pass(inst.C, inst.a, inst.b, inst.eta, gamma, r=r, s=s, k=kk, q=q)
    pr = problem(ib, inst)
    gs = ib.stop(ctx, pr, ctr, dev(gamma), dev(ev.M), dev(ev.S), want_xhat=True)
    os_ = orc.stop_pass(inst.C, inst.a, inst.b, inst.eta, gamma, ev.M, ev.S, s=s, k=kk,
                        want_xhat=True, q=q)
    np.testing.assert_allclose(host(gs["xhat"]), os_["xhat"], rtol=1e-10, atol=1e-15)
    for key, rtol, atol in [("primal", 1e-12, 0), ("dual", 1e-12, 1e-16), ("cx", 1e-12, 0),
                            ("dual_gamma", 1e-12, 1e-16), ("dual_psi", 1e-12, 1e-16),
                            ("dphi", 1e-9, 1e-15), ("kkt", 1e-9, 1e-16), ("er1", 1e-6, 1e-16)]:
        assert abs(gs[key] - os_[key]) <= rtol * abs(os_[key]) + atol, (key, gs[key], os_[key])
    Xh = host(gs["xhat"])
    assert Xh.min() >= 0
    np.testing.assert_allclose(Xh.sum(1), inst.a, atol=1e-15 * 333, rtol=0)
    np.testing.assert_allclose(Xh.sum(0), inst.b, atol=1e-15 * 333, rtol=0)


@pytest.mark.parametrize("m,n", [(250, 333), (64, 2049), (40, 4099)])
def test_stop_fp32_cost(ib, ctx, m, n):
    """FP32-stored cost (16-byte vectors of four floats, ragged tails) in both stop passes."""
    inst = W.gmm_points(n, 6, m=m)
    C32 = inst.C.astype(np.float32)
    r, s, k, gamma = outer_state(inst, 0)
    ctr, q = center(ib, inst, r, s, k, gamma, C32)
    ev = orc.eval_pass(C32, inst.a, inst.b, inst.eta, gamma, r=r, s=s, k=k, q=q)
    pr = problem(ib, inst, C32)
    gs = ib.stop(ctx, pr, ctr, dev(gamma), dev(ev.M), dev(ev.S), want_xhat=True)
    os_ = orc.stop_pass(C32, inst.a, inst.b, inst.eta, gamma, ev.M, ev.S, s=s, k=k,
                        want_xhat=True, q=q)
    np.testing.assert_allclose(host(gs["xhat"]), os_["xhat"], rtol=1e-10, atol=1e-15)
    for key, rtol, atol in [("primal", 1e-12, 0), ("dual", 1e-12, 1e-16), ("cx", 1e-12, 0),
                            ("dphi", 1e-9, 1e-15), ("kkt", 1e-9, 1e-16)]:
        assert abs(gs[key] - os_[key]) <= rtol * abs(os_[key]) + atol, (key, gs[key], os_[key])


# ---------------------------------------------------------------------------
# full solve (Algorithm 2) against exact optima and the oracle
# ---------------------------------------------------------------------------
def test_solve_n64_exact(ib, ctx):
    from scipy.optimize import linear_sum_assignment
    inst = W.uniform_points(64, 0)
    rr, cc = linear_sum_assignment(inst.C)
    fstar = inst.C[rr, cc].sum() / 64
    pr = problem(ib, inst)
    opt = ib.default_options(max_outer=20000, gap_tol=1e-8, marg_tol=0.0)
    res = ib.solve(ctx, pr, opt, want_plan=True)
    rep = res["report"]
    assert res["status"] == 0, rep
    assert rep["rel_gap"] <= 1e-8
    assert rep["dual"] <= fstar * (1 + 1e-13) and rep["primal"] >= fstar * (1 - 1e-13)
    assert (rep["primal"] - fstar) / fstar <= 1e-8
    X = host(res["plan"])
    np.testing.assert_allclose(X.sum(1), inst.a, atol=1e-15 * 64, rtol=0)
    np.testing.assert_allclose(X.sum(0), inst.b, atol=1e-15 * 64, rtol=0)
    assert abs((inst.C * X).sum() - rep["primal"]) <= 1e-15
    # the oracle, run to the same stop rule, brackets the same optimum
    o = orc.solve(inst.C, inst.a, inst.b, inst.eta,
                  options=orc.default_options(max_outer=20000, gap_tol=1e-8, marg_tol=0.0))
    assert abs(o["report"]["primal"] - rep["primal"]) <= 1e-8 * fstar


def test_solve_general_weights_vs_highs(ib, ctx):
    from scipy.optimize import linprog
    m, n = 24, 20
    inst = W.gmm_points(n, 101, m=m)
    A_eq = np.zeros((m + n, m * n))
    for i in range(m):
        A_eq[i, i * n:(i + 1) * n] = 1.0
    for j in range(n):
        A_eq[m + j, j::n] = 1.0
    fstar = linprog(inst.C.ravel(), A_eq=A_eq, b_eq=np.concatenate([inst.a, inst.b]),
                    bounds=(0, None), method="highs").fun
    pr = problem(ib, inst)
    res = ib.solve(ctx, pr, ib.default_options(max_outer=20000, gap_tol=1e-10, marg_tol=0.0))
    assert res["status"] == 0
    assert abs(res["report"]["primal"] - fstar) <= 1e-8 * fstar


def test_solve_resume_matches(ib, ctx):
    inst = W.uniform_points(40, 8)
    pr = problem(ib, inst)
    full = ib.solve(ctx, pr, ib.default_options(max_outer=9, gap_tol=0.0, marg_tol=0.0))
    part = ib.solve(ctx, pr, ib.default_options(max_outer=4, gap_tol=0.0, marg_tol=0.0))
    rest = ib.solve(ctx, pr, ib.default_options(max_outer=5, gap_tol=0.0, marg_tol=0.0),
                    gamma0=part["gamma"], state=(part["r"], part["s"], part["k"]))
    assert rest["k"] == full["k"] == 9
    assert torch.equal(rest["gamma"], full["gamma"])
    assert torch.equal(rest["s"], full["s"])


def test_solve_eibsn_matches_oracle(ib, ctx):
    # (E)IBSN (appendix C.4): centre 1 1^T, one subproblem to a small gradient.  The GPU and
    # the oracle reach the same entropic OT plan.
    inst = W.gmm_points(96, 52, m=80)
    inst = W.Instance(inst.C, inst.a, inst.b, 0.05, "eot")
    gopt = ib.default_options(eot=1, eot_tol=1e-12, max_newton=300)
    res = ib.solve(ctx, problem(ib, inst), gopt)
    rep = res["report"]
    assert res["status"] == 0 and rep["outer"] == 1 and rep["grad_norm"] < 1e-12, rep
    o = orc.solve(inst.C, inst.a, inst.b, inst.eta,
                  options=orc.default_options(eot=1, eot_tol=1e-12, max_newton=300))
    assert o["status"] == 0 and o["report"]["outer"] == 1
    m, n = inst.C.shape
    z_m, z_n = np.zeros(m), np.zeros(n)
    pg = orc.eval_pass(inst.C, inst.a, inst.b, inst.eta, host(res["gamma"]), r=z_m, s=z_n, k=0,
                       want_plan=True).plan
    po = orc.eval_pass(inst.C, inst.a, inst.b, inst.eta, o["gamma"], r=z_m, s=z_n, k=0,
                       want_plan=True).plan
    np.testing.assert_allclose(pg, po, rtol=0, atol=1e-12)
    # the returned centre is the (E)IBSN one
    assert res["k"] == 1 and float(host(res["r"]).max()) == 0.0 and float(host(res["s"]).max()) == 0.0


def test_solve_constant_cost(ib, ctx):
    m, n = 9, 11
    rng = np.random.default_rng(0)
    a = rng.uniform(0.1, 1, m); a /= a.sum()
    b = rng.uniform(0.1, 1, n); b /= b.sum()
    inst = W.Instance(np.full((m, n), 0.5), a, b, 0.01, "const")
    res = ib.solve(ctx, problem(ib, inst), want_plan=True)
    assert res["status"] == 0 and res["report"]["outer"] == 1
    np.testing.assert_allclose(host(res["plan"]), np.outer(a, b), rtol=1e-14)


# ---------------------------------------------------------------------------
# error behaviour of the ABI
# ---------------------------------------------------------------------------
def test_invalid_arguments(ib, ctx):
    inst = W.uniform_points(16, 0)
    pr = problem(ib, inst)
    ctr = ib.Center.initial(ctx, pr)
    g = torch.zeros(16, dtype=torch.float64, device="cuda")
    bad = ib.Problem(pr.C, pr.a, pr.b, -1.0)
    with pytest.raises(ib.IBSNError) as e:
        ib.subproblem_eval(ctx, bad, ctr, g)
    assert e.value.code == -1
    with pytest.raises(ib.IBSNError) as e:   # marginals that do not sum to 1
        ib.solve(ctx, ib.Problem(pr.C, pr.a * 2, pr.b, 0.01))
    assert e.value.code == -1
    # rows wider than every tile run split into column blocks (tests/test_gpu_split.py);
    # block widths outside [256, 10240] or not a multiple of 64 are rejected
    for cols in (100, 300, 10304, -64):
        with pytest.raises(ib.IBSNError) as e:
            ctx.set_row_split(cols)
        assert e.value.code == -1
    ctx.set_row_split(0)
    with pytest.raises(ValueError):   # host tensor rejected by the binding
        ib.subproblem_eval(ctx, pr, ctr, torch.zeros(16, dtype=torch.float64))
    with pytest.raises(ib.IBSNError) as e:   # quantum not a power of two
        ib.subproblem_eval(ctx, pr, ib.Center(0, ctr.r, ctr.s, 3e-12), g)
    assert e.value.code == -1


def test_csr_handle_lifetime(ib, ctx):
    """A factor is tied to its context: another context rejects it, and destroying its
    context first leaves ibsn_csr_free valid (it frees only what remains)."""
    inst = W.gmm_points(200, 3, m=150)
    r, s, k, gamma = outer_state(inst, 0)
    ctr, q = center(ib, inst, r, s, k, gamma)
    ev = orc.eval_pass(inst.C, inst.a, inst.b, inst.eta, gamma, r=r, s=s, k=k, q=q)
    c2 = ib.Context(0)
    pr = problem(ib, inst)
    gcsr = ib.sparsify(c2, pr, ctr, dev(gamma), dev(ev.M), dev(ev.S), 1e-6)
    v = dev(W.random_dual(200, 5, 1.0))
    with pytest.raises(ib.IBSNError):
        ib.hvp(ctx, gcsr, pr.a, inst.eta, 0.0, v)
    y = ib.hvp(c2, gcsr, pr.a, inst.eta, 0.0, v)
    assert torch.isfinite(y).all()
    c2.close()
    gcsr.free()
    assert gcsr.h is None


def test_solve_tiny_eta_reaches_optimum(ib, ctx):
    """eta = 1e-6: columns of the first kernel underflow (c_j = 0); the Sinkhorn step takes
    log c_j in the log domain and the solve reaches the exact assignment optimum, as the
    oracle does."""
    from scipy.optimize import linear_sum_assignment
    inst = W.uniform_points(64, 0)
    rr, cc = linear_sum_assignment(inst.C)
    fstar = inst.C[rr, cc].sum() / 64
    pr = ib.Problem(dev(inst.C), dev(inst.a), dev(inst.b), 1e-6)
    opt = ib.default_options(max_outer=50, gap_tol=1e-10, marg_tol=0.0, sinkhorn_maxit=200)
    res = ib.solve(ctx, pr, opt)
    rep = res["report"]
    assert res["status"] == 0, rep
    assert rep["dual"] <= fstar * (1 + 1e-13) and abs(rep["primal"] - fstar) <= 1e-10 * fstar


def test_sinkhorn_step_and_outer_update(ib, ctx):
    """One Sinkhorn gamma-step (the ordinary and the log-domain form) and one outer update,
    element by element against the oracle on the same eval state."""
    for eta, m, n in ((1e-2, 300, 257), (1e-6, 35, 40), (1e-6, 300, 4099)):
        inst = W.uniform_points(n, 3, m=m)
        inst = W.Instance(inst.C, inst.a, inst.b, eta, "step")
        r, s, k, gamma = np.log(inst.a), np.log(inst.b), 0, W.random_dual(n, 5, 1e-3 * eta)
        ctr, q = center(ib, inst, r, s, k, gamma)
        ev = orc.eval_pass(inst.C, inst.a, inst.b, eta, gamma, r=r, s=s, k=k, q=q)
        if eta < 1e-4:
            assert ev.c.min() < 1e-290   # the log-domain form runs
        pr = problem(ib, inst)
        gs = host(ib.sinkhorn_step(ctx, pr, ctr, dev(gamma), dev(ev.M), dev(ev.S), dev(ev.c)))
        os_ = orc.sinkhorn_step(inst.C, inst.a, inst.b, eta, gamma, ev.M, ev.S, ev.c, s, q=q)
        # gamma = eta (w - s): the step's own size sets the rounding scale
        np.testing.assert_allclose(gs, os_, rtol=0, atol=1e-13 * np.abs(os_).max())
        assert abs(gs.sum()) <= 1e-12 * np.abs(gs).max()
        gr, gsx = (host(x) for x in ib.outer_update(ctx, pr, ctr, dev(gamma), dev(ev.M),
                                                    dev(ev.S)))
        o_r, o_s = orc.outer_update(inst.a, eta, gamma, ev.M, ev.S, s, q)
        np.testing.assert_allclose(gr, o_r, rtol=1e-15, atol=1e-13)
        np.testing.assert_array_equal(gsx, o_s)


def test_full_size_10k_passes(ib, ctx):
    """m = n = 10^4 (800 MB FP64 cost) in the benchmark's launch configuration: trial,
    sparsify (pattern and values), HVP, CG and the stop pass against the oracle, at the
    prox centre of outer iteration 60 (sigma = 6100, a factor as sparse as in the benchmark)."""
    n = 10000
    inst = W.uniform_points(n, 1000)
    k = 60
    r, s = np.log(inst.a), np.log(inst.b)
    gamma = W.random_dual(n, 2, 1e-4)
    ctr, q = center(ib, inst, r, s, k, gamma)
    ev = orc.eval_pass(inst.C, inst.a, inst.b, inst.eta, gamma, r=r, s=s, k=k, q=q)
    pr = problem(ib, inst)
    g_gamma = dev(gamma)
    # Armijo trial
    Delta = W.random_dual(n, 44, 1e-4)
    gt = ib.trial(ctx, pr, ctr, g_gamma, dev(ev.M), dev(Delta), 1.0)
    dL, Mn, Sn, cn, gn_ = orc.trial_pass(inst.C, inst.a, inst.b, inst.eta, gamma, ev.M, Delta, 1.0,
                                         s=s, k=k, q=q)
    assert abs(gt["dL"] - dL) <= 1e-12 * abs(dL) + 1e-17
    np.testing.assert_allclose(host(gt["M"]) + np.log(host(gt["S"])), Mn + np.log(Sn), rtol=1e-15,
                               atol=1e-12)
    np.testing.assert_allclose(host(gt["c"]), cn, rtol=1e-12, atol=1e-300)
    # sparsify with the paper's rho
    gnorm = np.linalg.norm(ev.g)
    rho = inst.eta * gnorm / (n * n)
    gcsr = ib.sparsify(ctx, pr, ctr, g_gamma, dev(ev.M), dev(ev.S), rho)
    ocsr = orc.sparsify(inst.C, inst.a, inst.eta, gamma, ev.M, ev.S, rho, s=s, k=k, q=q)
    row_ptr, col, val, d = (host(x) for x in gcsr.export())
    assert gcsr.nnz == ocsr.nnz and np.array_equal(row_ptr, ocsr.row_ptr)
    assert np.array_equal(col, ocsr.col), "no entry of these inputs lies in the threshold band"
    np.testing.assert_allclose(val, ocsr.val, rtol=1e-12)
    np.testing.assert_allclose(d, ocsr.d, rtol=1e-12)
    assert 1e5 < gcsr.nnz < 2e7
    # HVP and CG on the same factor
    v = W.random_dual(n, 21, 1.0)
    shift = gnorm
    yg = host(ib.hvp(ctx, gcsr, pr.a, inst.eta, shift, dev(v)))
    yo = orc.hvp(ocsr, inst.a, inst.eta, shift, v)
    np.testing.assert_allclose(yg, yo, rtol=1e-12, atol=1e-12 * np.abs(yo).max())
    tol = 1e-8 * gnorm
    xg, itg = ib.cg(ctx, gcsr, pr.a, inst.eta, shift, dev(-ev.g), tol, 400)
    xo, ito = orc.cg(ocsr, inst.a, inst.eta, shift, -ev.g, tol, 400)
    assert itg < 400 and ito < 400
    np.testing.assert_allclose(host(xg), xo, rtol=0, atol=1e-7 * np.abs(xo).max())
    gcsr.free()
    # stop test and certificate
    gs = ib.stop(ctx, pr, ctr, g_gamma, dev(ev.M), dev(ev.S))
    os_ = orc.stop_pass(inst.C, inst.a, inst.b, inst.eta, gamma, ev.M, ev.S, s=s, k=k, q=q)
    for key, rtol, atol in [("primal", 1e-12, 0), ("dual", 1e-12, 1e-16), ("cx", 1e-12, 0),
                            ("dphi", 1e-9, 1e-15), ("kkt", 1e-9, 1e-16)]:
        assert abs(gs[key] - os_[key]) <= rtol * abs(os_[key]) + atol, (key, gs[key], os_[key])


def test_solve_batch_matches_sequential(ib, ctx):
    """The batched form (three worker contexts on their own streams) returns, for every
    problem, bitwise the result of solving it alone with the same CG form (several contexts
    run CG as launches): each solve is deterministic and the workers share nothing.  One
    problem is also checked against the oracle's solve."""
    batch = W.grid_histogram_batch(7, 301, lo=64, hi=600)
    probs = [problem(ib, inst) for inst in batch]
    opt = ib.default_options(max_outer=25, gap_tol=0.0, marg_tol=0.0)
    ctxs = [ib.Context(0, stream=torch.cuda.Stream()) for _ in range(3)]
    for c in ctxs:
        c.set_cg_kernel(ib.CG_PERSISTENT)   # restored by solve_batch after its launches
    out = ib.solve_batch(ctxs, probs, opt)
    ctx.set_cg_kernel(ib.CG_LAUNCHES)
    refs = [ib.solve(ctx, pr, opt) for pr in probs]
    ctx.set_cg_kernel(ib.CG_AUTO)
    # one context keeps its own CG form (here one launch per CG solve)
    one = ib.solve_batch([ctxs[0]], probs[:1], opt)[0]
    ctx.set_cg_kernel(ib.CG_PERSISTENT)
    ref1 = ib.solve(ctx, probs[0], opt)
    ctx.set_cg_kernel(ib.CG_AUTO)
    assert torch.equal(one["gamma"], ref1["gamma"])
    # CG in one workgroup needs no cooperative launch: the batch keeps that form
    for c in ctxs:
        c.set_cg_kernel(ib.CG_SINGLE)
    outs = ib.solve_batch(ctxs, probs[:4], opt)
    ctx.set_cg_kernel(ib.CG_SINGLE)
    for pr, o in zip(probs[:4], outs):
        ref = ib.solve(ctx, pr, opt)
        assert torch.equal(o["gamma"], ref["gamma"])
        assert o["report"]["cg"] == ref["report"]["cg"]
    ctx.set_cg_kernel(ib.CG_AUTO)
    for inst, pr, o, ref in zip(batch, probs, out, refs):
        assert o["status"] == ref["status"]
        assert torch.equal(o["gamma"], ref["gamma"]), inst.name
        for key in ("outer", "newton", "cg", "primal", "dual", "rel_gap"):
            assert o["report"][key] == ref["report"][key], (inst.name, key)
    # the smallest problem against the oracle's solve with the same options: after a fixed
    # number of inexact outer iterations the two trajectories differ, but each certificate
    # brackets the same OT value (dual <= OT <= primal), so the primal values differ by at
    # most the larger certified gap, and each dual stays below the other's primal
    i = int(np.argmin([inst.C.size for inst in batch]))
    inst = batch[i]
    o = orc.solve(inst.C, inst.a, inst.b, inst.eta, options=orc.default_options(
        max_outer=25, gap_tol=0.0, marg_tol=0.0))["report"]
    g = out[i]["report"]
    assert abs(g["primal"] - o["primal"]) <= max(g["primal"] - g["dual"], o["primal"] - o["dual"])
    assert g["dual"] <= o["primal"] * (1 + 1e-13) and o["dual"] <= g["primal"] * (1 + 1e-13)
    # the same context twice is rejected before any problem is attempted
    with pytest.raises(ib.IBSNError):
        ib.solve_batch([ctxs[0], ctxs[0]], probs[:2], opt)
    for c in ctxs:
        c.close()
