"""Rows split into column blocks (ibsn_set_row_split) against the CPU oracle.

Every dense pass holds a whole row of C in registers up to 10240 columns (FP64 cost, points)
or 20000 (FP32 cost); wider rows run as column blocks whose per-row results are joined
(row maxima and sums, kept entries, the stop test's sums and minima).  The oracle knows
nothing of blocks, so these tests hold the split passes to the whole-row tolerances:
- small problems with a forced block width (256 .. 1024 columns: several blocks and a
  ragged last block) for every pass, cost type and precision;
- the solve to a certified gap with split rows, against the oracle's solve;
- rows wider than the tiles: 12000 columns (FP64 cost and 2-D points) and the 20000 x 20000
  3-D points configuration (the precision form's third workload, cost formed on the fly).
"""
import numpy as np
import pytest

import oracle as orc
from paper_2603_07156_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U = 2.0 ** -22   # relative error bound of the FP32 exponential (mixed precision)


@pytest.fixture(scope="module")
def ib():
    from paper_2603_07156_amd import ibsn
    return ibsn


@pytest.fixture(scope="module")
def ctx(ib):
    return ib.Context(0)


@pytest.fixture
def split(ctx):
    """Set the block width for one test; whole rows again afterwards."""
    def set_(cols):
        ctx.set_row_split(cols)
    yield set_
    ctx.set_row_split(0)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def points_instance(m, n, d, seed, eta=1e-2):
    rng = np.random.default_rng(seed)
    x, y = rng.random((m, d)), rng.random((n, d))
    scale = W.points_scale(x, y)
    a = W._normalise(rng.uniform(0.1, 1.0, m))
    b = W._normalise(rng.uniform(0.1, 1.0, n))
    return W.Instance(W.points_cost(x, y, scale), a, b, eta, f"pts{d}d_{m}x{n}", x, y), scale


def make(ib, kind, m, n, seed, precision=0):
    """(instance, problem, cost the oracle sees) for kind 'f64', 'f32', 'pts2' or 'pts3'."""
    if kind.startswith("pts"):
        inst, scale = points_instance(m, n, int(kind[3]), seed)
        pr = ib.Problem.from_points(dev(inst.x), dev(inst.y), dev(inst.a), dev(inst.b), inst.eta,
                                    scale, precision)
        return inst, pr, inst.C
    inst = W.gmm_points(n, seed, m=m)
    C = inst.C.astype(np.float32) if kind == "f32" else inst.C
    return inst, ib.Problem(dev(C), dev(inst.a), dev(inst.b), inst.eta, precision=precision), C


def state(inst, C, k):
    """(r, s, k, gamma, q) after k oracle outer iterations (k = 0: the initial centre)."""
    if k == 0:
        r, s, kk, gamma = np.log(inst.a), np.log(inst.b), 0, W.random_dual(inst.n, 17, 0.02)
    else:
        res = orc.solve(C, inst.a, inst.b, inst.eta,
                        options=orc.default_options(max_outer=k, gap_tol=0.0, marg_tol=0.0))
        r, s, kk = res["r"], res["s"], res["k"]
        gamma = res["gamma"] + W.random_dual(inst.n, 3, 1e-4)
    return r, s, kk, gamma, orc.center_quantum(C, s, gamma, inst.eta, kk)


def check_eval(ib, ctx, inst, pr, C, r, s, k, gamma, q, mixed=False, want_plan=True):
    ctr = ib.Center(k, dev(r), dev(s), q)
    print(f"eval {inst.name} k={k} mixed={mixed}", flush=True)
    gv = ib.subproblem_eval(ctx, pr, ctr, dev(gamma), want_obj=True, want_plan=want_plan)
    ov = orc.eval_pass(C, inst.a, inst.b, inst.eta, gamma, r=r, s=s, k=k, want_plan=want_plan,
                       q=q)
    # the row maximum of the whole row is the largest block maximum: identical bits
    np.testing.assert_array_equal(host(gv["M"]), ov.M)
    if mixed:
        np.testing.assert_allclose(host(gv["S"]), ov.S, rtol=2 * U)
        np.testing.assert_allclose(host(gv["c"]), ov.c, rtol=4 * U, atol=1e-300)
        np.testing.assert_allclose(host(gv["g"]), ov.g, rtol=0, atol=4 * U * ov.c.max())
        return gv, ov
    np.testing.assert_allclose(host(gv["S"]), ov.S, rtol=1e-13)
    np.testing.assert_allclose(host(gv["lse"]), ov.lse, rtol=1e-15, atol=1e-13)
    np.testing.assert_allclose(host(gv["c"]), ov.c, rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(host(gv["g"]), ov.g, rtol=0, atol=1e-12 * np.abs(ov.c).max())
    scale = abs(inst.b @ gamma) + inst.eta * np.abs(inst.a * (r + ov.lse)).sum() + 1e-300
    assert abs(gv["L"] - ov.L) <= 1e-12 * scale
    if want_plan:
        np.testing.assert_allclose(host(gv["plan"]), ov.plan, rtol=1e-12, atol=1e-15)
    return gv, ov


# block widths (equal widths rounded up to a multiple of 64, the last one narrower):
# 700 = 2 x 256 + 188; 1025 = 2 x 384 + 257; 4099 = 4 x 832 + 771; 769 = 3 x 256 + 1 (a
# one-column last block); 2049 = 4 x 448 + 257; 3001 = 2 x 1024 + 953; 3000 = 2 x 1024 + 952;
# 2500 = 3 x 640 + 580
SHAPES = [("f64", 37, 700, 256), ("f64", 70, 1025, 512), ("f64", 5, 4099, 1024),
          ("f64", 33, 769, 256), ("f32", 64, 2049, 512), ("f32", 41, 3001, 1024),
          ("pts2", 40, 3000, 1024), ("pts3", 9, 2500, 768)]


@pytest.mark.parametrize("kind,m,n,cols", SHAPES)
@pytest.mark.parametrize("k", [0, 4])
def test_eval_split(ib, ctx, split, kind, m, n, cols, k):
    inst, pr, C = make(ib, kind, m, n, 5)
    r, s, kk, gamma, q = state(inst, C, k)
    split(cols)
    check_eval(ib, ctx, inst, pr, C, r, s, kk, gamma, q)


@pytest.mark.parametrize("kind", ["f64", "pts2"])
def test_eval_split_mixed(ib, ctx, split, kind):
    """FP32 exponentials with split rows: the mixed form's error bounds."""
    inst, pr, C = make(ib, kind, 50, 1500, 6, precision=ib.PREC_MIXED)
    r, s, k, gamma, q = state(inst, C, 0)
    split(512)
    check_eval(ib, ctx, inst, pr, C, r, s, k, gamma, q, mixed=True, want_plan=False)


def test_eval_split_deterministic(ib, ctx, split):
    inst, pr, C = make(ib, "f64", 300, 1800, 3)
    split(640)
    gamma = dev(W.random_dual(1800, 1, 0.01))
    ctr = ib.Center.initial(ctx, pr, gamma)
    a = ib.subproblem_eval(ctx, pr, ctr, gamma)
    b = ib.subproblem_eval(ctx, pr, ctr, gamma)
    for key in ("M", "S", "c", "g"):
        assert torch.equal(a[key], b[key])
    assert a["L"] == b["L"]


@pytest.mark.parametrize("t", [1.0, 1e-3])
@pytest.mark.parametrize("kind,cols", [("f64", 256), ("f32", 512), ("pts3", 384)])
def test_trial_split(ib, ctx, split, kind, cols, t):
    inst, pr, C = make(ib, kind, 61, 1100, 12)
    r, s, k, gamma, q = state(inst, C, 3)
    ev = orc.eval_pass(C, inst.a, inst.b, inst.eta, gamma, r=r, s=s, k=k, q=q)
    Delta = W.random_dual(1100, 44, 0.02)
    split(cols)
    print(f"trial {inst.name} t={t}", flush=True)
    gt = ib.trial(ctx, pr, ib.Center(k, dev(r), dev(s), q), dev(gamma), dev(ev.M), dev(Delta), t)
    dL, Mn, Sn, cn, gn = orc.trial_pass(C, inst.a, inst.b, inst.eta, gamma, ev.M, Delta, t, s=s,
                                        k=k, q=q)
    assert abs(gt["dL"] - dL) <= 1e-12 * abs(dL) + 1e-17 * t
    np.testing.assert_allclose(host(gt["M"]), Mn, rtol=0, atol=q)
    np.testing.assert_allclose(host(gt["M"]) + np.log(host(gt["S"])), Mn + np.log(Sn),
                               rtol=1e-15, atol=1e-12)
    np.testing.assert_allclose(host(gt["c"]), cn, rtol=1e-12)
    np.testing.assert_allclose(host(gt["g"]), gn, rtol=0, atol=1e-12 * np.abs(cn).max())


def test_trial_split_big_step(ib, ctx, split):
    """Steps with t Delta / eta > 500 (the shifted form) with split rows."""
    inst = W.gmm_points(900, 2, m=120)
    inst = W.Instance(inst.C, inst.a, inst.b, 1e-3, "big")
    r, s, gamma = np.log(inst.a), np.log(inst.b), np.zeros(900)
    q = orc.center_quantum(inst.C, s, gamma, inst.eta, 0)
    ev = orc.eval_pass(inst.C, inst.a, inst.b, inst.eta, gamma, q=q)
    Delta = W.random_dual(900, 7, 0.5)
    pr = ib.Problem(dev(inst.C), dev(inst.a), dev(inst.b), inst.eta)
    split(256)
    gt = ib.trial(ctx, pr, ib.Center(0, dev(r), dev(s), q), dev(gamma), dev(ev.M), dev(Delta), 1.0)
    dL, Mn, Sn, cn, gn = orc.trial_pass(inst.C, inst.a, inst.b, inst.eta, gamma, ev.M, Delta, 1.0,
                                        s=s, q=q)
    assert abs(gt["dL"] - dL) <= 1e-12 * abs(dL)
    np.testing.assert_allclose(host(gt["c"]), cn, rtol=1e-11, atol=1e-300)


def compare_csr(gcsr, ocsr, P, rho):
    row_ptr, col, val, d = (host(x) for x in gcsr.export())
    assert gcsr.istar == ocsr.istar
    assert int(row_ptr[-1]) == gcsr.nnz == len(col)
    for i in range(len(row_ptr) - 1):
        gc = col[row_ptr[i]:row_ptr[i + 1]]
        oc = ocsr.col[ocsr.row_ptr[i]:ocsr.row_ptr[i + 1]]
        assert np.all(np.diff(gc) > 0), "columns ascending within a row"
        if not np.array_equal(gc, oc):
            diff = np.setxor1d(gc, oc)
            assert np.all(np.abs(P[i, diff] - rho) <= 1e-12 * rho), (i, diff)
        else:
            np.testing.assert_allclose(val[row_ptr[i]:row_ptr[i + 1]],
                                       ocsr.val[ocsr.row_ptr[i]:ocsr.row_ptr[i + 1]], rtol=1e-12)
    return d


@pytest.mark.parametrize("kind,m,n,cols,rho", [("f64", 120, 700, 256, 1e-4),
                                               ("f64", 40, 2049, 512, 1e-6),
                                               ("f32", 64, 1500, 512, 1e-5),
                                               ("pts2", 90, 1300, 448, 1e-5),
                                               ("f64", 30, 900, 256, 0.0)])
def test_sparsify_split(ib, ctx, split, kind, m, n, cols, rho):
    """Kept entries joined across blocks (pattern, values, d) and the HVP on the factor;
    rho = 0 keeps every entry, so every block's segment moves."""
    inst, pr, C = make(ib, kind, m, n, 8)
    r, s, k, gamma, q = state(inst, C, 2)
    ev = orc.eval_pass(C, inst.a, inst.b, inst.eta, gamma, r=r, s=s, k=k, want_plan=True, q=q)
    P = ev.plan / inst.a[:, None]
    split(cols)
    print(f"sparsify {inst.name} rho={rho}", flush=True)
    gcsr = ib.sparsify(ctx, pr, ib.Center(k, dev(r), dev(s), q), dev(gamma), dev(ev.M),
                       dev(ev.S), rho)
    ocsr = orc.sparsify(C, inst.a, inst.eta, gamma, ev.M, ev.S, rho, s=s, k=k, q=q)
    d = compare_csr(gcsr, ocsr, P, rho)
    assert gcsr.nnz == ocsr.nnz
    np.testing.assert_allclose(d, ocsr.d, rtol=1e-12)
    row_ptr = host(gcsr.export()[0])
    assert row_ptr[gcsr.istar + 1] - row_ptr[gcsr.istar] == n   # the dense row, whole
    for shift in (0.0, 1e-3):
        v = W.random_dual(n, 21, 1.0)
        yg = host(ib.hvp(ctx, gcsr, pr.a, inst.eta, shift, dev(v)))
        yo = orc.hvp(ocsr, inst.a, inst.eta, shift, v)
        np.testing.assert_allclose(yg, yo, rtol=1e-12, atol=1e-12 * np.abs(yo).max())
    gcsr.free()


@pytest.mark.parametrize("kind,cols", [("f64", 256), ("f32", 512), ("pts3", 320)])
@pytest.mark.parametrize("k", [0, 5])
def test_stop_split(ib, ctx, split, kind, cols, k):
    """Both stop passes (Algorithm 3 and the certificate) with split rows."""
    inst, pr, C = make(ib, kind, 150, 1333, 6)
    r, s, kk, gamma, q = state(inst, C, k)
    ev = orc.eval_pass(C, inst.a, inst.b, inst.eta, gamma, r=r, s=s, k=kk, q=q)
    split(cols)
    print(f"stop {inst.name} k={kk}", flush=True)
    gs = ib.stop(ctx, pr, ib.Center(kk, dev(r), dev(s), q), dev(gamma), dev(ev.M), dev(ev.S),
                 want_xhat=True)
    os_ = orc.stop_pass(C, inst.a, inst.b, inst.eta, gamma, ev.M, ev.S, s=s, k=kk,
                        want_xhat=True, q=q)
    np.testing.assert_allclose(host(gs["xhat"]), os_["xhat"], rtol=1e-10, atol=1e-15)
    for key, rtol, atol in [("primal", 1e-12, 0), ("dual", 1e-12, 1e-16), ("cx", 1e-12, 0),
                            ("dual_gamma", 1e-12, 1e-16), ("dual_psi", 1e-12, 1e-16),
                            ("dphi", 1e-9, 1e-15), ("kkt", 1e-9, 1e-16), ("er1", 1e-6, 1e-16)]:
        assert abs(gs[key] - os_[key]) <= rtol * abs(os_[key]) + atol, (key, gs[key], os_[key])


def test_solve_split_matches_oracle(ib, ctx, split):
    """Algorithm 2 to a certified gap of 1e-10 with every dense pass on 3 column blocks,
    against the oracle's solve: objectives bracket one value and plans agree to 1e-9."""
    inst = W.uniform_points(700, 31, m=160)
    eta, gap = 1e-5, 1e-10
    pr = ib.Problem(dev(inst.C), dev(inst.a), dev(inst.b), eta)
    split(256)
    print("solve split 160x700", flush=True)
    g = ib.solve(ctx, pr, ib.default_options(max_outer=5000, gap_tol=gap, marg_tol=0.0),
                 want_plan=True)
    o = orc.solve(inst.C, inst.a, inst.b, eta, want_plan=True,
                  options=orc.default_options(max_outer=5000, gap_tol=gap, marg_tol=0.0))
    assert g["status"] == 0 and o["status"] == 0, (g["report"], o["report"])
    gr, orp = g["report"], o["report"]
    assert gr["rel_gap"] <= gap and orp["rel_gap"] <= gap
    assert gr["dual"] <= orp["primal"] * (1 + 1e-15) and orp["dual"] <= gr["primal"] * (1 + 1e-15)
    assert abs(gr["primal"] - orp["primal"]) <= 2 * gap * orp["primal"]
    np.testing.assert_allclose(host(g["plan"]), o["plan"], rtol=0, atol=1e-9)


@pytest.mark.parametrize("kind", ["f64", "pts2"])
def test_rows_wider_than_tiles(ib, ctx, kind):
    """12000 columns: split by default (two blocks of 6016 and 5984); eval, sparsify and the
    stop test against the oracle."""
    inst, pr, C = make(ib, kind, 64, 12000, 9)
    r, s, k, gamma, q = state(inst, C, 0)
    gv, ov = check_eval(ib, ctx, inst, pr, C, r, s, k, gamma, q, want_plan=False)
    ctr = ib.Center(k, dev(r), dev(s), q)
    rho = 1e-7
    ev = orc.eval_pass(C, inst.a, inst.b, inst.eta, gamma, r=r, s=s, k=k, want_plan=True, q=q)
    gcsr = ib.sparsify(ctx, pr, ctr, dev(gamma), dev(ev.M), dev(ev.S), rho)
    ocsr = orc.sparsify(C, inst.a, inst.eta, gamma, ev.M, ev.S, rho, s=s, k=k, q=q)
    d = compare_csr(gcsr, ocsr, ev.plan / inst.a[:, None], rho)
    np.testing.assert_allclose(d, ocsr.d, rtol=1e-12)
    gcsr.free()
    gs = ib.stop(ctx, pr, ctr, dev(gamma), dev(ev.M), dev(ev.S))
    os_ = orc.stop_pass(C, inst.a, inst.b, inst.eta, gamma, ev.M, ev.S, s=s, k=k, q=q)
    for key, rtol, atol in [("primal", 1e-12, 0), ("dual", 1e-12, 1e-16), ("cx", 1e-12, 0),
                            ("dphi", 1e-9, 1e-15), ("kkt", 1e-9, 1e-16)]:
        assert abs(gs[key] - os_[key]) <= rtol * abs(os_[key]) + atol, (key, gs[key], os_[key])


def test_cfg3_points_20000(ib, ctx):
    """20000 x 20000, 3-D unit-cube points vs an 8-component mixture with the cost formed
    from the points in every pass (no stored matrix; two blocks of 10048 and 9952 columns):
    eval and the stop test against the oracle on the same cost formed in numpy, and a
    short solve that runs every pass on the split rows."""
    # the cube_vs_gmm generator's points (seed 200), without its stored cost
    rng = np.random.default_rng(200)
    x = rng.random((20000, 3))
    y = W._gmm(rng, 20000, 8, 3, 0.08)
    scale = W.points_scale(x, y)
    C = W.points_cost(x, y, scale)
    a, b = np.full(20000, 1.0 / 20000), np.full(20000, 1.0 / 20000)
    inst = W.Instance(C, a, b, 1e-2, "cube_vs_gmm_pts_20000", x, y)
    pr = ib.Problem.from_points(dev(x), dev(y), dev(a), dev(b), inst.eta, scale)
    r, s, k = np.log(a), np.log(b), 0
    gamma = W.random_dual(20000, 4, 0.01)
    q = orc.center_quantum(C, s, gamma, inst.eta, k)
    gv, ov = check_eval(ib, ctx, inst, pr, C, r, s, k, gamma, q, want_plan=False)
    gs = ib.stop(ctx, pr, ib.Center(k, dev(r), dev(s), q), dev(gamma), dev(ov.M), dev(ov.S))
    os_ = orc.stop_pass(C, a, b, inst.eta, gamma, ov.M, ov.S, s=s, k=k, q=q)
    # 4e8 terms: both sides sum per row (GPU: per thread) before the totals
    for key in ("primal", "cx"):
        assert abs(gs[key] - os_[key]) <= 1e-12 * abs(os_[key]), (key, gs[key], os_[key])
    for key, rtol in (("dual", 1e-12), ("dphi", 1e-9), ("kkt", 1e-9)):
        assert abs(gs[key] - os_[key]) <= rtol * abs(os_[key]) + 1e-16, (key, gs[key], os_[key])
    print("cfg3 points: short solve", flush=True)
    res = ib.solve(ctx, pr, ib.default_options(max_outer=3, gap_tol=0.0, marg_tol=0.0))
    rep = res["report"]
    assert res["status"] == 1, rep   # IBSN_WARN_MAXITER: three outer iterations as asked
    assert rep["outer"] == 3 and rep["primal"] >= rep["dual"] - 1e-14
