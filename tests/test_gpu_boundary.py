"""Boundary calls through the C ABI: the initial prox centre and the per-outer-iteration
records of ibsn_solve.

ibsn_center_init forms X^0 = a b^T's implicit centre (r = log a, s = log b, Algorithm 2
input) on the device.  The trace records one entry per outer iteration; their counts and
phase times add up to the report's totals and the last record carries the report's
certificate.
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


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def test_center_init(ib, ctx):
    inst = W.gmm_points(777, 3, m=555)
    pr = ib.Problem(dev(inst.C), dev(inst.a), dev(inst.b), inst.eta)
    r, s = torch.empty(555, dtype=torch.float64, device="cuda"), torch.empty(
        777, dtype=torch.float64, device="cuda")
    ib.center_init(ctx, pr, r, s)
    r0, s0, _ = orc.default_state(inst.a, inst.b)
    np.testing.assert_allclose(host(r), r0, rtol=4e-16, atol=0)
    np.testing.assert_allclose(host(s), s0, rtol=4e-16, atol=0)
    c = ib.Center.initial(ctx, pr)
    assert c.k == 0 and torch.equal(c.r, r) and torch.equal(c.s, s)


SUMMED = ("newton", "cg", "sinkhorn", "backtracks", "stop_tests", "passes", "mixed_passes")
TIMES = ("t_eval", "t_sparsify", "t_cg", "t_linesearch", "t_stop")


@pytest.mark.parametrize("precision", [0, 1])
def test_solve_trace_reconciles_with_report(ib, ctx, precision):
    inst = W.uniform_points(64, 2)
    pr = ib.Problem(dev(inst.C), dev(inst.a), dev(inst.b), inst.eta, precision=precision)
    opt = ib.default_options(max_outer=20000, gap_tol=1e-8, marg_tol=0.0)
    res = ib.solve(ctx, pr, opt, trace_cap=100000)
    rep, tr = res["report"], res["trace"]
    assert res["status"] == 0
    assert rep["trace_len"] == rep["outer"] == len(tr) > 10
    assert [t["k"] for t in tr] == list(range(rep["outer"]))
    for key in SUMMED:
        assert sum(t[key] for t in tr) == rep[key], key
    for key in TIMES:
        assert abs(sum(t[key] for t in tr) - rep[key]) <= 1e-9 * max(rep[key], 1e-3), key
    assert sum(t["t_total"] for t in tr) <= rep["t_total"] * (1 + 1e-9)
    last = tr[-1]
    for key in ("primal", "dual", "rel_gap", "kkt", "dphi", "grad_norm", "marg_l1"):
        assert last[key] == rep[key], key
    # every outer iteration reports a valid certificate (weak duality) and a gap that the
    # report's stop rule reaches only at the end
    assert all(t["primal"] >= t["dual"] - 1e-14 for t in tr)
    assert all(t["rel_gap"] > 1e-8 for t in tr[:-1]) and last["rel_gap"] <= 1e-8
    # the mean stored entries of the last record's factors agree with the report's
    assert last["nnz_mean"] > 0
    if precision == 1:
        assert rep["mixed_passes"] > 0


def test_solve_trace_cap_and_resume(ib, ctx):
    """A cap below the outer count keeps the first records; a resumed solve numbers its
    records from the resumed k."""
    inst = W.uniform_points(40, 8)
    pr = ib.Problem(dev(inst.C), dev(inst.a), dev(inst.b), inst.eta)
    opt = ib.default_options(max_outer=9, gap_tol=0.0, marg_tol=0.0)
    res = ib.solve(ctx, pr, opt, trace_cap=5)
    assert res["report"]["outer"] == 9 and res["report"]["trace_len"] == 5
    assert [t["k"] for t in res["trace"]] == [0, 1, 2, 3, 4]
    part = ib.solve(ctx, pr, ib.default_options(max_outer=4, gap_tol=0.0, marg_tol=0.0))
    rest = ib.solve(ctx, pr, ib.default_options(max_outer=5, gap_tol=0.0, marg_tol=0.0),
                    gamma0=part["gamma"], state=(part["r"], part["s"], part["k"]), trace_cap=10)
    assert [t["k"] for t in rest["trace"]] == [4, 5, 6, 7, 8]
    # the same outer iterations as the uninterrupted run
    full = ib.solve(ctx, pr, opt, trace_cap=9)
    assert len(full["trace"]) == 9
    for a, b in zip(rest["trace"], full["trace"][4:]):
        assert a["newton"] == b["newton"] and a["cg"] == b["cg"] and a["primal"] == b["primal"]
