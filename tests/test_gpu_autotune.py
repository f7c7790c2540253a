"""The dense-pass tile autotuner (ibsn_autotune).

It times every compiled tile that can hold the row on the problem itself and records the
fastest for problems of that shape on the context.  Checked here: the choice is a valid
tile for n and no slower than the built-in table's tiles (the table's choice is among the
candidates, so up to timing noise); passes on the tuned tiles hold the oracle's tolerances
(results differ from the default tiles' by summation order only); the tuned solve reaches
the same certified value; clearing the records restores the default tiles bit for bit.
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


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("n", [700, 3000, 10000])
def test_autotune_choice_and_parity(ib, n):
    inst = W.uniform_points(n, 5, eta=1e-4)
    pr = ib.Problem(dev(inst.C), dev(inst.a), dev(inst.b), inst.eta)
    ctx = ib.Context(0)
    t = ctx.autotune(pr)
    print(f"n {n}: {t}", flush=True)
    vec = 2
    assert t["nt"] * t["q"] * vec >= n and t["nt"] * t["qf"] * vec <= n
    assert t["nt_h"] * t["q_h"] * vec >= n and t["nt_h"] * t["qf_h"] * vec <= n
    assert 1 <= t["grid"] <= 4 * ctx.num_cus
    assert np.isfinite(t["light_ms"]) and np.isfinite(t["heavy_ms"])
    assert t["light_ms"] + t["heavy_ms"] <= 1.15 * (t["default_light_ms"] + t["default_heavy_ms"])
    # an eval pass on the tuned tiles against the oracle
    gamma = W.random_dual(n, 3, 1e-3)
    ctr = ib.Center.initial(ctx, pr, dev(gamma))
    ev = ib.subproblem_eval(ctx, pr, ctr, dev(gamma))
    ov = orc.eval_pass(inst.C, inst.a, inst.b, inst.eta, gamma, q=ctr.quantum)
    np.testing.assert_allclose(ev["c"].cpu().numpy(), ov.c, rtol=1e-12, atol=1e-300)
    assert abs(ev["L"] - ov.L) <= 1e-12 * (abs(ov.L) + 1)
    if n <= 3000:
        # a solve of the same shape (the records are per shape, not per eta) on the tuned
        # tiles and, after clearing, on the default ones
        pr5 = ib.Problem(pr.C, pr.a, pr.b, 1e-5)
        opt = ib.default_options(max_outer=3000, gap_tol=1e-8, marg_tol=0.0)
        a = ib.solve(ctx, pr5, opt)["report"]
        ctx.autotune(None)
        b = ib.solve(ctx, pr5, opt)["report"]
        assert a["rel_gap"] <= 1e-8 and b["rel_gap"] <= 1e-8, (a, b)
        assert a["dual"] <= b["primal"] * (1 + 1e-15) and b["dual"] <= a["primal"] * (1 + 1e-15)
    ctx.close()


def test_autotune_clear_restores_default(ib):
    inst = W.uniform_points(1500, 6, eta=1e-4)
    pr = ib.Problem(dev(inst.C), dev(inst.a), dev(inst.b), inst.eta)
    gamma = dev(W.random_dual(1500, 4, 1e-3))
    ref_ctx = ib.Context(0)
    ctr = ib.Center.initial(ref_ctx, pr, gamma)
    ref = ib.subproblem_eval(ref_ctx, pr, ctr, gamma)
    ctx = ib.Context(0)
    ctx.autotune(pr)
    ctx.autotune(None)
    out = ib.subproblem_eval(ctx, pr, ctr, gamma)
    assert torch.equal(out["c"], ref["c"]) and out["L"] == ref["L"]
    ctx.close()
    ref_ctx.close()
