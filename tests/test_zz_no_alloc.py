"""ibsn_hvp_noalloc (the entry point that allocates nothing) against ibsn_hvp.

Both run the same kernels; the no-allocation variant keeps its intermediate in the
library's fixed per-device array.  Two calls in a row, the second on a smaller factor
(fewer rows and columns), each compared with ibsn_hvp on the same factor and vector:
bit-identical results are expected (same kernels, same summation order), and the bar for
an HVP (1e-12 relative) is asserted as well.  A factor with more rows than the array holds
is rejected with an error.
"""
import numpy as np
import pytest

import oracle as orc
from paper_2603_07156_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def factor(ib, ctx, n, m, seed, rho):
    inst = W.gmm_points(n, seed, m=m)
    gamma = W.random_dual(n, seed + 1, 0.01)
    pr = ib.Problem(dev(inst.C), dev(inst.a), dev(inst.b), inst.eta)
    s = np.log(inst.b)
    q = orc.center_quantum(inst.C, s, gamma, inst.eta, 0)
    ctr = ib.Center(0, dev(np.log(inst.a)), dev(s), q)
    ev = ib.subproblem_eval(ctx, pr, ctr, dev(gamma), want_obj=False)
    csr = ib.sparsify(ctx, pr, ctr, dev(gamma), ev["M"], ev["S"], rho)
    return inst, pr, csr


def test_hvp_noalloc_matches_hvp():
    from paper_2603_07156_amd import ibsn as ib
    ctx = ib.Context(0)
    for (n, m, seed, rho, shift) in [(3000, 2500, 41, 1e-7, 0.3), (700, 300, 42, 1e-5, 0.0)]:
        inst, pr, csr = factor(ib, ctx, n, m, seed, rho)
        assert csr.nnz > n   # several rows besides the dense one
        for vseed in (1, 2):
            v = dev(W.random_dual(n, vseed, 1.0))
            y_ref = ib.hvp(ctx, csr, pr.a, inst.eta, shift, v)
            y = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
            ib.hvp_noalloc(ctx, csr, pr.a, inst.eta, shift, v, y)
            torch.cuda.synchronize()
            yr, yn = y_ref.cpu().numpy(), y.cpu().numpy()
            assert np.all(np.isfinite(yn))
            np.testing.assert_allclose(yn, yr, rtol=1e-12, atol=1e-12 * np.abs(yr).max())
            assert np.array_equal(yn, yr)
        csr.free()
    ctx.close()


def test_hvp_noalloc_rejects_too_many_rows():
    """m above the fixed array's capacity: an error, nothing launched."""
    from paper_2603_07156_amd import ibsn as ib
    m, n = ib.NOALLOC_MAX_M + 1, 1
    ctx = ib.Context(0)
    C = torch.zeros((m, n), dtype=torch.float64, device="cuda")
    a = torch.full((m,), 1.0 / m, dtype=torch.float64, device="cuda")
    b = torch.ones(n, dtype=torch.float64, device="cuda")
    pr = ib.Problem(C, a, b, 1e-2)
    z = torch.zeros(n, dtype=torch.float64, device="cuda")
    ctr = ib.Center(0, torch.log(a), torch.log(b), 2.0 ** -40)
    ev = ib.subproblem_eval(ctx, pr, ctr, z, want_obj=False)
    csr = ib.sparsify(ctx, pr, ctr, z, ev["M"], ev["S"], 0.0)
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    with pytest.raises(ib.IBSNError) as e:
        ib.hvp_noalloc(ctx, csr, a, 1e-2, 0.0, torch.ones(n, dtype=torch.float64, device="cuda"), y)
    assert "exceeds" in str(e.value)
    csr.free()
    ctx.close()
