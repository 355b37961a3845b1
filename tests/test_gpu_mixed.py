"""Mixed precision (FP32 inner s-step, FP64 iterative refinement) against
the FP64 oracle.

The inner solves run the matrix powers and block updates in FP32 while the
moments, the s x s solves and the outer residual r = b - A x stay FP64.  The
refined result must reach the FP64 stopping test ||b - A x|| <= rtol ||b||
computed from the returned x; its distance to the oracle's FP64 solution is
then bounded by cond(A) times the two residual levels, which is what the
tests check (with the closed-form condition number of the operator).
"""
import math

import numpy as np
import pytest

import oracle
from paper_2501_03743_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    from paper_2501_03743_amd import sstep
    with sstep.Handle(0) as h:
        yield h


def _kappa_3d(kind, N):
    c1, cN = math.cos(math.pi / (N + 1)), math.cos(N * math.pi / (N + 1))
    if kind == "3d7":
        return (6 - 6 * cN) / (6 - 6 * c1)
    vals = [27 - (1 + 2 * a) * (1 + 2 * b) * (1 + 2 * c) for a in (c1, cN) for b in (c1, cN)
            for c in (c1, cN)]
    return max(vals) / min(vals)


@pytest.mark.parametrize("kind,N,form,s", [("3d27", 32, "csr", 4), ("3d27", 32, "stencil", 4),
                                           ("3d7", 40, "csr", 4), ("3d7", 40, "stencil", 2)])
def test_mixed_ir_reaches_fp64_accuracy(H, kind, N, form, s):
    shape = (N, N, N)
    n = N ** 3
    b = wl.normal_rhs(n, 0)
    ref = oracle.sstep(oracle.Operator(kind, shape), b, s, rtol=1e-13, maxit=50000)
    A = (H.matrix_csr_from_stencil if form == "csr" else H.matrix_stencil)(kind, shape)
    bd = torch.from_numpy(b).cuda()
    x = torch.zeros_like(bd)
    rtol = 1e-10
    res = H.solve(A, bd, x, s=s, rtol=rtol, maxit=20000, precision="mixed_ir",
                  inner_rtol=1e-5, max_refine=10)
    torch.cuda.synchronize()
    xg = x.cpu().numpy()
    assert res.status == 0, res
    assert res.true_rel <= rtol
    # the returned x really satisfies the FP64 residual test
    r = b - oracle.Operator(kind, shape).apply(xg)
    assert np.linalg.norm(r) <= rtol * np.linalg.norm(b) * 1.001
    err = np.linalg.norm(xg - ref.x) / np.linalg.norm(ref.x)
    print("mixed %s %s N=%d s=%d: refinements=%d inner outer iterations=%d err=%.2e"
          % (kind, form, N, s, len(res.hist) - 1, res.outer, err))
    assert err <= _kappa_3d(kind, N) * (rtol + 1e-13)
    # history: one FP64 true residual per refinement step, decreasing to rtol
    assert res.hist[0] == pytest.approx(1.0) and res.hist[-1] <= rtol
    assert len(res.hist) >= 2
    A.close()


def test_mixed_ir_vark_and_jacobi(H):
    shape = (24, 20, 22)
    n = int(np.prod(shape))
    k = np.exp(wl.gaussian_random_field(shape, 1.0, 0.1, 5))
    kd = torch.from_numpy(k).cuda()
    A = H.matrix_stencil("3d7_vark", shape, k=kd)
    b = wl.normal_rhs(n, 1)
    bd = torch.from_numpy(b).cuda()
    x = torch.zeros_like(bd)
    res = H.solve(A, bd, x, s=3, rtol=1e-10, precision="mixed_ir")
    assert res.status == 0 and res.true_rel <= 1e-10
    ref = oracle.sstep(oracle.Operator("3d7_vark", shape, k=k), b, 3, rtol=1e-13, maxit=50000)
    xg = x.cpu().numpy()
    err = np.linalg.norm(xg - ref.x) / np.linalg.norm(ref.x)
    print("mixed vark: err=%.2e refinements=%d" % (err, len(res.hist) - 1))
    assert err <= 1e-6
    A.close()


def test_mixed_ir_edge_cases(H):
    from paper_2501_03743_amd import sstep
    A = H.matrix_stencil("3d7", (10, 10, 10))
    bd = torch.zeros(1000, dtype=torch.float64, device="cuda")
    x = torch.ones_like(bd)
    res = H.solve(A, bd, x, s=4, precision="mixed_ir")
    assert res.status == 0 and not x.cpu().numpy().any()
    b = torch.from_numpy(wl.normal_rhs(1000, 2)).cuda()
    x = torch.zeros_like(b)
    res = H.solve(A, b, x, s=4, rtol=1e-14, precision="mixed_ir", max_refine=1)
    assert res.status == sstep.NOT_CONVERGED and np.isfinite(x.cpu().numpy()).all()
    with pytest.raises(sstep.SspError):
        H.solve(A, b, x, s=9, precision="mixed_ir")
    with pytest.raises(sstep.SspError):
        H.solve(A, b, x, method="pcg", precision="mixed_ir")
    A.close()
