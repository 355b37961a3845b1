"""Temporally blocked matrix powers of the 3D 7-point operator (Sec. IV's
communication-avoiding powers, one z-marching launch per up to 4 powers).

Bars: the basis [Z; AZ] is bit-exact against the oracle's Alg. 4 (and against
the one-launch-per-power path); the moments of Alg. 5 agree to 1e-12
relative (only the reduction order differs); solves that use the blocked
launches meet the oracle's iteration count and the 1e-9 iterate bar.
Grids are chosen to span several 32 x 32 tiles and several z chunks, with
ragged tails in every dimension.
"""
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _matrix(H, shape, temporal, monkeypatch):
    # "2": the blocked launches also on grids too small to fill the GPU
    monkeypatch.setenv("SSP_MPK_TEMPORAL", "2" if temporal else "0")
    A = H.matrix_stencil("3d7", shape)
    monkeypatch.delenv("SSP_MPK_TEMPORAL", raising=False)
    return A


@pytest.mark.parametrize("shape", [(70, 45, 37), (33, 64, 17), (5, 7, 40)])
@pytest.mark.parametrize("s", [2, 3, 4, 5, 7, 8])
def test_temporal_basis_bitexact(H, monkeypatch, shape, s):
    n = int(np.prod(shape))
    r = wl.normal_rhs(n, 11)
    Pref, vmref = oracle.mpk_cvm(oracle.Operator("3d7", shape), r, s)
    rd = dev(r)
    A = _matrix(H, shape, True, monkeypatch)
    P, vm = H.mpk(A, rd, s)
    got = host(P)
    bad = np.argwhere(got != Pref)
    assert bad.size == 0, (shape, s, bad[:5])
    assert np.allclose(vm, vmref, rtol=1e-12, atol=0), (vm, vmref)
    # the one-launch-per-power path: the same basis, moments to rounding
    B = _matrix(H, shape, False, monkeypatch)
    P2, vm2 = H.mpk(B, rd, s)
    assert np.array_equal(host(P2), got)
    assert np.allclose(vm2, vm, rtol=1e-12, atol=0)
    A.close()
    B.close()


@pytest.mark.parametrize("shape,s,K", [((40, 36, 29), 4, 6), ((40, 36, 29), 8, 3),
                                       ((33, 33, 65), 3, 5)])
def test_temporal_fixed_iterations(H, monkeypatch, shape, s, K):
    """Fixed-iteration s-step runs: the blocked launches against the oracle
    (iterate to 1e-9 at s <= 4, beyond that 4096 eps times the largest
    condition number of the W_i) and against the one-launch-per-power path."""
    n = int(np.prod(shape))
    b = wl.normal_rhs(n, 3)
    ref = oracle.sstep(oracle.Operator("3d7", shape), b, s, fixed_outer=K, trace_cap=K)
    bd = dev(b)
    xs = []
    for temporal in (True, False):
        A = _matrix(H, shape, temporal, monkeypatch)
        x = torch.zeros_like(bd)
        res = H.solve(A, bd, x, s=s, fixed_outer=K)
        assert res.outer == K
        xs.append(host(x))
        A.close()
    # beyond s = 4 the reduction-order difference of the moments is amplified
    # by the condition of the monomial-basis W_i (as in the parity tests)
    kappa = max(np.linalg.cond(W) for W in ref.trace["W"][:K])
    tol = 1e-9 if s <= 4 else max(1e-9, 4096 * 2.0 ** -52 * kappa)
    assert _rel(xs[0], ref.x) <= tol, _rel(xs[0], ref.x)
    assert _rel(xs[0], xs[1]) <= tol, _rel(xs[0], xs[1])


@pytest.mark.parametrize("N,s", [(64, 4), (96, 2)])
def test_temporal_converged_solve(H, monkeypatch, N, s):
    """Converged solve on the blocked launches: the oracle's outer count
    within 2 and the iterate within 1e-9."""
    shape = (N, N, N)
    b = wl.normal_rhs(N ** 3, 0)
    ref = oracle.sstep(oracle.Operator("3d7", shape), b, s, rtol=1e-8, maxit=20000)
    A = _matrix(H, shape, True, monkeypatch)
    bd = dev(b)
    x = torch.zeros_like(bd)
    res = H.solve(A, bd, x, s=s, rtol=1e-8)
    assert res.status == 0
    assert abs(res.outer - ref.outer) <= 2, (res.outer, ref.outer)
    assert _rel(host(x), ref.x) <= 1e-9
    assert res.true_rel <= 1e-8
    A.close()
