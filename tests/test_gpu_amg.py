"""The AMG preconditioner (aggregation hierarchy, weighted-Jacobi V-cycle;
Sec. III-A) on the GPU against the oracle (oracle/amg.py).

Bars: the level sizes equal the oracle's (the aggregation is integer work on
the same matrix); one V-cycle agrees to 1e-12 relative (the coarse operators'
sums run in other orders); the basis of Alg. 4 with B^-1 = one V-cycle to
1e-11 per column; s-step solves with it reach the oracle's outer count
within 2 and its iterate within 1e-9 (s <= 4).
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from oracle import amg
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


def _case(H, kind, shape, **amg_kw):
    from paper_2501_03743_amd import sstep
    rp, ci, v = wl.stencil_csr(kind, shape)
    n = rp.size - 1
    A = H.matrix_csr(dev(rp), dev(ci), dev(v), flags=sstep.COPY)
    H.set_amg(A, **amg_kw)
    S = sp.csr_matrix((v, ci, rp), shape=(n, n))
    kw = {("nu" if k == "sweeps" else k): val for k, val in amg_kw.items()}
    return A, S, amg.Hierarchy(S, **kw)


CASES = [("2d5", (64, 64)), ("3d7", (24, 20, 18)), ("2d5", (37, 29))]


@pytest.mark.parametrize("kind,shape", CASES)
def test_levels_and_vcycle(H, kind, shape):
    A, S, ref = _case(H, kind, shape)
    assert H.amg_levels(A) == ref.sizes
    assert len(ref.sizes) >= 3, ref.sizes
    for seed in (0, 1):
        y = wl.normal_rhs(S.shape[0], 10 + seed)
        z = torch.full((S.shape[0],), np.nan, dtype=torch.float64, device="cuda")
        H.amg_apply(A, dev(y), z)
        assert _rel(host(z), ref(y)) <= 1e-12
    A.close()


def test_two_sweeps_and_few_levels(H):
    A, S, ref = _case(H, "3d7", (14, 13, 12), sweeps=2, max_levels=2, max_coarse=64, omega=0.6)
    assert H.amg_levels(A) == ref.sizes == [S.shape[0], ref.sizes[1]]
    y = wl.normal_rhs(S.shape[0], 3)
    z = torch.empty(S.shape[0], dtype=torch.float64, device="cuda")
    H.amg_apply(A, dev(y), z)
    assert _rel(host(z), ref(y)) <= 1e-12
    A.close()


@pytest.mark.parametrize("s", [2, 4])
def test_mpk_basis_with_amg(H, s):
    A, S, ref = _case(H, "3d7", (24, 20, 18))
    r = wl.normal_rhs(S.shape[0], 4)
    P, vm = H.mpk(A, dev(r), s)
    got = host(P)
    Z = [ref(r)]
    AZ = []
    for j in range(s):
        AZ.append(S @ Z[j])
        if j + 1 < s:
            Z.append(ref(AZ[j]))
    cols = Z + AZ
    for c in range(2 * s):
        assert _rel(got[c], cols[c]) <= 1e-11, c
    vref = np.array([Z[a] @ r for a in range(s)] + [Z[a] @ AZ[s - 1] for a in range(s)])
    assert np.allclose(vm, vref, rtol=1e-10, atol=0)
    A.close()


@pytest.mark.parametrize("kind,shape,s,K", [("3d7", (24, 20, 18), 4, 3), ("2d5", (64, 64), 2, 5)])
def test_fixed_iterations_with_amg(H, kind, shape, s, K):
    A, S, ref = _case(H, kind, shape)
    b = wl.normal_rhs(S.shape[0], 5)
    xr, kr, _ = amg.sstep(S, b, ref, s, fixed_outer=K)
    x = torch.zeros(S.shape[0], dtype=torch.float64, device="cuda")
    res = H.solve(A, dev(b), x, s=s, fixed_outer=K)
    assert res.outer == kr == K
    assert _rel(host(x), xr) <= 1e-9
    A.close()


@pytest.mark.parametrize("kind,shape,s", [("3d7", (40, 40, 40), 4), ("2d5", (128, 128), 2),
                                          ("3d7", (33, 31, 29), 1)])
def test_converged_solve_with_amg(H, kind, shape, s):
    A, S, ref = _case(H, kind, shape)
    b = wl.normal_rhs(S.shape[0], 0)
    xr, kr, _ = amg.sstep(S, b, ref, s, rtol=1e-8)
    x = torch.zeros(S.shape[0], dtype=torch.float64, device="cuda")
    res = H.solve(A, dev(b), x, s=s, rtol=1e-8)
    assert res.status == 0
    assert abs(res.outer - kr) <= 2, (res.outer, kr)
    assert _rel(host(x), xr) <= 1e-9
    assert res.true_rel <= 1e-8 * 1.01
    # the same system with Jacobi takes many more outer iterations
    A.set_preconditioner("jacobi")
    xj = torch.zeros_like(x)
    rj = H.solve(A, dev(b), xj, s=s, rtol=1e-8)
    assert rj.outer >= 3 * res.outer, (rj.outer, res.outer)
    A.set_preconditioner("amg")
    A.close()


def test_amg_errors(H):
    from paper_2501_03743_amd import sstep
    As = H.matrix_stencil("3d7", (8, 8, 8))
    with pytest.raises(sstep.SspError) as e:
        H.set_amg(As)
    assert e.value.code == sstep.EUNSUPPORTED
    with pytest.raises(sstep.SspError):
        As.set_preconditioner("amg")   # no hierarchy
    As.close()
    A, S, ref = _case(H, "3d7", (12, 12, 12))
    b = dev(wl.normal_rhs(S.shape[0], 0))
    x = torch.zeros_like(b)
    for kw in (dict(method="pcg"), dict(precision="mixed_ir"), dict(basis="chebyshev")):
        with pytest.raises(sstep.SspError) as e:
            H.solve(A, b, x, s=2, **kw)
        assert e.value.code == sstep.EUNSUPPORTED, kw
    with pytest.raises(sstep.SspError):
        H.set_amg(A, max_coarse=100000)
    A.close()


def test_amg_at_128_cubed(H):
    """The 3D 7-point 128^3 CSR system, s = 4, rtol 1e-8: converged, true
    residual at the bar, far fewer outer iterations than Jacobi's 113."""
    from paper_2501_03743_amd import sstep
    rp, ci, v = wl.stencil_csr("3d7", (128, 128, 128))
    A = H.matrix_csr(dev(rp), dev(ci), dev(v), flags=sstep.COPY)
    H.set_amg(A)
    sizes = H.amg_levels(A)
    assert sizes[0] == 128 ** 3 and sizes[-1] <= 64, sizes
    b = dev(wl.normal_rhs(128 ** 3, 0))
    x = torch.zeros_like(b)
    res = H.solve(A, b, x, s=4, rtol=1e-8)
    assert res.status == 0 and res.true_rel <= 1.01e-8
    assert res.outer <= 40, res.outer
    A.close()
