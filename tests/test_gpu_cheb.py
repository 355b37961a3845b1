"""The Chebyshev-basis s-step path (the stabilised bases of the related work,
Sec. IV) on the GPU against the oracle's sstep_cheb / cheb_basis, through the
C ABI.

Bars:
  * the basis block [Z | AZ]: bit for bit (same recurrence, same rounding,
    no contraction on either side);
  * the block Gram product Z^T [AZ | r] from the FP64 matrix cores: to
    rounding (a different summation order), relative 1e-12 of the entries'
    magnitudes;
  * per-iteration alpha, beta, W at a fixed iteration count: within a bound
    that grows with cond(W) (rounding differences amplified by the s x s
    solves); the iterate within 1e-9 for s <= 4;
  * converged solves: outer count within 2 and x within 1e-9 for s <= 4; at
    s = 8 and 12 the true residual meets rtol without a restart.
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


class Ops:
    """A grid operator in the oracle (matrix-free and CSR) and on the GPU
    (matrix-free and library-built CSR)."""

    def __init__(self, H, kind, shape, seed=0):
        k = kd = None
        if kind == "3d7_vark":
            k = np.exp(wl.gaussian_random_field(shape, 1.0, 0.1, seed))
            kd = dev(k)
        self.mf = oracle.Operator(kind, shape, k=k)
        self.csr = oracle.Operator("csr", csr=wl.stencil_csr(kind, shape, k=k))
        self.n = self.mf.n
        self.keep = kd
        self.mats = [("stencil", H.matrix_stencil(kind, shape, k=kd)),
                     ("csr_lib", H.matrix_csr_from_stencil(kind, shape, k=kd))]

    def oracle_for(self, label):
        return self.mf if label == "stencil" else self.csr

    def close(self):
        for _, A in self.mats:
            A.close()


@pytest.fixture
def make_ops(H):
    made = []

    def mk(kind, shape, seed=0):
        o = Ops(H, kind, shape, seed)
        made.append(o)
        return o
    yield mk
    for o in made:
        o.close()


@pytest.mark.parametrize("kind,shape,s", [
    ("2d5", (13, 11), 3), ("3d7", (17, 9, 7), 4), ("3d7", (33, 20, 21), 8),
    ("3d27", (11, 13, 9), 5), ("3d7_vark", (15, 12, 10), 4), ("3d7", (9, 8, 7), 16),
    ("2d5", (64, 64), 1)])
def test_cheb_basis_bitexact_and_gram(H, make_ops, kind, shape, s):
    ops = make_ops(kind, shape)
    r = wl.normal_rhs(ops.n, 3)
    rd = dev(r)
    for label, A in ops.mats:
        for prec in ("jacobi", "none"):
            A.set_preconditioner(prec)
            op = ops.oracle_for(label)
            pk = oracle.PREC_JACOBI if prec == "jacobi" else oracle.PREC_NONE
            lo, hi = oracle.basis_interval(op, pk)
            Pref = oracle.cheb_basis(op, r, s, lo, hi, pk)
            P, gram = H.cheb_basis(A, rd, s)          # the library's default interval
            Pg = host(P)
            assert np.array_equal(Pg, Pref), (label, prec, np.max(np.abs(Pg - Pref)))
            Z, AZ = Pref[:s], Pref[s:]
            ref = np.concatenate([Z @ AZ.T, (Z @ r)[:, None]], axis=1)
            scale = np.abs(Z) @ np.abs(np.concatenate([AZ, r[None]], axis=0)).T
            assert np.all(np.abs(gram - ref) <= 1e-12 * scale + 1e-300), (label, prec)
        A.set_preconditioner("jacobi")


@pytest.mark.parametrize("kind,shape,s,K", [
    ("2d5", (64, 64), 4, 10), ("2d5", (64, 64), 1, 20), ("3d7", (24, 24, 24), 2, 10),
    ("3d7", (24, 24, 24), 4, 8), ("3d27", (20, 20, 20), 3, 6), ("3d7_vark", (20, 18, 16), 4, 10),
    ("3d7_vark", (20, 18, 16), 8, 5)])
def test_cheb_fixed_iteration_trace_parity(H, make_ops, kind, shape, s, K):
    ops = make_ops(kind, shape)
    b = wl.normal_rhs(ops.n, 7)
    bd = dev(b)
    for label, A in ops.mats:
        ref = oracle.sstep_cheb(ops.oracle_for(label), b, s, fixed_outer=K, trace_cap=K)
        tr = ref.trace
        x = torch.zeros_like(bd)
        res = H.solve(A, bd, x, s=s, fixed_outer=K, trace_cap=K, basis="chebyshev")
        assert res.outer == ref.outer == K, label
        g = res.trace
        kappa = 1.0
        for i in range(K):
            tol = max(1e-10, 4096 * 2.0 ** -52 * kappa)
            # vm holds Z^T r and diag(Z^T A Z) on both sides; the inner
            # products z_a^T r of a well-conditioned basis nearly cancel, so
            # each half is compared relative to its largest entry
            for part in (slice(0, s), slice(s, 2 * s)):
                gv, tv = g["vm"][i][part], tr["vm"][i][part]
                assert np.max(np.abs(gv - tv)) <= tol * np.max(np.abs(tv)), (label, i, tol)
            sc = np.max(np.abs(tr["W"][i]))
            assert np.max(np.abs(g["W"][i] - tr["W"][i])) <= tol * sc, (label, i)
            kappa = max(kappa, np.linalg.cond(tr["W"][i]))
            tol = max(1e-10, 4096 * 2.0 ** -52 * kappa)
            assert _rel(g["alpha"][i], tr["alpha"][i]) <= tol, (label, i, tol)
            if i > 0:
                assert _rel(g["beta"][i], tr["beta"][i]) <= tol, (label, i)
        xtol = 1e-9 if s <= 4 else max(1e-9, 4096 * 2.0 ** -52 * kappa)
        assert _rel(host(x), ref.x) <= xtol, (label, _rel(host(x), ref.x))
        assert np.allclose(res.hist, ref.hist, rtol=max(1e-8, xtol), atol=0)


@pytest.mark.parametrize("kind,shape,s", [
    ("2d5", (64, 64), 4), ("3d7", (40, 40, 40), 2), ("3d7", (40, 40, 40), 4),
    ("3d27", (32, 32, 32), 4), ("3d7_vark", (28, 28, 28), 3)])
def test_cheb_converged_solve_parity(H, make_ops, kind, shape, s):
    ops = make_ops(kind, shape)
    b = wl.normal_rhs(ops.n, 0)
    bd = dev(b)
    for label, A in ops.mats:
        ref = oracle.sstep_cheb(ops.oracle_for(label), b, s, rtol=1e-8, maxit=20000)
        assert ref.status == oracle.OK
        x = torch.zeros_like(bd)
        res = H.solve(A, bd, x, s=s, rtol=1e-8, maxit=20000, basis="chebyshev")
        assert res.status == 0, label
        assert abs(res.outer - ref.outer) <= 2, (label, res.outer, ref.outer)
        assert _rel(host(x), ref.x) <= 1e-9, (label, _rel(host(x), ref.x))
        assert res.true_rel <= 1e-8


@pytest.mark.parametrize("s", [8, 12, 16])
def test_cheb_large_s_reaches_rtol_without_restart(H, make_ops, s):
    # the monomial basis breaks down or misses the true-residual target here
    ops = make_ops("3d7", (48, 48, 48))
    b = wl.normal_rhs(ops.n, 0)
    bd = dev(b)
    _, A = ops.mats[1]
    ref = oracle.sstep_cheb(ops.csr, b, s, rtol=1e-8, maxit=20000)
    x = torch.zeros_like(bd)
    res = H.solve(A, bd, x, s=s, rtol=1e-8, maxit=20000, basis="chebyshev")
    assert res.status == 0 and res.restarts == 0
    assert res.true_rel <= 1e-8, res.true_rel
    assert abs(res.outer - ref.outer) <= 2, (res.outer, ref.outer)
    r = ops.csr.apply(host(x))
    assert np.linalg.norm(b - r) <= 1e-8 * np.linalg.norm(b)


def test_cheb_mixed_precision(H, make_ops):
    ops = make_ops("3d7", (40, 40, 40))
    b = wl.normal_rhs(ops.n, 0)
    bd = dev(b)
    ref = oracle.sstep(ops.csr, b, 4, rtol=1e-12, maxit=20000)
    lam_min = 6 - 6 * np.cos(np.pi / 41)
    cond = (6 + 6 * np.cos(np.pi / 41)) / lam_min
    for label, A in ops.mats:
        for s in (4, 8):
            x = torch.zeros_like(bd)
            res = H.solve(A, bd, x, s=s, rtol=1e-8, precision="mixed_ir", basis="chebyshev")
            assert res.status == 0, (label, s)
            xh = host(x)
            assert np.linalg.norm(b - ops.csr.apply(xh)) <= 1e-8 * np.linalg.norm(b)
            assert _rel(xh, ref.x) <= cond * (2e-8 + 1e-13), (label, s, _rel(xh, ref.x))


def test_cheb_deterministic_and_errors(H, make_ops):
    from paper_2501_03743_amd import sstep
    ops = make_ops("3d7_vark", (20, 18, 16))
    b = dev(wl.normal_rhs(ops.n, 1))
    _, A = ops.mats[1]
    xs = []
    for _ in range(2):
        x = torch.zeros_like(b)
        H.solve(A, b, x, s=6, rtol=1e-8, basis="chebyshev")
        xs.append(host(x))
    assert np.array_equal(xs[0], xs[1])
    with pytest.raises(sstep.SspError):
        H.solve(A, b, torch.zeros_like(b), s=4, basis="chebyshev", interval=(-np.inf, 2.0))
    # an interval with hi <= lo selects the default one
    x = torch.zeros_like(b)
    H.solve(A, b, x, s=6, rtol=1e-8, basis="chebyshev", interval=(1.0, 1.0))
    assert np.array_equal(host(x), xs[0])
    with pytest.raises(sstep.SspError):
        H.solve(A, b, torch.zeros_like(b), method="pcg", basis="chebyshev")
