"""Pins of the oracle's PCG (Alg. 1) and s-step PCG (Alg. 3-6).

What fixes the answers here is outside the oracle: exact rational arithmetic
(s-step iterate x_i equals PCG iterate x_{is}; finite termination at the exact
solution), dense direct solves, closed-form condition numbers with the
Chebyshev bound, the algebraic identities of Sec. II-A (W_i = P_i^T A P_i,
A-conjugacy, residual orthogonality, Hankel structure of P_{i-1}^T A Z_i), and
hand-derived special cases of Alg. 6.
"""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from oracle import exact
from paper_2501_03743_amd import workloads as wl
from golden.paper import PAPER_250  # values the paper prints (Sec. V-B)


# ---------------------------------------------------------------- helpers

def _tridiag(c):
    """1D SPD matrix with integer coefficients c_0..c_n (face weights):
    A_ii = c_i + c_{i+1}, A_{i,i+1} = -c_{i+1}."""
    n = len(c) - 1
    A = [[Fr(0)] * n for _ in range(n)]
    for i in range(n):
        A[i][i] = Fr(c[i] + c[i + 1])
        if i + 1 < n:
            A[i][i + 1] = A[i + 1][i] = Fr(-c[i + 1])
    return A


def _csr_from_dense(A):
    M = sp.csr_matrix(np.array([[float(v) for v in row] for row in A]))
    M.sort_indices()
    return M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data.astype(np.float64)


def _dense_solve_exact(A, b):
    return exact._solve(A, list(map(Fr, b)))


PROBLEMS = {
    # constant coefficients: Jacobi is a scalar multiple of I
    "laplace1d": [1] * 13,
    # variable coefficients: Jacobi changes the Krylov space
    "varcoef1d": [1, 3, 2, 5, 1, 4, 2, 6, 3, 1, 2, 5, 3],
}


# ---------------------------------------------------------------- exact arithmetic

@pytest.mark.parametrize("name", list(PROBLEMS))
def test_exact_pcg_terminates_at_solution(name):
    A = _tridiag(PROBLEMS[name])
    n = len(A)
    b = [(-1) ** i * (i % 5 + 1) for i in range(n)]
    bdiag = [A[i][i] for i in range(n)]
    xs = exact.pcg(A, b, bdiag, n)
    assert xs[-1] == _dense_solve_exact(A, b)


@pytest.mark.parametrize("name", list(PROBLEMS))
@pytest.mark.parametrize("s", [1, 2, 3, 4])
def test_exact_sstep_iterates_equal_pcg_every_s_steps(name, s):
    A = _tridiag(PROBLEMS[name])
    n = len(A)                         # 12: a multiple of 1, 2, 3, 4
    b = [(-1) ** i * (i % 5 + 1) for i in range(n)]
    bdiag = [A[i][i] for i in range(n)]
    ref = exact.pcg(A, b, bdiag, n)
    got = exact.sstep(A, b, bdiag, s, n // s)
    for i, xi in enumerate(got["x"]):
        assert xi == ref[i * s], (s, i)
    assert got["x"][-1] == _dense_solve_exact(A, b)
    # W_i is SPD and symmetric exactly
    for W in got["W"]:
        assert all(W[i][j] == W[j][i] for i in range(s) for j in range(s))


@pytest.mark.parametrize("s", [2, 3, 4])
def test_printed_b1_bound_breaks_equivalence(s):
    """With the inner loop bound of Alg. 6 read literally (j = 1..i-1), part
    of P_{i-1}^T A Z_i is dropped and the iterates leave the PCG ones; the
    full-range reading keeps them equal (previous test)."""
    A = _tridiag(PROBLEMS["varcoef1d"])
    n = len(A)
    b = [(-1) ** i * (i % 5 + 1) for i in range(n)]
    bdiag = [A[i][i] for i in range(n)]
    ref = exact.pcg(A, b, bdiag, n)
    got = exact.sstep(A, b, bdiag, s, 2, b1_printed_bound=True)
    assert got["x"][2] != ref[2 * s]


@pytest.mark.parametrize("name", list(PROBLEMS))
@pytest.mark.parametrize("s", [1, 2, 3, 4])
def test_c_oracle_matches_exact_arithmetic(name, s):
    A = _tridiag(PROBLEMS[name])
    n = len(A)
    b = [(-1) ** i * (i % 5 + 1) for i in range(n)]
    bdiag = [A[i][i] for i in range(n)]
    outer = max(1, min(n // s - 1, 3))       # stay clear of the final (degenerate) step
    ex = exact.sstep(A, b, bdiag, s, outer)
    op = oracle.Operator("csr", csr=_csr_from_dense(A))
    got = oracle.sstep(op, np.array(b, float), s, prec=oracle.PREC_JACOBI,
                       fixed_outer=outer, trace_cap=outer)
    tr = got.trace
    for k in range(outer):
        def rel(a, e):
            e = np.array([[float(v) for v in row] for row in e]) if isinstance(e[0], list) \
                else np.array([float(v) for v in e])
            return np.max(np.abs(np.asarray(a) - e)) / max(np.max(np.abs(e)), 1e-300)
        assert rel(tr["vm"][k], ex["vm"][k]) < 1e-10
        assert rel(tr["W"][k], ex["W"][k]) < 1e-9
        assert rel(tr["alpha"][k], ex["alpha"][k]) < 1e-6
        if k > 0:
            assert rel(tr["beta"][k], ex["beta"][k]) < 1e-6
    xe = np.array([float(v) for v in ex["x"][outer]])
    assert np.linalg.norm(got.x - xe) <= 1e-9 * np.linalg.norm(xe)


# ---------------------------------------------------------------- PCG in FP64

def _kappa(kind, N):
    c1 = math.cos(math.pi / (N + 1))
    cN = math.cos(N * math.pi / (N + 1))
    if kind == "2d5":
        return (4 - 4 * cN) / (4 - 4 * c1)
    if kind == "3d7":
        return (6 - 6 * cN) / (6 - 6 * c1)
    # 27-point: lambda = 27 - prod(1 + 2 cos); extremes over a in {1, N}
    vals = []
    for a in (1, N):
        for bb in (1, N):
            for cc in (1, N):
                cs = [math.cos(t * math.pi / (N + 1)) for t in (a, bb, cc)]
                vals.append(27 - (1 + 2 * cs[0]) * (1 + 2 * cs[1]) * (1 + 2 * cs[2]))
    return max(vals) / min(vals)


@pytest.mark.parametrize("kind,shape", [("2d5", (16, 16)), ("2d5", (22, 22)), ("3d7", (8, 8, 8)),
                                        ("3d27", (7, 7, 7))])
def test_pcg_matches_dense_solve(kind, shape):
    n = int(np.prod(shape))
    csr = wl.stencil_csr(kind, shape)
    Ad = sp.csr_matrix((csr[2], csr[1], csr[0]), shape=(n, n)).toarray()
    b = wl.normal_rhs(n, 0)
    xd = np.linalg.solve(Ad, b)
    kap = _kappa(kind, shape[0])
    rtol = 1e-10
    for op in (oracle.Operator(kind, shape), oracle.Operator("csr", csr=csr)):
        res = oracle.pcg(op, b, rtol=rtol)
        assert res.status == oracle.OK
        err = np.linalg.norm(res.x - xd) / np.linalg.norm(xd)
        assert err <= kap * rtol
        assert res.true_rel <= 10 * rtol


@pytest.mark.parametrize("kind,N", [("2d5", 64), ("3d7", 24), ("3d27", 16)])
def test_pcg_chebyshev_bound_and_manufactured_solution(kind, N):
    shape = (N, N) if kind == "2d5" else (N, N, N)
    n = int(np.prod(shape))
    xs = wl.uniform_solution(n, 0)
    b = wl.csr_matvec(wl.stencil_csr(kind, shape), xs)
    rtol = 1e-8
    res = oracle.pcg(oracle.Operator(kind, shape), b, rtol=rtol)
    kap = _kappa(kind, N)
    bound = math.ceil(0.5 * math.sqrt(kap) * math.log(2 * math.sqrt(kap) / rtol)) + 1
    assert res.status == oracle.OK and 1 <= res.outer <= bound
    assert np.linalg.norm(res.x - xs) / np.linalg.norm(xs) <= kap * rtol
    # residual history is monotone enough to end below rtol and starts at 1
    assert res.hist[0] == pytest.approx(1.0) and res.hist[-1] <= rtol


def test_jacobi_on_constant_diagonal_changes_nothing():
    shape = (20, 20, 20)
    b = wl.normal_rhs(8000, 2)
    op = oracle.Operator("3d7", shape)
    a = oracle.pcg(op, b, rtol=1e-8, prec=oracle.PREC_JACOBI)
    c = oracle.pcg(op, b, rtol=1e-8, prec=oracle.PREC_NONE)
    assert a.outer == c.outer
    assert np.linalg.norm(a.x - c.x) <= 1e-12 * np.linalg.norm(c.x)
    for s in (2, 4):
        a = oracle.sstep(op, b, s, rtol=1e-8, prec=oracle.PREC_JACOBI)
        c = oracle.sstep(op, b, s, rtol=1e-8, prec=oracle.PREC_NONE)
        assert a.outer == c.outer
        assert np.linalg.norm(a.x - c.x) <= 1e-9 * np.linalg.norm(c.x)


# ---------------------------------------------------------------- s-step in FP64

def _vark_problem(N=12, seed=7):
    shape = (N, N, N)
    k = np.exp(wl.gaussian_random_field(shape, 1.0, 0.1, seed))
    return oracle.Operator("3d7_vark", shape, k=k), wl.normal_rhs(N ** 3, seed)


def test_s1_is_pcg():
    op, b = _vark_problem()
    p = oracle.pcg(op, b, rtol=1e-9)
    s1 = oracle.sstep(op, b, 1, rtol=1e-9)
    assert p.status == s1.status == oracle.OK
    assert p.outer == s1.outer
    assert np.linalg.norm(p.x - s1.x) <= 1e-11 * np.linalg.norm(p.x)
    assert np.allclose(p.hist, s1.hist, rtol=1e-8, atol=0)


@pytest.mark.parametrize("s", [2, 3, 4])
def test_sstep_iterates_track_pcg_every_s_steps(s):
    op, b = _vark_problem()
    for i in (1, 2, 3, 5):
        xs = oracle.sstep(op, b, s, fixed_outer=i).x
        xp = oracle.pcg(op, b, rtol=0.0, maxit=i * s).x
        assert np.linalg.norm(xs - xp) <= 1e-8 * np.linalg.norm(xp), (s, i)


@pytest.mark.parametrize("s", [1, 2, 3, 4, 5])
def test_sstep_converges_like_pcg(s):
    op, b = _vark_problem(N=14, seed=3)
    rtol = 1e-8
    p = oracle.pcg(op, b, rtol=rtol)
    r = oracle.sstep(op, b, s, rtol=rtol)
    assert r.status == oracle.OK
    # in exact arithmetic the s-step stops at outer ceil(k/s) for PCG's k
    assert abs(r.outer - math.ceil(p.outer / s)) <= 1
    assert r.true_rel <= 10 * rtol
    assert np.linalg.norm(r.x - p.x) <= 1e-5 * np.linalg.norm(p.x)


@pytest.mark.parametrize("s", [2, 3, 4])
def test_block_identities(s):
    """W_i = P_i^T A P_i; P_i^T A P_{i-1} = 0; P_{i-1}^T A Z_i is Hankel with
    zeros where l + j <= s; P_i^T r_{i+1} = 0 (all relative to the sizes of
    the terms)."""
    N = 8
    shape = (N, N, N)
    k = np.exp(wl.gaussian_random_field(shape, 1.0, 0.1, 11))
    op = oracle.Operator("3d7_vark", shape, k=k)
    Acsr = oracle.stencil_csr("3d7_vark", shape, k=k)
    n = N ** 3
    A = sp.csr_matrix((Acsr[2], Acsr[1], Acsr[0]), shape=(n, n))
    b = wl.normal_rhs(n, 11)
    K = 4
    res = oracle.sstep(op, b, s, fixed_outer=K, trace_cap=K, trace_P=True)
    tr = res.trace
    r = b.copy()
    for i in range(K):
        P = tr["P"][i][:s].T                      # n x s
        AP = tr["P"][i][s:].T
        assert np.allclose(AP, A @ P, rtol=0, atol=1e-10 * np.abs(AP).max())
        G = P.T @ (A @ P)
        assert np.max(np.abs(G - tr["W"][i])) <= 1e-9 * np.max(np.abs(G))
        if i > 0:
            Pp = tr["P"][i - 1][:s].T
            X = P.T @ (A @ Pp)
            assert np.max(np.abs(X)) <= 1e-9 * np.sqrt(np.max(np.abs(G)) *
                                                        np.max(np.abs(Pp.T @ (A @ Pp))))
            Z = P - Pp @ tr["beta"][i]
            Cm = Pp.T @ (A @ Z)
            scale = np.max(np.abs(Cm))
            for l in range(s):
                for j in range(s):
                    if l + j + 2 <= s:
                        assert abs(Cm[l, j]) <= 1e-9 * scale
                    if l + 1 < s and j >= 1:
                        assert abs(Cm[l, j] - Cm[l + 1, j - 1]) <= 1e-9 * scale
        r = r - AP @ tr["alpha"][i]
        orth = P.T @ r
        assert np.max(np.abs(orth)) <= 1e-9 * np.linalg.norm(r) * np.max(np.linalg.norm(P, axis=0))


def test_sw_special_cases_by_hand():
    # s = 1: beta = mu0 / (alpha_prev W_prev), W = mu1 - b1 beta, alpha = mu0 / W
    mu0, mu1, ap, Wp = 2.0, 30.0, 0.25, 3.0
    st, beta, W, alpha = oracle.sw([mu0, mu1], [ap], [[Wp]])
    assert st == 0
    b1 = mu0 / ap
    assert beta[0, 0] == pytest.approx(b1 / Wp, rel=1e-15)
    assert W[0, 0] == pytest.approx(mu1 - b1 * b1 / Wp, rel=1e-15)
    assert alpha[0] == pytest.approx(mu0 / (mu1 - b1 * b1 / Wp), rel=1e-14)
    # s = 2: h2 = -mu0/alpha(2), h3 = -(mu1 + alpha(1) h2)/alpha(2), C = [[0,h2],[h2,h3]]
    vm = np.array([1.5, 5.0, 0.7, 6.0])          # mu0..mu3
    apv = np.array([0.3, -8.0])
    Wp = np.array([[4.0, 1.0], [1.0, 3.0]])
    st, beta, W, alpha = oracle.sw(vm, apv, Wp)
    assert st == 0
    h2 = -vm[0] / apv[1]
    h3 = -(vm[1] + apv[0] * h2) / apv[1]
    Cm = np.array([[0.0, h2], [h2, h3]])
    beta_ref = np.linalg.solve(Wp, -Cm)
    assert np.allclose(beta, beta_ref, rtol=1e-14, atol=1e-14)
    H = np.array([[vm[1], vm[2]], [vm[2], vm[3]]])
    W_ref = H + Cm @ beta_ref
    assert np.allclose(W, W_ref, rtol=1e-14, atol=1e-14)
    assert np.allclose(alpha, np.linalg.solve(W_ref, vm[:2]), rtol=1e-12)


def test_small_spd_solve_matches_numpy():
    g = np.random.default_rng(0)
    for s in range(1, 17):
        M = g.standard_normal((s, s))
        W = M @ M.T + s * np.eye(s)
        c = g.standard_normal(s)
        st, y = oracle.spd_solve(W, c)
        assert st == 0
        assert np.allclose(y, np.linalg.solve(W, c), rtol=1e-12, atol=1e-12)
    st, _ = oracle.spd_solve(np.array([[1.0, 1.0], [1.0, 1.0]]), [1.0, 1.0])
    assert st == 1


# ---------------------------------------------------------------- failure modes

def test_failure_modes():
    shape = (10, 10)
    op = oracle.Operator("2d5", shape)
    b = wl.normal_rhs(100, 0)
    r = oracle.sstep(op, b, 4, maxit=4)
    assert r.status == oracle.NOT_CONVERGED and r.outer == 1 and np.isfinite(r.x).all()
    r = oracle.sstep(op, np.zeros(100), 4)
    assert r.status == oracle.OK and r.outer == 0 and not r.x.any()
    # b an eigenvector: the Krylov space has dimension 1, so W is singular for s >= 2
    v = np.outer(np.sin(np.pi * np.arange(1, 11) / 11), np.sin(2 * np.pi * np.arange(1, 11) / 11))
    r = oracle.sstep(op, v.reshape(-1), 3, rtol=1e-10)
    assert r.status in (oracle.OK, oracle.BREAKDOWN) and np.isfinite(r.x).all()
    if r.status == oracle.OK:
        assert r.true_rel <= 1e-8
    # not SPD: the negated operator breaks down at k = 0
    neg = oracle.Operator("2d5", shape, coef=(-4.0, 1.0))
    r = oracle.sstep(neg, b, 2, prec=oracle.PREC_NONE)
    assert r.status == oracle.BREAKDOWN and r.outer == 0 and not r.x.any()
    assert oracle.sstep(op, b, 17).status == oracle.EINVAL
    assert oracle.sstep(op, b, 0).status == oracle.EINVAL
    # non-finite input never yields OK
    bb = b.copy()
    bb[3] = np.nan
    assert oracle.sstep(op, bb, 2).status != oracle.OK


# ---------------------------------------------------------------- the paper's number

@pytest.mark.slow
def test_paper_iteration_count_250cubed():
    """Sec. V: 3D Poisson 250^3, Dirichlet, b = 1, no preconditioner, relative
    residual 1e-6: PFCG and PCGs with s = 1 need 514 iterations on one GPU.
    The stopping details are not fully stated, so a few percent is allowed."""
    N = 250
    op = oracle.Operator("3d7", (N, N, N))
    b = np.ones(N ** 3)
    r = oracle.sstep(op, b, 1, rtol=1e-6, maxit=2000, prec=oracle.PREC_NONE)
    assert r.status == oracle.OK
    assert abs(r.outer - PAPER_250) <= 0.03 * PAPER_250, r.outer


def test_mpk_basis_and_moment_identities():
    """Alg. 4 fills [z, Kz, .., K^{s-1} z | A z, .., A K^{s-1} z] with z = B^-1 r;
    Alg. 5's vm(j) are the moments mu_{j-1} = r^T K^{j-1} B^-1 r, and the
    Gram matrix Z^T A Z is the Hankel matrix (vm(i+j))."""
    shape = (6, 7, 5)
    k = np.exp(wl.gaussian_random_field(shape, 1.0, 0.1, 2))
    op = oracle.Operator("3d7_vark", shape, k=k)
    r = wl.normal_rhs(op.n, 4)
    dinv = 1.0 / op.diag()
    for s in (1, 2, 3, 5):
        P, vm = oracle.mpk_cvm(op, r, s)
        z = dinv * r
        for j in range(s):
            assert np.array_equal(P[j], z)
            Az = op.apply(z)
            assert np.array_equal(P[s + j], Az)
            z = dinv * Az
        Z = P[:s].T
        AZ = np.stack([op.apply(Z[:, b]) for b in range(s)], axis=1)
        G = Z.T @ AZ
        for a in range(s):
            for b in range(s):
                assert G[a, b] == pytest.approx(vm[a + b + 1], rel=1e-10)
        # moments from their definition: mu_q = r^T K^q B^-1 r
        u = dinv * r
        for q in range(2 * s):
            assert vm[q] == pytest.approx(r @ u, rel=1e-10)
            u = dinv * op.apply(u)
