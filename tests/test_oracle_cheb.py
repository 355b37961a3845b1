"""Pins of the oracle's s-step PCG on a Chebyshev basis (the stabilised-basis
variant of Alg. 3; the related work of Sec. IV names Newton and Chebyshev
bases, Sec. II-A notes that the monomial basis loses independence).

What fixes the answers here is outside the oracle:
  * exact rational arithmetic: the Chebyshev basis spans the same Krylov
    space as the monomial one, so the iterate x_i must EQUAL standard PCG's
    x_{is}, the directions must be exactly A-conjugate and W_i = P_i^T A P_i;
  * the closed form of the Chebyshev polynomials on an eigenvector
    (z_{j+1} = T_j((mu - c)/h) z_1 for K z_1 = mu z_1);
  * dense direct solves and the FP64 oracle's agreement with the exact one.
A flipped sign of the conjugation coefficients is planted in the exact
version to show that these pins catch it.
"""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from oracle import exact
from paper_2501_03743_amd import workloads as wl


def _tridiag(c):
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


PROBLEMS = {
    "laplace1d": [1] * 13,
    "varcoef1d": [1, 3, 2, 5, 1, 4, 2, 6, 3, 1, 2, 5, 3],
}
INTERVALS = [(Fr(0), Fr(2)), (Fr(1, 4), Fr(7, 4))]


def _rhs(n):
    return [(-1) ** i * (i % 5 + 1) for i in range(n)]


# ---------------------------------------------------------------- exact arithmetic

@pytest.mark.parametrize("name", list(PROBLEMS))
@pytest.mark.parametrize("s", [1, 2, 3, 4])
@pytest.mark.parametrize("iv", INTERVALS)
def test_exact_cheb_iterates_equal_pcg_every_s_steps(name, s, iv):
    A = _tridiag(PROBLEMS[name])
    n = len(A)                         # 12: a multiple of 1, 2, 3, 4
    b = _rhs(n)
    bdiag = [A[i][i] for i in range(n)]
    ref = exact.pcg(A, b, bdiag, n)
    got = exact.sstep_cheb(A, b, bdiag, s, n // s, *iv)
    for i, xi in enumerate(got["x"]):
        assert xi == ref[i * s], (s, i)
    assert got["x"][-1] == exact._solve(A, list(map(Fr, b)))


@pytest.mark.parametrize("s", [2, 3, 4])
def test_exact_cheb_directions_conjugate_and_gram(s):
    A = _tridiag(PROBLEMS["varcoef1d"])
    n = len(A)
    bdiag = [A[i][i] for i in range(n)]
    got = exact.sstep_cheb(A, _rhs(n), bdiag, s, n // s - 1, Fr(0), Fr(2))
    for i, blk in enumerate(got["P"]):
        P, AP = blk[:s], blk[s:]
        for j in range(s):
            assert AP[j] == exact._mv(A, P[j])           # A P recurrence exact
        # W_i = P_i^T A P_i (the Gram the step solves with)
        for a in range(s):
            for q in range(s):
                assert got["W"][i][a][q] == exact._dot(P[a], AP[q])
        if i > 0:
            Po = got["P"][i - 1][:s]
            for a in range(s):
                for q in range(s):
                    assert exact._dot(P[a], exact._mv(A, Po[q])) == 0


def test_exact_planted_sign_slip_is_caught():
    A = _tridiag(PROBLEMS["varcoef1d"])
    n = len(A)
    b = _rhs(n)
    bdiag = [A[i][i] for i in range(n)]
    ref = exact.pcg(A, b, bdiag, n)
    bad = exact.sstep_cheb(A, b, bdiag, 3, 3, Fr(0), Fr(2), ap_conj_sign=-1)
    assert bad["x"][1] == ref[3]            # k = 0 has no conjugation
    assert bad["x"][2] != ref[6]


# ---------------------------------------------------------------- the FP64 oracle

@pytest.mark.parametrize("name", list(PROBLEMS))
@pytest.mark.parametrize("s", [1, 2, 4])
def test_c_oracle_matches_exact_arithmetic(name, s):
    A = _tridiag(PROBLEMS[name])
    n = len(A)
    b = _rhs(n)
    bdiag = [A[i][i] for i in range(n)]
    outer = n // s - 1
    ex = exact.sstep_cheb(A, b, bdiag, s, outer, Fr(0), Fr(2))
    op = oracle.Operator("csr", csr=_csr_from_dense(A))
    res = oracle.sstep_cheb(op, np.array(b, float), s, fixed_outer=outer, trace_cap=outer,
                            interval=(0.0, 2.0))
    tr = res.trace
    assert len(tr["W"]) == outer
    for i in range(outer):
        W = np.array([[float(v) for v in row] for row in ex["W"][i]])
        assert np.allclose(tr["W"][i], W, rtol=1e-12, atol=1e-12 * np.abs(W).max())
        al = np.array([float(v) for v in ex["alpha"][i]])
        assert np.allclose(tr["alpha"][i], al, rtol=1e-10, atol=1e-12 * np.abs(al).max())
    xe = np.array([float(v) for v in ex["x"][outer]])
    assert np.linalg.norm(res.x - xe) <= 1e-11 * np.linalg.norm(xe)


@pytest.mark.parametrize("kind,shape,iv", [("2d5", (23, 17), (0.0, 2.0)),
                                           ("3d7", (9, 8, 7), (0.25, 1.75)),
                                           ("3d27", (7, 6, 5), (0.0, 2.0))])
def test_cheb_basis_closed_form_on_an_eigenvector(kind, shape, iv):
    """For a constant-diagonal operator and Jacobi, K = A / d; on the Dirichlet
    eigenvector v (A v = lam v) the basis is z_{j+1} = T_j((mu - c)/h) z_1 with
    mu = lam / d and z_1 = v / d: a dropped -z_{j-1} term, a lost factor 2 or
    a wrong shift fails."""
    sh3 = tuple(shape) + (1,) * (3 - len(shape))
    a = (2, 3, 1)[:len(shape)] + (1,) * (3 - len(shape))
    vs = [np.sin(ad * math.pi * (np.arange(m) + 1.0) / (m + 1)) for m, ad in zip(sh3, a)]
    v = (vs[2][:, None, None] * vs[1][None, :, None] * vs[0][None, None, :]).ravel()
    cs = [math.cos(ad * math.pi / (m + 1)) for m, ad in zip(shape, a)]
    if kind == "2d5":
        lam, d = 4 - 2 * cs[0] - 2 * cs[1], 4.0
    elif kind == "3d7":
        lam, d = 6 - 2 * sum(cs), 6.0
    else:
        lam, d = 27 - (1 + 2 * cs[0]) * (1 + 2 * cs[1]) * (1 + 2 * cs[2]), 26.0
    op = oracle.Operator(kind, shape)
    s = 6
    P = oracle.cheb_basis(op, v, s, *iv)
    lo, hi = iv
    c, h = (hi + lo) / 2, (hi - lo) / 2
    t = (lam / d - c) / h
    z1 = v / d
    for j in range(s):
        Tj = math.cos(j * math.acos(t)) if abs(t) <= 1 else math.cosh(j * math.acosh(abs(t))) * (
            np.sign(t) ** j)
        assert np.allclose(P[j], Tj * z1, rtol=0, atol=1e-13 * np.abs(z1).max()), j
        assert np.allclose(P[s + j], lam * Tj * z1, rtol=0, atol=1e-12 * np.abs(z1).max()), j


def test_cheb_s1_is_pcg():
    shape = (20, 18, 16)
    n = int(np.prod(shape))
    op = oracle.Operator("3d7", shape)
    b = wl.normal_rhs(n, 3)
    a = oracle.pcg(op, b, rtol=1e-10)
    c = oracle.sstep_cheb(op, b, 1, rtol=1e-10)
    assert a.status == c.status == 0 and a.outer == c.outer
    assert np.linalg.norm(a.x - c.x) <= 1e-12 * np.linalg.norm(a.x)


@pytest.mark.parametrize("kind,shape,prec", [("2d5", (16, 16), oracle.PREC_JACOBI),
                                             ("3d7", (8, 8, 8), oracle.PREC_NONE),
                                             ("3d7_vark", (7, 6, 9), oracle.PREC_JACOBI)])
@pytest.mark.parametrize("s", [2, 4, 6])
def test_cheb_matches_dense_solve(kind, shape, prec, s):
    n = int(np.prod(shape))
    k = np.exp(wl.gaussian_random_field(shape, 1.0, 0.1, 2)) if kind == "3d7_vark" else None
    csr = oracle.stencil_csr(kind, shape, k=k)
    Ad = sp.csr_matrix((csr[2], csr[1], csr[0]), shape=(n, n)).toarray()
    xs = wl.uniform_solution(n, 1)
    b = Ad @ xs
    op = oracle.Operator(kind, shape, k=k)
    r = oracle.sstep_cheb(op, b, s, rtol=1e-10, prec=prec)
    assert r.status == 0 and r.true_rel <= 1e-9
    kappa = np.linalg.cond(Ad)
    assert np.linalg.norm(r.x - xs) <= kappa * 2e-10 * np.linalg.norm(xs)


def test_default_interval_encloses_spectrum():
    for kind, shape in (("3d7", (6, 5, 4)), ("3d27", (5, 4, 4)), ("2d5", (9, 7))):
        op = oracle.Operator(kind, shape)
        csr = oracle.stencil_csr(kind, shape)
        n = op.n
        Ad = sp.csr_matrix((csr[2], csr[1], csr[0]), shape=(n, n)).toarray()
        ev = np.linalg.eigvalsh(Ad)
        lo, hi = oracle.basis_interval(op, oracle.PREC_NONE)
        assert lo <= ev.min() and ev.max() <= hi
        d = np.diag(Ad)
        evk = np.linalg.eigvals(Ad / d[:, None]).real
        lo, hi = oracle.basis_interval(op, oracle.PREC_JACOBI)
        assert (lo, hi) == (0.0, 2.0) and lo <= evk.min() and evk.max() <= hi


@pytest.mark.slow
def test_cheb_keeps_true_residual_at_s8_where_monomial_drifts():
    """The purpose of the stabilised basis: at s = 8 the monomial recurrences
    stop on a recursive residual that the true residual no longer follows;
    the Chebyshev basis ends with a true residual below the tolerance."""
    shape = (48, 48, 48)
    n = int(np.prod(shape))
    op = oracle.Operator("3d7", shape)
    b = wl.normal_rhs(n, 0)
    mono = oracle.sstep(op, b, 8, rtol=1e-8)
    cheb = oracle.sstep_cheb(op, b, 8, rtol=1e-8)
    assert cheb.status == 0 and cheb.true_rel <= 1e-8, cheb.true_rel
    pcg = oracle.pcg(op, b, rtol=1e-8)
    assert abs(cheb.outer * 8 - pcg.outer) <= 8 + 0.02 * pcg.outer
    print("s=8 48^3: monomial true_rel %.2e (%d outer), chebyshev %.2e (%d outer), pcg %d"
          % (mono.true_rel, mono.outer, cheb.true_rel, cheb.outer, pcg.outer))
