"""Pins of the oracle's grid operators and inner product against closed forms.

Eigenpairs of the Dirichlet Laplacians: with theta_a = a pi / (N+1), the
vectors prod_d sin(a_d theta (i_d+1)) are eigenvectors with eigenvalues
  2D 5-point   4 - 2 cos th_a - 2 cos th_b
  3D 7-point   6 - 2 sum_d cos th_{a_d}
  3D 27-point  27 - prod_d (1 + 2 cos th_{a_d})   (A = 27 I - J(x)J(x)J, J = tridiag(1,1,1))
"""
import math

import numpy as np
import pytest

import oracle
from paper_2501_03743_amd import workloads as wl


def _mode(shape, a):
    nx, ny, nz = (tuple(shape) + (1,))[:3]
    vs = []
    for m, ad in zip((nx, ny, nz), a):
        i = np.arange(m) + 1.0
        vs.append(np.sin(ad * math.pi * i / (m + 1)))
    v = vs[2][:, None, None] * vs[1][None, :, None] * vs[0][None, None, :]
    return v.reshape(-1)


def _lam(kind, shape, a):
    cs = [math.cos(ad * math.pi / (m + 1)) for m, ad in zip(shape, a)]
    if kind == "2d5":
        return 4 - 2 * cs[0] - 2 * cs[1]
    if kind == "3d7":
        return 6 - 2 * sum(cs)
    return 27 - (1 + 2 * cs[0]) * (1 + 2 * cs[1]) * (1 + 2 * cs[2])


@pytest.mark.parametrize("kind,shape,modes", [
    ("2d5", (13, 9), [(1, 1), (3, 5), (13, 9), (7, 2)]),
    ("3d7", (6, 7, 5), [(1, 1, 1), (2, 3, 4), (6, 7, 5)]),
    ("3d27", (5, 6, 7), [(1, 1, 1), (4, 2, 6), (5, 6, 7)]),
])
def test_closed_form_eigenpairs(kind, shape, modes):
    op = oracle.Operator(kind, shape)
    csr = oracle.Operator("csr", csr=oracle.stencil_csr(kind, shape))
    for a in modes:
        a3 = tuple(a) + (1,) * (3 - len(a))
        sh3 = tuple(shape) + (1,) * (3 - len(shape))
        v = _mode(sh3, a3)
        lam = _lam(kind, shape, a)
        for o in (op, csr):
            Av = o.apply(v)
            assert np.max(np.abs(Av - lam * v)) <= 1e-13 * max(1.0, abs(lam)) * np.max(np.abs(v)) * 4


@pytest.mark.parametrize("kind,N,formula", [
    ("2d5", 17, lambda N: 5 * N * N - 4 * N),
    ("3d7", 9, lambda N: 7 * N ** 3 - 6 * N ** 2),
    ("3d27", 8, lambda N: (3 * N - 2) ** 3),
])
def test_nnz_formulas_and_symmetry(kind, N, formula):
    shape = (N, N) if kind == "2d5" else (N, N, N)
    assert oracle.stencil_nnz(kind, shape) == formula(N)
    rowptr, colind, val = oracle.stencil_csr(kind, shape)
    assert rowptr[-1] == formula(N)
    import scipy.sparse as sp
    n = len(rowptr) - 1
    A = sp.csr_matrix((val, colind, rowptr), shape=(n, n))
    assert (abs(A - A.T)).max() == 0
    # columns ascending within rows
    for i in range(0, n, max(1, n // 50)):
        c = colind[rowptr[i]:rowptr[i + 1]]
        assert np.all(np.diff(c) > 0)
    # interior rows sum to zero for the unscaled Laplacians (27-pt: 26 - 26)
    rs = np.asarray(A.sum(axis=1)).ravel()
    nnzrow = np.diff(rowptr)
    full = nnzrow == nnzrow.max()
    assert np.all(rs[full] == 0)


def test_vark_hand_example():
    # 2 x 1 x 1 grid, k = (1, 3): the shared face has weight 2*1*3/(1+3) = 1.5,
    # each of the other 5 faces of a cell weighs k_p.
    k = np.array([1.0, 3.0])
    rowptr, colind, val = oracle.stencil_csr("3d7_vark", (2, 1, 1), k=k)
    import scipy.sparse as sp
    A = sp.csr_matrix((val, colind, rowptr), shape=(2, 2)).toarray()
    assert np.array_equal(A, np.array([[6.5, -1.5], [-1.5, 16.5]]))


def test_vark_matrix_free_diagonal():
    """The Jacobi diagonal of the matrix-free variable-coefficient operator
    (Sec. III-A's Jacobi building block) against the hand-derived 2-cell
    matrix above and, on ragged grids, against the diagonal of the CSR matrix
    that the hand example and the product test pin.  Every cell of these
    grids has faces on the Dirichlet boundary, so a diagonal that drops the
    k_p weight of those faces fails here."""
    k = np.array([1.0, 3.0])
    d = oracle.Operator("3d7_vark", (2, 1, 1), k=k).diag()
    assert np.array_equal(d, np.array([6.5, 16.5]))
    import scipy.sparse as sp
    for shape, seed in (((6, 5, 4), 3), ((7, 3, 5), 4), ((1, 4, 3), 5)):
        n = int(np.prod(shape))
        kk = np.exp(wl.gaussian_random_field(shape, 1.0, 0.1, seed))
        rowptr, colind, val = oracle.stencil_csr("3d7_vark", shape, k=kk)
        A = sp.csr_matrix((val, colind, rowptr), shape=(n, n))
        assert np.array_equal(oracle.Operator("3d7_vark", shape, k=kk).diag(), A.diagonal())


def test_vark_constant_k_is_scaled_poisson():
    shape = (5, 4, 6)
    k = np.full(5 * 4 * 6, 2.5)
    ra, ca, va = oracle.stencil_csr("3d7_vark", shape, k=k)
    rb, cb, vb = oracle.stencil_csr("3d7", shape)
    assert np.array_equal(ra, rb) and np.array_equal(ca, cb)
    # interior: 6 * 2.5 and -2.5; boundary rows carry the Dirichlet faces, so
    # the diagonal stays 6 k everywhere (6 faces of weight k each)
    assert np.allclose(va, 2.5 * vb, rtol=0, atol=1e-15)


@pytest.mark.parametrize("kind,shape", [("2d5", (11, 7)), ("3d7", (5, 6, 4)), ("3d27", (4, 5, 6)),
                                        ("3d7_vark", (6, 5, 4))])
def test_matrix_free_equals_csr_and_workload_csr(kind, shape):
    n = int(np.prod(shape))
    k = np.exp(wl.gaussian_random_field(shape, 0.5, 0.1, 3)) if kind == "3d7_vark" else None
    csr_o = oracle.stencil_csr(kind, shape, k=k)
    csr_w = wl.stencil_csr(kind, shape, k=k)
    for a, b in zip(csr_o, csr_w):
        assert a.dtype == b.dtype and np.array_equal(a, b)
    x = np.random.default_rng(1).standard_normal(n)
    mf = oracle.Operator(kind, shape, k=k).apply(x)
    cs = oracle.Operator("csr", csr=csr_o).apply(x)
    assert np.allclose(mf, cs, rtol=1e-14, atol=1e-14)
    # SPD: the symmetric matrix is diagonally dominant with positive diagonal
    d = oracle.Operator(kind, shape, k=k).diag()
    assert np.all(d > 0)


def test_dot_is_accurate_and_deterministic():
    g = np.random.default_rng(5)
    for n in (1, 7, 4096, 4097, 100_003):
        a = g.standard_normal(n)
        b = g.standard_normal(n)
        exact = math.fsum(a * b)  # products are rounded once; fsum sums them exactly
        got = oracle.dot(a, b)
        assert abs(got - exact) <= 1e-13 * math.fsum(np.abs(a * b))
    a = g.standard_normal(50_000)
    assert oracle.dot(a, a) == oracle.dot(a, a)


def test_workload_generators_are_seeded():
    assert np.array_equal(wl.normal_rhs(100, 4), wl.normal_rhs(100, 4))
    assert not np.array_equal(wl.normal_rhs(100, 4), wl.normal_rhs(100, 5))
    g = wl.gaussian_random_field((16, 16, 16), 0.5, 0.1, 0)
    assert g.shape == (4096,) and abs(g.std() - 0.5) < 1e-12 and abs(g.mean()) < 1e-12
    f = wl.fourier_source((8, 9, 10), 1)
    assert f.shape == (720,) and np.isfinite(f).all()
    L = wl.batch_sides(0)
    assert L.shape == (32,) and L.min() >= 32 and L.max() <= 160
