"""Residual replacement by restart in the oracle (the CPU side of
opts.restarts).

With the monomial basis the s-step recurrences drift from the true residual
by rounding, most at large s (Sec. V-B reports instability there): at s = 8
the recursive test holds while ||b - A x|| / ||b|| stays above rtol.  A
restart from the current x starts from the true residual; the pins check that
the drift is real without restarts, that one restart brings the true residual
below rtol, that the result then agrees with a dense direct solve to
cond(A) times the tolerance, and the bookkeeping (counts add up, histories
concatenate, each run starts with its true residual, the CG-step budget
holds)."""
import numpy as np
import pytest

import oracle
from paper_2501_03743_amd import workloads as wl


@pytest.mark.parametrize("kind,shape", [("2d5", (64, 64, 1)), ("2d5", (96, 80, 1)),
                                        ("3d7", (32, 32, 32))])
def test_restart_meets_the_true_residual(kind, shape):
    op = oracle.Operator(kind, shape)
    b = wl.normal_rhs(op.n, 0)
    plain = oracle.sstep(op, b, 8, rtol=1e-8, maxit=20000)
    assert plain.status == oracle.OK and plain.true_rel > 1e-8   # the drift
    r = oracle.sstep(op, b, 8, rtol=1e-8, maxit=20000, restarts=3)
    assert r.status == oracle.OK and r.restarts >= 1 and r.true_rel <= 1e-8
    # bookkeeping: the first run is the plain one; the next starts from its x
    # with its true residual as the first history entry
    assert r.hist.size == r.outer + 1 + r.restarts
    assert np.array_equal(r.hist[:plain.outer + 1], plain.hist)
    assert r.hist[plain.outer + 1] == plain.true_rel
    again = oracle.sstep(op, b, 8, x0=plain.x, rtol=1e-8, maxit=20000)
    if r.restarts == 1:
        assert np.array_equal(r.x, again.x) and r.outer == plain.outer + again.outer


def test_restarted_solution_against_dense_solve():
    shape = (48, 40, 1)
    op = oracle.Operator("2d5", shape)
    b = wl.normal_rhs(op.n, 3)
    r = oracle.sstep(op, b, 8, rtol=1e-8, maxit=20000, restarts=3)
    assert r.status == oracle.OK and r.true_rel <= 1e-8
    D = np.stack([op.apply(e) for e in np.eye(op.n)], axis=1)
    xd = np.linalg.solve(D, b)
    cond = np.linalg.cond(D)
    assert np.linalg.norm(r.x - xd) / np.linalg.norm(xd) <= cond * 1.1e-8


def test_no_restart_when_not_needed_and_budget():
    op = oracle.Operator("3d7", (20, 18, 16))
    b = wl.normal_rhs(op.n, 1)
    for run in (lambda **k: oracle.pcg(op, b, rtol=1e-8, **k),
                lambda **k: oracle.pfcg(op, b, rtol=1e-8, **k),
                lambda **k: oracle.sstep(op, b, 4, rtol=1e-8, **k)):
        a, c = run(), run(restarts=5)
        assert a.true_rel <= 1e-8 and c.restarts == 0
        assert np.array_equal(a.x, c.x) and a.outer == c.outer
    # a budget used up by the first run allows no restart
    op2 = oracle.Operator("2d5", (64, 64, 1))
    b2 = wl.normal_rhs(op2.n, 0)
    plain = oracle.sstep(op2, b2, 8, rtol=1e-8, maxit=20000)
    r = oracle.sstep(op2, b2, 8, rtol=1e-8, maxit=plain.outer * 8, restarts=3)
    assert r.restarts == 0 and r.true_rel == plain.true_rel
