"""Aggregation AMG preconditioner and the solvers that use it (CPU oracle).

TEST INFRASTRUCTURE ONLY: imported by tests/, the package's smoke check and
the bench's CPU baseline; never by the product path.

The paper's weak-scaling runs (Sec. III-A, Sec. V-B) precondition with an
algebraic multigrid whose B^-1 is a few weighted-Jacobi sweeps on each level
of a hierarchy of coarser matrices built from A.  The paper refers to its
library for the details; this oracle takes a standard reading, the smoothed
aggregation of Vanek, Mandel and Brezina (1996), written out plainly:

* strength: j != i is a strong neighbour of i when a_ij^2 >= theta_l^2 |a_ii a_jj|,
  theta_l = theta 2^-l on level l (the coarse operators' couplings are
  weaker relative to their diagonals; with a fixed theta the 3D hierarchy
  stalls after one level);
* aggregation in three passes over the rows in index order: (1) a row whose
  strong neighbours are all free starts an aggregate with them; (2) a row
  still free joins the pass-1 aggregate of its strongest aggregated strong
  neighbour (weights within a relative 1e-9 count as ties, won by the
  smallest column, so that rounding in the Galerkin sums of a coarse level
  cannot decide the choice); (3) a row still free starts an aggregate with
  its free strong neighbours;
* tentative prolongator P_t(i, agg(i)) = 1, smoothed
  P = (I - omega_p D^-1 A) P_t with omega_p = 4 / (3 rho_G), rho_G the
  Gershgorin bound max_i sum_j |a_ij| / |a_ii| of rho(D^-1 A);
* Galerkin coarse operator A_c = P^T A P, restriction R = P^T;
* coarsening stops at max_coarse rows, max_levels levels, or when a level
  keeps more than 90 % of the rows; the coarsest level is solved exactly;
* V-cycle with nu sweeps of weighted Jacobi (weight omega) before and after
  the coarse correction, the first from a zero guess, so B^-1 is symmetric
  and, for omega < 2 / rho(D^-1 A), positive definite.

Sparse products are scipy's; nothing is blocked or fused.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

import oracle

THETA = 0.08
OMEGA = 2.0 / 3.0
NU = 1
MAX_COARSE = 64
MAX_LEVELS = 10
TIE = 1e-9          # relative width of a tie between neighbour weights


def strength(A: sp.csr_matrix, theta: float = THETA):
    """Strong-neighbour lists (column order of the stored row), i excluded."""
    A = sp.csr_matrix(A)
    d = A.diagonal()
    out = []
    for i in range(A.shape[0]):
        lo, hi = A.indptr[i], A.indptr[i + 1]
        nb = []
        for jj in range(lo, hi):
            j = int(A.indices[jj])
            if j == i:
                continue
            a = float(A.data[jj])
            if a * a >= theta * theta * abs(d[i] * d[j]):
                nb.append((j, abs(a)))
        out.append(nb)
    return out


def aggregate(A: sp.csr_matrix, theta: float = THETA):
    """Aggregate index of every row (three passes, see the module text)."""
    S = strength(A, theta)
    n = len(S)
    agg = np.full(n, -1, dtype=np.int64)
    k = 0
    for i in range(n):                       # pass 1
        if agg[i] >= 0:
            continue
        if all(agg[j] < 0 for j, _ in S[i]):
            agg[i] = k
            for j, _ in S[i]:
                agg[j] = k
            k += 1
    first = agg.copy()
    for i in range(n):                       # pass 2: join a pass-1 aggregate
        if agg[i] >= 0:
            continue
        best, bw = -1, -1.0
        for j, w in S[i]:
            if first[j] < 0:
                continue
            if best < 0 or w > bw * (1.0 + TIE) or (w >= bw * (1.0 - TIE) and j < best):
                best, bw = j, w
        if best >= 0:
            agg[i] = first[best]
    for i in range(n):                       # pass 3: the rest
        if agg[i] >= 0:
            continue
        agg[i] = k
        for j, _ in S[i]:
            if agg[j] < 0:
                agg[j] = k
        k += 1
    return agg, k


def tentative(agg, nc):
    n = agg.size
    return sp.csr_matrix((np.ones(n), (np.arange(n), agg)), shape=(n, nc))


def gershgorin(A: sp.csr_matrix) -> float:
    """max_i sum_j |a_ij| / |a_ii| (an upper bound of rho(D^-1 A))."""
    A = sp.csr_matrix(A)
    d = np.abs(A.diagonal())
    rows = np.asarray(abs(A).sum(axis=1)).ravel()
    return float(np.max(rows / d))


def prolongator(A: sp.csr_matrix, agg, nc):
    """Smoothed P = (I - omega_p D^-1 A) P_t."""
    Pt = tentative(agg, nc)
    wp = 4.0 / (3.0 * gershgorin(A))
    Dinv = sp.diags(1.0 / A.diagonal())
    return sp.csr_matrix(Pt - wp * (Dinv @ (A @ Pt)))


class Hierarchy:
    def __init__(self, A, theta=THETA, omega=OMEGA, nu=NU, max_coarse=MAX_COARSE,
                 max_levels=MAX_LEVELS):
        A = sp.csr_matrix(A, dtype=np.float64)
        A.sort_indices()
        self.omega, self.nu = omega, nu
        self.A, self.P, self.R, self.aggs = [A], [], [], []
        while (self.A[-1].shape[0] > max_coarse and len(self.A) < max_levels):
            Al = self.A[-1]
            agg, nc = aggregate(Al, theta * 0.5 ** (len(self.A) - 1))
            if nc >= 0.9 * Al.shape[0] or nc == 0:
                break
            P = prolongator(Al, agg, nc)
            R = sp.csr_matrix(P.T)
            Ac = sp.csr_matrix(R @ Al @ P)
            Ac.sort_indices()
            self.aggs.append(agg)
            self.P.append(P)
            self.R.append(R)
            self.A.append(Ac)
        self.coarse = np.linalg.inv(self.A[-1].toarray())
        self.dinv = [1.0 / Al.diagonal() for Al in self.A]

    @property
    def sizes(self):
        return [Al.shape[0] for Al in self.A]

    def vcycle(self, y, level=0):
        """z = B^-1 y on the given level."""
        if level == len(self.A) - 1:
            return self.coarse @ y
        A, dinv, w = self.A[level], self.dinv[level], self.omega
        z = w * (dinv * y)
        for _ in range(self.nu - 1):
            z = z + w * (dinv * (y - A @ z))
        r = y - A @ z
        zc = self.vcycle(self.R[level] @ r, level + 1)
        z = z + self.P[level] @ zc
        for _ in range(self.nu):
            z = z + w * (dinv * (y - A @ z))
        return z

    __call__ = vcycle


def pcg(A, b, H, rtol=1e-8, maxit=10000):
    """Alg. 1 with B^-1 = one V-cycle.  Returns (x, iterations, hist)."""
    A = sp.csr_matrix(A)
    x = np.zeros_like(b)
    r = b.copy()
    u = H(r)
    p = u.copy()
    rho = float(u @ r)
    bn = float(np.linalg.norm(b))
    hist = [float(np.linalg.norm(r)) / bn]
    k = 0
    while k < maxit and hist[-1] > rtol:
        s = A @ p
        alpha = rho / float(p @ s)
        x = x + alpha * p
        r = r - alpha * s
        u = H(r)
        rho_new = float(u @ r)
        p = u + (rho_new / rho) * p
        rho = rho_new
        k += 1
        hist.append(float(np.linalg.norm(r)) / bn)
    return x, k, np.array(hist)


def sstep(A, b, H, s, rtol=1e-8, maxit=10000, fixed_outer=0):
    """Alg. 3 (with Alg. 4-6) with B^-1 = one V-cycle: the block Z is
    stored, Z(:,1) = B^-1 r and Z(:,j+1) = B^-1 A Z(:,j); the s x s part
    is the CPU oracle's (oracle.sw).  Returns (x, outer iterations, hist)."""
    A = sp.csr_matrix(A)
    n = b.size
    x = np.zeros(n)
    r = b.copy()
    bn = float(np.linalg.norm(b))
    hist = [float(np.linalg.norm(r)) / bn]
    Pold = None
    ap = np.zeros(s)
    Wp = np.zeros((s, s))
    outer_max = fixed_outer if fixed_outer else -(-maxit // s)
    k = 0
    while k < outer_max and (fixed_outer or hist[-1] > rtol):
        Z = np.zeros((s, n))
        AZ = np.zeros((s, n))
        Z[0] = H(r)                                 # Alg. 4
        for j in range(s):
            AZ[j] = A @ Z[j]
            if j + 1 < s:
                Z[j + 1] = H(AZ[j])
        vm = np.concatenate([Z @ r, Z @ AZ[s - 1]])  # Alg. 5
        if k == 0:
            W = np.array([[vm[i + j + 1] for j in range(s)] for i in range(s)])
            beta = np.zeros((s, s))
            st, alpha = oracle.spd_solve(W, vm[:s])
            if st != 0:
                break
        else:
            st, beta, W, alpha = oracle.sw(vm, ap, Wp)   # Alg. 6
            if st != 0:
                break
        if Pold is not None:                         # P = Z + P_old beta
            Z = Z + beta.T @ Pold[0]
            AZ = AZ + beta.T @ Pold[1]
        x = x + alpha @ Z
        r = r - alpha @ AZ
        Pold = (Z, AZ)
        ap, Wp = alpha, W
        k += 1
        hist.append(float(np.linalg.norm(r)) / bn)
    return x, k, np.array(hist)
