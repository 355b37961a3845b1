"""Exact rational versions of Alg. 1 (PCG-HS), Alg. 2 (PFCG) and Alg. 3-6
(s-step PCG).

TEST INFRASTRUCTURE ONLY.  Pure Python with ``fractions.Fraction`` for tiny
dense problems (n up to a few dozen): every operation is exact, so the s-step
iterate x_i must EQUAL the standard PCG iterate x_{i*s} (both minimise the
A-norm of the error over the same preconditioned Krylov space; Sec. II-A), and
both reach the exact solution after n standard steps.  With a fixed
preconditioner, PFCG's iterates equal PCG's step for step.

The matrix A and the diagonal preconditioner B are given as integer/Fraction
lists.  Index names follow the paper (1-based in comments).
"""
from __future__ import annotations

from fractions import Fraction as Fr


def _mv(A, x):
    return [sum((a * b for a, b in zip(row, x)), Fr(0)) for row in A]


def _dot(a, b):
    return sum((p * q for p, q in zip(a, b)), Fr(0))


def _binv(bdiag, v):
    return [vi / di for vi, di in zip(v, bdiag)]


def pcg(A, b, bdiag, iters):
    """Alg. 1 for exactly ``iters`` steps (or until r = 0).  Returns [x_0, x_1, ...]."""
    n = len(b)
    x = [Fr(0)] * n
    r = list(map(Fr, b))                       # r0 = b - A x0, x0 = 0
    u = _binv(bdiag, r)                        # u0 = B^{-1} r0
    p = list(u)                                # p0 = u0
    xs = [list(x)]
    ur = _dot(u, r)
    for _ in range(iters):
        if all(v == 0 for v in r):
            break
        s = _mv(A, p)                          # s_k = A p_k
        alpha = ur / _dot(p, s)
        x = [xi + alpha * pi for xi, pi in zip(x, p)]
        r = [ri - alpha * si for ri, si in zip(r, s)]
        u = _binv(bdiag, r)
        ur_new = _dot(u, r)
        beta = ur_new / ur
        p = [ui + beta * pi for ui, pi in zip(u, p)]
        ur = ur_new
        xs.append(list(x))
    return xs


def pfcg(A, b, bdiag, iters):
    """Alg. 2 for exactly ``iters`` steps in all (the one before the loop
    included; fewer if r = 0).  Returns ([x_0, x_1, ...], [p_0, p_1, ...])."""
    n = len(b)
    x = [Fr(0)] * n
    r = list(map(Fr, b))                       # r0 = b - A x0, x0 = 0
    xs, ps = [list(x)], []
    if iters < 1 or all(v == 0 for v in r):
        return xs, ps
    u = _binv(bdiag, r)                        # u0 = p0 = B^{-1} r0
    p = list(u)
    w = _mv(A, u)                              # w0 = s0 = A u0
    s = list(w)
    alpha = _dot(u, r)                         # alpha0 = u0^T r0
    rho = _dot(p, s)                           # beta0 = rho0 = p0^T s0
    x = [xi + alpha / rho * pi for xi, pi in zip(x, p)]
    r = [ri - alpha / rho * si for ri, si in zip(r, s)]
    xs.append(list(x))
    ps.append(list(p))
    for _ in range(1, iters):
        if all(v == 0 for v in r):
            break
        u = _binv(bdiag, r)                    # u_k = B^{-1} r_k
        w = _mv(A, u)                          # w_k = A u_k
        alpha = _dot(u, r)
        beta = _dot(u, w)
        gamma = _dot(u, s)                     # u_k^T s_{k-1}
        rho_k = beta - gamma * gamma / rho
        p = [ui - gamma / rho * pi for ui, pi in zip(u, p)]
        x = [xi + alpha / rho_k * pi for xi, pi in zip(x, p)]
        s = [wi - gamma / rho * si for wi, si in zip(w, s)]
        r = [ri - alpha / rho_k * si for ri, si in zip(r, s)]
        rho = rho_k
        xs.append(list(x))
        ps.append(list(p))
    return xs, ps


def _solve(M, rhs):
    """Exact Gaussian elimination (M is SPD here, no pivoting needed)."""
    s = len(M)
    a = [list(row) + [rhs[i]] for i, row in enumerate(M)]
    for c in range(s):
        piv = a[c][c]
        for i in range(c + 1, s):
            f = a[i][c] / piv
            for j in range(c, s + 1):
                a[i][j] -= f * a[c][j]
    y = [Fr(0)] * s
    for i in range(s - 1, -1, -1):
        y[i] = (a[i][s] - sum((a[i][j] * y[j] for j in range(i + 1, s)), Fr(0))) / a[i][i]
    return y


def sstep(A, b, bdiag, s, outer, b1_printed_bound=False):
    """Alg. 3 for ``outer`` outer iterations.  Returns a dict with the iterates
    x_i and, per iteration, vm, alpha, beta and W (exact).

    ``b1_printed_bound`` fills b1 only for j < i, as the printed loop bound of
    Alg. 6 reads (tests use it to show that this reading breaks the method)."""
    n = len(b)
    x = [Fr(0)] * n
    r = list(map(Fr, b))
    Pold = None                                 # P1 = 0
    xs, vms, alphas, betas, Ws = [list(x)], [], [], [], []
    alpha_prev = W_prev = None
    for k in range(outer):
        # Alg. 4: P(:,1) = B^{-1} r, then alternate A and B^{-1}
        cols = [None] * (2 * s)
        cols[0] = _binv(bdiag, r)
        pin, pout = 1, s + 1
        for j in range(2, 2 * s + 1):
            src = cols[pin - 1]
            cols[pout - 1] = _mv(A, src) if j % 2 == 0 else _binv(bdiag, src)
            pin, pout = pout, pin + 1
        # Alg. 5
        vm = [_dot(cols[c], r) for c in range(s)] + [_dot(cols[c], cols[2 * s - 1]) for c in range(s)]
        # W(i,j) = vm(i+j)
        H = [[vm[i + j + 1] for j in range(s)] for i in range(s)]
        if k == 0:
            beta = [[Fr(0)] * s for _ in range(s)]
            W = H
        else:
            # Alg. 6: moment recurrence for rhs(s..2s-1), b1(i,j) = -rhs(i+j-1)
            rhs = [Fr(0)] * (2 * s - 1)
            for i in range(1, s + 1):
                t = vm[i - 1]
                for j in range(1, i):
                    t += rhs[s - 1 + j - 1] * alpha_prev[s - i + j - 1]
                rhs[s - 1 + i - 1] = -t / alpha_prev[s - 1]
            b1 = [[-rhs[i + j] if (not b1_printed_bound or j < i) else Fr(0)
                   for j in range(s)] for i in range(s)]
            bcols = [_solve(W_prev, [b1[i][j] for i in range(s)]) for j in range(s)]
            beta = [[bcols[j][i] for j in range(s)] for i in range(s)]
            W = [[H[i][j] - sum((b1[i][q] * beta[q][j] for q in range(s)), Fr(0))
                  for j in range(s)] for i in range(s)]
        alpha = _solve(W, vm[:s])
        if Pold is not None:
            for j in range(s):
                for l in range(s):
                    if beta[l][j] != 0:
                        cols[j] = [c + po * beta[l][j] for c, po in zip(cols[j], Pold[l])]
                        cols[s + j] = [c + po * beta[l][j]
                                       for c, po in zip(cols[s + j], Pold[s + l])]
        for j in range(s):
            x = [xi + cj * alpha[j] for xi, cj in zip(x, cols[j])]
            r = [ri - cj * alpha[j] for ri, cj in zip(r, cols[s + j])]
        Pold = cols
        alpha_prev, W_prev = alpha, W
        xs.append(list(x))
        vms.append(vm)
        alphas.append(alpha)
        betas.append(beta)
        Ws.append(W)
        if all(v == 0 for v in r):
            break
    return dict(x=xs, vm=vms, alpha=alphas, beta=betas, W=Ws)


def sstep_cheb(A, b, bdiag, s, outer, lo, hi, ap_conj_sign=1):
    """Alg. 3 on a Chebyshev basis with the block Gram product taken directly
    (the stabilised-basis variant; see ``orc_sstep_cheb``), exactly, for
    ``outer`` outer iterations.  [lo, hi] (Fractions) encloses the spectrum of
    K = B^-1 A: z_1 = B^-1 r, z_2 = (K - c) z_1 / h,
    z_{j+1} = 2 (K - c) z_j / h - z_{j-1}, c = (hi + lo)/2, h = (hi - lo)/2.
    With C = P_{i-1}^T A Z_i: W_{i-1} beta = -C, W_i = Z^T A Z + C^T beta,
    W_i alpha = Z^T r.  Returns a dict with the iterates and, per iteration,
    alpha, beta, W and the block [P_i | A P_i].

    ``ap_conj_sign`` = -1 flips the sign of the conjugation coefficients
    (tests use it to show that the pins catch such a slip)."""
    n = len(b)
    lo, hi = Fr(lo), Fr(hi)
    c, h = (hi + lo) / 2, (hi - lo) / 2
    x = [Fr(0)] * n
    r = list(map(Fr, b))
    Pold = None
    W_prev = None
    xs, alphas, betas, Ws, blocks = [list(x)], [], [], [], []
    for k in range(outer):
        Z = [_binv(bdiag, r)]
        AZ = []
        for j in range(s):
            AZ.append(_mv(A, Z[j]))
            if j + 1 == s:
                break
            Kz = _binv(bdiag, AZ[j])
            u = [t - c * zz for t, zz in zip(Kz, Z[j])]
            if j == 0:
                Z.append([v / h for v in u])
            else:
                Z.append([2 * v / h - zm for v, zm in zip(u, Z[j - 1])])
        ZAZ = [[_dot(Z[a], AZ[q]) for q in range(s)] for a in range(s)]
        m = [_dot(Z[a], r) for a in range(s)]
        if k == 0:
            beta = [[Fr(0)] * s for _ in range(s)]
            W = ZAZ
        else:
            Cm = [[_dot(Pold[s + l], Z[j]) for j in range(s)] for l in range(s)]
            bcols = [_solve(W_prev, [-ap_conj_sign * Cm[i][j] for i in range(s)])
                     for j in range(s)]
            beta = [[bcols[j][i] for j in range(s)] for i in range(s)]
            W = [[ZAZ[i][j] + sum((Cm[l][i] * beta[l][j] for l in range(s)), Fr(0))
                  for j in range(s)] for i in range(s)]
        alpha = _solve(W, m)
        cols = [list(v) for v in Z] + [list(v) for v in AZ]
        if Pold is not None:
            for j in range(s):
                for l in range(s):
                    if beta[l][j] != 0:
                        cols[j] = [cc + po * beta[l][j] for cc, po in zip(cols[j], Pold[l])]
                        cols[s + j] = [cc + po * beta[l][j]
                                       for cc, po in zip(cols[s + j], Pold[s + l])]
        for j in range(s):
            x = [xi + cj * alpha[j] for xi, cj in zip(x, cols[j])]
            r = [ri - cj * alpha[j] for ri, cj in zip(r, cols[s + j])]
        Pold = cols
        W_prev = W
        xs.append(list(x))
        alphas.append(alpha)
        betas.append(beta)
        Ws.append(W)
        blocks.append(cols)
        if all(v == 0 for v in r):
            break
    return dict(x=xs, alpha=alphas, beta=betas, W=Ws, P=blocks)
