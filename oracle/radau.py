"""Gauss-Radau companion of the Lanczos Gauss rule (test infrastructure).

For f(x) = exp(-t x) every even-order derivative is positive and every odd-order
one negative.  The Gauss rule built by Lanczos (§3.1, eq. "quadratic"; Golub and
Welsch) therefore underestimates each quadratic form q^T f(L) q, and the
Gauss-Radau rule with one node fixed at a <= lambda_min overestimates it (the
error term of a Radau rule has the sign of f^(2k+1) times a non-negative
integral; Golub and Meurant, "Matrices, Moments and Quadrature", 2010).  The
pair brackets the exact value.  The paper cites the Gauss rule only; the
bracket is used to gate the learned closure.

The (k+1)-point Radau rule comes from the Jacobi matrix T_k extended by one row:
    T~ = [[T_k, beta_k e_k], [beta_k e_k^T, phi]],  phi = a + delta_k,
with delta the solution of (T_k - a I) delta = beta_k^2 e_k; then a is an
eigenvalue of T~ and its eigenpairs give nodes and weights as in the Gauss case.
"""
import numpy as np

from .slq import tridiagonal


def radau_rule(alpha_p, beta_p, k, a=0.0):
    """Nodes and weights of the (k+1)-point Gauss-Radau rule with node a."""
    T = tridiagonal(alpha_p, beta_p, k)
    bk = float(beta_p[k - 1])
    rhs = np.zeros(k)
    rhs[-1] = bk * bk
    delta = np.linalg.solve(T - a * np.eye(k), rhs)
    Tx = np.zeros((k + 1, k + 1))
    Tx[:k, :k] = T
    Tx[k - 1, k] = Tx[k, k - 1] = bk
    Tx[k, k] = a + delta[-1]
    lam, U = np.linalg.eigh(Tx)
    return lam, U[0, :] ** 2


def heat_bracket(alpha, beta, steps, t, a=0.0):
    """Per-probe Gauss (lower) and Radau (upper) values of q^T exp(-tL) q.

    Returns two arrays [nv, nt].  A probe whose Krylov space became invariant
    (steps < m) has an exact Gauss rule; its Radau value is set equal to it."""
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    nv = alpha.shape[0]
    lo = np.zeros((nv, t.size))
    hi = np.zeros((nv, t.size))
    m = alpha.shape[1]
    for p in range(nv):
        k = int(steps[p])
        lam, U = np.linalg.eigh(tridiagonal(alpha[p], beta[p], k))
        g = (U[0, :] ** 2)[None, :] * np.exp(-t[:, None] * lam[None, :])
        lo[p] = g.sum(axis=1)
        if k < m:
            hi[p] = lo[p]
        else:
            rl, rw = radau_rule(alpha[p], beta[p], k, a)
            hi[p] = (rw[None, :] * np.exp(-t[:, None] * rl[None, :])).sum(axis=1)
    return lo, hi
