"""Exact (O(n^3)) route for tiny graphs: test-only ground truth.

The paper's "exact" baseline computes every eigenvalue and sums f(lambda_i)
(§2.3).  Brute-force Hutchinson evaluates v^T f(L) v with a dense f(L) on the
same probes as SLQ (§3.1, eq. "trace"), so it isolates the Lanczos/Gauss error
from the Monte-Carlo error.
"""
import numpy as np

from .slq import NORMALIZED, Graph, rademacher, xlogx


def dense_laplacian(g: Graph):
    """Dense L (§2): I - D^-1/2 A D^-1/2 with zero rows/columns for isolated
    nodes, or D - A."""
    A = g.A.toarray()
    if g.kind == NORMALIZED:
        S = g.dinv[:, None] * A * g.dinv[None, :]
        return np.diag((g.deg > 0).astype(np.float64)) - S
    return np.diag(g.deg) - A


def spectrum(g: Graph):
    return np.linalg.eigvalsh(dense_laplacian(g))


def exact_heat(lam, t):
    return np.array([np.sum(np.exp(-tt * lam)) for tt in np.atleast_1d(t)])


def exact_wave(lam, t):
    return np.array([np.sum(np.cos(tt * lam)) for tt in np.atleast_1d(t)])


def exact_vnge(lam, trace):
    return -float(np.sum(xlogx(lam / trace)))


def matrix_function(g: Graph, f):
    """f(L) = Phi f(Lambda) Phi^T (§2.2, eq. "heat-solution")."""
    lam, Phi = np.linalg.eigh(dense_laplacian(g))
    return (Phi * f(lam)[None, :]) @ Phi.T


def hutchinson(g: Graph, nv, seed, f, probes=None):
    """(n/nv) sum_p q_p^T f(L) q_p with q_p = v_p/sqrt(n): Hutchinson on the
    same probes SLQ uses (for Rademacher v this is (1/nv) sum v^T f(L) v)."""
    V = rademacher(g.n, nv, seed) if probes is None else probes
    F = matrix_function(g, f)
    Q = V / np.sqrt(g.n)
    per_probe = np.einsum("ip,ij,jp->p", Q, F, Q)
    return (g.n / V.shape[1]) * float(per_probe.sum()), per_probe
