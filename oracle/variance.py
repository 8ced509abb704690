"""FP64 oracle of the variance-reduced trace estimate (test infrastructure).

Paper §3.1 closes with one sentence: the Monte Carlo trace estimate is
improved by a "2-term polynomial variance reduction".  Reading (the paper
gives no formula): the two terms are control variates whose exact means the
graph gives in O(nnz),

    Z1_p = n q_p^T L q_p     with mean tr L,
    Z2_p = n q_p^T L^2 q_p   with mean tr L^2 = ||L||_F^2 (L symmetric),

for the unit start vectors q_p = v_p / sqrt(n).  The m-point Gauss rule of
probe p integrates polynomials up to degree 2m - 1 exactly, so for m >= 2
Z1_p = n sum_k tau2 theta and Z2_p = n sum_k tau2 theta^2 come with the
probe's Ritz pairs.  With X_p = n sum_k tau2 f(theta) (plain SLQ is mean X)
the estimate is

    mean(X) - g1 (mean(Z1) - tr L) - g2 (mean(Z2) - tr L^2),

unbiased for fixed (g1, g2).  Two choices of the coefficients:
  * "taylor": the degree-2 Taylor polynomial of f at 0 that the paper's own
    Taylor baselines expand (§2.2 for the heat kernel: 1 - t x + t^2 x^2 / 2),
    i.e. g = (-t, t^2/2) for the heat trace and (0, -t^2/2) for the wave
    trace; for VNGE the quadratic -x ln x ~ x - x^2 of the FINGER expansion
    (§2.1's Taylor form) on x = lambda / tr L, i.e. g = (1/c, -1/c^2);
  * "fitted": the least-squares regression of X on (Z1, Z2) over the probes
    (the optimal control-variate coefficients, estimated; bias O(1/nv)).
Fallbacks of "fitted" (both implementations): fewer than 3 probes, or no
spread in Z1 -> plain; 3 probes, no spread in Z2, or a 2x2 system with
det <= 1e-10 S11 S22 -> Z1 alone.
"""
import numpy as np
import scipy.sparse as sp

from .slq import NORMALIZED, xlogx

PLAIN, TAYLOR, FITTED = 0, 1, 2


def laplacian_matrix(g):
    """Sparse L (§2): normalized I - D^-1/2 A D^-1/2 with zero rows/columns for
    isolated nodes (Chung's convention), or D - A."""
    if g.kind == NORMALIZED:
        Dh = sp.diags(g.dinv)
        return (sp.diags((g.deg > 0).astype(np.float64)) - Dh @ g.A @ Dh).tocsr()
    return (sp.diags(g.deg) - g.A).tocsr()


def laplacian_traces(g):
    """(tr L, tr L^2); tr L^2 = sum of squares of L's entries since L = L^T."""
    L = laplacian_matrix(g)
    return float(L.diagonal().sum()), float(L.multiply(L).sum())


def probe_moments(theta, tau2, n):
    """Z1_p = n sum_k tau2 theta, Z2_p = n sum_k tau2 theta^2 (Gauss rule)."""
    return n * np.sum(tau2 * theta, axis=1), n * np.sum(tau2 * theta * theta, axis=1)


def fitted_coefficients(X, Z1, Z2):
    """Least-squares (g1, g2) of X on (Z1, Z2) with an intercept, from the
    centered sums, with the fallbacks stated in the module docstring."""
    nv = X.size
    if nv < 3:
        return 0.0, 0.0
    x = X - X.mean()
    z1 = Z1 - Z1.mean()
    z2 = Z2 - Z2.mean()
    s11, s22, s12 = float(z1 @ z1), float(z2 @ z2), float(z1 @ z2)
    s1x, s2x = float(z1 @ x), float(z2 @ x)
    if not s11 > 0.0:
        return 0.0, 0.0
    det = s11 * s22 - s12 * s12
    if nv >= 4 and s22 > 0.0 and det > 1e-10 * s11 * s22:
        return (s22 * s1x - s12 * s2x) / det, (s11 * s2x - s12 * s1x) / det
    return s1x / s11, 0.0


def cv_estimate(X, Z1, Z2, traces, gamma):
    """mean(X) - g1 (mean(Z1) - tr L) - g2 (mean(Z2) - tr L^2)."""
    g1, g2 = gamma
    return float(X.mean() - g1 * (Z1.mean() - traces[0]) - g2 * (Z2.mean() - traces[1]))


def _signature_cv(theta, tau2, n, t, traces, mode, f, taylor):
    Z1, Z2 = probe_moments(theta, tau2, n)
    out = []
    for tt in np.atleast_1d(np.asarray(t, dtype=np.float64)):
        X = n * np.sum(tau2 * f(tt, theta), axis=1)
        if mode == PLAIN:
            gamma = (0.0, 0.0)
        elif mode == TAYLOR:
            gamma = taylor(tt)
        else:
            gamma = fitted_coefficients(X, Z1, Z2)
        out.append(cv_estimate(X, Z1, Z2, traces, gamma))
    return np.array(out)


def heat_trace_cv(theta, tau2, n, t, traces, mode):
    """Variance-reduced h_t = tr exp(-t L) at every t."""
    return _signature_cv(theta, tau2, n, t, traces, mode, lambda tt, x: np.exp(-tt * x),
                         lambda tt: (-tt, 0.5 * tt * tt))


def wave_trace_cv(theta, tau2, n, t, traces, mode):
    """Variance-reduced w_t = sum_i cos(t lambda_i) at every t."""
    return _signature_cv(theta, tau2, n, t, traces, mode, lambda tt, x: np.cos(tt * x),
                         lambda tt: (0.0, -0.5 * tt * tt))


def vnge_cv(theta, tau2, n, trace, traces, mode):
    """Variance-reduced H = -tr g(L / c), c = tr L (the graph's trace)."""
    if trace <= 0:
        return 0.0
    c = float(trace)
    Z1, Z2 = probe_moments(theta, tau2, n)
    X = -n * np.sum(tau2 * xlogx(theta / c), axis=1)
    if mode == PLAIN:
        gamma = (0.0, 0.0)
    elif mode == TAYLOR:
        gamma = (1.0 / c, -1.0 / (c * c))
    else:
        gamma = fitted_coefficients(X, Z1, Z2)
    return cv_estimate(X, Z1, Z2, traces, gamma)
