"""FP64 oracle of the SLaQ estimator (test infrastructure, never the product path).

The method (paper §3, Algorithm 1): for a graph Laplacian L and a spectral
function f, estimate tr f(L) by Hutchinson's estimator over nv random probes
(§3.1, eq. "trace"), each quadratic form by the m-point Gauss rule that s-step
Lanczos builds (§3.1, eq. "quadratic"), giving the SLQ estimate Gamma
(eq. "slq").  NetLSD is the heat trace sum_i exp(-t lambda_i) (§2.2, eq.
"heat-trace"); VNGE is -sum_i lambda_i ln lambda_i of the density matrix
L / tr(L) (§2.1, Definition).

Readings where the paper is silent or inconsistent (each is repeated where used):
  * isolated nodes: the normalized Laplacian's row and column are zero (Chung's
    convention), so they add eigenvalue 0;
  * Hutchinson factor n/nv with unit-norm start q1 = v/sqrt(n) (eq. "trace",
    eq. "slq"); Algorithm 1's bare 1/nv drops the n;
  * VNGE carries the minus sign of the Definition; 0 ln 0 = 0, and a Ritz value
    <= 0 from rounding contributes 0;
  * probes are Rademacher, drawn from SplitMix64 keyed on (seed, node, probe);
  * Lanczos order: w = L q_j - beta_{j-1} q_{j-1}; alpha_j = q_j.w;
    w -= alpha_j q_j; beta_j = ||w|| (the three-term recurrence of §3.1);
  * breakdown: stop when beta_j <= eps_bd * S with S the spectral bound of §2
    (2 for the normalized Laplacian, 2 max_i D_ii for the combinatorial one).
"""
import warnings
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

NORMALIZED = 0
COMBINATORIAL = 1

EPS_BREAKDOWN = 1e-6


# --------------------------------------------------------------------------
# Graph quantities (§2: A symmetric with positive weights, D_ii = sum_j A_ij,
# L = D - A, normalized L = I - D^-1/2 A D^-1/2)
# --------------------------------------------------------------------------
@dataclass
class Graph:
    n: int
    A: object                 # symmetric adjacency: scipy CSR, or torch CPU CSR (large graphs), float64
    deg: np.ndarray           # D_ii, float64[n]
    dinv: np.ndarray          # D_ii^-1/2, 0 for isolated nodes
    kind: int
    self_w: np.ndarray = None  # A_ii (self-loop weights), float64[n]

    @property
    def trace(self):
        """tr(L), the sum of the Laplacian's diagonal (§2): L_ii = 1 - A_ii / D_ii
        on a non-isolated node of the normalized Laplacian (0 on an isolated
        one), L_ii = D_ii - A_ii for L = D - A.  Without self-loops this is the
        number of non-isolated nodes, or sum_i D_ii."""
        a = np.zeros(self.n) if self.self_w is None else self.self_w
        if self.kind == NORMALIZED:
            pos = self.deg > 0
            return float(np.sum(1.0 - a[pos] / self.deg[pos]))
        return float(np.sum(self.deg - a))

    @property
    def n_isolated(self):
        return int(np.count_nonzero(self.deg == 0))

    @property
    def spectral_bound(self):
        """Upper end of the spectrum (§2, Gershgorin): 2, or 2 max_i D_ii."""
        if self.kind == NORMALIZED:
            return 2.0
        return 2.0 * float(self.deg.max()) if self.n else 0.0


def _row_sums(n, row_ptr, col_idx, w, chunk=1 << 22):
    """D_ii = sum_j A_ij and A_ii of a CSR, rows taken in chunks (no n x n or
    nnz-sized index arrays at once)."""
    deg = np.zeros(n)
    diag = np.zeros(n)
    for r0 in range(0, n, chunk):
        r1 = min(n, r0 + chunk)
        k0, k1 = int(row_ptr[r0]), int(row_ptr[r1])
        rows = np.repeat(np.arange(r0, r1, dtype=np.int64), np.diff(row_ptr[r0:r1 + 1]))
        ww = np.ones(k1 - k0) if w is None else np.asarray(w[k0:k1], dtype=np.float64)
        deg[r0:r1] = np.bincount(rows - r0, weights=ww, minlength=r1 - r0)
        on = np.asarray(col_idx[k0:k1], dtype=np.int64) == rows
        diag[r0:r1] = np.bincount(rows[on] - r0, weights=ww[on], minlength=r1 - r0)
    return deg, diag


def build_graph(n, row_ptr, col_idx, weights=None, kind=NORMALIZED, backend="scipy"):
    """CSR (row_ptr[n+1], col_idx[nnz], optional positive weights) -> Graph.

    Degrees follow §2: D_ii = sum_j A_ij (self-loops are taken literally).
    backend "scipy" keeps A as a scipy CSR matrix; "torch" as a torch CPU CSR
    tensor (int32 indices when nnz < 2^31), whose matrix product uses every
    host core -- for graphs of billions of entries.  The arithmetic is the same
    (an FP64 product of A with a block)."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    nnz = int(row_ptr[-1])
    if backend == "scipy":
        col_idx = np.asarray(col_idx, dtype=np.int64)
        w = np.ones(nnz) if weights is None else np.asarray(weights, dtype=np.float64)
        A = sp.csr_matrix((w, col_idx, row_ptr), shape=(n, n))
        deg = np.asarray(A.sum(axis=1)).ravel()
        self_w = np.asarray(A.diagonal(), dtype=np.float64)
    elif backend == "torch":
        import torch
        deg, self_w = _row_sums(n, row_ptr, col_idx, weights)
        it = torch.int32 if nnz < 2**31 - 1 else torch.int64
        vals = (torch.ones(nnz, dtype=torch.float64) if weights is None
                else torch.from_numpy(np.asarray(weights, dtype=np.float64)))
        with warnings.catch_warnings():
            warnings.simplefilter("ignore")  # torch marks its CSR layout as beta
            A = torch.sparse_csr_tensor(torch.from_numpy(row_ptr).to(it),
                                        torch.from_numpy(np.asarray(col_idx)).to(it), vals, size=(n, n))
    else:
        raise ValueError(f"unknown backend {backend}")
    dinv = np.zeros(n)
    pos = deg > 0
    dinv[pos] = 1.0 / np.sqrt(deg[pos])
    return Graph(n=n, A=A, deg=deg, dinv=dinv, kind=kind, self_w=self_w)


def _product(A, X):
    """A X for the adjacency A (scipy or torch CSR) and a dense FP64 block X."""
    if sp.issparse(A):
        return A @ X
    import torch
    return (A @ torch.from_numpy(np.ascontiguousarray(X))).numpy()


def apply_laplacian(g, X):
    """Y = L X for a block X (n x k).

    Normalized (§2): Y = X - D^-1/2 A D^-1/2 X, except that rows of isolated
    nodes are 0 (the reading above).  Combinatorial: Y = D X - A X."""
    X = np.asarray(X, dtype=np.float64)
    if g.kind == NORMALIZED:
        nonisolated = (g.deg > 0).astype(np.float64)
        scaled = g.dinv[:, None] * X
        return nonisolated[:, None] * X - g.dinv[:, None] * _product(g.A, scaled)
    return g.deg[:, None] * X - _product(g.A, X)


# --------------------------------------------------------------------------
# Probes (§3.1: zero-mean, unit-variance random vectors; Rademacher chosen)
# --------------------------------------------------------------------------
_MASK = (1 << 64) - 1
GOLDEN_GAMMA = 0x9E3779B97F4A7C15


def splitmix64(seed, counter):
    """Output number counter+1 of SplitMix64 seeded with `seed` (Steele, Lea and
    Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014, with
    the 64-bit finalizer of Java's SplittableRandom).  Vectorized over
    `counter` (uint64 numpy array); all arithmetic is modulo 2^64."""
    c = np.asarray(counter, dtype=np.uint64)
    z = (np.uint64(seed & _MASK) + (c + np.uint64(1)) * np.uint64(GOLDEN_GAMMA))
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def rademacher(n, nv, seed, node_ids=None, columns=None):
    """Probe block V (n x nv) with entries +-1.

    Entry (i, p) is bit (p mod 64) of splitmix64(seed, 64*i + p div 64): a set
    bit gives -1.  Keys use the node id, so a probe does not depend on how the
    rows are stored.  `node_ids` selects rows (default all); `columns` selects
    probes (default 0..nv-1), e.g. a few probes of a very large graph."""
    if nv > 4096:
        raise ValueError("nv > 4096")
    ids = np.arange(n, dtype=np.uint64) if node_ids is None else np.asarray(node_ids, dtype=np.uint64)
    cols = np.arange(nv) if columns is None else np.asarray(columns, dtype=np.int64)
    V = np.empty((ids.size, cols.size))
    for word in np.unique(cols // 64):
        z = splitmix64(seed, ids * np.uint64(64) + np.uint64(word))
        for k in np.flatnonzero(cols // 64 == word):
            bit = (z >> np.uint64(int(cols[k]) % 64)) & np.uint64(1)
            V[:, k] = 1.0 - 2.0 * bit.astype(np.float64)
    return V


# --------------------------------------------------------------------------
# Lanczos (§3.1: s-step Lanczos, Q^T L Q = T tridiagonal, three-term recurrence)
# --------------------------------------------------------------------------
def lanczos(g, nv, m, seed, eps_bd=EPS_BREAKDOWN, probes=None):
    """m Lanczos steps per probe, all probes as columns of one block.

    Start vector q1 = v_p / sqrt(n) (unit norm, §3.1 "starting unit-vector").
    No reorthogonalization.  Returns alpha[nv, m], beta[nv, m] (beta_j couples
    q_j and q_{j+1}; beta of the last step is kept) and steps[nv] (< m when the
    Krylov space became invariant; entries past it are 0).
    `probes` lets a caller pass the +-1 block directly (n x nv)."""
    n = g.n
    V = rademacher(n, nv, seed) if probes is None else np.asarray(probes, dtype=np.float64)
    nv = V.shape[1]
    q = V / np.sqrt(n)
    q_prev = np.zeros_like(q)
    beta_prev = np.zeros(nv)
    alpha = np.zeros((nv, m))
    beta = np.zeros((nv, m))
    steps = np.full(nv, m, dtype=np.int32)
    active = np.ones(nv, dtype=bool)
    threshold = eps_bd * g.spectral_bound
    for j in range(m):
        w = apply_laplacian(g, q) - beta_prev[None, :] * q_prev
        a = np.sum(q * w, axis=0)
        w = w - a[None, :] * q
        b = np.sqrt(np.sum(w * w, axis=0))
        alpha[active, j] = a[active]
        beta[active, j] = b[active]
        stop = active & (b <= threshold) & (j < m - 1)
        steps[stop] = j + 1
        active = active & ~stop
        safe_b = np.where(active, b, 1.0)
        q_prev, q = q, np.where(active[None, :], w / safe_b[None, :], 0.0)
        beta_prev = np.where(active, b, 0.0)
    return alpha, beta, steps


# --------------------------------------------------------------------------
# Gauss rule (§3.1, eq. "quadratic": nodes = eigenvalues of T, weights = the
# squared first components of its normalized eigenvectors)
# --------------------------------------------------------------------------
def tridiagonal(alpha_p, beta_p, k):
    """Dense k x k Jacobi matrix T from alpha_1..k and beta_1..k-1."""
    T = np.diag(np.asarray(alpha_p[:k], dtype=np.float64))
    if k > 1:
        off = np.asarray(beta_p[: k - 1], dtype=np.float64)
        T += np.diag(off, 1) + np.diag(off, -1)
    return T


def ritz(alpha, beta, steps):
    """theta[nv, m], tau2[nv, m]: Gauss nodes and weights per probe.
    Columns past steps[p] hold theta = 0, tau2 = 0 (they add nothing)."""
    nv, m = alpha.shape
    theta = np.zeros((nv, m))
    tau2 = np.zeros((nv, m))
    for p in range(nv):
        k = int(steps[p])
        lam, U = np.linalg.eigh(tridiagonal(alpha[p], beta[p], k))
        theta[p, :k] = lam
        tau2[p, :k] = U[0, :] ** 2
    return theta, tau2


# --------------------------------------------------------------------------
# Quadrature: Gamma = n/nv sum_p sum_k tau2 f(theta)  (§3.1, eq. "slq")
# --------------------------------------------------------------------------
def t_grid(nt=256, lo=-2.0, hi=2.0):
    """Log-spaced time scales t_k = 10^(lo + (hi-lo) k/(nt-1)) (§2.2: a small
    logarithmically spaced grid; the endpoints 1e-2 and 1e2 are the workload's)."""
    k = np.arange(nt, dtype=np.float64)
    return 10.0 ** (lo + (hi - lo) * k / max(nt - 1, 1))


def quadrature(theta, tau2, n, f):
    """Gamma = (n / nv) sum_p sum_k tau2[p,k] f(theta[p,k])."""
    nv = theta.shape[0]
    return (n / nv) * float(np.sum(tau2 * f(theta)))


def heat_trace(theta, tau2, n, t):
    """h_t = tr exp(-t L) (§2.2, eq. "heat-trace") at every t."""
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    return np.array([quadrature(theta, tau2, n, lambda x, tt=tt: np.exp(-tt * x)) for tt in t])


def wave_trace(theta, tau2, n, t):
    """w_t = Re tr exp(-i t L) = sum_i cos(t lambda_i).  The paper defines only
    the heat trace; the wave trace is its oscillatory counterpart (reading)."""
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    return np.array([quadrature(theta, tau2, n, lambda x, tt=tt: np.cos(tt * x)) for tt in t])


def xlogx(x):
    """g(x) = x ln x for x > 0, else 0 (0 ln 0 = 0 by the convention of §2.1;
    non-positive Ritz values only arise from rounding)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    pos = x > 0
    out[pos] = x[pos] * np.log(x[pos])
    return out


def vnge(theta, tau2, n, trace):
    """H = -tr g(L / tr L) (§2.1 Definition on the density matrix L / tr(L);
    Algorithm 1 applies slq to that matrix).  The minus sign follows the
    Definition (Algorithm 1 omits it).  A graph without edges has L = 0 and no
    density matrix; its entropy is taken as 0."""
    if trace <= 0:
        return 0.0
    return -quadrature(theta, tau2, n, lambda x: xlogx(x / trace))


# --------------------------------------------------------------------------
# Algorithm 1 entry points
# --------------------------------------------------------------------------
def slaq_lsd(g, nv, m, seed, t, wave=False):
    """SLaQ_LSD: heat (or wave) trace signature at every t (Algorithm 1)."""
    a, b, s = lanczos(g, nv, m, seed)
    th, w2 = ritz(a, b, s)
    return wave_trace(th, w2, g.n, t) if wave else heat_trace(th, w2, g.n, t)


def slaq_vnge(g, nv, m, seed):
    """SLaQ_VNGE (Algorithm 1)."""
    a, b, s = lanczos(g, nv, m, seed)
    th, w2 = ritz(a, b, s)
    return vnge(th, w2, g.n, g.trace)
