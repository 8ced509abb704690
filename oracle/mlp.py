"""FP64 reference of the learned closure network (test infrastructure).

The paper has no learned component; this is the reference for the closure's
BF16 kernels.  The network maps per-probe features to a per-time correction
of the log Gauss value:
    x (d_in) -> SiLU(x W1 + b1) -> SiLU(. W2 + b2) -> SiLU(. W3 + b3) -> . W4 + b4
with SiLU(z) = z / (1 + exp(-z)) and loss L = mean over batch and outputs of
(y_hat - y)^2.  Weights are (d_in x d_out) matrices, activations are rows.

Also here: the features and targets the closure is trained on, computed from
the Gauss rule of §3.1 (eq. "quadratic"): for probe p with m-step nodes and
weights, Q_m(t) = sum_k tau2_k exp(-t theta_k), features are the first five
nodes (ascending) and their weights, the target is log Q_30(t) - log Q_5(t).
"""
import numpy as np


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(params, X):
    """params: list of (W, b); returns (Y, cache)."""
    H = np.asarray(X, dtype=np.float64)
    cache = []
    for li, (W, b) in enumerate(params):
        Z = H @ W + b
        cache.append((H, Z))
        H = Z if li == len(params) - 1 else silu(Z)
    return H, cache


def loss_and_grads(params, X, Y):
    """MSE loss and its gradients with respect to every W and b."""
    Yh, cache = forward(params, X)
    B, N = Yh.shape
    loss = float(np.mean((Yh - Y) ** 2))
    dY = 2.0 * (Yh - Y) / (B * N)
    grads = [None] * len(params)
    d = dY
    for li in range(len(params) - 1, -1, -1):
        Hin, Z = cache[li]
        if li != len(params) - 1:
            d = d * dsilu(Z)
        W, _ = params[li]
        grads[li] = (Hin.T @ d, d.sum(axis=0))
        d = d @ W.T
    return loss, grads


def gauss_values(theta, tau2, t):
    """Q(t) = sum_k tau2_k exp(-t theta_k) per probe: [P, nt]."""
    t = np.asarray(t, dtype=np.float64)
    return np.einsum("pk,pkt->pt", tau2, np.exp(-theta[:, :, None] * t[None, None, :]))


def features(theta, tau2, steps, m_feat=5):
    """First m_feat Gauss nodes of each probe sorted ascending, then their
    weights; nodes past the probe's step count are 0 with weight 0."""
    P = theta.shape[0]
    F = np.zeros((P, 2 * m_feat))
    for p in range(P):
        k = min(int(steps[p]), m_feat)
        o = np.argsort(theta[p, :k], kind="stable")
        F[p, :k] = theta[p, :k][o]
        F[p, m_feat:m_feat + k] = tau2[p, :k][o]
    return F


def targets(theta5, tau25, theta30, tau230, t):
    """log Q_30(t) - log Q_5(t) per probe and time."""
    return np.log(gauss_values(theta30, tau230, t)) - np.log(gauss_values(theta5, tau25, t))
