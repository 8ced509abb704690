"""Pins of the closure's FP64 reference: gradients against central finite
differences, SiLU against its definition, features/targets against the Gauss
rule of the oracle."""
import numpy as np

from oracle import mlp, slq
from paper_2003_01282_amd import inputs


def small_net(rng, dims=(6, 9, 7, 5, 4)):
    return [(rng.standard_normal((a, b)) * 0.5, rng.standard_normal(b) * 0.1) for a, b in zip(dims[:-1], dims[1:])]


def test_silu_and_derivative():
    z = np.linspace(-6, 6, 101)
    assert np.allclose(mlp.silu(z), z * (1 / (1 + np.exp(-z))))
    h = 1e-6
    fd = (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h)
    assert np.allclose(mlp.dsilu(z), fd, atol=1e-8)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(0)
    params = small_net(rng)
    X = rng.standard_normal((11, 6))
    Y = rng.standard_normal((11, 4))
    _, grads = mlp.loss_and_grads(params, X, Y)
    h = 1e-6
    for li, (W, b) in enumerate(params):
        for arr, g in ((W, grads[li][0]), (b, grads[li][1])):
            flat = arr.reshape(-1)
            for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
                old = flat[idx]
                flat[idx] = old + h
                lp = mlp.loss_and_grads(params, X, Y)[0]
                flat[idx] = old - h
                lm = mlp.loss_and_grads(params, X, Y)[0]
                flat[idx] = old
                fd = (lp - lm) / (2 * h)
                assert abs(g.reshape(-1)[idx] - fd) <= 1e-6 * max(1.0, abs(fd)), (li, idx)


def test_features_and_targets_follow_the_gauss_rule():
    csr = inputs.chung_lu(800, 3000, 2.5, seed=2)
    g = slq.build_graph(csr.n, csr.row_ptr, csr.col_idx)
    a, b, s = slq.lanczos(g, 6, 30, seed=3)
    t = slq.t_grid(16)
    th30, w30 = slq.ritz(a, b, s)
    th5, w5 = slq.ritz(a[:, :5], b[:, :5], np.minimum(s, 5))
    F = mlp.features(th5, w5, np.minimum(s, 5))
    assert np.all(np.diff(F[:, :5], axis=1) >= 0)
    assert np.allclose(F[:, 5:].sum(axis=1), 1.0)
    Y = mlp.targets(th5, w5, th30, w30, t)
    # Gauss monotonicity for exp(-tx): Q_30 >= Q_5, so the target is >= 0
    assert np.all(Y >= -1e-12)
    # at t -> 0 both rules integrate 1 exactly
    assert np.allclose(mlp.targets(th5, w5, th30, w30, [0.0]), 0.0, atol=1e-14)
    # the per-probe Gauss values reproduce the heat trace
    Q = mlp.gauss_values(th30, w30, t)
    assert np.allclose(csr.n / 6 * Q.sum(axis=0), slq.heat_trace(th30, w30, csr.n, t))
