"""Pins of the variance-reduced estimate in the FP64 oracle (oracle/variance.py)
against facts from outside it: traces from the dense Laplacian, the probes'
quadratic forms from dense products, the exact trace when the probe set is
every sign vector (Hutchinson is then exact and the control variates have
their exact means), the O(t^3) residual of the Taylor control variate at small
t, and a lower mean squared error than plain SLQ over many seeds."""
import itertools

import numpy as np
import pytest

from oracle import exact, slq
from oracle import variance as OV
from paper_2003_01282_amd import inputs


def graph(csr, kind=slq.NORMALIZED, weights=None):
    return slq.build_graph(csr.n, csr.row_ptr, csr.col_idx, weights, kind)


def with_self_loop_and_isolated():
    # path 0-1-2-3 with a self-loop on 2 and two isolated nodes (4, 5)
    e = np.array([[0, 1], [1, 2], [2, 3]])
    n = 6
    r = np.r_[e[:, 0], e[:, 1], 2]
    c = np.r_[e[:, 1], e[:, 0], 2]
    return _csr(n, r, c)


def _csr(n, r, c):
    order = np.lexsort((c, r))
    r, c = r[order], c[order]
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, r + 1, 1)
    return inputs.CSR(n=n, row_ptr=np.cumsum(rp), col_idx=c.astype(np.int32))


@pytest.mark.parametrize("kind", [slq.NORMALIZED, slq.COMBINATORIAL])
@pytest.mark.parametrize("weighted", [False, True])
def test_traces_match_the_dense_laplacian(kind, weighted):
    for csr in (inputs.chung_lu(400, 1500, 2.4, seed=2), with_self_loop_and_isolated()):
        w = None
        if weighted:
            r = np.repeat(np.arange(csr.n), np.diff(csr.row_ptr))
            c = csr.col_idx.astype(np.int64)
            w = 0.5 + ((np.minimum(r, c) * 31 + np.maximum(r, c) * 7) % 13) / 6.0
        g = graph(csr, kind, w)
        L = exact.dense_laplacian(g)
        t1, t2 = OV.laplacian_traces(g)
        assert abs(t1 - np.trace(L)) <= 1e-12 * max(1.0, abs(np.trace(L)))
        assert abs(t2 - np.trace(L @ L)) <= 1e-12 * np.trace(L @ L)


@pytest.mark.parametrize("kind", [slq.NORMALIZED, slq.COMBINATORIAL])
def test_probe_moments_are_the_quadratic_forms(kind):
    csr = inputs.erdos_renyi(60, 0.08, seed=3)
    g = graph(csr, kind)
    nv = 9
    a, b, s = slq.lanczos(g, nv, 6, seed=21)
    th, w2 = slq.ritz(a, b, s)
    Z1, Z2 = OV.probe_moments(th, w2, csr.n)
    L = exact.dense_laplacian(g)
    Q = slq.rademacher(csr.n, nv, 21) / np.sqrt(csr.n)
    np.testing.assert_allclose(Z1, csr.n * np.einsum("ip,ij,jp->p", Q, L, Q), rtol=1e-11)
    LQ = L @ Q
    np.testing.assert_allclose(Z2, csr.n * np.sum(LQ * LQ, axis=0), rtol=1e-11)


def all_sign_vectors(n):
    return np.array(list(itertools.product([1.0, -1.0], repeat=n))).T  # n x 2^n


@pytest.mark.parametrize("kind", [slq.NORMALIZED, slq.COMBINATORIAL])
@pytest.mark.parametrize("mode", [OV.PLAIN, OV.TAYLOR, OV.FITTED])
def test_exact_with_every_sign_vector(kind, mode):
    # Hutchinson over all 2^n sign vectors is exact, the control variates then
    # have exactly their means, and m = n makes every Gauss rule exact: every
    # mode must return the exact trace
    csr = _csr(7, np.array([0, 1, 1, 2, 2, 3, 3, 4, 4, 0, 2, 5]), np.array([1, 0, 2, 1, 3, 2, 4, 3, 0, 4, 5, 2]))
    g = graph(csr, kind)
    V = all_sign_vectors(csr.n)
    a, b, s = slq.lanczos(g, V.shape[1], csr.n, seed=0, probes=V)
    th, w2 = slq.ritz(a, b, s)
    tr = OV.laplacian_traces(g)
    lam = exact.spectrum(g)
    t = np.array([0.05, 0.7, 3.0])
    np.testing.assert_allclose(OV.heat_trace_cv(th, w2, csr.n, t, tr, mode), exact.exact_heat(lam, t), rtol=1e-10)
    np.testing.assert_allclose(OV.wave_trace_cv(th, w2, csr.n, t, tr, mode), exact.exact_wave(lam, t),
                               rtol=1e-9, atol=1e-9)
    c = g.trace
    assert abs(OV.vnge_cv(th, w2, csr.n, c, tr, mode) - exact.exact_vnge(lam, c)) <= 1e-10


def test_taylor_control_variate_removes_the_first_two_orders():
    # heat at small t: plain SLQ's error is the Hutchinson error of
    # 1 - t tr L + t^2/2 tr L^2 - ..., first order in t; after the Taylor
    # control variate only the O(t^3) remainder's Hutchinson error is left
    csr = inputs.chung_lu(300, 1200, 2.5, seed=8)
    g = graph(csr)
    lam = exact.spectrum(g)
    a, b, s = slq.lanczos(g, 10, 20, seed=5)
    th, w2 = slq.ritz(a, b, s)
    tr = OV.laplacian_traces(g)
    for t in (1e-3, 1e-2):
        ex = exact.exact_heat(lam, [t])[0]
        e_plain = abs(OV.heat_trace_cv(th, w2, csr.n, [t], tr, OV.PLAIN)[0] - ex)
        e_tay = abs(OV.heat_trace_cv(th, w2, csr.n, [t], tr, OV.TAYLOR)[0] - ex)
        assert e_plain > 0
        assert e_tay <= 10.0 * t * t * e_plain, (t, e_plain, e_tay)
    # the plain mode is the ordinary SLQ estimate
    np.testing.assert_allclose(OV.heat_trace_cv(th, w2, csr.n, [0.3, 3.0], tr, OV.PLAIN),
                               slq.heat_trace(th, w2, csr.n, [0.3, 3.0]), rtol=1e-13)


def test_fitted_control_variates_lower_the_mean_squared_error():
    csr = inputs.chung_lu(400, 1600, 2.5, seed=4)
    g = graph(csr)
    lam = exact.spectrum(g)
    tr = OV.laplacian_traces(g)
    t = np.array([0.1, 1.0, 5.0])
    ex_h = exact.exact_heat(lam, t)
    ex_v = exact.exact_vnge(lam, g.trace)
    se = {m: np.zeros(len(t) + 1) for m in (OV.PLAIN, OV.FITTED)}
    for seed in range(30):
        a, b, s = slq.lanczos(g, 12, 15, seed=1000 + seed)
        th, w2 = slq.ritz(a, b, s)
        for m in se:
            h = OV.heat_trace_cv(th, w2, csr.n, t, tr, m)
            v = OV.vnge_cv(th, w2, csr.n, g.trace, tr, m)
            se[m] += np.r_[(h - ex_h) ** 2, (v - ex_v) ** 2]
    assert np.all(se[OV.FITTED] < se[OV.PLAIN]), (se[OV.FITTED], se[OV.PLAIN])
    # at t = 0.1 the two moments explain almost all of the probe-to-probe spread
    assert se[OV.FITTED][0] < 0.05 * se[OV.PLAIN][0]


def test_fitted_fallbacks():
    rng = np.random.default_rng(0)
    X, Z1, Z2 = rng.standard_normal((3, 2))
    assert OV.fitted_coefficients(X, Z1, Z2) == (0.0, 0.0)              # < 3 probes
    X, Z1, Z2 = rng.standard_normal((3, 3))
    g1, g2 = OV.fitted_coefficients(X, Z1, Z2)                          # 3 probes: Z1 alone
    assert g2 == 0.0 and np.isclose(g1, np.polyfit(Z1, X, 1)[0])
    X, Z1 = rng.standard_normal((2, 8))
    assert OV.fitted_coefficients(X, Z1, 2.0 * Z1)[1] == 0.0             # collinear moments
    assert OV.fitted_coefficients(X, np.ones(8), Z1) == (0.0, 0.0)      # no spread in Z1
    Z2 = rng.standard_normal(8)
    g = OV.fitted_coefficients(X, Z1, Z2)
    coef = np.linalg.lstsq(np.c_[np.ones(8), Z1, Z2], X, rcond=None)[0]
    np.testing.assert_allclose(g, coef[1:], rtol=1e-12)
