"""Pins of the FP64 oracle against facts that do not come from the oracle itself:
published test vectors, closed-form spectra, the paper's worked example
(Figure 1), the exact route by dense eigendecomposition, brute-force Hutchinson
on the same probes, quadrature invariants and the paper's Lanczos error bound.
"""
import math
from pathlib import Path

import numpy as np
import pytest

from oracle import exact, radau, slq
from paper_2003_01282_amd import inputs

GOLDEN = Path(__file__).parent / "golden"


def load_fig1(name):
    rows = [ln.split() for ln in (GOLDEN / f"{name}_edges.txt").read_text().splitlines()
            if ln and not ln.startswith("#")]
    e = np.array(rows, dtype=np.int64)
    n = {"karate": 34, "dolphins": 62}[name]
    return inputs.from_edges(n, e)


def graph(csr, kind=slq.NORMALIZED, weights=None):
    return slq.build_graph(csr.n, csr.row_ptr, csr.col_idx, weights, kind)


# ---------------------------------------------------------------- probes ----
def test_splitmix64_published_vectors():
    # first outputs of SplitMix64 for seeds 0 and 1234567 (reference
    # implementation by Vigna, splitmix64.c)
    z0 = slq.splitmix64(0, np.arange(3, dtype=np.uint64))
    assert [int(x) for x in z0] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    z1 = slq.splitmix64(1234567, np.arange(3, dtype=np.uint64))
    assert [int(x) for x in z1] == [6457827717110365317, 3203168211198807973, 9817491932198370423]


def test_rademacher_statistics_and_prefix():
    V = slq.rademacher(4000, 130, seed=7)
    assert set(np.unique(V)) == {-1.0, 1.0}
    assert abs(V.mean()) < 4 / math.sqrt(V.size)
    C = (V.T @ V) / V.shape[0]
    off = C - np.eye(130)
    assert np.abs(off).max() < 6 / math.sqrt(V.shape[0])
    # probe p does not depend on how many probes are drawn or which rows
    assert np.array_equal(slq.rademacher(4000, 64, seed=7), V[:, :64])
    ids = np.array([5, 3999, 17])
    assert np.array_equal(slq.rademacher(4000, 130, seed=7, node_ids=ids), V[ids])
    assert not np.array_equal(slq.rademacher(4000, 130, seed=8), V)


# ------------------------------------------------------ closed-form spectra --
def closed_form(name, n, kind):
    k = np.arange(n)
    if kind == slq.NORMALIZED:
        return {
            "complete": np.r_[0.0, np.full(n - 1, n / (n - 1))],
            "cycle": 1 - np.cos(2 * np.pi * k / n),
            "path": 1 - np.cos(np.pi * k / (n - 1)),
            "star": np.r_[0.0, np.ones(n - 2), 2.0],
        }[name]
    return {
        "complete": np.r_[0.0, np.full(n - 1, float(n))],
        "cycle": 2 - 2 * np.cos(2 * np.pi * k / n),
        "path": 2 - 2 * np.cos(np.pi * k / n),
        "star": np.r_[0.0, np.ones(n - 2), float(n)],
    }[name]


@pytest.mark.parametrize("kind", [slq.NORMALIZED, slq.COMBINATORIAL])
@pytest.mark.parametrize("name", ["complete", "cycle", "path", "star"])
@pytest.mark.parametrize("n", [5, 12, 31])
def test_dense_laplacian_closed_forms(name, n, kind):
    g = graph(getattr(inputs, name)(n), kind)
    lam = exact.spectrum(g)
    assert np.allclose(np.sort(lam), np.sort(closed_form(name, n, kind)), atol=1e-12, rtol=0)


def test_complete_graph_vnge_and_heat_closed_form():
    n = 9
    g = graph(inputs.complete(n))
    lam = exact.spectrum(g)
    # density matrix eigenvalues 1/(n-1), (n-1) times -> H = ln(n-1)
    assert abs(exact.exact_vnge(lam, g.trace) - math.log(n - 1)) < 1e-12
    t = np.array([0.0, 0.3, 5.0])
    assert np.allclose(exact.exact_heat(lam, t), 1 + (n - 1) * np.exp(-t * n / (n - 1)), rtol=1e-13)


def test_isolated_nodes_follow_chung_convention():
    base = inputs.complete(5)
    iso = inputs.CSR(n=8, row_ptr=np.r_[base.row_ptr, [base.nnz] * 3], col_idx=base.col_idx)
    g = graph(iso)
    assert g.n_isolated == 3 and g.trace == 5
    lam = np.sort(exact.spectrum(g))
    assert np.allclose(lam, [0, 0, 0, 0, 1.25, 1.25, 1.25, 1.25], atol=1e-12)


@pytest.mark.parametrize("kind", [slq.NORMALIZED, slq.COMBINATORIAL])
def test_sparse_operator_matches_dense(kind):
    csr = inputs.erdos_renyi(60, 0.08, seed=3)   # has isolated nodes at this p
    rng = np.random.default_rng(0)
    w = None
    for weighted in (False, True):
        if weighted:
            # symmetric positive weights: w(i,j) = 1 + ((i*j) mod 7) / 3
            r = np.repeat(np.arange(csr.n), np.diff(csr.row_ptr))
            w = 1.0 + ((r * csr.col_idx) % 7) / 3.0
        g = graph(csr, kind, w)
        X = rng.standard_normal((csr.n, 5))
        assert np.allclose(slq.apply_laplacian(g, X), exact.dense_laplacian(g) @ X, atol=1e-13)
    assert graph(csr).n_isolated > 0


# ------------------------------------------------- Figure 1 worked example --
@pytest.mark.parametrize("name,printed", [("karate", 3.154), ("dolphins", 3.846)])
def test_fig1_exact_vnge(name, printed):
    g = graph(load_fig1(name), slq.COMBINATORIAL)
    lam = exact.spectrum(g)
    assert abs(exact.exact_vnge(lam, g.trace) - printed) < 5e-4


@pytest.mark.parametrize("name,printed", [("karate", 3.154), ("dolphins", 3.846)])
def test_fig1_slq_vnge_default_parameters(name, printed):
    # paper defaults nv=100, s=10 (§4): SLQ lands close to the printed value
    g = graph(load_fig1(name), slq.COMBINATORIAL)
    est = slq.slaq_vnge(g, nv=100, m=10, seed=2020)
    assert abs(est - printed) / printed < 1e-2


# ------------------------------------------------ brute force on tiny graphs --
def tiny_cases():
    return [
        ("karate", load_fig1("karate")),
        ("dolphins", load_fig1("dolphins")),
        ("K7", inputs.complete(7)),
        ("S9", inputs.star(9)),
        ("P11", inputs.path(11)),
        ("ER40", inputs.erdos_renyi(40, 0.1, seed=11)),
        ("SBM30", inputs.sbm(30, 3, 0.5, 0.05, seed=5)),
    ]


FUNCS = {
    "heat0.1": lambda x: np.exp(-0.1 * x),
    "heat3": lambda x: np.exp(-3.0 * x),
    "heat50": lambda x: np.exp(-50.0 * x),
    "wave2": lambda x: np.cos(2.0 * x),
}


@pytest.mark.parametrize("kind", [slq.NORMALIZED, slq.COMBINATORIAL])
@pytest.mark.parametrize("case", tiny_cases(), ids=lambda c: c[0])
def test_slq_equals_bruteforce_hutchinson_when_krylov_space_is_exhausted(case, kind):
    # the Gauss rule is exact once the Krylov space is invariant, so with m = n
    # SLQ equals Hutchinson on the same probes (§3.1, eqs. "trace", "slq")
    _, csr = case
    g = graph(csr, kind)
    nv, seed = 12, 99
    a, b, s = slq.lanczos(g, nv, csr.n, seed)
    th, w2 = slq.ritz(a, b, s)
    for fname, f in FUNCS.items():
        if kind == slq.COMBINATORIAL and fname.startswith("heat") and fname != "heat0.1":
            continue  # exp(-t x) underflows on the wide combinatorial spectrum
        est = slq.quadrature(th, w2, csr.n, f)
        ref, _ = exact.hutchinson(g, nv, seed, f)
        assert abs(est - ref) <= 1e-10 * max(abs(ref), 1.0), fname
    tr = g.trace
    est = slq.vnge(th, w2, csr.n, tr)
    ref, _ = exact.hutchinson(g, nv, seed, lambda x: -slq.xlogx(x / tr))
    assert abs(est - ref) <= 1e-10 * abs(ref)


def distinct_eigenvalues_seen(g, q):
    """Number of distinct eigenvalues whose eigenspace holds part of q: the
    dimension of the Krylov space q generates."""
    lam, Phi = np.linalg.eigh(exact.dense_laplacian(g))
    groups = np.split(np.arange(lam.size), np.flatnonzero(np.diff(lam) > 1e-8) + 1)
    return sum(1 for grp in groups if np.sum((Phi[:, grp].T @ q) ** 2) > 1e-12)


@pytest.mark.parametrize("csr", [inputs.complete(20), inputs.star(15), inputs.cycle(16),
                                 inputs.path(9)], ids=["K20", "S15", "C16", "P9"])
def test_breakdown_length_is_krylov_dimension(csr):
    # K_n has 2 distinct normalized eigenvalues, the star 3, C_n about n/2: the
    # Krylov space of a start vector is invariant once it holds every
    # eigen-direction the vector touches (a zero-sum probe on K_n is itself an
    # eigenvector and stops after one step)
    g = graph(csr)
    nv = 16
    _, b, s = slq.lanczos(g, nv, 14, seed=1)
    V = slq.rademacher(csr.n, nv, 1)
    for p in range(nv):
        k = distinct_eigenvalues_seen(g, V[:, p] / math.sqrt(csr.n))
        assert s[p] == min(k, 14), p
        assert np.all(b[p, : s[p] - 1] > 1e-3)


def test_edgeless_graph_is_exact():
    csr = inputs.CSR(n=6, row_ptr=np.zeros(7, dtype=np.int64), col_idx=np.zeros(0, dtype=np.int32))
    g = graph(csr)
    a, b, s = slq.lanczos(g, 4, 5, seed=3)
    th, w2 = slq.ritz(a, b, s)
    assert np.all(s == 1)
    assert np.allclose(slq.heat_trace(th, w2, 6, [0.0, 1.0, 10.0]), 6.0)
    assert slq.vnge(th, w2, 6, max(g.trace, 1.0)) == 0.0


# ------------------------------------------------------------- invariants ---
@pytest.fixture(scope="module")
def chung_lu_run():
    csr = inputs.chung_lu(3000, 15000, 2.5, seed=4)
    g = graph(csr)
    a, b, s = slq.lanczos(g, 10, 15, seed=5)
    th, w2 = slq.ritz(a, b, s)
    return csr, g, a, b, s, th, w2


def test_invariants(chung_lu_run):
    csr, g, a, b, s, th, w2 = chung_lu_run
    n = csr.n
    assert np.allclose(w2.sum(axis=1), 1.0, atol=1e-12)
    assert th.min() >= -1e-12 and th.max() <= 2 + 1e-12
    t = slq.t_grid(256)
    h = slq.heat_trace(th, w2, n, np.r_[0.0, t])
    assert abs(h[0] - n) < 1e-9 * n
    assert np.all(np.diff(h) <= 1e-9 * n)
    assert abs(slq.wave_trace(th, w2, n, [0.0])[0] - n) < 1e-9 * n
    H = slq.vnge(th, w2, n, g.trace)
    assert 0 < H <= math.log(g.trace) + 1e-9


def test_t_grid():
    t = slq.t_grid(256)
    assert t.size == 256 and t[0] == 0.01 and abs(t[-1] - 100.0) < 1e-12
    assert np.allclose(np.diff(np.log10(t)), 4 / 255)


def per_probe_gauss(a, b, s, m, t):
    out = []
    for p in range(a.shape[0]):
        k = min(int(s[p]), m)
        lam, U = np.linalg.eigh(slq.tridiagonal(a[p], b[p], k))
        out.append((U[0] ** 2 * np.exp(-t * lam)).sum())
    return np.array(out)


def test_gauss_monotone_and_bracketed_by_radau():
    csr = inputs.chung_lu(400, 1500, 2.5, seed=8)
    g = graph(csr)
    nv = 6
    a, b, s = slq.lanczos(g, nv, 12, seed=2)
    Q = slq.rademacher(csr.n, nv, 2) / math.sqrt(csr.n)
    for t in (0.5, 3.0, 20.0):
        F = exact.matrix_function(g, lambda x: np.exp(-t * x))
        ex = np.einsum("ip,ij,jp->p", Q, F, Q)
        prev = None
        for m in range(1, 12):
            cur = per_probe_gauss(a, b, s, m, t)
            assert np.all(cur <= ex + 1e-12)
            if prev is not None:
                assert np.all(cur >= prev - 1e-12)
            prev = cur
            lo, hi = radau.heat_bracket(a[:, :m], b[:, :m], np.minimum(s, m), [t])
            assert np.allclose(lo[:, 0], cur, rtol=1e-12, atol=1e-15)
            assert np.all(hi[:, 0] >= ex - 1e-12)


def eps2(s, t):
    """Error bound of the Lanczos approximation of q^T exp(-tL) q (§3.1,
    eq. "eps2"; applies to the normalized Laplacian and unit q)."""
    if math.sqrt(2 * t) <= s <= t:
        return 20 * math.exp(-s * s / (2.5 * t))
    if s >= t:
        return 40 / t * math.exp(-0.5 * t) * (0.5 * math.e * t / s) ** s
    return None


def test_lanczos_error_bound_eps2():
    csr = inputs.chung_lu(500, 2000, 2.5, seed=9)
    g = graph(csr)
    nv = 5
    a, b, s = slq.lanczos(g, nv, 30, seed=4)
    Q = slq.rademacher(csr.n, nv, 4) / math.sqrt(csr.n)
    checked = 0
    for t in (1.0, 4.0, 10.0, 30.0):
        F = exact.matrix_function(g, lambda x: np.exp(-t * x))
        ex = np.einsum("ip,ij,jp->p", Q, F, Q)
        for m in range(2, 31):
            bound = eps2(m, t)
            if bound is None:
                continue
            err = np.abs(per_probe_gauss(a, b, s, m, t) - ex)
            assert np.all(err <= bound + 1e-13), (t, m)  # + FP64 rounding floor
            checked += 1
    assert checked > 50


def test_slq_accuracy_against_exact_spectrum_is_monte_carlo_sized(chung_lu_run):
    # soft: SLQ vs the exact trace is limited by Hutchinson noise (nv = 10)
    csr, g, a, b, s, th, w2 = chung_lu_run
    lam = exact.spectrum(g)
    t = slq.t_grid(32)
    est = slq.heat_trace(th, w2, csr.n, t)
    ref = exact.exact_heat(lam, t)
    assert np.linalg.norm(est - ref) / np.linalg.norm(ref) < 2e-2


# ------------------------------------------------ self-loops and tr L ------
def with_self_loops(csr, nodes, weight=1.0):
    """csr plus a self-loop of the given weight on each of `nodes` (weights
    returned for every stored entry, 1 elsewhere)."""
    rows = np.repeat(np.arange(csr.n), np.diff(csr.row_ptr))
    r = np.r_[rows, nodes]
    c = np.r_[csr.col_idx, nodes].astype(np.int64)
    w = np.r_[np.ones(csr.nnz), np.full(len(nodes), weight)]
    order = np.lexsort((c, r))
    r, c, w = r[order], c[order], w[order]
    rp = np.zeros(csr.n + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=csr.n), out=rp[1:])
    return inputs.CSR(n=csr.n, row_ptr=rp, col_idx=c.astype(np.int32)), w


@pytest.mark.parametrize("kind", [slq.NORMALIZED, slq.COMBINATORIAL])
def test_trace_is_sum_of_eigenvalues_with_self_loops(kind):
    # tr L is the sum of the spectrum whatever the diagonal of A holds (§2;
    # the density matrix L / tr L of §2.1 needs it), and the entropy of the
    # density matrix from the dense spectrum equals SLQ at m = n on the same
    # probes (brute-force Hutchinson with that trace)
    csr, w = with_self_loops(inputs.erdos_renyi(30, 0.15, seed=21), [0, 4, 9, 17], 2.5)
    g = graph(csr, kind, w)
    lam = exact.spectrum(g)
    assert abs(g.trace - lam.sum()) <= 1e-10 * abs(lam.sum())
    # without the loops' share the trace would be off by a visible amount
    assert abs(lam.sum() - (np.count_nonzero(g.deg > 0) if kind == slq.NORMALIZED else g.deg.sum())) > 0.1
    nv, seed = 10, 5
    a, b, s = slq.lanczos(g, nv, csr.n, seed)
    th, w2 = slq.ritz(a, b, s)
    c = lam.sum()
    ref, _ = exact.hutchinson(g, nv, seed, lambda x: -slq.xlogx(x / c))
    assert abs(slq.vnge(th, w2, csr.n, g.trace) - ref) <= 1e-10 * abs(ref)


def test_torch_backend_equals_scipy_backend():
    # the two sparse-product primitives give the same recurrence (weights,
    # self-loops and isolated nodes included)
    base = inputs.chung_lu(1500, 6000, 2.5, seed=13)
    csr, w = with_self_loops(base, [3, 50, 700], 0.5)
    w = w * (1.0 + 0.25 * (np.arange(w.size) % 3 == 0))  # asymmetric would be wrong: keep loops only
    w[np.repeat(np.arange(csr.n), np.diff(csr.row_ptr)) != csr.col_idx] = 1.0
    for kind in (slq.NORMALIZED, slq.COMBINATORIAL):
        g1 = slq.build_graph(csr.n, csr.row_ptr, csr.col_idx, w, kind)
        g2 = slq.build_graph(csr.n, csr.row_ptr, csr.col_idx, w, kind, backend="torch")
        assert np.array_equal(g1.deg, g2.deg) and np.array_equal(g1.self_w, g2.self_w)
        a1, b1, s1 = slq.lanczos(g1, 5, 12, seed=8)
        a2, b2, s2 = slq.lanczos(g2, 5, 12, seed=8)
        assert np.array_equal(s1, s2)
        assert np.allclose(a1, a2, rtol=1e-12, atol=1e-14) and np.allclose(b1, b2, rtol=1e-12, atol=1e-14)


# ---------------------------------------------- Gauss-Radau companion rule --
@pytest.mark.parametrize("fixed", [0.0, -0.5])
def test_radau_rule_has_the_fixed_node_and_degree_2k_exactness(fixed):
    # a (k+1)-point rule with one prescribed node integrates polynomials of
    # degree <= 2k exactly; the k-point Gauss rule only up to 2k - 1
    # (Golub and Meurant; the spectral measure of q is sum_i (phi_i^T q)^2
    # delta(lambda_i), so the moments are q^T L^j q)
    csr = inputs.erdos_renyi(40, 0.12, seed=17)
    g = graph(csr)
    L = exact.dense_laplacian(g)
    nv, seed = 3, 6
    a, b, s = slq.lanczos(g, nv, 6, seed)
    Q = slq.rademacher(csr.n, nv, seed) / math.sqrt(csr.n)
    for p in range(nv):
        for k in (2, 3, 5):
            assert s[p] > k
            nodes, weights = radau.radau_rule(a[p], b[p], k, fixed)
            assert nodes.size == k + 1
            assert np.min(np.abs(nodes - fixed)) < 1e-10
            lam, U = np.linalg.eigh(slq.tridiagonal(a[p], b[p], k))
            gw = U[0] ** 2
            mom = Q[:, p].copy()
            for j in range(2 * k + 1):
                exact_j = Q[:, p] @ mom  # q^T L^j q
                assert abs(np.sum(weights * nodes ** j) - exact_j) <= 1e-9 * max(1.0, abs(exact_j)), (k, j)
                gauss_j = np.sum(gw * lam ** j)
                if j < 2 * k:
                    assert abs(gauss_j - exact_j) <= 1e-9 * max(1.0, abs(exact_j))
                else:  # the Gauss rule misses the degree-2k moment
                    assert abs(gauss_j - exact_j) > 1e-6
                mom = L @ mom


# ------------------------------------------------------ Algorithm 1 entries --
@pytest.mark.parametrize("kind", [slq.NORMALIZED, slq.COMBINATORIAL])
def test_algorithm1_entry_points_equal_bruteforce(kind):
    # SLaQ_LSD and SLaQ_VNGE at m = n equal Hutchinson on the same probes,
    # heat and wave kept apart (a swapped branch fails)
    csr = inputs.sbm(36, 3, 0.4, 0.05, seed=2)
    g = graph(csr, kind)
    nv, seed = 8, 31
    t = np.array([0.05, 0.4, 1.7])
    heat = slq.slaq_lsd(g, nv, csr.n, seed, t)
    wave = slq.slaq_lsd(g, nv, csr.n, seed, t, wave=True)
    for k, tt in enumerate(t):
        h, _ = exact.hutchinson(g, nv, seed, lambda x: np.exp(-tt * x))
        w, _ = exact.hutchinson(g, nv, seed, lambda x: np.cos(tt * x))
        assert abs(heat[k] - h) <= 1e-10 * abs(h)
        assert abs(wave[k] - w) <= 1e-10 * max(abs(w), 1.0)
        assert abs(heat[k] - wave[k]) > 1e-3
    c = g.trace
    H, _ = exact.hutchinson(g, nv, seed, lambda x: -slq.xlogx(x / c))
    assert abs(slq.slaq_vnge(g, nv, csr.n, seed) - H) <= 1e-10 * abs(H)


# ------------------------------------- combinatorial spectral bound / breakdown
def test_combinatorial_spectral_bound_covers_the_spectrum():
    # Gershgorin (§2): every eigenvalue of D - A lies in [0, 2 max D_ii]
    for seed in range(4):
        csr = inputs.chung_lu(200, 700, 2.5, seed=seed)
        r = np.repeat(np.arange(csr.n), np.diff(csr.row_ptr))
        w = 0.5 + ((r + csr.col_idx) % 5)  # symmetric positive weights
        g = graph(csr, slq.COMBINATORIAL, w)
        lam = exact.spectrum(g)
        assert g.spectral_bound == 2.0 * g.deg.max()
        assert lam.max() <= g.spectral_bound * (1 + 1e-12)
        assert lam.max() >= 0.5 * g.spectral_bound  # the bound is not loose by more than 2x (lambda_max >= max D)


@pytest.mark.parametrize("scale", [1.0, 1e-9, 1e7])
def test_combinatorial_breakdown_is_scale_invariant(scale):
    # K_n under D - A has eigenvalues {0, n}: a probe's Krylov space has
    # dimension <= 2, whatever the weight of the edges; the breakdown test is
    # relative to the spectral bound 2 max D_ii, so tiny weights do not stop
    # the recurrence early and large ones still stop it at the Krylov dimension
    csr = inputs.complete(12)
    g = graph(csr, slq.COMBINATORIAL, np.full(csr.nnz, scale))
    nv = 8
    a, b, s = slq.lanczos(g, nv, 6, seed=4)
    V = slq.rademacher(csr.n, nv, 4)
    for p in range(nv):
        k = distinct_eigenvalues_seen(graph(csr, slq.COMBINATORIAL), V[:, p] / math.sqrt(csr.n))
        assert k <= 2
        assert s[p] == k, (p, s[p], k)
        assert np.all(b[p, : k - 1] > 1e-3 * scale)
    th, w2 = slq.ritz(a, b, s)
    assert np.allclose(th[w2 > 1e-12], np.where(th[w2 > 1e-12] > 1e-6 * scale, 12.0 * scale, 0.0),
                       rtol=1e-9, atol=1e-9 * scale)
