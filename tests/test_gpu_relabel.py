"""GPU tests of the graph build's node relabelling: the internal order and CSR
equal the numpy reference exactly (index work), and relabelled graphs give
the oracle's results within the parity tolerances (the probes stay keyed by
the caller's ids, so only rounding order changes)."""
import numpy as np
import pytest
import torch

from oracle import slq as O
from paper_2003_01282_amd import inputs
from paper_2003_01282_amd import slaq as S

from gpu_helpers import assert_signature_parity, gpu_run, oracle_run
from relabel_ref import piece_count, relabel

pytestmark = pytest.mark.gpu

T256 = O.t_grid(256)


def header(msg):
    print(f"\n[gpu] {msg}", flush=True)


def with_isolated(csr, n_iso, seed=0):
    """csr plus n_iso isolated nodes spread among the others."""
    rng = np.random.default_rng(seed)
    n = csr.n + n_iso
    new_id = np.sort(rng.choice(n, csr.n, replace=False))
    lens = np.zeros(n, dtype=np.int64)
    lens[new_id] = np.diff(csr.row_ptr)
    rp = np.zeros(n + 1, dtype=np.int64)
    rp[1:] = np.cumsum(lens)
    return inputs.CSR(n=n, row_ptr=rp, col_idx=new_id[csr.col_idx].astype(np.int32))


CASES = {
    "chung_lu_iso": lambda: with_isolated(inputs.chung_lu(5000, 20000, 2.3, seed=7), 700),
    "star_iso": lambda: with_isolated(inputs.star(3000), 50),
    "path5_iso": lambda: with_isolated(inputs.path(5), 9),        # n_act < 8
    "k9": lambda: inputs.complete(9),                              # one node per range + 1
    "edgeless": lambda: inputs.CSR(n=6, row_ptr=np.zeros(7, dtype=np.int64), col_idx=np.zeros(0, dtype=np.int32)),
    "rmat14": lambda: inputs.rmat(14, seed=3),
    "er_iso": lambda: with_isolated(inputs.erdos_renyi(3000, 0.003, seed=4), 400, seed=2),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_internal_layout_matches_reference(case):
    header(f"relabel layout {case}")
    csr = CASES[case]()
    rp, ci = S.to_device(csr)
    g = S.build_graph(rp, ci, relabel=True, check=True)
    got = g.internal()
    ref = relabel(csr.row_ptr, csr.col_idx)
    assert got["relabeled"]
    assert got["n_rows"] == ref["n_rows"]
    assert np.array_equal(got["perm"].cpu().numpy(), ref["perm"])
    assert np.array_equal(got["row_ptr"].cpu().numpy(), ref["row_ptr"])
    assert np.array_equal(got["col_idx"].cpu().numpy(), ref["col_idx"])
    # without relabelling the handle reads the caller's CSR as is
    g0 = S.build_graph(rp, ci, relabel=False)
    raw = g0.internal()
    assert not raw["relabeled"] and raw["n_rows"] == csr.n
    assert np.array_equal(raw["perm"].cpu().numpy(), np.arange(csr.n))
    assert np.array_equal(raw["col_idx"].cpu().numpy(), csr.col_idx)


PARITY = [(c, S.SLAQ_LAP_NORMALIZED) for c in ("chung_lu_iso", "star_iso", "path5_iso", "k9", "edgeless", "rmat14",
                                                  "er_iso")]
# D - A (FP64 vectors by default)
PARITY += [(c, S.SLAQ_LAP_COMBINATORIAL) for c in ("chung_lu_iso", "star_iso", "path5_iso", "k9", "edgeless",
                                                     "er_iso", "rmat14")]


@pytest.mark.parametrize("case,lap", PARITY)
def test_relabelled_parity(case, lap):
    header(f"relabel parity {case} lap={lap}")
    csr = CASES[case]()
    nv, m = 20, 15
    gpu = gpu_run(csr, nv, m, 99, T256, laplacian=lap, relabel=True)
    ora = oracle_run(csr, nv, m, 99, T256, laplacian=lap)
    # dinv_out stays in caller order (D^-1/2, or D for the combinatorial Laplacian)
    want = ora["graph"].dinv if lap == S.SLAQ_LAP_NORMALIZED else ora["graph"].deg
    np.testing.assert_allclose(gpu["dinv"], want, rtol=1e-7)
    # coefficients to the 1e-4 bar of the signatures (on skewed degree
    # distributions the FP32 recurrence drifts by a few 1e-5 at the last
    # steps); absolute floor: FP32 rounding of an operator of spectral bound S
    # (2, or 2 max D_ii) over m steps
    S_bound = 2.0 if lap == S.SLAQ_LAP_NORMALIZED else 2.0 * max(float(ora["graph"].deg.max()), 1.0)
    atol = max(1e-5, 1e-8 * S_bound * m)
    for p in range(nv):
        k = int(min(gpu["steps"][p], ora["steps"][p]))
        np.testing.assert_allclose(gpu["alpha"][p, :k], ora["alpha"][p, :k], rtol=1e-4, atol=atol)
        np.testing.assert_allclose(gpu["beta"][p, :k - 1], ora["beta"][p, :k - 1], rtol=1e-4, atol=atol)
    assert_signature_parity(gpu, ora, csr.n, f"relabel {case}")


def test_combinatorial_hub_graph_precision():
    # D - A of a power-law graph (max degree ~900, spectrum [0, ~1800]): its
    # top eigenvalues converge within a few steps and the recurrence, without
    # reorthogonalization, then loses orthogonality to them.  With FP64
    # vectors (the default for D - A) that happens as late as in the FP64
    # oracle and the parity bar holds; with FP32 vectors it starts from step
    # ~10 and the low Ritz values and VNGE move by ~1e-4 relative, while the
    # first steps and the heat trace up to t = 0.1 still agree to 1e-4.
    header("combinatorial hub graph, FP64 and FP32 vectors")
    csr = CASES["chung_lu_iso"]()
    nv, m = 20, 15
    lap = S.SLAQ_LAP_COMBINATORIAL
    ora = oracle_run(csr, nv, m, 99, T256, laplacian=lap)
    for r in (True, False):
        gpu = gpu_run(csr, nv, m, 99, T256, laplacian=lap, relabel=r)
        np.testing.assert_allclose(gpu["alpha"], ora["alpha"], rtol=1e-7)
        np.testing.assert_allclose(gpu["beta"], ora["beta"], rtol=1e-7)
        assert_signature_parity(gpu, ora, csr.n, f"D - A FP64 relabel={r}")
    early = T256 <= 0.1
    runs = [gpu_run(csr, nv, m, 99, T256, laplacian=lap, relabel=r, precision=S.SLAQ_PREC_FP32) for r in (True, False)]
    for gpu in runs:
        np.testing.assert_allclose(gpu["alpha"][:, :8], ora["alpha"][:, :8], rtol=1e-5)
        np.testing.assert_allclose(gpu["beta"][:, :7], ora["beta"][:, :7], rtol=1e-5)
        assert abs(gpu["vnge"] - ora["vnge"]) / abs(ora["vnge"]) <= 1e-3
        rel = np.abs(gpu["heat"][early] - ora["heat"][early]) / ora["heat"][early]
        assert rel.max() <= 1e-4
    # heat counts nodes (h_0 = n): an absolute floor of 1e-4 for its decayed tail
    np.testing.assert_allclose(runs[0]["heat"], runs[1]["heat"], rtol=1e-3, atol=1e-4)


@pytest.mark.parametrize("relabel", [False, True])
def test_fp64_vectors_match_the_oracle_tightly(relabel):
    # the same kernels in FP64 differ from the FP64 oracle only in summation
    # order: a tight pin on the SpMM / update / reduction arithmetic
    header(f"FP64 vectors, normalized, relabel={relabel}")
    csr = CASES["chung_lu_iso"]()
    gpu = gpu_run(csr, 36, 15, 4, T256, relabel=relabel, precision=S.SLAQ_PREC_FP64)
    ora = oracle_run(csr, 36, 15, 4, T256)
    np.testing.assert_allclose(gpu["alpha"], ora["alpha"], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(gpu["beta"], ora["beta"], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(gpu["heat"], ora["heat"], rtol=1e-9)
    assert abs(gpu["vnge"] - ora["vnge"]) <= 1e-9 * abs(ora["vnge"])


def test_relabelled_weighted():
    header("relabel weighted SBM + isolated")
    base = inputs.sbm(2500, 4, 0.02, 0.001, seed=3)
    csr = with_isolated(base, 300, seed=5)
    r = np.repeat(np.arange(csr.n), np.diff(csr.row_ptr))
    c = csr.col_idx.astype(np.int64)
    lo, hi = np.minimum(r, c), np.maximum(r, c)
    w = (0.25 + ((lo * 2654435761 + hi * 40503) % 1000) / 500.0).astype(np.float32)  # symmetric weights
    for lap in (S.SLAQ_LAP_NORMALIZED, S.SLAQ_LAP_COMBINATORIAL):
        gpu = gpu_run(csr, 16, 12, 8, T256, laplacian=lap, weights=w, relabel=True)
        ora = oracle_run(csr, 16, 12, 8, T256, laplacian=lap, weights=w.astype(np.float64))
        np.testing.assert_allclose(gpu["alpha"], ora["alpha"], rtol=1e-5, atol=1e-6)
        np.testing.assert_allclose(gpu["beta"], ora["beta"], rtol=1e-5, atol=1e-6)
        assert_signature_parity(gpu, ora, csr.n, f"relabel weighted lap={lap}")


@pytest.mark.parametrize("lap", [S.SLAQ_LAP_NORMALIZED, S.SLAQ_LAP_COMBINATORIAL])
def test_relabelled_weighted_hub_rows(lap):
    # rows of more than 1024 entries take the chunked relabelling path; their
    # weights must travel with their columns
    header(f"relabel weighted hubs lap={lap}")
    csr = with_isolated(inputs.chung_lu(6000, 60000, 2.1, seed=13), 200, seed=4)
    assert np.diff(csr.row_ptr).max() > 1024
    r = np.repeat(np.arange(csr.n), np.diff(csr.row_ptr))
    c = csr.col_idx.astype(np.int64)
    lo, hi = np.minimum(r, c), np.maximum(r, c)
    w = (0.5 + ((lo * 977 + hi * 131) % 23) / 11.0).astype(np.float32)
    gpu = gpu_run(csr, 16, 12, 21, T256, laplacian=lap, weights=w, relabel=True)
    ora = oracle_run(csr, 16, 12, 21, T256, laplacian=lap, weights=w.astype(np.float64))
    np.testing.assert_allclose(gpu["alpha"][:, :6], ora["alpha"][:, :6], rtol=1e-5)
    assert_signature_parity(gpu, ora, csr.n, f"relabel weighted hubs lap={lap}")


@pytest.mark.parametrize("heavy_min,piece", [(128, 64), (256, 256), (128, 1024)])
def test_relabelled_schedules(heavy_min, piece):
    header(f"relabel schedule {heavy_min}/{piece}")
    csr = inputs.rmat(15, seed=2)
    rp, ci = S.to_device(csr)
    g = S.build_graph(rp, ci, relabel=True)
    g.set_schedule(heavy_min, piece)
    sch = g.schedule()
    ref = relabel(csr.row_ptr, csr.col_idx)
    lens = np.diff(ref["row_ptr"])
    assert sch["n_heavy"] == int(np.count_nonzero(lens >= heavy_min))
    assert sch["n_pieces"] == piece_count(ref["row_ptr"], ref["col_idx"], ref["bounds"], heavy_min, piece)
    a, b, s = S.lanczos(g, 36, 12, 5)
    ora = oracle_run(csr, 36, 12, 5, T256[::8])
    np.testing.assert_allclose(a.cpu().numpy(), ora["alpha"], rtol=1e-4, atol=1e-6)
    np.testing.assert_allclose(b.cpu().numpy(), ora["beta"], rtol=1e-4, atol=1e-6)


def test_size_rule_and_determinism():
    # from SLAQ_RELABEL_MIN_NNZ stored entries up the build relabels by itself
    header("relabel size rule")
    n = 180_000
    csr = inputs.erdos_renyi(n, 26.0 / n, seed=11)
    assert csr.nnz >= S.SLAQ_RELABEL_MIN_NNZ
    small = inputs.erdos_renyi(2000, 0.01, seed=1)
    rp, ci = S.to_device(small)
    assert not S.build_graph(rp, ci).internal()["relabeled"]
    rp, ci = S.to_device(csr)
    g = S.build_graph(rp, ci)
    assert g.internal()["relabeled"]
    a1, b1, s1 = S.lanczos(g, 8, 10, 3)
    a2, b2, s2 = S.lanczos(S.build_graph(rp, ci), 8, 10, 3)
    assert torch.equal(a1, a2) and torch.equal(b1, b2) and torch.equal(s1, s2)
    ora = O.lanczos(O.build_graph(csr.n, csr.row_ptr, csr.col_idx), 8, 10, 3)
    np.testing.assert_allclose(a1.cpu().numpy(), ora[0], rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(b1.cpu().numpy(), ora[1], rtol=1e-5, atol=1e-6)


def test_flag_conflict_rejected():
    csr = inputs.path(10)
    rp, ci = S.to_device(csr)
    n = csr.n
    dinv = torch.empty(n, dtype=torch.float32, device="cuda")
    nb = S._sz()
    S._check(S.lib().slaq_graph_scratch_bytes(n, csr.nnz, S.ctypes.byref(nb)))
    scratch = S._empty_aligned(nb.value, "cuda")
    h = S._vp()
    st = S.lib().slaq_build_graph(n, csr.nnz, S._ptr(rp), S._ptr(ci), None, 0,
                                  S.SLAQ_FLAG_RELABEL | S.SLAQ_FLAG_NO_RELABEL, S._ptr(dinv), S._ptr(scratch),
                                  scratch.numel(), None, S.ctypes.byref(h))
    assert st == 1  # SLAQ_ERR_INVALID_ARG


@pytest.mark.parametrize("precision", [S.SLAQ_PREC_FP32, S.SLAQ_PREC_FP64])
def test_cache_window_hints_leave_results_unchanged(precision):
    # the hot window only chooses load hints: every window gives the same
    # coefficients bit for bit (hub rows in pieces, light rows, all ranges)
    print(f"\n[gpu] cache window sweep, precision {precision}", flush=True)
    csr = inputs.chung_lu(20_000, 150_000, 2.2, seed=3)
    rp, ci = S.to_device(csr)
    g = S.build_graph(rp, ci, relabel=True)
    g.set_precision(precision)
    assert g.cache_rows() == -1
    ref = [x.cpu().numpy() for x in S.lanczos(g, 37, 8, 5)]
    assert g.schedule()["n_heavy"] > 0
    for rows in (0, 1, 100, 2500, 10**9):
        g.set_cache_rows(rows)
        assert g.cache_rows() == rows
        got = [x.cpu().numpy() for x in S.lanczos(g, 37, 8, 5)]
        for r, x in zip(ref, got):
            np.testing.assert_array_equal(x, r)
    with pytest.raises(S.SlaqError):
        g.set_cache_rows(-2)
