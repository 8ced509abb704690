"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs (same graphs, same SplitMix64 probes)."""
import math

import numpy as np
import pytest
import torch

from oracle import slq as O
from paper_2003_01282_amd import inputs
from paper_2003_01282_amd import slaq as S

from gpu_helpers import assert_signature_parity, gpu_run, oracle_run
from test_oracle_pins import load_fig1

pytestmark = pytest.mark.gpu

T256 = O.t_grid(256)


def header(msg):
    print(f"\n[gpu] {msg}", flush=True)


def test_chung_lu_small_config():
    # Chung-Lu power law, n=1e4, 5e4 endpoint pairs, nv=10, m=15, 256 t + VNGE
    header("chung_lu n=1e4 nv=10 m=15")
    csr = inputs.chung_lu(10_000, 50_000, 2.5, seed=1)
    gpu = gpu_run(csr, 10, 15, 2024, T256)
    ora = oracle_run(csr, 10, 15, 2024, T256)
    assert gpu["info"]["n_isolated"] == ora["graph"].n_isolated
    assert gpu["info"]["trace"] == ora["graph"].trace
    np.testing.assert_allclose(gpu["dinv"], ora["graph"].dinv, rtol=1e-7)
    assert np.array_equal(gpu["steps"], ora["steps"])
    np.testing.assert_allclose(gpu["alpha"], ora["alpha"], rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(gpu["beta"], ora["beta"], rtol=1e-5, atol=1e-6)
    rh, rw = assert_signature_parity(gpu, ora, csr.n, "C1")
    print(f"heat rel {rh:.2e} wave |d|/n {rw:.2e}")


@pytest.mark.parametrize("nv", [1, 3, 64, 100, 130, 300])
def test_probe_counts_and_tiles(nv):
    # ragged ld (nv not a multiple of 4), several SplitMix64 words, two tiles
    header(f"ER n=3000 nv={nv}")
    csr = inputs.erdos_renyi(3000, 0.004, seed=nv)
    gpu = gpu_run(csr, nv, 12, 77, T256[::8])
    ora = oracle_run(csr, nv, 12, 77, T256[::8])
    assert np.array_equal(gpu["steps"], ora["steps"])
    # ER's normalized spectrum is narrow and its Ritz values converge within
    # 12 steps, so the late coefficients carry amplified FP32 rounding (about
    # 1e-5): compared at the signatures' 1e-4
    np.testing.assert_allclose(gpu["alpha"], ora["alpha"], rtol=1e-4, atol=1e-6)
    np.testing.assert_allclose(gpu["beta"], ora["beta"], rtol=1e-4, atol=1e-6)
    assert_signature_parity(gpu, ora, csr.n, f"nv={nv}")


@pytest.mark.parametrize("lap", [S.SLAQ_LAP_NORMALIZED, S.SLAQ_LAP_COMBINATORIAL])
@pytest.mark.parametrize("name", ["karate", "dolphins"])
def test_fig1_graphs(name, lap):
    header(f"fig1 {name} lap={lap}")
    csr = load_fig1(name)
    gpu = gpu_run(csr, 100, 10, 2020, T256, laplacian=lap)
    ora = oracle_run(csr, 100, 10, 2020, T256, laplacian=lap)
    assert np.array_equal(gpu["steps"], ora["steps"])
    assert_signature_parity(gpu, ora, csr.n, name)
    if lap == S.SLAQ_LAP_COMBINATORIAL:
        printed = {"karate": 3.154, "dolphins": 3.846}[name]
        assert abs(gpu["vnge"] - printed) / printed < 1e-2


def star_with_isolated(n_leaves, n_iso):
    s = inputs.star(n_leaves + 1)
    rp = np.r_[s.row_ptr, np.full(n_iso, s.nnz, dtype=np.int64)]
    return inputs.CSR(n=s.n + n_iso, row_ptr=rp, col_idx=s.col_idx)


@pytest.mark.parametrize("case", ["K30", "star2000", "star_iso", "cycle64", "path50", "edgeless", "single"])
def test_degenerate_graphs(case):
    # breakdown (K_n: 2 distinct eigenvalues, star: 3), a heavy row (star
    # centre of degree 1999), isolated nodes, no edges, a single node
    header(f"degenerate {case}")
    csr = {
        "K30": lambda: inputs.complete(30),
        "star2000": lambda: inputs.star(2000),
        "star_iso": lambda: star_with_isolated(500, 300),
        "cycle64": lambda: inputs.cycle(64),
        "path50": lambda: inputs.path(50),
        "edgeless": lambda: inputs.CSR(n=7, row_ptr=np.zeros(8, dtype=np.int64), col_idx=np.zeros(0, dtype=np.int32)),
        "single": lambda: inputs.CSR(n=1, row_ptr=np.zeros(2, dtype=np.int64), col_idx=np.zeros(0, dtype=np.int32)),
    }[case]()
    nv, m = 16, 15
    gpu = gpu_run(csr, nv, m, 5, T256)
    ora = oracle_run(csr, nv, m, 5, T256)
    # After an exact breakdown the FP32 residual is rounding noise amplified by
    # 1/(beta_1 ... beta_{k-1}) (beta_1 ~ sqrt(2/n) on a star; an FP32
    # emulation of the same recurrence on star(2000) gives beta_3 up to 5e-4),
    # so the GPU may carry on past the FP64 stopping step into directions whose
    # Gauss weights are O(beta_k^2).  Coefficients are compared up to the
    # shorter run, the signatures in full.
    for p in range(nv):
        k = int(min(gpu["steps"][p], ora["steps"][p]))
        np.testing.assert_allclose(gpu["alpha"][p, :k], ora["alpha"][p, :k], rtol=1e-5, atol=1e-5)
        np.testing.assert_allclose(gpu["beta"][p, :k - 1], ora["beta"][p, :k - 1], rtol=1e-5, atol=1e-5)
        if gpu["steps"][p] > ora["steps"][p]:
            assert gpu["beta"][p, k - 1] < 5e-3
    assert_signature_parity(gpu, ora, csr.n, case)
    np.testing.assert_allclose(gpu["tau2"].sum(axis=1), 1.0, atol=1e-9)


@pytest.mark.parametrize("heavy_min,piece", [(32, 64), (64, 128), (128, 64), (256, 512), (128, 1024), (100000, 64)])
def test_row_schedules(heavy_min, piece):
    # every schedule computes the same recurrence; heavy rows with partial
    # pieces, rows just below / above the threshold, no heavy rows at all
    header(f"schedule heavy_min={heavy_min} piece={piece}")
    csr = inputs.chung_lu(10_000, 50_000, 2.5, seed=4)
    rp, ci = S.to_device(csr)
    g = S.build_graph(rp, ci)
    g.set_schedule(heavy_min, piece)
    sch = g.schedule()
    deg = np.diff(csr.row_ptr)
    heavy = deg >= heavy_min
    assert sch["n_heavy"] == int(heavy.sum())
    # pieces: every heavy row is cut at the 8 column-id boundaries of equal nnz
    # mass (first id whose row offset reaches nnz//8 * x), then into pieces
    bnd = [0] + [int(np.searchsorted(csr.row_ptr, csr.nnz // 8 * x, side="left")) for x in range(1, 8)] + [csr.n]
    expect = 0
    for r in np.flatnonzero(heavy):
        cols = csr.col_idx[csr.row_ptr[r]:csr.row_ptr[r + 1]]
        lens = np.diff(np.searchsorted(cols, bnd[1:8], side="left"), prepend=0, append=cols.size)
        expect += int(((lens + piece - 1) // piece).sum())
    assert sch["n_pieces"] == expect
    a, b, s = S.lanczos(g, 24, 15, 31)
    th, w2 = S.ritz(a, b, s)
    tt = torch.from_numpy(T256).cuda()
    gpu = dict(heat=S.signature(th, w2, csr.n, tt).cpu().numpy(),
               wave=S.signature(th, w2, csr.n, tt, S.SLAQ_SIG_WAVE).cpu().numpy(),
               vnge=float(S.vnge(g, th, w2).cpu().numpy()[0]))
    ora = oracle_run(csr, 24, 15, 31, T256)
    np.testing.assert_allclose(a.cpu().numpy(), ora["alpha"], rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(b.cpu().numpy(), ora["beta"], rtol=1e-5, atol=1e-6)
    assert_signature_parity(gpu, ora, csr.n, f"schedule {heavy_min}/{piece}")


@pytest.mark.parametrize("tile_quads", [0, 25, 7, 1])
def test_probe_tiles(tile_quads):
    # the gather kernels run once per probe tile; every tiling gives the same
    # recurrence (auto = two tiles of 13 and 12 quads for nv = 100)
    header(f"probe tiles {tile_quads}")
    csr = inputs.chung_lu(6000, 30000, 2.5, seed=12)
    rp, ci = S.to_device(csr)
    g = S.build_graph(rp, ci)
    g.set_tile(tile_quads)
    a, b, s = S.lanczos(g, 100, 12, 77)
    ora = oracle_run(csr, 100, 12, 77, T256[::16])
    np.testing.assert_allclose(a.cpu().numpy(), ora["alpha"], rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(b.cpu().numpy(), ora["beta"], rtol=1e-5, atol=1e-6)


def test_weighted_graph():
    header("weighted SBM")
    csr = inputs.sbm(2500, 4, 0.02, 0.001, seed=3)
    r = np.repeat(np.arange(csr.n), np.diff(csr.row_ptr))
    c = csr.col_idx.astype(np.int64)
    lo, hi = np.minimum(r, c), np.maximum(r, c)
    w = (1.0 + ((lo * 7 + hi * 13) % 10) / 4.0).astype(np.float32)   # symmetric by construction
    for lap in (S.SLAQ_LAP_NORMALIZED, S.SLAQ_LAP_COMBINATORIAL):
        gpu = gpu_run(csr, 20, 12, 9, T256, laplacian=lap, weights=w)
        ora = oracle_run(csr, 20, 12, 9, T256, laplacian=lap, weights=w.astype(np.float64))
        assert np.array_equal(gpu["steps"], ora["steps"])
        assert_signature_parity(gpu, ora, csr.n, f"weighted lap={lap}")


def test_ritz_against_lapack_on_oracle_tridiagonals():
    # the eigensolve alone, fed with the oracle's alpha/beta
    header("ritz on oracle tridiagonals")
    csr = inputs.chung_lu(2000, 8000, 2.5, seed=2)
    for m in (5, 15, 40, 64):
        ora = oracle_run(csr, 33, m, 1, T256[:4])
        a = torch.from_numpy(ora["alpha"]).cuda()
        b = torch.from_numpy(ora["beta"]).cuda()
        s = torch.from_numpy(ora["steps"]).cuda()
        th, w2 = S.ritz(a, b, s)
        th, w2 = th.cpu().numpy(), w2.cpu().numpy()
        for p in range(33):
            k = ora["steps"][p]
            np.testing.assert_allclose(np.sort(th[p, :k]), np.sort(ora["theta"][p, :k]), atol=1e-12)
            assert abs(w2[p].sum() - 1.0) < 1e-12
            for tt in (0.1, 1.0, 10.0):
                g1 = np.sum(w2[p] * np.exp(-tt * th[p]))
                g0 = np.sum(ora["tau2"][p] * np.exp(-tt * ora["theta"][p]))
                assert abs(g1 - g0) < 1e-12


def test_quadrature_alone_on_oracle_nodes():
    header("signature/vnge on oracle nodes")
    csr = inputs.chung_lu(1500, 6000, 2.5, seed=6)
    ora = oracle_run(csr, 25, 15, 3, T256)
    th = torch.from_numpy(ora["theta"]).cuda()
    w2 = torch.from_numpy(ora["tau2"]).cuda()
    tt = torch.from_numpy(T256).cuda()
    heat = S.signature(th, w2, csr.n, tt, S.SLAQ_SIG_HEAT).cpu().numpy()
    wave = S.signature(th, w2, csr.n, tt, S.SLAQ_SIG_WAVE).cpu().numpy()
    np.testing.assert_allclose(heat, ora["heat"], rtol=1e-13)
    np.testing.assert_allclose(wave, ora["wave"], rtol=0, atol=1e-11 * csr.n)
    rp, ci = S.to_device(csr)
    g = S.build_graph(rp, ci)
    H = S.vnge(g, th, w2).cpu().numpy()[0]
    assert abs(H - ora["vnge"]) <= 1e-13 * abs(ora["vnge"])


def test_maximum_probe_and_step_counts():
    # nv = SLAQ_MAX_PROBES, m = SLAQ_MAX_STEPS, with isolated nodes; FP32
    # vectors in caller order, FP64 vectors relabelled.  Without
    # reorthogonalisation the coefficients after the first Ritz values
    # converge carry amplified rounding (an FP32 emulation of this recurrence
    # on the CPU differs from the FP64 one by 1e-5 at step 16 and by 35% at
    # step 24), while the Gauss rules they define stay equivalent: the
    # coefficients are compared over the first 12 steps, the signatures in full.
    nv, m = S.SLAQ_MAX_PROBES, S.SLAQ_MAX_STEPS
    header(f"Chung-Lu n=1000 nv={nv} m={m}")
    csr = inputs.chung_lu(1000, 4000, 2.4, seed=64)
    assert np.any(np.diff(csr.row_ptr) == 0)
    ora = oracle_run(csr, nv, m, 7, T256)
    for prec, relabel, tol in ((S.SLAQ_PREC_FP32, False, 1e-4), (S.SLAQ_PREC_FP64, True, 1e-9)):
        print(f"precision {prec} relabel {relabel}", flush=True)
        gpu = gpu_run(csr, nv, m, 7, T256, relabel=relabel, precision=prec)
        assert np.array_equal(gpu["steps"], ora["steps"])
        np.testing.assert_allclose(gpu["alpha"][:, :12], ora["alpha"][:, :12], rtol=tol, atol=tol * 1e-2)
        np.testing.assert_allclose(gpu["beta"][:, :12], ora["beta"][:, :12], rtol=tol, atol=tol * 1e-2)
        rh, rw = assert_signature_parity(gpu, ora, csr.n, f"max sizes prec={prec}")
        print(f"heat rel {rh:.2e} wave |d|/n {rw:.2e}", flush=True)
        np.testing.assert_allclose(gpu["tau2"].sum(axis=1), 1.0, atol=1e-9)


def test_deterministic_bitwise():
    header("determinism")
    csr = inputs.chung_lu(10_000, 50_000, 2.5, seed=11)
    r1 = gpu_run(csr, 10, 15, 3, T256[:8])
    r2 = gpu_run(csr, 10, 15, 3, T256[:8])
    assert np.array_equal(r1["alpha"], r2["alpha"]) and np.array_equal(r1["beta"], r2["beta"])
    assert np.array_equal(r1["heat"], r2["heat"])


def test_check_flag_reports_bad_input():
    header("CHECK flag")
    csr = inputs.erdos_renyi(50, 0.2, seed=1)
    rp, ci = S.to_device(csr)
    S.build_graph(rp, ci, check=True)  # valid
    bad = ci.clone()
    bad[3] = 10_000
    with pytest.raises(S.SlaqError) as e:
        S.build_graph(rp, bad, check=True)
    assert e.value.status == 7
    # in the row of a neighbour j of node 0, replace the entry 0 by a node c
    # that j does not touch: (j,c) and (0,j) lose their mirrors
    col = csr.col_idx.copy()
    j = int(col[csr.row_ptr[1] - 1])
    rj = slice(csr.row_ptr[j], csr.row_ptr[j + 1])
    seg = col[rj].copy()
    c = max(set(range(50)) - set(seg.tolist()) - {j})
    seg[np.flatnonzero(seg == 0)[0]] = c
    seg.sort()
    col[rj] = seg
    with pytest.raises(S.SlaqError) as e:
        S.build_graph(rp, torch.from_numpy(col).cuda(), check=True)
    assert e.value.status == 2
    w = torch.ones(csr.nnz, dtype=torch.float32, device="cuda")
    w[5] = -1.0
    with pytest.raises(S.SlaqError) as e:
        S.build_graph(rp, ci, w, check=True)
    assert e.value.status in (2, 3)


def test_argument_errors_before_launch():
    header("host argument errors")
    csr = inputs.cycle(10)
    rp, ci = S.to_device(csr)
    g = S.build_graph(rp, ci)
    for nv, m in ((0, 5), (5000, 5), (4, 0), (4, 65)):  # lanczos: nv <= 4096, m <= 64
        with pytest.raises(S.SlaqError) as e:
            S.lanczos(g, nv, m, 1, workspace=torch.empty(1 << 20, dtype=torch.uint8, device="cuda"))
        assert e.value.status == 1
    small = torch.empty(256, dtype=torch.uint8, device="cuda")
    with pytest.raises(S.SlaqError) as e:
        S.lanczos(g, 4, 5, 1, workspace=small)
    assert e.value.status == 4


def test_schedule_defaults_and_bounds_follow_graph_size():
    # below 2^22 stored entries: heavy rows from 32 nonzeros, pieces of 64,
    # and the scratch sized for that; above: 128 / 128 and heavy_min >= 128
    header("schedule bounds by size")
    csr = inputs.chung_lu(10_000, 50_000, 2.5, seed=4)
    g = S.build_graph(*S.to_device(csr))
    sch = g.schedule()
    assert (sch["heavy_min"], sch["piece"]) == (32, 64)
    with pytest.raises(S.SlaqError):
        g.set_schedule(16, 64)
    g.set_schedule(32, 128)
    rp, ci = inputs.rmat_device(19, seed=3)
    assert ci.numel() >= S.SLAQ_RELABEL_MIN_NNZ
    big = S.build_graph(rp, ci)
    sch = big.schedule()
    assert (sch["heavy_min"], sch["piece"]) == (128, 128)
    with pytest.raises(S.SlaqError):
        big.set_schedule(64, 128)
    big.set_schedule(256, 128)


def loop_graph(n=600, pairs=2500, loops=(0, 3, 17, 250), weight=None, seed=6):
    """Chung-Lu graph with self-loops on `loops` (symmetric by construction)."""
    csr = inputs.chung_lu(n, pairs, 2.4, seed=seed)
    r = np.r_[np.repeat(np.arange(csr.n), np.diff(csr.row_ptr)), list(loops)]
    c = np.r_[csr.col_idx.astype(np.int64), list(loops)]
    o = np.lexsort((c, r))
    rp = np.zeros(csr.n + 1, dtype=np.int64)
    np.add.at(rp, r[o] + 1, 1)
    out = inputs.CSR(n=csr.n, row_ptr=np.cumsum(rp), col_idx=c[o].astype(np.int32))
    w = None
    if weight is not None:
        w = np.ones(out.nnz, dtype=np.float32)
        rr = np.repeat(np.arange(out.n), np.diff(out.row_ptr))
        w[rr == out.col_idx] = weight
    return out, w


@pytest.mark.parametrize("lap", [S.SLAQ_LAP_NORMALIZED, S.SLAQ_LAP_COMBINATORIAL])
@pytest.mark.parametrize("weight", [None, 3.5])
def test_self_loops_trace_and_vnge(lap, weight):
    # tr L is the sum of L's diagonal (§2), so self-loops lower it; the
    # density matrix of §2.1 divides by it.  The build's trace equals the sum
    # of the dense spectrum, and VNGE matches the oracle's
    header(f"self-loops lap={lap} weight={weight}")
    from oracle import exact
    csr, w = loop_graph(weight=weight)
    gpu = gpu_run(csr, 16, 15, 5, T256, laplacian=lap, weights=w, check=True)
    ora = oracle_run(csr, 16, 15, 5, T256, laplacian=lap, weights=None if w is None else w.astype(np.float64))
    lam = exact.spectrum(ora["graph"])
    assert abs(gpu["info"]["trace"] - lam.sum()) <= 1e-6 * lam.sum()
    assert abs(ora["graph"].trace - lam.sum()) <= 1e-9 * lam.sum()
    assert np.array_equal(gpu["steps"], ora["steps"])
    assert_signature_parity(gpu, ora, csr.n, f"self-loops lap={lap}")
