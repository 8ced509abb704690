"""The first Lanczos step's gathers from compact sign records (the first basis
block of §3.1's recurrence is Rademacher signs times one scale per row)
against the same step gathering the vector rows: alpha, beta and step counts
bit-identical, for both Laplacians, FP32 and FP64 vectors, weights, caller
order and relabelled graphs with heavy rows, probe counts whose records take
8 to 64 bytes, and isolated nodes; and the default path against the oracle."""
import numpy as np
import pytest
import torch

from paper_2003_01282_amd import inputs
from paper_2003_01282_amd import slaq as S

from gpu_helpers import assert_signature_parity, gpu_run, oracle_run

pytestmark = pytest.mark.gpu


def with_isolated(csr, n_iso, seed=0):
    rng = np.random.default_rng(seed)
    n = csr.n + n_iso
    new_id = np.sort(rng.choice(n, csr.n, replace=False))
    lens = np.zeros(n, dtype=np.int64)
    lens[new_id] = np.diff(csr.row_ptr)
    rp = np.zeros(n + 1, dtype=np.int64)
    rp[1:] = np.cumsum(lens)
    return inputs.CSR(n=n, row_ptr=rp, col_idx=new_id[csr.col_idx].astype(np.int32))


def coeffs(csr, nv, m, seed, sign_step, laplacian, relabel, precision=None, weights=None):
    rp, ci = S.to_device(csr)
    w = None if weights is None else torch.from_numpy(np.asarray(weights, dtype=np.float32)).cuda()
    g = S.build_graph(rp, ci, w, laplacian=laplacian, relabel=relabel)
    if precision is not None:
        g.set_precision(precision)
    g.set_fused(0)  # the stage kernels (the single launch has no separate first step)
    g.set_sign_step(sign_step)
    a, b, s = S.lanczos(g, nv, m, seed)
    torch.cuda.synchronize()
    assert S.device_status(clear=True) == 0
    return a.cpu().numpy(), b.cpu().numpy(), s.cpu().numpy()


CASES = {
    "rmat14_relabel_nv100": lambda: (inputs.rmat(14, seed=3), 100, 8, True),
    "rmat14_caller_nv20": lambda: (inputs.rmat(14, seed=5), 20, 6, False),
    "chung_lu_iso_nv130": lambda: (with_isolated(inputs.chung_lu(4000, 16000, 2.2, seed=7), 500), 130, 5, True),
    "star_nv300": lambda: (inputs.star(2000), 300, 4, True),
    "er_nv1": lambda: (inputs.erdos_renyi(2000, 0.004, seed=2), 1, 10, False),
    "sbm_nv64": lambda: (inputs.sbm(1500, 3, 0.02, 0.002, seed=3), 64, 7, True),
}


@pytest.mark.parametrize("lap", [S.SLAQ_LAP_NORMALIZED, S.SLAQ_LAP_COMBINATORIAL])
@pytest.mark.parametrize("case", sorted(CASES))
def test_sign_records_bit_identical(case, lap):
    csr, nv, m, relabel = CASES[case]()
    print(f"\n[gpu] sign step {case} lap={lap}: n={csr.n} nnz={csr.nnz} nv={nv} m={m}", flush=True)
    for prec in (S.SLAQ_PREC_FP32, S.SLAQ_PREC_FP64):
        on = coeffs(csr, nv, m, 11, True, lap, relabel, prec)
        off = coeffs(csr, nv, m, 11, False, lap, relabel, prec)
        for x, y, name in zip(on, off, ("alpha", "beta", "steps")):
            assert np.array_equal(x, y), (case, lap, prec, name)


def test_sign_records_weighted_with_heavy_rows():
    csr = with_isolated(inputs.chung_lu(6000, 40000, 2.0, seed=9), 300, seed=4)
    # symmetric weights: w(i, j) = w(j, i) from a per-pair key
    r = np.repeat(np.arange(csr.n), np.diff(csr.row_ptr))
    c = csr.col_idx.astype(np.int64)
    key = np.minimum(r, c) * csr.n + np.maximum(r, c)
    w = (0.5 + (key * 2654435761 % 1000) / 666.0).astype(np.float32)
    print(f"\n[gpu] sign step weighted: n={csr.n} nnz={csr.nnz}", flush=True)
    for lap in (S.SLAQ_LAP_NORMALIZED, S.SLAQ_LAP_COMBINATORIAL):
        on = coeffs(csr, 100, 6, 3, True, lap, True, weights=w)
        off = coeffs(csr, 100, 6, 3, False, lap, True, weights=w)
        for x, y in zip(on, off):
            assert np.array_equal(x, y), lap


def test_default_first_step_against_oracle():
    csr = inputs.rmat(13, seed=8)
    nv, m, seed = 100, 10, 21
    print(f"\n[gpu] sign step oracle parity: n={csr.n} nnz={csr.nnz}", flush=True)
    T = inputs.t_grid(64)
    gpu = gpu_run(csr, nv, m, seed, T, relabel=True)
    ora = oracle_run(csr, nv, m, seed, T)
    np.testing.assert_array_equal(gpu["steps"], ora["steps"])
    np.testing.assert_allclose(gpu["alpha"][:, 0], ora["alpha"][:, 0], rtol=1e-6, atol=1e-7)
    assert_signature_parity(gpu, ora, csr.n, "sign step rmat13")
