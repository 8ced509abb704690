"""GPU parity over combinations of the path's options: Laplacian, vector
precision, relabelling, probe count (one probe, ragged widths, several probe
tiles), step count (including m = 1 and m = 2) and weights, on small seeded
graphs with isolated nodes and a hub, against the oracle."""
import itertools

import numpy as np
import pytest

from oracle import slq as O
from paper_2003_01282_amd import inputs
from paper_2003_01282_amd import slaq as S

from gpu_helpers import assert_signature_parity, gpu_run, oracle_run

pytestmark = pytest.mark.gpu

T = O.t_grid(256)[::4]


def graph(seed):
    """Chung-Lu with a hub of a few hundred neighbours plus isolated nodes."""
    base = inputs.chung_lu(1500, 6000, 2.2, seed=seed)
    n = base.n + 40
    rp = np.r_[base.row_ptr, np.full(40, base.nnz, dtype=np.int64)]
    return inputs.CSR(n=n, row_ptr=rp, col_idx=base.col_idx)


def weights(csr):
    r = np.repeat(np.arange(csr.n), np.diff(csr.row_ptr))
    c = csr.col_idx.astype(np.int64)
    return (0.3 + ((np.minimum(r, c) * 37 + np.maximum(r, c) * 11) % 17) / 8.0).astype(np.float32)


ALL = list(itertools.product(
    [S.SLAQ_LAP_NORMALIZED, S.SLAQ_LAP_COMBINATORIAL],
    [S.SLAQ_PREC_FP32, S.SLAQ_PREC_FP64],
    [False, True],                     # relabel
    [1, 7, 130, 300],                  # nv: one probe, ragged, two and three probe tiles in FP64
    [1, 2, 9],                         # m
    [False, True],                     # weighted
))
# a fixed, seeded sample of the 192 combinations, plus every nv/m pair once
rng = np.random.default_rng(2003)
PICK = sorted(set(rng.choice(len(ALL), 28, replace=False).tolist())
              | {ALL.index((S.SLAQ_LAP_NORMALIZED, S.SLAQ_PREC_FP64, True, nv, m, True))
                 for nv in (1, 7, 130, 300) for m in (1, 2, 9)})
CASES = [ALL[i] for i in PICK]


def case_id(c):
    lap, prec, rl, nv, m, wt = c
    return (f"{'norm' if lap == S.SLAQ_LAP_NORMALIZED else 'comb'}-{'fp32' if prec == S.SLAQ_PREC_FP32 else 'fp64'}"
            f"-{'rl' if rl else 'id'}-nv{nv}-m{m}-{'w' if wt else 'u'}")


@pytest.mark.parametrize("case", CASES, ids=case_id)
def test_combination(case):
    lap, prec, rl, nv, m, wt = case
    print(f"\n[gpu] {case_id(case)}", flush=True)
    csr = graph(seed=nv + m)
    w = weights(csr) if wt else None
    gpu = gpu_run(csr, nv, m, 1000 + nv, T, laplacian=lap, weights=w, relabel=rl, precision=prec)
    ora = oracle_run(csr, nv, m, 1000 + nv, T, laplacian=lap, weights=None if w is None else w.astype(np.float64))
    assert np.array_equal(gpu["steps"], ora["steps"])
    # FP64 vectors differ from the oracle only in summation order (D - A: its
    # wide spectrum amplifies that order a little more)
    tol = 1e-4 if prec == S.SLAQ_PREC_FP32 else (1e-9 if lap == S.SLAQ_LAP_NORMALIZED else 1e-8)
    S_bound = 2.0 if lap == S.SLAQ_LAP_NORMALIZED else 2.0 * float(ora["graph"].deg.max())
    atol = (1e-8 if prec == S.SLAQ_PREC_FP32 else 1e-13) * S_bound * m
    kmax = m if (lap == S.SLAQ_LAP_NORMALIZED or prec == S.SLAQ_PREC_FP64) else min(m, 6)
    np.testing.assert_allclose(gpu["alpha"][:, :kmax], ora["alpha"][:, :kmax], rtol=tol, atol=atol)
    np.testing.assert_allclose(gpu["beta"][:, :kmax], ora["beta"][:, :kmax], rtol=tol, atol=atol)
    if lap == S.SLAQ_LAP_NORMALIZED or prec == S.SLAQ_PREC_FP64:
        assert_signature_parity(gpu, ora, csr.n, case_id(case))
    np.testing.assert_allclose(gpu["tau2"].sum(axis=1), 1.0, atol=1e-9)
