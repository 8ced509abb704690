"""The single-launch Lanczos path (all m steps of §3.1's recurrence in one
kernel with device-wide barriers) against the stage kernels and the FP64
oracle on the same probes: step counts equal, coefficients and signatures at
the parity bars, run-to-run bitwise determinism, every workgroup count from
one to one per CU, and no barrier that ran out (SLAQ_STATUS_GRID)."""
import numpy as np
import pytest
import torch

from oracle import slq as O
from paper_2003_01282_amd import inputs
from paper_2003_01282_amd import slaq as S

from gpu_helpers import assert_signature_parity, oracle_run

pytestmark = pytest.mark.gpu

T = O.t_grid(64)


def run(csr, nv, m, seed, fused, laplacian=S.SLAQ_LAP_NORMALIZED, weights=None, precision=None):
    rp, ci = S.to_device(csr)
    w = None if weights is None else torch.from_numpy(np.asarray(weights, dtype=np.float32)).cuda()
    g = S.build_graph(rp, ci, w, laplacian=laplacian, relabel=False)
    if precision is not None:
        g.set_precision(precision)
    g.set_fused(fused)
    S.profile_reset()
    S.profile_enable(True)
    a, b, s = S.lanczos(g, nv, m, seed)
    torch.cuda.synchronize()
    S.profile_enable(False)
    launches = S.profile_read("lanczos_fused")[0]
    S.profile_reset()
    th, w2 = S.ritz(a, b, s)
    tt = torch.from_numpy(T).cuda()
    out = dict(alpha=a.cpu().numpy(), beta=b.cpu().numpy(), steps=s.cpu().numpy(),
               heat=S.signature(th, w2, csr.n, tt).cpu().numpy(),
               wave=S.signature(th, w2, csr.n, tt, S.SLAQ_SIG_WAVE).cpu().numpy(),
               vnge=float(S.vnge(g, th, w2).cpu().numpy()[0]), launches=launches)
    assert S.device_status(clear=True) == 0
    return out


CASES = {
    "chung_lu_c1": lambda: (inputs.chung_lu(10_000, 50_000, 2.5, seed=1), 10, 15),
    "hub_and_isolated": lambda: (inputs.chung_lu(3000, 6000, 2.1, seed=4), 7, 12),
    "star_breakdown": lambda: (inputs.star(800), 5, 10),
    "er_wide_probe_rows": lambda: (inputs.erdos_renyi(1500, 0.01, seed=2), 64, 9),
    "one_probe": lambda: (inputs.sbm(900, 3, 0.05, 0.005, seed=3), 1, 15),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_fused_matches_stage_kernels_and_oracle(case):
    csr, nv, m = CASES[case]()
    print(f"\n[gpu] fused path {case}: n={csr.n} nnz={csr.nnz} nv={nv} m={m}", flush=True)
    fu = run(csr, nv, m, 9, -1)
    st = run(csr, nv, m, 9, 0)
    assert fu["launches"] == 1 and st["launches"] == 0
    if np.all(st["steps"] == m):
        np.testing.assert_array_equal(fu["steps"], st["steps"])
    # after an exact breakdown FP32 rounding, amplified by the recurrence, can
    # sit above the threshold: either run may carry on into rounding-noise
    # directions of Gauss weight O(beta^2), so coefficients are compared up to
    # the FP64 oracle's breakdown step (and the signatures, below, at the
    # usual bars)
    # (absolute floor: FP32 rounding of an operator of spectral bound 2 over m
    # steps, 1e-8 * 2 * m)
    ora = oracle_run(csr, nv, m, 9, T)
    floor = 1e-8 * 2 * m
    for p in range(nv):
        k = int(min(fu["steps"][p], st["steps"][p], ora["steps"][p]))
        np.testing.assert_allclose(fu["alpha"][p, :k], st["alpha"][p, :k], rtol=1e-5, atol=floor)
        np.testing.assert_allclose(fu["beta"][p, :k - 1], st["beta"][p, :k - 1], rtol=1e-5, atol=floor)
    assert_signature_parity(fu, ora, csr.n, case)
    # run to run: fixed-order sums, the same bits
    again = run(csr, nv, m, 9, -1)
    for key in ("alpha", "beta", "steps"):
        np.testing.assert_array_equal(again[key], fu[key])


@pytest.mark.parametrize("blocks", [1, 3, 64, 256])
def test_fused_any_workgroup_count(blocks):
    csr = inputs.chung_lu(4000, 16_000, 2.3, seed=7)
    print(f"\n[gpu] fused path with {blocks} workgroups", flush=True)
    fu = run(csr, 12, 10, 3, blocks)
    ora = oracle_run(csr, 12, 10, 3, T)
    np.testing.assert_array_equal(fu["steps"], ora["steps"])
    assert_signature_parity(fu, ora, csr.n, f"blocks={blocks}")


@pytest.mark.parametrize("lap,prec,weighted", [(S.SLAQ_LAP_COMBINATORIAL, S.SLAQ_PREC_FP64, False),
                                               (S.SLAQ_LAP_NORMALIZED, S.SLAQ_PREC_FP64, True),
                                               (S.SLAQ_LAP_NORMALIZED, S.SLAQ_PREC_FP32, True)])
def test_fused_laplacians_precisions_weights(lap, prec, weighted):
    csr = inputs.chung_lu(2500, 9000, 2.4, seed=11)
    print(f"\n[gpu] fused path lap={lap} prec={prec} weighted={weighted}", flush=True)
    rng = np.random.default_rng(5)
    w = None
    if weighted:
        # symmetric positive weights: w_ij = f(min(i,j), max(i,j))
        rows = np.repeat(np.arange(csr.n), np.diff(csr.row_ptr))
        lo, hi = np.minimum(rows, csr.col_idx), np.maximum(rows, csr.col_idx)
        w = 0.5 + ((lo * 7919 + hi * 104729) % 1000) / 1000.0
    fu = run(csr, 16, 12, 21, -1, laplacian=lap, weights=w, precision=prec)
    ol = O.NORMALIZED if lap == S.SLAQ_LAP_NORMALIZED else O.COMBINATORIAL
    ora = oracle_run(csr, 16, 12, 21, T, laplacian=ol, weights=w)
    np.testing.assert_array_equal(fu["steps"], ora["steps"])
    if prec == S.SLAQ_PREC_FP64:
        np.testing.assert_allclose(fu["alpha"], ora["alpha"], rtol=1e-8, atol=1e-10)
    assert_signature_parity(fu, ora, csr.n, f"lap={lap}")


def test_fused_not_used_where_ineligible():
    # probe rows wider than 16 quads and relabelled graphs take the stage kernels
    csr = inputs.chung_lu(2000, 8000, 2.5, seed=2)
    print("\n[gpu] fused path eligibility", flush=True)
    assert run(csr, 65, 4, 1, -1)["launches"] == 0
    assert run(csr, 64, 4, 1, -1)["launches"] == 1
    with pytest.raises(S.SlaqError):
        rp, ci = S.to_device(csr)
        S.build_graph(rp, ci).set_fused(257)
