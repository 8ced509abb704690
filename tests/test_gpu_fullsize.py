"""Parity at full size, in the bench's launch configuration (nv = 100,
m = 15, default schedule): R-MAT scale 22 and scale 26 (about 2.1e9 stored
nonzeros, generated on the device), each on sampled probes the oracle runs
for all 15 steps, plus properties that hold at any size.  The scale-26
oracle sample needs ~45 GB of host memory and its sparse product uses every
host core."""
import math

import numpy as np
import pytest
import torch

from oracle import slq as O
from paper_2003_01282_amd import inputs
from paper_2003_01282_amd import slaq as S

pytestmark = pytest.mark.gpu

T = O.t_grid(256)


def gpu_full(rp, ci, n, nv, m, seed):
    g = S.build_graph(rp, ci)
    a, b, s = S.lanczos(g, nv, m, seed)
    th, w2 = S.ritz(a, b, s)
    tt = torch.from_numpy(T).cuda()
    heat = S.signature(th, w2, n, tt).cpu().numpy()
    wave = S.signature(th, w2, n, tt, S.SLAQ_SIG_WAVE).cpu().numpy()
    H = float(S.vnge(g, th, w2).cpu().numpy()[0])
    info = g.info()
    return (a.cpu().numpy(), b.cpu().numpy(), s.cpu().numpy(), th.cpu().numpy(), w2.cpu().numpy(), heat, wave, H,
            info)


def check_properties(n, th, w2, heat, wave, H, info):
    assert np.allclose(w2.sum(axis=1), 1.0, atol=1e-9)
    assert th.min() > -1e-6 and th.max() < 2 + 1e-6
    assert np.all(np.diff(heat) <= 1e-9 * n)
    # every isolated node keeps heat 1 for all t; the rest decays
    assert heat[-1] >= 0.9 * info["n_isolated"]
    assert np.all(np.abs(wave) <= n * (1 + 1e-9))
    assert 0 < H <= math.log(info["trace"]) + 1e-9


def compare_sampled(og, Vs, idx, m, seed, a, b, steps, th, w2, rtol_ab, trace):
    """The oracle's Lanczos on the probe columns Vs (n x len(idx), probes idx
    of the GPU run): coefficients, and every probe's heat / wave / VNGE
    quadrature (its share of eq. "slq") at the signatures' bars."""
    oa, ob, os_ = O.lanczos(og, len(idx), m, seed, probes=Vs)
    oth, ow2 = O.ritz(oa, ob, os_)
    for k, p in enumerate(idx):
        assert steps[p] == os_[k]
        np.testing.assert_allclose(a[p], oa[k], rtol=rtol_ab, atol=rtol_ab)
        np.testing.assert_allclose(b[p], ob[k], rtol=rtol_ab, atol=rtol_ab)
        q_gpu = (w2[p][None, :] * np.exp(-T[:, None] * th[p][None, :])).sum(axis=1)
        q_ora = (ow2[k][None, :] * np.exp(-T[:, None] * oth[k][None, :])).sum(axis=1)
        np.testing.assert_allclose(q_gpu, q_ora, rtol=1e-4)
        c_gpu = (w2[p][None, :] * np.cos(T[:, None] * th[p][None, :])).sum(axis=1)
        c_ora = (ow2[k][None, :] * np.cos(T[:, None] * oth[k][None, :])).sum(axis=1)
        assert np.max(np.abs(c_gpu - c_ora)) <= 1e-4  # wave: 1e-4 of w_0 (a unit probe's w_0 is 1)
        v_gpu = -np.sum(w2[p] * O.xlogx(th[p] / trace))
        v_ora = -np.sum(ow2[k] * O.xlogx(oth[k] / trace))
        assert abs(v_gpu - v_ora) <= 1e-4 * abs(v_ora)
    return oa, ob


def test_rmat22_bench_configuration_sampled_probes():
    print("\n[gpu] R-MAT 22, nv=100, m=15 (the bench's graph and seed)", flush=True)
    csr = inputs.rmat(22, seed=1)
    nv, m, seed = 100, 15, 20200302
    rp, ci = S.to_device(csr)
    a, b, s, th, w2, heat, wave, H, info = gpu_full(rp, ci, csr.n, nv, m, seed)
    check_properties(csr.n, th, w2, heat, wave, H, info)
    assert info["n_isolated"] == int(np.count_nonzero(np.diff(csr.row_ptr) == 0))
    og = O.build_graph(csr.n, csr.row_ptr, csr.col_idx)
    idx = [0, 57, 99]
    Vs = O.rademacher(csr.n, nv, seed, columns=idx)
    compare_sampled(og, Vs, idx, m, seed, a, b, s, th, w2, 1e-4, info["trace"])


@pytest.mark.timeout(1500)
def test_rmat26_bench_configuration_sampled_probes():
    # the bench's headline configuration: the graph is generated on the device,
    # the GPU runs all 100 probes for 15 steps; the oracle repeats two of them
    # (one per 64-probe word) for all 15 steps on a host copy, its sparse
    # product on every host core (torch CPU CSR)
    import time
    print("\n[gpu] R-MAT 26, nv=100, m=15 (the bench's graph and seed)", flush=True)
    t0 = time.perf_counter()
    rp, ci = inputs.rmat_device(26, seed=1)
    n = rp.numel() - 1
    print(f"n={n} nnz={ci.numel()} generated in {time.perf_counter() - t0:.1f} s", flush=True)
    nv, m, seed = 100, 15, 20200302
    a, b, s, th, w2, heat, wave, H, info = gpu_full(rp, ci, n, nv, m, seed)
    check_properties(n, th, w2, heat, wave, H, info)
    row_ptr = rp.cpu().numpy()
    col = ci.cpu().numpy()
    del rp, ci
    torch.cuda.empty_cache()
    t0 = time.perf_counter()
    og = O.build_graph(n, row_ptr, col, backend="torch")
    del col
    assert og.n_isolated == info["n_isolated"] and abs(og.trace - info["trace"]) <= 1e-9 * og.trace
    print(f"oracle graph in {time.perf_counter() - t0:.1f} s ({torch.get_num_threads()} threads)", flush=True)
    t0 = time.perf_counter()
    idx = [0, 99]
    Vs = O.rademacher(n, nv, seed, columns=idx)
    compare_sampled(og, Vs, idx, m, seed, a, b, s, th, w2, 1e-4, info["trace"])
    print(f"oracle Lanczos (2 probes, 15 steps) in {time.perf_counter() - t0:.1f} s", flush=True)
