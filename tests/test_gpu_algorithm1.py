"""Algorithm 1's SLaQ_LSD and SLaQ_VNGE from the Lanczos coefficients
(slaq_lsd, slaq_vnge_slq: the eigensolve of §3.1, eq. "quadratic", inside)
against the two-call route (slaq_ritz, then slaq_signature / slaq_vnge) and
against the FP64 oracle on the same probes."""
import numpy as np
import pytest
import torch

from oracle import slq as O
from paper_2003_01282_amd import inputs
from paper_2003_01282_amd import slaq as S

from gpu_helpers import TOL_HEAT_REL, TOL_VNGE_REL, TOL_WAVE_ABS_N

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nv,m,nt", [(10, 15, 256), (130, 40, 70), (1, 1, 1), (64, 33, 33)])
def test_lsd_and_vnge_from_coefficients(nv, m, nt):
    print(f"\n[gpu] slaq_lsd / slaq_vnge_slq nv={nv} m={m} nt={nt}", flush=True)
    csr = inputs.chung_lu(1200, 5000, 2.5, seed=12)
    rp, ci = S.to_device(csr)
    g = S.build_graph(rp, ci)
    if m > 15:
        # beyond the FP32 configurations (m = 15) the FP32 recurrence, run
        # without reorthogonalization, drifts from the FP64 one (ghost Ritz
        # values), and cos(t theta) at t = 100 magnifies that drift t-fold:
        # the long recurrences compare with FP64 vectors
        g.set_precision(S.SLAQ_PREC_FP64)
    a, b, s = S.lanczos(g, nv, m, seed=77)
    t = O.t_grid(nt) if nt > 1 else np.array([0.3])
    tt = torch.from_numpy(t).cuda()
    heat = S.lsd(a, b, s, csr.n, tt).cpu().numpy()
    wave = S.lsd(a, b, s, csr.n, tt, S.SLAQ_SIG_WAVE).cpu().numpy()
    tr = g.info()["trace"]
    H = float(S.vnge_slq(a, b, s, csr.n, tr).cpu().numpy()[0])
    th, w2 = S.ritz(a, b, s)
    heat2 = S.signature(th, w2, csr.n, tt).cpu().numpy()
    wave2 = S.signature(th, w2, csr.n, tt, S.SLAQ_SIG_WAVE).cpu().numpy()
    H2 = float(S.vnge(g, th, w2).cpu().numpy()[0])
    # same eigensolves, other summation order
    np.testing.assert_allclose(heat, heat2, rtol=1e-12)
    np.testing.assert_allclose(wave, wave2, rtol=1e-12, atol=1e-12 * csr.n)
    assert abs(H - H2) <= 1e-12 * abs(H2)
    og = O.build_graph(csr.n, csr.row_ptr, csr.col_idx)
    oa, ob, os_ = O.lanczos(og, nv, m, 77)
    oth, ow2 = O.ritz(oa, ob, os_)
    oh = O.heat_trace(oth, ow2, csr.n, t)
    ow = O.wave_trace(oth, ow2, csr.n, t)
    oH = O.vnge(oth, ow2, csr.n, og.trace)
    assert np.max(np.abs(heat - oh) / np.abs(oh)) <= TOL_HEAT_REL
    assert np.max(np.abs(wave - ow)) / csr.n <= TOL_WAVE_ABS_N
    assert abs(H - oH) / abs(oH) <= TOL_VNGE_REL
    assert S.device_status(clear=True) == 0


def test_hutchinson_mean_of_per_probe_values():
    # eq. "trace": n_g / nv times the sum over the graph's probes, per time
    print("\n[gpu] slaq_hutchinson_mean, 7 graphs x 9 probes x 33 times", flush=True)
    rng = np.random.default_rng(4)
    G, nv, nt = 7, 9, 33
    q = rng.random((G * nv, nt))
    gn = rng.integers(10, 10_000, G)
    heat = S.hutchinson_mean(torch.from_numpy(q).cuda(), torch.from_numpy(gn).cuda(), nv).cpu().numpy()
    ref = q.reshape(G, nv, nt).sum(axis=1) * (gn / nv)[:, None]
    np.testing.assert_allclose(heat, ref, rtol=1e-14)
