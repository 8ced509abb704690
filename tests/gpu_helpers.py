"""Shared helpers of the GPU tests: run the HIP path through the binding and
the oracle on the same inputs, and compare with the stated tolerances."""
import numpy as np
import torch

from oracle import slq as O
from paper_2003_01282_amd import slaq as S

# GPU (FP32 vectors, FP64 reductions) vs FP64 oracle on the same probes
TOL_HEAT_REL = 1e-4      # per entry, relative
TOL_VNGE_REL = 1e-4      # relative
TOL_WAVE_ABS_N = 1e-4    # |gpu - oracle| <= 1e-4 * n (w_t crosses zero)


def gpu_run(csr, nv, m, seed, t, laplacian=S.SLAQ_LAP_NORMALIZED, weights=None, check=True, relabel=None,
            precision=None):
    rp, ci = S.to_device(csr)
    w = None if weights is None else torch.from_numpy(np.asarray(weights, dtype=np.float32)).cuda()
    g = S.build_graph(rp, ci, w, laplacian=laplacian, check=check, relabel=relabel)
    if precision is not None:
        g.set_precision(precision)
    a, b, s = S.lanczos(g, nv, m, seed)
    th, w2 = S.ritz(a, b, s)
    tt = torch.from_numpy(np.asarray(t, dtype=np.float64)).cuda()
    heat = S.signature(th, w2, csr.n, tt, S.SLAQ_SIG_HEAT)
    wave = S.signature(th, w2, csr.n, tt, S.SLAQ_SIG_WAVE)
    H = S.vnge(g, th, w2)
    torch.cuda.synchronize()
    out = dict(alpha=a.cpu().numpy(), beta=b.cpu().numpy(), steps=s.cpu().numpy(), theta=th.cpu().numpy(),
               tau2=w2.cpu().numpy(), heat=heat.cpu().numpy(), wave=wave.cpu().numpy(),
               vnge=float(H.cpu().numpy()[0]), info=g.info(), dinv=g.dinv.cpu().numpy())
    return out


def oracle_run(csr, nv, m, seed, t, laplacian=O.NORMALIZED, weights=None):
    g = O.build_graph(csr.n, csr.row_ptr, csr.col_idx, weights, laplacian)
    a, b, s = O.lanczos(g, nv, m, seed)
    th, w2 = O.ritz(a, b, s)
    return dict(graph=g, alpha=a, beta=b, steps=s, theta=th, tau2=w2,
                heat=O.heat_trace(th, w2, csr.n, t), wave=O.wave_trace(th, w2, csr.n, t),
                vnge=O.vnge(th, w2, csr.n, g.trace))


def assert_signature_parity(gpu, ora, n, label=""):
    # identical entries (a heat trace that underflowed to 0 on both sides) count as exact
    same = gpu["heat"] == ora["heat"]
    rel = np.where(same, 0.0, np.abs(gpu["heat"] - ora["heat"]) / np.where(same, 1.0, np.abs(ora["heat"])))
    assert rel.max() <= TOL_HEAT_REL, f"{label} heat rel {rel.max():.3e}"
    dw = np.abs(gpu["wave"] - ora["wave"]).max() / n
    assert dw <= TOL_WAVE_ABS_N, f"{label} wave |d|/n {dw:.3e}"
    if ora["vnge"] != 0.0:
        rv = abs(gpu["vnge"] - ora["vnge"]) / abs(ora["vnge"])
        assert rv <= TOL_VNGE_REL, f"{label} vnge rel {rv:.3e}"
    else:
        assert abs(gpu["vnge"]) < 1e-12
    return rel.max(), dw
