"""The paper's Erdos-Renyi accuracy sweep (§4, the ER figure): relative error
of SLQ against the exact spectrum (a) at n = 1000 over the density and (b)
over n at average degree 10, with the paper's defaults nv = 100, s = 10.  The
paper's claim checked here is that the error neither grows with the size nor
with the density; its comparison systems (linear interpolation, FINGER) are
not implemented here.  VNGE on L = D - A (the paper's density matrix,
FP64 vectors), the heat signature on the normalized Laplacian (relative l2
over the 256 time scales, the paper's error metric)."""
import numpy as np
import pytest
import torch

from oracle import exact, slq as O
from paper_2003_01282_amd import inputs
from paper_2003_01282_amd import slaq as S

pytestmark = pytest.mark.gpu

T256 = O.t_grid(256)
NV, M = 100, 10


def errors(csr, seed):
    rp, ci = S.to_device(csr)
    tt = torch.from_numpy(T256).cuda()
    out = {}
    # VNGE, L = D - A
    g = S.build_graph(rp, ci, laplacian=S.SLAQ_LAP_COMBINATORIAL)
    a, b, s = S.lanczos(g, NV, M, seed)
    th, w2 = S.ritz(a, b, s)
    H = float(S.vnge(g, th, w2).cpu().numpy()[0])
    ogc = O.build_graph(csr.n, csr.row_ptr, csr.col_idx, None, O.COMBINATORIAL)
    Hx = exact.exact_vnge(exact.spectrum(ogc), ogc.trace)
    out["vnge"] = abs(H - Hx) / abs(Hx)
    # heat signature, normalized L
    g = S.build_graph(rp, ci)
    a, b, s = S.lanczos(g, NV, M, seed)
    th, w2 = S.ritz(a, b, s)
    h = S.signature(th, w2, csr.n, tt).cpu().numpy()
    ogn = O.build_graph(csr.n, csr.row_ptr, csr.col_idx)
    hx = exact.exact_heat(exact.spectrum(ogn), T256)
    out["heat_l2"] = float(np.linalg.norm(h - hx) / np.linalg.norm(hx))
    return out


def test_er_density_sweep():
    print("\n[gpu] ER sweep (a): n = 1000, G(n, p)", flush=True)
    rows = []
    for p in (0.001, 0.002, 0.005, 0.01, 0.02, 0.05, 0.1):
        csr = inputs.erdos_renyi(1000, p, seed=int(p * 1e4))
        e = errors(csr, 11)
        dens = csr.nnz / (csr.n * (csr.n - 1))
        rows.append((p, dens, e["vnge"], e["heat_l2"]))
        print(f"p={p:<6} density={dens:.4g}  VNGE rel.err {e['vnge']:.3e}  heat rel-l2 {e['heat_l2']:.3e}", flush=True)
    v = np.array([r[2] for r in rows])
    h = np.array([r[3] for r in rows])
    assert v.max() <= 1e-2 and h.max() <= 1e-2
    # no growth with density: the densest half is not worse than 5x the sparsest half
    assert v[3:].mean() <= 5 * v[:3].mean() + 1e-4


def test_er_size_sweep():
    print("\n[gpu] ER sweep (b): average degree 10", flush=True)
    rows = []
    for n in (100, 300, 1000, 3000):
        csr = inputs.erdos_renyi(n, 20.0 / (n - 1), seed=n)
        e = errors(csr, 12)
        rows.append((n, e["vnge"], e["heat_l2"]))
        print(f"n={n:<6} edges={csr.nnz // 2:<7} VNGE rel.err {e['vnge']:.3e}  heat rel-l2 {e['heat_l2']:.3e}",
              flush=True)
    v = np.array([r[1] for r in rows])
    h = np.array([r[2] for r in rows])
    assert v.max() <= 1e-2 and h.max() <= 1e-2
    # no growth with n
    assert v[2:].mean() <= 5 * v[:2].mean() + 1e-4
