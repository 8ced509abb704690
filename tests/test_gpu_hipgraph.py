"""The plain path captured into a HIP graph: one whole step (graph build,
Lanczos, Gauss rules, heat and wave trace, VNGE) recorded on torch's capture
stream and replayed several times, with eager work and synchronizations
between replays; every replay must equal the eager step bit for bit."""
import numpy as np
import pytest
import torch

from oracle import slq as O
from paper_2003_01282_amd import inputs
from paper_2003_01282_amd import slaq as S

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("relabel", [False, True])
def test_captured_step_replays_match_eager(relabel):
    print(f"\n[gpu] hipgraph capture of one step, relabel={relabel}", flush=True)
    csr = inputs.chung_lu(10_000, 50_000, 2.5, seed=1)
    nv, m, seed = 10, 15, 5
    rp, ci = S.to_device(csr)
    t = torch.from_numpy(O.t_grid(256)).cuda()
    g0 = S.build_graph(rp, ci, relabel=relabel)
    dinv, scratch = g0.dinv, g0._keep["scratch"]
    ws = S._empty_aligned(S.lanczos_workspace(g0, nv, m), "cuda")
    f64 = dict(dtype=torch.float64, device="cuda")
    out = {"alpha": torch.empty((nv, m), **f64), "beta": torch.empty((nv, m), **f64),
           "steps": torch.empty(nv, dtype=torch.int32, device="cuda"), "theta": torch.empty((nv, m), **f64),
           "tau2": torch.empty((nv, m), **f64), "heat": torch.empty(256, **f64), "wave": torch.empty(256, **f64),
           "vnge": torch.empty(1, **f64)}
    keep = []

    def step():
        g = S.build_graph(rp, ci, dinv=dinv, scratch=scratch, relabel=relabel)
        S.lanczos(g, nv, m, seed, workspace=ws, out=(out["alpha"], out["beta"], out["steps"]))
        S.ritz(out["alpha"], out["beta"], out["steps"], out=(out["theta"], out["tau2"]))
        S.signature(out["theta"], out["tau2"], csr.n, t, S.SLAQ_SIG_HEAT, out=out["heat"])
        S.signature(out["theta"], out["tau2"], csr.n, t, S.SLAQ_SIG_WAVE, out=out["wave"])
        S.vnge(g, out["theta"], out["tau2"], out=out["vnge"])
        keep.append(g)

    step()
    torch.cuda.synchronize()
    ref = {k: v.cpu().numpy().copy() for k, v in out.items()}
    hg = torch.cuda.CUDAGraph()
    with torch.cuda.graph(hg):
        step()
    for r in range(4):
        for v in out.values():
            v.fill_(-7)
        torch.cuda.synchronize()
        hg.replay()
        torch.cuda.synchronize()
        for k, v in out.items():
            assert np.array_equal(v.cpu().numpy(), ref[k]), (r, k)
        (torch.randn(4096, device="cuda") * 3).sum().item()  # eager work between replays
    # and the eager step still agrees with the oracle on these probes
    og = O.build_graph(csr.n, csr.row_ptr, csr.col_idx)
    a, b, s = O.lanczos(og, nv, m, seed)
    th, w2 = O.ritz(a, b, s)
    heat = O.heat_trace(th, w2, csr.n, O.t_grid(256))
    assert np.max(np.abs(ref["heat"] - heat) / heat) <= 1e-4
