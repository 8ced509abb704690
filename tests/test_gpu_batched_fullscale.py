"""The batched engine at the sizes of its two workloads, against the FP64
oracle: the whole 5,000-graph small mix of the batched benchmark (n 20-500,
nv = 20, m = 10) in one plan, with every 100th graph checked by the oracle and
every graph checked against invariants; and graphs of the learned-closure
population (n log-uniform on 10^3 - 10^5, mean degree 10, made on the device)
in the global bucket at the closure's m = 5 and the labels' m = 30."""
import numpy as np
import pytest
import torch

from oracle import slq as O
from paper_2003_01282_amd import closure as C
from paper_2003_01282_amd import inputs
from paper_2003_01282_amd import slaq as S

from gpu_helpers import TOL_HEAT_REL, TOL_VNGE_REL

pytestmark = pytest.mark.gpu

T = O.t_grid(256)


def oracle_heat_vnge(csr, nv, m, seed):
    og = O.build_graph(csr.n, csr.row_ptr, csr.col_idx)
    a, b, s = O.lanczos(og, nv, m, seed)
    th, w2 = O.ritz(a, b, s)
    return O.heat_trace(th, w2, csr.n, T), O.vnge(th, w2, csr.n, og.trace)


def check(heat_g, H_g, heat_o, H_o, label):
    rel = np.abs(heat_g - heat_o) / np.abs(heat_o)
    assert rel.max() <= TOL_HEAT_REL, (label, rel.max())
    if H_o != 0.0:
        assert abs(H_g - H_o) <= TOL_VNGE_REL * abs(H_o), label
    return rel.max()


def test_small_mix_5000_graphs():
    print("\n[gpu] batched: the 5,000-graph mix (seed 1), nv=20, m=10", flush=True)
    gs = inputs.small_graph_mix(5000, seed=1)
    union, off = inputs.disjoint_union(gs)
    b = S.batch_plan(union, off, nv=20, m=10, nt=T.size)
    t = torch.from_numpy(T).cuda()
    out = {k: v.cpu().numpy() for k, v in S.batch_run(b, 20200302, t, heat=True, vnge=True).items()}
    n = np.diff(off)
    # invariants on every graph: heat(t_0 = 0.01) within 2% of n (the spectrum
    # lies in [0, 2]), heat positive and non-increasing up to the rounding of
    # Ritz values at 0 (an FP32 recurrence leaves them within ~1e-6 of it, so
    # e^{-t theta} may grow by 1e-4 relative up to t = 100), VNGE finite and >= 0
    assert np.all(np.isfinite(out["heat"])) and np.all(out["heat"] > 0)
    assert np.all(out["heat"][:, 1:] <= out["heat"][:, :-1] * (1 + 1e-4))
    assert np.all(np.abs(out["heat"][:, 0] - n) <= 0.0201 * n)
    assert np.all(np.isfinite(out["vnge"])) and np.all(out["vnge"] >= 0)
    worst = 0.0
    for g in range(0, 5000, 100):
        ho, Ho = oracle_heat_vnge(gs[g], 20, 10, 20200302 + g)
        worst = max(worst, check(out["heat"][g], out["vnge"][g], ho, Ho, g))
    print(f"50 graphs against the oracle: worst heat rel {worst:.2e}", flush=True)


@pytest.mark.timeout(600)
def test_closure_population_global_bucket():
    print("\n[gpu] batched: closure population (n 1e3-1e5), nv=20, m=5 and m=30", flush=True)
    idx = [0, 1, 2, 5, 7, 11, 13, 17]
    dev = [inputs.closure_graph_device(i, seed=1) for i in idx]
    sizes = [C.graph_nodes(g) for g in dev]
    print(f"sizes {sizes}", flush=True)
    assert max(sizes) > 20_000 and min(sizes) < 5_000
    t = torch.from_numpy(T).cuda()
    for m in (5, 30):
        heat = C.heat_batched(dev, 20, m, t, 500).cpu().numpy()
        for k, (rp, ci) in enumerate(dev):
            csr = inputs.CSR(n=rp.numel() - 1, row_ptr=rp.cpu().numpy(), col_idx=ci.cpu().numpy())
            ho, _ = oracle_heat_vnge(csr, 20, m, 500 + k)
            check(heat[k], 0.0, ho, 0.0, (m, k, csr.n))
