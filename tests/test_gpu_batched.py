"""GPU parity of the batched engine: every graph of a batch against the FP64
oracle run on that graph alone (seed + g), against the plain GPU path, and
hipGraph replays against the eager launch."""
import numpy as np
import pytest
import torch

from oracle import slq as O
from paper_2003_01282_amd import inputs
from paper_2003_01282_amd import slaq as S

from gpu_helpers import TOL_HEAT_REL, TOL_VNGE_REL

pytestmark = pytest.mark.gpu

T = O.t_grid(256)


def mixed_batch(count, seed):
    gs = inputs.small_graph_mix(count, seed=seed)
    # degenerate members: a single node, no edges, a complete graph, a star,
    # a star followed by isolated nodes (rows with and without edges mixed)
    gs[3] = inputs.CSR(n=1, row_ptr=np.zeros(2, dtype=np.int64), col_idx=np.zeros(0, dtype=np.int32))
    gs[5] = inputs.CSR(n=9, row_ptr=np.zeros(10, dtype=np.int64), col_idx=np.zeros(0, dtype=np.int32))
    gs[7] = inputs.complete(40)
    gs[9] = inputs.star(300)
    st = inputs.star(50)
    gs[11] = inputs.CSR(n=80, row_ptr=np.r_[st.row_ptr, np.full(30, st.nnz, dtype=np.int64)], col_idx=st.col_idx)
    return gs


@pytest.fixture(scope="module")
def batch60():
    gs = mixed_batch(60, seed=8)
    union, off = inputs.disjoint_union(gs)
    b = S.batch_plan(union, off, nv=20, m=10, nt=T.size)
    t = torch.from_numpy(T).cuda()
    out = S.batch_run(b, 1234, t, heat=True, vnge=True, coeffs=True, ritz=True)
    torch.cuda.synchronize()
    return gs, b, t, {k: v.cpu().numpy() for k, v in out.items()}


def test_batched_against_oracle(batch60):
    gs, b, t, out = batch60
    print(f"\n[gpu] batched 60 graphs buckets {b.buckets()}", flush=True)
    worst = 0.0
    for g, csr in enumerate(gs):
        og = O.build_graph(csr.n, csr.row_ptr, csr.col_idx)
        a, be, st = O.lanczos(og, 20, 10, 1234 + g)
        th, w2 = O.ritz(a, be, st)
        heat = O.heat_trace(th, w2, csr.n, T)
        H = O.vnge(th, w2, csr.n, og.trace)
        rel = np.abs(out["heat"][g] - heat) / np.abs(heat)
        worst = max(worst, rel.max())
        assert rel.max() <= TOL_HEAT_REL, (g, rel.max())
        if H != 0.0:
            assert abs(out["vnge"][g] - H) <= TOL_VNGE_REL * abs(H), g
        else:
            assert abs(out["vnge"][g]) < 1e-12
        # On these small graphs Ritz values converge within m = 10 steps and the
        # later Lanczos coefficients amplify FP32 rounding (up to ~5e-5 by step
        # 5), while each probe's Gauss rule stays accurate.  Compared: the first
        # step's coefficients, and every probe's own quadrature value.
        np.testing.assert_allclose(out["alpha"][g, :, 0], a[:, 0], rtol=1e-6, atol=1e-7)
        np.testing.assert_allclose(out["beta"][g, :, 0], be[:, 0], rtol=1e-6, atol=1e-7)
        for tt in (0.1, 1.0, 10.0):
            q_gpu = (out["tau2"][g] * np.exp(-tt * out["theta"][g])).sum(axis=1)
            q_ora = (w2 * np.exp(-tt * th)).sum(axis=1)
            np.testing.assert_allclose(q_gpu, q_ora, rtol=1e-4)
    print(f"worst heat rel {worst:.2e}")


def test_batched_matches_plain_gpu_path(batch60):
    gs, b, t, out = batch60
    for g in (0, 1, 2, 7, 9, 20, 41):
        csr = gs[g]
        rp, ci = S.to_device(csr)
        gr = S.build_graph(rp, ci)
        a, be, st = S.lanczos(gr, 20, 10, 1234 + g)
        th, w2 = S.ritz(a, be, st)
        heat = S.signature(th, w2, csr.n, t).cpu().numpy()
        # two FP32 paths with different summation orders, each within 1e-4 of
        # the FP64 oracle
        np.testing.assert_allclose(out["heat"][g], heat, rtol=1e-4)


def test_hipgraph_replays_match_eager(batch60):
    gs, b, t, out = batch60
    eager = S.batch_run(b, 99, t)
    torch.cuda.synchronize()
    ref = eager["heat"].cpu().numpy().copy()
    outs = {"heat": torch.empty_like(eager["heat"]), "vnge": torch.empty_like(eager["vnge"])}
    for r in range(4):
        outs["heat"].fill_(-1.0)
        S.batch_run(b, 99, t, graph=True, out=outs)
        torch.cuda.synchronize()
        assert np.array_equal(outs["heat"].cpu().numpy(), ref), r
        # eager work between replays
        x = torch.randn(1000, device="cuda")
        (x * 2).sum().item()


def test_autotune_keeps_results():
    gs = inputs.small_graph_mix(200, seed=3)
    union, off = inputs.disjoint_union(gs)
    b = S.batch_plan(union, off, nv=20, m=10, nt=T.size)
    t = torch.from_numpy(T).cuda()
    before = S.batch_run(b, 5, t)["heat"].cpu().numpy()
    choice = S.batch_autotune(b, t, reps=2)
    print(f"\n[gpu] autotune {choice} buckets {b.buckets()}", flush=True)
    assert all(c[0] in (128, 256, 512, 1024) for c in choice)
    after = S.batch_run(b, 5, t)["heat"].cpu().numpy()
    np.testing.assert_allclose(after, before, rtol=1e-6)


def test_bucket_edge_growth_against_oracle(batch60):
    """Plans with finer and coarser LDS bucket edges (growth 1.5 and 3) and
    the edge tuner's pick: every graph still within tolerance of the oracle."""
    gs, b2, t, _ = batch60
    rp, ci = b2._keep["rp"], b2._keep["ci"]
    off = b2._keep["goff"].cpu().numpy()
    plans = {gr: S.batch_plan_device(rp, ci, off, nv=20, m=10, nt=T.size, growth=gr) for gr in (1.5, 3.0)}
    tuned, growth, ms = S.batch_autotune_edges(rp, ci, off, nv=20, m=10, nt=T.size, t=t, reps=2)
    print(f"\n[gpu] edge tuner picked growth {growth} ({ms:.3f} ms), buckets {tuned.buckets()}", flush=True)
    assert growth in (1.5, 2.0, 3.0) and ms > 0.0
    n_lds = {gr: sum(k["in_lds"] for k in p.buckets()) for gr, p in plans.items()}
    assert n_lds[1.5] >= sum(k["in_lds"] for k in b2.buckets()) >= n_lds[3.0]
    plans["tuned"] = tuned
    ref = {}
    for g, csr in enumerate(gs):
        og = O.build_graph(csr.n, csr.row_ptr, csr.col_idx)
        a, be, st = O.lanczos(og, 20, 10, 77 + g)
        th, w2 = O.ritz(a, be, st)
        ref[g] = (O.heat_trace(th, w2, csr.n, T), O.vnge(th, w2, csr.n, og.trace))
    for name, p in plans.items():
        out = S.batch_run(p, 77, t)
        torch.cuda.synchronize()
        heat, vn = out["heat"].cpu().numpy(), out["vnge"].cpu().numpy()
        for g in range(len(gs)):
            h, H = ref[g]
            assert (np.abs(heat[g] - h) / np.abs(h)).max() <= TOL_HEAT_REL, (name, g)
            assert abs(vn[g] - H) <= TOL_VNGE_REL * abs(H) + 1e-12, (name, g)


def with_loops(csr, nodes):
    r = np.r_[np.repeat(np.arange(csr.n), np.diff(csr.row_ptr)), nodes]
    c = np.r_[csr.col_idx.astype(np.int64), nodes]
    o = np.lexsort((c, r))
    rp = np.zeros(csr.n + 1, dtype=np.int64)
    np.add.at(rp, r[o] + 1, 1)
    return inputs.CSR(n=csr.n, row_ptr=np.cumsum(rp), col_idx=c[o].astype(np.int32))


def test_batched_self_loops_trace():
    # graphs with self-loops in the LDS and in the global bucket: VNGE divides
    # by tr L = sum_i (1 - A_ii / D_ii) (§2, §2.1), as the oracle does
    print("\n[gpu] batched graphs with self-loops", flush=True)
    gs = [with_loops(inputs.erdos_renyi(60, 0.1, seed=1), [0, 5, 9]),
          inputs.erdos_renyi(50, 0.1, seed=2),
          with_loops(inputs.sbm(300, 3, 0.3, 0.02, seed=3), [1, 2, 299]),
          with_loops(inputs.chung_lu(6000, 24000, 2.5, seed=4), [0, 10, 5999])]
    union, off = inputs.disjoint_union(gs)
    b = S.batch_plan(union, off, nv=20, m=10, nt=T.size)
    assert any(not bk["in_lds"] for bk in b.buckets())
    t = torch.from_numpy(T).cuda()
    out = S.batch_run(b, 55, t, heat=True, vnge=True)
    H = out["vnge"].cpu().numpy()
    for g, csr in enumerate(gs):
        og = O.build_graph(csr.n, csr.row_ptr, csr.col_idx)
        a, be, st = O.lanczos(og, 20, 10, 55 + g)
        th, w2 = O.ritz(a, be, st)
        oH = O.vnge(th, w2, csr.n, og.trace)
        assert abs(H[g] - oH) <= TOL_VNGE_REL * abs(oH), (g, H[g], oH)
