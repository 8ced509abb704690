"""GPU parity of the batched engine's global-workspace buckets (graphs whose
probe block does not fit in LDS): every graph against the plain GPU path and,
up to a few thousand nodes, against the FP64 oracle on that graph alone
(seed + g); LDS and global buckets in one batch; hipGraph replay; autotune."""
import numpy as np
import pytest
import torch

from oracle import slq as O
from paper_2003_01282_amd import inputs
from paper_2003_01282_amd import slaq as S

from gpu_helpers import TOL_HEAT_REL, TOL_VNGE_REL

pytestmark = pytest.mark.gpu

T = O.t_grid(256)[::4]


def with_isolated(csr, k):
    return inputs.CSR(n=csr.n + k, row_ptr=np.r_[csr.row_ptr, np.full(k, csr.nnz, dtype=np.int64)],
                      col_idx=csr.col_idx)


def mixed(seed):
    """Small graphs (LDS buckets) and graphs of 900 to 20,000 nodes (global
    buckets for nv = 20), a hub graph with isolated nodes, an edgeless one."""
    gs = [inputs.chung_lu(n, 3 * n, 2.3, seed=seed + n) for n in (40, 300, 900, 1500, 3000, 9000, 20000)]
    gs.append(with_isolated(inputs.star(2500), 700))
    gs.append(inputs.erdos_renyi(5000, 0.002, seed=seed))
    gs.append(inputs.CSR(n=1200, row_ptr=np.zeros(1201, dtype=np.int64), col_idx=np.zeros(0, dtype=np.int32)))
    return gs


@pytest.mark.parametrize("nv", [20, 6, 100, 160, 256])  # 160, 256: more probes than first-level sum slots; 256 the maximum
def test_global_buckets_against_plain_path_and_oracle(nv):
    print(f"\n[gpu] batched global buckets nv={nv}", flush=True)
    gs = mixed(5)
    union, off = inputs.disjoint_union(gs)
    m, seed = 10, 77
    b = S.batch_plan(union, off, nv=nv, m=m, nt=T.size)
    kinds = b.buckets()
    print(kinds, flush=True)
    assert any(k["in_lds"] for k in kinds) and any(not k["in_lds"] for k in kinds)
    t = torch.from_numpy(T).cuda()
    out = {k: v.cpu().numpy() for k, v in S.batch_run(b, seed, t, heat=True, vnge=True, coeffs=True).items()}
    for g, csr in enumerate(gs):
        rp, ci = S.to_device(csr)
        gr = S.build_graph(rp, ci)
        a, be, st = S.lanczos(gr, nv, m, seed + g)
        th, w2 = S.ritz(a, be, st)
        heat = S.signature(th, w2, csr.n, t).cpu().numpy()
        # the star's exact breakdown (3 distinct eigenvalues) sits in FP32
        # rounding noise, so either FP32 path may carry on past it
        if g != 7:
            assert np.array_equal(out["steps"][g], st.cpu().numpy()), g
        np.testing.assert_allclose(out["heat"][g], heat, rtol=1e-4, err_msg=f"graph {g}")
        og = O.build_graph(csr.n, csr.row_ptr, csr.col_idx)
        oa, ob, os_ = O.lanczos(og, nv, m, seed + g)
        oth, ow2 = O.ritz(oa, ob, os_)
        oh = O.heat_trace(oth, ow2, csr.n, T)
        rel = np.abs(out["heat"][g] - oh) / np.abs(oh)
        assert rel.max() <= TOL_HEAT_REL, (g, rel.max())
        H = O.vnge(oth, ow2, csr.n, og.trace)
        if H != 0.0:
            assert abs(out["vnge"][g] - H) <= TOL_VNGE_REL * abs(H), g
        else:
            assert abs(out["vnge"][g]) < 1e-12
        np.testing.assert_allclose(out["alpha"][g, :, 0], oa[:, 0], rtol=1e-6, atol=1e-7)


def test_global_buckets_graph_replay_and_autotune():
    print("\n[gpu] batched global buckets: replay and autotune", flush=True)
    gs = mixed(9)
    union, off = inputs.disjoint_union(gs)
    b = S.batch_plan(union, off, nv=20, m=8, nt=T.size)
    t = torch.from_numpy(T).cuda()
    ref = S.batch_run(b, 3, t)["heat"].cpu().numpy().copy()
    outs = {"heat": torch.empty((b.G, T.size), dtype=torch.float64, device="cuda"),
            "vnge": torch.empty(b.G, dtype=torch.float64, device="cuda")}
    for r in range(3):
        outs["heat"].fill_(-1.0)
        S.batch_run(b, 3, t, graph=True, out=outs)
        torch.cuda.synchronize()
        assert np.array_equal(outs["heat"].cpu().numpy(), ref), r
        (torch.randn(1000, device="cuda") * 2).sum().item()
    choice = S.batch_autotune(b, t, reps=2)
    print(choice, b.buckets(), flush=True)
    after = S.batch_run(b, 3, t)["heat"].cpu().numpy()
    np.testing.assert_allclose(after, ref, rtol=1e-6)


def test_caller_workspace():
    print("\n[gpu] batched global bucket: caller-owned workspace", flush=True)
    gs = mixed(13)
    union, off = inputs.disjoint_union(gs)
    t = torch.from_numpy(T).cuda()
    b = S.batch_plan(union, off, nv=20, m=6, nt=T.size)
    need = b.workspace_bytes()
    assert need > 0
    own = S.batch_run(b, 21, t)["heat"].cpu().numpy()
    with pytest.raises(S.SlaqError):
        b.set_workspace(S._empty_aligned(need // 2, "cuda"))
    b.set_workspace(S._empty_aligned(need, "cuda"))
    np.testing.assert_array_equal(S.batch_run(b, 21, t)["heat"].cpu().numpy(), own)
    # small graphs only: no global bucket, no workspace
    small = inputs.small_graph_mix(20, seed=4)
    u2, o2 = inputs.disjoint_union(small)
    assert S.batch_plan(u2, o2, nv=20, m=6, nt=T.size).workspace_bytes() == 0


def test_long_recurrence_lds_and_global():
    # m = 40 (the eigensolve's wide-m configuration), graphs in an LDS bucket
    # and in the global one; no breakdown on these sizes, so step counts match
    print("\n[gpu] batched m=40", flush=True)
    gs = [inputs.chung_lu(n, 4 * n, 2.4, seed=n) for n in (300, 900, 3000)]
    union, off = inputs.disjoint_union(gs)
    nv, m, seed = 12, 40, 5
    b = S.batch_plan(union, off, nv=nv, m=m, nt=T.size)
    kinds = b.buckets()
    assert any(k["in_lds"] for k in kinds) and any(not k["in_lds"] for k in kinds)
    t = torch.from_numpy(T).cuda()
    out = {k: v.cpu().numpy() for k, v in S.batch_run(b, seed, t, heat=True, vnge=True, coeffs=True).items()}
    for g, csr in enumerate(gs):
        rp, ci = S.to_device(csr)
        a, be, st = S.lanczos(S.build_graph(rp, ci), nv, m, seed + g)
        th, w2 = S.ritz(a, be, st)
        heat = S.signature(th, w2, csr.n, t).cpu().numpy()
        assert np.array_equal(out["steps"][g], st.cpu().numpy()), g
        np.testing.assert_allclose(out["heat"][g], heat, rtol=1e-4, err_msg=f"graph {g}")
        og = O.build_graph(csr.n, csr.row_ptr, csr.col_idx)
        oa, ob, os_ = O.lanczos(og, nv, m, seed + g)
        oth, ow2 = O.ritz(oa, ob, os_)
        oh = O.heat_trace(oth, ow2, csr.n, T)
        assert (np.abs(out["heat"][g] - oh) / np.abs(oh)).max() <= TOL_HEAT_REL, g
        np.testing.assert_allclose(out["alpha"][g, :, :3], oa[:, :3], rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("nv", [20, 6, 100, 256])
def test_global_buckets_sign_records_bit_identical(nv):
    """The global buckets' first step from sign records against the same step
    gathering the rows of X_1: every coefficient, step count and output equal
    bit for bit (edgeless, isolated-node and hub members included), also as a
    replayed hipGraph captured before the setting changed."""
    print(f"\n[gpu] batched global sign records nv={nv}", flush=True)
    gs = mixed(9)
    union, off = inputs.disjoint_union(gs)
    b = S.batch_plan(union, off, nv=nv, m=8, nt=T.size)
    t = torch.from_numpy(T).cuda()
    runs = {}
    for on in (True, False):
        b.set_sign_step(on)
        o = S.batch_run(b, 31, t, heat=True, vnge=True, coeffs=True)
        torch.cuda.synchronize()
        runs[on] = {k: v.cpu().numpy() for k, v in o.items()}
    for k in runs[True]:
        assert np.array_equal(runs[True][k], runs[False][k]), k
    # a graph captured with the rows, then the setting flipped: the replay follows it
    cap = S.batch_run(b, 31, t, graph=True)
    torch.cuda.synchronize()
    b.set_sign_step(True)
    rep = S.batch_run(b, 31, t, graph=True)
    torch.cuda.synchronize()
    assert np.array_equal(rep["heat"].cpu().numpy(), runs[True]["heat"])
    assert np.array_equal(cap["heat"].cpu().numpy(), runs[False]["heat"])
