"""Host checks of the seeded input generators that the benchmark's stress
variants use."""
import numpy as np

from paper_2003_01282_amd import inputs


def edge_set(csr):
    r = np.repeat(np.arange(csr.n, dtype=np.int64), np.diff(csr.row_ptr))
    return set(zip(r.tolist(), csr.col_idx.astype(np.int64).tolist()))


def test_permute_is_an_isomorphism_in_csr_form():
    g = inputs.chung_lu(3000, 9000, 2.4, seed=5)
    h, p = inputs.permute(g, seed=1, return_perm=True)
    assert h.n == g.n and h.nnz == g.nnz
    assert np.array_equal(np.sort(p), np.arange(g.n))
    assert not np.array_equal(p, np.arange(g.n))
    assert edge_set(h) == {(int(p[i]), int(p[j])) for i, j in edge_set(g)}
    # degrees follow the renaming; rows stay sorted, no self-loops
    assert np.array_equal(np.diff(h.row_ptr)[p], np.diff(g.row_ptr))
    for i in range(h.n):
        row = h.col_idx[h.row_ptr[i]:h.row_ptr[i + 1]]
        assert np.all(np.diff(row) > 0) and not np.any(row == i)
    # seeded: the same seed gives the same graph, another seed another one
    h2 = inputs.permute(g, seed=1)
    assert np.array_equal(h2.row_ptr, h.row_ptr) and np.array_equal(h2.col_idx, h.col_idx)
    assert not np.array_equal(inputs.permute(g, seed=2).col_idx, h.col_idx)


def test_union_device_matches_host_union():
    # the binding's union of (row_ptr, col_idx) pairs (here on CPU tensors)
    # equals the host block-diagonal union: offsets, shifted ids, row starts
    import torch
    from paper_2003_01282_amd import slaq as S
    gs = [inputs.chung_lu(50 + 7 * i, 150, 2.5, seed=i) for i in range(5)]
    gs.insert(2, inputs.erdos_renyi(30, 0.0, seed=2))  # a graph without edges
    rp, ci, off = S.union_device([(torch.from_numpy(g.row_ptr), torch.from_numpy(g.col_idx)) for g in gs])
    u, uoff = inputs.disjoint_union(gs)
    assert ci.dtype == torch.int32 and rp.dtype == torch.int64
    assert np.array_equal(rp.numpy(), u.row_ptr) and np.array_equal(ci.numpy(), u.col_idx)
    assert np.array_equal(off, uoff)
