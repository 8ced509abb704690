"""CPU checks of the relabelling reference (tests/relabel_ref.py): the bucket
rule, a permutation of the nodes that keeps the graph, the degree order, the
dealing over column ranges and the range-partitioned rows."""
import numpy as np

from paper_2003_01282_amd import inputs
from relabel_ref import N_BUCKETS, RANGES, degree_bucket, range_base, relabel


def test_bucket_rule():
    d = np.arange(0, 1024)
    assert np.array_equal(degree_bucket(d), d)
    assert degree_bucket([1024, 1087, 1088, 2047, 2048])[:].tolist() == [1024, 1024, 1025, 1039, 1040]
    big = np.unique(np.r_[np.arange(1, 200_000), (1 << np.arange(11, 31)) - 1, 1 << np.arange(11, 31)])
    b = degree_bucket(big)
    assert np.all(np.diff(b) >= 0)
    assert degree_bucket([2**31 - 1])[0] == N_BUCKETS - 1


def test_range_bases():
    for n_act in (0, 1, 5, 8, 9, 15, 16, 1001):
        base = range_base(np.arange(RANGES + 1), n_act)
        assert base[0] == 0 and base[-1] == n_act
        sizes = np.diff(base)
        assert sizes.max() - sizes.min() <= 1


def test_relabel_is_a_graph_isomorphism():
    csr = inputs.chung_lu(3000, 9000, 2.3, seed=3)  # has isolated nodes
    w = np.random.default_rng(0).uniform(0.5, 2.0, csr.nnz).astype(np.float32)
    R = relabel(csr.row_ptr, csr.col_idx, w)
    n = csr.n
    lens = np.diff(csr.row_ptr)
    assert R["n_rows"] == int(np.count_nonzero(lens))
    assert np.array_equal(np.sort(R["perm"]), np.arange(n))
    assert np.array_equal(R["inv"][R["perm"]], np.arange(n))
    # labels below n_rows: non-isolated, dealt round-robin from the degree order
    nr = R["n_rows"]
    assert np.all(lens[R["perm"][:nr]] > 0) and np.all(lens[R["perm"][nr:]] == 0)
    keys = degree_bucket(lens)
    rank_of_label = np.empty(nr, dtype=np.int64)
    for x in range(RANGES):
        lo, hi = R["bounds"][x], R["bounds"][x + 1]
        rank_of_label[lo:hi] = x + RANGES * np.arange(hi - lo)
    by_rank = np.empty(nr, dtype=np.int64)
    by_rank[rank_of_label] = R["perm"][:nr]
    assert np.all(np.diff(keys[by_rank]) <= 0)
    # same edge set (and weights) under the map
    r_old = np.repeat(np.arange(n), lens)
    e_old = sorted(zip(R["inv"][r_old].tolist(), R["inv"][csr.col_idx].tolist(), w.tolist()))
    l2 = np.diff(R["row_ptr"])
    r_new = np.repeat(np.arange(n), l2)
    e_new = sorted(zip(r_new.tolist(), R["col_idx"].tolist(), R["weights"].tolist()))
    assert e_old == e_new
    # rows list their entries range by range
    for r in range(0, nr, 37):
        c = R["col_idx"][R["row_ptr"][r]:R["row_ptr"][r + 1]]
        x = np.searchsorted(R["bounds"][1:RANGES], c, side="right")
        assert np.all(np.diff(x) >= 0)
    # near-equal nonzero mass per column range
    mass = np.array([l2[R["bounds"][x]:R["bounds"][x + 1]].sum() for x in range(RANGES)])
    assert mass.max() <= 1.25 * mass.mean()
