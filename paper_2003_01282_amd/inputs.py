"""Seeded synthetic graph workloads (shared by the tests, the benchmark and the
oracle's callers; holds none of the method's arithmetic).

All graphs are undirected and unweighted, returned as symmetric CSR with
int64 row offsets and int32 column indices, rows sorted, no self-loops and no
duplicate edges (nnz = 2|E|).  The paper measures on public graphs that are not
available here; these generators take their shapes instead:

  chung_lu  power-law expected degrees (Chung-Lu), e.g. n=1e4, 5e4 endpoint
            pairs, degree exponent 2.5;
  rmat      recursive-matrix graphs (Chakrabarti et al.), scale 22 stands in
            for LiveJournal/Orkut-sized social graphs, scale 26 for Friendster;
  er / sbm  Erdos-Renyi and stochastic block model graphs, the small-graph
            mix of the batched workload (tens to hundreds of nodes, like the
            graph-classification collections the paper uses).
"""
from dataclasses import dataclass

import numpy as np


@dataclass
class CSR:
    n: int
    row_ptr: np.ndarray   # int64[n+1]
    col_idx: np.ndarray   # int32[nnz]

    @property
    def nnz(self):
        return int(self.row_ptr[-1])


def t_grid(nt=256, lo=-2.0, hi=2.0):
    """Workload time scales t_k = 10^(lo + (hi-lo) k/(nt-1)), log-spaced
    (1e-2 .. 1e2 by default)."""
    k = np.arange(nt, dtype=np.float64)
    return 10.0 ** (lo + (hi - lo) * k / max(nt - 1, 1))


def csr_from_pairs(n, u, v):
    """Undirected pairs (any order, duplicates and self-loops allowed) ->
    symmetric CSR without self-loops or duplicates."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    lo = np.minimum(u, v)
    hi = np.maximum(u, v)
    key = np.unique(lo * n + hi)
    lo = key // n
    hi = key - lo * n
    del key
    both = np.concatenate([lo * n + hi, hi * n + lo])
    del lo, hi
    both.sort()
    rows = both // n
    cols = (both - rows * n).astype(np.int32)
    del both
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return CSR(n=n, row_ptr=row_ptr, col_idx=cols)


def _rng(seed, *stream):
    return np.random.default_rng(np.random.SeedSequence([int(seed), *[int(s) for s in stream]]))


def permute(csr, seed=0, return_perm=False):
    """The same graph under a seeded uniformly random renaming of its nodes
    (node i becomes p[i]): the stress input for layouts that lean on the
    generator's id order.  With return_perm, also p."""
    p = _rng(seed, 9).permutation(csr.n).astype(np.int64)
    rows = p[np.repeat(np.arange(csr.n, dtype=np.int64), np.diff(csr.row_ptr))]
    key = rows * csr.n + p[csr.col_idx]
    del rows
    key.sort()
    r = key // csr.n
    cols = (key - r * csr.n).astype(np.int32)
    del key
    row_ptr = np.zeros(csr.n + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=csr.n), out=row_ptr[1:])
    out = CSR(n=csr.n, row_ptr=row_ptr, col_idx=cols)
    return (out, p) if return_perm else out


def chung_lu(n, n_pairs, gamma=2.5, seed=0):
    """Chung-Lu power-law graph: node i has weight (i+1)^(-1/(gamma-1)); each of
    n_pairs endpoint pairs draws both ends independently with probability
    proportional to weight; self-loops and duplicates are dropped."""
    rng = _rng(seed, 1)
    w = (np.arange(n, dtype=np.float64) + 1.0) ** (-1.0 / (gamma - 1.0))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    u = np.searchsorted(cdf, rng.random(n_pairs), side="right")
    v = np.searchsorted(cdf, rng.random(n_pairs), side="right")
    return csr_from_pairs(n, np.minimum(u, n - 1), np.minimum(v, n - 1))


def rmat(scale, edge_factor=16, a=0.57, b=0.19, c=0.19, seed=0):
    """R-MAT graph on n = 2^scale nodes from edge_factor * n edge samples.
    At every level the quadrant is (0,0), (0,1), (1,0), (1,1) with
    probabilities a, b, c, 1-a-b-c; no noise, ids not permuted."""
    rng = _rng(seed, 2)
    n = 1 << scale
    e = edge_factor * n
    src = np.zeros(e, dtype=np.int64)
    dst = np.zeros(e, dtype=np.int64)
    ab, abc = a + b, a + b + c
    for _ in range(scale):
        r = rng.random(e, dtype=np.float32)
        src <<= 1
        dst <<= 1
        src += r >= ab
        dst += ((r >= a) & (r < ab)) | (r >= abc)
        del r
    return csr_from_pairs(n, src, dst)


def erdos_renyi(n, p, seed=0):
    """G(n, p).  Exact Bernoulli draws on the upper triangle for n <= 4096;
    above that, Binomial(n(n-1)/2, p) uniform pairs (duplicates dropped)."""
    rng = _rng(seed, 3)
    if n <= 4096:
        iu, ju = np.triu_indices(n, 1)
        keep = rng.random(iu.size) < p
        return csr_from_pairs(n, iu[keep], ju[keep])
    m = rng.binomial(n * (n - 1) // 2, p)
    return csr_from_pairs(n, rng.integers(0, n, m), rng.integers(0, n, m))


def sbm(n, k, p_in, p_out, seed=0):
    """Stochastic block model with k blocks, uniform random labels, edge
    probability p_in inside a block and p_out across blocks.  Exact Bernoulli
    draws for n <= 4096, block-pair Binomial sampling above."""
    rng = _rng(seed, 4)
    lab = rng.integers(0, k, n)
    if n <= 4096:
        iu, ju = np.triu_indices(n, 1)
        prob = np.where(lab[iu] == lab[ju], p_in, p_out)
        keep = rng.random(iu.size) < prob
        return csr_from_pairs(n, iu[keep], ju[keep])
    members = [np.flatnonzero(lab == b) for b in range(k)]
    us, vs = [], []
    for x in range(k):
        for y in range(x, k):
            nx, ny = members[x].size, members[y].size
            pairs = nx * (nx - 1) // 2 if x == y else nx * ny
            cnt = rng.binomial(pairs, p_in if x == y else p_out)
            us.append(members[x][rng.integers(0, max(nx, 1), cnt)])
            vs.append(members[y][rng.integers(0, max(ny, 1), cnt)])
    return csr_from_pairs(n, np.concatenate(us), np.concatenate(vs))


def complete(n):
    i, j = np.triu_indices(n, 1)
    return csr_from_pairs(n, i, j)


def cycle(n):
    i = np.arange(n)
    return csr_from_pairs(n, i, (i + 1) % n)


def path(n):
    i = np.arange(n - 1)
    return csr_from_pairs(n, i, i + 1)


def star(n):
    return csr_from_pairs(n, np.zeros(n - 1, dtype=np.int64), np.arange(1, n))


def from_edges(n, edges):
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    return csr_from_pairs(n, e[:, 0], e[:, 1])


def disjoint_union(graphs):
    """Block-diagonal union: (CSR of the union, node offsets int64[G+1])."""
    offs = np.zeros(len(graphs) + 1, dtype=np.int64)
    np.cumsum([g.n for g in graphs], out=offs[1:])
    nnz = np.zeros(len(graphs) + 1, dtype=np.int64)
    np.cumsum([g.nnz for g in graphs], out=nnz[1:])
    row_ptr = np.zeros(int(offs[-1]) + 1, dtype=np.int64)
    col = np.empty(int(nnz[-1]), dtype=np.int32)
    for k, g in enumerate(graphs):
        row_ptr[offs[k] + 1: offs[k + 1] + 1] = g.row_ptr[1:] + nnz[k]
        col[nnz[k]: nnz[k + 1]] = g.col_idx + np.int32(offs[k])
    return CSR(n=int(offs[-1]), row_ptr=row_ptr, col_idx=col), offs


def small_graph_mix(count, seed=0, n_lo=20, n_hi=500):
    """Batched workload: `count` graphs, n uniform on [n_lo, n_hi]; even
    indices Erdos-Renyi with p ~ U[0.05, 0.3], odd indices a 2-5 block SBM
    (p_in 0.3, p_out 0.02)."""
    rng = _rng(seed, 5)
    ns = rng.integers(n_lo, n_hi + 1, count)
    ps = rng.uniform(0.05, 0.3, count)
    ks = rng.integers(2, 6, count)
    out = []
    for g in range(count):
        gs = int(seed) * 1_000_003 + g
        if g % 2 == 0:
            out.append(erdos_renyi(int(ns[g]), float(ps[g]), seed=gs))
        else:
            out.append(sbm(int(ns[g]), int(ks[g]), 0.3, 0.02, seed=gs))
    return out


def closure_graph(idx, seed=0, n_lo=1_000, n_hi=100_000, mean_degree=10.0):
    """One graph of the closure's training/evaluation population: n
    log-uniform on [n_lo, n_hi]; family by idx mod 3: Chung-Lu (gamma 2.5),
    SBM (2-5 blocks, p_in/p_out = 15) or Erdos-Renyi, all with the given
    expected mean degree."""
    rng = _rng(seed, 6, idx)
    n = int(round(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi)))))
    gs = int(seed) * 7_919 + idx
    fam = idx % 3
    if fam == 0:
        return chung_lu(n, int(mean_degree * n / 2), 2.5, seed=gs)
    if fam == 1:
        k = int(rng.integers(2, 6))
        # mean degree = (n/k) p_in + (n - n/k) p_out with p_in = 15 p_out
        p_out = mean_degree / (15.0 * n / k + (n - n / k))
        return sbm(n, k, min(15.0 * p_out, 1.0), p_out, seed=gs)
    return erdos_renyi(n, mean_degree / (n - 1), seed=gs)


# ---------------------------------------------------------------------------
# Device generators for large graph populations (same families and
# parameters as closure_graph, drawn with torch's device RNG; the graphs are
# not the same draws as the numpy generators').  Return (row_ptr int64,
# col_idx int32) device tensors.
# ---------------------------------------------------------------------------
def _csr_from_pairs_torch(n, u, v):
    import torch
    keep = u != v
    u, v = u[keep], v[keep]
    lo = torch.minimum(u, v)
    hi = torch.maximum(u, v)
    key = torch.unique(lo * n + hi)
    lo = key // n
    hi = key - lo * n
    both, _ = torch.sort(torch.cat([lo * n + hi, hi * n + lo]))
    rows = both // n
    cols = (both - rows * n).to(torch.int32)
    counts = torch.bincount(rows, minlength=n)
    row_ptr = torch.zeros(n + 1, dtype=torch.int64, device=u.device)
    row_ptr[1:] = torch.cumsum(counts, 0)
    return row_ptr, cols


def closure_graph_device(idx, seed=0, n_lo=1_000, n_hi=100_000, mean_degree=10.0, device="cuda"):
    """Device counterpart of closure_graph: n log-uniform on [n_lo, n_hi],
    family idx mod 3 (Chung-Lu gamma 2.5 / 2-5 block SBM with p_in = 15 p_out /
    Erdos-Renyi), expected mean degree `mean_degree`."""
    import torch
    rng = _rng(seed, 7, idx)
    n = int(round(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi)))))
    gen = torch.Generator(device=device)
    gen.manual_seed(int(rng.integers(0, 2**62)))
    fam = idx % 3
    if fam == 0:
        w = (torch.arange(n, dtype=torch.float64, device=device) + 1.0) ** (-1.0 / 1.5)
        cdf = torch.cumsum(w, 0)
        cdf /= cdf[-1].clone()
        m = int(mean_degree * n / 2)
        u = torch.searchsorted(cdf, torch.rand(m, dtype=torch.float64, device=device, generator=gen), right=True)
        v = torch.searchsorted(cdf, torch.rand(m, dtype=torch.float64, device=device, generator=gen), right=True)
        return _csr_from_pairs_torch(n, u.clamp_(max=n - 1), v.clamp_(max=n - 1))
    if fam == 2:
        m = int(rng.binomial(n * (n - 1) // 2, mean_degree / (n - 1)))
        u = torch.randint(0, n, (m,), device=device, generator=gen)
        v = torch.randint(0, n, (m,), device=device, generator=gen)
        return _csr_from_pairs_torch(n, u, v)
    k = int(rng.integers(2, 6))
    p_out = mean_degree / (15.0 * n / k + (n - n / k))
    p_in = min(15.0 * p_out, 1.0)
    lab = torch.randint(0, k, (n,), device=device, generator=gen)
    order = torch.argsort(lab)
    sizes = torch.bincount(lab, minlength=k).cpu().numpy()
    starts = np.concatenate([[0], np.cumsum(sizes)])
    us, vs = [], []
    for x in range(k):
        for y in range(x, k):
            nx, ny = int(sizes[x]), int(sizes[y])
            if nx == 0 or ny == 0:
                continue
            pairs = nx * (nx - 1) // 2 if x == y else nx * ny
            cnt = int(rng.binomial(pairs, p_in if x == y else p_out))
            iu = torch.randint(0, nx, (cnt,), device=device, generator=gen) + int(starts[x])
            iv = torch.randint(0, ny, (cnt,), device=device, generator=gen) + int(starts[y])
            us.append(order[iu])
            vs.append(order[iv])
    if not us:
        e = torch.zeros(0, dtype=torch.int64, device=device)
        return _csr_from_pairs_torch(n, e, e)
    return _csr_from_pairs_torch(n, torch.cat(us), torch.cat(vs))


def rmat_device(scale, edge_factor=16, a=0.57, b=0.19, c=0.19, seed=0, device="cuda", chunk_log2=27):
    """Device R-MAT (same recipe as rmat; torch's RNG, so not the same draws):
    n = 2^scale, edge_factor * n samples drawn in chunks of 2^chunk_log2,
    self-loops and duplicates dropped, symmetrized.  Returns (row_ptr int64,
    col_idx int32) device tensors."""
    import torch
    n = 1 << scale
    e = edge_factor * n
    gen = torch.Generator(device=device)
    gen.manual_seed(int(_rng(seed, 8).integers(0, 2**62)))
    ab, abc = a + b, a + b + c
    keys = []
    for start in range(0, e, 1 << chunk_log2):
        cnt = min(1 << chunk_log2, e - start)
        src = torch.zeros(cnt, dtype=torch.int64, device=device)
        dst = torch.zeros(cnt, dtype=torch.int64, device=device)
        for _ in range(scale):
            r = torch.rand(cnt, dtype=torch.float32, device=device, generator=gen)
            src = (src << 1) | (r >= ab).to(torch.int64)
            dst = (dst << 1) | (((r >= a) & (r < ab)) | (r >= abc)).to(torch.int64)
            del r
        keep = src != dst
        lo = torch.minimum(src[keep], dst[keep])
        hi = torch.maximum(src[keep], dst[keep])
        del src, dst, keep
        keys.append(torch.unique(lo * n + hi))
        del lo, hi
    key = torch.unique(torch.cat(keys))
    del keys
    lo = key // n
    hi = key - lo * n
    del key
    both = torch.cat([lo * n + hi, hi * n + lo])
    del lo, hi
    both, _ = torch.sort(both)
    rows = both // n
    cols = (both - rows * n).to(torch.int32)
    del both
    counts = torch.bincount(rows, minlength=n)
    del rows
    row_ptr = torch.zeros(n + 1, dtype=torch.int64, device=device)
    row_ptr[1:] = torch.cumsum(counts, 0)
    return row_ptr, cols
