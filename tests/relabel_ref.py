"""Reference (numpy) of the graph build's node relabelling, the storage order
that slaq_build_graph documents: nodes stably ordered by decreasing row-length
bucket, isolated nodes last, rank r of the n_act non-isolated nodes at label
base(r mod 8) + r div 8 with base(x) = x q + min(x, n_act mod 8), and each
relabelled row listed column range by column range, caller order within a
range.  Index work: the HIP build must match it exactly."""
import numpy as np

N_BUCKETS = 1024 + 16 * 21
RANGES = 8


def degree_bucket(d):
    """Exact below 1024, 16 buckets per octave above (lengths < 2^31)."""
    d = np.asarray(d, dtype=np.int64)
    out = d.copy()
    big = d >= 1024
    if np.any(big):
        db = d[big]
        lg = np.floor(np.log2(db.astype(np.float64))).astype(np.int64)
        lg += ((np.int64(1) << (lg + 1)) <= db).astype(np.int64)
        lg -= ((np.int64(1) << lg) > db).astype(np.int64)
        out[big] = 1024 + 16 * (lg - 10) + ((db >> (lg - 4)) & 15)
    return out


def range_base(x, n_act):
    q, rem = divmod(n_act, RANGES)
    x = np.asarray(x, dtype=np.int64)
    return x * q + np.minimum(x, rem)


def relabel(row_ptr, col_idx, weights=None):
    """Returns dict(perm, inv, n_rows, row_ptr, col_idx, weights, bounds)."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col_idx = np.asarray(col_idx)
    n = row_ptr.size - 1
    lens = np.diff(row_ptr)
    key = (N_BUCKETS - 1) - degree_bucket(lens)
    order = np.argsort(key, kind="stable")  # rank -> caller id
    n_act = int(np.count_nonzero(lens > 0))
    r = np.arange(n, dtype=np.int64)
    label = np.where(r < n_act, range_base(r % RANGES, n_act) + r // RANGES, r)
    perm = np.empty(n, dtype=np.int64)
    perm[label] = order
    inv = np.empty(n, dtype=np.int64)
    inv[order] = label
    bounds = range_base(np.arange(RANGES + 1), n_act)
    new_lens = np.zeros(n, dtype=np.int64)
    new_lens[:n_act] = lens[perm[:n_act]]
    rp2 = np.zeros(n + 1, dtype=np.int64)
    rp2[1:] = np.cumsum(new_lens)
    # entries: new row, range of the new column, original position (stable)
    src_row = np.repeat(np.arange(n, dtype=np.int64), lens)
    c_new = inv[col_idx.astype(np.int64)]
    x = np.searchsorted(bounds[1:RANGES], c_new, side="right")
    idx = np.lexsort((np.arange(c_new.size), x, inv[src_row]))
    out = dict(perm=perm, inv=inv, n_rows=n_act, row_ptr=rp2, col_idx=c_new[idx].astype(np.int32),
               weights=None if weights is None else np.asarray(weights, dtype=np.float32)[idx], bounds=bounds)
    return out


def piece_count(rp2, col2, bounds, heavy_min, piece):
    """Heavy rows (length >= heavy_min) cut at the range bounds, then into
    pieces of at most `piece` entries."""
    lens = np.diff(rp2)
    total = 0
    for r in np.flatnonzero(lens >= heavy_min):
        cols = col2[rp2[r]:rp2[r + 1]]
        cuts = np.searchsorted(cols, bounds[1:RANGES], side="left")  # rows are range-partitioned
        seg = np.diff(np.r_[0, cuts, cols.size])
        total += int(((seg + piece - 1) // piece).sum())
    return total
