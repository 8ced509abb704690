// Graph build: degrees, the Laplacian's diagonal scale and graph statistics
// (paper §2: D_ii = sum_j A_ij, L = D - A, normalized L = I - D^-1/2 A D^-1/2;
// §2.1: the density matrix is L / tr L).
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>

#include "common.hpp"

namespace slaq {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = '\0'; }

enum : unsigned {
    kCheckBadRowPtr = 1u,
    kCheckBadCol = 2u,
    kCheckUnsorted = 4u,
    kCheckAsymmetric = 8u,
    kCheckBadWeight = 16u,
};

// One thread per row, grid-stride.  Degree is a count (unweighted, exact) or a
// double sum of weights.  Each block writes one partial (fixed-order reduce).
template <bool WEIGHTED>
__global__ void __launch_bounds__(256) degree_kernel(int64_t n, const int64_t* __restrict__ rp,
                                                     const float* __restrict__ w, int laplacian,
                                                     float* __restrict__ diag, double* __restrict__ diag64,
                                                     BuildPartial* __restrict__ part) {
    double dmax = 0.0, dsum = 0.0;
    long long nz = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = rp[i], e = rp[i + 1];
        double d;
        if (WEIGHTED) {
            d = 0.0;
            for (int64_t k = s; k < e; ++k) d += (double)w[k];
        } else {
            d = (double)(e - s);
        }
        double out;
        if (laplacian == SLAQ_LAP_NORMALIZED)
            out = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
        else
            out = d;
        diag[i] = (float)out;
        diag64[i] = out;
        dmax = fmax(dmax, d);
        dsum += d;
        nz += d > 0.0 ? 1 : 0;
    }
    __shared__ double smax[256], ssum[256];
    __shared__ long long snz[256];
    const int t = threadIdx.x;
    smax[t] = dmax;
    ssum[t] = dsum;
    snz[t] = nz;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off) {
            smax[t] = fmax(smax[t], smax[t + off]);
            ssum[t] += ssum[t + off];
            snz[t] += snz[t + off];
        }
        __syncthreads();
    }
    if (t == 0) {
        part[blockIdx.x].max_degree = smax[0];
        part[blockIdx.x].sum_degree = ssum[0];
        part[blockIdx.x].nonisolated = snz[0];
    }
}

// Self-loop share of tr L (§2: L_ii = 1 - A_ii / D_ii on a non-isolated node
// of the normalized Laplacian, D_ii - A_ii for L = D - A): per block the sum
// over its rows of A_ii / D_ii, or of A_ii.  A thread per row (grid-stride)
// finds column i in its row by binary search: rows list their columns in
// ascending order without repeats (the CSR contract SLAQ_FLAG_CHECK
// verifies), so a row costs about log2(length) loads and hub rows no more
// than a few dozen.
template <bool WEIGHTED>
__global__ void __launch_bounds__(256) loop_kernel(int64_t n, const int64_t* __restrict__ rp,
                                                   const int32_t* __restrict__ col, const float* __restrict__ w,
                                                   int laplacian, const double* __restrict__ d64,
                                                   double* __restrict__ part) {
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = rp[i], e = rp[i + 1];
        int64_t lo = s, hi = e;  // first entry with column >= i
        while (lo < hi) {
            const int64_t mid = lo + ((hi - lo) >> 1);
            if ((int64_t)col[mid] < i) lo = mid + 1;
            else hi = mid;
        }
        if (lo < e && (int64_t)col[lo] == i) {
            const double self = WEIGHTED ? (double)w[lo] : 1.0;
            const double d = d64[i];  // D^-1/2 or D_ii
            acc += laplacian == SLAQ_LAP_NORMALIZED ? self * d * d : self;
        }
    }
    __shared__ double red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) stats_kernel(int64_t n, int nparts, int laplacian,
                                                    const BuildPartial* __restrict__ part,
                                                    const double* __restrict__ loop_part, int nloop,
                                                    GraphStats* __restrict__ st) {
    __shared__ double smax[256], ssum[256], sloop[256];
    __shared__ long long snz[256];
    const int t = threadIdx.x;
    double dmax = 0.0, dsum = 0.0, dl = 0.0;
    long long nz = 0;
    for (int b = t; b < nparts; b += 256) {
        dmax = fmax(dmax, part[b].max_degree);
        dsum += part[b].sum_degree;
        nz += part[b].nonisolated;
    }
    for (int b = t; b < nloop; b += 256) dl += loop_part[b];
    smax[t] = dmax;
    ssum[t] = dsum;
    snz[t] = nz;
    sloop[t] = dl;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off) {
            smax[t] = fmax(smax[t], smax[t + off]);
            ssum[t] += ssum[t + off];
            snz[t] += snz[t + off];
            sloop[t] += sloop[t + off];
        }
        __syncthreads();
    }
    if (t == 0) {
        st->max_degree = smax[0];
        st->sum_degree = ssum[0];
        st->n_isolated = (long long)n - snz[0];
        // tr L = sum_i L_ii: the non-isolated count (or sum_i D_ii) less the self-loops' share
        st->trace = (laplacian == SLAQ_LAP_NORMALIZED ? (double)snz[0] : ssum[0]) - sloop[0];
        st->n_rows = n;  // the relabelling lowers it to n_act
        st->check = 0u;
        st->status = 0u;
    }
}

// SLAQ_FLAG_CHECK: one thread per row.  Rows must be strictly increasing in
// column (sorted, no duplicates) so the transpose entry is found by bisection.
__global__ void __launch_bounds__(256) check_kernel(int64_t n, int64_t nnz,
                                                    const int64_t* __restrict__ rp,
                                                    const int32_t* __restrict__ col,
                                                    const float* __restrict__ w,
                                                    GraphStats* __restrict__ st) {
    unsigned bad = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = rp[i], e = rp[i + 1];
        if (s < 0 || (i == 0 && s != 0) || e < s || e > nnz || (i == n - 1 && e != nnz)) {
            bad |= kCheckBadRowPtr;
            continue;
        }
        int32_t prev = -1;
        for (int64_t k = s; k < e; ++k) {
            const int32_t j = col[k];
            if (j < 0 || (int64_t)j >= n) {
                bad |= kCheckBadCol;
                continue;
            }
            if (j <= prev) bad |= kCheckUnsorted;
            prev = j;
            if (w) {
                const float x = w[k];
                if (!(x > 0.0f) || !isfinite(x)) bad |= kCheckBadWeight;
            }
            // bisection for i in row j
            int64_t lo = rp[j], hi = rp[j + 1];
            if (lo < 0 || hi > nnz || hi < lo) {
                bad |= kCheckBadRowPtr;
                continue;
            }
            while (lo < hi) {
                const int64_t mid = lo + (hi - lo) / 2;
                if ((int64_t)col[mid] < i) lo = mid + 1; else hi = mid;
            }
            if (lo >= rp[j + 1] || (int64_t)col[lo] != i) bad |= kCheckAsymmetric;
            else if (w && w[lo] != w[k]) bad |= kCheckAsymmetric;
        }
    }
    if (bad) atomicOr(&st->check, bad);
}


// ------------------------------------------------------------ row plan ----
// Heavy rows (degree >= heavy_min) are listed in increasing id order with the
// offset of their first piece (ceil(degree / piece) pieces each).  Three
// kernels: per-block counts, one-block exclusive scan, per-block writes, so
// the list is deterministic.
__global__ void __launch_bounds__(kPlanBlock) plan_count(int64_t n, const int64_t* __restrict__ rp,
                                                         int heavy_min, int piece,
                                                         long long* __restrict__ counts) {
    const int64_t i = (int64_t)blockIdx.x * kPlanBlock + threadIdx.x;
    long long h = 0, p = 0;
    if (i < n) {
        const int64_t d = rp[i + 1] - rp[i];
        if (d >= heavy_min) {
            h = 1;
            p = (d + piece - 1) / piece;
        }
    }
    __shared__ long long sh[kPlanBlock], sp[kPlanBlock];
    sh[threadIdx.x] = h;
    sp[threadIdx.x] = p;
    __syncthreads();
    for (int off = kPlanBlock / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            sh[threadIdx.x] += sh[threadIdx.x + off];
            sp[threadIdx.x] += sp[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        counts[2 * (int64_t)blockIdx.x] = sh[0];
        counts[2 * (int64_t)blockIdx.x + 1] = sp[0];
    }
}

// One block: exclusive scan of the per-block counts into offs (same layout).
__global__ void __launch_bounds__(1024) plan_scan(int64_t nblocks, const long long* __restrict__ counts,
                                                  long long* __restrict__ offs, GraphStats* __restrict__ st,
                                                  int64_t* __restrict__ hoff) {
    const int t = threadIdx.x;
    const int64_t per = (nblocks + 1023) / 1024;
    const int64_t b0 = t * per, b1 = b0 + per < nblocks ? b0 + per : nblocks;
    long long h = 0, p = 0;
    for (int64_t b = b0; b < b1; ++b) {
        h += counts[2 * b];
        p += counts[2 * b + 1];
    }
    __shared__ long long sh[1024], sp[1024];
    sh[t] = h;
    sp[t] = p;
    __syncthreads();
    // inclusive Hillis-Steele scan over the 1024 thread sums
    for (int off = 1; off < 1024; off <<= 1) {
        long long ah = 0, ap = 0;
        if (t >= off) {
            ah = sh[t - off];
            ap = sp[t - off];
        }
        __syncthreads();
        sh[t] += ah;
        sp[t] += ap;
        __syncthreads();
    }
    long long run_h = t > 0 ? sh[t - 1] : 0, run_p = t > 0 ? sp[t - 1] : 0;
    for (int64_t b = b0; b < b1; ++b) {
        offs[2 * b] = run_h;
        offs[2 * b + 1] = run_p;
        run_h += counts[2 * b];
        run_p += counts[2 * b + 1];
    }
    if (t == 1023) {
        st->n_heavy = sh[1023];
        st->n_pieces = sp[1023];
        hoff[sh[1023]] = sp[1023];
    }
}

__global__ void __launch_bounds__(kPlanBlock) plan_write(int64_t n, const int64_t* __restrict__ rp,
                                                         int heavy_min, int piece,
                                                         const long long* __restrict__ offs,
                                                         int32_t* __restrict__ hrow, int64_t* __restrict__ hoff) {
    const int64_t i = (int64_t)blockIdx.x * kPlanBlock + threadIdx.x;
    long long h = 0, p = 0;
    if (i < n) {
        const int64_t d = rp[i + 1] - rp[i];
        if (d >= heavy_min) {
            h = 1;
            p = (d + piece - 1) / piece;
        }
    }
    __shared__ long long sh[kPlanBlock], sp[kPlanBlock];
    const int t = threadIdx.x;
    sh[t] = h;
    sp[t] = p;
    __syncthreads();
    for (int off = 1; off < kPlanBlock; off <<= 1) {
        long long ah = 0, ap = 0;
        if (t >= off) {
            ah = sh[t - off];
            ap = sp[t - off];
        }
        __syncthreads();
        sh[t] += ah;
        sp[t] += ap;
        __syncthreads();
    }
    if (h) {
        const long long oh = offs[2 * (int64_t)blockIdx.x] + sh[t] - 1;
        const long long op = offs[2 * (int64_t)blockIdx.x + 1] + sp[t] - p;
        hrow[oh] = (int32_t)i;
        hoff[oh] = op;
    }
}

// ---- column-range segments of heavy rows (x-major layout, stride cap) ----
__global__ void __launch_bounds__(64) xcd_bounds(int64_t n, int64_t nnz, const int64_t* __restrict__ rp,
                                                 int64_t* __restrict__ bounds) {
    const int x = threadIdx.x;
    if (x > kColRanges) return;
    const int64_t target = nnz / kColRanges * x;
    int64_t lo = 0, hi = n;  // smallest i with rp[i] >= target
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (rp[mid] < target) lo = mid + 1; else hi = mid;
    }
    bounds[x] = x == 0 ? 0 : (x == kColRanges ? n : lo);
}

__global__ void __launch_bounds__(256) seg_count(int64_t cap, const GraphStats* __restrict__ st,
                                                 const int32_t* __restrict__ hrow, const int64_t* __restrict__ rp,
                                                 const int32_t* __restrict__ col, const int64_t* __restrict__ bounds,
                                                 int piece, int64_t* __restrict__ segk, long long* __restrict__ cnt) {
    const int64_t h = blockIdx.x * 256LL + threadIdx.x;
    if (h >= cap) return;
    const int64_t nh = st->n_heavy;
    if (h >= nh) {
        for (int x = 0; x < kColRanges; ++x) cnt[x * cap + h] = 0;
        return;
    }
    const int64_t row = hrow[h], s = rp[row], e = rp[row + 1];
    int64_t prev = s;
    segk[h] = s;
    for (int x = 1; x <= kColRanges; ++x) {
        int64_t k = e;
        if (x < kColRanges) {
            const int64_t b = bounds[x];
            int64_t lo = prev, hi = e;  // first nonzero with column >= b
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if ((int64_t)col[mid] < b) lo = mid + 1; else hi = mid;
            }
            k = lo;
        }
        segk[x * cap + h] = k;
        cnt[(x - 1) * cap + h] = (k - prev + piece - 1) / piece;
        prev = k;
    }
}

__global__ void __launch_bounds__(256) iota_kernel(int64_t n, int32_t* __restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        out[i] = (int32_t)i;
}

// ------------------------------------------------ exclusive scan (int64) ----
// Three fixed-order passes: per-block sums, one-block scan of the sums, and
// per-block scans offset by them.
__global__ void __launch_bounds__(1024) scan_blocks(int64_t len, const long long* __restrict__ in,
                                                    long long* __restrict__ bsum) {
    __shared__ long long red[1024];
    const int64_t i = blockIdx.x * 1024LL + threadIdx.x;
    red[threadIdx.x] = i < len ? in[i] : 0;
    __syncthreads();
    for (int off = 512; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(1024) scan_top(int64_t nb, long long* __restrict__ bsum,
                                                 long long* __restrict__ total_a, int64_t* __restrict__ total_b) {
    const int t = threadIdx.x;
    const int64_t per = (nb + 1023) / 1024;
    const int64_t b0 = t * per, b1 = b0 + per < nb ? b0 + per : nb;
    long long s = 0;
    for (int64_t b = b0; b < b1; ++b) s += bsum[b];
    __shared__ long long sh[1024];
    sh[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        long long a = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += a;
        __syncthreads();
    }
    long long run = t > 0 ? sh[t - 1] : 0;
    for (int64_t b = b0; b < b1; ++b) {
        const long long v = bsum[b];
        bsum[b] = run;
        run += v;
    }
    if (t == 1023) {
        if (total_a) *total_a = sh[1023];
        if (total_b) *total_b = sh[1023];
    }
}

__global__ void __launch_bounds__(1024) scan_apply(int64_t len, const long long* __restrict__ in,
                                                   const long long* __restrict__ boff, int64_t* __restrict__ out) {
    __shared__ long long sh[1024];
    const int t = threadIdx.x;
    const int64_t i = blockIdx.x * 1024LL + t;
    const long long v = i < len ? in[i] : 0;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        long long a = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += a;
        __syncthreads();
    }
    if (i < len) out[i] = boff[blockIdx.x] + sh[t] - v;
}

slaq_status exclusive_scan(const long long* in, int64_t len, int64_t* out, long long* bsum, long long* total_a,
                           int64_t* total_b, hipStream_t st) {
    const int64_t nb = (len + 1023) / 1024;
    if (nb == 0) return SLAQ_OK;
    hipLaunchKernelGGL(scan_blocks, dim3((unsigned)nb), dim3(1024), 0, st, len, in, bsum);
    SLAQ_LAUNCHED();
    hipLaunchKernelGGL(scan_top, dim3(1), dim3(1024), 0, st, nb, bsum, total_a, total_b);
    SLAQ_LAUNCHED();
    hipLaunchKernelGGL(scan_apply, dim3((unsigned)nb), dim3(1024), 0, st, len, in, bsum, out);
    SLAQ_LAUNCHED();
    return SLAQ_OK;
}

struct ScratchLayout {
    size_t off_stats, off_part, off_counts, off_hrow, off_hoff, off_bounds, off_segk, off_cnt, off_segoff, off_bsum,
        off_perm, off_inv, off_rp2, off_col2, off_w2, off_tmp, off_diag2, off_d64, off_d64r, off_len, off_sortcnt,
        off_sortoff, off_tpart, off_lpart, off_choff, off_ccnt, off_coff, total;
    int64_t nplan, max_heavy, sort_chunks;
};

static ScratchLayout scratch_layout(int64_t n, int64_t nnz) {
    ScratchLayout L{};
    L.nplan = (n + kPlanBlock - 1) / kPlanBlock;
    L.max_heavy = nnz / heavy_min_bound(nnz);
    if (L.max_heavy > n) L.max_heavy = n;
    L.sort_chunks = (n + kSortChunk - 1) / kSortChunk;
    size_t off = 0;
    auto take = [&off](size_t bytes) {
        const size_t o = off;
        off += align_up(bytes, 256);
        return o;
    };
    const size_t cap = (size_t)(L.max_heavy > 0 ? L.max_heavy : 1);
    const size_t sort_len = (size_t)kDegBuckets * (size_t)L.sort_chunks;
    size_t scan_max = kColRanges * cap;
    if (sort_len > scan_max) scan_max = sort_len;
    if ((size_t)n + 1 > scan_max) scan_max = (size_t)n + 1;
    L.off_stats = take(sizeof(GraphStats));
    L.off_part = take(sizeof(BuildPartial) * kBuildBlocks);
    L.off_counts = take(sizeof(long long) * 4 * (size_t)L.nplan);
    L.off_hrow = take(sizeof(int32_t) * (size_t)(L.max_heavy + 1));
    L.off_hoff = take(sizeof(int64_t) * (size_t)(L.max_heavy + 1));
    L.off_bounds = take(sizeof(int64_t) * (kColRanges + 1));
    L.off_segk = take(sizeof(int64_t) * (kColRanges + 1) * cap);
    L.off_cnt = take(sizeof(long long) * kColRanges * cap);
    L.off_segoff = take(sizeof(int64_t) * (kColRanges * cap + 1));
    L.off_bsum = take(sizeof(long long) * ((scan_max + 1023) / 1024));
    // relabelled CSR
    L.off_perm = take(sizeof(int32_t) * (size_t)n);
    L.off_inv = take(sizeof(int32_t) * (size_t)n);
    L.off_rp2 = take(sizeof(int64_t) * ((size_t)n + 1));
    L.off_col2 = take(sizeof(int32_t) * (size_t)nnz);
    L.off_w2 = take(sizeof(float) * (size_t)nnz);
    L.off_tmp = take(sizeof(int32_t) * (size_t)nnz);
    L.off_diag2 = take(sizeof(float) * (size_t)n);
    L.off_d64 = take(sizeof(double) * (size_t)n);
    L.off_d64r = take(sizeof(double) * (size_t)n);
    L.off_len = take(sizeof(long long) * ((size_t)n + 1));
    L.off_sortcnt = take(sizeof(long long) * sort_len);
    L.off_sortoff = take(sizeof(int64_t) * sort_len);
    L.off_tpart = take(sizeof(double) * 2 * kTraceBlocks);
    L.off_lpart = take(sizeof(double) * kLoopBlocks);
    L.off_choff = take(sizeof(int64_t) * ((size_t)n + 1));
    L.off_ccnt = take(sizeof(int32_t) * kColRanges * (size_t)relabel_max_chunks(nnz));
    L.off_coff = take(sizeof(int32_t) * kColRanges * (size_t)relabel_max_chunks(nnz));
    L.total = off;
    return L;
}

slaq_status build_plan(slaq_graph_s* g, hipStream_t st) {
    const int64_t nplan = (g->n + kPlanBlock - 1) / kPlanBlock;
    long long* counts = g->blockcounts;
    long long* offs = g->blockcounts + 2 * nplan;
    hipLaunchKernelGGL(plan_count, dim3((unsigned)nplan), dim3(kPlanBlock), 0, st, g->n, g->row_ptr,
                       g->heavy_min, g->piece, counts);
    SLAQ_LAUNCHED();
    hipLaunchKernelGGL(plan_scan, dim3(1), dim3(1024), 0, st, nplan, counts, offs, g->stats, g->hoff);
    SLAQ_LAUNCHED();
    hipLaunchKernelGGL(plan_write, dim3((unsigned)nplan), dim3(kPlanBlock), 0, st, g->n, g->row_ptr,
                       g->heavy_min, g->piece, offs, g->hrow, g->hoff);
    SLAQ_LAUNCHED();
    // column-range segments and their pieces
    const int64_t cap = g->max_heavy > 0 ? g->max_heavy : 1;
    const int64_t len = kColRanges * cap;
    if (!g->relabeled) {  // relabelled graphs got their range starts from the relabelling
        hipLaunchKernelGGL(xcd_bounds, dim3(1), dim3(64), 0, st, g->n, g->nnz, g->row_ptr, g->bounds);
        SLAQ_LAUNCHED();
    }
    hipLaunchKernelGGL(seg_count, dim3((unsigned)((cap + 255) / 256)), dim3(256), 0, st, cap, g->stats, g->hrow,
                       g->row_ptr, g->col_idx, g->bounds, g->piece, g->segk, g->segcnt);
    SLAQ_LAUNCHED();
    return exclusive_scan(g->segcnt, len, g->segoff, g->scanbuf, &g->stats->n_pieces, g->segoff + len, st);
}

}  // namespace slaq

using namespace slaq;

extern "C" {

const char* slaq_last_error(void) { return g_err; }

slaq_status slaq_graph_scratch_bytes(int64_t n, int64_t nnz, size_t* bytes) {
    SLAQ_REQUIRE(bytes, SLAQ_ERR_INVALID_ARG, "bytes is NULL");
    SLAQ_REQUIRE(n > 0 && nnz >= 0, SLAQ_ERR_INVALID_ARG, "need n > 0 and nnz >= 0");
    *bytes = scratch_layout(n, nnz).total;
    return SLAQ_OK;
}

slaq_status slaq_build_graph(int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                             const float* weights, int laplacian, unsigned flags, float* dinv_out,
                             void* scratch, size_t scratch_bytes, void* stream, slaq_graph_t* out) {
    clear_error();
    SLAQ_REQUIRE(out, SLAQ_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    SLAQ_REQUIRE(n > 0, SLAQ_ERR_INVALID_ARG, "n must be positive (got %lld)", (long long)n);
    SLAQ_REQUIRE(n < (int64_t)INT32_MAX, SLAQ_ERR_UNSUPPORTED, "n must fit int32 column indices");
    SLAQ_REQUIRE(nnz >= 0, SLAQ_ERR_INVALID_ARG, "nnz must be >= 0");
    SLAQ_REQUIRE(row_ptr && dinv_out && scratch, SLAQ_ERR_INVALID_ARG,
                 "row_ptr, dinv_out and scratch must be non-NULL");
    SLAQ_REQUIRE(nnz == 0 || col_idx, SLAQ_ERR_INVALID_ARG, "col_idx is NULL");
    SLAQ_REQUIRE(laplacian == SLAQ_LAP_NORMALIZED || laplacian == SLAQ_LAP_COMBINATORIAL,
                 SLAQ_ERR_INVALID_ARG, "unknown laplacian kind %d", laplacian);
    SLAQ_REQUIRE((flags & ~(unsigned)(SLAQ_FLAG_CHECK | SLAQ_FLAG_RELABEL | SLAQ_FLAG_NO_RELABEL)) == 0,
                 SLAQ_ERR_INVALID_ARG, "unknown flags");
    SLAQ_REQUIRE((flags & (SLAQ_FLAG_RELABEL | SLAQ_FLAG_NO_RELABEL)) !=
                     (unsigned)(SLAQ_FLAG_RELABEL | SLAQ_FLAG_NO_RELABEL),
                 SLAQ_ERR_INVALID_ARG, "SLAQ_FLAG_RELABEL and SLAQ_FLAG_NO_RELABEL both set");
    size_t need = 0;
    slaq_graph_scratch_bytes(n, nnz, &need);
    SLAQ_REQUIRE(scratch_bytes >= need, SLAQ_ERR_WORKSPACE, "graph scratch needs %zu bytes, got %zu",
                 need, scratch_bytes);
    SLAQ_REQUIRE(((uintptr_t)scratch & 255) == 0, SLAQ_ERR_INVALID_ARG, "scratch must be 256-byte aligned");

    hipStream_t st = (hipStream_t)stream;
    char* base = (char*)scratch;
    const ScratchLayout SL = scratch_layout(n, nnz);
    GraphStats* stats = (GraphStats*)(base + SL.off_stats);
    BuildPartial* part = (BuildPartial*)(base + SL.off_part);

    int blocks = (int)((n + 255) / 256);
    if (blocks > kBuildBlocks) blocks = kBuildBlocks;

    if (flags & SLAQ_FLAG_CHECK) {
        // validate before anything reads the CSR through row_ptr
        SLAQ_HIP(hipMemsetAsync(&stats->check, 0, sizeof(unsigned), st));
        hipLaunchKernelGGL(check_kernel, dim3(blocks), dim3(256), 0, st, n, nnz, row_ptr, col_idx,
                           weights, stats);
        SLAQ_LAUNCHED();
        unsigned found = 0;
        SLAQ_HIP(hipMemcpyAsync(&found, &stats->check, sizeof(found), hipMemcpyDeviceToHost, st));
        SLAQ_HIP(hipStreamSynchronize(st));
        SLAQ_REQUIRE(!(found & (kCheckBadRowPtr | kCheckBadCol | kCheckUnsorted)), SLAQ_ERR_BAD_CSR,
                     "CSR check failed (flags 0x%x: 1 row_ptr, 2 column range, 4 unsorted/duplicate)",
                     found);
        SLAQ_REQUIRE(!(found & kCheckBadWeight), SLAQ_ERR_NUMERIC, "a weight is <= 0 or not finite");
        SLAQ_REQUIRE(!(found & kCheckAsymmetric), SLAQ_ERR_NOT_SYMMETRIC,
                     "adjacency is not symmetric (pattern or weights)");
    }

    double* d64 = (double*)(base + SL.off_d64);
    if (weights)
        hipLaunchKernelGGL(degree_kernel<true>, dim3(blocks), dim3(256), 0, st, n, row_ptr, weights,
                           laplacian, dinv_out, d64, part);
    else
        hipLaunchKernelGGL(degree_kernel<false>, dim3(blocks), dim3(256), 0, st, n, row_ptr, weights,
                           laplacian, dinv_out, d64, part);
    SLAQ_LAUNCHED();
    double* loop_part = (double*)(base + SL.off_lpart);
    int lblocks = (int)((n + 255) / 256);
    if (lblocks > kLoopBlocks) lblocks = kLoopBlocks;
    if (weights)
        hipLaunchKernelGGL(loop_kernel<true>, dim3(lblocks), dim3(256), 0, st, n, row_ptr, col_idx, weights,
                           laplacian, d64, loop_part);
    else
        hipLaunchKernelGGL(loop_kernel<false>, dim3(lblocks), dim3(256), 0, st, n, row_ptr, col_idx, weights,
                           laplacian, d64, loop_part);
    SLAQ_LAUNCHED();
    hipLaunchKernelGGL(stats_kernel, dim3(1), dim3(256), 0, st, n, blocks, laplacian, part, loop_part, lblocks,
                       stats);
    SLAQ_LAUNCHED();

    const bool relabel = (flags & SLAQ_FLAG_RELABEL) ||
                         (!(flags & SLAQ_FLAG_NO_RELABEL) && nnz >= (int64_t)SLAQ_RELABEL_MIN_NNZ);

    slaq_graph_s* g = new (std::nothrow) slaq_graph_s;
    SLAQ_REQUIRE(g, SLAQ_ERR_INVALID_ARG, "out of host memory");
    g->blockcounts = (long long*)(base + SL.off_counts);
    g->hrow = (int32_t*)(base + SL.off_hrow);
    g->hoff = (int64_t*)(base + SL.off_hoff);
    g->bounds = (int64_t*)(base + SL.off_bounds);
    g->segk = (int64_t*)(base + SL.off_segk);
    g->segcnt = (long long*)(base + SL.off_cnt);
    g->segoff = (int64_t*)(base + SL.off_segoff);
    g->scanbuf = (long long*)(base + SL.off_bsum);
    g->trace_part = (double*)(base + SL.off_tpart);
    g->max_heavy = SL.max_heavy;
    const bool small = nnz < (int64_t)SLAQ_RELABEL_MIN_NNZ;
    g->heavy_min = small ? kSmallHeavyMin : kDefaultHeavyMin;
    g->piece = small ? kSmallPiece : kDefaultPiece;
    g->tile_quads = 0;
    g->cache_rows = -1;
    g->fused = -1;
    g->sign_step = 1;
    g->precision = laplacian == SLAQ_LAP_COMBINATORIAL ? SLAQ_PREC_FP64 : SLAQ_PREC_FP32;
    g->n = n;
    g->nnz = nnz;
    g->laplacian = laplacian;
    g->dinv_out = dinv_out;
    g->stats = stats;
    g->partials = part;
    g->stream = st;
    if (relabel) {
        RelabelBuffers B;
        B.perm = (int32_t*)(base + SL.off_perm);
        B.inv = (int32_t*)(base + SL.off_inv);
        B.row_ptr = (int64_t*)(base + SL.off_rp2);
        B.col = (int32_t*)(base + SL.off_col2);
        B.w = (float*)(base + SL.off_w2);
        B.tmp = (int32_t*)(base + SL.off_tmp);
        B.diag = (float*)(base + SL.off_diag2);
        B.diag64 = (double*)(base + SL.off_d64r);
        B.len = (long long*)(base + SL.off_len);
        B.sort_cnt = (long long*)(base + SL.off_sortcnt);
        B.sort_off = (int64_t*)(base + SL.off_sortoff);
        B.bsum = g->scanbuf;
        B.chunk_off = (int64_t*)(base + SL.off_choff);
        B.ccnt = (int32_t*)(base + SL.off_ccnt);
        B.coff = (int32_t*)(base + SL.off_coff);
        const slaq_status rs = relabel_build(B, n, row_ptr, col_idx, weights, dinv_out, d64, stats, g->bounds, st);
        if (rs != SLAQ_OK) {
            delete g;
            return rs;
        }
        g->row_ptr = B.row_ptr;
        g->col_idx = B.col;
        g->weights = weights ? B.w : nullptr;
        g->diag = B.diag;
        g->diag64 = B.diag64;
        g->perm = B.perm;
        g->relabeled = 1;
    } else {
        g->row_ptr = row_ptr;
        g->col_idx = col_idx;
        g->weights = weights;
        g->diag = dinv_out;
        g->diag64 = d64;
        g->perm = nullptr;
        g->relabeled = 0;
    }
    const slaq_status ps = build_plan(g, st);
    if (ps != SLAQ_OK) {
        delete g;
        return ps;
    }
    *out = g;
    return SLAQ_OK;
}

slaq_status slaq_graph_info(slaq_graph_t g, int64_t* n, int64_t* nnz, double* trace,
                            int64_t* n_isolated, double* max_degree) {
    clear_error();
    SLAQ_REQUIRE(g, SLAQ_ERR_INVALID_ARG, "graph is NULL");
    GraphStats hs;
    SLAQ_HIP(hipMemcpyAsync(&hs, g->stats, sizeof(hs), hipMemcpyDeviceToHost, g->stream));
    SLAQ_HIP(hipStreamSynchronize(g->stream));
    if (n) *n = g->n;
    if (nnz) *nnz = g->nnz;
    if (trace) *trace = hs.trace;
    if (n_isolated) *n_isolated = hs.n_isolated;
    if (max_degree) *max_degree = hs.max_degree;
    SLAQ_REQUIRE(hs.status == 0u, SLAQ_ERR_NUMERIC,
                 "the last Lanczos run on this graph found a non-finite coefficient (status 0x%x)", hs.status);
    return SLAQ_OK;
}

slaq_status slaq_graph_set_schedule(slaq_graph_t g, int heavy_min, int piece, void* stream) {
    clear_error();
    SLAQ_REQUIRE(g, SLAQ_ERR_INVALID_ARG, "graph is NULL");
    SLAQ_REQUIRE(heavy_min >= heavy_min_bound(g->nnz), SLAQ_ERR_INVALID_ARG, "heavy_min must be >= %d",
                 heavy_min_bound(g->nnz));
    SLAQ_REQUIRE(piece >= kMinPiece && piece % 64 == 0, SLAQ_ERR_INVALID_ARG,
                 "piece must be a multiple of 64 and >= %d", kMinPiece);
    g->heavy_min = heavy_min;
    g->piece = piece;
    return build_plan(g, (hipStream_t)stream);
}

slaq_status slaq_graph_set_tile(slaq_graph_t g, int tile_quads) {
    clear_error();
    SLAQ_REQUIRE(g, SLAQ_ERR_INVALID_ARG, "graph is NULL");
    SLAQ_REQUIRE(tile_quads >= 0 && tile_quads <= 64, SLAQ_ERR_INVALID_ARG, "tile_quads must be in [0, 64]");
    g->tile_quads = tile_quads;
    return SLAQ_OK;
}

slaq_status slaq_graph_set_cache_rows(slaq_graph_t g, int64_t rows) {
    clear_error();
    SLAQ_REQUIRE(g, SLAQ_ERR_INVALID_ARG, "graph is NULL");
    SLAQ_REQUIRE(rows >= -1, SLAQ_ERR_INVALID_ARG, "rows must be >= -1 (-1 = automatic)");
    g->cache_rows = rows;
    return SLAQ_OK;
}

slaq_status slaq_graph_cache_rows(slaq_graph_t g, int64_t* rows) {
    clear_error();
    SLAQ_REQUIRE(g && rows, SLAQ_ERR_INVALID_ARG, "graph or rows is NULL");
    *rows = g->cache_rows;
    return SLAQ_OK;
}

slaq_status slaq_graph_set_fused(slaq_graph_t g, int blocks) {
    clear_error();
    SLAQ_REQUIRE(g, SLAQ_ERR_INVALID_ARG, "graph is NULL");
    SLAQ_REQUIRE(blocks >= -1 && blocks <= 256, SLAQ_ERR_INVALID_ARG,
                 "blocks must be -1 (automatic), 0 (never) or 1..256");
    g->fused = blocks;
    return SLAQ_OK;
}

slaq_status slaq_graph_set_sign_step(slaq_graph_t g, int on) {
    clear_error();
    SLAQ_REQUIRE(g, SLAQ_ERR_INVALID_ARG, "graph is NULL");
    SLAQ_REQUIRE(on == 0 || on == 1, SLAQ_ERR_INVALID_ARG, "on must be 0 or 1");
    g->sign_step = on;
    return SLAQ_OK;
}

slaq_status slaq_graph_set_precision(slaq_graph_t g, int precision) {
    clear_error();
    SLAQ_REQUIRE(g, SLAQ_ERR_INVALID_ARG, "graph is NULL");
    SLAQ_REQUIRE(precision == SLAQ_PREC_FP32 || precision == SLAQ_PREC_FP64, SLAQ_ERR_INVALID_ARG,
                 "unknown precision %d", precision);
    g->precision = precision;
    return SLAQ_OK;
}

slaq_status slaq_graph_precision(slaq_graph_t g, int* precision) {
    clear_error();
    SLAQ_REQUIRE(g && precision, SLAQ_ERR_INVALID_ARG, "graph or precision is NULL");
    *precision = g->precision;
    return SLAQ_OK;
}

slaq_status slaq_graph_schedule(slaq_graph_t g, int* heavy_min, int* piece, int64_t* n_heavy,
                                int64_t* n_pieces) {
    clear_error();
    SLAQ_REQUIRE(g, SLAQ_ERR_INVALID_ARG, "graph is NULL");
    if (heavy_min) *heavy_min = g->heavy_min;
    if (piece) *piece = g->piece;
    if (n_heavy || n_pieces) {
        GraphStats hs;
        SLAQ_HIP(hipMemcpyAsync(&hs, g->stats, sizeof(hs), hipMemcpyDeviceToHost, g->stream));
        SLAQ_HIP(hipStreamSynchronize(g->stream));
        if (n_heavy) *n_heavy = hs.n_heavy;
        if (n_pieces) *n_pieces = hs.n_pieces;
    }
    return SLAQ_OK;
}

slaq_status slaq_graph_internal(slaq_graph_t g, int* relabeled, int64_t* n_rows, int32_t* perm,
                                int64_t* row_ptr, int32_t* col_idx) {
    clear_error();
    SLAQ_REQUIRE(g, SLAQ_ERR_INVALID_ARG, "graph is NULL");
    hipStream_t st = g->stream;
    if (relabeled) *relabeled = g->relabeled;
    if (n_rows) {
        GraphStats hs;
        SLAQ_HIP(hipMemcpyAsync(&hs, g->stats, sizeof(hs), hipMemcpyDeviceToHost, st));
        SLAQ_HIP(hipStreamSynchronize(st));
        *n_rows = hs.n_rows;
    }
    if (perm) {
        if (g->perm) {
            SLAQ_HIP(hipMemcpyAsync(perm, g->perm, sizeof(int32_t) * (size_t)g->n, hipMemcpyDeviceToDevice, st));
        } else {
            hipLaunchKernelGGL(iota_kernel, dim3(256), dim3(256), 0, st, g->n, perm);
            SLAQ_LAUNCHED();
        }
    }
    if (row_ptr)
        SLAQ_HIP(hipMemcpyAsync(row_ptr, g->row_ptr, sizeof(int64_t) * (size_t)(g->n + 1), hipMemcpyDeviceToDevice, st));
    if (col_idx && g->nnz > 0)
        SLAQ_HIP(hipMemcpyAsync(col_idx, g->col_idx, sizeof(int32_t) * (size_t)g->nnz, hipMemcpyDeviceToDevice, st));
    SLAQ_HIP(hipStreamSynchronize(st));
    return SLAQ_OK;
}

slaq_status slaq_graph_destroy(slaq_graph_t g) {
    delete g;
    return SLAQ_OK;
}

}  // extern "C"
