// Node relabelling of the graph build.  It changes the storage order of the
// SpMM only: every result is a function of the graph and of the probes, whose
// entries stay keyed by the caller's node ids.
//
// Why: a gather of node c reads its whole probe row (ld floats), and the
// number of gathers of c is its row length.  Sorting nodes by decreasing row
// length puts the rows that are gathered most next to each other, so a cache
// line of one hot row is shared with other hot rows rather than with cold
// ones, and isolated nodes (no vector data at all) leave the label space.
// Dealing the degree order round-robin over the eight column ranges of the
// row schedule gives every range (and so every XCD, which owns one range in
// the piece kernel) the same mix of hot and cold columns.  Generators such as
// R-MAT place their hubs at ids of few set bits, which in the caller's order
// concentrates the hottest rows on few memory channels; the relabelled order
// spreads them.
//
// Steps (all deterministic):
//   sort_count     per chunk of caller ids, a histogram of order keys
//   scan           exclusive scan, key-major, over (key, chunk)
//   sort_scatter   stable ranks within (key, chunk) by wave ballots; rank r
//                  of the n_act non-isolated nodes gets label
//                  base(r mod 8) + r div 8, isolated nodes labels >= n_act
//   relabel_len    row lengths and diagonal scale (FP32 and FP64) in label order
//   scan           row offsets of the relabelled CSR
//   range bounds   base(x), x = 0..8
//   relabel_short_rows / relabel_rows / long_row_*   thread per row up to 32
//                  entries, wave per row up to 1024, chunks of 256 above (count,
//                  offsets, place): columns mapped to labels and listed range by
//                  range (caller order within a range), weights alongside
#include "common.hpp"

namespace slaq {

// Row-length bucket: exact below 1024, then 16 buckets per octave.
__device__ __forceinline__ int degree_bucket(int64_t d) {
    if (d < 1024) return (int)d;
    const int lg = 63 - __clzll((unsigned long long)d);
    if (lg > 30) return kDegBuckets - 1;
    return 1024 + 16 * (lg - 10) + (int)((d >> (lg - 4)) & 15);
}

// Sort key in increasing order = decreasing row length; isolated nodes last.
__device__ __forceinline__ int order_key(const int64_t* __restrict__ rp, int64_t i) {
    return kDegBuckets - 1 - degree_bucket(rp[i + 1] - rp[i]);
}

// First label of column range x when n_act labels are dealt over kColRanges.
__device__ __forceinline__ int64_t range_base(int x, int64_t q, int64_t rem) {
    return (int64_t)x * q + (x < rem ? x : rem);
}

__global__ void __launch_bounds__(256) sort_count(int64_t n, const int64_t* __restrict__ rp, int64_t nblk,
                                                  long long* __restrict__ counts) {
    __shared__ int hist[kDegBuckets];
    for (int b = threadIdx.x; b < kDegBuckets; b += 256) hist[b] = 0;
    __syncthreads();
    const int64_t i0 = (int64_t)blockIdx.x * kSortChunk;
    for (int k = threadIdx.x; k < kSortChunk; k += 256) {
        const int64_t i = i0 + k;
        if (i < n) atomicAdd(&hist[order_key(rp, i)], 1);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kDegBuckets; b += 256) counts[(int64_t)b * nblk + blockIdx.x] = hist[b];
}

// One wave per chunk, sub-chunks of 64 ids in increasing order: lanes sharing
// a key are ranked by a ballot, then the key's running offset advances, so
// ties keep caller order.
__global__ void __launch_bounds__(64) sort_scatter(int64_t n, const int64_t* __restrict__ rp, int64_t nblk,
                                                   const int64_t* __restrict__ offs, GraphStats* __restrict__ st,
                                                   int32_t* __restrict__ perm, int32_t* __restrict__ inv) {
    __shared__ int64_t next[kDegBuckets];
    const int lane = threadIdx.x;
    for (int b = lane; b < kDegBuckets; b += 64) next[b] = offs[(int64_t)b * nblk + blockIdx.x];
    __syncthreads();
    // the isolated key is the last one: its first offset counts the others
    const int64_t nact = offs[(int64_t)(kDegBuckets - 1) * nblk];
    if (blockIdx.x == 0 && lane == 0) st->n_rows = nact;
    const int64_t q = nact / kColRanges, rem = nact % kColRanges;
    const uint64_t lt = (1ull << lane) - 1ull;
    const int64_t i0 = (int64_t)blockIdx.x * kSortChunk;
    for (int k0 = 0; k0 < kSortChunk; k0 += 64) {
        const int64_t i = i0 + k0 + lane;
        const int key = i < n ? order_key(rp, i) : -1;
        uint64_t todo = __ballot(key >= 0);
        while (todo) {
            const int leader = __ffsll((unsigned long long)todo) - 1;
            const int lk = __shfl(key, leader);
            const uint64_t same = __ballot(key == lk);
            const int64_t b0 = next[lk];
            if (key == lk) {
                const int64_t r = b0 + __popcll(same & lt);
                const int64_t label =
                    r < nact ? range_base((int)(r % kColRanges), q, rem) + r / kColRanges : r;
                perm[label] = (int32_t)i;
                inv[i] = (int32_t)label;
            }
            if (lane == leader) next[lk] = b0 + __popcll(same);
            todo &= ~same;
        }
    }
}

// Row lengths (len[n] = 0 closes the scan) and the diagonal scale by label.
__global__ void __launch_bounds__(256) relabel_len(int64_t n, const GraphStats* __restrict__ st,
                                                   const int64_t* __restrict__ rp, const int32_t* __restrict__ perm,
                                                   const float* __restrict__ diag_caller,
                                                   const double* __restrict__ diag64_caller, long long* __restrict__ len,
                                                   float* __restrict__ diag2, double* __restrict__ diag64) {
    const int64_t nr = st->n_rows;
    for (int64_t L = (int64_t)blockIdx.x * 256 + threadIdx.x; L <= n; L += (int64_t)gridDim.x * 256) {
        long long d = 0;
        float dg = 0.0f;
        double dg64 = 0.0;
        if (L < nr) {
            const int64_t o = perm[L];
            d = rp[o + 1] - rp[o];
            dg = diag_caller[o];
            dg64 = diag64_caller[o];
        }
        len[L] = d;
        if (L < n) {
            diag2[L] = dg;
            diag64[L] = dg64;
        }
    }
}

__global__ void __launch_bounds__(64) range_bounds(const GraphStats* __restrict__ st, int64_t* __restrict__ bounds) {
    const int x = threadIdx.x;
    if (x > kColRanges) return;
    const int64_t nr = st->n_rows;
    bounds[x] = range_base(x, nr / kColRanges, nr % kColRanges);
}

__device__ __forceinline__ int range_of(int64_t c, const int64_t (&bnd)[kColRanges]) {
    int x = 0;
#pragma unroll
    for (int r = 1; r < kColRanges; ++r) x += c >= bnd[r] ? 1 : 0;
    return x;
}

// Short rows (at most kShortRow entries): one thread per row, so a wave keeps
// 64 rows' label gathers in flight.  Pass 1 maps and counts per range, pass 2
// maps again (the labels are in L2 by then) and places the entries range by
// range in caller order: the same layout as the wave kernel below.
constexpr int kShortRow = 32;
// Long rows (more than kBigRow entries): cut into chunks of kRelabelChunk
// entries that workgroups process in parallel (one wave walking a hub row of
// 10^5 entries would be the critical path of the build).
constexpr int kBigRow = 1024;
constexpr int kRelabelChunk = 256;

template <bool WEIGHTED>
__global__ void __launch_bounds__(256) relabel_short_rows(const GraphStats* __restrict__ st,
                                                          const int64_t* __restrict__ rp,
                                                          const int32_t* __restrict__ col,
                                                          const float* __restrict__ w,
                                                          const int32_t* __restrict__ perm,
                                                          const int32_t* __restrict__ inv,
                                                          const int64_t* __restrict__ bounds,
                                                          const int64_t* __restrict__ rp2,
                                                          int32_t* __restrict__ col2, float* __restrict__ w2) {
    const int64_t nr = st->n_rows;
    int64_t bnd[kColRanges];
#pragma unroll
    for (int r = 0; r < kColRanges; ++r) bnd[r] = bounds[r];
    for (int64_t L = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; L < nr;
         L += (int64_t)gridDim.x * blockDim.x) {
        const int64_t o = perm[L], s = rp[o], e = rp[o + 1];
        if (e - s > kShortRow) continue;
        int cnt[kColRanges];
#pragma unroll
        for (int r = 0; r < kColRanges; ++r) cnt[r] = 0;
        for (int64_t k = s; k < e; ++k) {
            const int x = range_of(inv[col[k]], bnd);
#pragma unroll
            for (int r = 0; r < kColRanges; ++r) cnt[r] += x == r ? 1 : 0;
        }
        int64_t pos[kColRanges];
        int64_t run = rp2[L];
#pragma unroll
        for (int r = 0; r < kColRanges; ++r) {
            pos[r] = run;
            run += cnt[r];
        }
        for (int64_t k = s; k < e; ++k) {
            const int32_t c = inv[col[k]];
            const int x = range_of(c, bnd);
            int64_t p = 0;
#pragma unroll
            for (int r = 0; r < kColRanges; ++r)
                if (x == r) p = pos[r]++;
            col2[p] = c;
            if (WEIGHTED) w2[p] = w[k];
        }
    }
}

// One wave per relabelled row.  Each caller column is mapped to its label
// once (the gather inv[col] is the costly part: random 4-byte reads): rows of
// at most 64 entries keep the labels in registers and are placed in one pass
// from 8 ballots (one per range); longer rows park the labels, in caller
// order, in `tmp` at the row's own offsets (coalesced), count per range, then
// read them back and place them.
template <bool WEIGHTED>
__global__ void __launch_bounds__(256) relabel_rows(const GraphStats* __restrict__ st, const int64_t* __restrict__ rp,
                                                    const int32_t* __restrict__ col, const float* __restrict__ w,
                                                    const int32_t* __restrict__ perm, const int32_t* __restrict__ inv,
                                                    const int64_t* __restrict__ bounds,
                                                    const int64_t* __restrict__ rp2, int32_t* __restrict__ col2,
                                                    float* __restrict__ w2, int32_t* __restrict__ tmp) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint64_t lt = (1ull << lane) - 1ull;
    const int64_t nr = st->n_rows;
    int64_t bnd[kColRanges];
#pragma unroll
    for (int r = 0; r < kColRanges; ++r) bnd[r] = bounds[r];
    for (int64_t L = (int64_t)blockIdx.x * 4 + wave; L < nr; L += (int64_t)gridDim.x * 4) {
        const int64_t o = perm[L], s = rp[o], e = rp[o + 1];
        if (e - s <= kShortRow || e - s > kBigRow) continue;  // relabel_short_rows / the chunk kernels
        const int64_t dst = rp2[L];
        if (e - s <= 64) {
            const int64_t k = s + lane;
            int32_t c = 0;
            int x = -1;
            if (k < e) {
                c = inv[col[k]];
                x = range_of(c, bnd);
            }
            int64_t run = dst;
#pragma unroll
            for (int r = 0; r < kColRanges; ++r) {
                const uint64_t mr = __ballot(x == r);
                if (x == r) {
                    const int64_t p = run + __popcll(mr & lt);
                    col2[p] = c;
                    if (WEIGHTED) w2[p] = w[k];
                }
                run += __popcll(mr);
            }
            continue;
        }
        int64_t pos[kColRanges];
#pragma unroll
        for (int r = 0; r < kColRanges; ++r) pos[r] = 0;
        for (int64_t k0 = s; k0 < e; k0 += 64) {
            const int64_t k = k0 + lane;
            int x = -1;
            if (k < e) {
                const int32_t c = inv[col[k]];
                tmp[dst + (k - s)] = c;
                x = range_of(c, bnd);
            }
#pragma unroll
            for (int r = 0; r < kColRanges; ++r) pos[r] += __popcll(__ballot(x == r));
        }
        int64_t run = dst;
#pragma unroll
        for (int r = 0; r < kColRanges; ++r) {
            const int64_t c = pos[r];
            pos[r] = run;
            run += c;
        }
        for (int64_t k0 = s; k0 < e; k0 += 64) {
            const int64_t k = k0 + lane;
            int32_t c = 0;
            int x = -1;
            if (k < e) {
                c = tmp[dst + (k - s)];
                x = range_of(c, bnd);
            }
#pragma unroll
            for (int r = 0; r < kColRanges; ++r) {
                const uint64_t mr = __ballot(x == r);
                if (x == r) {
                    const int64_t p = pos[r] + __popcll(mr & lt);
                    col2[p] = c;
                    if (WEIGHTED) w2[p] = w[k];
                }
                pos[r] += __popcll(mr);
            }
        }
    }
}

// Chunks per long row (0 for the others); len[n] = 0 closes the scan.
__global__ void __launch_bounds__(256) long_row_chunks(int64_t n, const GraphStats* __restrict__ st,
                                                       const int64_t* __restrict__ rp2, long long* __restrict__ cnt) {
    const int64_t nr = st->n_rows;
    for (int64_t L = (int64_t)blockIdx.x * 256 + threadIdx.x; L <= n; L += (int64_t)gridDim.x * 256) {
        const int64_t len = L < nr ? rp2[L + 1] - rp2[L] : 0;
        cnt[L] = len > kBigRow ? (len + kRelabelChunk - 1) / kRelabelChunk : 0;
    }
}

// Row of global chunk g: the largest L with chunk_off[L] <= g (chunk_off,
// n + 1 entries, is non-decreasing; chunk_off[L + 1] > g for the owning row).
// A workgroup walks a contiguous run of chunks, so given the previous
// chunk's row `prev` (or -1) the row is almost always prev or prev + 1; only
// otherwise (the run's first chunk, a row without chunks in between) does it
// search the offsets, from prev + 1 on.
__device__ __forceinline__ int64_t chunk_row(const int64_t* __restrict__ chunk_off, int64_t n, int64_t g,
                                             int64_t prev) {
    int64_t lo = 0;
    if (prev >= 0) {
        if (g < chunk_off[prev + 1]) return prev;
        if (prev + 2 <= n && g < chunk_off[prev + 2]) return prev + 1;
        lo = prev + 1;
    }
    int64_t hi = n - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (chunk_off[mid] <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// The contiguous run of chunks of this workgroup: [*g0, *g1).
__device__ __forceinline__ void chunk_run(int64_t C, int64_t* g0, int64_t* g1) {
    const int64_t per = (C + gridDim.x - 1) / gridDim.x;
    const int64_t a = (int64_t)blockIdx.x * per;
    *g0 = a < C ? a : C;
    *g1 = a + per < C ? a + per : C;
}

// Phase 1: each chunk maps its columns to labels (parked in tmp at the row's
// offsets, caller order) and counts them per range.
__global__ void __launch_bounds__(256) long_row_count(int64_t n, const int64_t* __restrict__ chunk_off,
                                                      const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                      const int32_t* __restrict__ perm,
                                                      const int32_t* __restrict__ inv,
                                                      const int64_t* __restrict__ bounds,
                                                      const int64_t* __restrict__ rp2, int32_t* __restrict__ tmp,
                                                      int32_t* __restrict__ ccnt) {
    __shared__ int hist[kColRanges];
    __shared__ int64_t row;
    int64_t bnd[kColRanges];
#pragma unroll
    for (int r = 0; r < kColRanges; ++r) bnd[r] = bounds[r];
    int64_t g0, g1, prev = -1;
    chunk_run(chunk_off[n], &g0, &g1);
    for (int64_t g = g0; g < g1; ++g) {
        if (threadIdx.x < kColRanges) hist[threadIdx.x] = 0;
        if (threadIdx.x == 0) row = prev = chunk_row(chunk_off, n, g, prev);
        __syncthreads();
        const int64_t L = row, q = g - chunk_off[L];
        const int64_t o = perm[L];
        const int64_t s = rp[o] + q * kRelabelChunk, e0 = rp[o + 1];
        const int64_t k = s + threadIdx.x;
        if (k < e0 && threadIdx.x < kRelabelChunk) {
            const int32_t c = inv[col[k]];
            tmp[rp2[L] + q * kRelabelChunk + threadIdx.x] = c;
            atomicAdd(&hist[range_of(c, bnd)], 1);  // integer counts: order does not matter
        }
        __syncthreads();
        if (threadIdx.x < kColRanges) ccnt[g * kColRanges + threadIdx.x] = hist[threadIdx.x];
        __syncthreads();
    }
}

// Phase 2: one thread per long row turns the chunk counts into each chunk's
// first position per range within the row (ranges in order, chunks in order).
__global__ void __launch_bounds__(256) long_row_offsets(int64_t n, const GraphStats* __restrict__ st,
                                                        const int64_t* __restrict__ chunk_off,
                                                        const int32_t* __restrict__ ccnt, int32_t* __restrict__ coff) {
    const int64_t nr = st->n_rows;
    for (int64_t L = (int64_t)blockIdx.x * 256 + threadIdx.x; L < nr; L += (int64_t)gridDim.x * 256) {
        const int64_t g0 = chunk_off[L], g1 = chunk_off[L + 1];
        if (g0 == g1) continue;
        int tot[kColRanges];
#pragma unroll
        for (int r = 0; r < kColRanges; ++r) tot[r] = 0;
        for (int64_t g = g0; g < g1; ++g)
#pragma unroll
            for (int r = 0; r < kColRanges; ++r) tot[r] += ccnt[g * kColRanges + r];
        int run[kColRanges];
        int base = 0;
#pragma unroll
        for (int r = 0; r < kColRanges; ++r) {
            run[r] = base;
            base += tot[r];
        }
        for (int64_t g = g0; g < g1; ++g)
#pragma unroll
            for (int r = 0; r < kColRanges; ++r) {
                coff[g * kColRanges + r] = run[r];
                run[r] += ccnt[g * kColRanges + r];
            }
    }
}

// Phase 3: each chunk places its labels, ranked within the chunk by wave
// ballots and a prefix over the 4 waves (caller order within a range).
template <bool WEIGHTED>
__global__ void __launch_bounds__(256) long_row_place(int64_t n, const int64_t* __restrict__ chunk_off,
                                                      const int64_t* __restrict__ rp, const float* __restrict__ w,
                                                      const int32_t* __restrict__ perm,
                                                      const int64_t* __restrict__ bounds,
                                                      const int64_t* __restrict__ rp2,
                                                      const int32_t* __restrict__ tmp,
                                                      const int32_t* __restrict__ coff, int32_t* __restrict__ col2,
                                                      float* __restrict__ w2) {
    __shared__ int wcnt[4][kColRanges];
    __shared__ int64_t row;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint64_t lt = (1ull << lane) - 1ull;
    int64_t bnd[kColRanges];
#pragma unroll
    for (int r = 0; r < kColRanges; ++r) bnd[r] = bounds[r];
    int64_t g0, g1, prev = -1;
    chunk_run(chunk_off[n], &g0, &g1);
    for (int64_t g = g0; g < g1; ++g) {
        if (threadIdx.x == 0) row = prev = chunk_row(chunk_off, n, g, prev);
        __syncthreads();
        const int64_t L = row, q = g - chunk_off[L];
        const int64_t o = perm[L];
        const int64_t s = rp[o] + q * kRelabelChunk, e0 = rp[o + 1];
        const int64_t k = s + threadIdx.x;
        const bool valid = k < e0 && threadIdx.x < kRelabelChunk;
        int32_t c = 0;
        int x = -1;
        if (valid) {
            c = tmp[rp2[L] + q * kRelabelChunk + threadIdx.x];
            x = range_of(c, bnd);
        }
        uint64_t m[kColRanges];
#pragma unroll
        for (int r = 0; r < kColRanges; ++r) {
            m[r] = __ballot(x == r);
            if (lane == 0) wcnt[wave][r] = __popcll(m[r]);
        }
        __syncthreads();
        if (valid) {
            int before = 0;
            for (int v = 0; v < wave; ++v) before += wcnt[v][x];
            const int64_t p = rp2[L] + coff[g * kColRanges + x] + before + __popcll(m[x] & lt);
            col2[p] = c;
            if (WEIGHTED) w2[p] = w[k];
        }
        __syncthreads();
    }
}

slaq_status relabel_build(const RelabelBuffers& B, int64_t n, const int64_t* rp, const int32_t* col,
                          const float* w, const float* diag_caller, const double* diag64_caller, GraphStats* st,
                          int64_t* bounds, hipStream_t stream) {
    const int64_t nblk = (n + kSortChunk - 1) / kSortChunk;
    hipLaunchKernelGGL(sort_count, dim3((unsigned)nblk), dim3(256), 0, stream, n, rp, nblk, B.sort_cnt);
    SLAQ_LAUNCHED();
    slaq_status s = exclusive_scan(B.sort_cnt, (int64_t)kDegBuckets * nblk, B.sort_off, B.bsum, nullptr, nullptr,
                                   stream);
    if (s != SLAQ_OK) return s;
    hipLaunchKernelGGL(sort_scatter, dim3((unsigned)nblk), dim3(64), 0, stream, n, rp, nblk, B.sort_off, st, B.perm,
                       B.inv);
    SLAQ_LAUNCHED();
    int lb = (int)((n + 1 + 255) / 256);
    if (lb > 4096) lb = 4096;
    hipLaunchKernelGGL(relabel_len, dim3(lb), dim3(256), 0, stream, n, st, rp, B.perm, diag_caller, diag64_caller,
                       B.len, B.diag, B.diag64);
    SLAQ_LAUNCHED();
    s = exclusive_scan(B.len, n + 1, B.row_ptr, B.bsum, nullptr, nullptr, stream);
    if (s != SLAQ_OK) return s;
    hipLaunchKernelGGL(range_bounds, dim3(1), dim3(64), 0, stream, st, bounds);
    SLAQ_LAUNCHED();
    int64_t sb = (n + 255) / 256;
    if (sb > 8192) sb = 8192;
    if (sb < 1) sb = 1;
    if (w)
        hipLaunchKernelGGL(relabel_short_rows<true>, dim3((unsigned)sb), dim3(256), 0, stream, st, rp, col, w, B.perm,
                           B.inv, bounds, B.row_ptr, B.col, B.w);
    else
        hipLaunchKernelGGL(relabel_short_rows<false>, dim3((unsigned)sb), dim3(256), 0, stream, st, rp, col, w, B.perm,
                           B.inv, bounds, B.row_ptr, B.col, B.w);
    SLAQ_LAUNCHED();
    int64_t rb = (n + 3) / 4;
    if (rb > 8192) rb = 8192;
    if (rb < 1) rb = 1;
    if (w)
        hipLaunchKernelGGL(relabel_rows<true>, dim3((unsigned)rb), dim3(256), 0, stream, st, rp, col, w, B.perm, B.inv,
                           bounds, B.row_ptr, B.col, B.w, B.tmp);
    else
        hipLaunchKernelGGL(relabel_rows<false>, dim3((unsigned)rb), dim3(256), 0, stream, st, rp, col, w, B.perm,
                           B.inv, bounds, B.row_ptr, B.col, B.w, B.tmp);
    SLAQ_LAUNCHED();
    // long rows in chunks (B.len is free again once the row offsets exist)
    hipLaunchKernelGGL(long_row_chunks, dim3(lb), dim3(256), 0, stream, n, st, B.row_ptr, B.len);
    SLAQ_LAUNCHED();
    s = exclusive_scan(B.len, n + 1, B.chunk_off, B.bsum, nullptr, nullptr, stream);
    if (s != SLAQ_OK) return s;
    const int cb = 8192;
    hipLaunchKernelGGL(long_row_count, dim3(cb), dim3(256), 0, stream, n, B.chunk_off, rp, col, B.perm, B.inv, bounds,
                       B.row_ptr, B.tmp, B.ccnt);
    SLAQ_LAUNCHED();
    hipLaunchKernelGGL(long_row_offsets, dim3(lb), dim3(256), 0, stream, n, st, B.chunk_off, B.ccnt, B.coff);
    SLAQ_LAUNCHED();
    if (w)
        hipLaunchKernelGGL(long_row_place<true>, dim3(cb), dim3(256), 0, stream, n, B.chunk_off, rp, w, B.perm, bounds,
                           B.row_ptr, B.tmp, B.coff, B.col, B.w);
    else
        hipLaunchKernelGGL(long_row_place<false>, dim3(cb), dim3(256), 0, stream, n, B.chunk_off, rp, w, B.perm,
                           bounds, B.row_ptr, B.tmp, B.coff, B.col, B.w);
    SLAQ_LAUNCHED();
    return SLAQ_OK;
}

}  // namespace slaq
