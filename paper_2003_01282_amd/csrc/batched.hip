// Batched SLQ for many graphs (paper §3.1 and Algorithm 1 applied to every
// graph of a collection).  One workgroup runs the Lanczos part of one
// whole graph - degrees, probes, m steps - with the current Lanczos vector in
// LDS and the previous one and w in registers, and writes alpha, beta, the
// step counts and tr L.  As in the plain path the vectors of rows with edges
// are kept in the scaled basis X = D^-1/2 R, so a gather adds neighbour rows
// with no per-nonzero scale (isolated rows keep R: L is zero there).  Graphs are grouped into size buckets; each bucket is
// one persistent launch whose workgroups pull graphs (largest first) from an
// atomic queue.  The FP64 Gauss rules of all G nv probes then come from the
// plain path's eigensolver (one thread per probe), and one block per graph
// forms the heat trace and VNGE; the FP64 tail lives in kernels of its own so
// that its registers do not limit the occupancy of the step kernel.  All
// launches of a run are replayed from one hipGraph.
//
// Probe p of graph g is the plain path's probe p for seed + g on that graph
// alone (SplitMix64 keyed on the graph-local node id), so a graph's batched
// result equals slaq_lanczos/slaq_signature on it, up to summation order.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <vector>

#include "common.hpp"
#include "profile.hpp"
#include "tridiag.hpp"

namespace slaq {

constexpr double kBatchEpsBreakdown = 1e-6;
constexpr int kRedSlots = 128;  // doubles of first-level probe sums
constexpr int kBatchUnroll = 4;  // nonzeros of a row gathered per round

__device__ __forceinline__ uint64_t bmix64(uint64_t seed, uint64_t counter) {
    uint64_t z = seed + (counter + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

struct BatchArgs {
    const int32_t* order;   // graph ids of this bucket, most expensive first
    int count;              // graphs in this bucket
    int* queue;             // work counter of this bucket (reset before launch)
    const int64_t* goff;    // node offsets [G+1] (device)
    const int64_t* rp;      // global row_ptr (device)
    const int32_t* col;     // global column ids (device)
    int nv, m, n_max;       // n_max: node count the LDS layout is sized for
    uint64_t seed;
    const uint64_t* seeds;  // [G] per-graph probe seeds, or NULL: seed + g
    double* alpha;          // [G][nv][m]
    double* beta;           // [G][nv][m]
    int32_t* steps;         // [G][nv]
    double* trace;          // [G]: tr L
    unsigned* dstat;        // device status word (SLAQ_STATUS_* bits)
    int sign_first;         // global buckets: first step gathers sign records
};

// First-step sign records of the global buckets: X_1 is +-1 times one scale
// per row, so row i's record is a power of two of 16-byte slots, each three
// dwords of sign bits (bit p of probe p's dword set for -1) and the scale.
// A gather loads the one slot with the lane's four probes (one cache line,
// against one or two for the 16 F-byte row) and expands it to exactly X_1's
// values; row n's record is zero, like X_1's zero row.
__host__ __device__ inline int sign_slots(int F) {
    const int need = ((4 * F + 31) / 32 + 2) / 3;
    int s = 1;
    while (s < need) s *= 2;
    return s;
}

__device__ __forceinline__ float4 sign_expand4(const uint4& r, int p0, int nv) {
    const int w = p0 >> 5, pos = w % 3;
    const unsigned wd = pos == 0 ? r.x : (pos == 1 ? r.y : r.z);
    float v[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const unsigned b = __builtin_amdgcn_ubfe(wd, (unsigned)((p0 & 31) + c), 1u);
        v[c] = __uint_as_float(p0 + c < nv ? (b << 31) | r.w : 0u);
    }
    return make_float4(v[0], v[1], v[2], v[3]);
}

// LDS layout (bytes), n_max nodes, ld = 4F floats per node
struct BatchLds {
    size_t r, dinv, st, red, red2, coef, total;
};

__host__ __device__ inline BatchLds batch_lds(int n_max, int nv, int B) {
    const int F = (nv + 3) / 4;
    BatchLds L{};
    size_t off = 0;
    L.r = off;  // n_max rows and one zero row after the graph's last
    off += (size_t)(n_max + 1) * F * 16;
    L.dinv = off;
    off += ((size_t)n_max * 4 + 15) / 16 * 16;
    L.st = off;  // per probe: sigma, tau, a, active, steps (doubles)
    off += (size_t)nv * 40;
    L.red = off;
    off += (size_t)B * 4 * 8;
    L.red2 = off;  // first-level sums of the partials (reduce_chunks)
    off += (size_t)(nv > kRedSlots ? nv : kRedSlots) * 8;  // K nv <= max(kRedSlots, nv)
    L.coef = off;  // float sigma[4F], tau[4F], a[4F]
    off += (size_t)3 * 4 * F * 4;
    L.total = (off + 15) / 16 * 16;
    return L;
}

// Per-graph recurrence state (LDS): pst[5 p ..] = sigma, tau, a, active,
// steps of probe p; coef[4F] x 3 = sigma, tau, a in FP32 for the vector math.
__device__ __forceinline__ void init_probe_state(int t, int B, int nv, int F, int m, double sigma1, double* pst,
                                                 float* coef) {
    for (int p = t; p < 4 * F; p += B) {
        const bool on = p < nv;
        coef[p] = on ? (float)sigma1 : 0.0f;
        coef[4 * F + p] = 0.0f;
        coef[8 * F + p] = 0.0f;
        if (on) {
            pst[5 * p + 0] = sigma1;
            pst[5 * p + 1] = 0.0;
            pst[5 * p + 2] = 0.0;
            pst[5 * p + 3] = 1.0;
            pst[5 * p + 4] = (double)m;
        }
    }
}

// chunks per probe of the first-level sums
__device__ __forceinline__ int red_chunks(int nv) {
    const int k = kRedSlots / nv;
    return k < 1 ? 1 : (k > 8 ? 8 : k);
}

// First level of the per-probe sums of the block's FP64 partials red[4 u + c]
// (threads u = q, q + F, ... hold probe 4 q + c): chunk k of probe p adds the
// row groups k, k + K, ... in order into red2[k nv + p], all chunks of all
// probes at once; the finish_* calls add the K chunks in order after a barrier.
__device__ __forceinline__ void reduce_chunks(int t, int B, int F, int bact, int nv, const double* red,
                                              double* red2) {
    const int K = red_chunks(nv), R = bact / F;
    for (int x = t; x < nv * K; x += B) {
        const int p = x % nv, k = x / nv, qq = p >> 2, cc = p & 3;
        double s = 0.0;
        for (int r = k; r < R; r += K) s += red[4 * (r * F + qq) + cc];
        red2[k * nv + p] = s;
    }
}

__device__ __forceinline__ double chunk_sum(int t, int nv, const double* red2) {
    const int K = red_chunks(nv);
    double s = 0.0;
    for (int k = 0; k < K; ++k) s += red2[k * nv + t];
    return s;
}

// alpha_j of probe t (t < nv) from the first-level sums red2 (reduce_chunks);
// writes gal[t m + j-1] (0 once the probe has stopped) and the FP32 update
// coefficient a_j.
__device__ __forceinline__ void finish_alpha(int t, int nv, int m, int j, const double* red2, double* pst, int F,
                                             float* coef, double* gal, unsigned* dstat) {
    const double s = chunk_sum(t, nv, red2);
    if (pst[5 * t + 3] != 0.0) {
        const double alpha = pst[5 * t + 0] * s;
        if (!isfinite(alpha)) raise_status(dstat, SLAQ_STATUS_NONFINITE);
        gal[t * m + j - 1] = alpha;
        pst[5 * t + 2] = alpha * pst[5 * t + 0];
        coef[8 * F + t] = (float)pst[5 * t + 2];
    } else {
        gal[t * m + j - 1] = 0.0;
        coef[8 * F + t] = 0.0f;
    }
}

// beta_j = ||R_{j+1}|| of probe t, the breakdown test and the next step's
// sigma and tau; writes gbe[t m + j-1] (0 once the probe has stopped).
__device__ __forceinline__ void finish_beta(int t, int nv, int m, int j, const double* red2, double* pst, int F,
                                            float* coef, double* gbe, unsigned* dstat) {
    const double s = chunk_sum(t, nv, red2);
    if (pst[5 * t + 3] == 0.0) {
        gbe[t * m + j - 1] = 0.0;
        return;
    }
    if (!isfinite(s)) raise_status(dstat, SLAQ_STATUS_NONFINITE);
    const double b = sqrt(fmax(s, 0.0));
    gbe[t * m + j - 1] = b;
    if (j < m && !(b > kBatchEpsBreakdown * 2.0)) {
        pst[5 * t + 3] = 0.0;
        pst[5 * t + 1] = 0.0;
        pst[5 * t + 0] = 0.0;
        coef[t] = 0.0f;
        coef[4 * F + t] = 0.0f;
        coef[8 * F + t] = 0.0f;
        pst[5 * t + 4] = (double)j;
    } else {
        const double tn = b * pst[5 * t + 0];
        pst[5 * t + 1] = tn;
        pst[5 * t + 0] = 1.0 / b;
        coef[t] = (float)(1.0 / b);
        coef[4 * F + t] = (float)tn;
    }
}

// Degrees and D^-1/2 of one graph (thread per row), its non-isolated count
// (LDS integer atomic) and the self-loops' share of tr L (§2: L_ii = 1 -
// A_ii / D_ii), summed in thread order only when the graph has a loop.  Rows
// list their columns in ascending order without repeats (the CSR contract),
// so a row's diagonal entry is found by binary search.  Uses red[0, B) and
// ends with a barrier.
__device__ __forceinline__ void degrees_and_loops(int t, int B, int n, const int64_t* __restrict__ rp,
                                                  const int32_t* __restrict__ col, int64_t base,
                                                  float* __restrict__ dinv, double* red, int* s_nz, int* s_loops,
                                                  double* s_corr) {
    int nonzero = 0, loops = 0;
    double share = 0.0;
    for (int i = t; i < n; i += B) {
        const int64_t s = rp[i], e = rp[i + 1], d = e - s;
        dinv[i] = d > 0 ? (float)(1.0 / sqrt((double)d)) : 0.0f;
        nonzero += d > 0 ? 1 : 0;
        int64_t lo = s, hi = e;  // first entry with column >= base + i
        while (lo < hi) {
            const int64_t mid = lo + ((hi - lo) >> 1);
            if ((int64_t)col[mid] < base + i) lo = mid + 1;
            else hi = mid;
        }
        const int self = lo < e && (int64_t)col[lo] == base + i ? 1 : 0;
        if (self) {
            ++loops;
            share += (double)self / (double)d;
        }
    }
    atomicAdd(s_nz, nonzero);
    if (loops) atomicAdd(s_loops, loops);
    red[t] = share;
    __syncthreads();
    if (t == 0) {
        double c = 0.0;
        if (*s_loops)
            for (int b = 0; b < B; ++b) c += red[b];
        *s_corr = c;
    }
}

template <int B, int IPT>
__global__ void __launch_bounds__(B) batch_slq(BatchArgs a) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int F = (a.nv + 3) / 4;
    const int ldq = F;  // quads per node
    const BatchLds L = batch_lds(a.n_max, a.nv, B);
    float4* R = (float4*)(lds + L.r);
    float* dinv = (float*)(lds + L.dinv);
    double* pst = (double*)(lds + L.st);  // [nv][5]: sigma, tau, a, active, steps
    double* red = (double*)(lds + L.red);
    double* red2 = (double*)(lds + L.red2);
    float* coef = (float*)(lds + L.coef);  // [3][4F]
    __shared__ int s_job;
    __shared__ int s_nz;     // non-isolated nodes of the graph (exact integer sum)
    __shared__ int s_loops;  // rows with a self-loop
    __shared__ double s_corr;  // self-loops' share of tr L, sum_i A_ii / D_ii

    const int t = threadIdx.x;
    const int bact = (B / F) * F;  // threads with a fixed quad
    const bool tact = t < bact;
    const int q = t % F;
    const int row0 = t / F;
    const int rstride = bact / F;

    for (;;) {
        if (t == 0) {
            s_job = atomicAdd(a.queue, 1);
            s_nz = 0;
            s_loops = 0;
        }
        __syncthreads();
        const int job = s_job;
        if (job >= a.count) break;
        const int g = a.order[job];
        const int64_t base = a.goff[g];
        const int n = (int)(a.goff[g + 1] - base);
        const int64_t* rp = a.rp + base;
        const int32_t* col = a.col;

        // ---- degrees, D^-1/2, tr L (non-isolated count less the loops' share)
        degrees_and_loops(t, B, n, rp, col, base, dinv, red, &s_nz, &s_loops, &s_corr);
        // ---- probes R_1 = v (graph-local ids, seed + g), stored as X_1 = D^-1/2 v
        //      on rows with edges --------------------------------------------------
        const uint64_t sg = a.seeds ? a.seeds[g] : a.seed + (uint64_t)g;
        for (int x = t; x < n * F; x += B) {
            const int i = x / F, qq = x % F, p0 = 4 * qq;
            const int64_t d = rp[i + 1] - rp[i];
            const float one = d > 0 ? (float)(1.0 / sqrt((double)d)) : 1.0f;  // the same value as dinv[i]
            const uint64_t z = bmix64(sg, 64ull * (uint64_t)i + (uint64_t)(p0 >> 6));
            float v[4];
#pragma unroll
            for (int c = 0; c < 4; ++c)
                v[c] = (p0 + c < a.nv) ? (((z >> ((p0 & 63) + c)) & 1ull) ? -one : one) : 0.0f;
            R[x] = make_float4(v[0], v[1], v[2], v[3]);
        }
        // row n stays zero: column ids outside the graph are clamped to it
        for (int x = t; x < F; x += B) R[n * ldq + x] = make_float4(0.f, 0.f, 0.f, 0.f);
        init_probe_state(t, B, a.nv, F, a.m, 1.0 / sqrt((double)n), pst, coef);
        // every (probe, step) entry of alpha and beta is written below (0 once
        // a probe has stopped)
        double* const gal = a.alpha + (int64_t)g * a.nv * a.m;
        double* const gbe = a.beta + (int64_t)g * a.nv * a.m;
        __syncthreads();

        float4 prev[IPT], wv[IPT];
#pragma unroll
        for (int k = 0; k < IPT; ++k) prev[k] = make_float4(0.f, 0.f, 0.f, 0.f);

        for (int j = 1; j <= a.m; ++j) {
            // ---- w = sigma L R_j - tau R_{j-1}; partial R_j . w -----------------
            const float4 sgm = make_float4(coef[4 * q], coef[4 * q + 1], coef[4 * q + 2], coef[4 * q + 3]);
            const float4 tau = make_float4(coef[4 * F + 4 * q], coef[4 * F + 4 * q + 1], coef[4 * F + 4 * q + 2],
                                           coef[4 * F + 4 * q + 3]);
            double s1[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int k = 0; k < IPT; ++k) {
                const int i = row0 + k * rstride;
                wv[k] = make_float4(0.f, 0.f, 0.f, 0.f);
                if (!tact || i >= n) continue;
                const int64_t s = rp[i], e = rp[i + 1];
                float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
                int64_t kk = s;
                // kBatchUnroll column ids, then their LDS reads, are in flight at
                // once; the products are added in nonzero order as below.  Row
                // offsets use the full-rate 24-bit multiply (rows and quads per
                // row are far below 2^24; the 32-bit one is quarter rate)
                for (; kk + kBatchUnroll <= e; kk += kBatchUnroll) {
                    // a column outside the graph reads the zero row n: ignored
                    unsigned c[kBatchUnroll];
#pragma unroll
                    for (int u = 0; u < kBatchUnroll; ++u) c[u] = min((unsigned)(int)(col[kk + u] - base), (unsigned)n);
                    float4 x[kBatchUnroll];
#pragma unroll
                    for (int u = 0; u < kBatchUnroll; ++u) x[u] = R[__umul24(c[u], (unsigned)ldq) + q];
#pragma unroll
                    for (int u = 0; u < kBatchUnroll; ++u) {
                        acc.x += x[u].x;
                        acc.y += x[u].y;
                        acc.z += x[u].z;
                        acc.w += x[u].w;
                    }
                }
                for (; kk < e; ++kk) {
                    const unsigned c = min((unsigned)(int)(col[kk] - base), (unsigned)n);
                    const float4 x = R[__umul24(c, (unsigned)ldq) + q];
                    acc.x += x.x;
                    acc.y += x.y;
                    acc.z += x.z;
                    acc.w += x.w;
                }
                // rows with edges: D^-1/2 w = sigma (X_i - dinv_i^2 (A X)_i) - tau X_{j-1,i}
                // in FP64 with one rounding, dot weight 1/dinv_i^2; isolated rows
                // (unscaled): L R = 0, w = -tau R_{j-1,i}, weight 1
                const float di = dinv[i];
                const double dd = (double)di, d2 = dd * dd, wgt = di != 0.0f ? 1.0 / d2 : 1.0;
                const float4 ri = R[i * ldq + q];
                const float* rv = &ri.x;
                const float* av = &acc.x;
                const float* pv = &prev[k].x;
                const float* sv = &sgm.x;
                const float* tv = &tau.x;
                float4 w;
                float* wp = &w.x;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const double lr = di != 0.0f ? fma(-d2, (double)av[c], (double)rv[c]) : 0.0;
                    wp[c] = (float)fma(-(double)tv[c], (double)pv[c], (double)sv[c] * lr);
                    s1[c] = fma((double)rv[c] * (double)wp[c], wgt, s1[c]);
                }
                wv[k] = w;
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) red[4 * t + c] = s1[c];
            __syncthreads();
            reduce_chunks(t, B, F, bact, a.nv, red, red2);
            __syncthreads();
            if (t < a.nv) finish_alpha(t, a.nv, a.m, j, red2, pst, F, coef, gal, a.dstat);
            __syncthreads();
            // ---- R_{j+1} = w - a R_j (in place); partial ||R_{j+1}||^2 ---------
            const float4 av = make_float4(coef[8 * F + 4 * q], coef[8 * F + 4 * q + 1], coef[8 * F + 4 * q + 2],
                                          coef[8 * F + 4 * q + 3]);
            double s2[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int k = 0; k < IPT; ++k) {
                const int i = row0 + k * rstride;
                if (!tact || i >= n) continue;
                const float4 ri = R[i * ldq + q];
                const float di = dinv[i];
                const double wgt = di != 0.0f ? 1.0 / ((double)di * (double)di) : 1.0;  // ||R||^2 from X
                float4 r;
                r.x = fmaf(-av.x, ri.x, wv[k].x);
                r.y = fmaf(-av.y, ri.y, wv[k].y);
                r.z = fmaf(-av.z, ri.z, wv[k].z);
                r.w = fmaf(-av.w, ri.w, wv[k].w);
                prev[k] = ri;
                R[i * ldq + q] = r;
                s2[0] = fma((double)r.x * (double)r.x, wgt, s2[0]);
                s2[1] = fma((double)r.y * (double)r.y, wgt, s2[1]);
                s2[2] = fma((double)r.z * (double)r.z, wgt, s2[2]);
                s2[3] = fma((double)r.w * (double)r.w, wgt, s2[3]);
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) red[4 * t + c] = s2[c];
            __syncthreads();
            reduce_chunks(t, B, F, bact, a.nv, red, red2);
            __syncthreads();
            if (t < a.nv) finish_beta(t, a.nv, a.m, j, red2, pst, F, coef, gbe, a.dstat);
            __syncthreads();
        }

        if (t < a.nv) a.steps[(int64_t)g * a.nv + t] = (int32_t)pst[5 * t + 4];
        if (t == 0) a.trace[g] = (double)s_nz - s_corr;  // tr L of the normalized Laplacian
        __syncthreads();
    }
}

// Graphs whose probe block does not fit in LDS: the same per-graph Lanczos
// with X_j, X_{j-1}, w and D^-1/2 in the workgroup's slot of a global
// workspace (slot = blockIdx.x: three buffers of slot_quads quads, the
// largest graph's rows plus one zero row, and slot_n floats of D^-1/2).  Rows are taken in passes of bact / F; nothing is held per row in
// registers, so the kernel serves any graph size.  X_{j+1} overwrites
// X_{j-1}, and the two buffers swap roles after every step.
template <int B>
__global__ void __launch_bounds__(B) batch_slq_global(BatchArgs a, float4* __restrict__ ws, int64_t slot_quads,
                                                      float* __restrict__ wsd, int64_t slot_n) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int F = (a.nv + 3) / 4;
    const BatchLds L = batch_lds(0, a.nv, B);
    double* pst = (double*)(lds + L.st);
    double* red = (double*)(lds + L.red);
    double* red2 = (double*)(lds + L.red2);
    float* coef = (float*)(lds + L.coef);
    __shared__ int s_job;
    __shared__ int s_nz;     // non-isolated nodes of the graph (exact integer sum)
    __shared__ int s_loops;  // rows with a self-loop
    __shared__ double s_corr;  // self-loops' share of tr L, sum_i A_ii / D_ii

    const int t = threadIdx.x;
    const int bact = (B / F) * F;
    const bool tact = t < bact;
    const int q = t % F;
    const int row0 = t / F;
    const int rstride = bact / F;
    float4* const slot = ws + (int64_t)blockIdx.x * 3 * slot_quads;
    float* const dinv = wsd + (int64_t)blockIdx.x * slot_n;
    const int slots = sign_slots(F), sh = ((4 * q) >> 5) / 3;  // record slots, the lane's slot

    for (;;) {
        if (t == 0) {
            s_job = atomicAdd(a.queue, 1);
            s_nz = 0;
            s_loops = 0;
        }
        __syncthreads();
        const int job = s_job;
        if (job >= a.count) break;
        const int g = a.order[job];
        const int64_t base = a.goff[g];
        const int n = (int)(a.goff[g + 1] - base);
        const int64_t* rp = a.rp + base;
        const int32_t* col = a.col;
        float4* X = slot;                    // X_j
        float4* P = slot + slot_quads;       // X_{j-1}, then X_{j+1}
        float4* W = slot + 2 * slot_quads;   // D^-1/2 w

        degrees_and_loops(t, B, n, rp, col, base, dinv, red, &s_nz, &s_loops, &s_corr);
        const uint64_t sg = a.seeds ? a.seeds[g] : a.seed + (uint64_t)g;
        // the first step's sign records live in the X_{j-1} buffer, which the
        // first step does not read (the first update overwrites them)
        uint4* const Rs = (uint4*)P;
        for (int64_t x = t; x < (int64_t)n * F; x += B) {
            const int i = (int)(x / F), qq = (int)(x % F), p0 = 4 * qq;
            const int64_t d = rp[i + 1] - rp[i];
            const float one = d > 0 ? (float)(1.0 / sqrt((double)d)) : 1.0f;
            const uint64_t z = bmix64(sg, 64ull * (uint64_t)i + (uint64_t)(p0 >> 6));
            float v[4];
#pragma unroll
            for (int c = 0; c < 4; ++c)
                v[c] = (p0 + c < a.nv) ? (((z >> ((p0 & 63) + c)) & 1ull) ? -one : one) : 0.0f;
            X[x] = make_float4(v[0], v[1], v[2], v[3]);
            if (a.sign_first && (p0 & 31) == 0) {
                const int w = p0 >> 5;
                unsigned* sl = (unsigned*)(Rs + (int64_t)i * slots + w / 3);
                sl[w % 3] = (unsigned)(z >> (p0 & 63));
                if (w % 3 == 0) sl[3] = __float_as_uint(one);
            }
        }
        // row n of both rotating buffers stays zero: column ids outside the
        // graph are clamped to it (and so is row n's sign record)
        for (int x = t; x < F; x += B) {
            X[(int64_t)n * F + x] = make_float4(0.f, 0.f, 0.f, 0.f);
            P[(int64_t)n * F + x] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
        if (a.sign_first)
            for (int x = t; x < slots; x += B) Rs[(int64_t)n * slots + x] = make_uint4(0u, 0u, 0u, 0u);
        init_probe_state(t, B, a.nv, F, a.m, 1.0 / sqrt((double)n), pst, coef);
        double* const gal = a.alpha + (int64_t)g * a.nv * a.m;
        double* const gbe = a.beta + (int64_t)g * a.nv * a.m;
        __syncthreads();

        for (int j = 1; j <= a.m; ++j) {
            const float4 sgm = make_float4(coef[4 * q], coef[4 * q + 1], coef[4 * q + 2], coef[4 * q + 3]);
            const float4 tau = make_float4(coef[4 * F + 4 * q], coef[4 * F + 4 * q + 1], coef[4 * F + 4 * q + 2],
                                           coef[4 * F + 4 * q + 3]);
            double s1[4] = {0.0, 0.0, 0.0, 0.0};
            const bool sgj = a.sign_first && j == 1;
            for (int i = row0; tact && i < n; i += rstride) {
                const int64_t s = rp[i], e = rp[i + 1];
                float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
                int64_t kk = s;
                if (sgj) {  // first step: gather sign records, expand after each round's loads
                    const uint4* const Rl = (const uint4*)P + sh;
                    for (; kk + kBatchUnroll <= e; kk += kBatchUnroll) {
                        unsigned c[kBatchUnroll];
#pragma unroll
                        for (int u = 0; u < kBatchUnroll; ++u)
                            c[u] = min((unsigned)(int)(col[kk + u] - base), (unsigned)n);
                        uint4 r[kBatchUnroll];
#pragma unroll
                        for (int u = 0; u < kBatchUnroll; ++u) r[u] = Rl[(int64_t)c[u] * slots];
#pragma unroll
                        for (int u = 0; u < kBatchUnroll; ++u) {
                            const float4 x = sign_expand4(r[u], 4 * q, a.nv);
                            acc.x += x.x;
                            acc.y += x.y;
                            acc.z += x.z;
                            acc.w += x.w;
                        }
                    }
                    for (; kk < e; ++kk) {
                        const unsigned c = min((unsigned)(int)(col[kk] - base), (unsigned)n);
                        const float4 x = sign_expand4(Rl[(int64_t)c * slots], 4 * q, a.nv);
                        acc.x += x.x;
                        acc.y += x.y;
                        acc.z += x.z;
                        acc.w += x.w;
                    }
                }
                for (; kk + kBatchUnroll <= e; kk += kBatchUnroll) {
                    // a column outside the graph reads the zero row n: ignored
                    unsigned c[kBatchUnroll];
#pragma unroll
                    for (int u = 0; u < kBatchUnroll; ++u) c[u] = min((unsigned)(int)(col[kk + u] - base), (unsigned)n);
                    float4 x[kBatchUnroll];
#pragma unroll
                    for (int u = 0; u < kBatchUnroll; ++u) x[u] = X[(int64_t)c[u] * F + q];
#pragma unroll
                    for (int u = 0; u < kBatchUnroll; ++u) {
                        acc.x += x[u].x;
                        acc.y += x[u].y;
                        acc.z += x[u].z;
                        acc.w += x[u].w;
                    }
                }
                for (; kk < e; ++kk) {
                    const unsigned c = min((unsigned)(int)(col[kk] - base), (unsigned)n);
                    const float4 x = X[(int64_t)c * F + q];
                    acc.x += x.x;
                    acc.y += x.y;
                    acc.z += x.z;
                    acc.w += x.w;
                }
                const float di = dinv[i];
                const double dd = (double)di, d2 = dd * dd, wgt = di != 0.0f ? 1.0 / d2 : 1.0;
                const int64_t at = (int64_t)i * F + q;
                const float4 ri = X[at];
                const float4 pr = j > 1 ? P[at] : make_float4(0.f, 0.f, 0.f, 0.f);
                const float* rv = &ri.x;
                const float* av = &acc.x;
                const float* pv = &pr.x;
                const float* sv = &sgm.x;
                const float* tv = &tau.x;
                float4 w;
                float* wp = &w.x;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const double lr = di != 0.0f ? fma(-d2, (double)av[c], (double)rv[c]) : 0.0;
                    wp[c] = (float)fma(-(double)tv[c], (double)pv[c], (double)sv[c] * lr);
                    s1[c] = fma((double)rv[c] * (double)wp[c], wgt, s1[c]);
                }
                W[at] = w;
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) red[4 * t + c] = s1[c];
            __syncthreads();
            reduce_chunks(t, B, F, bact, a.nv, red, red2);
            __syncthreads();
            if (t < a.nv) finish_alpha(t, a.nv, a.m, j, red2, pst, F, coef, gal, a.dstat);
            __syncthreads();
            const float4 av = make_float4(coef[8 * F + 4 * q], coef[8 * F + 4 * q + 1], coef[8 * F + 4 * q + 2],
                                          coef[8 * F + 4 * q + 3]);
            double s2[4] = {0.0, 0.0, 0.0, 0.0};
            for (int i = row0; tact && i < n; i += rstride) {
                const int64_t at = (int64_t)i * F + q;
                const float4 ri = X[at];
                const float4 wv = W[at];
                const float di = dinv[i];
                const double wgt = di != 0.0f ? 1.0 / ((double)di * (double)di) : 1.0;
                float4 r;
                r.x = fmaf(-av.x, ri.x, wv.x);
                r.y = fmaf(-av.y, ri.y, wv.y);
                r.z = fmaf(-av.z, ri.z, wv.z);
                r.w = fmaf(-av.w, ri.w, wv.w);
                P[at] = r;
                s2[0] = fma((double)r.x * (double)r.x, wgt, s2[0]);
                s2[1] = fma((double)r.y * (double)r.y, wgt, s2[1]);
                s2[2] = fma((double)r.z * (double)r.z, wgt, s2[2]);
                s2[3] = fma((double)r.w * (double)r.w, wgt, s2[3]);
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) red[4 * t + c] = s2[c];
            __syncthreads();
            reduce_chunks(t, B, F, bact, a.nv, red, red2);
            __syncthreads();
            if (t < a.nv) finish_beta(t, a.nv, a.m, j, red2, pst, F, coef, gbe, a.dstat);
            __syncthreads();
            float4* const tmp = X;  // X_{j+1} now lives in P; X_j becomes the previous block
            X = P;
            P = tmp;
        }
        if (t < a.nv) a.steps[(int64_t)g * a.nv + t] = (int32_t)pst[5 * t + 4];
        if (t == 0) a.trace[g] = (double)s_nz - s_corr;  // tr L of the normalized Laplacian
        __syncthreads();
    }
}

__global__ void reset_queues(int* q, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) q[i] = 0;
}

// Per graph from its Gauss rules: heat[g][b] = n_g/nv sum tau2 exp(-t_b theta)
// and vnge[g] = -n_g/nv sum tau2 g(theta / tr L_g), g(x) = x ln x for x > 0
// (fixed-order tree for the VNGE sum).  Blocks stride over the graphs.
__global__ void __launch_bounds__(256) batch_outputs(const int64_t* __restrict__ goff, int64_t G, int nv, int m,
                                                     const double* __restrict__ theta,
                                                     const double* __restrict__ tau2,
                                                     const double* __restrict__ trace, int nt,
                                                     const double* __restrict__ tgrid, double* __restrict__ heat,
                                                     double* __restrict__ vnge) {
    __shared__ double red[256];
    const int tid = threadIdx.x;
    const int cnt = nv * m;
    for (int64_t g = blockIdx.x; g < G; g += gridDim.x) {
        const double scale = (double)(goff[g + 1] - goff[g]) / (double)nv;
        const double* th = theta + g * cnt;
        const double* w2 = tau2 + g * cnt;
        if (heat)
            for (int b = tid; b < nt; b += 256) {
                const double tt = tgrid[b];
                double s = 0.0;
                for (int i = 0; i < cnt; ++i) s += w2[i] * exp(-tt * th[i]);
                heat[g * nt + b] = scale * s;
            }
        if (vnge) {
            const double c = trace[g];
            double s = 0.0;
            if (c > 0.0)
                for (int i = tid; i < cnt; i += 256) {
                    const double x = th[i] / c;
                    if (x > 0.0) s += w2[i] * (x * log(x));
                }
            red[tid] = s;
            __syncthreads();
            for (int off = 128; off > 0; off >>= 1) {
                if (tid < off) red[tid] += red[tid + off];
                __syncthreads();
            }
            if (tid == 0) vnge[g] = -scale * red[0];
            __syncthreads();
        }
    }
}

// ------------------------------------------------------------- host plan --
struct BucketCfg {
    int n_lo, n_hi;   // graphs with n in (n_lo, n_hi]
    int block;        // threads per workgroup
    int ipt;          // items per thread (ceil(n_hi*F / active threads)); 0 for global buckets
    int grid;         // persistent workgroups
    size_t lds;
    bool global;      // probe blocks in the global workspace (batch_slq_global)
    int slots;        // workspace slots of a global bucket (caps its grid)
};

typedef void (*BatchKernel)(BatchArgs);
typedef void (*BatchGlobalKernel)(BatchArgs, float4*, int64_t, float*, int64_t);

// probe blocks above this size go to the global-workspace kernel (an LDS
// block this large would leave one workgroup per CU)
constexpr size_t kLdsVecMax = 64 * 1024;
// global workspace of a plan: slots of 3 n_hi F quads + n_hi floats, as many
// as fit this budget (at most 8 per CU)
constexpr size_t kGlobalWsBudget = size_t(16) << 30;

// Largest graph the LDS kernels serve for nv probes: the probe block within
// kLdsVecMax, and rows per thread within the largest instantiation of each
// workgroup size (pick_kernel: 32, 16, 8, 4 rows at 128, 256, 512, 1024).
static int64_t lds_node_cap(int nv) {
    const int F = (nv + 3) / 4;
    static const int table[4][2] = {{128, 32}, {256, 16}, {512, 8}, {1024, 4}};
    int64_t rows = 0;
    for (const auto& e : table) rows = std::max<int64_t>(rows, (int64_t)(e[0] / F) * e[1]);
    return std::min<int64_t>((int64_t)(kLdsVecMax / ((size_t)F * 16)), rows);
}

static BatchGlobalKernel pick_global(int block) {
    switch (block) {
        case 128: return batch_slq_global<128>;
        case 256: return batch_slq_global<256>;
        case 512: return batch_slq_global<512>;
        case 1024: return batch_slq_global<1024>;
        default: return nullptr;
    }
}

static BatchKernel pick_kernel(int block, int ipt) {
#define SLAQ_BK(Bv, Iv) if (block == Bv && ipt <= Iv) return batch_slq<Bv, Iv>;
    SLAQ_BK(128, 1) SLAQ_BK(128, 2) SLAQ_BK(128, 3) SLAQ_BK(128, 4) SLAQ_BK(128, 6) SLAQ_BK(128, 8)
    SLAQ_BK(128, 12) SLAQ_BK(128, 16) SLAQ_BK(128, 24) SLAQ_BK(128, 32)
    SLAQ_BK(256, 1) SLAQ_BK(256, 2) SLAQ_BK(256, 3) SLAQ_BK(256, 4) SLAQ_BK(256, 6) SLAQ_BK(256, 8)
    SLAQ_BK(256, 12) SLAQ_BK(256, 16)
    SLAQ_BK(512, 1) SLAQ_BK(512, 2) SLAQ_BK(512, 3) SLAQ_BK(512, 4) SLAQ_BK(512, 6) SLAQ_BK(512, 8)
    SLAQ_BK(1024, 1) SLAQ_BK(1024, 2) SLAQ_BK(1024, 3) SLAQ_BK(1024, 4)
#undef SLAQ_BK
    return nullptr;
}

}  // namespace slaq

struct slaq_batch_s {
    int64_t G;
    int nv, m, nt;
    const int64_t* goff;  // device
    const int64_t* rp;    // device
    const int32_t* col;   // device
    std::vector<slaq::BucketCfg> buckets;
    std::vector<int> bucket_start;  // offset into order per bucket
    int32_t* order_dev;             // library-owned
    int* queues_dev;                // library-owned, one counter per bucket
    std::vector<std::vector<int32_t>> order_host;
    // library-owned results of the last run when the caller passes no buffer:
    // alpha, beta, theta, tau2 [G][nv][m], steps [G][nv], tr L [G]
    double *al_dev, *be_dev, *th_dev, *w2_dev, *tr_dev;
    int32_t* st_dev;
    // workspace of the global bucket (probe blocks, then D^-1/2, per slot):
    // the caller's (slaq_batch_set_workspace) or allocated at the first run
    int64_t ws_quads, ws_floats;
    size_t ws_bytes;
    void* ws;
    bool ws_owned;
    hipGraphExec_t exec;
    hipGraph_t graph;
    hipStream_t cap;  // private stream used only for capture (the NULL stream cannot be captured)
    // side streams and events: the buckets of a run are launched concurrently
    // (bucket k > 0 on side[k - 1], forked from and joined to the caller's stream)
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> joins;
    hipEvent_t fork;
    const uint64_t* seeds;  // caller's per-graph seeds (device) or NULL
    int sign_step;          // global buckets: first step from sign records (default 1)
    const void* exec_key[9];
    uint64_t exec_seed;
};

namespace slaq {

static void free_plan(slaq_batch_s* b) {
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        (void)hipGraphDestroy(b->graph);
    }
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (hipStream_t x : b->side) (void)hipStreamDestroy(x);
    for (hipEvent_t e : b->joins) (void)hipEventDestroy(e);
    if (b->fork) (void)hipEventDestroy(b->fork);
    for (void* p : {(void*)b->order_dev, (void*)b->queues_dev, (void*)b->al_dev, (void*)b->be_dev,
                    (void*)b->th_dev, (void*)b->w2_dev, (void*)b->st_dev, (void*)b->tr_dev,
                    b->ws_owned ? b->ws : nullptr})
        if (p) (void)hipFree(p);
    delete b;
}

static int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 256;
    return cus > 0 ? cus : 256;
}

static slaq_status configure_bucket(BucketCfg& b, int nv, int block) {
    const int F = (nv + 3) / 4;
    const int bact = (block / F) * F;
    SLAQ_REQUIRE(bact >= F && bact >= nv, SLAQ_ERR_UNSUPPORTED, "block %d too small for nv=%d", block, nv);
    if (b.global) {
        BatchGlobalKernel k = pick_global(block);
        SLAQ_REQUIRE(k, SLAQ_ERR_UNSUPPORTED, "no global batched kernel for block %d", block);
        b.block = block;
        b.ipt = 0;
        b.lds = batch_lds(0, nv, block).total;
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, block, b.lds) != hipSuccess || per_cu < 1)
            per_cu = 1;
        b.grid = std::min(device_cus() * per_cu, b.slots);
        return SLAQ_OK;
    }
    const int rows_per_pass = bact / F;
    const int ipt = (b.n_hi + rows_per_pass - 1) / rows_per_pass;
    static const int sizes[] = {1, 2, 3, 4, 6, 8, 12, 16, 24, 32};
    int ipt_r = 0;
    for (int v : sizes)
        if (v >= ipt && pick_kernel(block, v)) {
            ipt_r = v;
            break;
        }
    SLAQ_REQUIRE(ipt_r > 0 && pick_kernel(block, ipt_r), SLAQ_ERR_UNSUPPORTED,
                 "no batched kernel for block %d, %d rows per thread (n up to %d)", block, ipt_r, b.n_hi);
    b.block = block;
    b.ipt = ipt_r;
    b.lds = batch_lds(b.n_hi, nv, block).total;
    SLAQ_REQUIRE(b.lds <= 160 * 1024, SLAQ_ERR_UNSUPPORTED, "graphs of %d nodes need %zu bytes of LDS", b.n_hi, b.lds);
    BatchKernel k = pick_kernel(block, ipt_r);
    int per_cu = 0;
    if (hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)b.lds) != hipSuccess)
        per_cu = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, block, b.lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
    b.grid = device_cus() * per_cu;
    return SLAQ_OK;
}

}  // namespace slaq

using namespace slaq;

extern "C" {

slaq_status slaq_batch_plan(int64_t n_graphs, const int64_t* node_off, const int64_t* nnz_off,
                            const int64_t* node_off_dev, const int64_t* row_ptr, const int32_t* col_idx, int nv,
                            int m, int nt, const int* bucket_blocks, int n_buckets_cfg, slaq_batch_t* out) {
    return slaq_batch_plan_grown(n_graphs, node_off, nnz_off, node_off_dev, row_ptr, col_idx, nv, m, nt, 2.0,
                                 bucket_blocks, n_buckets_cfg, out);
}

slaq_status slaq_batch_plan_grown(int64_t n_graphs, const int64_t* node_off, const int64_t* nnz_off,
                                  const int64_t* node_off_dev, const int64_t* row_ptr, const int32_t* col_idx,
                                  int nv, int m, int nt, double growth, const int* bucket_blocks, int n_buckets_cfg,
                                  slaq_batch_t* out) {
    clear_error();
    SLAQ_REQUIRE(growth >= 1.25 && growth <= 8.0, SLAQ_ERR_INVALID_ARG, "bucket growth must be in [1.25, 8]");
    SLAQ_REQUIRE(out, SLAQ_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    SLAQ_REQUIRE(n_graphs >= 1 && node_off && nnz_off && node_off_dev && row_ptr && col_idx, SLAQ_ERR_INVALID_ARG,
                 "need n_graphs >= 1 and non-NULL offsets / CSR");
    SLAQ_REQUIRE(nv >= 1 && nv <= 256, SLAQ_ERR_INVALID_ARG, "batched nv must be in [1, 256]");
    SLAQ_REQUIRE(m >= 1 && m <= SLAQ_MAX_STEPS, SLAQ_ERR_INVALID_ARG, "m must be in [1, %d]", SLAQ_MAX_STEPS);
    SLAQ_REQUIRE(nt >= 0, SLAQ_ERR_INVALID_ARG, "nt must be >= 0");
    // size buckets by node count: (0,64], (64,128], (128,256], (256,512], ... up to the batch maximum
    int64_t nmax = 0;
    for (int64_t g = 0; g < n_graphs; ++g) {
        const int64_t n = node_off[g + 1] - node_off[g];
        SLAQ_REQUIRE(n >= 1, SLAQ_ERR_INVALID_ARG, "graph %lld has no nodes", (long long)g);
        SLAQ_REQUIRE(nnz_off[g + 1] >= nnz_off[g], SLAQ_ERR_INVALID_ARG, "nnz offsets decrease at %lld", (long long)g);
        nmax = std::max(nmax, n);
    }
    SLAQ_REQUIRE(node_off[n_graphs] <= INT32_MAX, SLAQ_ERR_UNSUPPORTED,
                 "a batch holds fewer than 2^31 nodes in all (column ids are int32)");
    SLAQ_REQUIRE(n_graphs * nv * m <= INT32_MAX, SLAQ_ERR_UNSUPPORTED,
                 "G * nv * m must stay below 2^31 (got %lld)", (long long)(n_graphs * nv * m));
    // LDS buckets by node counts growing from 64 by `growth` (doubling by
    // default) up to the largest probe block that stays in LDS, then one global bucket for every larger graph (a single
    // persistent launch pulling them largest first keeps the CUs busy where
    // size classes of their own would each leave most of the chip idle)
    const int64_t lds_cap_n = lds_node_cap(nv);
    std::vector<int64_t> edges = {0, std::min<int64_t>(64, lds_cap_n)};
    while (edges.back() < nmax && edges.back() < lds_cap_n) {
        const int64_t next = std::max<int64_t>(edges.back() + 1, (int64_t)std::ceil((double)edges.back() * growth));
        edges.push_back(std::min<int64_t>(next, lds_cap_n));
    }
    if (edges.back() < nmax) edges.push_back(nmax);
    slaq_batch_s* b = new (std::nothrow) slaq_batch_s();
    SLAQ_REQUIRE(b, SLAQ_ERR_INVALID_ARG, "out of host memory");
    b->G = n_graphs;
    b->sign_step = 1;
    b->nv = nv;
    b->m = m;
    b->nt = nt;
    b->goff = node_off_dev;
    b->rp = row_ptr;
    b->col = col_idx;
    const int nb = (int)edges.size() - 1;
    std::vector<std::vector<std::pair<int64_t, int32_t>>> members(nb);
    for (int64_t g = 0; g < n_graphs; ++g) {
        const int64_t n = node_off[g + 1] - node_off[g];
        int k = 0;
        while (n > edges[k + 1]) ++k;
        // cost ~ nnz * nv * m + n * nt (gathers, quadrature)
        members[k].push_back({(nnz_off[g + 1] - nnz_off[g]) + n, (int32_t)g});
    }
    std::vector<int32_t> order;
    for (int k = 0; k < nb; ++k) {
        if (members[k].empty()) continue;
        std::stable_sort(members[k].begin(), members[k].end(),
                         [](const std::pair<int64_t, int32_t>& x, const std::pair<int64_t, int32_t>& y) {
                             return x.first > y.first;
                         });
        BucketCfg c{};
        c.n_lo = (int)edges[k];
        c.n_hi = std::min<int64_t>(edges[k + 1], nmax);
        int64_t top = 0;
        for (auto& pr : members[k]) top = std::max<int64_t>(top, node_off[pr.second + 1] - node_off[pr.second]);
        c.n_hi = (int)top;
        const int Fq = (nv + 3) / 4;
        c.global = c.n_hi > lds_cap_n;
        const size_t slot_bytes = (size_t)3 * (c.n_hi + 1) * Fq * 16 + (size_t)c.n_hi * 4;
        if (c.global)
            c.slots = (int)std::max<size_t>(1, std::min<size_t>(kGlobalWsBudget / slot_bytes,
                                                                (size_t)device_cus() * 8));
        const int bidx = (int)b->buckets.size();
        // defaults (slaq_batch_autotune refines them); a global bucket is led by
        // its largest graphs, each on one workgroup: the widest one finishes
        // them soonest (1024 threads: 80 ms against 97 at 512 for 2,000 graphs
        // of 1e3 to 1e5 nodes, nv = 20, m = 5)
        int block = c.global ? 1024 : (c.n_hi <= 64 ? 128 : (c.n_hi <= 256 ? 256 : 512));
        const bool forced = bucket_blocks && bidx < n_buckets_cfg && bucket_blocks[bidx] > 0;
        if (forced) block = bucket_blocks[bidx];
        slaq_status s = configure_bucket(c, nv, block);
        // a default size too small for the probe count (one thread per probe
        // finishes the sums) or for the bucket's rows: the next larger one
        for (int wider = block * 2; s != SLAQ_OK && !forced && wider <= 1024; wider *= 2) {
            s = configure_bucket(c, nv, wider);
            if (s == SLAQ_OK) clear_error();
        }
        if (s != SLAQ_OK) {
            delete b;
            return s;
        }
        if (c.global) {
            // one slot per workgroup the chosen block keeps resident (the
            // autotuner's other sizes are capped to as many)
            c.slots = std::min(c.slots, c.grid);
            b->ws_quads = (int64_t)c.slots * 3 * (c.n_hi + 1) * Fq;  // + a zero row per buffer
            b->ws_floats = (int64_t)c.slots * c.n_hi;
            b->ws_bytes = align_up((size_t)b->ws_quads * 16, 256) + align_up((size_t)b->ws_floats * 4, 256);
        }
        b->bucket_start.push_back((int)order.size());
        std::vector<int32_t> ids;
        for (auto& pr : members[k]) {
            order.push_back(pr.second);
            ids.push_back(pr.second);
        }
        b->order_host.push_back(ids);
        b->buckets.push_back(c);
    }
    b->bucket_start.push_back((int)order.size());
    const size_t coeffs = (size_t)n_graphs * nv * m * sizeof(double);
    if (hipMalloc(&b->order_dev, order.size() * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&b->queues_dev, b->buckets.size() * sizeof(int)) != hipSuccess ||
        hipMalloc(&b->al_dev, coeffs) != hipSuccess || hipMalloc(&b->be_dev, coeffs) != hipSuccess ||
        hipMalloc(&b->th_dev, coeffs) != hipSuccess || hipMalloc(&b->w2_dev, coeffs) != hipSuccess ||
        hipMalloc(&b->st_dev, (size_t)n_graphs * nv * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&b->tr_dev, (size_t)n_graphs * sizeof(double)) != hipSuccess) {
        free_plan(b);
        set_error("hipMalloc of the batch plan failed");
        return SLAQ_ERR_HIP;
    }
    if (hipMemcpy(b->order_dev, order.data(), order.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess) {
        free_plan(b);
        set_error("copy of the batch order failed");
        return SLAQ_ERR_HIP;
    }
    *out = b;
    return SLAQ_OK;
}

slaq_status slaq_batch_buckets(slaq_batch_t b, int* n_buckets, int* n_hi, int* blocks, int* graphs, int* in_lds) {
    clear_error();
    SLAQ_REQUIRE(b && n_buckets, SLAQ_ERR_INVALID_ARG, "NULL argument");
    *n_buckets = (int)b->buckets.size();
    for (size_t k = 0; k < b->buckets.size(); ++k) {
        if (n_hi) n_hi[k] = b->buckets[k].n_hi;
        if (blocks) blocks[k] = b->buckets[k].block;
        if (graphs) graphs[k] = b->bucket_start[k + 1] - b->bucket_start[k];
        if (in_lds) in_lds[k] = b->buckets[k].global ? 0 : 1;
    }
    return SLAQ_OK;
}

// the global bucket's workspace (allocated here at the first run unless the
// caller gave one) and the side streams of the bucket launches; never while a
// stream is being captured
static slaq_status ensure_workspace(slaq_batch_t b) {
    if (b->side.empty() && b->buckets.size() > 1) {
        SLAQ_HIP(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
        for (size_t k = 1; k < b->buckets.size(); ++k) {
            hipStream_t x = nullptr;
            hipEvent_t e = nullptr;
            SLAQ_HIP(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
            b->side.push_back(x);
            SLAQ_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            b->joins.push_back(e);
        }
    }
    if (b->ws_bytes == 0 || b->ws) return SLAQ_OK;
    SLAQ_HIP(hipMalloc(&b->ws, b->ws_bytes));
    b->ws_owned = true;
    return SLAQ_OK;
}

static slaq_status enqueue_batch(slaq_batch_t b, uint64_t seed, const double* t, double* heat, double* vnge,
                                 double* alpha, double* beta, int32_t* steps, double* theta, double* tau2,
                                 hipStream_t st, int only_bucket) {
    const int nbk = (int)b->buckets.size();
    double* al = alpha ? alpha : b->al_dev;
    double* be = beta ? beta : b->be_dev;
    int32_t* sp = steps ? steps : b->st_dev;
    hipLaunchKernelGGL(reset_queues, dim3(1), dim3(64), 0, st, b->queues_dev, nbk);
    SLAQ_LAUNCHED();
    // every bucket of a full run on a stream of its own: their persistent grids
    // fill one another's tails
    const bool fan = only_bucket < 0 && nbk > 1 && (int)b->side.size() == nbk - 1;
    if (fan) SLAQ_HIP(hipEventRecord(b->fork, st));
    for (int k = 0; k < nbk; ++k) {
        if (only_bucket >= 0 && k != only_bucket) continue;
        const BucketCfg& c = b->buckets[k];
        hipStream_t bs = st;
        if (fan && k > 0) {
            bs = b->side[k - 1];
            SLAQ_HIP(hipStreamWaitEvent(bs, b->fork, 0));
        }
        BatchArgs a{};
        a.order = b->order_dev + b->bucket_start[k];
        a.count = b->bucket_start[k + 1] - b->bucket_start[k];
        a.queue = b->queues_dev + k;
        a.goff = b->goff;
        a.rp = b->rp;
        a.col = b->col;
        a.nv = b->nv;
        a.m = b->m;
        a.n_max = c.n_hi;
        a.seed = seed;
        a.seeds = b->seeds;
        a.alpha = al;
        a.beta = be;
        a.steps = sp;
        a.trace = b->tr_dev;
        a.dstat = device_status_word();
        a.sign_first = b->sign_step;
        SLAQ_REQUIRE(a.dstat, SLAQ_ERR_HIP, "device status word unavailable");
        const int grid = std::min(c.grid, a.count);
        if (c.global) {
            const int Fq = (b->nv + 3) / 4;
            BatchGlobalKernel kern = pick_global(c.block);
            SLAQ_REQUIRE(b->ws, SLAQ_ERR_WORKSPACE, "the batch plan has no workspace");
            float4* gws = (float4*)b->ws;
            float* gwsd = (float*)((char*)b->ws + align_up((size_t)b->ws_quads * 16, 256));
            SLAQ_TIMED("batch_slq", bs,
                       hipLaunchKernelGGL(kern, dim3(grid), dim3(c.block), c.lds, bs, a, gws,
                                          (int64_t)(c.n_hi + 1) * Fq, gwsd, (int64_t)c.n_hi));
        } else {
            BatchKernel kern = pick_kernel(c.block, c.ipt);
            SLAQ_TIMED("batch_slq", bs, hipLaunchKernelGGL(kern, dim3(grid), dim3(c.block), c.lds, bs, a));
        }
        SLAQ_LAUNCHED();
        if (fan && k > 0) {
            SLAQ_HIP(hipEventRecord(b->joins[k - 1], bs));
            SLAQ_HIP(hipStreamWaitEvent(st, b->joins[k - 1], 0));
        }
    }
    if (only_bucket >= 0) return SLAQ_OK;  // autotuner trial: the Lanczos part of one bucket
    if (!(heat || vnge || theta)) return SLAQ_OK;
    double* th = theta ? theta : b->th_dev;
    double* w2 = tau2 ? tau2 : b->w2_dev;
    SLAQ_TRY(slaq_ritz(al, be, sp, (int)(b->G * b->nv), b->m, th, w2, st));
    if (heat || vnge) {
        const int grid = (int)std::min<int64_t>(b->G, 8192);
        SLAQ_TIMED("batch_outputs", st,
                   hipLaunchKernelGGL(batch_outputs, dim3(grid), dim3(256), 0, st, b->goff, b->G, b->nv, b->m, th,
                                      w2, b->tr_dev, b->nt, t, heat, vnge));
        SLAQ_LAUNCHED();
    }
    return SLAQ_OK;
}

slaq_status slaq_batch_run(slaq_batch_t b, uint64_t seed, const double* t, double* heat, double* vnge, double* alpha,
                           double* beta, int32_t* steps, double* theta, double* tau2, unsigned flags, void* stream) {
    clear_error();
    SLAQ_REQUIRE(b, SLAQ_ERR_INVALID_ARG, "batch plan is NULL");
    SLAQ_REQUIRE(!heat || (t && b->nt > 0), SLAQ_ERR_INVALID_ARG, "heat needs the time grid t (nt > 0)");
    SLAQ_REQUIRE((!beta || alpha) && (!tau2 || theta), SLAQ_ERR_INVALID_ARG, "beta needs alpha, tau2 needs theta");
    hipStream_t st = (hipStream_t)stream;
    SLAQ_TRY(ensure_workspace(b));
    if (!(flags & SLAQ_BATCH_GRAPH)) return enqueue_batch(b, seed, t, heat, vnge, alpha, beta, steps, theta, tau2, st, -1);
    // replay one captured hipGraph; (re)capture when the buffers or the seed change
    const void* key[9] = {t, heat, vnge, alpha, beta, steps, theta, tau2, b->seeds};
    const bool same = b->exec && std::memcmp(key, b->exec_key, sizeof(key)) == 0 && b->exec_seed == seed;
    if (!same) {
        if (b->exec) {
            (void)hipGraphExecDestroy(b->exec);
            (void)hipGraphDestroy(b->graph);
            b->exec = nullptr;
        }
        if (!b->cap) SLAQ_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
        SLAQ_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
        slaq_status s = enqueue_batch(b, seed, t, heat, vnge, alpha, beta, steps, theta, tau2, b->cap, -1);
        hipGraph_t gr = nullptr;
        hipError_t e = hipStreamEndCapture(b->cap, &gr);
        SLAQ_REQUIRE(s == SLAQ_OK, s, "%s", slaq_last_error());
        SLAQ_HIP(e);
        SLAQ_HIP(hipGraphInstantiate(&b->exec, gr, nullptr, nullptr, 0));
        b->graph = gr;
        std::memcpy(b->exec_key, key, sizeof(key));
        b->exec_seed = seed;
    }
    SLAQ_HIP(hipGraphLaunch(b->exec, st));
    return SLAQ_OK;
}

// Host autotuner: for every bucket, time each candidate block size (HIP events,
// median of `reps` runs of that bucket alone) and keep the fastest.  Writes the
// chosen block per bucket to blocks_out (n_buckets entries) when non-NULL.
slaq_status slaq_batch_autotune(slaq_batch_t b, const double* t, double* heat, double* vnge, int reps,
                                int* blocks_out, float* best_ms_out, void* stream) {
    clear_error();
    SLAQ_REQUIRE(b, SLAQ_ERR_INVALID_ARG, "batch plan is NULL");
    SLAQ_REQUIRE(reps >= 1 && reps <= 100, SLAQ_ERR_INVALID_ARG, "reps must be in [1, 100]");
    hipStream_t st = (hipStream_t)stream;
    SLAQ_TRY(ensure_workspace(b));
    const int cand[4] = {128, 256, 512, 1024};
    hipEvent_t e0, e1;
    SLAQ_HIP(hipEventCreate(&e0));
    SLAQ_HIP(hipEventCreate(&e1));
    for (size_t k = 0; k < b->buckets.size(); ++k) {
        BucketCfg best = b->buckets[k];
        float best_ms = 1e30f;
        for (int ci = 0; ci < 4; ++ci) {
            BucketCfg c = b->buckets[k];
            if (configure_bucket(c, b->nv, cand[ci]) != SLAQ_OK) continue;
            const BucketCfg keep = b->buckets[k];
            b->buckets[k] = c;
            std::vector<float> ts;
            for (int r = 0; r < reps; ++r) {
                SLAQ_HIP(hipEventRecord(e0, st));
                slaq_status s = enqueue_batch(b, 12345, t, heat, vnge, nullptr, nullptr, nullptr, nullptr, nullptr, st,
                                              (int)k);
                if (s != SLAQ_OK) {
                    b->buckets[k] = keep;
                    return s;
                }
                SLAQ_HIP(hipEventRecord(e1, st));
                SLAQ_HIP(hipEventSynchronize(e1));
                float ms = 0.0f;
                SLAQ_HIP(hipEventElapsedTime(&ms, e0, e1));
                ts.push_back(ms);
            }
            std::sort(ts.begin(), ts.end());
            const float med = ts[ts.size() / 2];
            if (med < best_ms) {
                best_ms = med;
                best = c;
            }
            b->buckets[k] = keep;
        }
        b->buckets[k] = best;
        if (blocks_out) blocks_out[k] = best.block;
        if (best_ms_out) best_ms_out[k] = best_ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (b->exec) {  // schedule changed: drop the captured graph
        (void)hipGraphExecDestroy(b->exec);
        (void)hipGraphDestroy(b->graph);
        b->exec = nullptr;
    }
    return SLAQ_OK;
}

slaq_status slaq_batch_workspace(slaq_batch_t b, size_t* bytes) {
    clear_error();
    SLAQ_REQUIRE(b && bytes, SLAQ_ERR_INVALID_ARG, "NULL argument");
    *bytes = b->ws_bytes;
    return SLAQ_OK;
}

slaq_status slaq_batch_set_workspace(slaq_batch_t b, void* workspace, size_t bytes) {
    clear_error();
    SLAQ_REQUIRE(b, SLAQ_ERR_INVALID_ARG, "batch plan is NULL");
    SLAQ_REQUIRE(!workspace || bytes >= b->ws_bytes, SLAQ_ERR_WORKSPACE,
                 "batch workspace needs %zu bytes, got %zu", b->ws_bytes, bytes);
    SLAQ_REQUIRE(((uintptr_t)workspace & 255) == 0, SLAQ_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (b->ws_owned) {
        SLAQ_HIP(hipFree(b->ws));
        b->ws_owned = false;
    }
    b->ws = b->ws_bytes ? workspace : nullptr;
    if (b->exec) {  // launches captured with the old workspace
        (void)hipGraphExecDestroy(b->exec);
        (void)hipGraphDestroy(b->graph);
        b->exec = nullptr;
    }
    return SLAQ_OK;
}

slaq_status slaq_batch_set_seeds(slaq_batch_t b, const uint64_t* seeds) {
    clear_error();
    SLAQ_REQUIRE(b, SLAQ_ERR_INVALID_ARG, "batch plan is NULL");
    b->seeds = seeds;
    return SLAQ_OK;
}

slaq_status slaq_batch_set_sign_step(slaq_batch_t b, int on) {
    clear_error();
    SLAQ_REQUIRE(b, SLAQ_ERR_INVALID_ARG, "batch plan is NULL");
    SLAQ_REQUIRE(on == 0 || on == 1, SLAQ_ERR_INVALID_ARG, "on must be 0 or 1");
    if (b->sign_step != on && b->exec) {  // the captured launches carry the old setting
        (void)hipGraphExecDestroy(b->exec);
        (void)hipGraphDestroy(b->graph);
        b->exec = nullptr;
    }
    b->sign_step = on;
    return SLAQ_OK;
}

slaq_status slaq_batch_autotune_edges(int64_t n_graphs, const int64_t* node_off, const int64_t* nnz_off,
                                      const int64_t* node_off_dev, const int64_t* row_ptr, const int32_t* col_idx,
                                      int nv, int m, int nt, const double* t, int reps, double* growth_out,
                                      float* ms_out, slaq_batch_t* out, void* stream) {
    clear_error();
    SLAQ_REQUIRE(out && t, SLAQ_ERR_INVALID_ARG, "NULL argument");
    SLAQ_REQUIRE(reps >= 1 && reps <= 100, SLAQ_ERR_INVALID_ARG, "reps must be in [1, 100]");
    SLAQ_REQUIRE(nt >= 1, SLAQ_ERR_INVALID_ARG, "need nt >= 1 time scales to time the runs");
    *out = nullptr;
    hipStream_t st = (hipStream_t)stream;
    double *heat = nullptr, *vn = nullptr;
    if (hipMalloc(&heat, (size_t)n_graphs * nt * sizeof(double)) != hipSuccess ||
        hipMalloc(&vn, (size_t)n_graphs * sizeof(double)) != hipSuccess) {
        if (heat) (void)hipFree(heat);
        set_error("hipMalloc of the tuning outputs failed");
        return SLAQ_ERR_HIP;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    slaq_status r = SLAQ_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        set_error("hipEventCreate failed");
        r = SLAQ_ERR_HIP;
    }
    slaq_batch_t best = nullptr;
    float best_ms = 1e30f;
    double best_g = 2.0;
    const double growths[] = {2.0, 1.5, 3.0};
    for (double gr : growths) {
        if (r != SLAQ_OK) break;
        slaq_batch_t b = nullptr;
        r = slaq_batch_plan_grown(n_graphs, node_off, nnz_off, node_off_dev, row_ptr, col_idx, nv, m, nt, gr,
                                  nullptr, 0, &b);
        if (r == SLAQ_OK) r = slaq_batch_autotune(b, t, heat, vn, reps, nullptr, nullptr, st);
        std::vector<float> ts;
        for (int k = 0; r == SLAQ_OK && k <= reps; ++k) {  // one untimed run first
            if (hipEventRecord(e0, st) != hipSuccess) r = SLAQ_ERR_HIP;
            if (r == SLAQ_OK)
                r = slaq_batch_run(b, 12345, t, heat, vn, nullptr, nullptr, nullptr, nullptr, nullptr, 0, st);
            float ms = 0.0f;
            if (r == SLAQ_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                 hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                r = SLAQ_ERR_HIP;
            if (k > 0) ts.push_back(ms);
        }
        if (r != SLAQ_OK) {
            if (b) slaq_batch_destroy(b);
            break;
        }
        std::sort(ts.begin(), ts.end());
        const float med = ts[ts.size() / 2];
        if (med < best_ms) {
            if (best) slaq_batch_destroy(best);
            best = b;
            best_ms = med;
            best_g = gr;
        } else {
            slaq_batch_destroy(b);
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(heat);
    (void)hipFree(vn);
    if (r != SLAQ_OK) {
        if (best) slaq_batch_destroy(best);
        return r;
    }
    *out = best;
    if (growth_out) *growth_out = best_g;
    if (ms_out) *ms_out = best_ms;
    return SLAQ_OK;
}

slaq_status slaq_batch_destroy(slaq_batch_t b) {
    if (!b) return SLAQ_OK;
    free_plan(b);
    return SLAQ_OK;
}

}  // extern "C"
