// Block Lanczos-quadrature front end: Rademacher probes and m steps of the
// three-term recurrence on nv probes at once (paper §3.1, "s-step Lanczos";
// Algorithm 1's lanczos(L, s, nv)).
//
// The vectors are kept unnormalized: R_j = beta_{j-1} q_j, R_1 = v (the +-1
// probe), sigma_j = 1/||R_j||.  Per step j
//   spmm_pieces   partial sums sum_k A_ik X_j[k] of the pieces of heavy rows
//   spmm_rows     w = sigma_j L R_j - tau_{j-1} R_{j-1}  (tau_{j-1} = beta_{j-1} sigma_{j-1})
//                 and FP64 partial sums of R_j . w
//   finalize_a    alpha_j = sigma_j sum(R_j . w);  a_j = alpha_j sigma_j
//   update        R_{j+1} = w - a_j R_j and FP64 partial sums of ||R_{j+1}||^2
//   finalize_b    beta_j = ||R_{j+1}||, breakdown test, sigma_{j+1}, tau_j
// which is the recurrence of §3.1 (w = L q_j - beta_{j-1} q_{j-1},
// alpha_j = q_j.w, beta_j = ||w - alpha_j q_j||) with the scalings folded into
// the reads.  Reductions are fixed-order (no floating-point atomics).
//
// Vector precision V: FP32 (products of two floats are exact in FP64, so the
// dot products are FP64 sums of exact terms) or FP64 (the whole recurrence in
// FP64, for operators of wide spectral range such as D - A of a graph with
// hubs, where FP32 vectors lose orthogonality to the converged top of the
// spectrum within a few steps).  A "quad" is 16 bytes of a probe row: 4 floats
// or 2 doubles; a lane holds one quad.
//
// Block layout: a probe row of F quads is split into a main part of
// Fm = 8 floor(F / 8) quads (whole 128-byte lines, rows line-aligned) and a
// tail of Ft = F - Fm quads kept in a region of its own.  A row gather then
// touches Fm / 8 lines plus one 16 Ft-byte tail slot, where tails of eight or
// more rows share a line and stay in cache far longer; an unsplit 400-byte
// row (nv = 100) straddles four lines at any alignment.  Each lane serves one
// quad and so reads one region with one stride (VecMap::lane).
//
// Normalized Laplacian: the probe blocks are stored in the scaled basis
// X_j = D^-1/2 R_j (per row, with the same D^-1/2 the kernels read), so the
// SpMM sums plain neighbour rows, (A X_j)_i, with no per-nonzero scale; the
// row epilogue forms D^-1/2 w = sigma (X_i - dinv_i^2 (A X_j)_i) - tau X_{j-1,i}
// (which is D^-1/2 times sigma (L R_j)_i - tau R_{j-1,i}), the update keeps its
// form, and the dot products weight row i by 1/dinv_i^2 so that they are the
// ones of R: R_j.w = sum_i X_i (D^-1/2 w)_i / dinv_i^2.  D - A needs no scale.
//
// Isolated nodes have zero rows and columns in L, so on them every R_j is a
// multiple of the probe: R_j[i] = rho_j v[i] with rho_1 = 1, rho_0 = 0 and
// rho_{j+1} = -tau_{j-1} rho_{j-1} - a_j rho_j.  Their rows are never stored
// or streamed; their share of the two dot products is added in FP64 from
// rho (v[i]^2 = 1) and the isolated-node count.
#include <cmath>

#include <mutex>
#include <type_traits>

#include "common.hpp"
#include "profile.hpp"

namespace slaq {

constexpr int kPieceUnroll = 8;  // gathers in flight per group in the piece kernel
constexpr int kUpdateRows = 4;   // rows per group with their loads in flight in the update

// breakdown threshold relative to the spectral bound (above the rounding
// noise of FP32 vectors; the same for FP64 ones, so both stop where the FP64
// reference recurrence stops)
constexpr double kEpsBreakdown = 1e-6;

template <typename V>
struct alignas(16) Quad {
    static constexpr int E = 16 / sizeof(V);
    V v[E];
};

// Split row layout of a probe block (see the top of this file): quad q < Fm
// of row i at quad index i Fm + q, quad q >= Fm at tail + i Ft + (q - Fm).
struct VecMap {
    int Fm, Ft;
    int64_t tail;
    // quad index of (row i, this lane's quad) = off + i * stride
    __device__ __forceinline__ void lane(int quad, int64_t& off, int& stride) const {
        if (quad < Fm) {
            off = quad;
            stride = Fm;
        } else {
            off = tail + (quad - Fm);
            stride = Ft;
        }
    }
};

// Per-probe FP64 recurrence state (workspace).
struct ProbeState {
    double sigma;     // 1 / ||R_j||
    double tau;       // beta_{j-1} sigma_{j-1}
    double rho;       // isolated-node coefficient of R_j
    double rho_prev;  // ... of R_{j-1}
    double a;         // alpha_j sigma_j
    int active;
    int pad;
};

// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) output number counter+1 for `seed`.
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t counter) {
    uint64_t z = seed + (counter + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ float vfma(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double vfma(double a, double b, double c) { return fma(a, b, c); }

template <typename V>
__device__ __forceinline__ Quad<V> qzero() {
    Quad<V> q;
#pragma unroll
    for (int e = 0; e < Quad<V>::E; ++e) q.v[e] = V(0);
    return q;
}

template <typename V>
__device__ __forceinline__ void qfma(V s, const Quad<V>& x, Quad<V>& acc) {
#pragma unroll
    for (int e = 0; e < Quad<V>::E; ++e) acc.v[e] = vfma(s, x.v[e], acc.v[e]);
}

template <typename V>
__device__ __forceinline__ void qadd(Quad<V>& a, const Quad<V>& b) {
#pragma unroll
    for (int e = 0; e < Quad<V>::E; ++e) a.v[e] += b.v[e];
}

// quad `q` of a per-probe coefficient vector
template <typename V>
__device__ __forceinline__ Quad<V> qload(const V* p, int q) {
    Quad<V> r;
#pragma unroll
    for (int e = 0; e < Quad<V>::E; ++e) r.v[e] = p[Quad<V>::E * q + e];
    return r;
}

// Gathers and the Infinity Cache.  On a relabelled graph the labels of each
// column range run in decreasing degree order, so the range's first rows are
// the ones every step gathers most.  Gathers of those rows are ordinary loads;
// gathers of the rest, and the once-read column indices and piece partials,
// carry the non-temporal hint, which keeps their lines from displacing the hot
// rows in the 256 MB last-level cache (measured at R-MAT 26: piece kernel
// 99.4 -> 92 ms; hinting every gather instead: 131 ms).  A gathered column
// travels between lanes with the hint folded into its sign bit (labels are
// below 2^31).
__device__ __forceinline__ Quad<float> qload_nt(const Quad<float>* p) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    const f4 v = __builtin_nontemporal_load((const f4*)p);
    Quad<float> q;
    q.v[0] = v.x;
    q.v[1] = v.y;
    q.v[2] = v.z;
    q.v[3] = v.w;
    return q;
}
__device__ __forceinline__ Quad<double> qload_nt(const Quad<double>* p) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 v = __builtin_nontemporal_load((const d2*)p);
    Quad<double> q;
    q.v[0] = v.x;
    q.v[1] = v.y;
    return q;
}

// a packed column: the label, negative when its gather is a cold one
__device__ __forceinline__ int32_t pack_col(int32_t c, bool hot) { return hot ? c : (int32_t)((uint32_t)c | 0x80000000u); }

// row `c` of the lane's quad column (stride ms), hint from the packed column
template <typename V>
__device__ __forceinline__ Quad<V> gather(const Quad<V>* __restrict__ Rl, int32_t packed, int ms) {
    const Quad<V>* p = Rl + (int64_t)(packed & 0x7fffffff) * ms;
    return packed >= 0 ? *p : qload_nt(p);
}

// The first step's probe block in compact form.  R_1 is +-1 times one scale
// per row, so its gathers need not read the FP32 rows: record i is a run of
// 16-byte slots, each holding 4 - sizeof(V)/4 dwords of sign bits (bit p of
// the probe's dword set for -1, as the probe generator draws them) and then
// the row's value of +1 in X_1 (dinv_i for the normalized Laplacian, 1 for
// D - A, 0 on rows without data).  A lane loads the one slot with its
// probes' bits and the scale in a single 16-byte load (records take a power
// of two of slots, so a gather touches one cache line, against
// ceil(4 ld / 128) lines for the FP32 row) and expands it to exactly the
// values of X_1 (probes at or past nv to 0).  The expansion waits until all
// loads of a gather round are issued: expanding each slot right after its
// load serializes the round and is slower than gathering the rows.  Measured
// with nv = 100, first-step pieces / light rows: R-MAT 22 2.30 / 2.63 ms
// against 2.34-2.42 / 3.29-3.32 ms gathering the rows, R-MAT 24 10.5 / 8.2
// against 13.9 / 11.9 ms.
struct SignRows {
    const uint32_t* rec;
    int rd, nv;  // record dwords, probes
};

// one 16-byte slot of a sign record, as loaded
struct Slot {
    uint32_t x, y, z, w;
};

// the lane's slot of record `packed` (the column, hint in its sign bit)
template <typename V>
__device__ __forceinline__ Slot sign_load(const SignRows& sr, int32_t packed, int quad) {
    constexpr int E = Quad<V>::E, HW = 4 - (int)(sizeof(V) / 4);
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
    const int h = ((E * quad) >> 5) / HW;
    const u4* r = (const u4*)(sr.rec + (int64_t)(packed & 0x7fffffff) * sr.rd) + h;
    const u4 v = packed >= 0 ? *r : __builtin_nontemporal_load(r);
    return Slot{v.x, v.y, v.z, v.w};
}

// the lane's E values of X_1 from its slot: the scale is never negative, so a
// probe's value is the scale with its sign bit set from the probe's bit
// (padding probes, p >= nv, are 0; an all-zero slot gives +0)
template <typename V>
__device__ __forceinline__ Quad<V> sign_expand(const Slot& v, const SignRows& sr, int quad) {
    constexpr int E = Quad<V>::E, HW = 4 - (int)(sizeof(V) / 4);
    const int p0 = E * quad, w = p0 >> 5, pos = w - (w / HW) * HW;
    const uint32_t wd = pos == 0 ? v.x : (HW > 1 && pos == 1 ? v.y : v.z);
    Quad<V> q;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const uint32_t b = __builtin_amdgcn_ubfe(wd, (uint32_t)((p0 & 31) + e), 1u);
        if constexpr (sizeof(V) == 4) {
            q.v[e] = __uint_as_float(p0 + e < sr.nv ? (b << 31) | v.w : 0u);
        } else {
            q.v[e] = p0 + e < sr.nv ? __hiloint2double((int)((b << 31) | v.w), (int)v.z) : 0.0;
        }
    }
    return q;
}

// What a gather loads: the lane's quad of the FP32 row, or (SG) the slot of
// the first step's sign record, expanded only where the values are summed
// (so the loads of a round stay in flight together).
template <bool SG, typename V>
using Fetched = typename std::conditional<SG, Slot, Quad<V>>::type;

template <bool SG, typename V>
__device__ __forceinline__ Fetched<SG, V> fetch(const Quad<V>* __restrict__ Rl, int32_t packed, int ms,
                                                const SignRows& sr, int quad) {
    if constexpr (SG) return sign_load<V>(sr, packed, quad);
    else return gather(Rl, packed, ms);
}

template <bool SG, typename V>
__device__ __forceinline__ Fetched<SG, V> fzero() {
    if constexpr (SG) return Slot{0u, 0u, 0u, 0u};
    else return qzero<V>();
}

template <bool SG, typename V>
__device__ __forceinline__ Quad<V> expand(const Fetched<SG, V>& f, const SignRows& sr, int quad) {
    if constexpr (SG) return sign_expand<V>(f, sr, quad);
    else return f;
}

// The column ranges' first labels (device, from the build) and the hot
// window (rows per range whose gathers stay cached); a window of at least n
// rows caches every gather.
struct CacheWindow {
    const int64_t* bounds;
    int64_t hot;
};

// the range starts in registers, for kernels whose gathers span all ranges
struct HotRanges {
    int64_t lo[kColRanges];
    int64_t hot;
    __device__ __forceinline__ explicit HotRanges(const CacheWindow& cw) : hot(cw.hot) {
#pragma unroll
        for (int x = 0; x < kColRanges; ++x) lo[x] = cw.bounds[x];
    }
    // label offset of column c within its range is below the window
    __device__ __forceinline__ bool hot_col(int64_t c) const {
        int64_t l = lo[0];
#pragma unroll
        for (int x = 1; x < kColRanges; ++x) l = c >= lo[x] ? lo[x] : l;
        return c - l < hot;
    }
};

template <typename V>
__device__ __forceinline__ Quad<V> qshfl(const Quad<V>& a, int src) {
    Quad<V> r;
#pragma unroll
    for (int e = 0; e < Quad<V>::E; ++e) r.v[e] = __shfl(a.v[e], src);
    return r;
}

// Fixed-order reduction of per-lane FP64 sums (E probes per lane) over the
// groups of each wave and the 4 waves of the block; writes one partial per
// probe of this block's tile: part[p * nb + block].
template <int E>
__device__ __forceinline__ void block_reduce_store(const double (&s)[E], double* __restrict__ part, int nb, int F,
                                                   int G, int K, int ld, int tile, int TQ, int col0 = 0) {
    __shared__ double red[4][64][E];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int c = 0; c < E; ++c) red[wave][lane][c] = s[c];
    __syncthreads();
    const int t = threadIdx.x;
    if (t < E * G) {
        const int q = t / E, comp = t % E;
        const int p = tile * (E * TQ) + t;
        if (tile * TQ + q < F && p < ld) {
            double a = 0.0;
            for (int wv = 0; wv < 4; ++wv)
                for (int g = 0; g < K; ++g) a += red[wv][g * G + q][comp];
            part[(int64_t)p * nb + col0 + blockIdx.x] = a;
        }
    }
}

// ------------------------------------------------------------- init -------
template <typename V>
__global__ void __launch_bounds__(256) state_init(int nv, int m, int ld, double sigma1,
                                                  double* __restrict__ alpha, double* __restrict__ beta,
                                                  int32_t* __restrict__ steps, ProbeState* __restrict__ ps,
                                                  V* __restrict__ coef, GraphStats* __restrict__ st) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int stride = gridDim.x * blockDim.x;
    if (t == 0) st->status = 0u;  // this run's findings only
    for (int k = t; k < nv * m; k += stride) {
        alpha[k] = 0.0;
        beta[k] = 0.0;
    }
    for (int p = t; p < ld; p += stride) {
        const bool on = p < nv;
        if (on) steps[p] = m;
        ps[p].sigma = on ? sigma1 : 0.0;
        ps[p].tau = 0.0;
        ps[p].rho = 1.0;
        ps[p].rho_prev = 0.0;
        ps[p].a = 0.0;
        ps[p].active = on ? 1 : 0;
        coef[p] = on ? (V)sigma1 : V(0);  // sigma_j
        coef[ld + p] = V(0);               // tau_{j-1}
        coef[2 * ld + p] = V(0);           // a_j
    }
}

// R_1[i][p] = +-1 (bit (p mod 64) of splitmix64(seed, 64 id + p div 64), id
// the caller's id of internal row i) on rows with data, stored as X_1 = dinv_i
// R_1 for the normalized Laplacian; padding probes are 0.
// One quad per thread, rows strided.
template <typename V>
__global__ void __launch_bounds__(256) probe_init(const GraphStats* __restrict__ st, int laplacian, int nv, int F,
                                                  VecMap vm, int rows_per_sweep, uint64_t seed,
                                                  const V* __restrict__ diag,
                                                  const int32_t* __restrict__ perm, Quad<V>* __restrict__ R,
                                                  uint32_t* __restrict__ rec, int rd) {
    constexpr int E = Quad<V>::E;
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int quad = tid % F;
    const int64_t row0 = tid / F;
    if (row0 >= rows_per_sweep) return;
    int64_t mo;
    int ms;
    vm.lane(quad, mo, ms);
    const int64_t n = st->n_rows;
    const int p0 = E * quad;
    const uint64_t word = (uint64_t)(p0 >> 6);
    const int bit0 = p0 & 63;
    for (int64_t i = row0; i < n; i += rows_per_sweep) {
        const uint64_t id = perm ? (uint64_t)perm[i] : (uint64_t)i;
        const uint64_t z = splitmix64(seed, 64ull * id + word);
        if (rec && (p0 & 31) == 0) {  // sign record of row i (every row: every gather reads written slots)
            constexpr int HW = 4 - (int)(sizeof(V) / 4);
            const int wi = p0 >> 5, h = wi / HW, pos = wi - h * HW;
            uint32_t* slot = rec + i * rd + 4 * h;
            slot[pos] = (uint32_t)(z >> bit0);
            if (pos == 0)
                *(V*)(slot + HW) = diag[i] == V(0) ? V(0) : (laplacian == SLAQ_LAP_NORMALIZED ? diag[i] : V(1));
        }
        if (diag[i] == V(0)) continue;
        const V one = laplacian == SLAQ_LAP_NORMALIZED ? diag[i] : V(1);  // X_1 = D^-1/2 v
        Quad<V> v;
#pragma unroll
        for (int c = 0; c < E; ++c) {
            const V sgn = ((z >> (bit0 + c)) & 1ull) ? -one : one;
            v.v[c] = (p0 + c < nv) ? sgn : V(0);
        }
        R[mo + i * ms] = v;
    }
}

// ------------------------------------------------------------- SpMM -------
// Gather-accumulate over nonzeros [k0, k1) of one row by the group of this
// lane: the group loads up to G column indices (and their scale) at once and
// broadcasts them with lane shuffles; gathers are issued four at a time.
template <int MODE, bool WEIGHTED, typename V, bool SG = false>
__device__ __forceinline__ void group_segment(Quad<V>& acc, int64_t k0, int64_t k1, int gbase, int gl, int G,
                                              const int32_t* __restrict__ col, const float* __restrict__ w,
                                              const V* __restrict__ diag, const Quad<V>* __restrict__ Rl,
                                              int ms, bool lane_ok, const HotRanges& hr,
                                              const SignRows& sr = SignRows{}, int quad = 0) {
    for (int64_t kb = k0; kb < k1; kb += G) {
        const int cnt = (int)((k1 - kb) < G ? (k1 - kb) : G);
        int32_t cl = 0;
        V sl = V(0);
        if (gl < cnt) {
            const int32_t c = __builtin_nontemporal_load(col + kb + gl);
            cl = pack_col(c, hr.hot_col(c));
            sl = WEIGHTED ? (V)w[kb + gl] : V(1);
        }
        int u = 0;
        for (; u + 4 <= cnt; u += 4) {
            int32_t c[4];
            V s[4];
            Fetched<SG, V> x[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                c[v] = __shfl(cl, gbase + u + v);
                s[v] = __shfl(sl, gbase + u + v);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) x[v] = lane_ok ? fetch<SG, V>(Rl, c[v], ms, sr, quad) : fzero<SG, V>();
#pragma unroll
            for (int v = 0; v < 4; ++v) qfma(s[v], expand<SG, V>(x[v], sr, quad), acc);
        }
        for (; u < cnt; ++u) {
            const int32_t c = __shfl(cl, gbase + u);
            const V s = __shfl(sl, gbase + u);
            if (lane_ok) qfma(s, expand<SG, V>(fetch<SG, V>(Rl, c, ms, sr, quad), sr, quad), acc);
        }
    }
}

// One wave per piece: P[p] = sum over the piece's nonzeros of scale * R_j[col].
// Pieces of column range x (x-major list) are taken by workgroups with
// blockIdx.x % 8 == x, which the dispatcher places on one XCD; each wave walks
// a contiguous run of its range's pieces so the owning heavy row advances
// incrementally.
template <int MODE, bool WEIGHTED, typename V, bool SG>
__global__ void __launch_bounds__(256) spmm_pieces(const GraphStats* __restrict__ st,
                                                   const int64_t* __restrict__ segk,
                                                   const int64_t* __restrict__ segoff, int64_t cap,
                                                   const int32_t* __restrict__ col,
                                                   const float* __restrict__ w,
                                                   const V* __restrict__ diag,
                                                   const Quad<V>* __restrict__ R,
                                                   Quad<V>* __restrict__ P, int F, VecMap vm, int G, int K, int piece,
                                                   int tile0, int TQ, CacheWindow cw, SignRows sr) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int gi = lane / G, gl = lane % G;
    const int tile = tile0 + (int)blockIdx.y;
    const int quad = tile * TQ + gl;
    const bool in_group = gi < K;
    const bool lane_ok = in_group && quad < F;
    const int64_t nh = st->n_heavy;
    if (nh == 0) return;
    int64_t mo;
    int ms;
    vm.lane(quad, mo, ms);
    const Quad<V>* __restrict__ Rl = R + mo;
    const int x = blockIdx.x % kColRanges;
    const int64_t rlo = cw.bounds[x];
    const int64_t waves_x = (int64_t)(gridDim.x / kColRanges) * 4;
    const int64_t wi = (int64_t)(blockIdx.x / kColRanges) * 4 + wave;
    const int64_t* so = segoff + (int64_t)x * cap;
    const int64_t p_lo = so[0], p_hi = so[cap];
    const int64_t per = (p_hi - p_lo + waves_x - 1) / waves_x;
    const int64_t pa = p_lo + wi * per;
    const int64_t pb = pa + per < p_hi ? pa + per : p_hi;
    if (pa >= pb) return;
    int64_t h;
    {  // largest h < nh with so[h] <= pa
        int64_t lo = 0, hi = nh - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (so[mid] <= pa) lo = mid; else hi = mid - 1;
        }
        h = lo;
    }
    for (int64_t p = pa; p < pb; ++p) {
        while (so[h + 1] <= p) ++h;
        const int64_t kstart = segk[(int64_t)x * cap + h];
        const int64_t kend = segk[(int64_t)(x + 1) * cap + h];
        const int64_t k0 = kstart + (p - so[h]) * piece;
        const int64_t k1 = k0 + piece < kend ? k0 + piece : kend;
        Quad<V> acc = qzero<V>();
        // the wave loads 64 column indices at a time; group gi takes u = gi, gi+K, ...
        for (int64_t kb = k0; kb < k1; kb += 64) {
            const int cnt = (int)((k1 - kb) < 64 ? (k1 - kb) : 64);
            int32_t cl = 0;
            V sl = V(0);
            if (lane < cnt) {
                const int32_t c = __builtin_nontemporal_load(col + kb + lane);
                cl = pack_col(c, (int64_t)c - rlo < cw.hot);
                sl = WEIGHTED ? (V)w[kb + lane] : V(1);
            }
            const int rounds = (cnt + K - 1) / K;
            int r = 0;
            for (; r + kPieceUnroll <= rounds; r += kPieceUnroll) {
                int32_t c[kPieceUnroll];
                V s[kPieceUnroll];
                Fetched<SG, V> xv[kPieceUnroll];
#pragma unroll
                for (int v = 0; v < kPieceUnroll; ++v) {
                    const int u = (r + v) * K + gi;
                    const int src = u < 64 ? u : 63;
                    c[v] = __shfl(cl, src);
                    s[v] = __shfl(sl, src);
                    if (!(in_group && u < cnt)) s[v] = V(0);
                }
#pragma unroll
                for (int v = 0; v < kPieceUnroll; ++v)
                    xv[v] = (lane_ok && s[v] != V(0)) ? fetch<SG, V>(Rl, c[v], ms, sr, quad) : fzero<SG, V>();
#pragma unroll
                for (int v = 0; v < kPieceUnroll; ++v) qfma(s[v], expand<SG, V>(xv[v], sr, quad), acc);
            }
            for (; r < rounds; ++r) {
                const int u = r * K + gi;
                const int src = u < 64 ? u : 63;
                const int32_t c = __shfl(cl, src);
                const V s = __shfl(sl, src);
                if (lane_ok && u < cnt) qfma(s, expand<SG, V>(fetch<SG, V>(Rl, c, ms, sr, quad), sr, quad), acc);
            }
        }
        // fixed-order tree over the K groups (lane + st*G)
        for (int sd = 1; sd < K; sd <<= 1) {
            const int src = lane + sd * G < 64 ? lane + sd * G : lane;
            const Quad<V> o = qshfl(acc, src);
            if (in_group && (gi % (2 * sd)) == 0 && gi + sd < K) qadd(acc, o);
        }
        if (gi == 0 && quad < F) P[p * F + quad] = acc;
    }
}

// Row epilogue shared by the row and heavy-row kernels: with acc = (A X_j)_i
// (normalized, scaled basis) or (A R_j)_i (D - A) it stores
//   normalized: D^-1/2 w_i = sigma (X_i - dinv_i^2 acc) - tau X_{j-1,i}
//   D - A:      w_i       = sigma (D_ii R_i - acc)     - tau R_{j-1,i}
// and accumulates R_j[i] * w_i in FP64 (normalized: X_i (D^-1/2 w)_i / dinv_i^2).
template <int MODE, typename V>
__device__ __forceinline__ void row_epilogue(int64_t i, const Quad<V>& acc, const V* __restrict__ diag,
                                             const Quad<V>* __restrict__ R, const Quad<V>* __restrict__ Rp,
                                             Quad<V>* __restrict__ W, const Quad<V>& sg, const Quad<V>& tp,
                                             int has_prev, int64_t mo, int ms, double (&s1)[Quad<V>::E]) {
    constexpr int E = Quad<V>::E;
    const int64_t at = mo + i * ms;
    const Quad<V> ri = R[at];
    const V di = diag[i];
    const double dd = (double)di, d2 = dd * dd;
    // per-row arithmetic in FP64, one rounding to the storage precision (the
    // scale dinv_i^2 stays exact, so the scaled operator stays symmetric)
    Quad<V> rq = qzero<V>();
    if (has_prev) rq = Rp[at];
    Quad<V> wi;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const double x = (double)ri.v[e], a = (double)acc.v[e];
        const double lr = MODE == SLAQ_LAP_NORMALIZED ? fma(-d2, a, x) : fma(dd, x, -a);
        double wv = (double)sg.v[e] * lr;
        if (has_prev) wv = fma(-(double)tp.v[e], (double)rq.v[e], wv);
        wi.v[e] = (V)wv;
    }
    W[at] = wi;
    // FP32: products of two floats are exact in double
    if (MODE == SLAQ_LAP_NORMALIZED) {
        const double wgt = di != V(0) ? 1.0 / d2 : 0.0;  // zero weight sum: no data
#pragma unroll
        for (int e = 0; e < E; ++e) s1[e] = fma((double)ri.v[e] * (double)wi.v[e], wgt, s1[e]);
    } else {
#pragma unroll
        for (int e = 0; e < E; ++e) s1[e] = fma((double)ri.v[e], (double)wi.v[e], s1[e]);
    }
}

// Heavy rows: one wave per row sums the row's pieces (all column ranges, the
// K groups taking every K-th piece, then a fixed-order tree), then the row
// epilogue.  Dot partials go to columns col0 + block of `part`.
template <int MODE, typename V>
__global__ void __launch_bounds__(256) spmm_heavy(const GraphStats* __restrict__ st,
                                                  const int32_t* __restrict__ hrow,
                                                  const int64_t* __restrict__ segoff, int64_t cap,
                                                  const Quad<V>* __restrict__ P, const V* __restrict__ diag,
                                                  const Quad<V>* __restrict__ R, const Quad<V>* __restrict__ Rp,
                                                  Quad<V>* __restrict__ W, const V* __restrict__ coef,
                                                  int has_prev, double* __restrict__ part, int nb, int col0, int F,
                                                  VecMap vm, int G, int K, int ld, int tile0, int TQ) {
    constexpr int E = Quad<V>::E;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int gi = lane / G, gl = lane % G;
    const int tile = tile0 + (int)blockIdx.y;
    const int quad = tile * TQ + gl;
    const bool in_group = gi < K;
    const bool lane_ok = in_group && quad < F;
    const int64_t nh = st->n_heavy;
    int64_t mo;
    int ms;
    vm.lane(quad, mo, ms);
    double s1[E];
#pragma unroll
    for (int e = 0; e < E; ++e) s1[e] = 0.0;
    Quad<V> sg = qzero<V>(), tp = qzero<V>();
    if (lane_ok) {
        sg = qload(coef, quad);
        if (has_prev) tp = qload(coef + ld, quad);
    }
    for (int64_t h = (int64_t)blockIdx.x * 4 + wave; h < nh; h += (int64_t)gridDim.x * 4) {
        Quad<V> acc = qzero<V>();
        int64_t idx = 0;  // position in the row's piece list (ranges in order)
        for (int x = 0; x < kColRanges; ++x) {
            const int64_t p0 = segoff[(int64_t)x * cap + h], p1 = segoff[(int64_t)x * cap + h + 1];
            // first piece of this range owned by group gi
            int64_t p = p0 + ((gi - idx) % K + K) % K;
            for (; p + 3 * K < p1; p += 4 * K) {
                Quad<V> xv[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) xv[v] = lane_ok ? qload_nt(&P[(p + v * K) * F + quad]) : qzero<V>();
#pragma unroll
                for (int v = 0; v < 4; ++v) qadd(acc, xv[v]);
            }
            for (; p < p1; p += K)
                if (lane_ok) qadd(acc, qload_nt(&P[p * F + quad]));
            idx += p1 - p0;
        }
        for (int sd = 1; sd < K; sd <<= 1) {
            const int src = lane + sd * G < 64 ? lane + sd * G : lane;
            const Quad<V> o = qshfl(acc, src);
            if (in_group && (gi % (2 * sd)) == 0 && gi + sd < K) qadd(acc, o);
        }
        if (gi == 0 && lane_ok)
            row_epilogue<MODE, V>((int64_t)hrow[h], acc, diag, R, Rp, W, sg, tp, has_prev, mo, ms, s1);
    }
    block_reduce_store<E>(s1, part, nb, F, G, K, ld, tile, TQ, col0);
}

// Every light row with data: w = sigma (L R_j)_i - tau R_{j-1}[i]; partial
// R_j.w.  A wave takes windows of rw rows (row offsets loaded by its lanes at
// once); group gi handles rows gi, gi+K, ... of the window.
template <int MODE, bool WEIGHTED, typename V, bool SG>
__global__ void __launch_bounds__(256) spmm_rows(const GraphStats* __restrict__ st, const int64_t* __restrict__ rp,
                                                 const int32_t* __restrict__ col,
                                                 const float* __restrict__ w,
                                                 const V* __restrict__ diag,
                                                 int heavy_min,
                                                 const Quad<V>* __restrict__ R,
                                                 const Quad<V>* __restrict__ Rp,
                                                 Quad<V>* __restrict__ W, const V* __restrict__ coef,
                                                 int has_prev, double* __restrict__ part, int nb, int F, VecMap vm,
                                                 int G, int K, int ld, int rw, int tile0, int TQ, CacheWindow cw,
                                                 SignRows sr) {
    constexpr int E = Quad<V>::E;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int gi = lane / G, gl = lane % G;
    const int gbase = gi * G;
    const HotRanges hr(cw);
    const int tile = tile0 + (int)blockIdx.y;
    const int quad = tile * TQ + gl;
    const bool in_group = gi < K;
    const bool lane_ok = in_group && quad < F;
    int64_t mo;
    int ms;
    vm.lane(quad, mo, ms);

    double s1[E];
#pragma unroll
    for (int e = 0; e < E; ++e) s1[e] = 0.0;
    Quad<V> sg = qzero<V>(), tp = qzero<V>();
    if (lane_ok) {
        sg = qload(coef, quad);
        if (has_prev) tp = qload(coef + ld, quad);
    }
    const int64_t n = st->n_rows;
    const int rounds = (rw + K - 1) / K;
    const int64_t nwin = (n + rw - 1) / rw;
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    for (int64_t win = (int64_t)blockIdx.x * 4 + wave; win < nwin; win += nwaves) {
        const int64_t r0 = win * rw;
        const int64_t ia = r0 + lane < n ? r0 + lane : n;
        const int64_t ib = r0 + lane + 1 < n ? r0 + lane + 1 : n;
        const int64_t rs_l = rp[ia], re_l = rp[ib];
        for (int rr = 0; rr < rounds; ++rr) {
            const int t = rr * K + gi;
            const int src = t < 64 ? t : 63;
            const int64_t s = __shfl(rs_l, src), e = __shfl(re_l, src);
            const int64_t i = r0 + t;
            if (!in_group || t >= rw || i >= n || e == s) continue;  // isolated: nothing stored
            if (e - s >= heavy_min) continue;  // heavy rows: spmm_heavy
            Quad<V> acc = qzero<V>();
            group_segment<MODE, WEIGHTED, V, SG>(acc, s, e, gbase, gl, G, col, w, diag, R + mo, ms, lane_ok, hr, sr,
                                                 quad);
            if (!lane_ok) continue;
            row_epilogue<MODE, V>(i, acc, diag, R, Rp, W, sg, tp, has_prev, mo, ms, s1);
        }
    }
    block_reduce_store<E>(s1, part, nb, F, G, K, ld, tile, TQ);
}

// R_{j+1} = w - a_j R_j on rows with data (stored when `store`; in the scaled
// basis for the normalized Laplacian), partial sums of ||R_{j+1}||^2.  Lane
// groups as in spmm_rows (a row's quads on one group), windows of 64 rows.
template <typename V>
__global__ void __launch_bounds__(256) update(const GraphStats* __restrict__ st, int laplacian,
                                              const V* __restrict__ diag,
                                              const Quad<V>* __restrict__ W, const Quad<V>* __restrict__ R,
                                              const V* __restrict__ coef, int store,
                                              Quad<V>* __restrict__ Rn, double* __restrict__ part, int nb,
                                              int F, VecMap vm, int G, int K, int ld, int tile0, int TQ) {
    constexpr int E = Quad<V>::E;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int gi = lane / G, gl = lane % G;
    const int tile = tile0 + (int)blockIdx.y;
    const int quad = tile * TQ + gl;
    const bool in_group = gi < K;
    const bool lane_ok = in_group && quad < F;
    int64_t mo;
    int ms;
    vm.lane(quad, mo, ms);
    double s2[E];
#pragma unroll
    for (int e = 0; e < E; ++e) s2[e] = 0.0;
    Quad<V> a = qzero<V>();
    if (lane_ok) a = qload(coef + 2 * ld, quad);
    // a streaming pass: windows of 64 rows (one D^-1/2 load per lane, shared
    // by lane shuffles), group gi taking rows gi, gi + K, ... of the window,
    // kUpdateRows of them with their loads in flight together
    const int64_t n = st->n_rows;
    const int per = (64 + K - 1) / K;  // rows of a window per group (the last round partly)
    const int64_t nwin = (n + 63) / 64;
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    for (int64_t win = (int64_t)blockIdx.x * 4 + wave; win < nwin; win += nwaves) {
        const int64_t r0 = win * 64;
        const V d_l = r0 + lane < n ? diag[r0 + lane] : V(0);
        for (int rr = 0; rr < per; rr += kUpdateRows) {
            bool ok[kUpdateRows];
            V d[kUpdateRows];
            int64_t at[kUpdateRows];
            Quad<V> wv[kUpdateRows], rv[kUpdateRows];
#pragma unroll
            for (int u = 0; u < kUpdateRows; ++u) {
                const int t = (rr + u) * K + gi;
                d[u] = __shfl(d_l, t < 64 ? t : 63);
                const int64_t i = r0 + t;
                ok[u] = lane_ok && t < 64 && i < n && d[u] != V(0);
                at[u] = mo + i * ms;
            }
#pragma unroll
            for (int u = 0; u < kUpdateRows; ++u) {
                wv[u] = ok[u] ? W[at[u]] : qzero<V>();
                rv[u] = ok[u] ? R[at[u]] : qzero<V>();
            }
#pragma unroll
            for (int u = 0; u < kUpdateRows; ++u) {
                if (!ok[u]) continue;
                Quad<V> r;
#pragma unroll
                for (int e = 0; e < E; ++e) r.v[e] = vfma(-a.v[e], rv[u].v[e], wv[u].v[e]);
                if (store) Rn[at[u]] = r;
                // normalized: ||R_{j+1}||^2 = sum_i X_{j+1,i}^2 / dinv_i^2
                const double wgt = laplacian == SLAQ_LAP_NORMALIZED ? 1.0 / ((double)d[u] * (double)d[u]) : 1.0;
#pragma unroll
                for (int e = 0; e < E; ++e) s2[e] = fma((double)r.v[e] * (double)r.v[e], wgt, s2[e]);
            }
        }
    }
    block_reduce_store<E>(s2, part, nb, F, G, K, ld, tile, TQ);
}

// ---------------------------------------------------------- finalize ------
__device__ __forceinline__ double sum_partials(const double* __restrict__ part, int nb, int p) {
    __shared__ double red[256];
    const int t = threadIdx.x;
    double a = 0.0;
    for (int b = t; b < nb; b += 256) a += part[(int64_t)p * nb + b];
    red[t] = a;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off) red[t] += red[t + off];
        __syncthreads();
    }
    return red[0];
}

// A non-finite coefficient sets SLAQ_STATUS_NONFINITE in the graph's status
// and in the device word.
__device__ __forceinline__ void check_finite(double x, GraphStats* st, unsigned* dstat) {
    if (!isfinite(x)) {
        atomicOr(&st->status, (unsigned)SLAQ_STATUS_NONFINITE);
        raise_status(dstat, SLAQ_STATUS_NONFINITE);
    }
}

template <typename V>
__global__ void __launch_bounds__(256) finalize_a(const double* __restrict__ part, int nb, int ld, int m, int j,
                                                  GraphStats* __restrict__ st, ProbeState* __restrict__ ps,
                                                  double* __restrict__ alpha, V* __restrict__ coef,
                                                  unsigned* dstat) {
    const int p = blockIdx.x;
    const double s1 = sum_partials(part, nb, p);
    if (threadIdx.x != 0) return;
    ProbeState s = ps[p];
    if (!s.active) {
        coef[2 * ld + p] = V(0);
        return;
    }
    // isolated rows: R_j[i] = rho_j v_i, w_i = -tau_{j-1} rho_{j-1} v_i
    const double iso = (double)st->n_isolated * s.rho * (-s.tau * s.rho_prev);
    const double al = s.sigma * (s1 + iso);
    check_finite(al, st, dstat);
    alpha[(int64_t)p * m + (j - 1)] = al;
    s.a = al * s.sigma;
    ps[p].a = s.a;
    coef[2 * ld + p] = (V)s.a;
}

template <typename V>
__global__ void __launch_bounds__(256) finalize_b(const double* __restrict__ part, int nb, int ld, int m, int j,
                                                  GraphStats* __restrict__ st, int laplacian, double eps_bd,
                                                  ProbeState* __restrict__ ps, double* __restrict__ beta,
                                                  int32_t* __restrict__ steps, V* __restrict__ coef,
                                                  unsigned* dstat) {
    const int p = blockIdx.x;
    const double s2 = sum_partials(part, nb, p);
    if (threadIdx.x != 0) return;
    ProbeState s = ps[p];
    if (!s.active) return;
    const double rho_next = -s.tau * s.rho_prev - s.a * s.rho;
    const double nrm2 = s2 + (double)st->n_isolated * rho_next * rho_next;
    const double be = sqrt(fmax(nrm2, 0.0));
    check_finite(nrm2, st, dstat);
    beta[(int64_t)p * m + (j - 1)] = be;
    const double bound = laplacian == SLAQ_LAP_NORMALIZED ? 2.0 : 2.0 * st->max_degree;
    if (j < m && !(be > eps_bd * bound)) {
        steps[p] = j;
        s.active = 0;
        s.sigma = 0.0;
        s.tau = 0.0;
        coef[p] = V(0);
        coef[ld + p] = V(0);
        coef[2 * ld + p] = V(0);
    } else {
        s.tau = be * s.sigma;
        s.sigma = 1.0 / be;
        s.rho_prev = s.rho;
        s.rho = rho_next;
        coef[p] = (V)s.sigma;
        coef[ld + p] = (V)s.tau;
    }
    ps[p] = s;
}

// ------------------------------------------------ single-launch path ------
// A graph too small to fill the chip runs the whole recurrence in one launch
// of at most one workgroup per CU instead of six launches per step: per step
//   A  heavy rows (degree >= heavy_min), one workgroup each (its 4K lane
//      groups split the row's nonzeros, fixed-order sums over groups, then
//      waves), then light rows in windows of rw rows per wave; the row
//      epilogue of spmm_rows; FP64 partials of R_j . w per workgroup
//   -- grid barrier --
//   B  every workgroup sums the partials in workgroup order and forms alpha_j
//      (the finalize_a arithmetic, the same in every workgroup, so the
//      per-probe state needs no broadcast); R_{j+1} = w - a_j R_j on its rows,
//      partials of ||R_{j+1}||^2
//   -- grid barrier --
//   C  beta_j, breakdown, sigma_{j+1}, tau_j as in finalize_b
// Workgroup 0 alone writes alpha, beta and the step counts.  The barrier is a
// device-wide arrival counter (zeroed by fused_reset before the launch) with
// release/acquire fences; its wait is bounded, so a grid whose workgroups are
// not all resident at once ends with SLAQ_STATUS_GRID set instead of hanging
// (the grid is sized to what the occupancy query says stays resident).
constexpr int kFusedMaxBlocks = 256;
constexpr int kFusedMaxQuads = 16;  // F <= 16: nv <= 64 (FP32) or 32 (FP64)
constexpr unsigned kSpinLimit = 1u << 20;

template <typename V>
struct FusedArgs {
    GraphStats* st;
    const int64_t* rp;
    const int32_t* col;
    const float* w;
    const V* diag;
    const int32_t* perm;
    const int32_t* hrow;
    int heavy_min;
    Quad<V>* R0;
    Quad<V>* R1;
    Quad<V>* R2;
    int F, G, K, ld, nv, m, rw;
    VecMap vm;
    uint64_t seed;
    double sigma1, eps_bd;
    double* alpha;
    double* beta;
    int32_t* steps;
    double* part;  // [2][ld][kFusedMaxBlocks]
    unsigned* bar;
    unsigned* dstat;
    CacheWindow cw;
};

// Barrier counters, each on a 128-byte line of its own: [0] the rounds the
// eight groups (workgroups b with b mod 8 = x, one XCD each) have completed,
// [1 + x] group x's arrivals.
constexpr int kBarStride = 32;  // unsigned words per counter line
constexpr size_t kBarBytes = (size_t)(1 + kColRanges) * kBarStride * sizeof(unsigned);

__global__ void fused_reset(unsigned* bar) {
    if (threadIdx.x <= kColRanges) bar[threadIdx.x * kBarStride] = 0u;
}

// Every workgroup has arrived `round` times; false if the wait ran out.  Two
// levels: a workgroup counts itself in its group's counter, the group's last
// arrival of the round counts the group in counter 0, and every workgroup
// waits for counter 0 to reach round x groups (256 arrivals on one address
// would serialize: ~6.6 us per barrier at 128 workgroups).
__device__ __forceinline__ bool grid_barrier(unsigned* bar, unsigned round, int* s_ok) {
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        const unsigned nb = gridDim.x;
        const unsigned x = blockIdx.x % kColRanges;
        const unsigned members = (nb - x + kColRanges - 1) / kColRanges;
        const unsigned groups = nb < (unsigned)kColRanges ? nb : (unsigned)kColRanges;
        // release: this workgroup's writes (L2 written back) before its arrival
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned old =
            __hip_atomic_fetch_add(bar + (1 + x) * kBarStride, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (old + 1 == round * members) {
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
            __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        // the wait polls with plain coherent loads; one acquire after it
        // (an acquiring poll would invalidate the L2 at every iteration)
        const unsigned target = round * groups;
        unsigned spins = 0;
        while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > kSpinLimit) {
                ok = 0;
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *s_ok = ok;
    }
    __syncthreads();
    return *s_ok != 0;
}

// Fixed-order sum over the workgroups' partials part[p][0..nb) of every
// probe p < ld into out[p] (chunks of workgroups summed by all threads, then
// the chunks in order by thread p).  Ends with a barrier.
__device__ __forceinline__ void sum_workgroup_partials(const double* __restrict__ part, int nb, int ld,
                                                       double* red, double* out) {
    const int t = threadIdx.x;
    int C = 256 / ld;
    if (C > 8) C = 8;
    if (C < 1) C = 1;
    if (t < C * ld) {
        const int p = t % ld, c = t / ld;
        double a = 0.0;
        for (int b = c; b < nb; b += C) a += __hip_atomic_load(part + (int64_t)p * kFusedMaxBlocks + b,
                                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        red[c * ld + p] = a;
    }
    __syncthreads();
    if (t < ld) {
        double a = 0.0;
        for (int c = 0; c < C; ++c) a += red[c * ld + t];
        out[t] = a;
    }
    __syncthreads();
}

template <int MODE, bool WEIGHTED, typename V>
__global__ void __launch_bounds__(256) lanczos_fused(FusedArgs<V> a) {
    constexpr int E = Quad<V>::E;
    __shared__ ProbeState sps[4 * kFusedMaxQuads];
    __shared__ V scoef[3 * 4 * kFusedMaxQuads];
    __shared__ double sred[256];
    __shared__ double ssum[4 * kFusedMaxQuads];
    __shared__ Quad<V> hacc[4][64];
    __shared__ int s_ok;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int G = a.G, K = a.K, F = a.F, ld = a.ld;
    const int gi = lane / G, gl = lane % G, gbase = gi * G;
    const bool in_group = gi < K;
    const int quad = gl;
    const bool lane_ok = in_group && quad < F;
    int64_t mo;
    int ms;
    a.vm.lane(quad, mo, ms);
    const HotRanges hr(a.cw);
    const int nb = gridDim.x;
    const bool lead = blockIdx.x == 0;
    GraphStats* st = a.st;
    const int64_t n = st->n_rows;
    const int64_t nh = st->n_heavy;
    const double n_iso = (double)st->n_isolated;
    const double bound = MODE == SLAQ_LAP_NORMALIZED ? 2.0 : 2.0 * st->max_degree;
    const V* __restrict__ diag = a.diag;
    double* part1 = a.part;
    double* part2 = a.part + (int64_t)ld * kFusedMaxBlocks;
    unsigned round = 0;

    // ---- per-probe state (every workgroup the same) and X_1 ----------------
    for (int p = threadIdx.x; p < ld; p += blockDim.x) {
        const bool on = p < a.nv;
        ProbeState z;
        z.sigma = on ? a.sigma1 : 0.0;
        z.tau = 0.0;
        z.rho = 1.0;
        z.rho_prev = 0.0;
        z.a = 0.0;
        z.active = on ? 1 : 0;
        z.pad = 0;
        sps[p] = z;
        scoef[p] = on ? (V)a.sigma1 : V(0);
        scoef[ld + p] = V(0);
        scoef[2 * ld + p] = V(0);
    }
    if (lead) {
        if (threadIdx.x == 0) st->status = 0u;
        for (int k = threadIdx.x; k < a.nv * a.m; k += blockDim.x) {
            a.alpha[k] = 0.0;
            a.beta[k] = 0.0;
        }
        for (int p = threadIdx.x; p < a.nv; p += blockDim.x) a.steps[p] = a.m;
    }
    {
        const int64_t total = n * F;
        for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total; x += (int64_t)nb * blockDim.x) {
            const int64_t i = x / F;
            const int q = (int)(x % F);
            if (diag[i] == V(0)) continue;
            int64_t o;
            int sd;
            a.vm.lane(q, o, sd);
            const uint64_t id = a.perm ? (uint64_t)a.perm[i] : (uint64_t)i;
            const int p0 = E * q;
            const uint64_t z = splitmix64(a.seed, 64ull * id + (uint64_t)(p0 >> 6));
            const V one = MODE == SLAQ_LAP_NORMALIZED ? diag[i] : V(1);
            Quad<V> v;
#pragma unroll
            for (int c = 0; c < E; ++c) {
                const V sgn = ((z >> ((p0 & 63) + c)) & 1ull) ? -one : one;
                v.v[c] = (p0 + c < a.nv) ? sgn : V(0);
            }
            a.R0[o + i * sd] = v;
        }
    }
    if (!grid_barrier(a.bar, ++round, &s_ok)) {
        if (threadIdx.x == 0) raise_status(a.dstat, SLAQ_STATUS_GRID);
        return;
    }

    Quad<V>* Rc = a.R0;
    Quad<V>* Rp = a.R1;
    Quad<V>* W = a.R2;
    const int64_t nwin = (n + a.rw - 1) / a.rw;
    const int rounds = (a.rw + K - 1) / K;
    const int64_t nwaves = (int64_t)nb * 4;
    for (int j = 1; j <= a.m; ++j) {
        const int hp = j > 1 ? 1 : 0;
        Quad<V> sg = qzero<V>(), tp = qzero<V>();
        if (lane_ok) {
            sg = qload(scoef, quad);
            if (hp) tp = qload(scoef + ld, quad);
        }
        double s1[E];
#pragma unroll
        for (int e = 0; e < E; ++e) s1[e] = 0.0;
        // -- A: heavy rows.  The longest (>= 8 nonzeros per lane group of the
        // workgroup) take a whole workgroup each: its 4K groups split the row,
        // fixed-order sums over groups, then over waves through LDS.  The
        // others take one wave each: its K groups split the row, fixed-order
        // sums over the groups by lane shuffles.
        const int64_t big = 32 * (int64_t)K;
        for (int64_t h = blockIdx.x; h < nh; h += nb) {
            const int64_t i = a.hrow[h];
            const int64_t rs = a.rp[i], re = a.rp[i + 1];
            if (re - rs < big) continue;  // workgroup-uniform
            const int64_t ng = 4 * (int64_t)K;
            const int64_t chunk = (re - rs + ng - 1) / ng;
            int64_t k0 = re, k1 = re;
            if (in_group) {
                const int64_t gg = (int64_t)wave * K + gi;
                k0 = rs + gg * chunk < re ? rs + gg * chunk : re;
                k1 = k0 + chunk < re ? k0 + chunk : re;
            }
            Quad<V> acc = qzero<V>();
            group_segment<MODE, WEIGHTED, V>(acc, k0, k1, gbase, gl, G, a.col, a.w, diag, Rc + mo, ms, lane_ok, hr);
            for (int sd = 1; sd < K; sd <<= 1) {
                const int src = lane + sd * G < 64 ? lane + sd * G : lane;
                const Quad<V> o = qshfl(acc, src);
                if (in_group && (gi % (2 * sd)) == 0 && gi + sd < K) qadd(acc, o);
            }
            if (gi == 0) hacc[wave][lane] = acc;
            __syncthreads();
            if (wave == 0 && gi == 0 && lane_ok) {
                Quad<V> r = hacc[0][lane];
                qadd(r, hacc[1][lane]);
                qadd(r, hacc[2][lane]);
                qadd(r, hacc[3][lane]);
                row_epilogue<MODE, V>(i, r, diag, Rc, Rp, W, sg, tp, hp, mo, ms, s1);
            }
            __syncthreads();
        }
        for (int64_t h = (int64_t)blockIdx.x * 4 + wave; h < nh; h += nwaves) {
            const int64_t i = a.hrow[h];
            const int64_t rs = a.rp[i], re = a.rp[i + 1];
            if (re - rs >= big) continue;  // wave-uniform
            const int64_t chunk = (re - rs + K - 1) / K;
            int64_t k0 = re, k1 = re;
            if (in_group) {
                k0 = rs + gi * chunk < re ? rs + gi * chunk : re;
                k1 = k0 + chunk < re ? k0 + chunk : re;
            }
            Quad<V> acc = qzero<V>();
            group_segment<MODE, WEIGHTED, V>(acc, k0, k1, gbase, gl, G, a.col, a.w, diag, Rc + mo, ms, lane_ok, hr);
            for (int sd = 1; sd < K; sd <<= 1) {
                const int src = lane + sd * G < 64 ? lane + sd * G : lane;
                const Quad<V> o = qshfl(acc, src);
                if (in_group && (gi % (2 * sd)) == 0 && gi + sd < K) qadd(acc, o);
            }
            if (gi == 0 && lane_ok) row_epilogue<MODE, V>(i, acc, diag, Rc, Rp, W, sg, tp, hp, mo, ms, s1);
        }
        // -- A: light rows, a lane group per row, windows of rw rows per wave
        for (int64_t win = (int64_t)blockIdx.x * 4 + wave; win < nwin; win += nwaves) {
            const int64_t r0 = win * a.rw;
            const int64_t ia = r0 + lane < n ? r0 + lane : n;
            const int64_t ib = r0 + lane + 1 < n ? r0 + lane + 1 : n;
            const int64_t rs_l = a.rp[ia], re_l = a.rp[ib];
            for (int rr = 0; rr < rounds; ++rr) {
                const int t = rr * K + gi;
                const int src = t < 64 ? t : 63;
                const int64_t rs = __shfl(rs_l, src), re = __shfl(re_l, src);
                const int64_t i = r0 + t;
                if (!in_group || t >= a.rw || i >= n || re == rs) continue;
                if (re - rs >= a.heavy_min) continue;
                Quad<V> acc = qzero<V>();
                group_segment<MODE, WEIGHTED, V>(acc, rs, re, gbase, gl, G, a.col, a.w, diag, Rc + mo, ms, lane_ok,
                                                 hr);
                if (!lane_ok) continue;
                row_epilogue<MODE, V>(i, acc, diag, Rc, Rp, W, sg, tp, hp, mo, ms, s1);
            }
        }
        block_reduce_store<E>(s1, part1, kFusedMaxBlocks, F, G, K, ld, 0, F);
        if (!grid_barrier(a.bar, ++round, &s_ok)) {
            if (threadIdx.x == 0) raise_status(a.dstat, SLAQ_STATUS_GRID);
            return;
        }
        // -- B: alpha_j (finalize_a in every workgroup)
        sum_workgroup_partials(part1, nb, ld, sred, ssum);
        if (threadIdx.x < ld) {
            const int p = threadIdx.x;
            ProbeState z = sps[p];
            if (z.active) {
                const double iso = n_iso * z.rho * (-z.tau * z.rho_prev);
                const double al = z.sigma * (ssum[p] + iso);
                if (lead) {
                    check_finite(al, st, a.dstat);
                    a.alpha[(int64_t)p * a.m + (j - 1)] = al;
                }
                z.a = al * z.sigma;
                sps[p] = z;
                scoef[2 * ld + p] = (V)z.a;
            } else {
                scoef[2 * ld + p] = V(0);
            }
        }
        __syncthreads();
        // -- B: R_{j+1} = w - a_j R_j (into R_{j-1}'s block), ||R_{j+1}||^2 partials
        Quad<V> av = qzero<V>();
        if (lane_ok) av = qload(scoef + 2 * ld, quad);
        double s2[E];
#pragma unroll
        for (int e = 0; e < E; ++e) s2[e] = 0.0;
        for (int64_t win = (int64_t)blockIdx.x * 4 + wave; win < nwin; win += nwaves) {
            const int64_t r0 = win * a.rw;
            const V d_l = r0 + lane < n ? diag[r0 + lane] : V(0);
            for (int rr = 0; rr < rounds; ++rr) {
                const int t = rr * K + gi;
                const V d = __shfl(d_l, t < 64 ? t : 63);
                const int64_t i = r0 + t;
                if (!lane_ok || t >= a.rw || i >= n || d == V(0)) continue;
                const int64_t at = mo + i * ms;
                const Quad<V> wv = W[at];
                const Quad<V> rv = Rc[at];
                Quad<V> r;
#pragma unroll
                for (int e = 0; e < E; ++e) r.v[e] = vfma(-av.v[e], rv.v[e], wv.v[e]);
                if (j < a.m) Rp[at] = r;
                const double wgt = MODE == SLAQ_LAP_NORMALIZED ? 1.0 / ((double)d * (double)d) : 1.0;
#pragma unroll
                for (int e = 0; e < E; ++e) s2[e] = fma((double)r.v[e] * (double)r.v[e], wgt, s2[e]);
            }
        }
        block_reduce_store<E>(s2, part2, kFusedMaxBlocks, F, G, K, ld, 0, F);
        if (!grid_barrier(a.bar, ++round, &s_ok)) {
            if (threadIdx.x == 0) raise_status(a.dstat, SLAQ_STATUS_GRID);
            return;
        }
        // -- C: beta_j, breakdown, next sigma and tau (finalize_b in every workgroup)
        sum_workgroup_partials(part2, nb, ld, sred, ssum);
        if (threadIdx.x < ld) {
            const int p = threadIdx.x;
            ProbeState z = sps[p];
            if (z.active) {
                const double rho_next = -z.tau * z.rho_prev - z.a * z.rho;
                const double nrm2 = ssum[p] + n_iso * rho_next * rho_next;
                const double be = sqrt(fmax(nrm2, 0.0));
                if (lead) {
                    check_finite(nrm2, st, a.dstat);
                    a.beta[(int64_t)p * a.m + (j - 1)] = be;
                }
                if (j < a.m && !(be > a.eps_bd * bound)) {
                    if (lead) a.steps[p] = j;
                    z.active = 0;
                    z.sigma = 0.0;
                    z.tau = 0.0;
                    scoef[p] = V(0);
                    scoef[ld + p] = V(0);
                    scoef[2 * ld + p] = V(0);
                } else {
                    z.tau = be * z.sigma;
                    z.sigma = 1.0 / be;
                    z.rho_prev = z.rho;
                    z.rho = rho_next;
                    scoef[p] = (V)z.sigma;
                    scoef[ld + p] = (V)z.tau;
                }
                sps[p] = z;
            }
        }
        __syncthreads();
        if (j < a.m) {
            Quad<V>* tq = Rc;
            Rc = Rp;
            Rp = tq;
        }
    }
}

// ------------------------------------------------------------ layout ------
struct Layout {
    int ld, F, G, K, ntiles, TQ, Gu, Ku, ntiles_u, nb_rows, nb_upd, piece_blocks, rw, nb_heavy;
    VecMap vm;
    int64_t max_pieces;
    size_t off_r[3], off_p, off_part1, off_part2, off_ps, off_coef, off_fused, off_bar, total;
};

constexpr int kRowBlocks = 2048;  // upper bound; the grid is sized to what stays resident
// Grid cap of the piece kernel: on R-MAT 22 (1.25M pieces) 65,536 workgroups
// give each wave ~5 consecutive pieces of its range and balance best (4,096:
// 3.84 ms, 16,384: 3.45 ms, 65,536: 3.40 ms, 262,144: 3.59 ms).
constexpr int kPieceBlocks = 65536;

// Blocks of `kernel` that fit on the current device at once (all CUs).
template <typename K>
static int resident_blocks(K kernel, int block) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return kRowBlocks;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return kRowBlocks;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) != hipSuccess || per_cu < 1)
        return kRowBlocks;
    return cus * per_cu;
}

template <typename V>
static Layout make_layout(const slaq_graph_s* g, int nv) {
    constexpr int E = Quad<V>::E;
    Layout L{};
    L.ld = lanczos_ld(nv);
    L.F = L.ld / E;
    // probe tiles of the gather kernels, run one after another (a tile's
    // gathered rows are narrower and stay in cache longer, but every nonzero
    // is visited once per tile; on R-MAT scale 22 with nv = 100 one tile is
    // fastest, so the default is one tile of up to 64 quads)
    int tq = g->tile_quads > 0 ? g->tile_quads : kQuadsPerTile;
    if (tq > kQuadsPerTile) tq = kQuadsPerTile;
    if (tq > L.F) tq = L.F;
    L.TQ = tq;
    L.G = tq;
    L.K = 64 / L.G;
    L.ntiles = (L.F + tq - 1) / tq;
    L.Gu = L.F < kQuadsPerTile ? L.F : kQuadsPerTile;
    L.Ku = 64 / L.Gu;
    L.ntiles_u = (L.F + kQuadsPerTile - 1) / kQuadsPerTile;
    // rows per wave window: up to kRowsPerWindow, fewer on small graphs so
    // that the windows still cover every resident wave (never fewer than K)
    const int64_t target_waves = 8192;
    int64_t rw = (g->n + target_waves - 1) / target_waves;
    if (rw > kRowsPerWindow) rw = kRowsPerWindow;
    if (rw < L.K) rw = L.K;
    L.rw = (int)rw;
    const int64_t nwin = (g->n + L.rw - 1) / L.rw;
    int64_t nb = (nwin + 3) / 4;
    if (nb < 1) nb = 1;
    static const int rows_cap = resident_blocks(spmm_rows<SLAQ_LAP_NORMALIZED, false, V, false>, kSpmmBlock);
    static const int upd_cap = resident_blocks(update<V>, kSpmmBlock);
    const int cap_r = rows_cap < kRowBlocks ? rows_cap : kRowBlocks;
    const int cap_u = upd_cap < kRowBlocks ? upd_cap : kRowBlocks;
    L.nb_rows = (int)(nb < cap_r ? nb : cap_r);
    L.nb_upd = (int)(nb < cap_u ? nb : cap_u);
    // pieces <= nnz/piece + one partial piece per (heavy row, column range)
    int64_t heavy_cap = g->nnz / g->heavy_min;
    if (heavy_cap > g->n) heavy_cap = g->n;
    L.max_pieces = g->nnz / g->piece + kColRanges * heavy_cap;
    int64_t pb = (L.max_pieces + 3) / 4;
    pb = pb < kPieceBlocks ? (pb > 0 ? pb : 1) : kPieceBlocks;
    L.piece_blocks = (int)((pb + kColRanges - 1) / kColRanges * kColRanges);  // a multiple of the ranges
    // split rows: main part of whole 128-byte lines, tail region after it
    L.vm.Fm = L.F / 8 * 8;
    L.vm.Ft = L.F - L.vm.Fm;
    const size_t main_bytes = align_up((size_t)g->n * L.vm.Fm * 16, 256);
    L.vm.tail = (int64_t)(main_bytes / 16);
    const size_t vec = main_bytes + align_up((size_t)g->n * L.vm.Ft * 16, 256);
    size_t off = 0;
    for (int b = 0; b < 3; ++b) {
        L.off_r[b] = off;
        off += vec;
    }
    L.off_p = off;
    off += align_up((size_t)L.max_pieces * L.ld * sizeof(V), 256);
    // heavy-row epilogue grid: one wave per heavy row, at most 1024 blocks
    {
        int64_t hb = (heavy_cap + 3) / 4;
        L.nb_heavy = (int)(hb < 1 ? 1 : (hb > 1024 ? 1024 : hb));
    }
    L.off_part1 = off;
    off += align_up((size_t)L.ld * (L.nb_rows + L.nb_heavy) * sizeof(double), 256);
    L.off_part2 = off;
    off += align_up((size_t)L.ld * L.nb_upd * sizeof(double), 256);
    L.off_ps = off;
    off += align_up((size_t)L.ld * sizeof(ProbeState), 256);
    L.off_coef = off;
    off += align_up((size_t)3 * L.ld * sizeof(V), 256);
    // single-launch path: FP64 partials [2][ld][kFusedMaxBlocks] and the
    // barrier's arrival counter
    L.off_fused = off;
    off += align_up((size_t)2 * L.ld * kFusedMaxBlocks * sizeof(double), 256);
    L.off_bar = off;
    off += align_up(kBarBytes, 256);
    L.total = off;
    return L;
}

// The hot window: rows per column range whose gathers keep their lines
// cached.  Only a relabelled graph has its hot rows at the front of each
// range; elsewhere every gather is cached.  Automatic: the window whose probe
// rows (F quads each, all ranges) fill kCacheBudget of the last-level cache.
static CacheWindow cache_window(const slaq_graph_s* g, int F) {
    CacheWindow cw{g->bounds, INT64_MAX / 2};
    if (!g->relabeled) return cw;
    cw.hot = g->cache_rows >= 0 ? g->cache_rows : (int64_t)(kCacheBudget / ((size_t)kColRanges * 16 * F));
    return cw;
}

// Workgroups of the single-launch path for this graph and probe count, or 0
// for the multi-kernel path.  Eligible: caller order (no relabelling), at most
// kFusedMaxQuads quads per row; automatic (fused = -1) below kFusedAutoNnz
// stored entries, with one workgroup per 80 rows between 8 and 128 (measured
// on Chung-Lu n = 10^4, nv = 10, m = 15: 8 / 32 / 128 / 256 workgroups take
// 3.55 / 1.11 / 0.67 / 0.77 ms; a 100-node path 0.15 ms at 8, where the stage
// kernels need ~90 launches).  At most one workgroup per CU
// and never more than stay resident at once.
constexpr int64_t kFusedAutoNnz = (int64_t)1 << 18;

template <typename V>
static int fused_blocks(const slaq_graph_s* g, const Layout& L) {
    if (g->fused == 0 || g->relabeled || L.F > kFusedMaxQuads || L.ntiles != 1) return 0;
    if (g->fused < 0 && g->nnz >= kFusedAutoNnz) return 0;
    static const int cap_res = resident_blocks(lanczos_fused<SLAQ_LAP_COMBINATORIAL, true, V>, 256);
    int cus = 0, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        return 0;
    int cap = cus < cap_res ? cus : cap_res;
    if (cap > kFusedMaxBlocks) cap = kFusedMaxBlocks;
    int64_t want = g->fused;
    if (want < 0) {
        want = (g->n + 79) / 80;
        want = want < 8 ? 8 : (want > 128 ? 128 : want);
    }
    return (int)(want < cap ? want : cap);
}

static int sweep_grid(int64_t n, int F, int* rows_per_sweep) {
    int64_t rows = n;
    const int64_t max_threads = 256LL * 8192;
    if ((int64_t)F * rows > max_threads) rows = max_threads / F;
    if (rows < 1) rows = 1;
    *rows_per_sweep = (int)rows;
    return (int)(((int64_t)F * rows + 255) / 256);
}

#define SLAQ_DISPATCH(MODE_, WEIGHTED_, KERNEL, ...)                                                  \
    do {                                                                                               \
        if ((MODE_) == SLAQ_LAP_NORMALIZED) {                                                          \
            if (WEIGHTED_) hipLaunchKernelGGL((KERNEL<SLAQ_LAP_NORMALIZED, true, V>), __VA_ARGS__);    \
            else hipLaunchKernelGGL((KERNEL<SLAQ_LAP_NORMALIZED, false, V>), __VA_ARGS__);             \
        } else {                                                                                       \
            if (WEIGHTED_) hipLaunchKernelGGL((KERNEL<SLAQ_LAP_COMBINATORIAL, true, V>), __VA_ARGS__); \
            else hipLaunchKernelGGL((KERNEL<SLAQ_LAP_COMBINATORIAL, false, V>), __VA_ARGS__);          \
        }                                                                                              \
    } while (0)

// the stage gather kernels with their first-step variant (SG_: sign records)
#define SLAQ_DISPATCH_SG(MODE_, WEIGHTED_, SG_, KERNEL, ...)                                                \
    do {                                                                                                     \
        if (SG_) {                                                                                           \
            if ((MODE_) == SLAQ_LAP_NORMALIZED) {                                                            \
                if (WEIGHTED_) hipLaunchKernelGGL((KERNEL<SLAQ_LAP_NORMALIZED, true, V, true>), __VA_ARGS__); \
                else hipLaunchKernelGGL((KERNEL<SLAQ_LAP_NORMALIZED, false, V, true>), __VA_ARGS__);          \
            } else {                                                                                         \
                if (WEIGHTED_) hipLaunchKernelGGL((KERNEL<SLAQ_LAP_COMBINATORIAL, true, V, true>), __VA_ARGS__); \
                else hipLaunchKernelGGL((KERNEL<SLAQ_LAP_COMBINATORIAL, false, V, true>), __VA_ARGS__);       \
            }                                                                                                \
        } else {                                                                                             \
            if ((MODE_) == SLAQ_LAP_NORMALIZED) {                                                            \
                if (WEIGHTED_) hipLaunchKernelGGL((KERNEL<SLAQ_LAP_NORMALIZED, true, V, false>), __VA_ARGS__); \
                else hipLaunchKernelGGL((KERNEL<SLAQ_LAP_NORMALIZED, false, V, false>), __VA_ARGS__);         \
            } else {                                                                                         \
                if (WEIGHTED_) hipLaunchKernelGGL((KERNEL<SLAQ_LAP_COMBINATORIAL, true, V, false>), __VA_ARGS__); \
                else hipLaunchKernelGGL((KERNEL<SLAQ_LAP_COMBINATORIAL, false, V, false>), __VA_ARGS__);      \
            }                                                                                                \
        }                                                                                                    \
    } while (0)

// Sign-record layout of the first step for ld probe slots: ceil(ld / 32)
// sign dwords, 4 - sizeof(V)/4 of them per 16-byte slot with the scale, a
// power of two of slots per record.
template <typename V>
static SignRows sign_layout(int ld, int nv) {
    const int words = (ld + 31) / 32, hw = 4 - (int)(sizeof(V) / 4);
    const int slots = (words + hw - 1) / hw;
    int rs = 1;
    while (rs < slots) rs *= 2;
    return SignRows{nullptr, 4 * rs, nv};
}

// diagonal scale of the internal rows in the vectors' precision
template <typename V> static const V* diag_of(const slaq_graph_s* g);
template <> const float* diag_of<float>(const slaq_graph_s* g) { return g->diag; }
template <> const double* diag_of<double>(const slaq_graph_s* g) { return g->diag64; }

template <typename V>
static slaq_status run_lanczos(slaq_graph_t g, int nv, int m, uint64_t seed, double* alpha, double* beta,
                               int32_t* steps, void* workspace, size_t workspace_bytes, hipStream_t st) {
    using Q = Quad<V>;
    const Layout L = make_layout<V>(g, nv);
    SLAQ_REQUIRE(workspace_bytes >= L.total, SLAQ_ERR_WORKSPACE, "lanczos workspace needs %zu bytes, got %zu",
                 L.total, workspace_bytes);
    char* ws = (char*)workspace;
    Q* Rb[3] = {(Q*)(ws + L.off_r[0]), (Q*)(ws + L.off_r[1]), (Q*)(ws + L.off_r[2])};
    Q* P = (Q*)(ws + L.off_p);
    double* part1 = (double*)(ws + L.off_part1);
    double* part2 = (double*)(ws + L.off_part2);
    ProbeState* ps = (ProbeState*)(ws + L.off_ps);
    V* coef = (V*)(ws + L.off_coef);
    const int mode = g->laplacian;
    const bool weighted = g->weights != nullptr;
    const V* diag = diag_of<V>(g);
    unsigned* const dstat = device_status_word();
    SLAQ_REQUIRE(dstat, SLAQ_ERR_HIP, "device status word unavailable");

    const CacheWindow cw = cache_window(g, L.F);
    const double sigma1 = 1.0 / sqrt((double)g->n);
    const int fused_nb = fused_blocks<V>(g, L);
    if (fused_nb > 0) {
        FusedArgs<V> fa{};
        fa.st = g->stats;
        fa.rp = g->row_ptr;
        fa.col = g->col_idx;
        fa.w = g->weights;
        fa.diag = diag;
        fa.perm = g->perm;
        fa.hrow = g->hrow;
        fa.heavy_min = g->heavy_min;
        fa.R0 = Rb[0];
        fa.R1 = Rb[1];
        fa.R2 = Rb[2];
        // lane groups of at least 8 lanes: a group loads 8 column indices per
        // round (its lanes beyond the row's F quads only load indices)
        fa.F = L.F;
        fa.G = L.F < 8 ? 8 : L.F;
        fa.K = 64 / fa.G;
        fa.ld = L.ld;
        fa.nv = nv;
        fa.m = m;
        fa.rw = fa.K;
        fa.vm = L.vm;
        fa.seed = seed;
        fa.sigma1 = sigma1;
        fa.eps_bd = kEpsBreakdown;
        fa.alpha = alpha;
        fa.beta = beta;
        fa.steps = steps;
        fa.part = (double*)(ws + L.off_fused);
        fa.bar = (unsigned*)(ws + L.off_bar);
        fa.dstat = dstat;
        fa.cw = cw;
        hipLaunchKernelGGL(fused_reset, dim3(1), dim3(64), 0, st, fa.bar);
        SLAQ_LAUNCHED();
        SLAQ_TIMED("lanczos_fused", st,
                   SLAQ_DISPATCH(mode, weighted, lanczos_fused, dim3(fused_nb), dim3(256), 0, st, fa));
        SLAQ_LAUNCHED();
        return SLAQ_OK;
    }
    hipLaunchKernelGGL(state_init<V>, dim3(4), dim3(256), 0, st, nv, m, L.ld, sigma1, alpha, beta, steps, ps, coef,
                       g->stats);
    SLAQ_LAUNCHED();
    // first step from sign records, kept in the third vector buffer (the
    // previous basis block, which the first step does not read; the first
    // update overwrites it after the step's gathers are done)
    SignRows sr = sign_layout<V>(L.ld, nv);
    const bool sg1 = g->sign_step != 0 && (size_t)g->n * sr.rd * 4 <= L.off_r[2] - L.off_r[1];
    if (sg1) sr.rec = (const uint32_t*)Rb[1];
    CacheWindow cw1 = cw;  // records are narrower: a wider hot window fills the same budget
    if (g->relabeled) cw1.hot = (int64_t)(kCacheBudget / ((size_t)kColRanges * 4 * sr.rd));
    int rps = 0;
    const int sgrid = sweep_grid(g->n, L.F, &rps);
    hipLaunchKernelGGL(probe_init<V>, dim3(sgrid), dim3(256), 0, st, g->stats, mode, nv, L.F, L.vm, rps, seed, diag,
                       g->perm, Rb[0], sg1 ? (uint32_t*)Rb[1] : nullptr, sr.rd);
    SLAQ_LAUNCHED();

    int cur = 0, prev = 1;
    const int wbuf = 2;
    const int64_t cap = g->max_heavy > 0 ? g->max_heavy : 1;
    const int nbp = L.nb_rows + L.nb_heavy;
    for (int j = 1; j <= m; ++j) {
        const int hp = j > 1 ? 1 : 0;
        const bool sg = sg1 && j == 1;
        for (int tile = 0; tile < L.ntiles; ++tile) {
            if (L.max_pieces > 0) {
                SLAQ_TIMED("spmm_pieces", st,
                           SLAQ_DISPATCH_SG(mode, weighted, sg, spmm_pieces, dim3(L.piece_blocks, 1), dim3(256), 0, st,
                                            g->stats, g->segk, g->segoff, cap, g->col_idx, g->weights, diag, Rb[cur],
                                            P, L.F, L.vm, L.G, L.K, g->piece, tile, L.TQ, sg ? cw1 : cw, sr));
                SLAQ_LAUNCHED();
            }
            SLAQ_TIMED("spmm_rows", st,
                       SLAQ_DISPATCH_SG(mode, weighted, sg, spmm_rows, dim3(L.nb_rows, 1), dim3(kSpmmBlock), 0, st,
                                        g->stats, g->row_ptr, g->col_idx, g->weights, diag, g->heavy_min, Rb[cur],
                                        Rb[prev], Rb[wbuf], coef, hp, part1, nbp, L.F, L.vm, L.G, L.K, L.ld, L.rw, tile,
                                        L.TQ, sg ? cw1 : cw, sr));
            SLAQ_LAUNCHED();
            {  // always launched: its blocks write their (zero) dot partials even without heavy rows
                SLAQ_TIMED("spmm_heavy", st, {
                    if (mode == SLAQ_LAP_NORMALIZED)
                        hipLaunchKernelGGL((spmm_heavy<SLAQ_LAP_NORMALIZED, V>), dim3(L.nb_heavy, 1), dim3(256), 0,
                                           st, g->stats, g->hrow, g->segoff, cap, P, diag, Rb[cur], Rb[prev],
                                           Rb[wbuf], coef, hp, part1, nbp, L.nb_rows, L.F, L.vm, L.G, L.K, L.ld, tile,
                                           L.TQ);
                    else
                        hipLaunchKernelGGL((spmm_heavy<SLAQ_LAP_COMBINATORIAL, V>), dim3(L.nb_heavy, 1), dim3(256), 0,
                                           st, g->stats, g->hrow, g->segoff, cap, P, diag, Rb[cur], Rb[prev],
                                           Rb[wbuf], coef, hp, part1, nbp, L.nb_rows, L.F, L.vm, L.G, L.K, L.ld, tile,
                                           L.TQ);
                });
                SLAQ_LAUNCHED();
            }
        }
        SLAQ_TIMED("finalize", st,
                   hipLaunchKernelGGL(finalize_a<V>, dim3(nv), dim3(256), 0, st, part1, nbp, L.ld, m, j,
                                      g->stats, ps, alpha, coef, dstat));
        SLAQ_LAUNCHED();
        SLAQ_TIMED("update", st,
                   hipLaunchKernelGGL(update<V>, dim3(L.nb_upd, L.ntiles_u), dim3(kSpmmBlock), 0, st, g->stats,
                                      mode, diag, Rb[wbuf], Rb[cur], coef, j < m ? 1 : 0, Rb[prev], part2, L.nb_upd, L.F,
                                      L.vm, L.Gu, L.Ku, L.ld, 0, kQuadsPerTile));
        SLAQ_LAUNCHED();
        SLAQ_TIMED("finalize", st,
                   hipLaunchKernelGGL(finalize_b<V>, dim3(nv), dim3(256), 0, st, part2, L.nb_upd, L.ld, m, j,
                                      g->stats, mode, kEpsBreakdown, ps, beta, steps, coef, dstat));
        SLAQ_LAUNCHED();
        if (j < m) {
            const int t = cur;
            cur = prev;
            prev = t;
        }
    }
    return SLAQ_OK;
}

// Workspace of slaq_lanczos_noalloc: a file-scope device array, one copy per
// GPU, held until the process ends.  Host code never passes the array's name
// to a kernel (on the host it is only a stand-in symbol): it takes the
// device's address from hipGetSymbolAddress once per device, with that device
// current, and uses that address everywhere.
__device__ __align__(256) unsigned char scratch[SLAQ_NOALLOC_WORKSPACE_BYTES];

static void* noalloc_workspace() {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        addr[dev] = p;
    }
    return addr[dev];
}

}  // namespace slaq

using namespace slaq;

extern "C" {

slaq_status slaq_lanczos_workspace(slaq_graph_t g, int nv, int m, size_t* bytes) {
    clear_error();
    SLAQ_REQUIRE(g && bytes, SLAQ_ERR_INVALID_ARG, "graph or bytes is NULL");
    SLAQ_REQUIRE(nv >= 1 && nv <= SLAQ_MAX_PROBES, SLAQ_ERR_INVALID_ARG, "nv must be in [1, %d]",
                 SLAQ_MAX_PROBES);
    SLAQ_REQUIRE(m >= 1 && m <= SLAQ_MAX_STEPS, SLAQ_ERR_INVALID_ARG, "m must be in [1, %d]", SLAQ_MAX_STEPS);
    *bytes = g->precision == SLAQ_PREC_FP64 ? make_layout<double>(g, nv).total : make_layout<float>(g, nv).total;
    return SLAQ_OK;
}

slaq_status slaq_lanczos(slaq_graph_t g, int nv, int m, uint64_t seed, double* alpha, double* beta,
                         int32_t* steps, void* workspace, size_t workspace_bytes, void* stream) {
    clear_error();
    SLAQ_REQUIRE(g, SLAQ_ERR_INVALID_ARG, "graph is NULL");
    SLAQ_REQUIRE(alpha && beta && steps && workspace, SLAQ_ERR_INVALID_ARG,
                 "alpha, beta, steps and workspace must be non-NULL");
    SLAQ_REQUIRE(nv >= 1 && nv <= SLAQ_MAX_PROBES, SLAQ_ERR_INVALID_ARG, "nv must be in [1, %d]",
                 SLAQ_MAX_PROBES);
    SLAQ_REQUIRE(m >= 1 && m <= SLAQ_MAX_STEPS, SLAQ_ERR_INVALID_ARG, "m must be in [1, %d]", SLAQ_MAX_STEPS);
    SLAQ_REQUIRE(((uintptr_t)workspace & 255) == 0, SLAQ_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    if (g->precision == SLAQ_PREC_FP64)
        return run_lanczos<double>(g, nv, m, seed, alpha, beta, steps, workspace, workspace_bytes, st);
    return run_lanczos<float>(g, nv, m, seed, alpha, beta, steps, workspace, workspace_bytes, st);
}

slaq_status slaq_lanczos_noalloc(slaq_graph_t g, int nv, int m, uint64_t seed, double* alpha, double* beta,
                                 int32_t* steps, void* stream) {
    clear_error();
    SLAQ_REQUIRE(g, SLAQ_ERR_INVALID_ARG, "graph is NULL");
    SLAQ_REQUIRE(alpha && beta && steps, SLAQ_ERR_INVALID_ARG, "alpha, beta and steps must be non-NULL");
    SLAQ_REQUIRE(nv >= 1 && nv <= SLAQ_MAX_PROBES, SLAQ_ERR_INVALID_ARG, "nv must be in [1, %d]",
                 SLAQ_MAX_PROBES);
    SLAQ_REQUIRE(m >= 1 && m <= SLAQ_MAX_STEPS, SLAQ_ERR_INVALID_ARG, "m must be in [1, %d]", SLAQ_MAX_STEPS);
    const size_t need =
        g->precision == SLAQ_PREC_FP64 ? make_layout<double>(g, nv).total : make_layout<float>(g, nv).total;
    SLAQ_REQUIRE(need <= (size_t)SLAQ_NOALLOC_WORKSPACE_BYTES, SLAQ_ERR_WORKSPACE,
                 "this graph and probe count need %zu bytes of workspace; the library's own is %zu bytes "
                 "(use slaq_lanczos with a caller workspace)",
                 need, (size_t)SLAQ_NOALLOC_WORKSPACE_BYTES);
    void* ws = noalloc_workspace();
    SLAQ_REQUIRE(ws, SLAQ_ERR_HIP, "library workspace unavailable on the current device");
    hipStream_t st = (hipStream_t)stream;
    // every kernel writes what it later reads (state_init the per-probe state
    // and coefficients, probe_init the first block, each block its partials):
    // nothing in the workspace has to start at zero
    if (g->precision == SLAQ_PREC_FP64)
        return run_lanczos<double>(g, nv, m, seed, alpha, beta, steps, ws, SLAQ_NOALLOC_WORKSPACE_BYTES, st);
    return run_lanczos<float>(g, nv, m, seed, alpha, beta, steps, ws, SLAQ_NOALLOC_WORKSPACE_BYTES, st);
}

}  // extern "C"
