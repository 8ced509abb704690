// Block Lanczos-quadrature front end: Rademacher probes and m steps of the
// three-term recurrence on nv probes at once (paper §3.1, "s-step Lanczos";
// Algorithm 1's lanczos(L, s, nv)).
//
// Per step j the work is
//   spmm_chunks  partial A-products of aligned kChunk-nonzero chunks of heavy rows
//   spmm_rows    w = L q_j - beta_{j-1} q_{j-1} for every row (FP32), and per
//                probe the FP64 partial sums q.w, w.w, q.q of this block
//   finalize     fixed-order sum of the partials: alpha_j = q.w,
//                beta_j^2 = w.w - 2 alpha q.w + alpha^2 q.q (= ||w - alpha q||^2),
//                breakdown test, FP32 coefficients for the next kernels
//   update       q_{j+1} = (w - alpha_j q_j) / beta_j
// so each step streams the probe block a fixed number of times and the
// reductions are deterministic (no floating-point atomics).
#include <cmath>

#include "common.hpp"
#include "profile.hpp"

namespace slaq {

constexpr double kEpsBreakdown = 1e-6;

// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) output number counter+1 for `seed`.
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t counter) {
    uint64_t z = seed + (counter + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ float4 f4(float a) { return make_float4(a, a, a, a); }

__device__ __forceinline__ void fma4(float s, const float4& x, float4& acc) {
    acc.x = fmaf(s, x.x, acc.x);
    acc.y = fmaf(s, x.y, acc.y);
    acc.z = fmaf(s, x.z, acc.z);
    acc.w = fmaf(s, x.w, acc.w);
}

__device__ __forceinline__ void add4(float4& a, const float4& b) {
    a.x += b.x;
    a.y += b.y;
    a.z += b.z;
    a.w += b.w;
}

// ------------------------------------------------------------- init -------
__global__ void __launch_bounds__(256) state_init(int nv, int m, int ld, double* __restrict__ alpha,
                                                  double* __restrict__ beta, int32_t* __restrict__ steps,
                                                  int* __restrict__ active, float* __restrict__ coef) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int stride = gridDim.x * blockDim.x;
    for (int k = t; k < nv * m; k += stride) {
        alpha[k] = 0.0;
        beta[k] = 0.0;
    }
    for (int p = t; p < ld; p += stride) {
        if (p < nv) steps[p] = m;
        active[p] = p < nv ? 1 : 0;
        coef[p] = 0.0f;           // alpha
        coef[ld + p] = 0.0f;      // 1 / beta
        coef[2 * ld + p] = 0.0f;  // beta_{j-1}, zero before the first step
    }
}

// q1[i][p] = +-1/sqrt(n): bit (p mod 64) of splitmix64(seed, 64 i + p div 64).
// Thread layout: quad fixed per thread, rows strided (F divides the stride).
__global__ void __launch_bounds__(256) probe_init(int64_t n, int nv, int F, int rows_per_sweep,
                                                  uint64_t seed, float scale, float4* __restrict__ Q) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int quad = tid % F;
    const int64_t row0 = tid / F;
    if (row0 >= rows_per_sweep) return;
    const int p0 = 4 * quad;
    const uint64_t word = (uint64_t)(p0 >> 6);
    const int bit0 = p0 & 63;
    for (int64_t i = row0; i < n; i += rows_per_sweep) {
        const uint64_t z = splitmix64(seed, 64ull * (uint64_t)i + word);
        float v[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const float sgn = ((z >> (bit0 + c)) & 1ull) ? -scale : scale;
            v[c] = (p0 + c < nv) ? sgn : 0.0f;
        }
        Q[i * F + quad] = make_float4(v[0], v[1], v[2], v[3]);
    }
}

// ------------------------------------------------------------- SpMM -------
// Lane layout inside a wave: G lanes per group hold one float4 of probes each
// (quad = tile*64 + lane%G), K = 64/G groups per wave work on different
// nonzeros (chunks) or different rows (row kernel).

// acc += sum_{k in [k0,k1), step} scale_k * Q[col_k], four loads in flight.
template <int MODE, bool WEIGHTED>
__device__ __forceinline__ void row_segment(float4& acc, int64_t k0, int64_t k1, int step,
                                            const int32_t* __restrict__ col,
                                            const float* __restrict__ w,
                                            const float* __restrict__ diag,
                                            const float4* __restrict__ Q, int F, int quad) {
    int64_t k = k0;
    for (; k + 3 * (int64_t)step < k1; k += 4 * (int64_t)step) {
        int32_t c[4];
        float s[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) c[u] = col[k + u * step];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            float sc = WEIGHTED ? w[k + u * step] : 1.0f;
            if (MODE == SLAQ_LAP_NORMALIZED) sc *= diag[c[u]];
            s[u] = sc;
        }
        float4 x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] = Q[(int64_t)c[u] * F + quad];
#pragma unroll
        for (int u = 0; u < 4; ++u) fma4(s[u], x[u], acc);
    }
    for (; k < k1; k += step) {
        const int32_t c = col[k];
        float sc = WEIGHTED ? w[k] : 1.0f;
        if (MODE == SLAQ_LAP_NORMALIZED) sc *= diag[c];
        fma4(sc, Q[(int64_t)c * F + quad], acc);
    }
}

// smallest r with rp[r+1] > k (the row holding nonzero k)
__device__ __forceinline__ int64_t row_of(const int64_t* __restrict__ rp, int64_t n, int64_t k) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (rp[mid + 1] <= k) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Heavy rows (degree >= kHeavyMin): chunk c = nonzeros [c*kChunk, (c+1)*kChunk)
// lying wholly inside one heavy row gets H[c] = sum scale_k Q[col_k].
template <int MODE, bool WEIGHTED>
__global__ void __launch_bounds__(256) spmm_chunks(int64_t n, int64_t nchunks,
                                                   const int64_t* __restrict__ rp,
                                                   const int32_t* __restrict__ col,
                                                   const float* __restrict__ w,
                                                   const float* __restrict__ diag,
                                                   const float4* __restrict__ Q,
                                                   float4* __restrict__ H, int F, int G, int K) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int gi = lane / G, gl = lane % G;
    const int quad = blockIdx.y * kQuadsPerTile + gl;
    const bool lane_ok = gi < K && quad < F;
    for (int64_t c = (int64_t)blockIdx.x * 4 + wave; c < nchunks; c += (int64_t)gridDim.x * 4) {
        const int64_t k0 = c * kChunk, k1 = k0 + kChunk;
        const int64_t r = row_of(rp, n, k0);
        const int64_t s = rp[r], e = rp[r + 1];
        if (e - s < kHeavyMin || s > k0 || e < k1) continue;  // wave-uniform
        float4 acc = f4(0.0f);
        if (lane_ok)
            row_segment<MODE, WEIGHTED>(acc, k0 + gi, k1, K, col, w, diag, Q, F, quad);
        // fixed-order tree over the K groups (lane + s*G)
        for (int st = 1; st < K; st <<= 1) {
            const int src = lane + st * G < 64 ? lane + st * G : lane;
            float4 o;
            o.x = __shfl(acc.x, src);
            o.y = __shfl(acc.y, src);
            o.z = __shfl(acc.z, src);
            o.w = __shfl(acc.w, src);
            if ((gi % (2 * st)) == 0 && gi + st < K) add4(acc, o);
        }
        if (gi == 0 && quad < F) H[c * F + quad] = acc;
    }
}

// Every row: w_i = L q_j (row i) - beta_{j-1} q_{j-1}[i]; FP64 partial dots.
template <int MODE, bool WEIGHTED>
__global__ void __launch_bounds__(256) spmm_rows(int64_t n, const int64_t* __restrict__ rp,
                                                 const int32_t* __restrict__ col,
                                                 const float* __restrict__ w,
                                                 const float* __restrict__ diag,
                                                 const float4* __restrict__ Q,
                                                 const float4* __restrict__ Qp,
                                                 const float4* __restrict__ H,
                                                 float4* __restrict__ W,
                                                 const float* __restrict__ cB, int has_prev,
                                                 double* __restrict__ part, int nb, int F, int G,
                                                 int K, int ld) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int gi = lane / G, gl = lane % G;
    const int quad = blockIdx.y * kQuadsPerTile + gl;
    const bool lane_ok = gi < K && quad < F;

    double s1[4] = {0, 0, 0, 0}, s2[4] = {0, 0, 0, 0}, s3[4] = {0, 0, 0, 0};
    float4 bprev = f4(0.0f);
    if (has_prev && lane_ok) bprev = make_float4(cB[4 * quad], cB[4 * quad + 1], cB[4 * quad + 2], cB[4 * quad + 3]);

    const int64_t nwin = (n + K - 1) / K;
    if (lane_ok) {
        for (int64_t win = (int64_t)blockIdx.x * 4 + wave; win < nwin; win += (int64_t)nb * 4) {
            const int64_t i = win * K + gi;
            if (i >= n) break;
            const int64_t s = rp[i], e = rp[i + 1];
            float4 acc = f4(0.0f);
            if (e - s >= kHeavyMin) {
                const int64_t c0 = (s + kChunk - 1) / kChunk, c1 = e / kChunk;
                for (int64_t c = c0; c < c1; ++c) add4(acc, H[c * F + quad]);
                row_segment<MODE, WEIGHTED>(acc, s, c0 * kChunk, 1, col, w, diag, Q, F, quad);
                row_segment<MODE, WEIGHTED>(acc, c1 * kChunk, e, 1, col, w, diag, Q, F, quad);
            } else {
                row_segment<MODE, WEIGHTED>(acc, s, e, 1, col, w, diag, Q, F, quad);
            }
            const float4 qi = Q[i * F + quad];
            const float di = diag[i];
            float4 wi;
            if (MODE == SLAQ_LAP_NORMALIZED) {
                const float id = di > 0.0f ? 1.0f : 0.0f;
                wi.x = fmaf(-di, acc.x, id * qi.x);
                wi.y = fmaf(-di, acc.y, id * qi.y);
                wi.z = fmaf(-di, acc.z, id * qi.z);
                wi.w = fmaf(-di, acc.w, id * qi.w);
            } else {
                wi.x = fmaf(di, qi.x, -acc.x);
                wi.y = fmaf(di, qi.y, -acc.y);
                wi.z = fmaf(di, qi.z, -acc.z);
                wi.w = fmaf(di, qi.w, -acc.w);
            }
            if (has_prev) {
                const float4 qp = Qp[i * F + quad];
                wi.x = fmaf(-bprev.x, qp.x, wi.x);
                wi.y = fmaf(-bprev.y, qp.y, wi.y);
                wi.z = fmaf(-bprev.z, qp.z, wi.z);
                wi.w = fmaf(-bprev.w, qp.w, wi.w);
            }
            W[i * F + quad] = wi;
            const float qv[4] = {qi.x, qi.y, qi.z, qi.w};
            const float wv[4] = {wi.x, wi.y, wi.z, wi.w};
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                // products of two floats are exact in double
                s1[c] = fma((double)qv[c], (double)wv[c], s1[c]);
                s2[c] = fma((double)wv[c], (double)wv[c], s2[c]);
                s3[c] = fma((double)qv[c], (double)qv[c], s3[c]);
            }
        }
    }

    // block reduction in fixed order: waves, then groups
    __shared__ double red[4][64][12];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        red[wave][lane][c] = s1[c];
        red[wave][lane][4 + c] = s2[c];
        red[wave][lane][8 + c] = s3[c];
    }
    __syncthreads();
    const int t = threadIdx.x;
    if (t < 4 * G) {
        const int q = t >> 2, comp = t & 3;
        const int p = blockIdx.y * (4 * kQuadsPerTile) + t;
        if (blockIdx.y * kQuadsPerTile + q < F && p < ld) {
            double a[3] = {0.0, 0.0, 0.0};
            for (int wv = 0; wv < 4; ++wv)
                for (int g = 0; g < K; ++g)
#pragma unroll
                    for (int sidx = 0; sidx < 3; ++sidx) a[sidx] += red[wv][g * G + q][4 * sidx + comp];
#pragma unroll
            for (int sidx = 0; sidx < 3; ++sidx) part[((int64_t)sidx * ld + p) * nb + blockIdx.x] = a[sidx];
        }
    }
}

// ---------------------------------------------------------- finalize ------
__global__ void __launch_bounds__(256) finalize(const double* __restrict__ part, int nb, int ld, int m,
                                                int j, const GraphStats* __restrict__ st, int laplacian,
                                                double eps_bd, double* __restrict__ alpha,
                                                double* __restrict__ beta, int32_t* __restrict__ steps,
                                                int* __restrict__ active, float* __restrict__ coef) {
    const int p = blockIdx.x, t = threadIdx.x;
    double a[3] = {0.0, 0.0, 0.0};
    for (int b = t; b < nb; b += 256)
#pragma unroll
        for (int s = 0; s < 3; ++s) a[s] += part[((int64_t)s * ld + p) * nb + b];
    __shared__ double red[3][256];
#pragma unroll
    for (int s = 0; s < 3; ++s) red[s][t] = a[s];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off)
#pragma unroll
            for (int s = 0; s < 3; ++s) red[s][t] += red[s][t + off];
        __syncthreads();
    }
    if (t != 0) return;
    if (!active[p]) {
        coef[p] = 0.0f;
        coef[ld + p] = 0.0f;
        coef[2 * ld + p] = 0.0f;
        return;
    }
    const double qw = red[0][0], ww = red[1][0], qq = red[2][0];
    const double al = qw;
    const double b2 = ww - 2.0 * al * qw + al * al * qq;
    const double be = sqrt(fmax(b2, 0.0));
    alpha[(int64_t)p * m + (j - 1)] = al;
    beta[(int64_t)p * m + (j - 1)] = be;
    const double bound = laplacian == SLAQ_LAP_NORMALIZED ? 2.0 : 2.0 * st->max_degree;
    if (j < m && !(be > eps_bd * bound)) {
        steps[p] = j;
        active[p] = 0;
        coef[p] = 0.0f;
        coef[ld + p] = 0.0f;
        coef[2 * ld + p] = 0.0f;
    } else {
        coef[p] = (float)al;
        coef[ld + p] = (float)(1.0 / be);
        coef[2 * ld + p] = (float)be;
    }
}

// q_{j+1} = (w - alpha q_j) / beta, per probe; zero for stopped probes.
__global__ void __launch_bounds__(256) update(int64_t n, int F, int rows_per_sweep,
                                              const float4* __restrict__ W,
                                              const float4* __restrict__ Q,
                                              const float* __restrict__ coef, int ld,
                                              float4* __restrict__ Qn) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int quad = tid % F;
    const int64_t row0 = tid / F;
    if (row0 >= rows_per_sweep) return;
    const float4 a = make_float4(coef[4 * quad], coef[4 * quad + 1], coef[4 * quad + 2], coef[4 * quad + 3]);
    const float4 ib = make_float4(coef[ld + 4 * quad], coef[ld + 4 * quad + 1], coef[ld + 4 * quad + 2],
                                  coef[ld + 4 * quad + 3]);
    for (int64_t i = row0; i < n; i += rows_per_sweep) {
        const float4 wv = W[i * F + quad];
        const float4 qv = Q[i * F + quad];
        float4 r;
        r.x = fmaf(-a.x, qv.x, wv.x) * ib.x;
        r.y = fmaf(-a.y, qv.y, wv.y) * ib.y;
        r.z = fmaf(-a.z, qv.z, wv.z) * ib.z;
        r.w = fmaf(-a.w, qv.w, wv.w) * ib.w;
        Qn[i * F + quad] = r;
    }
}

// ------------------------------------------------------------ layout ------
struct Layout {
    int ld, F, G, K, ntiles, nb;
    int64_t nchunks;
    size_t vec_bytes, off_q[3], off_h, off_part, off_coef, off_active, total;
};

static Layout make_layout(const slaq_graph_s* g, int nv) {
    Layout L{};
    L.ld = lanczos_ld(nv);
    L.F = L.ld / 4;
    L.G = L.F < kQuadsPerTile ? L.F : kQuadsPerTile;
    L.K = 64 / L.G;
    L.ntiles = (L.F + kQuadsPerTile - 1) / kQuadsPerTile;
    const int64_t nwin = (g->n + L.K - 1) / L.K;
    int64_t nb = (nwin + 3) / 4;
    L.nb = (int)(nb < kSpmmMaxBlocks ? (nb > 0 ? nb : 1) : kSpmmMaxBlocks);
    L.nchunks = g->nnz / kChunk;
    L.vec_bytes = align_up((size_t)g->n * L.ld * sizeof(float), 256);
    size_t off = 0;
    for (int b = 0; b < 3; ++b) {
        L.off_q[b] = off;
        off += L.vec_bytes;
    }
    L.off_h = off;
    off += align_up((size_t)L.nchunks * L.ld * sizeof(float), 256);
    L.off_part = off;
    off += align_up((size_t)3 * L.ld * L.nb * sizeof(double), 256);
    L.off_coef = off;
    off += align_up((size_t)3 * L.ld * sizeof(float), 256);
    L.off_active = off;
    off += align_up((size_t)L.ld * sizeof(int), 256);
    L.total = off;
    return L;
}

static int sweep_grid(int64_t n, int F, int* rows_per_sweep) {
    // threads = F * rows, capped; every thread keeps one quad
    int64_t rows = n;
    const int64_t max_threads = 256LL * 8192;
    if ((int64_t)F * rows > max_threads) rows = max_threads / F;
    if (rows < 1) rows = 1;
    *rows_per_sweep = (int)rows;
    return (int)(((int64_t)F * rows + 255) / 256);
}

}  // namespace slaq

using namespace slaq;

#define SLAQ_DISPATCH(MODE_, WEIGHTED_, KERNEL, ...)                                         \
    do {                                                                                      \
        if ((MODE_) == SLAQ_LAP_NORMALIZED) {                                                 \
            if (WEIGHTED_) hipLaunchKernelGGL((KERNEL<SLAQ_LAP_NORMALIZED, true>), __VA_ARGS__);   \
            else hipLaunchKernelGGL((KERNEL<SLAQ_LAP_NORMALIZED, false>), __VA_ARGS__);            \
        } else {                                                                              \
            if (WEIGHTED_) hipLaunchKernelGGL((KERNEL<SLAQ_LAP_COMBINATORIAL, true>), __VA_ARGS__); \
            else hipLaunchKernelGGL((KERNEL<SLAQ_LAP_COMBINATORIAL, false>), __VA_ARGS__);         \
        }                                                                                     \
    } while (0)

extern "C" {

slaq_status slaq_lanczos_workspace(slaq_graph_t g, int nv, int m, size_t* bytes) {
    clear_error();
    SLAQ_REQUIRE(g && bytes, SLAQ_ERR_INVALID_ARG, "graph or bytes is NULL");
    SLAQ_REQUIRE(nv >= 1 && nv <= SLAQ_MAX_PROBES, SLAQ_ERR_INVALID_ARG, "nv must be in [1, %d]",
                 SLAQ_MAX_PROBES);
    SLAQ_REQUIRE(m >= 1 && m <= SLAQ_MAX_STEPS, SLAQ_ERR_INVALID_ARG, "m must be in [1, %d]", SLAQ_MAX_STEPS);
    *bytes = make_layout(g, nv).total;
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
    const Layout L = make_layout(g, nv);
    SLAQ_REQUIRE(workspace_bytes >= L.total, SLAQ_ERR_WORKSPACE, "lanczos workspace needs %zu bytes, got %zu",
                 L.total, workspace_bytes);
    hipStream_t st = (hipStream_t)stream;
    char* ws = (char*)workspace;
    float4* Qb[3] = {(float4*)(ws + L.off_q[0]), (float4*)(ws + L.off_q[1]), (float4*)(ws + L.off_q[2])};
    float4* H = (float4*)(ws + L.off_h);
    double* part = (double*)(ws + L.off_part);
    float* coef = (float*)(ws + L.off_coef);
    int* active = (int*)(ws + L.off_active);
    const int mode = g->laplacian;
    const bool weighted = g->weights != nullptr;

    hipLaunchKernelGGL(state_init, dim3(4), dim3(256), 0, st, nv, m, L.ld, alpha, beta, steps, active, coef);
    SLAQ_LAUNCHED();
    int rps = 0;
    const int sgrid = sweep_grid(g->n, L.F, &rps);
    const float scale = (float)(1.0 / sqrt((double)g->n));
    hipLaunchKernelGGL(probe_init, dim3(sgrid), dim3(256), 0, st, g->n, nv, L.F, rps, seed, scale, Qb[0]);
    SLAQ_LAUNCHED();

    int cur = 0, prev = 1;
    const int wbuf = 2;
    const int64_t chunk_blocks64 = (L.nchunks + 3) / 4;
    const int chunk_blocks = (int)(chunk_blocks64 < 4096 ? chunk_blocks64 : 4096);
    for (int j = 1; j <= m; ++j) {
        if (L.nchunks > 0) {
            SLAQ_TIMED("spmm_chunks", st,
                       SLAQ_DISPATCH(mode, weighted, spmm_chunks, dim3(chunk_blocks, L.ntiles), dim3(256), 0, st,
                                     g->n, L.nchunks, g->row_ptr, g->col_idx, g->weights, g->diag, Qb[cur], H,
                                     L.F, L.G, L.K));
            SLAQ_LAUNCHED();
        }
        SLAQ_TIMED("spmm_rows", st,
                   SLAQ_DISPATCH(mode, weighted, spmm_rows, dim3(L.nb, L.ntiles), dim3(kSpmmBlock), 0, st, g->n,
                                 g->row_ptr, g->col_idx, g->weights, g->diag, Qb[cur], Qb[prev], H, Qb[wbuf],
                                 coef + 2 * L.ld, j > 1 ? 1 : 0, part, L.nb, L.F, L.G, L.K, L.ld));
        SLAQ_LAUNCHED();
        SLAQ_TIMED("finalize", st,
                   hipLaunchKernelGGL(finalize, dim3(nv), dim3(256), 0, st, part, L.nb, L.ld, m, j, g->stats, mode,
                                      kEpsBreakdown, alpha, beta, steps, active, coef));
        SLAQ_LAUNCHED();
        if (j < m) {
            SLAQ_TIMED("update", st,
                       hipLaunchKernelGGL(update, dim3(sgrid), dim3(256), 0, st, g->n, L.F, rps, Qb[wbuf], Qb[cur],
                                          coef, L.ld, Qb[prev]));
            SLAQ_LAUNCHED();
            const int t = cur;
            cur = prev;
            prev = t;
        }
    }
    return SLAQ_OK;
}

}  // extern "C"
