// Gauss rule per probe and the SLQ estimate (paper §3.1, eqs. "quadratic" and
// "slq"; Algorithm 1's eigh(T) and the final weighted sum), all in FP64.
#include <cmath>

#include "common.hpp"
#include "tridiag.hpp"

namespace slaq {

constexpr int kRitzWaves = 2048;  // probe counts solved one wave per probe

// The first B threads of a block each take one probe; T_p lives in LDS
// interleaved across them (stride B, 3 * B * m doubles).  With many probes
// B = blockDim.x (a lane per probe); with few, B = 1 and one wave per probe,
// since the lanes of a wave run their probes' QR sweeps in lockstep and a
// wave of divergent lanes takes about the sum of their times (10 probes at
// m = 15: 181 us as one wave).
__global__ void __launch_bounds__(64) ritz_kernel(const double* __restrict__ alpha,
                                                          const double* __restrict__ beta,
                                                          const int32_t* __restrict__ steps, int nv, int m,
                                                          int B, double* __restrict__ theta,
                                                          double* __restrict__ tau2, unsigned* dstat) {
    extern __shared__ double lds[];
    const int t = threadIdx.x;
    const int p = blockIdx.x * B + t;
    double* d = lds + t;
    double* e = lds + B * m + t;
    double* u = lds + 2 * B * m + t;
    // the block's coefficients into LDS with all threads at once (coalesced,
    // every load in flight together), then one thread per probe
    {
        const int64_t first = (int64_t)blockIdx.x * B * m;
        const int64_t count = (int64_t)(nv - blockIdx.x * B < B ? nv - blockIdx.x * B : B) * m;
        for (int64_t x = t; x < count; x += blockDim.x) {
            const int pl = (int)(x / m), i = (int)(x % m);
            lds[i * B + pl] = alpha[first + x];
            lds[B * m + i * B + pl] = beta[first + x];
        }
    }
    __syncthreads();
    if (t >= B || p >= nv) return;
    int k = steps[p];
    k = k < 0 ? 0 : (k > m ? m : k);
    bool finite = true;
    if (k > 0) e[(k - 1) * B] = 0.0;
    for (int i = 0; i < k; ++i) finite = finite && isfinite(d[i * B]) && isfinite(e[i * B]);
    if (!finite) raise_status(dstat, SLAQ_STATUS_NONFINITE);
    if (tridiag_eig_first_row(d, e, u, k, B) < 0) raise_status(dstat, SLAQ_STATUS_NO_CONVERGENCE);
    for (int i = 0; i < m; ++i) {
        const bool in = i < k;
        const double ui = in ? u[i * B] : 0.0;
        theta[(int64_t)p * m + i] = in ? d[i * B] : 0.0;
        tau2[(int64_t)p * m + i] = ui * ui;
    }
}

// Block b evaluates out[b] = n/nv sum_{p,k} tau2 f(t_b theta); threads stride
// over the nv*m pairs and reduce in a fixed tree (deterministic).
__global__ void __launch_bounds__(256) signature_kernel(const double* __restrict__ theta,
                                                        const double* __restrict__ tau2, int count,
                                                        double scale, const double* __restrict__ tgrid,
                                                        int kind, double* __restrict__ out) {
    const int b = blockIdx.x, tid = threadIdx.x;
    const double tt = tgrid[b];
    double acc = 0.0;
    for (int i = tid; i < count; i += 256) {
        const double w = tau2[i];
        const double x = theta[i];
        acc += w * (kind == SLAQ_SIG_HEAT ? exp(-tt * x) : cos(tt * x));
    }
    __shared__ double red[256];
    red[tid] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (tid < off) red[tid] += red[tid + off];
        __syncthreads();
    }
    if (tid == 0) out[b] = scale * red[0];
}

// H = -n/nv sum tau2 g(theta / tr L), g(x) = x ln x for x > 0, else 0.
__global__ void __launch_bounds__(256) vnge_kernel(const double* __restrict__ theta,
                                                   const double* __restrict__ tau2, int count, double scale,
                                                   const GraphStats* __restrict__ st, double* __restrict__ out) {
    const int tid = threadIdx.x;
    const double c = st->trace;
    double acc = 0.0;
    if (c > 0.0) {
        for (int i = tid; i < count; i += 256) {
            const double x = theta[i] / c;
            if (x > 0.0) acc += tau2[i] * (x * log(x));
        }
    }
    __shared__ double red[256];
    red[tid] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (tid < off) red[tid] += red[tid + off];
        __syncthreads();
    }
    if (tid == 0) out[0] = -scale * red[0];
}

// ---- Algorithm 1 end to end from the Lanczos coefficients ---------------
// Each block of CH threads re-solves the nv tridiagonals in chunks of CH (one
// thread per probe, T_p interleaved in LDS as in ritz_kernel; CH = 64, or 32
// for m > 32 to keep the tile under 64 KB) and accumulates its probes'
// tau2 f(theta) for its kSigPerBlock time values in registers; a fixed-order
// tree over the CH threads gives out[b].  The eigensolves are repeated by
// every block (ceil(nt / kSigPerBlock) of them): no workspace is needed.
constexpr int kSigPerBlock = 32;

template <int CH>
__device__ __forceinline__ void solve_chunk(const double* __restrict__ alpha, const double* __restrict__ beta,
                                            const int32_t* __restrict__ steps, int nv, int m, int p, double* d,
                                            double* e, double* u, int& k, unsigned* dstat) {
    k = 0;
    if (p >= nv) return;
    k = steps[p];
    k = k < 0 ? 0 : (k > m ? m : k);
    bool finite = true;
    for (int i = 0; i < k; ++i) {
        d[i * CH] = alpha[(int64_t)p * m + i];
        e[i * CH] = i + 1 < k ? beta[(int64_t)p * m + i] : 0.0;
        finite = finite && isfinite(d[i * CH]) && isfinite(e[i * CH]);
    }
    if (!finite) raise_status(dstat, SLAQ_STATUS_NONFINITE);
    if (tridiag_eig_first_row(d, e, u, k, CH) < 0) raise_status(dstat, SLAQ_STATUS_NO_CONVERGENCE);
}

template <int CH>
__device__ __forceinline__ double tree_sum(double v, double* red) {
    const int t = threadIdx.x;
    __syncthreads();
    red[t] = v;
    __syncthreads();
    for (int off = CH / 2; off > 0; off >>= 1) {
        if (t < off) red[t] += red[t + off];
        __syncthreads();
    }
    return red[0];
}

template <int CH>
__global__ void __launch_bounds__(CH) lsd_kernel(const double* __restrict__ alpha, const double* __restrict__ beta,
                                                 const int32_t* __restrict__ steps, int nv, int m, double scale,
                                                 const double* __restrict__ tgrid, int nt, int kind,
                                                 double* __restrict__ out, unsigned* dstat) {
    extern __shared__ double lds[];
    const int t = threadIdx.x;
    double* d = lds + t;
    double* e = lds + CH * m + t;
    double* u = lds + 2 * CH * m + t;
    double* red = lds + 3 * CH * m;
    const int b0 = blockIdx.x * kSigPerBlock;
    const int nb = nt - b0 < kSigPerBlock ? nt - b0 : kSigPerBlock;
    double acc[kSigPerBlock];
#pragma unroll
    for (int c = 0; c < kSigPerBlock; ++c) acc[c] = 0.0;
    for (int p0 = 0; p0 < nv; p0 += CH) {
        int k = 0;
        solve_chunk<CH>(alpha, beta, steps, nv, m, p0 + t, d, e, u, k, dstat);
#pragma unroll
        for (int c = 0; c < kSigPerBlock; ++c) {
            if (c >= nb) break;
            const double tt = tgrid[b0 + c];
            double s = 0.0;
            for (int i = 0; i < k; ++i) {
                const double w = u[i * CH] * u[i * CH];
                const double x = d[i * CH];
                s += w * (kind == SLAQ_SIG_HEAT ? exp(-tt * x) : cos(tt * x));
            }
            acc[c] += s;
        }
    }
    for (int c = 0; c < nb; ++c) {
        const double v = tree_sum<CH>(acc[c], red);
        if (t == 0) out[b0 + c] = scale * v;
    }
}

template <int CH>
__global__ void __launch_bounds__(CH) vnge_ab_kernel(const double* __restrict__ alpha, const double* __restrict__ beta,
                                                     const int32_t* __restrict__ steps, int nv, int m, double scale,
                                                     double c, double* __restrict__ out, unsigned* dstat) {
    extern __shared__ double lds[];
    const int t = threadIdx.x;
    double* d = lds + t;
    double* e = lds + CH * m + t;
    double* u = lds + 2 * CH * m + t;
    double* red = lds + 3 * CH * m;
    double acc = 0.0;
    for (int p0 = 0; p0 < nv; p0 += CH) {
        int k = 0;
        solve_chunk<CH>(alpha, beta, steps, nv, m, p0 + t, d, e, u, k, dstat);
        if (c > 0.0)
            for (int i = 0; i < k; ++i) {
                const double x = d[i * CH] / c;
                if (x > 0.0) acc += u[i * CH] * u[i * CH] * (x * log(x));
            }
    }
    const double v = tree_sum<CH>(acc, red);
    if (t == 0) out[0] = -scale * v;
}

}  // namespace slaq

using namespace slaq;

extern "C" {

slaq_status slaq_ritz(const double* alpha, const double* beta, const int32_t* steps, int nv, int m,
                      double* theta, double* tau2, void* stream) {
    clear_error();
    SLAQ_REQUIRE(alpha && beta && steps && theta && tau2, SLAQ_ERR_INVALID_ARG, "NULL pointer argument");
    SLAQ_REQUIRE(nv >= 1 && (int64_t)nv * m <= INT32_MAX, SLAQ_ERR_INVALID_ARG, "need nv >= 1 and nv * m < 2^31");
    SLAQ_REQUIRE(m >= 1 && m <= SLAQ_MAX_STEPS, SLAQ_ERR_INVALID_ARG, "m must be in [1, %d]", SLAQ_MAX_STEPS);
    unsigned* const dstat = device_status_word();
    SLAQ_REQUIRE(dstat, SLAQ_ERR_HIP, "device status word unavailable");
    // up to kRitzWaves probes: a wave each; more: a lane each, 64 (32 for
    // m > 32: the LDS tile stays at <= 48 KB) per block
    const int B = nv <= kRitzWaves ? 1 : (m <= 32 ? 64 : 32);
    const int threads = B == 1 ? 64 : B;
    const size_t lds = (size_t)3 * B * m * sizeof(double);
    hipLaunchKernelGGL(ritz_kernel, dim3((nv + B - 1) / B), dim3(threads), lds,
                       (hipStream_t)stream, alpha, beta, steps, nv, m, B, theta, tau2, dstat);
    SLAQ_LAUNCHED();
    return SLAQ_OK;
}

slaq_status slaq_signature(const double* theta, const double* tau2, int nv, int m, int64_t n,
                           const double* t, int nt, int kind, double* out, void* stream) {
    clear_error();
    SLAQ_REQUIRE(theta && tau2 && t && out, SLAQ_ERR_INVALID_ARG, "NULL pointer argument");
    SLAQ_REQUIRE(nv >= 1 && (int64_t)nv * m <= INT32_MAX, SLAQ_ERR_INVALID_ARG, "need nv >= 1 and nv * m < 2^31");
    SLAQ_REQUIRE(m >= 1 && m <= SLAQ_MAX_STEPS, SLAQ_ERR_INVALID_ARG, "m must be in [1, %d]", SLAQ_MAX_STEPS);
    SLAQ_REQUIRE(n > 0, SLAQ_ERR_INVALID_ARG, "n must be positive");
    SLAQ_REQUIRE(nt >= 1 && nt <= 65535, SLAQ_ERR_INVALID_ARG, "nt must be in [1, 65535]");
    SLAQ_REQUIRE(kind == SLAQ_SIG_HEAT || kind == SLAQ_SIG_WAVE, SLAQ_ERR_INVALID_ARG, "unknown signature kind");
    const double scale = (double)n / (double)nv;
    hipLaunchKernelGGL(signature_kernel, dim3(nt), dim3(256), 0, (hipStream_t)stream, theta, tau2, nv * m, scale,
                       t, kind, out);
    SLAQ_LAUNCHED();
    return SLAQ_OK;
}

slaq_status slaq_vnge(slaq_graph_t g, const double* theta, const double* tau2, int nv, int m, double* out,
                      void* stream) {
    clear_error();
    SLAQ_REQUIRE(g && theta && tau2 && out, SLAQ_ERR_INVALID_ARG, "NULL pointer argument");
    SLAQ_REQUIRE(nv >= 1 && nv <= SLAQ_MAX_PROBES, SLAQ_ERR_INVALID_ARG, "nv must be in [1, %d]",
                 SLAQ_MAX_PROBES);
    SLAQ_REQUIRE(m >= 1 && m <= SLAQ_MAX_STEPS, SLAQ_ERR_INVALID_ARG, "m must be in [1, %d]", SLAQ_MAX_STEPS);
    const double scale = (double)g->n / (double)nv;
    hipLaunchKernelGGL(vnge_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream, theta, tau2, nv * m, scale,
                       g->stats, out);
    SLAQ_LAUNCHED();
    return SLAQ_OK;
}

slaq_status slaq_lsd(const double* alpha, const double* beta, const int32_t* steps, int nv, int m, int64_t n,
                     const double* t, int nt, int kind, double* out, void* stream) {
    clear_error();
    SLAQ_REQUIRE(alpha && beta && steps && t && out, SLAQ_ERR_INVALID_ARG, "NULL pointer argument");
    SLAQ_REQUIRE(nv >= 1 && nv <= SLAQ_MAX_PROBES, SLAQ_ERR_INVALID_ARG, "nv must be in [1, %d]", SLAQ_MAX_PROBES);
    SLAQ_REQUIRE(m >= 1 && m <= SLAQ_MAX_STEPS, SLAQ_ERR_INVALID_ARG, "m must be in [1, %d]", SLAQ_MAX_STEPS);
    SLAQ_REQUIRE(n > 0, SLAQ_ERR_INVALID_ARG, "n must be positive");
    SLAQ_REQUIRE(nt >= 1 && nt <= 65535, SLAQ_ERR_INVALID_ARG, "nt must be in [1, 65535]");
    SLAQ_REQUIRE(kind == SLAQ_SIG_HEAT || kind == SLAQ_SIG_WAVE, SLAQ_ERR_INVALID_ARG, "unknown signature kind");
    unsigned* const dstat = device_status_word();
    SLAQ_REQUIRE(dstat, SLAQ_ERR_HIP, "device status word unavailable");
    const int blocks = (nt + kSigPerBlock - 1) / kSigPerBlock;
    const double scale = (double)n / (double)nv;
    if (m <= 32)
        hipLaunchKernelGGL(lsd_kernel<64>, dim3(blocks), dim3(64), (size_t)(3 * 64 * m + 64) * sizeof(double),
                           (hipStream_t)stream, alpha, beta, steps, nv, m, scale, t, nt, kind, out, dstat);
    else
        hipLaunchKernelGGL(lsd_kernel<32>, dim3(blocks), dim3(32), (size_t)(3 * 32 * m + 32) * sizeof(double),
                           (hipStream_t)stream, alpha, beta, steps, nv, m, scale, t, nt, kind, out, dstat);
    SLAQ_LAUNCHED();
    return SLAQ_OK;
}

slaq_status slaq_vnge_slq(const double* alpha, const double* beta, const int32_t* steps, int nv, int m, int64_t n,
                          double trace, double* out, void* stream) {
    clear_error();
    SLAQ_REQUIRE(alpha && beta && steps && out, SLAQ_ERR_INVALID_ARG, "NULL pointer argument");
    SLAQ_REQUIRE(nv >= 1 && nv <= SLAQ_MAX_PROBES, SLAQ_ERR_INVALID_ARG, "nv must be in [1, %d]", SLAQ_MAX_PROBES);
    SLAQ_REQUIRE(m >= 1 && m <= SLAQ_MAX_STEPS, SLAQ_ERR_INVALID_ARG, "m must be in [1, %d]", SLAQ_MAX_STEPS);
    SLAQ_REQUIRE(n > 0, SLAQ_ERR_INVALID_ARG, "n must be positive");
    SLAQ_REQUIRE(trace >= 0.0, SLAQ_ERR_INVALID_ARG, "trace must be >= 0");
    unsigned* const dstat = device_status_word();
    SLAQ_REQUIRE(dstat, SLAQ_ERR_HIP, "device status word unavailable");
    const double scale = (double)n / (double)nv;
    if (m <= 32)
        hipLaunchKernelGGL(vnge_ab_kernel<64>, dim3(1), dim3(64), (size_t)(3 * 64 * m + 64) * sizeof(double),
                           (hipStream_t)stream, alpha, beta, steps, nv, m, scale, trace, out, dstat);
    else
        hipLaunchKernelGGL(vnge_ab_kernel<32>, dim3(1), dim3(32), (size_t)(3 * 32 * m + 32) * sizeof(double),
                           (hipStream_t)stream, alpha, beta, steps, nv, m, scale, trace, out, dstat);
    SLAQ_LAUNCHED();
    return SLAQ_OK;
}

}  // extern "C"
