// Variance reduction of the trace estimate (paper §3.1, last paragraph: a
// "2-term polynomial variance reduction", no formula given).  Reading: the two
// terms are control variates with exactly known means,
//   Z1_p = n q_p^T L q_p    (mean tr L)
//   Z2_p = n q_p^T L^2 q_p  (mean tr L^2 = ||L||_F^2, L symmetric),
// which the m-point Gauss rule gives exactly for m >= 2 (degree <= 2m - 1):
// Z1_p = n sum_k tau2 theta, Z2_p = n sum_k tau2 theta^2.  With the plain
// per-probe values X_p = n sum_k tau2 f(theta) the estimate is
//   mean(X) - g1 (mean(Z1) - tr L) - g2 (mean(Z2) - tr L^2)
// with (g1, g2) from the degree-2 Taylor polynomial of f (SLAQ_CV_TAYLOR:
// heat (-t, t^2/2), wave (0, -t^2/2), VNGE (1/c, -1/c^2) from -x ln x ~ x - x^2)
// or from the least-squares regression of X on (Z1, Z2) over the probes
// (SLAQ_CV_FITTED).  Everything in FP64 with fixed-order reductions.
#include <cmath>

#include "common.hpp"

namespace slaq {

// tr L and tr L^2 (sum of squared entries) over the internal rows, one wave
// per row, lanes over its entries; per-lane sums, then a fixed-order block
// reduction into part[2 * block].
template <int MODE, bool WEIGHTED>
__global__ void __launch_bounds__(256) traces_kernel(const GraphStats* __restrict__ st,
                                                     const int64_t* __restrict__ rp,
                                                     const int32_t* __restrict__ col,
                                                     const float* __restrict__ w,
                                                     const double* __restrict__ diag,
                                                     double* __restrict__ part) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t nr = st->n_rows;
    double s_tr = 0.0, s_sq = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 4 + wave; i < nr; i += (int64_t)gridDim.x * 4) {
        const double di = diag[i];
        if (di == 0.0) continue;  // no data: a zero row of L (isolated node)
        const int64_t s = rp[i], e = rp[i + 1];
        double sq = 0.0, self = 0.0;  // sum_j N_ij^2 (or A_ij^2), and N_ii (or A_ii)
        for (int64_t k = s + lane; k < e; k += 64) {
            const int64_t j = col[k];
            const double a = WEIGHTED ? (double)w[k] : 1.0;
            const double v = MODE == SLAQ_LAP_NORMALIZED ? a * di * diag[j] : a;
            sq += v * v;
            if (j == i) self += v;
        }
        // fixed-order wave tree
        for (int off = 32; off > 0; off >>= 1) {
            sq += __shfl_down(sq, off);
            self += __shfl_down(self, off);
        }
        if (lane == 0) {
            if (MODE == SLAQ_LAP_NORMALIZED) {  // L_ii = 1 - N_ii, L_ij = -N_ij
                s_tr += 1.0 - self;
                s_sq += 1.0 - 2.0 * self + sq;
            } else {  // L_ii = D_ii - A_ii, L_ij = -A_ij
                s_tr += di - self;
                s_sq += di * di - 2.0 * di * self + sq;
            }
        }
    }
    __shared__ double r_tr[256], r_sq[256];
    r_tr[threadIdx.x] = s_tr;
    r_sq[threadIdx.x] = s_sq;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            r_tr[threadIdx.x] += r_tr[threadIdx.x + off];
            r_sq[threadIdx.x] += r_sq[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = r_tr[0];
        part[2 * blockIdx.x + 1] = r_sq[0];
    }
}

__global__ void __launch_bounds__(256) traces_final(const double* __restrict__ part, int nb,
                                                    double* __restrict__ out) {
    __shared__ double r_tr[256], r_sq[256];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) {
        a += part[2 * i];
        b += part[2 * i + 1];
    }
    r_tr[threadIdx.x] = a;
    r_sq[threadIdx.x] = b;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            r_tr[threadIdx.x] += r_tr[threadIdx.x + off];
            r_sq[threadIdx.x] += r_sq[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = r_tr[0];
        out[1] = r_sq[0];
    }
}

// fixed-order sum of one value per thread over the 256-thread block
__device__ __forceinline__ double block_sum(double v, double* red) {
    __syncthreads();
    red[threadIdx.x] = v;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    return red[0];
}

enum { kFunHeat = 0, kFunWave = 1, kFunVnge = 2 };

__device__ __forceinline__ double fval(int fun, double tt, double c, double x) {
    if (fun == kFunHeat) return exp(-tt * x);
    if (fun == kFunWave) return cos(tt * x);
    const double y = x / c;  // VNGE: -g(x / c), g(y) = y ln y for y > 0
    return y > 0.0 ? -(y * log(y)) : 0.0;
}

// Per probe: X (f), Z1 (theta), Z2 (theta^2), each n sum_k tau2 (.).
__device__ __forceinline__ void probe_values(const double* __restrict__ theta, const double* __restrict__ tau2,
                                             int p, int m, double n, int fun, double tt, double c, double& X,
                                             double& Z1, double& Z2) {
    double x = 0.0, z1 = 0.0, z2 = 0.0;
    for (int k = 0; k < m; ++k) {
        const double w = tau2[(int64_t)p * m + k];
        const double th = theta[(int64_t)p * m + k];
        x += w * fval(fun, tt, c, th);
        z1 += w * th;
        z2 += w * th * th;
    }
    X = n * x;
    Z1 = n * z1;
    Z2 = n * z2;
}

// Block b: the estimate at tgrid[b] (one block for VNGE).  Two passes over the
// probes: means, then centered second moments for the regression.
__global__ void __launch_bounds__(256) cv_kernel(const double* __restrict__ theta, const double* __restrict__ tau2,
                                                 int nv, int m, double n, const double* __restrict__ traces,
                                                 const double* __restrict__ tgrid, int fun, int mode,
                                                 const GraphStats* __restrict__ st, double* __restrict__ out) {
    __shared__ double red[256];
    const double tt = fun == kFunVnge ? 0.0 : tgrid[blockIdx.x];
    const double c = fun == kFunVnge ? st->trace : 1.0;
    if (fun == kFunVnge && !(c > 0.0)) {  // no density matrix: entropy 0
        if (threadIdx.x == 0) out[0] = 0.0;
        return;
    }
    double sx = 0.0, s1 = 0.0, s2 = 0.0;
    for (int p = threadIdx.x; p < nv; p += 256) {
        double X, Z1, Z2;
        probe_values(theta, tau2, p, m, n, fun, tt, c, X, Z1, Z2);
        sx += X;
        s1 += Z1;
        s2 += Z2;
    }
    const double mx = block_sum(sx, red) / nv;
    const double m1 = block_sum(s1, red) / nv;
    const double m2 = block_sum(s2, red) / nv;
    double g1 = 0.0, g2 = 0.0;
    if (mode == SLAQ_CV_TAYLOR) {
        if (fun == kFunHeat) {
            g1 = -tt;
            g2 = 0.5 * tt * tt;
        } else if (fun == kFunWave) {
            g2 = -0.5 * tt * tt;
        } else {
            g1 = 1.0 / c;
            g2 = -1.0 / (c * c);
        }
    } else if (mode == SLAQ_CV_FITTED && nv >= 3) {
        double a11 = 0.0, a22 = 0.0, a12 = 0.0, a1x = 0.0, a2x = 0.0;
        for (int p = threadIdx.x; p < nv; p += 256) {
            double X, Z1, Z2;
            probe_values(theta, tau2, p, m, n, fun, tt, c, X, Z1, Z2);
            const double x = X - mx, z1 = Z1 - m1, z2 = Z2 - m2;
            a11 += z1 * z1;
            a22 += z2 * z2;
            a12 += z1 * z2;
            a1x += z1 * x;
            a2x += z2 * x;
        }
        const double S11 = block_sum(a11, red), S22 = block_sum(a22, red), S12 = block_sum(a12, red);
        const double S1X = block_sum(a1x, red), S2X = block_sum(a2x, red);
        if (S11 > 0.0) {
            const double det = S11 * S22 - S12 * S12;
            if (nv >= 4 && S22 > 0.0 && det > 1e-10 * S11 * S22) {
                g1 = (S22 * S1X - S12 * S2X) / det;
                g2 = (S11 * S2X - S12 * S1X) / det;
            } else {
                g1 = S1X / S11;
            }
        }
    }
    if (threadIdx.x == 0) out[blockIdx.x] = mx - g1 * (m1 - traces[0]) - g2 * (m2 - traces[1]);
}

}  // namespace slaq

using namespace slaq;

#define SLAQ_TRACES_LAUNCH(MODE_, W_)                                                                            \
    hipLaunchKernelGGL((traces_kernel<MODE_, W_>), dim3(nb), dim3(256), 0, st, g->stats, g->row_ptr, g->col_idx, \
                       g->weights, g->diag64, g->trace_part)

extern "C" {

slaq_status slaq_graph_traces(slaq_graph_t g, double* traces, void* stream) {
    clear_error();
    SLAQ_REQUIRE(g && traces, SLAQ_ERR_INVALID_ARG, "NULL pointer argument");
    hipStream_t st = (hipStream_t)stream;
    int64_t nb = (g->n + 3) / 4;
    if (nb > kTraceBlocks) nb = kTraceBlocks;
    if (nb < 1) nb = 1;
    const bool wtd = g->weights != nullptr;
    if (g->laplacian == SLAQ_LAP_NORMALIZED) {
        if (wtd) SLAQ_TRACES_LAUNCH(SLAQ_LAP_NORMALIZED, true);
        else SLAQ_TRACES_LAUNCH(SLAQ_LAP_NORMALIZED, false);
    } else {
        if (wtd) SLAQ_TRACES_LAUNCH(SLAQ_LAP_COMBINATORIAL, true);
        else SLAQ_TRACES_LAUNCH(SLAQ_LAP_COMBINATORIAL, false);
    }
    SLAQ_LAUNCHED();
    hipLaunchKernelGGL(traces_final, dim3(1), dim3(256), 0, st, g->trace_part, (int)nb, traces);
    SLAQ_LAUNCHED();
    return SLAQ_OK;
}

slaq_status slaq_signature_cv(const double* theta, const double* tau2, int nv, int m, int64_t n,
                              const double* traces, const double* t, int nt, int kind, int mode, double* out,
                              void* stream) {
    clear_error();
    SLAQ_REQUIRE(theta && tau2 && traces && t && out, SLAQ_ERR_INVALID_ARG, "NULL pointer argument");
    SLAQ_REQUIRE(nv >= 1 && (int64_t)nv * m <= INT32_MAX, SLAQ_ERR_INVALID_ARG, "need nv >= 1 and nv * m < 2^31");
    SLAQ_REQUIRE(m >= 1 && m <= SLAQ_MAX_STEPS, SLAQ_ERR_INVALID_ARG, "m must be in [1, %d]", SLAQ_MAX_STEPS);
    SLAQ_REQUIRE(n > 0, SLAQ_ERR_INVALID_ARG, "n must be positive");
    SLAQ_REQUIRE(nt >= 1 && nt <= 65535, SLAQ_ERR_INVALID_ARG, "nt must be in [1, 65535]");
    SLAQ_REQUIRE(kind == SLAQ_SIG_HEAT || kind == SLAQ_SIG_WAVE, SLAQ_ERR_INVALID_ARG, "unknown signature kind");
    SLAQ_REQUIRE(mode == SLAQ_CV_NONE || mode == SLAQ_CV_TAYLOR || mode == SLAQ_CV_FITTED, SLAQ_ERR_INVALID_ARG,
                 "unknown control-variate mode %d", mode);
    hipLaunchKernelGGL(cv_kernel, dim3(nt), dim3(256), 0, (hipStream_t)stream, theta, tau2, nv, m, (double)n, traces,
                       t, kind == SLAQ_SIG_HEAT ? (int)kFunHeat : (int)kFunWave, mode, (const GraphStats*)nullptr,
                       out);
    SLAQ_LAUNCHED();
    return SLAQ_OK;
}

slaq_status slaq_vnge_cv(slaq_graph_t g, const double* theta, const double* tau2, int nv, int m,
                         const double* traces, int mode, double* out, void* stream) {
    clear_error();
    SLAQ_REQUIRE(g && theta && tau2 && traces && out, SLAQ_ERR_INVALID_ARG, "NULL pointer argument");
    SLAQ_REQUIRE(nv >= 1 && nv <= SLAQ_MAX_PROBES, SLAQ_ERR_INVALID_ARG, "nv must be in [1, %d]",
                 SLAQ_MAX_PROBES);
    SLAQ_REQUIRE(m >= 1 && m <= SLAQ_MAX_STEPS, SLAQ_ERR_INVALID_ARG, "m must be in [1, %d]", SLAQ_MAX_STEPS);
    SLAQ_REQUIRE(mode == SLAQ_CV_NONE || mode == SLAQ_CV_TAYLOR || mode == SLAQ_CV_FITTED, SLAQ_ERR_INVALID_ARG,
                 "unknown control-variate mode %d", mode);
    hipLaunchKernelGGL(cv_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream, theta, tau2, nv, m, (double)g->n,
                       traces, (const double*)nullptr, (int)kFunVnge, mode, g->stats, out);
    SLAQ_LAUNCHED();
    return SLAQ_OK;
}

}  // extern "C"
