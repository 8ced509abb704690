// Learned closure: an MLP maps a probe's 5-step Gauss rule (nodes and weights)
// to a correction of log Q_5(t), so that Q_5(t) exp(y_hat(t)) approximates the
// 30-step value Q_30(t) (Q_m(t) = sum_k tau2_k exp(-t theta_k), §3.1 eq.
// "quadratic").  Predictions are clamped to the Gauss / Gauss-Radau bracket
// Q_5 <= Q <= Q_R of each probe; a graph with a prediction outside the bracket
// by more than a tolerance is flagged for plain SLQ.  The paper has no learned
// component: this is an addition on top of its method.
//
// Network: d_in (padded to 32) -> 256 -> 256 -> 256 -> nt, SiLU between,
// MSE loss, Adam on FP32 master weights; every product runs on BF16 MFMA
// (v_mfma_f32_16x16x32_bf16) with FP32 accumulation.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "common.hpp"
#include "profile.hpp"
#include "tridiag.hpp"

typedef __bf16 bf16;
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

namespace slaq {

// tile sizes: 64 x 64 outputs per block, K staged 128 deep (four MFMA K-steps
// of 32); LDS row stride 136 bf16 = 68 dwords puts the 16 rows a fragment read
// touches on distinct 4-bank groups
constexpr int kTM = 64, kTN = 64, kTK = 128, kLdsK = kTK + 8;
constexpr int kDinPad = 32;

enum { EPI_STORE = 0, EPI_BIAS_SILU = 1, EPI_BIAS = 2, EPI_DSILU = 3 };

struct GemmArgs {
    int M, N, K;
    const bf16* A;
    int lda;
    const bf16* B;
    int ldb;
    float* C;
    int ldc;
    const float* bias;
    float* Z;        // EPI_BIAS_SILU: pre-activation out
    bf16* H;         // EPI_BIAS_SILU: activation out; EPI_DSILU: gradient out
    const float* Zin;  // EPI_DSILU: pre-activation in
    int kslice;        // split K: rows of K per blockIdx.z (0: the whole of K)
    float* part;       // split K: FP32 partial products [gridDim.z][M][ldc]
};

__device__ __forceinline__ float silu_f(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float dsilu_f(float z) {
    const float s = 1.0f / (1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

// C (M x N) = op(A) (M x K) * op(B) (K x N).  TA: A stored K x M (lda over m);
// TB: B stored N x K (ldb over k).  64x64 tile per block of 4 waves, each wave
// a 32x32 sub-tile of 2x2 MFMA 16x16x32 blocks; operands staged through LDS
// with K contiguous so each lane's fragment is one 16-byte read.  A stage of
// kTK rows of K is fetched with all of a thread's loads in flight at once: one
// 16-byte load per 8 elements when the tile is wholly in bounds and the operand
// rows are 16-byte aligned, element by element (zero outside) otherwise.
template <bool TRANS>
__device__ __forceinline__ void stage_operand(bf16 (*S)[kLdsK], const bf16* __restrict__ X, int ld, int o0, int olim,
                                              int k0, int klim, bool vec, int t) {
    // TRANS: X stored K x (outer), rows of K at stride ld; else (outer) x K
    constexpr int kVec = kTM * kTK / 8 / 256;  // 16-byte vectors per thread
    if (vec) {
        bf16x8 v[kVec];
#pragma unroll
        for (int j = 0; j < kVec; ++j) {
            const int q = t + 256 * j;
            if (TRANS) {
                const int kk = q / (kTM / 8), oc = (q % (kTM / 8)) * 8;
                v[j] = *(const bf16x8*)&X[(int64_t)(k0 + kk) * ld + o0 + oc];
            } else {
                const int r = q / (kTK / 8), kc = (q % (kTK / 8)) * 8;
                v[j] = *(const bf16x8*)&X[(int64_t)(o0 + r) * ld + k0 + kc];
            }
        }
#pragma unroll
        for (int j = 0; j < kVec; ++j) {
            const int q = t + 256 * j;
            if (TRANS) {
                const int kk = q / (kTM / 8), oc = (q % (kTM / 8)) * 8;
#pragma unroll
                for (int i = 0; i < 8; ++i) S[oc + i][kk] = v[j][i];
            } else {
                const int r = q / (kTK / 8), kc = (q % (kTK / 8)) * 8;
                *(bf16x8*)&S[r][kc] = v[j];
            }
        }
        return;
    }
    const bf16 zero = (bf16)0.0f;
#pragma unroll
    for (int j = 0; j < kVec; ++j) {
        const int q = t + 256 * j;
        if (TRANS) {
            const int kk = q / (kTM / 8), oc = (q % (kTM / 8)) * 8;
            const int gk = k0 + kk;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int go = o0 + oc + i;
                S[oc + i][kk] = (go < olim && gk < klim) ? X[(int64_t)gk * ld + go] : zero;
            }
        } else {
            const int r = q / (kTK / 8), kc = (q % (kTK / 8)) * 8;
            const int go = o0 + r;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int gk = k0 + kc + i;
                S[r][kc + i] = (go < olim && gk < klim) ? X[(int64_t)go * ld + gk] : zero;
            }
        }
    }
}

template <int EPI, bool TA, bool TB>
__global__ void __launch_bounds__(256) mlp_gemm(GemmArgs g) {
    static_assert(kTM == kTN, "one staging routine serves both operands");
    __shared__ __align__(16) bf16 As[kTM][kLdsK];
    __shared__ __align__(16) bf16 Bs[kTN][kLdsK];
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int m0 = blockIdx.y * kTM, n0 = blockIdx.x * kTN;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int kb = g.kslice > 0 ? (int)blockIdx.z * g.kslice : 0;
    const int ke = g.kslice > 0 ? min(g.K, kb + g.kslice) : g.K;
    const bool vec_ok = (g.lda % 8) == 0 && (g.ldb % 8) == 0 && (((uintptr_t)g.A | (uintptr_t)g.B) & 15) == 0 &&
                        m0 + kTM <= g.M && n0 + kTN <= g.N;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = kb; k0 < ke; k0 += kTK) {
        const bool vec = vec_ok && k0 + kTK <= ke;
        stage_operand<TA>(As, g.A, g.lda, m0, g.M, k0, ke, vec, t);
        stage_operand<!TB>(Bs, g.B, g.ldb, n0, g.N, k0, ke, vec, t);
        __syncthreads();
        const int kn = min(kTK, ke - k0);
        for (int kk = 0; kk < kn; kk += 32) {
            bf16x8 a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i)
                a[i] = *(const bf16x8*)&As[wm + i * 16 + (lane & 15)][kk + (lane >> 4) * 8];
#pragma unroll
            for (int j = 0; j < 2; ++j)
                b[j] = *(const bf16x8*)&Bs[wn + j * 16 + (lane & 15)][kk + (lane >> 4) * 8];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    // ---- epilogue: lane holds rows (lane/16)*4 + r of column lane%16
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm + i * 16 + (lane >> 4) * 4 + r;
                const int col = n0 + wn + j * 16 + (lane & 15);
                if (row >= g.M || col >= g.N) continue;
                const int64_t o = (int64_t)row * g.ldc + col;
                const float v = acc[i][j][r];
                if (EPI == EPI_STORE && g.kslice > 0) {
                    g.part[(int64_t)blockIdx.z * g.M * g.ldc + o] = v;
                } else if (EPI == EPI_STORE) {
                    g.C[o] = v;
                } else if (EPI == EPI_BIAS) {
                    g.C[o] = v + g.bias[col];
                } else if (EPI == EPI_BIAS_SILU) {
                    const float z = v + g.bias[col];
                    g.Z[o] = z;
                    g.H[o] = (bf16)silu_f(z);
                } else {
                    g.H[o] = (bf16)(v * dsilu_f(g.Zin[o]));
                }
            }
}

// C = the S split-K partial products summed in slice order (deterministic).
__global__ void __launch_bounds__(256) splitk_sum(int M, int N, int ldc, int S, const float* __restrict__ part,
                                                  float* __restrict__ C) {
    const int64_t total = (int64_t)M * N, plane = (int64_t)M * ldc;
    for (int64_t x = blockIdx.x * 256LL + threadIdx.x; x < total; x += (int64_t)gridDim.x * 256) {
        const int64_t o = (x / N) * ldc + x % N;
        float s = 0.0f;
        for (int z = 0; z < S; ++z) s += part[z * plane + o];
        C[o] = s;
    }
}

// dY = 2 (Y - T) / (B N) as BF16; per-block partial sums of (Y - T)^2.
__global__ void __launch_bounds__(256) mse_grad(int64_t total, const float* __restrict__ Y, const float* __restrict__ T,
                                                float scale, bf16* __restrict__ dY, float* __restrict__ dYf,
                                                double* __restrict__ part) {
    double s = 0.0;
    for (int64_t i = blockIdx.x * 256LL + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
        const float d = Y[i] - T[i];
        s += (double)d * d;
        dY[i] = (bf16)(scale * d);
        dYf[i] = scale * d;
    }
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) loss_final(const double* __restrict__ part, int nparts, double inv_count,
                                                  float* __restrict__ loss) {
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = (float)(red[0] * inv_count);
}

// db[n] = sum over rows of D[row][n] (BF16 or FP32 input), fixed order: 16
// row groups per column, each summing every 16th row into four interleaved
// accumulators, then the groups in order.
template <typename T>
__global__ void __launch_bounds__(1024) col_sum(int rows, int N, const T* __restrict__ D, float* __restrict__ db) {
    const int lane = threadIdx.x & 63, r0 = threadIdx.x >> 6;
    const int c = blockIdx.x * 64 + lane;
    float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
    if (c < N) {
        int r = r0;
        for (; r + 48 < rows; r += 64) {
            s0 += (float)D[(int64_t)r * N + c];
            s1 += (float)D[(int64_t)(r + 16) * N + c];
            s2 += (float)D[(int64_t)(r + 32) * N + c];
            s3 += (float)D[(int64_t)(r + 48) * N + c];
        }
        for (; r < rows; r += 16) s0 += (float)D[(int64_t)r * N + c];
    }
    __shared__ float red[16][64];
    red[r0][lane] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    if (threadIdx.x < 64 && c < N) {
        float t = 0.0f;
#pragma unroll
        for (int g = 0; g < 16; ++g) t += red[g][lane];
        db[c] = t;
    }
}

__global__ void __launch_bounds__(256) adam_step(int64_t P, float* __restrict__ w, bf16* __restrict__ wb,
                                                 const float* __restrict__ grad, float* __restrict__ m1,
                                                 float* __restrict__ m2, float lr, float b1, float b2, float eps,
                                                 float c1, float c2) {
    for (int64_t i = blockIdx.x * 256LL + threadIdx.x; i < P; i += (int64_t)gridDim.x * 256) {
        const float gr = grad[i];
        const float a = b1 * m1[i] + (1.0f - b1) * gr;
        const float v = b2 * m2[i] + (1.0f - b2) * gr * gr;
        m1[i] = a;
        m2[i] = v;
        const float wn = w[i] - lr * (a / c1) / (sqrtf(v / c2) + eps);
        w[i] = wn;
        wb[i] = (bf16)wn;
    }
}

// Glorot-uniform init from SplitMix64 keyed on (seed, index); biases 0.
__global__ void __launch_bounds__(256) init_params(int64_t P, uint64_t seed, const int64_t* __restrict__ off,
                                                   const int* __restrict__ fan, int nlayers, float* __restrict__ w,
                                                   bf16* __restrict__ wb, float* __restrict__ m1,
                                                   float* __restrict__ m2, int d_in) {
    for (int64_t i = blockIdx.x * 256LL + threadIdx.x; i < P; i += (int64_t)gridDim.x * 256) {
        float v = 0.0f;
        for (int l = 0; l < nlayers; ++l) {
            const int64_t wo = off[2 * l], bo = off[2 * l + 1];
            if (i >= wo && i < bo) {
                const int fi = fan[2 * l], fo = fan[2 * l + 1];
                const int64_t r = (i - wo) / fo;
                if (l == 0 && r >= d_in) break;  // padded input rows stay 0
                uint64_t z = seed + ((uint64_t)i + 1ull) * 0x9E3779B97F4A7C15ull;
                z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
                z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
                z ^= z >> 31;
                const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);  // [0, 1)
                const double a = sqrt(6.0 / (double)((l == 0 ? d_in : fi) + fo));
                v = (float)((2.0 * u - 1.0) * a);
                break;
            }
        }
        w[i] = v;
        wb[i] = (bf16)v;
        m1[i] = 0.0f;
        m2[i] = 0.0f;
    }
}

// ------------------------------------------------------ per-probe rules ---
// From a probe's Lanczos coefficients (row stride ms): the mf-node Gauss rule
// (nodes ascending) and the (mf+1)-node Gauss-Radau rule with a node fixed at
// a = 0.  A probe that stopped before mf steps has an exact Gauss rule; its
// Radau rule is set equal to it.
__global__ void __launch_bounds__(64) probe_rules(int64_t count, const double* __restrict__ alpha,
                                                  const double* __restrict__ beta, const int32_t* __restrict__ steps,
                                                  int ms, int mf, double* __restrict__ th, double* __restrict__ w2,
                                                  double* __restrict__ thr, double* __restrict__ w2r,
                                                  unsigned* dstat) {
    const int64_t p = blockIdx.x * 64LL + threadIdx.x;
    if (p >= count) return;
    double d[SLAQ_MAX_STEPS + 1], e[SLAQ_MAX_STEPS + 1], u[SLAQ_MAX_STEPS + 1];
    int k = steps[p] < mf ? steps[p] : mf;
    if (k < 1) k = 1;
    const double* a = alpha + p * ms;
    const double* b = beta + p * ms;
    for (int i = 0; i < k; ++i) {
        d[i] = a[i];
        e[i] = i + 1 < k ? b[i] : 0.0;
    }
    if (tridiag_eig_first_row(d, e, u, k, 1) < 0) raise_status(dstat, SLAQ_STATUS_NO_CONVERGENCE);
    // insertion sort ascending
    for (int i = 1; i < k; ++i) {
        const double x = d[i], y = u[i] * u[i];
        int jj = i - 1;
        while (jj >= 0 && d[jj] > x) {
            d[jj + 1] = d[jj];
            u[jj + 1] = u[jj];
            --jj;
        }
        d[jj + 1] = x;
        u[jj + 1] = sqrt(y);
    }
    for (int i = 0; i < mf; ++i) {
        th[p * mf + i] = i < k ? d[i] : 0.0;
        w2[p * mf + i] = i < k ? u[i] * u[i] : 0.0;
    }
    const bool exact = steps[p] < mf;
    if (exact) {
        for (int i = 0; i <= mf; ++i) {
            thr[p * (mf + 1) + i] = i < k ? d[i] : 0.0;
            w2r[p * (mf + 1) + i] = i < k ? u[i] * u[i] : 0.0;
        }
        return;
    }
    // Radau: (T_k - 0 I) delta = beta_k^2 e_k  ->  phi = beta_k^2 / (last LDL^T pivot)
    double piv = a[0];
    for (int i = 1; i < k && piv > 0.0; ++i) piv = a[i] - b[i - 1] * b[i - 1] / piv;
    if (!(piv > 1e-300)) {
        // T_k numerically singular at the fixed node: fall back to the trivial
        // upper bound Q <= ||q||^2 = 1 (one node at 0, weight 1)
        for (int i = 0; i <= mf; ++i) {
            thr[p * (mf + 1) + i] = 0.0;
            w2r[p * (mf + 1) + i] = i == 0 ? 1.0 : 0.0;
        }
        return;
    }
    const double bk = b[k - 1];
    const double phi = bk * bk / piv;
    for (int i = 0; i < k; ++i) {
        d[i] = a[i];
        e[i] = b[i];
    }
    d[k] = phi;
    e[k - 1] = bk;
    e[k] = 0.0;
    if (tridiag_eig_first_row(d, e, u, k + 1, 1) < 0) raise_status(dstat, SLAQ_STATUS_NO_CONVERGENCE);
    for (int i = 0; i <= mf; ++i) {
        thr[p * (mf + 1) + i] = i <= k ? d[i] : 0.0;
        w2r[p * (mf + 1) + i] = i <= k ? u[i] * u[i] : 0.0;
    }
}

// x = (theta_1..mf ascending, tau2_1..mf), zero-padded to kDinPad, BF16.
__global__ void __launch_bounds__(256) make_features(int64_t count, int mf, const double* __restrict__ th,
                                                     const double* __restrict__ w2, bf16* __restrict__ X) {
    const int64_t i = blockIdx.x * 256LL + threadIdx.x;
    if (i >= count * kDinPad) return;
    const int64_t p = i / kDinPad;
    const int c = (int)(i % kDinPad);
    float v = 0.0f;
    if (c < mf) v = (float)th[p * mf + c];
    else if (c < 2 * mf) v = (float)w2[p * mf + c - mf];
    X[i] = (bf16)v;
}

// Q[p][b] = sum_k w2[p][k] exp(-t_b th[p][k]) for k < kn (row stride ks).
__global__ void __launch_bounds__(256) gauss_values(int64_t count, int kn, int ks, const double* __restrict__ th,
                                                    const double* __restrict__ w2, const double* __restrict__ t,
                                                    int nt, double* __restrict__ Q) {
    const int64_t i = blockIdx.x * 256LL + threadIdx.x;
    if (i >= count * nt) return;
    const int64_t p = i / nt;
    const double tt = t[i % nt];
    double s = 0.0;
    for (int k = 0; k < kn; ++k) s += w2[p * ks + k] * exp(-tt * th[p * ks + k]);
    Q[i] = s;
}

__global__ void __launch_bounds__(256) log_ratio(int64_t total, const double* __restrict__ Qa,
                                                 const double* __restrict__ Qb, float* __restrict__ y) {
    const int64_t i = blockIdx.x * 256LL + threadIdx.x;
    if (i < total) y[i] = (float)(log(Qa[i]) - log(Qb[i]));
}

// Q_hat = Q5 exp(y_hat) clamped to [Q5, QR] per probe; heat[g][b] =
// n_g / nv sum_p Q_hat.  Where the graph's bracket is narrower than tol
// (relative) the clamped value is within tol of every value the bracket
// allows, whatever the network said.  flags[g] = 1 when, at some time, the
// bracket is wider than tol AND clamping moved the graph's heat by more than
// tol: there the prediction disagrees with a bound that cannot vouch for it.
// One block per graph.
__global__ void __launch_bounds__(256) closure_apply(int G, int nv, int nt, const float* __restrict__ yhat,
                                                     const double* __restrict__ Q5, const double* __restrict__ QR,
                                                     const int64_t* __restrict__ gn, double tol,
                                                     double* __restrict__ heat, int* __restrict__ flags) {
    const int g = blockIdx.x;
    int bad = 0;
    for (int b = threadIdx.x; b < nt; b += blockDim.x) {
        double s = 0.0, raw = 0.0, slo = 0.0, shi = 0.0;
        for (int p = 0; p < nv; ++p) {
            const int64_t o = ((int64_t)g * nv + p) * nt + b;
            const double lo = Q5[o], hi = QR[o];
            const double q = lo * exp((double)yhat[o]);
            raw += q;
            slo += lo;
            shi += hi;
            s += q < lo ? lo : (q > hi ? hi : q);
        }
        if (!(shi - slo <= tol * s) && !(fabs(raw - s) <= tol * s)) bad = 1;
        heat[(int64_t)g * nt + b] = (double)gn[g] / nv * s;
    }
    __shared__ int any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    if (bad) atomicOr(&any, 1);
    __syncthreads();
    if (threadIdx.x == 0) flags[g] = any;
}

// Hutchinson's estimate from per-probe quadratic forms (§3.1, eq. "trace"):
// heat[g][b] = n_g / nv sum_p Q[g nv + p][b], probes added in order.  One
// block per graph, threads over the times.
__global__ void __launch_bounds__(256) hutchinson_mean(int nv, int nt, const double* __restrict__ Q,
                                                       const int64_t* __restrict__ gn, double* __restrict__ heat) {
    const int g = blockIdx.x;
    for (int b = threadIdx.x; b < nt; b += blockDim.x) {
        double s = 0.0;
        for (int p = 0; p < nv; ++p) s += Q[((int64_t)g * nv + p) * nt + b];
        heat[(int64_t)g * nt + b] = (double)gn[g] / nv * s;
    }
}

__global__ void __launch_bounds__(256) to_bf16(int64_t n, const float* __restrict__ a, bf16* __restrict__ b) {
    for (int64_t i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) b[i] = (bf16)a[i];
}

}  // namespace slaq

// --------------------------------------------------------------- handle ---
struct slaq_closure_s {
    int d_in, hidden, nt, nlayers;
    int dims[5];            // layer widths: kDinPad, hidden, hidden, hidden, nt
    int64_t P;              // parameters
    int64_t off[8];         // W0 b0 W1 b1 ... offsets in the parameter vector
    float* w;               // FP32 master weights
    bf16* wb;               // BF16 copies (weights and biases)
    float* grad;
    float* m1;
    float* m2;
    int64_t* off_dev;
    int* fan_dev;
    int step;
};

namespace slaq {

struct ClosureWs {
    size_t x, z[3], h[3], y, dy, dyf, dh, dz, part, kpart, total;
};

constexpr int kSplitKMin = kTK;               // fewest rows of K per slice
constexpr size_t kSplitKBytes = 16u << 20;    // largest partial-product buffer

// slices of K for a weight-gradient product (M x N, K = batch rows): enough
// workgroups to fill the chip while each slice keeps at least kSplitKMin rows
// and the partials fit kSplitKBytes; 1 means no split
static int splitk_slices(int M, int N, int64_t K) {
    const int64_t tiles = (int64_t)((N + kTN - 1) / kTN) * ((M + kTM - 1) / kTM);
    int64_t s = K / kSplitKMin;
    s = std::min<int64_t>(s, std::max<int64_t>(1, 256 / tiles));
    s = std::min<int64_t>(s, (int64_t)(kSplitKBytes / ((size_t)M * N * 4)));
    return (int)std::max<int64_t>(1, s);
}

static ClosureWs closure_ws(const slaq_closure_s* c, int64_t B) {
    ClosureWs L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align_up(bytes, 256);
        return o;
    };
    const int H = c->hidden, N = c->nt;
    for (int l = 0; l < 3; ++l) {
        L.z[l] = take((size_t)B * H * 4);
        L.h[l] = take((size_t)B * H * 2);
    }
    L.y = take((size_t)B * N * 4);
    L.dy = take((size_t)B * (N > H ? N : H) * 2);
    L.dyf = take((size_t)B * N * 4);
    L.dh = take((size_t)B * H * 4);
    L.dz = take((size_t)B * H * 2);
    L.part = take(1024 * 8);
    size_t kp = 0;
    for (int l = 0; l < 4; ++l) {
        const int S = splitk_slices(c->dims[l], c->dims[l + 1], B);
        if (S > 1) kp = std::max(kp, (size_t)S * c->dims[l] * c->dims[l + 1] * 4);
    }
    L.kpart = take(kp);
    L.total = off;
    return L;
}

template <int EPI, bool TA, bool TB>
static slaq_status gemm(const GemmArgs& a, hipStream_t st, const char* tag) {
    dim3 grid((a.N + kTN - 1) / kTN, (a.M + kTM - 1) / kTM);
    SLAQ_TIMED(tag, st, hipLaunchKernelGGL((mlp_gemm<EPI, TA, TB>), grid, dim3(256), 0, st, a));
    SLAQ_LAUNCHED();
    return SLAQ_OK;
}

// C = A^T B with A stored K x M: split over K when that fills more of the chip
// (partials into the workspace, then a fixed-order sum)
static slaq_status gemm_wgrad(GemmArgs a, float* kpart, hipStream_t st, const char* tag) {
    const int S = splitk_slices(a.M, a.N, a.K);
    if (S <= 1) return gemm<EPI_STORE, true, false>(a, st, tag);
    const int per = (a.K + S - 1) / S;
    a.kslice = (per + kTK - 1) / kTK * kTK;
    const int Z = (a.K + a.kslice - 1) / a.kslice;
    a.part = kpart;
    dim3 grid((a.N + kTN - 1) / kTN, (a.M + kTM - 1) / kTM, Z);
    SLAQ_TIMED(tag, st, hipLaunchKernelGGL((mlp_gemm<EPI_STORE, true, false>), grid, dim3(256), 0, st, a));
    SLAQ_LAUNCHED();
    const int64_t total = (int64_t)a.M * a.N;
    const int nb = (int)std::min<int64_t>(1024, (total + 255) / 256);
    hipLaunchKernelGGL(splitk_sum, dim3(nb), dim3(256), 0, st, a.M, a.N, a.ldc, Z, (const float*)kpart, a.C);
    SLAQ_LAUNCHED();
    return SLAQ_OK;
}


// forward for a batch of B rows: fills z/h of the hidden layers and y
static slaq_status closure_fwd(slaq_closure_s* c, const bf16* X, int64_t B, char* ws, const ClosureWs& L,
                               hipStream_t st) {
    const bf16* in = X;
    for (int l = 0; l < 3; ++l) {
        GemmArgs a{};
        a.M = (int)B;
        a.N = c->dims[l + 1];
        a.K = c->dims[l];
        a.A = in;
        a.lda = c->dims[l];
        a.B = c->wb + c->off[2 * l];
        a.ldb = c->dims[l + 1];
        a.ldc = c->dims[l + 1];
        a.bias = c->w + c->off[2 * l + 1];
        a.Z = (float*)(ws + L.z[l]);
        a.H = (bf16*)(ws + L.h[l]);
        SLAQ_TRY((gemm<EPI_BIAS_SILU, false, false>(a, st, "mlp_fwd")));
        in = a.H;
    }
    GemmArgs a{};
    a.M = (int)B;
    a.N = c->dims[4];
    a.K = c->dims[3];
    a.A = in;
    a.lda = c->dims[3];
    a.B = c->wb + c->off[6];
    a.ldb = c->dims[4];
    a.C = (float*)(ws + L.y);
    a.ldc = c->dims[4];
    a.bias = c->w + c->off[7];
    return gemm<EPI_BIAS, false, false>(a, st, "mlp_fwd");
}

// gradients of the mean squared error into c->grad; loss (device float) optional
static slaq_status closure_bwd(slaq_closure_s* c, const bf16* X, const float* Yt, int64_t B, float* loss, char* ws,
                               const ClosureWs& L, hipStream_t st) {
    const int N = c->dims[4];
    const int64_t total = B * N;
    int nb = (int)((total + 255) / 256);
    if (nb > 1024) nb = 1024;
    bf16* dy = (bf16*)(ws + L.dy);
    float* dyf = (float*)(ws + L.dyf);
    double* part = (double*)(ws + L.part);
    SLAQ_TIMED("mlp_bwd", st,
               hipLaunchKernelGGL(mse_grad, dim3(nb), dim3(256), 0, st, total, (const float*)(ws + L.y), Yt,
                                  (float)(2.0 / (double)total), dy, dyf, part));
    SLAQ_LAUNCHED();
    if (loss) {
        hipLaunchKernelGGL(loss_final, dim3(1), dim3(256), 0, st, part, nb, 1.0 / (double)total, loss);
        SLAQ_LAUNCHED();
    }
    // layer l = 3 (output, no activation) down to 0
    const bf16* dcur = dy;  // gradient w.r.t. the output of layer l's affine map
    for (int l = 3; l >= 0; --l) {
        const int din = c->dims[l], dout = c->dims[l + 1];
        const bf16* Hin = l == 0 ? X : (const bf16*)(ws + L.h[l - 1]);
        // dW_l = Hin^T dcur  (din x dout), K = B
        GemmArgs gw{};
        gw.M = din;
        gw.N = dout;
        gw.K = (int)B;
        gw.A = Hin;
        gw.lda = din;
        gw.B = dcur;
        gw.ldb = dout;
        gw.C = c->grad + c->off[2 * l];
        gw.ldc = dout;
        SLAQ_TRY(gemm_wgrad(gw, (float*)(ws + L.kpart), st, "mlp_bwd"));
        // db_l = column sums of dcur (FP32 for the output layer)
        if (l == 3)
            hipLaunchKernelGGL(col_sum<float>, dim3((dout + 63) / 64), dim3(1024), 0, st, (int)B, dout, dyf,
                               c->grad + c->off[2 * l + 1]);
        else
            hipLaunchKernelGGL(col_sum<bf16>, dim3((dout + 63) / 64), dim3(1024), 0, st, (int)B, dout, dcur,
                               c->grad + c->off[2 * l + 1]);
        SLAQ_LAUNCHED();
        if (l == 0) break;
        // d(pre-activation of layer l-1) = (dcur W_l^T) * SiLU'(z_{l-1})
        GemmArgs gd{};
        gd.M = (int)B;
        gd.N = din;
        gd.K = dout;
        gd.A = dcur;
        gd.lda = dout;
        gd.B = c->wb + c->off[2 * l];
        gd.ldb = dout;
        gd.ldc = din;
        gd.Zin = (const float*)(ws + L.z[l - 1]);
        bf16* dnext = (bf16*)(ws + ((l & 1) ? L.dz : L.dy));
        if (dnext == dcur) dnext = (bf16*)(ws + L.dz);
        gd.H = dnext;
        SLAQ_TRY((gemm<EPI_DSILU, false, true>(gd, st, "mlp_bwd")));
        dcur = dnext;
    }
    return SLAQ_OK;
}

}  // namespace slaq

using namespace slaq;

extern "C" {

slaq_status slaq_closure_create(int d_in, int hidden, int nt, uint64_t seed, void* stream, slaq_closure_t* out) {
    clear_error();
    SLAQ_REQUIRE(out, SLAQ_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    SLAQ_REQUIRE(d_in >= 1 && d_in <= kDinPad, SLAQ_ERR_INVALID_ARG, "d_in must be in [1, %d]", kDinPad);
    SLAQ_REQUIRE(hidden >= 16 && hidden % 16 == 0 && hidden <= 4096, SLAQ_ERR_INVALID_ARG,
                 "hidden must be a multiple of 16 in [16, 4096]");
    SLAQ_REQUIRE(nt >= 1 && nt <= 4096, SLAQ_ERR_INVALID_ARG, "nt must be in [1, 4096]");
    slaq_closure_s* c = new (std::nothrow) slaq_closure_s();
    SLAQ_REQUIRE(c, SLAQ_ERR_INVALID_ARG, "out of host memory");
    c->d_in = d_in;
    c->hidden = hidden;
    c->nt = nt;
    c->nlayers = 4;
    c->dims[0] = kDinPad;
    c->dims[1] = c->dims[2] = c->dims[3] = hidden;
    c->dims[4] = nt;
    int64_t o = 0;
    int fan[8];
    for (int l = 0; l < 4; ++l) {
        c->off[2 * l] = o;
        o += (int64_t)c->dims[l] * c->dims[l + 1];
        c->off[2 * l + 1] = o;
        o += c->dims[l + 1];
        fan[2 * l] = c->dims[l];
        fan[2 * l + 1] = c->dims[l + 1];
    }
    c->P = o;
    hipStream_t st = (hipStream_t)stream;
    bool ok = hipMalloc(&c->w, o * 4) == hipSuccess && hipMalloc(&c->wb, o * 2) == hipSuccess &&
              hipMalloc(&c->grad, o * 4) == hipSuccess && hipMalloc(&c->m1, o * 4) == hipSuccess &&
              hipMalloc(&c->m2, o * 4) == hipSuccess && hipMalloc(&c->off_dev, 8 * 8) == hipSuccess &&
              hipMalloc(&c->fan_dev, 8 * 4) == hipSuccess;
    ok = ok && hipMemcpy(c->off_dev, c->off, 8 * 8, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(c->fan_dev, fan, 8 * 4, hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) {
        slaq_closure_destroy(c);
        set_error("allocation of the closure parameters failed");
        return SLAQ_ERR_HIP;
    }
    hipLaunchKernelGGL(init_params, dim3(256), dim3(256), 0, st, o, seed, c->off_dev, c->fan_dev, 4, c->w, c->wb,
                       c->m1, c->m2, d_in);
    SLAQ_LAUNCHED();
    *out = c;
    return SLAQ_OK;
}

slaq_status slaq_closure_destroy(slaq_closure_t c) {
    if (!c) return SLAQ_OK;
    (void)hipFree(c->w);
    (void)hipFree(c->wb);
    (void)hipFree(c->grad);
    (void)hipFree(c->m1);
    (void)hipFree(c->m2);
    (void)hipFree(c->off_dev);
    (void)hipFree(c->fan_dev);
    delete c;
    return SLAQ_OK;
}

slaq_status slaq_closure_info(slaq_closure_t c, int64_t* n_params, int64_t* offsets /*[8]*/, int* dims /*[5]*/) {
    clear_error();
    SLAQ_REQUIRE(c, SLAQ_ERR_INVALID_ARG, "closure is NULL");
    if (n_params) *n_params = c->P;
    if (offsets) std::memcpy(offsets, c->off, sizeof(c->off));
    if (dims) std::memcpy(dims, c->dims, sizeof(c->dims));
    return SLAQ_OK;
}

slaq_status slaq_closure_workspace(slaq_closure_t c, int64_t batch, size_t* bytes) {
    clear_error();
    SLAQ_REQUIRE(c && bytes && batch >= 1, SLAQ_ERR_INVALID_ARG, "bad argument");
    *bytes = closure_ws(c, batch).total;
    return SLAQ_OK;
}

// which: 0 = FP32 master weights, 1 = gradients of the last backward pass
slaq_status slaq_closure_get(slaq_closure_t c, int which, float* dst, void* stream) {
    clear_error();
    SLAQ_REQUIRE(c && dst && which >= 0 && which <= 3, SLAQ_ERR_INVALID_ARG, "bad argument");
    const float* src[4] = {c->w, c->grad, c->m1, c->m2};
    SLAQ_HIP(hipMemcpyAsync(dst, src[which], c->P * 4, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return SLAQ_OK;
}

slaq_status slaq_closure_get_step(slaq_closure_t c, int* step) {
    clear_error();
    SLAQ_REQUIRE(c && step, SLAQ_ERR_INVALID_ARG, "bad argument");
    *step = c->step;
    return SLAQ_OK;
}

slaq_status slaq_closure_set_optimizer(slaq_closure_t c, const float* m1, const float* m2, int step, void* stream) {
    clear_error();
    SLAQ_REQUIRE(c && m1 && m2 && step >= 0, SLAQ_ERR_INVALID_ARG, "bad argument");
    hipStream_t st = (hipStream_t)stream;
    SLAQ_HIP(hipMemcpyAsync(c->m1, m1, c->P * 4, hipMemcpyDeviceToDevice, st));
    SLAQ_HIP(hipMemcpyAsync(c->m2, m2, c->P * 4, hipMemcpyDeviceToDevice, st));
    c->step = step;
    return SLAQ_OK;
}

slaq_status slaq_closure_set(slaq_closure_t c, const float* src, int reset_optimizer, void* stream) {
    clear_error();
    SLAQ_REQUIRE(c && src, SLAQ_ERR_INVALID_ARG, "bad argument");
    hipStream_t st = (hipStream_t)stream;
    SLAQ_HIP(hipMemcpyAsync(c->w, src, c->P * 4, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(to_bf16, dim3(256), dim3(256), 0, st, c->P, c->w, c->wb);
    SLAQ_LAUNCHED();
    if (reset_optimizer) {
        SLAQ_HIP(hipMemsetAsync(c->m1, 0, c->P * 4, st));
        SLAQ_HIP(hipMemsetAsync(c->m2, 0, c->P * 4, st));
        c->step = 0;
    }
    return SLAQ_OK;
}

slaq_status slaq_closure_forward(slaq_closure_t c, const void* x, int64_t batch, float* yhat, void* workspace,
                                 size_t ws_bytes, void* stream) {
    clear_error();
    SLAQ_REQUIRE(c && x && yhat && workspace && batch >= 1 && batch <= INT32_MAX, SLAQ_ERR_INVALID_ARG,
                 "bad argument");
    const ClosureWs L = closure_ws(c, batch);
    SLAQ_REQUIRE(ws_bytes >= L.total, SLAQ_ERR_WORKSPACE, "closure workspace needs %zu bytes", L.total);
    hipStream_t st = (hipStream_t)stream;
    char* ws = (char*)workspace;
    SLAQ_TRY(closure_fwd(c, (const bf16*)x, batch, ws, L, st));
    SLAQ_HIP(hipMemcpyAsync(yhat, ws + L.y, (size_t)batch * c->nt * 4, hipMemcpyDeviceToDevice, st));
    return SLAQ_OK;
}

// Gradients of the MSE between the network's output and y (FP32 [batch][nt]);
// lr > 0 also applies one Adam step (beta1 0.9, beta2 0.999, eps 1e-8).
slaq_status slaq_closure_train_step(slaq_closure_t c, const void* x, const float* y, int64_t batch, float lr,
                                    float* loss, void* workspace, size_t ws_bytes, void* stream) {
    clear_error();
    SLAQ_REQUIRE(c && x && y && workspace && batch >= 1 && batch <= INT32_MAX, SLAQ_ERR_INVALID_ARG, "bad argument");
    const ClosureWs L = closure_ws(c, batch);
    SLAQ_REQUIRE(ws_bytes >= L.total, SLAQ_ERR_WORKSPACE, "closure workspace needs %zu bytes", L.total);
    hipStream_t st = (hipStream_t)stream;
    char* ws = (char*)workspace;
    SLAQ_TRY(closure_fwd(c, (const bf16*)x, batch, ws, L, st));
    SLAQ_TRY(closure_bwd(c, (const bf16*)x, y, batch, loss, ws, L, st));
    if (lr > 0.0f) {
        c->step += 1;
        const float c1 = 1.0f - powf(0.9f, (float)c->step), c2 = 1.0f - powf(0.999f, (float)c->step);
        SLAQ_TIMED("mlp_adam", st,
                   hipLaunchKernelGGL(adam_step, dim3(256), dim3(256), 0, st, c->P, c->w, c->wb, c->grad, c->m1,
                                      c->m2, lr, 0.9f, 0.999f, 1e-8f, c1, c2));
        SLAQ_LAUNCHED();
    }
    return SLAQ_OK;
}

slaq_status slaq_closure_rules(const double* alpha, const double* beta, const int32_t* steps, int64_t count, int ms,
                               int mf, double* theta, double* tau2, double* theta_r, double* tau2_r, void* stream) {
    clear_error();
    SLAQ_REQUIRE(alpha && beta && steps && theta && tau2 && theta_r && tau2_r, SLAQ_ERR_INVALID_ARG, "NULL pointer");
    SLAQ_REQUIRE(count >= 1 && mf >= 1 && mf <= ms && ms <= SLAQ_MAX_STEPS, SLAQ_ERR_INVALID_ARG,
                 "need count >= 1 and 1 <= mf <= ms <= %d", SLAQ_MAX_STEPS);
    unsigned* const dstat = device_status_word();
    SLAQ_REQUIRE(dstat, SLAQ_ERR_HIP, "device status word unavailable");
    hipLaunchKernelGGL(probe_rules, dim3((unsigned)((count + 63) / 64)), dim3(64), 0, (hipStream_t)stream, count,
                       alpha, beta, steps, ms, mf, theta, tau2, theta_r, tau2_r, dstat);
    SLAQ_LAUNCHED();
    return SLAQ_OK;
}

slaq_status slaq_closure_features(const double* theta, const double* tau2, int64_t count, int mf, void* x,
                                  void* stream) {
    clear_error();
    SLAQ_REQUIRE(theta && tau2 && x && count >= 1 && mf >= 1 && 2 * mf <= kDinPad, SLAQ_ERR_INVALID_ARG,
                 "bad argument");
    hipLaunchKernelGGL(make_features, dim3((unsigned)((count * kDinPad + 255) / 256)), dim3(256), 0,
                       (hipStream_t)stream, count, mf, theta, tau2, (bf16*)x);
    SLAQ_LAUNCHED();
    return SLAQ_OK;
}

slaq_status slaq_closure_gauss_values(const double* theta, const double* tau2, int64_t count, int kn, int ks,
                                      const double* t, int nt, double* Q, void* stream) {
    clear_error();
    SLAQ_REQUIRE(theta && tau2 && t && Q && count >= 1 && kn >= 1 && ks >= kn && nt >= 1, SLAQ_ERR_INVALID_ARG,
                 "bad argument");
    hipLaunchKernelGGL(gauss_values, dim3((unsigned)((count * nt + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       count, kn, ks, theta, tau2, t, nt, Q);
    SLAQ_LAUNCHED();
    return SLAQ_OK;
}

slaq_status slaq_closure_targets(const double* q_hi, const double* q_lo, int64_t total, float* y, void* stream) {
    clear_error();
    SLAQ_REQUIRE(q_hi && q_lo && y && total >= 1, SLAQ_ERR_INVALID_ARG, "bad argument");
    hipLaunchKernelGGL(log_ratio, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, (hipStream_t)stream, total,
                       q_hi, q_lo, y);
    SLAQ_LAUNCHED();
    return SLAQ_OK;
}

slaq_status slaq_closure_apply(const float* yhat, const double* q5, const double* qr, int n_graphs, int nv, int nt,
                               const int64_t* graph_n, double tol, double* heat, int* flags, void* stream) {
    clear_error();
    SLAQ_REQUIRE(yhat && q5 && qr && graph_n && heat && flags && n_graphs >= 1 && nv >= 1 && nt >= 1,
                 SLAQ_ERR_INVALID_ARG, "bad argument");
    SLAQ_TIMED("closure_apply", (hipStream_t)stream,
               hipLaunchKernelGGL(closure_apply, dim3(n_graphs), dim3(256), 0, (hipStream_t)stream, n_graphs, nv, nt,
                                  yhat, q5, qr, graph_n, tol, heat, flags));
    SLAQ_LAUNCHED();
    return SLAQ_OK;
}

slaq_status slaq_hutchinson_mean(const double* q, int n_graphs, int nv, int nt, const int64_t* graph_n,
                                 double* heat, void* stream) {
    clear_error();
    SLAQ_REQUIRE(q && graph_n && heat, SLAQ_ERR_INVALID_ARG, "NULL pointer argument");
    SLAQ_REQUIRE(n_graphs >= 1 && nv >= 1 && nt >= 1, SLAQ_ERR_INVALID_ARG, "need n_graphs, nv, nt >= 1");
    hipLaunchKernelGGL(hutchinson_mean, dim3(n_graphs), dim3(256), 0, (hipStream_t)stream, nv, nt, q, graph_n, heat);
    SLAQ_LAUNCHED();
    return SLAQ_OK;
}

}  // extern "C"
