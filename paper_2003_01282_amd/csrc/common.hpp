// Internal helpers shared by the HIP sources of libslaq.so (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstddef>
#include <cstdint>
#include <cstdio>

#include "slaq.h"

namespace slaq {

// ---------------------------------------------------------------- errors ----
void set_error(const char* fmt, ...);
void clear_error();

#define SLAQ_REQUIRE(cond, code, ...)          \
    do {                                       \
        if (!(cond)) {                         \
            ::slaq::set_error(__VA_ARGS__);    \
            return (code);                     \
        }                                      \
    } while (0)

#define SLAQ_HIP(expr)                                                              \
    do {                                                                            \
        hipError_t e_ = (expr);                                                     \
        if (e_ != hipSuccess) {                                                     \
            ::slaq::set_error("%s failed: %s", #expr, hipGetErrorString(e_));       \
            return SLAQ_ERR_HIP;                                                    \
        }                                                                           \
    } while (0)

// launch-error check right after a <<<>>> launch
#define SLAQ_LAUNCHED() SLAQ_HIP(hipGetLastError())

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ----------------------------------------------------------- graph state ----
// Device-resident statistics written by the graph build (in caller scratch).
struct GraphStats {
    double trace;          // tr L: #non-isolated nodes, or sum_i D_ii
    double max_degree;     // max_i D_ii
    double sum_degree;     // sum_i D_ii
    long long n_isolated;  // #{i : D_ii = 0}
    unsigned int check;    // SLAQ_FLAG_CHECK findings (bit mask, see graph.hip)
    unsigned int pad;
};

constexpr int kBuildBlocks = 1024;  // grid of the degree kernel (partials size)

struct BuildPartial {
    double max_degree;
    double sum_degree;
    long long nonisolated;
    long long pad;
};

}  // namespace slaq

struct slaq_graph_s {
    int64_t n;
    int64_t nnz;
    const int64_t* row_ptr;
    const int32_t* col_idx;
    const float* weights;   // NULL = unweighted
    int laplacian;          // SLAQ_LAP_*
    float* diag;            // dinv (normalized) or degree (combinatorial)
    slaq::GraphStats* stats;
    slaq::BuildPartial* partials;
    hipStream_t stream;     // stream of the build (slaq_graph_info waits on it)
};

namespace slaq {

// ------------------------------------------------------- Lanczos layout ----
// Probe block row-major [n][ld], ld = nv rounded up to a multiple of 4 floats,
// so one node's probes are ld/4 float4 words.  Rows of degree >= kHeavyMin are
// split into aligned chunks of kChunk nonzeros whose partial products are
// computed by a separate kernel (bounded work per wave).
constexpr int kChunk = 128;
constexpr int kHeavyMin = 2 * kChunk;
constexpr int kSpmmBlock = 256;       // 4 waves
constexpr int kSpmmMaxBlocks = 2048;  // persistent grid of the SpMM kernel
constexpr int kQuadsPerTile = 64;     // float4 words per probe tile (256 probes)

inline int lanczos_ld(int nv) { return (nv + 3) / 4 * 4; }

}  // namespace slaq
