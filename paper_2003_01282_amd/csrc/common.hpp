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

// returns a non-OK status of a library call to the caller
#define SLAQ_TRY(x)                   \
    do {                              \
        const slaq_status s_ = (x);   \
        if (s_ != SLAQ_OK) return s_; \
    } while (0)

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

// launch-error check right after a launch
#define SLAQ_LAUNCHED() SLAQ_HIP(hipGetLastError())

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ----------------------------------------------------------- graph state ----
// Device-resident statistics written by the graph build (in caller scratch).
struct GraphStats {
    double trace;          // tr L: #non-isolated nodes, or sum_i D_ii
    double max_degree;     // max_i D_ii
    double sum_degree;     // sum_i D_ii
    long long n_isolated;  // #{i : D_ii = 0}
    long long n_heavy;     // rows split into pieces (degree >= heavy_min)
    long long n_pieces;    // total pieces of the heavy rows
    long long n_rows;      // rows of the internal CSR (n_act when relabelled, else n)
    unsigned int check;    // SLAQ_FLAG_CHECK findings (bit mask, see graph.hip)
    unsigned int status;   // SLAQ_STATUS_* bits of this graph's Lanczos runs
};

// Address of the current device's status word (SLAQ_STATUS_* bits), or NULL
// if the runtime cannot give it.  Kernels OR into it with raise_status.
unsigned* device_status_word();

__device__ __forceinline__ void raise_status(unsigned* word, unsigned bits) {
    if (word) atomicOr(word, bits);
}

constexpr int kBuildBlocks = 1024;  // grid of the degree kernel (partials size)
constexpr int kPlanBlock = 256;     // rows per block of the plan kernels

struct BuildPartial {
    double max_degree;
    double sum_degree;
    long long nonisolated;
    long long pad;
};

// Bytes of the last-level (Infinity) cache the automatic hot window fills with
// the hottest probe rows (of 256 MB; the rest holds tails, indices and the
// streamed vectors).
constexpr size_t kCacheBudget = (size_t)200 << 20;

// Grid of the self-loop pass of the build (one FP64 partial per block).
constexpr int kLoopBlocks = 4096;

// Row schedule of the SpMM: rows of degree >= heavy_min are cut into pieces of
// at most `piece` nonzeros (a piece never crosses a row).  heavy_min and piece
// are tunable (slaq_graph_set_schedule); these are the defaults and bounds.
constexpr int kDefaultHeavyMin = 128;
constexpr int kDefaultPiece = 128;
// below SLAQ_RELABEL_MIN_NNZ stored entries the SpMM does not fill the chip and
// its time is the serial gather chain of the longest light row: shorter light
// rows, more pieces (Chung-Lu 10^4: 1.39 -> 0.96 ms per step)
constexpr int kSmallHeavyMin = 32;
constexpr int kSmallPiece = 64;
// lowest heavy_min a schedule may set: it sizes the heavy-row scratch
// (nnz / bound rows), so small graphs get the low bound they default to and
// large ones keep their scratch at nnz / 128
constexpr int kMinHeavyMin = 128;
inline int heavy_min_bound(int64_t nnz) {
    return nnz < (int64_t)SLAQ_RELABEL_MIN_NNZ ? kSmallHeavyMin : kMinHeavyMin;
}
constexpr int kMinPiece = 64;
// Heavy rows are also cut at kColRanges column-id boundaries of equal nnz
// mass; the pieces of range x are reduced by workgroups b with b % 8 == x,
// i.e. on one XCD, whose L2 then holds only that range's hot rows.
constexpr int kColRanges = 8;

// Relabelling: nodes are counting-sorted by row-length bucket (exact below
// 1024, 16 buckets per octave above; lengths < 2^31), in chunks of
// kSortChunk caller ids per workgroup.
constexpr int kDegBuckets = 1024 + 16 * 21;

// Partial sums of slaq_graph_traces (two doubles per workgroup).
constexpr int kTraceBlocks = 1024;
constexpr int kSortChunk = 4096;

}  // namespace slaq

struct slaq_graph_s {
    int64_t n;
    int64_t nnz;
    // internal CSR the kernels read: the caller's, or its relabelled copy in scratch
    const int64_t* row_ptr;
    const int32_t* col_idx;
    const float* weights;   // NULL = unweighted
    int laplacian;          // SLAQ_LAP_*
    float* diag;            // per internal row: dinv (normalized) or degree (combinatorial); 0 <=> no data
    double* diag64;         // the same in FP64 (read by the FP64-vector kernels)
    const int32_t* perm;    // internal label -> caller id (NULL = identity)
    int relabeled;
    float* dinv_out;        // caller's diagonal scale, caller order
    slaq::GraphStats* stats;
    slaq::BuildPartial* partials;
    long long* blockcounts;  // [nplan] heavy rows, pieces per plan block, then offsets
    int32_t* hrow;           // heavy row ids, increasing
    int64_t* hoff;           // (row-major piece offsets; kept for the counts)
    int64_t* bounds;         // [kColRanges + 1] column-id boundaries of equal nnz mass
    int64_t* segk;           // [(kColRanges + 1) * max_heavy]: first nonzero of range x in heavy row h
    int64_t* segoff;         // [kColRanges * max_heavy + 1]: first piece of (x, h), x-major
    long long* segcnt;       // [kColRanges * max_heavy] pieces of (x, h) before the scan
    long long* scanbuf;      // block sums of the segment scan
    double* trace_part;      // [2 * kTraceBlocks] partials of slaq_graph_traces
    int64_t max_heavy;       // capacity of hrow / hoff / segk (stride of the x-major arrays)
    int heavy_min;
    int piece;
    int tile_quads;          // probe tile of the gather kernels in 16-byte words (0 = automatic)
    int64_t cache_rows;      // hot window of the gathers, rows per column range (-1 = automatic)
    int fused;               // single-launch Lanczos: -1 automatic, 0 never, > 0 that many workgroups
    int sign_step;           // first step's gathers from the compact sign records (1) or the rows (0)
    int precision;           // SLAQ_PREC_* of the Lanczos vectors
    hipStream_t stream;      // stream of the build (slaq_graph_info waits on it)
};

namespace slaq {

// Builds (or rebuilds) the heavy-row plan of g on `st` with its heavy_min/piece.
slaq_status build_plan(slaq_graph_s* g, hipStream_t st);

// Exclusive scan of in[0, len) into out (fixed-order, blocks of 1024);
// bsum holds ceil(len / 1024) partials.  The total goes to *total_a and
// *total_b when they are non-NULL.
slaq_status exclusive_scan(const long long* in, int64_t len, int64_t* out, long long* bsum, long long* total_a,
                           int64_t* total_b, hipStream_t st);

// Scratch arrays of the relabelled CSR (see relabel.hip).
struct RelabelBuffers {
    int32_t* perm;       // [n] label -> caller id
    int32_t* inv;        // [n] caller id -> label
    int64_t* row_ptr;    // [n + 1]
    int32_t* col;        // [nnz]
    float* w;            // [nnz]
    int32_t* tmp;        // [nnz] labels of long rows in caller order
    float* diag;         // [n]
    double* diag64;      // [n]
    long long* len;      // [n + 1] row lengths before the scan
    long long* sort_cnt; // [kDegBuckets * chunks]
    int64_t* sort_off;   // [kDegBuckets * chunks]
    long long* bsum;     // scan partials
    int64_t* chunk_off;  // [n + 1] first chunk of each long row
    int32_t* ccnt;       // [max_chunks * 8] entries per (chunk, range)
    int32_t* coff;       // [max_chunks * 8] first position per (chunk, range) within the row
};

// Upper bound of the chunks the relabelling cuts long rows into.
inline int64_t relabel_max_chunks(int64_t nnz) { return nnz / 256 + nnz / 1024 + 1; }

// Relabels the caller's CSR into B (sets st->n_rows and the range bounds).
slaq_status relabel_build(const RelabelBuffers& B, int64_t n, const int64_t* rp, const int32_t* col,
                          const float* w, const float* diag_caller, const double* diag64_caller, GraphStats* st,
                          int64_t* bounds, hipStream_t stream);

// ------------------------------------------------------- Lanczos layout ----
// Vector blocks are row-major [n][ld], ld = nv rounded up to a multiple of 4
// floats, so one node's probes are ld/4 float4 words ("quads").  A wave splits
// into K = 64/G groups of G = min(ld/4, 64) lanes; one group covers one node's
// quads of a probe tile (64 quads = 256 probes).
constexpr int kQuadsPerTile = 64;
constexpr int kSpmmBlock = 256;       // 4 waves
// Rows a wave takes per window of the light-row and update kernels (at least
// one per group: the layout raises it to K).  Small windows balance the
// waves: relabelled rows of similar cost sit next to each other, so wide
// windows hand some waves far more work (R-MAT 22: 64 rows 2.87 ms, 8 rows
// 2.41 ms, 2 rows 2.35 ms for the light-row kernel).
constexpr int kRowsPerWindow = 2;

inline int lanczos_ld(int nv) { return (nv + 3) / 4 * 4; }

}  // namespace slaq
