/*
 * slaq.h -- C ABI of libslaq.so, stochastic Lanczos quadrature (SLQ) of graph
 * Laplacian spectral functions on one AMD Instinct MI355X (gfx950).
 *
 * The method is SLaQ (Tsitsulin, Munkhoeva, Perozzi, "Just SLaQ When You
 * Approximate: Accurate Spectral Distances for Web-Scale Graphs", WWW 2020,
 * arXiv 2003.01282): tr f(L) is estimated by Hutchinson's estimator over nv
 * random probes (§3.1, eq. "trace"); each quadratic form v^T f(L) v by the
 * m-point Gauss rule whose nodes and weights are the eigenvalues of the
 * Lanczos tridiagonal T and the squared first components of its eigenvectors
 * (§3.1, eq. "quadratic"); the estimate is Gamma = n/nv sum_p sum_k
 * tau_pk^2 f(theta_pk) (§3.1, eq. "slq"; Algorithm 1).  The spectral
 * functions are the heat trace of NetLSD (§2.2, eq. "heat-trace"), its wave
 * counterpart, and the von Neumann graph entropy of §2.1.
 *
 * Conventions shared by every entry point
 *  - Every array argument is a DEVICE pointer owned by the caller (e.g. a
 *    torch tensor's storage).  The library never allocates, frees or keeps
 *    caller memory beyond the documented lifetime of a handle.
 *  - Every call is asynchronous and ordered on `stream` (a hipStream_t, NULL
 *    = the default stream); outputs are valid once that stream has reached
 *    the call.  Only slaq_graph_info and a build with SLAQ_FLAG_CHECK wait.
 *  - Argument errors detectable on the host (NULL pointers, sizes out of
 *    range, a workspace that is too small) return an error before anything
 *    is enqueued.  slaq_last_error() then describes it (thread-local).
 *  - No C++ exception crosses this boundary.
 *  - Graph layout: CSR of a symmetric adjacency matrix A with positive
 *    weights (§2): row_ptr int64[n+1] (row_ptr[0] = 0, non-decreasing,
 *    row_ptr[n] = nnz), col_idx int32[nnz] in [0, n), optional weights
 *    float[nnz] (NULL = every edge has weight 1).  Both directions of an
 *    undirected edge are stored, so nnz = 2|E| for a loop-free graph.
 *  - Probe vectors are FP32; alpha/beta reductions accumulate in FP64; the
 *    tridiagonal eigensolve and the quadrature are FP64.
 */
#ifndef SLAQ_H
#define SLAQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SLAQ_OK = 0,
    SLAQ_ERR_INVALID_ARG = 1,   /* NULL pointer, size out of range, bad enum */
    SLAQ_ERR_NOT_SYMMETRIC = 2, /* SLAQ_FLAG_CHECK found (i,j) without (j,i) */
    SLAQ_ERR_NUMERIC = 3,       /* weight <= 0 or not finite (SLAQ_FLAG_CHECK), or a
                                   device-detected problem (slaq_device_status) */
    SLAQ_ERR_WORKSPACE = 4,     /* workspace smaller than the size query says */
    SLAQ_ERR_HIP = 5,           /* a HIP runtime call failed */
    SLAQ_ERR_UNSUPPORTED = 6,   /* valid request the library does not serve */
    SLAQ_ERR_BAD_CSR = 7        /* SLAQ_FLAG_CHECK: row_ptr / col_idx malformed */
} slaq_status;

/* Which Laplacian (§2): L = I - D^-1/2 A D^-1/2 (isolated nodes get a zero row
 * and column, so they add eigenvalue 0), or L = D - A. */
enum { SLAQ_LAP_NORMALIZED = 0, SLAQ_LAP_COMBINATORIAL = 1 };

/* Which trace signature: heat h_t = tr exp(-tL) (§2.2, eq. "heat-trace"), or
 * wave w_t = Re tr exp(-itL) = sum_i cos(t lambda_i). */
enum { SLAQ_SIG_HEAT = 0, SLAQ_SIG_WAVE = 1 };

/* slaq_build_graph flags.  SLAQ_FLAG_RELABEL / SLAQ_FLAG_NO_RELABEL force
 * the internal node relabelling on or off (default: on from
 * SLAQ_RELABEL_MIN_NNZ stored entries up); setting both is an error. */
enum { SLAQ_FLAG_CHECK = 1u, SLAQ_FLAG_RELABEL = 2u, SLAQ_FLAG_NO_RELABEL = 4u };
enum { SLAQ_RELABEL_MIN_NNZ = 1 << 22 };

/* Precision of the Lanczos vectors (slaq_graph_set_precision).  The dot
 * products, alpha, beta and everything after them are FP64 either way. */
enum { SLAQ_PREC_FP32 = 0, SLAQ_PREC_FP64 = 1 };

/* Size limits of the library. */
enum { SLAQ_MAX_PROBES = 4096, SLAQ_MAX_STEPS = 64 };

typedef struct slaq_graph_s* slaq_graph_t;

/* Bytes of device scratch slaq_build_graph needs for a graph of n nodes and
 * nnz stored entries. */
slaq_status slaq_graph_scratch_bytes(int64_t n, int64_t nnz, size_t* bytes);

/* Degrees D_ii = sum_j A_ij, the diagonal scale of the Laplacian and the
 * graph statistics (§2; tr L per §2.1's density matrix).
 *   dinv_out  float[n], caller-owned: D_ii^-1/2 (0 for an isolated node) for
 *             the normalized Laplacian, D_ii for the combinatorial one.
 *   scratch   device memory of slaq_graph_scratch_bytes(); holds tr(L), the
 *             number of isolated nodes and max_i D_ii.
 * CSR: row_ptr int64[n+1] (row_ptr[0] = 0, non-decreasing, row_ptr[n] =
 * nnz), col_idx int32[nnz] in [0, n), each row's columns ascending without
 * repeats (the self-loop entry A_ii is found by binary search), weights
 * float[nnz] > 0 or NULL for 1; the pattern and weights symmetric.
 * The handle stores the pointers it was given: row_ptr, col_idx, weights,
 * dinv_out and scratch must stay valid and unchanged until
 * slaq_graph_destroy.  With SLAQ_FLAG_CHECK the call validates the CSR
 * (monotone row_ptr, columns in range, symmetric pattern and weights,
 * positive finite weights) and waits for the result.
 *
 * Relabelling (a storage order only; every result is a function of the
 * graph and the probes, which stay keyed by the caller's node ids): the
 * handle keeps its own copy of the CSR in scratch whose nodes are ordered by
 * decreasing row length (stable, i.e. ties in caller id order; rows are
 * bucketed exactly below 1024 entries and by 16 steps per octave above),
 * isolated nodes dropped, and rank r of the n_act non-isolated nodes placed
 * at label base(r mod 8) + r div 8 with base(x) = x q + min(x, n_act mod 8),
 * q = n_act div 8: each eighth of the label space holds every eighth node of
 * the degree order, so the eight column ranges of the row schedule carry
 * near-equal nonzero mass and each range stores its hot rows together.
 * Each relabelled row lists its entries range by range, in caller order
 * within a range.  Without relabelling the caller's CSR is used as is. */
slaq_status slaq_build_graph(int64_t n, int64_t nnz, const int64_t* row_ptr,
                             const int32_t* col_idx, const float* weights,
                             int laplacian, unsigned flags, float* dinv_out,
                             void* scratch, size_t scratch_bytes, void* stream,
                             slaq_graph_t* out);

/* Waits for the build (and any later work) on its stream and reports n, nnz,
 * tr(L) = sum_i L_ii (the number of non-isolated nodes, or sum_i D_ii, less
 * the self-loops' share A_ii / D_ii, or A_ii), the isolated-node count and
 * max D_ii.  Any output pointer may be NULL.  Returns SLAQ_ERR_NUMERIC (with
 * the outputs written) when the graph's last slaq_lanczos run produced a
 * non-finite coefficient (see slaq_device_status). */
slaq_status slaq_graph_info(slaq_graph_t g, int64_t* n, int64_t* nnz, double* trace,
                            int64_t* n_isolated, double* max_degree);

/* Row schedule of the SpMM.  Rows with at least heavy_min nonzeros are cut
 * at 8 column-label boundaries (relabelled: the range starts base(x); else
 * the first id whose row offset reaches nnz/8 * x, i.e. equal nnz mass) and
 * each part into pieces of at most `piece`
 * nonzeros that separate waves reduce in parallel; the pieces of column range
 * x run on workgroups b with b % 8 == x, i.e. one XCD, so that XCD's L2 holds
 * only that range's rows (defaults 128 and 128, or 32 and 64 for graphs of
 * fewer than SLAQ_RELABEL_MIN_NNZ stored entries; heavy_min >= 128, >= 32 for
 * those graphs, which is what their scratch is sized for; piece a multiple of
 * 64 and >= 64).  Setting it rebuilds the piece plan on `stream`; query
 * slaq_lanczos_workspace again afterwards, its size depends on the schedule.
 * slaq_graph_schedule reports the schedule and (waiting for the stream of the
 * build) the number of heavy rows and pieces; any pointer may be NULL. */
slaq_status slaq_graph_set_schedule(slaq_graph_t g, int heavy_min, int piece, void* stream);
slaq_status slaq_graph_schedule(slaq_graph_t g, int* heavy_min, int* piece, int64_t* n_heavy,
                                int64_t* n_pieces);

/* Probe tile of the gather kernels, in float4 words (4 probes): the SpMM
 * runs once per tile of the probe block, tiles one after another, so the
 * gathered rows of a tile stay in cache longer, at the price of visiting
 * every nonzero once per tile.  0 (default) = tiles of 64 words (256 probes).
 * Changes the workspace size. */
slaq_status slaq_graph_set_tile(slaq_graph_t g, int tile_quads);

/* Hot window of the SpMM gathers on a relabelled graph: the first `rows`
 * labels of each of the 8 column ranges (the range's highest-degree rows)
 * are gathered with ordinary loads, every other row, the column indices and
 * the piece partials with the non-temporal hint, so that the hottest probe
 * rows keep the last-level cache.  -1 (default) = automatic: the window whose
 * probe rows fill 200 MB (65,536 rows per range at nv = 100 in FP32).  A
 * window of at least n caches every gather; graphs that are not relabelled
 * always do.  Storage hints only: results are identical for every value. */
slaq_status slaq_graph_set_cache_rows(slaq_graph_t g, int64_t rows);
slaq_status slaq_graph_cache_rows(slaq_graph_t g, int64_t* rows);

/* Single-launch Lanczos (the recurrence of §3.1 with its m steps in one
 * kernel): one workgroup per CU at most, two device-wide barriers per step,
 * the per-probe sums formed in workgroup order by every workgroup.  For
 * graphs too small to fill the chip, where six launches per step cost more
 * than the work.  blocks: -1 (default) = automatic, used below 2^18 stored
 * entries with one workgroup per 80 rows (8 to 128); 0 = never; 1..256 =
 * that many workgroups (capped at the CU count and at what stays resident).  Applies to graphs kept in caller order with
 * at most 16 quads per probe row (nv <= 64 in FP32, 32 in FP64); otherwise,
 * and for any other setting, the stage kernels run.  The workgroups wait for
 * each other: they must all be resident at once, so no other work should
 * hold the device's CUs during the call (a wait that runs out sets
 * SLAQ_STATUS_GRID). */
slaq_status slaq_graph_set_fused(slaq_graph_t g, int blocks);

/* Gathers of the first Lanczos step (stage kernels).  The first basis block
 * is +-1 per probe times one scale per row (§3.1: Rademacher probes; X_1 =
 * D^-1/2 R_1 for the normalized Laplacian), so with on = 1 (the default) the
 * first step's SpMM reads a compact record per column (16-byte slots of the
 * row's sign bits and its scale, a power of two of them: one slot for up to
 * 96 probes in FP32 (64 in FP64), two for up to 192, ...; a gather loads the
 * one slot with its lane's probes) instead of its row of vector values, and
 * expands it in registers to the same values: results are bit-identical
 * either way.  The records live in the workspace's third
 * vector buffer, unused during the first step, so the workspace size does
 * not change.  on = 0 gathers the FP32 rows in every step. */
slaq_status slaq_graph_set_sign_step(slaq_graph_t g, int on);

/* Autotuner of the schedule above (row schedule heavy_min / piece, hot window,
 * single launch and its workgroups): none of these changes what §3.1's
 * recurrence computes, only where its work runs, so results differ at most by
 * rounding order.  Times each candidate with HIP events over `reps` Lanczos
 * runs after one untimed run (graphs of 2^22 stored entries and more on their
 * first 4 steps), searching coordinate-wise from the current settings, and
 * leaves the fastest set on the graph.  alpha, beta, steps and workspace are
 * the caller's slaq_lanczos buffers, used as scratch (overwritten); the
 * workspace should hold slaq_graph_autotune_workspace() bytes (a candidate
 * that needs more is skipped).  Waits for `stream`.  cache_path (NULL = no
 * cache): a JSON file mapping "<GPU arch>|<shape bucket>" (Laplacian,
 * precision, relabelling, padded nv, ceil(log2) of n and nnz) to the chosen
 * settings; a hit applies them without timing (*from_cache = 1), a miss tunes
 * and rewrites the file with the new entry.  A file that is not a cache is
 * an error (SLAQ_ERR_INVALID_ARG), as is one that cannot be written.
 * reps = 0: cache lookup only (a miss leaves the graph as it is). */
slaq_status slaq_graph_autotune(slaq_graph_t g, int nv, int m, uint64_t seed, double* alpha,
                                double* beta, int32_t* steps, void* workspace,
                                size_t workspace_bytes, int reps, const char* cache_path,
                                int* from_cache, void* stream);
slaq_status slaq_graph_autotune_workspace(slaq_graph_t g, int nv, int m, size_t* bytes);
/* The graph's current schedule settings (any output may be NULL). */
slaq_status slaq_graph_settings(slaq_graph_t g, int* heavy_min, int* piece, int64_t* cache_rows,
                                int* fused);

/* Precision of the Lanczos vectors of this graph.  Default: FP32 for the
 * normalized Laplacian (spectrum in [0, 2]; GPU and FP64 results agree to
 * ~1e-5 relative), FP64 for the combinatorial one, whose spectrum spans
 * [0, 2 max D_ii]: with hubs its top eigenvalues converge within a few steps
 * and FP32 vectors then lose orthogonality to them far sooner than FP64 ones
 * (no reorthogonalization, as in §3.1), which moves the low Ritz values and
 * VNGE by ~1e-4 relative.  FP64 doubles the vector traffic.  Changes the
 * workspace size (query slaq_lanczos_workspace again). */
slaq_status slaq_graph_set_precision(slaq_graph_t g, int precision);
slaq_status slaq_graph_precision(slaq_graph_t g, int* precision);

/* Internal storage order of the handle (waits for the build's stream).
 * relabeled: 1 if the handle relabelled its nodes; n_rows: rows of the
 * internal CSR (n_act when relabelled, else n).  perm (int32[n]), row_ptr
 * (int64[n + 1]) and col_idx (int32[nnz]) are caller device buffers that
 * receive the internal label -> caller id map (labels >= n_rows: the isolated
 * nodes in caller order; identity without relabelling) and the internal
 * CSR (rows >= n_rows empty).  Any pointer may be NULL. */
slaq_status slaq_graph_internal(slaq_graph_t g, int* relabeled, int64_t* n_rows, int32_t* perm,
                                int64_t* row_ptr, int32_t* col_idx);

/* Variance reduction of the trace estimate (§3.1, last paragraph: a "2-term
 * polynomial variance reduction"; the paper gives no formula).  The two terms
 * are control variates with exact means: Z1_p = n q_p^T L q_p (mean tr L) and
 * Z2_p = n q_p^T L^2 q_p (mean tr L^2), which the Gauss rule of each probe
 * gives exactly for m >= 2 as n sum_k tau2 theta and n sum_k tau2 theta^2.
 * With X_p = n sum_k tau2 f(theta) the estimate is
 *   mean(X) - g1 (mean(Z1) - tr L) - g2 (mean(Z2) - tr L^2).
 * SLAQ_CV_NONE: g = 0 (plain SLQ).  SLAQ_CV_TAYLOR: the degree-2 Taylor
 * polynomial of f at 0 (heat (-t, t^2/2), wave (0, -t^2/2), VNGE (1/c, -1/c^2)
 * from -x ln x ~ x - x^2 on x = lambda / c): unbiased, for small t only
 * (its coefficients grow like t^2 and multiply the probes' spread of Z2).
 * SLAQ_CV_FITTED: least-squares regression of X on (Z1, Z2) over the probes
 * (bias O(1/nv)); fewer than 3 probes or no spread in Z1 -> plain; 3 probes,
 * no spread in Z2 or a 2x2 system with det <= 1e-10 S11 S22 -> Z1 alone. */
enum { SLAQ_CV_NONE = 0, SLAQ_CV_TAYLOR = 1, SLAQ_CV_FITTED = 2 };

/* tr L and tr L^2 = sum_ij L_ij^2 of the graph's Laplacian (§2), FP64, into
 * traces[0..1] (device), one O(nnz) pass on `stream` (self-loops taken
 * literally; isolated nodes have zero rows).  Uses the handle's scratch:
 * calls on one graph must not overlap. */
slaq_status slaq_graph_traces(slaq_graph_t g, double* traces, void* stream);

/* Variance-reduced heat / wave trace at nt times (as slaq_signature, plus the
 * device traces[2] of slaq_graph_traces and a SLAQ_CV_* mode). */
slaq_status slaq_signature_cv(const double* theta, const double* tau2, int nv, int m, int64_t n,
                              const double* traces, const double* t, int nt, int kind, int mode,
                              double* out, void* stream);

/* Variance-reduced VNGE (as slaq_vnge, c = the graph's tr L of §2.1). */
slaq_status slaq_vnge_cv(slaq_graph_t g, const double* theta, const double* tau2, int nv, int m,
                         const double* traces, int mode, double* out, void* stream);

/* Frees the host handle (never caller memory). */
slaq_status slaq_graph_destroy(slaq_graph_t g);

/* Bytes of device workspace slaq_lanczos needs for nv probes. */
slaq_status slaq_lanczos_workspace(slaq_graph_t g, int nv, int m, size_t* bytes);

/* m steps of the Lanczos three-term recurrence (§3.1) on nv Rademacher probes
 * at once, without reorthogonalization.  Probe p's start vector is
 * q1[i] = v[i,p] / sqrt(n) with v[i,p] = +-1 given by bit (p mod 64) of
 * SplitMix64 output number 64*i + (p div 64) + 1 for `seed` (a set bit gives
 * -1), so q1 has unit norm (§3.1's "starting unit-vector").  Per probe and
 * step j = 1..m:
 *     w = L q_j - beta_{j-1} q_{j-1};  alpha_j = q_j . w;
 *     beta_j = || w - alpha_j q_j ||;   q_{j+1} = (w - alpha_j q_j) / beta_j.
 * Outputs (device, caller-owned, row-major by probe):
 *   alpha, beta  double[nv*m]: T_p = tridiag(beta, alpha, beta); beta[p*m+j-1]
 *                couples q_j and q_{j+1} (the last one is kept).
 *   steps        int32[nv]: Lanczos steps taken; < m when the Krylov space of
 *                the probe became invariant (beta_j <= 1e-6 * spectral bound,
 *                i.e. 2 or 2 max D_ii); entries past steps[p] are 0.  This is
 *                not an error.
 * workspace: device memory of slaq_lanczos_workspace() bytes; 1 <= nv <=
 * SLAQ_MAX_PROBES, 1 <= m <= SLAQ_MAX_STEPS.  Isolated nodes (zero rows of L)
 * are not stored in the workspace: on them every Lanczos vector is a multiple
 * of the probe, carried as an FP64 scalar per probe. */
slaq_status slaq_lanczos(slaq_graph_t g, int nv, int m, uint64_t seed, double* alpha,
                         double* beta, int32_t* steps, void* workspace,
                         size_t workspace_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): slaq_lanczos
 * with its workspace taken from a library-owned device array of
 * SLAQ_NOALLOC_WORKSPACE_BYTES (64 MiB) per GPU, held until the process ends.
 * Same arguments, kernels and results as slaq_lanczos (bit for bit).  Returns
 * SLAQ_ERR_WORKSPACE, with nothing enqueued, when slaq_lanczos_workspace()
 * for this graph and nv exceeds that size.  Calls no allocating routine
 * (with slaq_profile_enable on, the stage timer creates HIP events).  All calls on one GPU share the array:
 * calls that overlap on a GPU (other streams, other threads) race, so the
 * caller orders them. */
#define SLAQ_NOALLOC_WORKSPACE_BYTES (64u << 20)
slaq_status slaq_lanczos_noalloc(slaq_graph_t g, int nv, int m, uint64_t seed, double* alpha,
                                 double* beta, int32_t* steps, void* stream);

/* Gauss nodes and weights (§3.1, eq. "quadratic"): theta[p*m+k] are the
 * eigenvalues of T_p (size steps[p]) and tau2[p*m+k] the squared first
 * components of its normalized eigenvectors; entries k >= steps[p] are 0.
 * FP64 implicit-shift QR per probe; nv may be any count of independent
 * probes (nv * m < 2^31), e.g. the probes of many graphs at once. */
slaq_status slaq_ritz(const double* alpha, const double* beta, const int32_t* steps,
                      int nv, int m, double* theta, double* tau2, void* stream);

/* Trace signature Gamma_f = n/nv sum_p sum_k tau2 f(theta) (§3.1, eq. "slq")
 * at the nt time scales t[0..nt) (device double[nt]) for f = exp(-t x)
 * (SLAQ_SIG_HEAT) or cos(t x) (SLAQ_SIG_WAVE); out double[nt]. */
slaq_status slaq_signature(const double* theta, const double* tau2, int nv, int m,
                           int64_t n, const double* t, int nt, int kind, double* out,
                           void* stream);

/* Von Neumann graph entropy H = -tr g(L / tr L), g(x) = x ln x (0 for x <= 0)
 * (§2.1 Definition; Algorithm 1's SLaQ_VNGE), estimated as
 * -n/nv sum_p sum_k tau2 g(theta / tr L) with n and tr L taken from the graph
 * (on the device, no wait); out double[1]. */
slaq_status slaq_vnge(slaq_graph_t g, const double* theta, const double* tau2, int nv,
                      int m, double* out, void* stream);

/* Algorithm 1 from the Lanczos coefficients: SLaQ_LSD and SLaQ_VNGE with the
 * eigensolve inside.  slaq_lsd takes alpha, beta, steps as slaq_lanczos
 * writes them (device, [nv*m], [nv*m], [nv]), solves each T_p (FP64
 * implicit QR, eq. "quadratic") and writes Gamma_f = n/nv sum_p sum_k
 * tau2 f(theta) (eq. "slq") for f = exp(-t x) or cos(t x) at the nt times
 * t[0..nt) into out double[nt]; slaq_vnge_slq writes -n/nv sum tau2
 * g(theta / trace), g(x) = x ln x (0 for x <= 0), into out double[1], with
 * the caller's trace = tr L (0 gives 0).  No workspace: every block of
 * slaq_lsd re-solves the nv tridiagonals for its 32 times (callers that
 * reuse the Gauss rules call slaq_ritz once and slaq_signature / slaq_vnge).
 * 1 <= nv <= SLAQ_MAX_PROBES, 1 <= m <= SLAQ_MAX_STEPS, 1 <= nt <= 65535. */
slaq_status slaq_lsd(const double* alpha, const double* beta, const int32_t* steps, int nv, int m, int64_t n,
                     const double* t, int nt, int kind, double* out, void* stream);
slaq_status slaq_vnge_slq(const double* alpha, const double* beta, const int32_t* steps, int nv, int m,
                          int64_t n, double trace, double* out, void* stream);

/* ---- Batched SLQ over many graphs -------------------------------------
 * A batch is the block-diagonal union of G graphs: node_off[g] .. node_off[g+1]
 * are graph g's nodes, row_ptr / col_idx its CSR rows with GLOBAL column ids
 * (each row's columns lie inside its own graph).  Graph g uses the probes of
 * slaq_lanczos with seed + g on that graph alone (keys are graph-local node
 * ids), so each output row equals the plain path on the graph by itself, up
 * to summation order.  Normalized Laplacian; nv <= 256; fewer than 2^31
 * nodes in the whole batch.  Graphs whose probe block (n ceil(nv/4) 16 bytes)
 * fits in 64 KB are bucketed by node count and keep it in LDS; all larger
 * graphs form one more bucket that runs the same per-graph Lanczos with the
 * probe blocks in a global workspace: one slot of 3 (n_max + 1) ceil(nv/4)
 * 16 + 4 n_max bytes per workgroup its launch keeps resident, at most 16 GB
 * (slaq_batch_workspace; the caller's via slaq_batch_set_workspace, else
 * allocated by the first run and freed by slaq_batch_destroy).
 *
 * slaq_batch_plan (host): node_off and nnz_off are HOST copies of the node
 * offsets and of row_ptr at the graph starts (G+1 entries each);
 * node_off_dev / row_ptr / col_idx are the device arrays, which must stay
 * valid until slaq_batch_destroy.  Graphs are bucketed by node count
 * (<= 64, 128, 256, ... up to the LDS limit, then the global bucket);
 * bucket_blocks (optional, n_buckets_cfg entries)
 * overrides each bucket's workgroup size; G nv m must stay below 2^31.  The
 * plan owns device memory until slaq_batch_destroy: the graph order, work
 * counters, and result buffers for whatever the caller does not ask for
 * (alpha, beta, theta, tau2: 32 G nv m bytes; steps; tr L per graph).
 *
 * slaq_batch_run enqueues one persistent launch per bucket on `stream`; each
 * workgroup pulls graphs, most expensive first, and computes degrees, probes
 * and m Lanczos steps; then the FP64 Gauss rules of all G nv probes
 * (slaq_ritz) and, per graph, the requested outputs (any may be NULL): heat
 * double[G][nt] (n_g/nv sum tau2 exp(-t theta)), vnge double[G], alpha,
 * beta, theta, tau2 double[G][nv][m], steps int32[G][nv].  With
 * SLAQ_BATCH_GRAPH the launches are captured once into a hipGraph and
 * replayed (re-captured when a buffer pointer or the seed changes).  Runs
 * that overlap on one plan race on its buffers.
 *
 * slaq_batch_buckets reports the bucket count and, per bucket (arrays of
 * n_buckets entries, any may be NULL), its largest node count, workgroup
 * size, graph count and whether its probe blocks live in LDS (1) or in the
 * global workspace (0).
 *
 * slaq_batch_autotune times every workgroup size in {128, 256, 512, 1024}
 * per bucket (median of reps runs, HIP events) and keeps the fastest; the
 * chosen sizes are returned in blocks_out[n_buckets] (optional).
 *
 * slaq_batch_plan_grown is slaq_batch_plan with the LDS buckets' node-count
 * edges growing by `growth` (in [1.25, 8]; slaq_batch_plan uses 2: 64, 128,
 * 256, ...).  slaq_batch_autotune_edges plans the batch with growth 2, 1.5
 * and 3, autotunes each plan's workgroup sizes, times `reps` full runs of it
 * (heat at the nt times of t and VNGE, after one untimed run; HIP events,
 * median) and returns the fastest plan in *out (the others are destroyed),
 * its growth and time.  It allocates and frees its own output buffers and
 * waits for `stream`. */
enum { SLAQ_BATCH_GRAPH = 1u };
typedef struct slaq_batch_s* slaq_batch_t;
slaq_status slaq_batch_plan(int64_t n_graphs, const int64_t* node_off, const int64_t* nnz_off,
                            const int64_t* node_off_dev, const int64_t* row_ptr,
                            const int32_t* col_idx, int nv, int m, int nt,
                            const int* bucket_blocks, int n_buckets_cfg, slaq_batch_t* out);
/* First step of the global-workspace buckets (graphs whose probe block does
 * not fit in LDS): with on = 1 (the default) its gathers read a record per
 * column (16-byte slots of the Rademacher sign bits of §3.1's probes and the
 * row's D^-1/2, one slot for up to 96 probes) instead of the row of X_1,
 * expanded in registers to the same values; results are bit-identical
 * either way.  The records use the
 * workspace's previous-vector buffer, which the first step does not read.
 * A captured hipGraph of the plan is dropped when the setting changes. */
slaq_status slaq_batch_set_sign_step(slaq_batch_t b, int on);
slaq_status slaq_batch_plan_grown(int64_t n_graphs, const int64_t* node_off, const int64_t* nnz_off,
                                  const int64_t* node_off_dev, const int64_t* row_ptr,
                                  const int32_t* col_idx, int nv, int m, int nt, double growth,
                                  const int* bucket_blocks, int n_buckets_cfg, slaq_batch_t* out);
slaq_status slaq_batch_autotune_edges(int64_t n_graphs, const int64_t* node_off, const int64_t* nnz_off,
                                      const int64_t* node_off_dev, const int64_t* row_ptr,
                                      const int32_t* col_idx, int nv, int m, int nt, const double* t,
                                      int reps, double* growth_out, float* ms_out, slaq_batch_t* out,
                                      void* stream);
slaq_status slaq_batch_buckets(slaq_batch_t b, int* n_buckets, int* n_hi, int* blocks, int* graphs,
                               int* in_lds);
slaq_status slaq_batch_run(slaq_batch_t b, uint64_t seed, const double* t, double* heat, double* vnge,
                           double* alpha, double* beta, int32_t* steps, double* theta, double* tau2,
                           unsigned flags, void* stream);
slaq_status slaq_batch_autotune(slaq_batch_t b, const double* t, double* heat, double* vnge, int reps,
                                int* blocks_out, float* best_ms_out, void* stream);
/* Workspace of the global bucket: slaq_batch_workspace gives its size in
 * bytes (0 when every graph runs in LDS); slaq_batch_set_workspace hands the
 * plan caller-owned device memory of at least that size (256-byte aligned,
 * valid for every later run; NULL returns to the plan's own), so that a
 * caller who builds many plans can keep one buffer instead of allocating per
 * plan.  A plan's runs use it in turn: runs that overlap on one workspace
 * race. */
slaq_status slaq_batch_workspace(slaq_batch_t b, size_t* bytes);
slaq_status slaq_batch_set_workspace(slaq_batch_t b, void* workspace, size_t bytes);
/* Per-graph probe seeds: with seeds (device uint64[G], caller-owned, valid for
 * every later run) graph g uses the probes of slaq_lanczos with seeds[g]
 * instead of seed + g; NULL restores seed + g.  Lets a batch of selected
 * graphs reuse the probes they had in another batch. */
slaq_status slaq_batch_set_seeds(slaq_batch_t b, const uint64_t* seeds);
slaq_status slaq_batch_destroy(slaq_batch_t b);

/* ---- Learned closure (an addition to the paper's method) ----------------
 * An MLP d_in (<= 32, zero-padded to 32) -> hidden -> hidden -> hidden -> nt
 * with SiLU activations, trained with MSE and Adam on FP32 master weights;
 * every matrix product is a BF16 MFMA (v_mfma_f32_16x16x32_bf16) with FP32
 * accumulation.  It maps a probe's mf-step Gauss rule (features: nodes
 * ascending, then weights) to y(t) = log Q_30(t) - log Q_mf(t), where
 * Q_m(t) = sum_k tau2_k exp(-t theta_k) is the probe's m-point Gauss value of
 * exp(-tL) (§3.1, eq. "quadratic").  The handle owns its parameters (device
 * memory, freed by slaq_closure_destroy); batch activations live in a
 * caller workspace of slaq_closure_workspace() bytes.  Not thread-safe per
 * handle.
 *
 * create: Glorot-uniform init from SplitMix64(seed); info: parameter count,
 * offsets of W1 b1 W2 b2 W3 b3 W4 b4 in the FP32 parameter vector
 * (W row-major d_in x d_out), layer widths.  get (which 0 = weights, 1 =
 * gradients of the last train_step, 2 / 3 = Adam first / second moments) /
 * set copy such a vector device-to-device (set: the weights, optionally
 * zeroing the optimizer state).  get_step: the number of Adam steps taken
 * (host int, no device work).  set_optimizer: restores the Adam moments and
 * the step count, so that a handle given a checkpoint's weights (set with
 * reset_optimizer = 0) and optimizer state continues training exactly as the
 * handle it was taken from.
 * train_step: x BF16 [batch][32], y FP32 [batch][nt]; writes the gradients,
 * the loss (device float, optional) and, when lr > 0, one Adam step.
 * forward: y_hat FP32 [batch][nt].
 * rules: from Lanczos coefficients (row stride ms, steps) the mf-node Gauss
 * rule (theta, tau2 [count][mf], ascending) and the (mf+1)-node Gauss-Radau
 * rule with a node at 0 (theta_r, tau2_r [count][mf+1]); for exp(-tx) they
 * bracket the exact quadratic form from below and above.
 * features: BF16 x [count][32] from an mf-node rule.
 * gauss_values: Q[count][nt] from the first kn of ks nodes per probe.
 * targets: y = log(q_hi) - log(q_lo) elementwise (FP32).
 * apply: per probe Q_hat = q5 exp(y_hat) clamped to [q5, qr]; heat[g][t] =
 * graph_n[g]/nv sum over the graph's nv probes; flags[g] = 1 when at some t
 * the graph's bracket is wider than tol (relative) and clamping moved the
 * graph's heat by more than tol - such graphs are to be recomputed by plain
 * SLQ (tol < 0 flags every graph). */
typedef struct slaq_closure_s* slaq_closure_t;
slaq_status slaq_closure_create(int d_in, int hidden, int nt, uint64_t seed, void* stream, slaq_closure_t* out);
slaq_status slaq_closure_destroy(slaq_closure_t c);
slaq_status slaq_closure_info(slaq_closure_t c, int64_t* n_params, int64_t* offsets, int* dims);
slaq_status slaq_closure_workspace(slaq_closure_t c, int64_t batch, size_t* bytes);
slaq_status slaq_closure_get(slaq_closure_t c, int which, float* dst, void* stream);
slaq_status slaq_closure_set(slaq_closure_t c, const float* src, int reset_optimizer, void* stream);
slaq_status slaq_closure_get_step(slaq_closure_t c, int* step);
slaq_status slaq_closure_set_optimizer(slaq_closure_t c, const float* m1, const float* m2, int step, void* stream);
slaq_status slaq_closure_forward(slaq_closure_t c, const void* x, int64_t batch, float* yhat, void* workspace,
                                 size_t ws_bytes, void* stream);
slaq_status slaq_closure_train_step(slaq_closure_t c, const void* x, const float* y, int64_t batch, float lr,
                                    float* loss, void* workspace, size_t ws_bytes, void* stream);
slaq_status slaq_closure_rules(const double* alpha, const double* beta, const int32_t* steps, int64_t count,
                               int ms, int mf, double* theta, double* tau2, double* theta_r, double* tau2_r,
                               void* stream);
slaq_status slaq_closure_features(const double* theta, const double* tau2, int64_t count, int mf, void* x,
                                  void* stream);
slaq_status slaq_closure_gauss_values(const double* theta, const double* tau2, int64_t count, int kn, int ks,
                                      const double* t, int nt, double* Q, void* stream);
slaq_status slaq_closure_targets(const double* q_hi, const double* q_lo, int64_t total, float* y, void* stream);
slaq_status slaq_closure_apply(const float* yhat, const double* q5, const double* qr, int n_graphs, int nv, int nt,
                               const int64_t* graph_n, double tol, double* heat, int* flags, void* stream);
/* Hutchinson's estimate (§3.1, eq. "trace") from per-probe quadratic forms:
 * heat[g][b] = graph_n[g] / nv sum_p q[g nv + p][b] (probes in order), for
 * q double[n_graphs nv][nt] (e.g. slaq_closure_gauss_values of the plain
 * Gauss rules), graph_n int64[n_graphs], heat double[n_graphs][nt]. */
slaq_status slaq_hutchinson_mean(const double* q, int n_graphs, int nv, int nt, const int64_t* graph_n,
                                 double* heat, void* stream);

/* Stage timing with HIP events (off by default).  While enabled, every launch
 * of a stage kernel ("spmm_pieces", "spmm_rows", "spmm_heavy", "finalize",
 * "update", "batch_slq", "mlp_fwd", "mlp_bwd", "mlp_adam", "closure_apply")
 * is bracketed by two events on its stream; launches captured into a hipGraph
 * are not timed (replays of the graph neither).  slaq_profile_read waits for
 * the recorded events of `kernel` and returns how many launches were recorded
 * and their summed duration in milliseconds; slaq_profile_reset drops the
 * records.  Intended for benchmarks: recording adds two event records per
 * launch. */
slaq_status slaq_profile_enable(int on);
slaq_status slaq_profile_reset(void);
slaq_status slaq_profile_read(const char* kernel, int64_t* launches, double* total_ms);

/* Device-detected numeric problems.  Kernels that find a non-finite Lanczos
 * coefficient alpha_j or beta_j (§3.1's recurrence; e.g. from a NaN weight
 * built without SLAQ_FLAG_CHECK) set SLAQ_STATUS_NONFINITE; a tridiagonal
 * eigensolve of the Gauss rule (§3.1, eq. "quadratic"; Algorithm 1's eigh)
 * that reaches its sweep cap (60 k implicit QR sweeps for a k x k matrix,
 * which only non-finite input reaches in practice) sets
 * SLAQ_STATUS_NO_CONVERGENCE.  The bits of a graph's last slaq_lanczos run
 * make slaq_graph_info return SLAQ_ERR_NUMERIC (its outputs are still
 * written).  Every kernel also ORs its bits into one status word per device:
 * slaq_device_status waits for `stream`, returns the word in *bits (may be
 * NULL), clears it when clear != 0, and returns SLAQ_ERR_NUMERIC when it was
 * non-zero.  Work on other streams of the device is not waited for.
 * SLAQ_STATUS_GRID: a single-launch Lanczos run (slaq_graph_set_fused) found
 * its workgroups not all resident at once and stopped early; its outputs are
 * incomplete. */
enum { SLAQ_STATUS_NONFINITE = 1u, SLAQ_STATUS_NO_CONVERGENCE = 2u, SLAQ_STATUS_GRID = 4u };
slaq_status slaq_device_status(unsigned* bits, int clear, void* stream);

/* Thread-local description of the last non-OK status ("" if none). */
const char* slaq_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SLAQ_H */
