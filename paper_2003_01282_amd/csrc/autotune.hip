// Schedule autotuner of the plain Lanczos path, with a tuning cache.
//
// The schedule is everything that changes where and how the recurrence's
// SpMM runs but not what it computes: the heavy-row threshold and piece size
// of the row schedule, the hot window of the gathers on a relabelled graph,
// and, on graphs small enough for it, the single launch and its workgroup
// count.  A candidate is timed with HIP events around `reps` Lanczos runs
// (after one untimed run) on the caller's graph, probes and buffers; large
// graphs are timed on the first few steps only (every step costs the same).
// The search is coordinate-wise: row schedule first, then the hot window, or
// single launch versus stage kernels on small graphs.
//
// Cache: a JSON object whose keys are "<GPU arch>|<shape bucket>" and whose
// values hold the chosen settings, e.g.
//   {"gfx950:sramecc+:xnack-|lap0-prec0-rel1-ld100-n26-nnz31":
//    {"heavy_min": 128, "piece": 128, "cache_rows": -1, "fused": 0, "ms": 352.1}}
// The shape bucket is the Laplacian kind, vector precision, relabelling,
// padded probe count and ceil(log2) of n and of the stored entries.  The file
// is read and rewritten whole (a reader that finds no entry, or no file, tunes
// and adds one); the library writes only the entries it tunes.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "common.hpp"
#include "tuning_cache.hpp"

namespace slaq {

namespace {

struct Setting {
    int heavy_min, piece, fused;
    int64_t cache_rows;
    double ms;
};

int ceil_log2(int64_t x) {
    int k = 0;
    while (((int64_t)1 << k) < x) ++k;
    return k;
}

std::string arch_name() {
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    return std::string(p.gcnArchName);
}

std::string shape_key(const slaq_graph_s* g, int nv) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "lap%d-prec%d-rel%d-ld%d-n%d-nnz%d", g->laplacian, g->precision, g->relabeled,
                  lanczos_ld(nv), ceil_log2(g->n), ceil_log2(g->nnz > 0 ? g->nnz : 1));
    return buf;
}

slaq_status apply(slaq_graph_t g, const Setting& s, hipStream_t st) {
    if (s.heavy_min != g->heavy_min || s.piece != g->piece) {
        const slaq_status r = slaq_graph_set_schedule(g, s.heavy_min, s.piece, st);
        if (r != SLAQ_OK) return r;
    }
    g->cache_rows = s.cache_rows;
    g->fused = s.fused;
    return SLAQ_OK;
}

}  // namespace

}  // namespace slaq

using namespace slaq;

extern "C" {

slaq_status slaq_graph_autotune(slaq_graph_t g, int nv, int m, uint64_t seed, double* alpha, double* beta,
                                int32_t* steps, void* workspace, size_t workspace_bytes, int reps,
                                const char* cache_path, int* from_cache, void* stream) {
    clear_error();
    SLAQ_REQUIRE(g && alpha && beta && steps && workspace, SLAQ_ERR_INVALID_ARG, "NULL pointer argument");
    SLAQ_REQUIRE(nv >= 1 && nv <= SLAQ_MAX_PROBES, SLAQ_ERR_INVALID_ARG, "nv must be in [1, %d]", SLAQ_MAX_PROBES);
    SLAQ_REQUIRE(m >= 1 && m <= SLAQ_MAX_STEPS, SLAQ_ERR_INVALID_ARG, "m must be in [1, %d]", SLAQ_MAX_STEPS);
    SLAQ_REQUIRE(reps >= 0 && reps <= 100, SLAQ_ERR_INVALID_ARG, "reps must be in [0, 100]");
    hipStream_t st = (hipStream_t)stream;
    if (from_cache) *from_cache = 0;
    const std::string key = arch_name() + "|" + shape_key(g, nv);
    tuning::Entries entries;
    if (cache_path) {
        std::string text;
        if (tuning::read_file(cache_path, text))
            SLAQ_REQUIRE(tuning::parse_cache(text, entries), SLAQ_ERR_INVALID_ARG, "tuning cache %s is not a valid cache file",
                         cache_path);
        auto it = entries.find(key);
        if (it != entries.end()) {
            auto field = [&](const char* name, double dflt) {
                auto f = it->second.find(name);
                return f == it->second.end() ? dflt : f->second;
            };
            Setting s{(int)field("heavy_min", g->heavy_min), (int)field("piece", g->piece),
                      (int)field("fused", -1), (int64_t)field("cache_rows", -1), field("ms", 0.0)};
            const slaq_status r = apply(g, s, st);
            if (r != SLAQ_OK) return r;
            if (from_cache) *from_cache = 1;
            return SLAQ_OK;
        }
    }

    if (reps == 0) return SLAQ_OK;  // cache lookup only

    // large graphs: time the first steps only (each step costs the same)
    const bool large = g->nnz >= (int64_t)SLAQ_RELABEL_MIN_NNZ;
    const int mt = large && m > 4 ? 4 : m;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    SLAQ_HIP(hipEventCreate(&e0));
    SLAQ_HIP(hipEventCreate(&e1));
    auto time_it = [&](const Setting& s, double* ms) -> slaq_status {
        slaq_status r = apply(g, s, st);
        if (r != SLAQ_OK) return r;
        size_t need = 0;
        r = slaq_lanczos_workspace(g, nv, mt, &need);
        if (r != SLAQ_OK) return r;
        if (need > workspace_bytes) {  // this candidate needs more than the caller gave
            *ms = INFINITY;
            return SLAQ_OK;
        }
        r = slaq_lanczos(g, nv, mt, seed, alpha, beta, steps, workspace, workspace_bytes, st);
        if (r != SLAQ_OK) return r;
        SLAQ_HIP(hipEventRecord(e0, st));
        for (int k = 0; k < reps; ++k) {
            r = slaq_lanczos(g, nv, mt, seed, alpha, beta, steps, workspace, workspace_bytes, st);
            if (r != SLAQ_OK) return r;
        }
        SLAQ_HIP(hipEventRecord(e1, st));
        SLAQ_HIP(hipEventSynchronize(e1));
        float t = 0.0f;
        SLAQ_HIP(hipEventElapsedTime(&t, e0, e1));
        *ms = (double)t / reps;
        return SLAQ_OK;
    };

    Setting best{g->heavy_min, g->piece, g->fused, g->cache_rows, INFINITY};
    std::vector<Setting> trials;
    slaq_status r = time_it(best, &best.ms);
    auto consider = [&](Setting s) -> slaq_status {
        slaq_status q = time_it(s, &s.ms);
        if (q != SLAQ_OK) return q;
        trials.push_back(s);
        if (s.ms < best.ms) best = s;
        return SLAQ_OK;
    };
    const int hb = heavy_min_bound(g->nnz);
    // row schedule (stage kernels)
    if (r == SLAQ_OK) {
        const Setting base = best;
        const int hms[] = {hb, 2 * hb, 4 * hb};
        const int pcs[] = {64, 128, 256};
        for (int hm : hms)
            for (int pc : pcs) {
                if (hm == base.heavy_min && pc == base.piece) continue;
                if (r == SLAQ_OK) r = consider(Setting{hm, pc, large ? base.fused : 0, base.cache_rows, 0.0});
            }
    }
    if (r == SLAQ_OK && large && g->relabeled) {
        // hot window around the automatic one (rows per range)
        const int64_t automatic = (int64_t)(kCacheBudget / ((size_t)kColRanges * 16 * (lanczos_ld(nv) / 4)));
        const Setting base = best;
        const int64_t wins[] = {automatic / 2, automatic * 3 / 2, g->n};
        for (int64_t w : wins)
            if (r == SLAQ_OK) r = consider(Setting{base.heavy_min, base.piece, base.fused, w, 0.0});
    }
    if (r == SLAQ_OK && !large) {
        // single launch (automatic size, half and double) against the best stage schedule
        const Setting base = best;
        const int64_t rows = g->n;
        int autob = (int)((rows + 79) / 80);
        autob = autob < 8 ? 8 : (autob > 128 ? 128 : autob);
        const int fs[] = {-1, autob / 2 > 0 ? autob / 2 : 1, autob * 2 > 256 ? 256 : autob * 2};
        for (int f : fs)
            if (r == SLAQ_OK) r = consider(Setting{base.heavy_min, base.piece, f, base.cache_rows, 0.0});
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (r != SLAQ_OK) return r;
    r = apply(g, best, st);
    if (r != SLAQ_OK) return r;
    if (cache_path) {
        std::map<std::string, double> f;
        f["heavy_min"] = best.heavy_min;
        f["piece"] = best.piece;
        f["fused"] = best.fused;
        f["cache_rows"] = (double)best.cache_rows;
        f["ms"] = best.ms;
        f["trials"] = (double)trials.size() + 1;
        entries[key] = f;
        SLAQ_REQUIRE(tuning::write_cache(cache_path, entries), SLAQ_ERR_INVALID_ARG, "cannot write tuning cache %s",
                     cache_path);
    }
    return SLAQ_OK;
}

slaq_status slaq_graph_autotune_workspace(slaq_graph_t g, int nv, int m, size_t* bytes) {
    clear_error();
    SLAQ_REQUIRE(g && bytes, SLAQ_ERR_INVALID_ARG, "graph or bytes is NULL");
    // the most demanding candidate: the lowest heavy-row threshold with the
    // smallest pieces (host-side sizing only; the graph is left as it was)
    const int hm = g->heavy_min, pc = g->piece;
    g->heavy_min = heavy_min_bound(g->nnz);
    g->piece = kMinPiece;
    size_t a = 0, b = 0;
    const slaq_status r1 = slaq_lanczos_workspace(g, nv, m, &a);
    g->heavy_min = hm;
    g->piece = pc;
    if (r1 != SLAQ_OK) return r1;
    const slaq_status r2 = slaq_lanczos_workspace(g, nv, m, &b);
    if (r2 != SLAQ_OK) return r2;
    *bytes = a > b ? a : b;
    return SLAQ_OK;
}

slaq_status slaq_graph_settings(slaq_graph_t g, int* heavy_min, int* piece, int64_t* cache_rows, int* fused) {
    clear_error();
    SLAQ_REQUIRE(g, SLAQ_ERR_INVALID_ARG, "graph is NULL");
    if (heavy_min) *heavy_min = g->heavy_min;
    if (piece) *piece = g->piece;
    if (cache_rows) *cache_rows = g->cache_rows;
    if (fused) *fused = g->fused;
    return SLAQ_OK;
}

}  // extern "C"
