// Path planner: chooses the fusion size and the execution path of a circuit
// from measured costs.
//
// The paper's adaptive fusion (Sec. III-C) asks, fusion by fusion, whether a
// fused gate is cheaper than its parts under a cost model measured on the
// target.  Here that question is asked of whole plans: the circuit is fused
// at each size limit in a range, and each fused list is priced on both
// execution paths -- one pass per fused gate (with diagonal runs merged) and
// cache-blocked segments -- from a table of measured rates; the cheapest
// (fused list, path) pair wins.  The rates come from the autotuner:
//  * a single pass costs a launch plus max(algorithmic bytes / its kernel's
//    measured rate, flops / the measured arithmetic rate), the matrix-core
//    kernels' arithmetic rate by block dimension;
//  * a segment of the blocked path costs a launch, one read and write of the
//    state at the measured segment rate, and a measured per-gate cost inside
//    the tile by block dimension (diagonal gates cheapest).
#include <cmath>
#include <cstring>
#include <string>

#include "internal.hpp"

namespace cast {

struct PathCost {
    double bw[7];        // GB/s of algorithmic bytes, by schedule kernel kind 0..6
    double fl[7];        // GFLOP/s of the matrix-core kernels (kinds 4, 5), by block dimension d
    double fl_vec;       // GFLOP/s of the vector kernels
    double launch_ms;    // fixed cost of one pass
    double seg_bw;       // GB/s of a segment's read and write of the state
    double seg_gate[4];  // ms per 2^30 amplitudes per fused gate inside a segment, by d (0: diagonal)
};

// Starting values: rates measured on the MI355X for the kernels as first
// built (replaced by the autotuner's measurements when it has run).
static PathCost g_pc[3] = {
    {},
    // CAST_C64
    {{5100, 4700, 4000, 5100, 4700, 4500, 5300}, {0, 0, 0, 0, 80000, 100000, 120000}, 60000, 0.005, 5000,
     {0.15, 0.30, 0.30, 0.40}},
    // CAST_C128
    {{5200, 4800, 4000, 5260, 4840, 4500, 5400}, {0, 0, 0, 0, 38000, 38700, 51900}, 60000, 0.005, 5000,
     {0.25, 0.50, 0.50, 0.60}},
};

static double *path_cost_field(const std::string &key, cast_dtype dt) {
    PathCost &c = g_pc[dt];
    if (key.size() == 3 && key.compare(0, 2, "bw") == 0 && key[2] >= '0' && key[2] <= '6') return &c.bw[key[2] - '0'];
    if (key.size() == 3 && key.compare(0, 2, "fl") == 0 && key[2] >= '4' && key[2] <= '6') return &c.fl[key[2] - '0'];
    if (key == "fl_vec") return &c.fl_vec;
    if (key == "launch_ms") return &c.launch_ms;
    if (key == "seg_bw") return &c.seg_bw;
    if (key.size() == 9 && key.compare(0, 8, "seg_gate") == 0 && key[8] >= '0' && key[8] <= '3')
        return &c.seg_gate[key[8] - '0'];
    return nullptr;
}

static double pass_ms(const PathCost &c, int kind, int d, double alg_bytes, double flops) {
    if (kind < 0) return 0.0;
    const double mem = alg_bytes / (c.bw[kind] * 1e6);
    const double rate = (kind == 4 || kind == 5) ? c.fl[d < 4 ? 4 : d] : c.fl_vec;
    return c.launch_ms + std::max(mem, flops / (rate * 1e6));
}

static cast_status predict(const cast_fused *f, int n, cast_dtype dt, int path, double *ms) {
    const PathCost &c = g_pc[dt];
    double t = 0;
    if (path == 0) {
        size_t np = 0;
        if (cast_status rc = circuit_passes(f, n, dt, &np)) return rc;
        for (size_t i = 0; i < np; ++i) {
            size_t first;
            int kind;
            double b, fl;
            if (cast_status rc = circuit_pass_info(f, n, dt, i, &first, nullptr, &kind, nullptr, &b, &fl)) return rc;
            const int d = kind == 6 || kind < 0 ? 0 : f->plans[first].d;
            t += pass_ms(c, kind, d, b, fl);
        }
    } else {
        size_t np = 0;
        if (cast_status rc = blocked_info(f, n, dt, &np)) return rc;
        const double S = std::ldexp(1.0, n) * (double)amp_bytes(dt), scale = std::ldexp(1.0, n - 30);
        for (size_t i = 0; i < np; ++i) {
            size_t first, count;
            int tb;
            if (cast_status rc = blocked_pass_info(f, n, dt, i, &first, &count, &tb, nullptr, nullptr)) return rc;
            if (tb == 0) {
                int kind, d;
                double b, fl;
                if (cast_status rc = fused_pass_info(f, first, n, dt, &kind, &d, &b, &fl)) return rc;
                t += pass_ms(c, kind, d, b, fl);
                continue;
            }
            double seg = c.launch_ms + 2.0 * S / (c.seg_bw * 1e6);
            for (size_t g = first; g < first + count; ++g) {
                const PassPlan &p = f->plans[g];
                if (p.identity()) continue;
                seg += c.seg_gate[p.d > 3 ? 3 : p.d] * scale;
            }
            t += seg;
        }
    }
    *ms = t;
    return CAST_OK;
}

}  // namespace cast

using namespace cast;

extern "C" {

cast_status path_cost_set(const char *key, cast_dtype dt, double value) {
    if (!key) return fail(CAST_EINVAL, "key is NULL");
    if (dt != CAST_C64 && dt != CAST_C128) return fail(CAST_EINVAL, "bad dtype");
    double *f = path_cost_field(key, dt);
    if (!f) return fail(CAST_EINVAL, std::string("unknown path-cost key ") + key);
    if (!(value > 0) || !std::isfinite(value)) return fail(CAST_EINVAL, std::string("value must be positive: ") + key);
    *f = value;
    return CAST_OK;
}

cast_status path_cost_get(const char *key, cast_dtype dt, double *value) {
    if (!key || !value) return fail(CAST_EINVAL, "NULL argument");
    if (dt != CAST_C64 && dt != CAST_C128) return fail(CAST_EINVAL, "bad dtype");
    double *f = path_cost_field(key, dt);
    if (!f) return fail(CAST_EINVAL, std::string("unknown path-cost key ") + key);
    *value = *f;
    return CAST_OK;
}

cast_status predict_ms(const cast_fused *f, int n, cast_dtype dt, int path, double *ms) {
    if (!f || !ms) return fail(CAST_EINVAL, "NULL argument");
    if (dt != CAST_C64 && dt != CAST_C128) return fail(CAST_EINVAL, "bad dtype");
    if (path != 0 && path != 1) return fail(CAST_EINVAL, "path must be 0 (per pass) or 1 (cache-blocked)");
    if (n != f->n) return fail(CAST_EINVAL, "n differs from the fused list's");
    return predict(f, n, dt, path, ms);
}

cast_status plan_circuit(int n, const cast_gate *gates, size_t n_gates, cast_dtype dt, const cast_fusion_opts *opts,
                         int k_lo, int k_hi, cast_fused **out, int *path, int *k_max, double *predicted) {
    if (!out || !path || !k_max) return fail(CAST_EINVAL, "NULL argument");
    *out = nullptr;
    if (dt != CAST_C64 && dt != CAST_C128) return fail(CAST_EINVAL, "bad dtype");
    if (k_lo < 1 || k_hi > kMaxK || k_lo > k_hi) return fail(CAST_EINVAL, "need 1 <= k_lo <= k_hi <= 6");
    cast_fusion_opts o;
    fusion_opts_default(&o);
    if (opts) o = *opts;
    cast_fused *best = nullptr;
    double best_ms = 0;
    int best_path = 0, best_k = 0;
    for (int k = k_lo; k <= k_hi; ++k) {
        o.k_max = k;
        cast_fused *f = nullptr;
        if (cast_status rc = fuse_circuit(n, gates, n_gates, &o, &f)) {
            fused_destroy(best);
            return rc;
        }
        bool kept = false;
        for (int p = 0; p <= 1; ++p) {
            double ms;
            if (cast_status rc = predict(f, n, dt, p, &ms)) {
                if (!kept) fused_destroy(f);
                fused_destroy(best);
                return rc;
            }
            if (!best || ms < best_ms) {
                if (best && best != f) fused_destroy(best);
                best = f;
                best_ms = ms;
                best_path = p;
                best_k = k;
                kept = true;
            }
        }
        if (!kept) fused_destroy(f);
    }
    *out = best;
    *path = best_path;
    *k_max = best_k;
    if (predicted) *predicted = best_ms;
    return CAST_OK;
}

}  // extern "C"
