// Host side of the cache-blocked executor (see blocked.hpp): groups a fused
// list into segments, builds each gate's in-tile description, and queues the
// passes.
#include <algorithm>
#include <cstring>

#include "blocked.hpp"
#include "internal.hpp"

namespace cast {

cast_status launch_blocked(void *psi, cast_dtype dt, const void *mats, const BlkGate *gates, const BlkSeg &s,
                           hipStream_t stream);

struct BlockedPlan {
    int tb = 0;
    struct Pass {
        size_t first = 0, count = 0;   // fused gates [first, first + count) covered by this pass
        bool segment = false;
        size_t gate = 0;               // ordinary pass: the fused gate it applies
        BlkSeg seg{};
    };
    std::vector<Pass> passes;
    std::vector<BlkGate> gates;
    void *dev = nullptr;               // device copy of `gates`
};

void blocked_free(BlockedPlan *b) {
    if (!b) return;
    dev_free(b->dev);
    delete b;
}

namespace {

// Qubits mixed by a plan's blocks: the targets its first d virtual basis
// vectors touch.
uint64_t span_qubits(const PassPlan &p) {
    uint64_t m = 0;
    for (int i = 0; i < p.d; ++i)
        for (int s = 0; s < p.k; ++s)
            if ((p.L[i] >> s) & 1u) m |= 1ull << p.q[s];
    return m;
}

// Window w of a tile of 2^tb amplitudes that holds the qubits `need`: the
// fixed point of w = tb - #{q in need : q >= w}; false if it drops below the
// smallest window.
bool window_of(uint64_t need, int tb, int *w_out) {
    int w = tb;
    for (;;) {
        const int w2 = tb - __builtin_popcountll(need >> w);
        if (w2 < kBlkMinWindow) return false;
        if (w2 == w) break;
        w = w2;
    }
    *w_out = w;
    return true;
}

BlkGate make_gate(const PassPlan &p, int w, const int *qh, int nh, uint64_t mat) {
    BlkGate g;
    std::memset(&g, 0, sizeof g);
    g.kind = p.d == 0 ? 0 : 1;
    g.k = p.k;
    g.d = p.d;
    g.mat = mat;
    g.mat_reals = p.d == 0 ? 2u << p.k : (uint32_t)(2 * p.mat.size());
    g.run = 1;
    g.tshift = std::max(p.k, 1);
    for (int s = 0; s < p.k; ++s) {
        const int q = p.q[s];
        g.q[s] = q;
        g.tpos[s] = -1;
        if (q < w) g.tpos[s] = q;
        for (int i = 0; i < nh; ++i)
            if (qh[i] == q) g.tpos[s] = w + i;
    }
    if (p.d == 0) {
        for (uint32_t b : p.blk) g.amask |= 1ull << b;
        return g;
    }
    // L^-1 by Gauss-Jordan: row r of [A | I] with A[r][c] = bit r of L[c]
    const int k = p.k;
    uint32_t rows[kMaxK];
    for (int r = 0; r < k; ++r) {
        rows[r] = 1u << (k + r);
        for (int c = 0; c < k; ++c)
            if ((p.L[c] >> r) & 1u) rows[r] |= 1u << c;
    }
    for (int c = 0; c < k; ++c) {
        int pr = c;
        while (!((rows[pr] >> c) & 1u)) ++pr;   // L is invertible
        std::swap(rows[c], rows[pr]);
        for (int r = 0; r < k; ++r)
            if (r != c && ((rows[r] >> c) & 1u)) rows[r] ^= rows[c];
    }
    for (int s = 0; s < k; ++s) {
        uint32_t col = 0;
        for (int i = 0; i < k; ++i) col |= ((rows[i] >> (k + s)) & 1u) << i;
        g.colv[s] = col;
    }
    // span offsets in tile coordinates (every span target is in the tile)
    for (int i = 0; i < p.d; ++i) {
        uint32_t o = 0;
        for (int s = 0; s < k; ++s)
            if ((p.L[i] >> s) & 1u) o |= 1u << g.tpos[s];
        g.span[i] = o;
    }
    // pivot bits of a reduced echelon basis of the span: the tile positions
    // with zeros there hold one element of every coset
    uint32_t b[kBlkMaxD];
    int piv[kBlkMaxD];
    for (int i = 0; i < p.d; ++i) {
        b[i] = g.span[i];
        for (int j = 0; j < i; ++j)
            if ((b[i] >> piv[j]) & 1u) b[i] ^= b[j];
        piv[i] = 31 - __builtin_clz(b[i]);
        for (int j = 0; j < i; ++j)
            if ((b[j] >> piv[i]) & 1u) b[j] ^= b[i];
    }
    std::sort(piv, piv + p.d);
    for (int i = 0; i < p.d; ++i) g.pivlow[i] = (1u << piv[i]) - 1;
    std::memset(g.slot, -1, sizeof g.slot);
    for (size_t i = 0; i < p.blk.size(); ++i) g.slot[p.blk[i]] = (int8_t)i;
    return g;
}

cast_status build(const cast_fused &f, cast_dtype dt, BlockedPlan **out) {
    const int tb = tuning().blocked_tile_bits[dt];
    if (((size_t)1 << tb) * amp_bytes(dt) > (64u << 10))
        return fail(CAST_EINVAL, "blocked_tile_bits: tile exceeds 64 KiB of LDS");
    auto *bp = new BlockedPlan;
    bp->tb = tb;
    const int n = f.n;
    const std::vector<PassPlan> &P = f.plans;
    const std::vector<size_t> off = plan_offsets(P, dt);
    // matrices / phase tables of one gate area: tile + two areas within the LDS budget
    const size_t tile_bytes = ((size_t)1 << tb) * amp_bytes(dt);
    const size_t area_max = std::min<size_t>(tile_bytes + 2 * kBlkAreaHead < kBlkLdsBudget
                                                 ? (kBlkLdsBudget - tile_bytes) / 2 - kBlkAreaHead : 0,
                                             (size_t)kBlkMaxMatChunks * 16);
    std::vector<size_t> cur;   // non-identity gates of the open segment
    size_t first = 0;
    uint64_t need = 0;
    auto close = [&](size_t end) {
        if (cur.size() == 1) {
            BlockedPlan::Pass ps;
            ps.first = first, ps.count = end - first, ps.gate = cur[0];
            bp->passes.push_back(ps);
        } else if (cur.size() > 1) {
            int w = tb;
            window_of(need, tb, &w);
            BlockedPlan::Pass ps;
            ps.first = first, ps.count = end - first, ps.segment = true;
            BlkSeg &s = ps.seg;
            s.tb = tb, s.w = w, s.nh = 0;
            s.ntiles = 1ull << (n - tb);
            for (int q = w; q < n; ++q)
                if ((need >> q) & 1u) {
                    s.qh[s.nh] = q;
                    s.hlowmask[s.nh] = (1ull << q) - 1;
                    ++s.nh;
                }
            s.g0 = (uint32_t)bp->gates.size();
            for (size_t i : cur) bp->gates.push_back(make_gate(P[i], w, s.qh, s.nh, off[i]));
            s.g1 = (uint32_t)bp->gates.size();
            // consecutive diagonal gates form runs applied in one sweep of the
            // tile; a run's phase tables sit at the stride of its largest table
            for (uint32_t gi = s.g0; gi < s.g1;) {
                uint32_t m = 0;
                int ts = 1;
                while (gi + m < s.g1 && m < kBlkRunMax && bp->gates[gi + m].kind == 0) {
                    const int ts2 = std::max(ts, bp->gates[gi + m].tshift);
                    if (((size_t)(m + 1) << ts2) * amp_bytes(dt) > area_max && m > 0) break;
                    ts = ts2;
                    ++m;
                }
                if (m == 0) {
                    ++gi;
                    continue;
                }
                bp->gates[gi].run = (int)m;
                bp->gates[gi].tshift = ts;
                for (uint32_t j = 1; j < m; ++j) bp->gates[gi + j].run = 0;
                gi += m;
            }
            uint32_t mbytes = 0;
            for (uint32_t gi = s.g0; gi < s.g1; ++gi) {
                const BlkGate &g = bp->gates[gi];
                if (g.kind == 0 && g.run == 0) continue;
                const uint32_t b = g.kind == 0 ? ((uint32_t)g.run << g.tshift) * (uint32_t)amp_bytes(dt)
                                               : g.mat_reals * (dt == CAST_C128 ? 8 : 4);
                mbytes = std::max(mbytes, b);
            }
            s.area = kBlkAreaHead + ((mbytes + 15) & ~15u);
            s.maxd = 0;
            for (uint32_t gi = s.g0; gi < s.g1; ++gi) s.maxd = std::max(s.maxd, bp->gates[gi].d);
            bp->passes.push_back(ps);
        }
        cur.clear();
        need = 0;
        first = end;
    };
    for (size_t i = 0; i < P.size(); ++i) {
        const PassPlan &p = P[i];
        if (p.identity()) continue;
        const uint64_t sp = span_qubits(p);
        int w;
        const size_t mbytes = (p.d == 0 ? ((size_t)2 << std::max(p.k, 1)) : 2 * p.mat.size()) * amp_bytes(dt) / 2;
        if (n < tb || p.d > kBlkMaxD || (mbytes + 15) / 16 > kBlkMaxMatChunks || mbytes > area_max ||
            !window_of(sp, tb, &w)) {
            // an ordinary pass of its own
            close(i);
            BlockedPlan::Pass ps;
            ps.first = i, ps.count = 1, ps.gate = i;
            bp->passes.push_back(ps);
            first = i + 1;
            continue;
        }
        if (window_of(need | sp, tb, &w)) {
            need |= sp;
        } else {
            close(i);
            need = sp;
        }
        cur.push_back(i);
    }
    close(P.size());
    *out = bp;
    return CAST_OK;
}

// The blocked grouping of a fused list for dtype dt (built on first use,
// rebuilt when the tile size knob has changed).  `device`: also upload the
// list's matrices and the grouping's gate table.
cast_status prepare(const cast_fused *fc, int n, cast_dtype dt, bool device, BlockedPlan **out) {
    if (!fc) return fail(CAST_EINVAL, "fused list is NULL");
    if (dt != CAST_C64 && dt != CAST_C128) return fail(CAST_EINVAL, "bad dtype");
    if (n != fc->n) return fail(CAST_EINVAL, "fused list was built for a different qubit count");
    cast_fused *f = const_cast<cast_fused *>(fc);
    BlockedPlan *&bp = f->blocked[dt];
    if (bp && bp->tb != tuning().blocked_tile_bits[dt]) {
        blocked_free(bp);
        bp = nullptr;
    }
    if (!bp) {
        if (cast_status rc = build(*f, dt, &bp)) return rc;
    }
    if (device) {
        if (!f->dev[dt].ptr && !f->plans.empty()) {
            if (cast_status rc = upload_plans(f->plans, dt, &f->dev[dt], &f->dev_off[dt])) return rc;
        }
        if (!bp->dev && !bp->gates.empty()) {
            const size_t bytes = bp->gates.size() * sizeof(BlkGate);
            if (cast_status rc = dev_alloc(&bp->dev, bytes)) return rc;
            const hipError_t e = hipMemcpy(bp->dev, bp->gates.data(), bytes, hipMemcpyHostToDevice);
            if (e != hipSuccess) {
                dev_free(bp->dev);
                bp->dev = nullptr;
                return fail(CAST_EHIP, std::string("blocked gate table upload: ") + hipGetErrorString(e));
            }
        }
    }
    *out = bp;
    return CAST_OK;
}

cast_status launch(cast_sv *sv, const cast_fused *f, const BlockedPlan &bp, size_t i) {
    const BlockedPlan::Pass &ps = bp.passes[i];
    const void *mats = f->dev[sv->dt].ptr;
    if (ps.segment)
        return launch_blocked(sv->data, sv->dt, mats, static_cast<const BlkGate *>(bp.dev), ps.seg, sv->stream);
    const size_t rsz = sv->dt == CAST_C128 ? 8 : 4;
    const void *dm = (const char *)mats + f->dev_off[sv->dt][ps.gate] * rsz;
    return launch_pass(sv->data, sv->n, sv->dt, f->plans[ps.gate], dm, sv->stream);
}

cast_status check(const cast_sv *sv) {
    if (!sv || !sv->data) return fail(CAST_EINVAL, "state is NULL");
    return CAST_OK;
}

}  // namespace
}  // namespace cast

using namespace cast;

extern "C" {

cast_status apply_circuit_blocked(cast_sv *sv, const cast_fused *f) {
    if (cast_status rc = check(sv)) return rc;
    BlockedPlan *bp;
    if (cast_status rc = prepare(f, sv->n, sv->dt, true, &bp)) return rc;
    for (size_t i = 0; i < bp->passes.size(); ++i)
        if (cast_status rc = launch(sv, f, *bp, i)) return rc;
    return CAST_OK;
}

cast_status apply_circuit_blocked_timed(cast_sv *sv, const cast_fused *f, float *pass_ms) {
    if (cast_status rc = check(sv)) return rc;
    if (!pass_ms) return fail(CAST_EINVAL, "NULL argument");
    BlockedPlan *bp;
    if (cast_status rc = prepare(f, sv->n, sv->dt, true, &bp)) return rc;
    const size_t np = bp->passes.size();
    std::vector<hipEvent_t> ev(np + 1, nullptr);
    cast_status rc = CAST_OK;
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) rc = fail(CAST_EHIP, "hipEventCreate failed");
    if (!rc && hipEventRecord(ev[0], sv->stream) != hipSuccess) rc = fail(CAST_EHIP, "hipEventRecord failed");
    for (size_t i = 0; i < np && !rc; ++i) {
        rc = launch(sv, f, *bp, i);
        if (!rc && hipEventRecord(ev[i + 1], sv->stream) != hipSuccess) rc = fail(CAST_EHIP, "hipEventRecord failed");
    }
    if (!rc && hipEventSynchronize(ev[np]) != hipSuccess) rc = fail(CAST_EHIP, "hipEventSynchronize failed");
    for (size_t i = 0; i < np && !rc; ++i)
        if (hipEventElapsedTime(&pass_ms[i], ev[i], ev[i + 1]) != hipSuccess)
            rc = fail(CAST_EHIP, "hipEventElapsedTime failed");
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    return rc;
}

cast_status blocked_info(const cast_fused *f, int n, cast_dtype dt, size_t *n_passes) {
    if (!n_passes) return fail(CAST_EINVAL, "NULL argument");
    BlockedPlan *bp;
    if (cast_status rc = prepare(f, n, dt, false, &bp)) return rc;
    *n_passes = bp->passes.size();
    return CAST_OK;
}

cast_status blocked_pass_info(const cast_fused *f, int n, cast_dtype dt, size_t i, size_t *first, size_t *count,
                              int *tile_bits, int *window, int *high_qubits) {
    BlockedPlan *bp;
    if (cast_status rc = prepare(f, n, dt, false, &bp)) return rc;
    if (i >= bp->passes.size()) return fail(CAST_EINVAL, "pass index out of range");
    const BlockedPlan::Pass &ps = bp->passes[i];
    if (first) *first = ps.first;
    if (count) *count = ps.count;
    if (tile_bits) *tile_bits = ps.segment ? ps.seg.tb : 0;
    if (window) *window = ps.segment ? ps.seg.w : 0;
    if (high_qubits) {
        for (int j = 0; j < kBlkMaxHigh; ++j) high_qubits[j] = -1;
        if (ps.segment)
            for (int j = 0; j < ps.seg.nh; ++j) high_qubits[j] = ps.seg.qh[j];
    }
    return CAST_OK;
}

}  // extern "C"
