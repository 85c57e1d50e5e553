// Host side of batched adjoint gradients (batch.hpp): builds the op programs
// of many parametrised circuits, binds parameters into a pinned matrix
// buffer, and runs the program as per-step launches, per-step launches
// captured in a hipGraph, or one persistent launch captured in a hipGraph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>

#include "batch.hpp"
#include "internal.hpp"

namespace cast {

static const cplx kIpowB[4] = {cplx(1, 0), cplx(0, 1), cplx(-1, 0), cplx(0, -1)};

struct HostOp {
    uint32_t kind;
    int gate;            // gate index (FWD/ADJ)
    int slot;
};

struct InstPlan {
    int n;
    std::vector<cast_gate> gates;          // copied descriptors
    std::vector<std::vector<cplx>> fixed;  // fixed matrices (sorted-qubit order), per gate
    std::vector<int> sq0, sq1;             // sorted targets per gate
    std::vector<int> form;                 // BatchForm of each gate's matrix (all parameter values)
    std::vector<uint32_t> neg;             // BF_SIGN: local indices of the -1 diagonal entries
    std::vector<uint32_t> xl, zl;          // local generator masks per gate
    std::vector<int> gen_sorted;           // generator letters in sorted local order
    std::vector<uint64_t> gx, gz;          // global generator masks per gate
    std::vector<int> gslot;                // result slot per gate (-1: none)
    std::vector<HostOp> ops;
    int tb = 0;                            // tile bits of this instance's segments
    std::vector<std::vector<int>> seg_gates;   // per op (FWD/ADJ): gates in processing order
    std::vector<uint64_t> mat_fwd, mat_adj;  // matrix offsets (complex entries) per gate
    size_t nparams = 0;
    int nslots = 0;
    uint32_t wgs = 1;
};

}  // namespace cast

struct cast_batch {
    int ninst = 0;
    cast_dtype dt = CAST_C128;
    int mode = 0;
    hipStream_t stream = nullptr;
    std::vector<cast::InstPlan> inst;
    // device
    void *states = nullptr;
    cast::BatchRec *d_recs = nullptr;
    cast::SegGate *d_segs = nullptr;
    cast::SegSweep *d_sweeps = nullptr;
    size_t lds_bytes = 0;
    uint64_t *d_step_rec = nullptr, *d_step_item = nullptr;
    cast::BatchInst *d_insts = nullptr;
    void *d_mats = nullptr;
    cast::PauliSumGroup *d_tg = nullptr;
    cast::PauliSumTerm *d_tt = nullptr;
    double *d_partials = nullptr, *d_results = nullptr;
    unsigned long long *d_counters = nullptr;
    // host
    void *h_mats = nullptr;      // pinned, matrices in the state dtype
    double *h_results = nullptr; // pinned
    size_t mat_entries = 0, result_doubles = 0;
    std::vector<uint64_t> step_rec, step_item;
    std::vector<uint64_t> step_items;   // items per step
    std::vector<size_t> step_lds;       // LDS bytes of each step's launch
    int nsteps = 0;
    uint64_t total_items = 0;
    cast::BatchDev dev;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int persistent_grid = 1024;
    uint32_t persistent_chunk = 16;
    uint32_t spin_limit = 1u << 24;
};

namespace cast {

static void sorted_matrix(int k, const int *qubits, const std::vector<cplx> &m, int *q0, int *q1,
                          std::vector<cplx> *out) {
    PassPlan p;
    make_plan(k, qubits, m.data(), 0.0, 0.0, &p);
    *q0 = p.q[0];
    *q1 = k == 2 ? p.q[1] : -1;
    *out = p.full;
}

// Writes a gate's matrix entry into the pinned table in the state dtype: its
// 2^k x 2^k entries row-major (dagger: those of the adjoint), or compactly
// for the forms the batched kernels read so: a two-qubit diagonal its four
// diagonal entries; a Pauli pair (BF_PAULI, masks xm / zm) a and b of
// y_r = a x_r + b (-1)^{popc(zm & (r ^ xm))} x_{r ^ xm}.
static void put_matrix(cast_batch *b, uint64_t off, const cplx *m, bool dagger, int k, int form, uint32_t xm,
                       uint32_t zm) {
    const int D = 1 << k;
    auto put = [&](uint64_t e, cplx z) {
        if (b->dt == CAST_C128) {
            ((double *)b->h_mats)[2 * e] = z.real();
            ((double *)b->h_mats)[2 * e + 1] = z.imag();
        } else {
            ((float *)b->h_mats)[2 * e] = (float)z.real();
            ((float *)b->h_mats)[2 * e + 1] = (float)z.imag();
        }
    };
    auto at = [&](int r, int c) { return dagger ? std::conj(m[(size_t)c * D + r]) : m[(size_t)r * D + c]; };
    if (k == 2 && (form == BF_DIAG || form == BF_PAULI)) {
        if (form == BF_DIAG) {
            for (int r = 0; r < D; ++r) put(off + r, at(r, r));
        } else {
            put(off, at(0, 0));
            put(off + 1, at(0, (int)xm) * ((__builtin_popcount(zm & xm) & 1) ? -1.0 : 1.0));
            for (int e = 2; e < D; ++e) put(off + e, 0.0);
        }
        for (int e = D; e < D * D; ++e) put(off + e, 0.0);
        return;
    }
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c) put(off + (uint64_t)r * D + c, at(r, c));
}

// Whether a two-qubit matrix is a I + b P for one Pauli string P that flips
// bits: nonzeros only on the diagonal (all equal) and at (r, r ^ x) for one
// x != 0, with the off-diagonal signs those of a Z mask z (the i^{|x & z|}
// of the Y letters folds into b).  On success, *xm and *zm (local bits).
static bool pauli_pair(const std::vector<cplx> &m, uint32_t *xm, uint32_t *zm) {
    const int D = 4;
    for (uint32_t x = 1; x < (uint32_t)D; ++x) {
        bool ok = true;
        for (int r = 0; r < D && ok; ++r)
            for (int c = 0; c < D && ok; ++c)
                if (c != r && c != (int)(r ^ x) && m[(size_t)r * D + c] != cplx(0, 0)) ok = false;
        for (int r = 1; r < D && ok; ++r)
            if (m[(size_t)r * D + r] != m[0]) ok = false;
        if (!ok) continue;
        for (uint32_t z = 0; z < (uint32_t)D; ++z) {
            const cplx b0 = m[x] * ((__builtin_popcount(z & x) & 1) ? -1.0 : 1.0);
            bool good = true;
            for (int r = 1; r < D && good; ++r) {
                const cplx br = m[(size_t)r * D + (r ^ x)] * ((__builtin_popcount(z & (r ^ x)) & 1) ? -1.0 : 1.0);
                if (std::abs(br - b0) > 1e-15 * (1.0 + std::abs(b0))) good = false;
            }
            if (good) {
                *xm = x;
                *zm = z;
                return true;
            }
        }
    }
    return false;
}

// exp(-i a P / 2) = cos(a/2) I - i sin(a/2) P with P a Pauli string (2-bit
// letters in local bit order): P has one nonzero per row, at column r ^ x.
static void bind_rotation(cast_batch *b, uint64_t off, int k, int gen, double angle, bool dagger, int form,
                          uint32_t xm, uint32_t zm) {
    const int D = 1 << k;
    const double c = std::cos(angle / 2), s = std::sin(angle / 2) * (dagger ? -1.0 : 1.0);
    uint32_t x = 0;
    for (int i = 0; i < k; ++i) {
        const int L = (gen >> (2 * i)) & 3;
        if (L == 1 || L == 2) x |= 1u << i;
    }
    cplx m[16];
    for (int e = 0; e < D * D; ++e) m[e] = 0.0;
    for (int r = 0; r < D; ++r) {
        // P[r][r ^ x] = prod_i f(letter_i, bit_i(r)); Y: [[0,-i],[i,0]], Z: diag(1,-1)
        cplx p = 1.0;
        for (int i = 0; i < k; ++i) {
            const int L = (gen >> (2 * i)) & 3, bit = (r >> i) & 1;
            if (L == 2) p *= bit ? cplx(0, 1) : cplx(0, -1);
            else if (L == 3 && bit) p = -p;
        }
        m[r * D + r] += c;
        m[r * D + (r ^ (int)x)] += cplx(0, -1) * s * p;  // dagger: conj of a Hermitian P's coefficient
    }
    // U^dag = cos I + i sin P; the loop above used -s for it, and P is Hermitian
    put_matrix(b, off, m, false, k, form, xm, zm);
}

static cast_status queue_program(cast_batch *b) {
    hipStream_t s = b->stream;
    const size_t rsz = b->dt == CAST_C128 ? 8 : 4;
    CAST_HIP_TRY(hipMemcpyAsync(b->d_mats, b->h_mats, b->mat_entries * 2 * rsz, hipMemcpyHostToDevice, s));
    if (cast_status rc = batch_init_states(b->dev, b->dt, s)) return rc;
    if (b->mode == 2) {
        if (cast_status rc = batch_zero(b->d_counters, 2 + (size_t)b->ninst, s)) return rc;
        if (cast_status rc = batch_launch_persistent(b->dev, b->dt, b->total_items, b->persistent_grid,
                                                     b->d_counters, b->spin_limit, b->persistent_chunk, b->lds_bytes, s))
            return rc;
    } else {
        for (int st = 0; st < b->nsteps; ++st)
            if (cast_status rc = batch_launch_step(b->dev, b->dt, st, b->step_items[st], b->step_lds[st], s)) return rc;
    }
    if (cast_status rc = batch_finish(b->dev, s)) return rc;
    CAST_HIP_TRY(hipMemcpyAsync(b->h_results, b->d_results, b->result_doubles * sizeof(double),
                                hipMemcpyDeviceToHost, s));
    if (b->mode == 2)
        CAST_HIP_TRY(hipMemcpyAsync(b->h_results + b->result_doubles, b->d_counters + 1, sizeof(unsigned long long),
                                    hipMemcpyDeviceToHost, s));
    return CAST_OK;
}

static void free_batch(cast_batch *b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    dev_free(b->states);
    dev_free(b->d_recs);
    dev_free(b->d_segs);
    dev_free(b->d_sweeps);
    dev_free(b->d_step_rec);
    dev_free(b->d_step_item);
    dev_free(b->d_insts);
    dev_free(b->d_mats);
    dev_free(b->d_tg);
    dev_free(b->d_tt);
    dev_free(b->d_partials);
    dev_free(b->d_results);
    dev_free(b->d_counters);
    if (b->h_mats) (void)hipHostFree(b->h_mats);
    if (b->h_results) (void)hipHostFree(b->h_results);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

// Tile of a segment: 2^batch_tile_bits amplitudes (the tuning knob, 11 by
// default for both dtypes: psi and lambda together 64 KiB of LDS in
// complex128, 32 KiB in complex64); CAST_BATCH_TILE_BITS overrides.
static int batch_tile_bits(cast_dtype dt) {
    int tb = tuning().batch_tile_bits[dt == CAST_C64 ? CAST_C64 : CAST_C128];
    if (const char *e = std::getenv("CAST_BATCH_TILE_BITS")) tb = std::min(12, std::max(4, atoi(e)));
    return tb;
}

// Low window a segment's tile keeps (the knob batch_min_window, at most
// tb - 2 so that a two-qubit gate on high qubits still fits);
// CAST_BATCH_MIN_WINDOW overrides.
static int batch_min_window(cast_dtype dt, int tb) {
    int w = tuning().batch_min_window[dt == CAST_C64 ? CAST_C64 : CAST_C128];
    if (const char *e = std::getenv("CAST_BATCH_MIN_WINDOW")) w = atoi(e);
    return std::max(0, std::min(w, tb - 2));
}

// Whether segments may take gates out of circuit order (CAST_BATCH_REORDER=0
// keeps the circuit order).
static bool batch_reorder() {
    const char *e = std::getenv("CAST_BATCH_REORDER");
    return !e || atoi(e) != 0;
}

// Cuts a gate list into segments whose qubits fit a tile of 2^tb amplitudes
// (at most kSegMaxGates gates each), returned in application order: the
// circuit's order (reverse: the reverse order) or, with `reorder`, another
// order of the same circuit.  Two gates that share a qubit keep their
// relative order unless both are diagonal (diagonal gates commute); gates on
// disjoint qubits commute.  So any order in which every such pair keeps its
// relative order applies the same operator, and the adjoint sweep evaluates
// each gate's derivative between the states that order gives before and
// after it.  The greedy schedule fills a segment with ready gates (all
// earlier dependent gates applied), preferring those whose qubits the
// segment already holds, then the earliest ready gate that still fits.  On
// a layered ansatz (rotations on every qubit, then an entangling ring) this
// roughly halves the segments of the circuit-order cut, since a layer's
// rotations on the qubits of one tile need not wait for the rest of the
// layer.
// Orders the gates of one segment (given in a valid application order) so
// that consecutive gates share few qubits: the kernel applies each run of
// gates on at most three qubits (a register sweep) with one LDS round trip
// and one barrier, so fewer, longer runs cost less.  List scheduling under
// the same dependence rule as the segments: a run is grown from ready gates,
// first those whose qubits it already holds, then the one adding the fewest
// new qubits (earliest on ties), until no ready gate fits three qubits.  On
// a layered ansatz this interleaves the rotations of neighbouring qubits
// with the entangling gates between them (RY, RZ on q and q + 1, then their
// CZ) instead of running each rotation layer across the whole tile.
static std::vector<int> cluster_sweeps(const std::vector<int> &seg, const std::vector<uint64_t> &gmask,
                                       const std::vector<char> &gdiag) {
    const int n = (int)seg.size();
    std::vector<std::vector<int>> succ(n);
    std::vector<int> indeg(n, 0);
    for (int a = 0; a < n; ++a)
        for (int b = a + 1; b < n; ++b)
            if ((gmask[seg[a]] & gmask[seg[b]]) && !(gdiag[seg[a]] && gdiag[seg[b]])) {
                succ[a].push_back(b);
                ++indeg[b];
            }
    std::vector<int> ready, out;
    for (int a = 0; a < n; ++a)
        if (!indeg[a]) ready.push_back(a);
    while ((int)out.size() < n) {
        uint64_t bits = 0;
        for (;;) {
            int pick = -1, best_new = 4;
            for (size_t r = 0; r < ready.size(); ++r) {
                const uint64_t m = gmask[seg[ready[r]]];
                const int nw = __builtin_popcountll(m & ~bits);
                if (__builtin_popcountll(bits | m) > 3) continue;
                if (nw < best_new) pick = (int)r, best_new = nw;   // ready is ascending: earliest on ties
            }
            if (pick < 0 && bits == 0) pick = 0;   // (a gate on more than three qubits runs alone)
            if (pick < 0) break;
            const int a = ready[pick];
            ready.erase(ready.begin() + pick);
            out.push_back(seg[a]);
            bits |= gmask[seg[a]];
            for (int b : succ[a])
                if (--indeg[b] == 0) ready.insert(std::lower_bound(ready.begin(), ready.end(), b), b);
        }
    }
    return out;
}

static std::vector<std::vector<int>> segment_gates(const std::vector<uint64_t> &gmask, const std::vector<char> &gdiag,
                                                   int tb, bool reverse, bool reorder, int wmin) {
    const int L = (int)gmask.size();
    // a segment's qubits fit a tile of 2^tb amplitudes whose low window
    // [0, W) keeps at least wmin bits: at most tb - wmin of them lie at or
    // above bit wmin, so the tile is read in runs of at least 2^wmin
    // consecutive amplitudes
    const uint64_t hi_mask = wmin >= 64 ? 0 : ~((1ull << wmin) - 1);
    auto fits = [&](uint64_t q) {
        return __builtin_popcountll(q) <= tb && __builtin_popcountll(q & hi_mask) <= tb - wmin;
    };
    auto gate_at = [&](int p) { return reverse ? L - 1 - p : p; };   // base order position -> gate
    std::vector<std::vector<int>> segs;
    if (!reorder) {
        std::vector<int> cur;
        uint64_t qm = 0;
        for (int p = 0; p < L; ++p) {
            const int l = gate_at(p);
            if (!cur.empty() && (!fits(qm | gmask[l]) || cur.size() >= (size_t)kSegMaxGates)) {
                segs.push_back(cur);
                cur.clear();
                qm = 0;
            }
            cur.push_back(l);
            qm |= gmask[l];
        }
        if (!cur.empty()) segs.push_back(cur);
        return segs;
    }
    // dependence graph over base positions: per qubit, the last non-diagonal
    // gate and the diagonal gates since it
    std::vector<std::vector<int>> succ(L);
    std::vector<int> indeg(L, 0);
    std::vector<int> last_nd(64, -1);
    std::vector<std::vector<int>> diag_since(64);
    auto edge = [&](int a, int b) {
        if (a < 0) return;
        succ[a].push_back(b);
        ++indeg[b];
    };
    for (int p = 0; p < L; ++p) {
        const int l = gate_at(p);
        std::vector<int> preds;
        for (int q = 0; q < 64; ++q) {
            if (!((gmask[l] >> q) & 1ull)) continue;
            if (gdiag[l]) {
                preds.push_back(last_nd[q]);
                diag_since[q].push_back(p);
            } else {
                preds.push_back(last_nd[q]);
                for (int d : diag_since[q]) preds.push_back(d);
                diag_since[q].clear();
                last_nd[q] = p;
            }
        }
        std::sort(preds.begin(), preds.end());
        preds.erase(std::unique(preds.begin(), preds.end()), preds.end());
        for (int a : preds) edge(a, p);
    }
    std::vector<int> ready;   // base positions, ascending
    for (int p = 0; p < L; ++p)
        if (!indeg[p]) ready.push_back(p);
    int done = 0;
    while (done < L) {
        std::vector<int> cur;
        uint64_t qm = 0;
        while (cur.size() < (size_t)kSegMaxGates && !ready.empty()) {
            int pick = -1;
            for (size_t r = 0; r < ready.size() && pick < 0; ++r)
                if (!(gmask[gate_at(ready[r])] & ~qm)) pick = (int)r;
            for (size_t r = 0; r < ready.size() && pick < 0; ++r)
                if (fits(qm | gmask[gate_at(ready[r])])) pick = (int)r;
            if (pick < 0) break;
            const int p = ready[pick];
            ready.erase(ready.begin() + pick);
            cur.push_back(gate_at(p));
            qm |= gmask[gate_at(p)];
            ++done;
            for (int b : succ[p])
                if (--indeg[b] == 0) ready.insert(std::lower_bound(ready.begin(), ready.end(), b), b);
        }
        segs.push_back(cluster_sweeps(cur, gmask, gdiag));
    }
    return segs;
}

template <typename T>
static cast_status upload(T **dst, const std::vector<T> &src) {
    if (cast_status rc = dev_alloc((void **)dst, std::max<size_t>(1, src.size()) * sizeof(T))) return rc;
    if (!src.empty()) CAST_HIP_TRY(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return CAST_OK;
}

}  // namespace cast

using namespace cast;

extern "C" {

cast_status batch_create(int n_inst, const int *n_qubits, cast_dtype dt, const cast_gate *const *circuits,
                         const size_t *n_gates, const size_t *n_params, const cast_pauli_term *const *hams,
                         const size_t *n_terms, const int *init_kind, const cast_sv *const *init_states, int mode,
                         cast_batch **out) {
    if (!out) return fail(CAST_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_inst < 1 || n_inst > 65535) return fail(CAST_EINVAL, "n_inst must be in [1, 65535]");
    if (!n_qubits || !circuits || !n_gates || !n_params || !hams || !n_terms)
        return fail(CAST_EINVAL, "NULL array argument");
    if (dt != CAST_C64 && dt != CAST_C128) return fail(CAST_EINVAL, "bad dtype");
    if (mode < 0 || mode > 2) return fail(CAST_EINVAL, "mode must be 0, 1 or 2");
    cast_batch *b = new cast_batch;
    b->ninst = n_inst;
    b->dt = dt;
    b->mode = mode;
    b->inst.resize(n_inst);
    std::vector<PauliSumGroup> tg;
    std::vector<PauliSumTerm> tt;
    std::vector<BatchInst> hinst(n_inst);
    size_t state_elems = 0;
    // amplitudes per work item, and the cache budget of an instance group
    // tile of a segment: 2^batch_tile_bits amplitudes of psi and of lambda
    const int tile_bits = batch_tile_bits(dt);
    // per-step launches: groups sized for the 256 MB last-level cache; the
    // persistent launch keeps every instance in one step-major stream
    double group_bytes = mode == 2 ? 0.0 : 192.0 * (1 << 20);
    if (const char *e = std::getenv("CAST_BATCH_GROUP_MB"))
        if (mode != 2) group_bytes = atof(e) * (1 << 20);
    if (const char *e = std::getenv("CAST_PERSISTENT_GROUP_MB"))
        if (mode == 2) group_bytes = atof(e) * (1 << 20);
    uint64_t mat_entries = 0, part = 0, res = 0;
    auto bail = [&](cast_status rc) {
        free_batch(b);
        return rc;
    };
    for (int i = 0; i < n_inst; ++i) {
        InstPlan &ip = b->inst[i];
        const int n = n_qubits[i];
        if (n < 3 || n > kMaxQubits) return bail(fail(CAST_EINVAL, "instance qubit count must be in [3, 34]"));
        if (n_gates[i] && !circuits[i]) return bail(fail(CAST_EINVAL, "circuit is NULL"));
        ip.n = n;
        ip.nparams = n_params[i];
        ip.gates.assign(circuits[i], circuits[i] + n_gates[i]);
        const size_t L = ip.gates.size();
        ip.fixed.resize(L);
        ip.form.assign(L, BF_GENERAL);
        ip.neg.assign(L, 0);
        ip.sq0.resize(L);
        ip.sq1.resize(L);
        ip.xl.assign(L, 0);
        ip.zl.assign(L, 0);
        ip.gen_sorted.assign(L, 0);
        ip.gx.assign(L, 0);
        ip.gz.assign(L, 0);
        ip.gslot.assign(L, -1);
        ip.mat_fwd.resize(L);
        ip.mat_adj.resize(L);
        int slot = 1;  // slot 0: energy
        for (size_t l = 0; l < L; ++l) {
            const cast_gate &g = ip.gates[l];
            if (g.k < 1 || g.k > 2) return bail(fail(CAST_EUNSUPPORTED, "batched programs take 1- and 2-qubit gates"));
            for (int a = 0; a < g.k; ++a) {
                if (g.qubits[a] < 0 || g.qubits[a] >= n) return bail(fail(CAST_EINVAL, "gate qubit out of range"));
                for (int c = 0; c < a; ++c)
                    if (g.qubits[a] == g.qubits[c]) return bail(fail(CAST_EINVAL, "duplicate gate qubit"));
            }
            const int D = 1 << g.k;
            std::vector<cplx> m((size_t)D * D);
            if (g.param_id >= 0) {
                if ((size_t)g.param_id >= ip.nparams) return bail(fail(CAST_EINVAL, "param_id out of range"));
                if (g.generator <= 0 || g.generator >= (1 << (2 * g.k)))
                    return bail(fail(CAST_EINVAL, "parametrised gate needs a Pauli generator"));
                m = rotation_matrix(g.k, g.generator, 0.0);  // placeholder; bound in batch_run
                ip.gslot[l] = slot++;
            } else {
                if (!g.matrix) return bail(fail(CAST_EINVAL, "fixed gate without a matrix"));
                for (int e = 0; e < D * D; ++e) m[e] = cplx(g.matrix[2 * e], g.matrix[2 * e + 1]);
            }
            sorted_matrix(g.k, g.qubits, m, &ip.sq0[l], &ip.sq1[l], &ip.fixed[l]);
            // generator masks: global and in sorted local bits
            for (int a = 0; a < g.k && g.param_id >= 0; ++a) {
                const int letter = (g.generator >> (2 * a)) & 3;
                const int q = g.qubits[a];
                const int lb = (q == ip.sq0[l]) ? 0 : 1;
                if (letter == 1 || letter == 2) ip.gx[l] |= 1ull << q, ip.xl[l] |= 1u << lb;
                if (letter == 2 || letter == 3) ip.gz[l] |= 1ull << q, ip.zl[l] |= 1u << lb;
                ip.gen_sorted[l] |= letter << (2 * lb);
            }
            // form: exp(-i a P / 2) = cos I - i sin P is diagonal when P has no X or Y
            // letter and real when P has an odd number of Y letters (P imaginary);
            // a fixed gate's form is read off its matrix
            if (g.param_id >= 0) {
                int nx = 0, ny = 0;
                for (int a = 0; a < g.k; ++a) {
                    const int letter = (g.generator >> (2 * a)) & 3;
                    nx += letter == 1;
                    ny += letter == 2;
                }
                if (nx == 0 && ny == 0) ip.form[l] = BF_DIAG;
                else if (ny % 2 == 1) ip.form[l] = BF_REAL;
                else if (g.k == 2) ip.form[l] = BF_PAULI;   // masks: the generator's
            } else {
                bool diag = true, real = true, sign = true;
                for (int r = 0; r < D; ++r)
                    for (int c = 0; c < D; ++c) {
                        const cplx z = ip.fixed[l][(size_t)r * D + c];
                        if (r != c && z != cplx(0, 0)) diag = false;
                        if (z.imag() != 0.0) real = false;
                        if (r == c && z != cplx(1, 0) && z != cplx(-1, 0)) sign = false;
                    }
                ip.form[l] = diag ? (sign ? BF_SIGN : BF_DIAG) : real ? BF_REAL : BF_GENERAL;
                for (int r = 0; r < D && ip.form[l] == BF_SIGN; ++r)
                    if (ip.fixed[l][(size_t)r * D + r] == cplx(-1, 0)) ip.neg[l] |= 1u << r;
                uint32_t xm, zm;
                if (ip.form[l] == BF_GENERAL && g.k == 2 && pauli_pair(ip.fixed[l], &xm, &zm)) {
                    ip.form[l] = BF_PAULI;
                    ip.xl[l] = xm;   // a fixed gate has no generator: its Pauli pair's masks
                    ip.zl[l] = zm;
                }
            }
            ip.mat_fwd[l] = mat_entries;
            mat_entries += (uint64_t)D * D;
            ip.mat_adj[l] = mat_entries;
            mat_entries += (uint64_t)D * D;
        }
        ip.nslots = slot;
        // segments (forward order, then reverse order) whose qubits together
        // fit one tile of 2^tb amplitudes
        ip.tb = std::min(n, tile_bits);
        std::vector<uint64_t> gmask(L, 0);
        std::vector<char> gdiag(L, 0);
        for (size_t l = 0; l < L; ++l) {
            for (int a = 0; a < ip.gates[l].k; ++a) gmask[l] |= 1ull << ip.gates[l].qubits[a];
            gdiag[l] = ip.form[l] == BF_DIAG || ip.form[l] == BF_SIGN;
        }
        auto segment = [&](bool reverse) {
            return segment_gates(gmask, gdiag, ip.tb, reverse, batch_reorder(), batch_min_window(dt, ip.tb));
        };
        for (auto &sg : segment(false)) {
            ip.ops.push_back(HostOp{BK_FWD, -1, -1});
            ip.seg_gates.push_back(sg);
        }
        ip.ops.push_back(HostOp{BK_HPSI, -1, 0});
        ip.seg_gates.emplace_back();
        for (auto &sg : segment(true)) {
            ip.ops.push_back(HostOp{BK_ADJ, -1, -1});
            ip.seg_gates.push_back(sg);
        }
        ip.wgs = 1u << (n - ip.tb);
        // Hamiltonian, grouped by x mask
        if (n_terms[i] && !hams[i]) return bail(fail(CAST_EINVAL, "Hamiltonian is NULL"));
        BatchInst &bi = hinst[i];
        bi.n = n;
        bi.nslots = ip.nslots;
        bi.wgs = ip.wgs;
        bi.tg_off = (uint32_t)tg.size();
        bi.tt_off = (uint32_t)tt.size();
        std::map<uint64_t, std::vector<size_t>> byx;
        std::vector<uint64_t> order;
        const uint64_t full = (1ull << n) - 1;
        for (size_t t = 0; t < n_terms[i]; ++t) {
            const cast_pauli_term &pt = hams[i][t];
            if ((pt.xmask | pt.zmask) & ~full) return bail(fail(CAST_EINVAL, "Pauli term acts outside the state"));
            if (!byx.count(pt.xmask)) order.push_back(pt.xmask);
            byx[pt.xmask].push_back(t);
        }
        int first = 0;
        for (uint64_t x : order) {
            tg.push_back(PauliSumGroup{x, first, (int)byx[x].size()});
            for (size_t t : byx[x]) {
                const cast_pauli_term &pt = hams[i][t];
                const cplx c = pt.coeff * kIpowB[__builtin_popcountll(pt.xmask & pt.zmask) & 3];
                tt.push_back(PauliSumTerm{pt.zmask, c.real(), c.imag()});
                ++first;
            }
        }
        bi.ngroups = (uint32_t)order.size();
        bi.part_off = part;
        part += 2ull * ip.nslots * ip.wgs;
        bi.res_off = res;
        res += 2ull * ip.nslots;
        bi.init_kind = init_kind ? init_kind[i] : 0;
        if (bi.init_kind < 0 || bi.init_kind > 2) return bail(fail(CAST_EINVAL, "bad init kind"));
        if (bi.init_kind == 2) {
            const cast_sv *src = init_states ? init_states[i] : nullptr;
            if (!src || !src->data || src->n != n || src->dt != dt)
                return bail(fail(CAST_EINVAL, "init state missing or of the wrong size/dtype"));
            bi.init_src = src->data;
        }
        state_elems += 2ull << n;  // psi and lambda
    }
    if (mat_entries > 0xffffffffull) return bail(fail(CAST_EUNSUPPORTED, "batch matrix table exceeds 2^32 entries"));
    b->mat_entries = mat_entries;
    b->result_doubles = res;
    // ---- instance groups (consecutive instances whose psi and lambda fit the
    // cache budget run their whole programs before the next group), then
    // steps: step (g, s) holds op s of every instance of group g
    std::vector<std::pair<int, int>> groups;  // [first, last)
    {
        int first = 0;
        double acc = 0;
        const double ab_d = (double)amp_bytes(dt);
        for (int i = 0; i < n_inst; ++i) {
            const double bytes = 2.0 * std::ldexp(1.0, n_qubits[i]) * ab_d;
            if (i > first && group_bytes > 0 && acc + bytes > group_bytes) {
                groups.emplace_back(first, i);
                first = i;
                acc = 0;
            }
            acc += bytes;
        }
        groups.emplace_back(first, n_inst);
        // keep a captured program below 65536 launches: merge groups if needed
        size_t max_ops_all = 0;
        for (auto &ip : b->inst) max_ops_all = std::max(max_ops_all, ip.ops.size());
        const size_t cap = 65536;
        if (groups.size() * max_ops_all > cap) {
            const size_t per = (groups.size() * max_ops_all + cap - 1) / cap;   // groups per merged group
            std::vector<std::pair<int, int>> merged;
            for (size_t gi = 0; gi < groups.size(); gi += per)
                merged.emplace_back(groups[gi].first, groups[std::min(groups.size(), gi + per) - 1].second);
            groups.swap(merged);
        }
    }
    std::vector<BatchRec> recs;
    std::vector<SegGate> segs;
    std::vector<SegSweep> sweeps;
    uint64_t item_base = 0;
    for (auto &gr : groups) {
    size_t max_ops = 0;
    for (int i = gr.first; i < gr.second; ++i) max_ops = std::max(max_ops, b->inst[i].ops.size());
    for (size_t s = 0; s < max_ops; ++s) {
        b->step_rec.push_back(recs.size());
        b->step_item.push_back(item_base);
        uint64_t items = 0;
        for (int i = gr.first; i < gr.second; ++i) {
            const InstPlan &ip = b->inst[i];
            if (s >= ip.ops.size()) continue;
            const HostOp &op = ip.ops[s];
            BatchRec r;
            memset(&r, 0, sizeof r);
            r.kind = op.kind;
            r.inst = (uint32_t)i;
            r.item0 = (uint32_t)items;
            r.wgs = ip.wgs;
            r.slot = op.slot;
            r.need = (uint64_t)s * ip.wgs;
            r.tb = ip.tb;
            if (op.kind != BK_HPSI) {
                // tile geometry: smallest khi with #{segment qubits >= tb - khi} == khi
                const std::vector<int> &gl = ip.seg_gates[s];
                uint64_t qm = 0;
                for (int l : gl)
                    for (int a = 0; a < ip.gates[l].k; ++a) qm |= 1ull << ip.gates[l].qubits[a];
                int khi = 0;
                for (;; ++khi) {
                    const int lim = ip.tb - khi;
                    const uint64_t above = lim >= 64 ? 0 : (qm & ~((1ull << lim) - 1));
                    if (__builtin_popcountll(above) == khi) break;
                }
                r.khi = khi;
                r.W = ip.tb - khi;
                int pos[64];
                int h = 0;
                for (int q = 0; q < ip.n; ++q) {
                    if (!((qm >> q) & 1ull)) continue;
                    if (q < r.W) pos[q] = q;
                    else { r.qhi[h] = (uint8_t)q; pos[q] = r.W + h; ++h; }
                }
                // sweeps: consecutive gates on at most three tile bits (padded
                // with the lowest other tile bits to exactly three)
                r.sg0 = (uint32_t)segs.size();
                r.sw0 = (uint32_t)sweeps.size();
                int nparam = 0;
                size_t gi = 0;
                while (gi < gl.size()) {
                    uint32_t bits = 0;
                    size_t gj = gi;
                    for (; gj < gl.size(); ++gj) {
                        const int l = gl[gj];
                        uint32_t gb = 1u << pos[ip.sq0[l]];
                        if (ip.gates[l].k == 2) gb |= 1u << pos[ip.sq1[l]];
                        if (__builtin_popcount(bits | gb) > 3) break;
                        bits |= gb;
                    }
                    for (int t = 0; __builtin_popcount(bits) < 3 && t < ip.tb; ++t) bits |= 1u << t;
                    SegSweep sw;
                    memset(&sw, 0, sizeof sw);
                    int loc[32];
                    for (int t = 0, c = 0; t < ip.tb; ++t)
                        if ((bits >> t) & 1u) sw.b[c] = t, loc[t] = c++;
                    sw.g0 = (uint32_t)segs.size();
                    sw.p0 = nparam;
                    for (size_t q = gi; q < gj; ++q) {
                        const int l = gl[q];
                        SegGate sgt;
                        memset(&sgt, 0, sizeof sgt);
                        const int k = ip.gates[l].k;
                        const int t0 = loc[pos[ip.sq0[l]]];
                        const int t1 = k == 2 ? loc[pos[ip.sq1[l]]] : -1;
                        sgt.slot = op.kind == BK_ADJ ? ip.gslot[l] : -1;
                        // generator masks: gate-local bit 0 / 1 -> sweep bits t0 / t1
                        uint32_t xl = 0, zl = 0;
                        for (int bb = 0; bb < k; ++bb) {
                            const int sb = bb == 0 ? t0 : t1;
                            if ((ip.xl[l] >> bb) & 1u) xl |= 1u << sb;
                            if ((ip.zl[l] >> bb) & 1u) zl |= 1u << sb;
                        }
                        // sign pattern: gate-local index -> sweep bits t0 / t1 stay in
                        // the same order (bit 0 <-> t0 < t1 <-> bit 1)
                        sgt.info = seg_info(k, t0, t1, ip.form[l], xl, zl, sgt.slot >= 0, ip.neg[l]);
                        sgt.mat = (uint32_t)(op.kind == BK_FWD ? ip.mat_fwd[l] : ip.mat_adj[l]);
                        if (sgt.slot >= 0) ++nparam;
                        segs.push_back(sgt);
                    }
                    sw.g1 = (uint32_t)segs.size();
                    sweeps.push_back(sw);
                    gi = gj;
                }
                r.sg1 = (uint32_t)segs.size();
                r.sw1 = (uint32_t)sweeps.size();
                r.slot = -1;
            }
            recs.push_back(r);
            items += ip.wgs;
        }
        if (items > 0x7fffffffull) return bail(fail(CAST_EUNSUPPORTED, "too many work items in one step"));
        b->step_items.push_back(items);
        {
            // LDS of this step's launch: the tables, then one tile (forward) or
            // two (adjoint: psi and lambda) of its largest tile
            int tbs = 0, tiles = 0;
            for (size_t q = b->step_rec.back(); q < recs.size(); ++q) {
                if (recs[q].kind == BK_HPSI) continue;
                tbs = std::max(tbs, recs[q].tb);
                tiles = std::max(tiles, recs[q].kind == BK_ADJ ? 2 : 1);
            }
            b->step_lds.push_back(kSegLdsExtra + (size_t)tiles * ((size_t)1 << tbs) * amp_bytes(dt));
        }
        item_base += items;
    }
    }
    b->nsteps = (int)b->step_items.size();
    b->step_rec.push_back(recs.size());
    b->step_item.push_back(item_base);
    b->total_items = item_base;
    // ---- device and pinned buffers
    const size_t rsz = dt == CAST_C128 ? 8 : 4;
    const size_t ab = amp_bytes(dt);
    if (cast_status rc = dev_alloc(&b->states, state_elems * ab)) return bail(rc);
    size_t off = 0;
    for (int i = 0; i < n_inst; ++i) {
        const size_t N = (size_t)1 << hinst[i].n;
        hinst[i].psi = (char *)b->states + off * ab;
        hinst[i].lam = (char *)b->states + (off + N) * ab;
        off += 2 * N;
    }
    if (cast_status rc = upload(&b->d_recs, recs)) return bail(rc);
    if (cast_status rc = upload(&b->d_segs, segs)) return bail(rc);
    if (cast_status rc = upload(&b->d_sweeps, sweeps)) return bail(rc);
    {
        int tbm = 0;
        for (auto &ip : b->inst) tbm = std::max(tbm, ip.tb);
        b->lds_bytes = 2 * ((size_t)1 << tbm) * amp_bytes(dt) + kSegLdsExtra;
    }
    if (cast_status rc = upload(&b->d_step_rec, b->step_rec)) return bail(rc);
    if (cast_status rc = upload(&b->d_step_item, b->step_item)) return bail(rc);
    if (cast_status rc = upload(&b->d_insts, hinst)) return bail(rc);
    if (cast_status rc = upload(&b->d_tg, tg)) return bail(rc);
    if (cast_status rc = upload(&b->d_tt, tt)) return bail(rc);
    if (cast_status rc = dev_alloc(&b->d_mats, std::max<size_t>(1, mat_entries) * 2 * rsz)) return bail(rc);
    if (cast_status rc = dev_alloc((void **)&b->d_partials, std::max<uint64_t>(1, part) * sizeof(double)))
        return bail(rc);
    if (cast_status rc = dev_alloc((void **)&b->d_results, std::max<uint64_t>(1, res) * sizeof(double)))
        return bail(rc);
    if (cast_status rc = dev_alloc((void **)&b->d_counters, (2 + (size_t)n_inst) * sizeof(unsigned long long)))
        return bail(rc);
    if (hipHostMalloc(&b->h_mats, std::max<size_t>(1, mat_entries) * 2 * rsz) != hipSuccess)
        return bail(fail(CAST_ENOMEM, "pinned matrix buffer"));
    if (hipHostMalloc((void **)&b->h_results, (res + 1) * sizeof(double)) != hipSuccess)
        return bail(fail(CAST_ENOMEM, "pinned result buffer"));
    for (auto &ip : b->inst)
        for (size_t l = 0; l < ip.gates.size(); ++l) {
            put_matrix(b, ip.mat_fwd[l], ip.fixed[l].data(), false, ip.gates[l].k, ip.form[l], ip.xl[l], ip.zl[l]);
            put_matrix(b, ip.mat_adj[l], ip.fixed[l].data(), true, ip.gates[l].k, ip.form[l], ip.xl[l], ip.zl[l]);
        }
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(CAST_EHIP, "hipStreamCreate failed"));
    BatchDev &d = b->dev;
    d.recs = b->d_recs;
    d.segs = b->d_segs;
    d.sweeps = b->d_sweeps;
    d.step_rec = b->d_step_rec;
    d.step_item = b->d_step_item;
    d.insts = b->d_insts;
    d.mats = b->d_mats;
    d.tg = b->d_tg;
    d.tt = b->d_tt;
    d.partials = b->d_partials;
    d.results = b->d_results;
    d.nsteps = b->nsteps;
    d.ninst = n_inst;
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    b->persistent_grid = cus * 4;
    b->spin_limit = (uint32_t)tuning().persistent_spin_limit[dt == CAST_C64 ? CAST_C64 : CAST_C128];
    if (const char *e = std::getenv("CAST_PERSISTENT_WG_PER_CU")) b->persistent_grid = cus * std::max(1, atoi(e));
    if (const char *e = std::getenv("CAST_PERSISTENT_CHUNK")) b->persistent_chunk = (uint32_t)std::max(1, atoi(e));
    if (mode >= 1) {
        // capture the whole program once; batch_run refreshes the pinned
        // matrices and replays it
        if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return bail(fail(CAST_EHIP, "hipStreamBeginCapture failed"));
        cast_status rc = queue_program(b);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(b->stream, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return bail(rc);
        }
        if (e != hipSuccess) return bail(fail(CAST_EHIP, std::string("graph capture: ") + hipGetErrorString(e)));
        b->graph = g;
        e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) return bail(fail(CAST_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e)));
    }
    *out = b;
    return CAST_OK;
}

cast_status batch_run(cast_batch *b, const double *const *theta, double *energies, double *const *grads) {
    if (!b) return fail(CAST_EINVAL, "batch is NULL");
    if (!energies) return fail(CAST_EINVAL, "energies is NULL");
    for (int i = 0; i < b->ninst; ++i) {
        const InstPlan &ip = b->inst[i];
        if (ip.nparams && (!theta || !theta[i] || !grads || !grads[i]))
            return fail(CAST_EINVAL, "theta/grads missing for an instance with parameters");
    }
    // bind parameters (host FP64, cast once into the pinned buffer)
    for (int i = 0; i < b->ninst; ++i) {
        const InstPlan &ip = b->inst[i];
        for (size_t l = 0; l < ip.gates.size(); ++l) {
            const cast_gate &g = ip.gates[l];
            if (g.param_id < 0) continue;
            const double a = g.param_coeff * theta[i][g.param_id];
            bind_rotation(b, ip.mat_fwd[l], g.k, ip.gen_sorted[l], a, false, ip.form[l], ip.xl[l], ip.zl[l]);
            bind_rotation(b, ip.mat_adj[l], g.k, ip.gen_sorted[l], a, true, ip.form[l], ip.xl[l], ip.zl[l]);
        }
    }
    if (b->mode >= 1) {
        CAST_HIP_TRY(hipGraphLaunch(b->exec, b->stream));
    } else {
        if (cast_status rc = queue_program(b)) return rc;
    }
    CAST_HIP_TRY(hipStreamSynchronize(b->stream));
    if (b->mode == 2) {
        unsigned long long err;
        memcpy(&err, b->h_results + b->result_doubles, sizeof err);
        if (err) return fail(CAST_EHIP, "persistent batch: a dependency wait exceeded its bound");
    }
    for (int i = 0; i < b->ninst; ++i) {
        const InstPlan &ip = b->inst[i];
        size_t off = 0;
        for (int j = 0; j < i; ++j) off += 2 * (size_t)b->inst[j].nslots;
        const double *r = b->h_results + off;
        energies[i] = r[0];
        if (!ip.nparams) continue;
        for (size_t p = 0; p < ip.nparams; ++p) grads[i][p] = 0.0;
        for (size_t l = ip.gates.size(); l-- > 0;) {
            const int s = ip.gslot[l];
            if (s < 0) continue;
            const cplx S(r[2 * s], r[2 * s + 1]);
            const cplx v = kIpowB[__builtin_popcountll(ip.gx[l] & ip.gz[l]) & 3] * S;
            grads[i][ip.gates[l].param_id] += ip.gates[l].param_coeff * v.imag();
        }
    }
    return CAST_OK;
}

void batch_destroy(cast_batch *b) { free_batch(b); }

cast_status adjoint_grad_batch(int n_inst, const int *n_qubits, cast_dtype dt, const cast_gate *const *circuits,
                               const size_t *n_gates, const double *const *theta, const size_t *n_params,
                               const cast_pauli_term *const *hams, const size_t *n_terms, const int *init_kind,
                               const cast_sv *const *init_states, int mode, double *energies, double *const *grads) {
    cast_batch *b = nullptr;
    if (cast_status rc = batch_create(n_inst, n_qubits, dt, circuits, n_gates, n_params, hams, n_terms, init_kind,
                                      init_states, mode, &b))
        return rc;
    cast_status rc = batch_run(b, theta, energies, grads);
    batch_destroy(b);
    return rc;
}

cast_status batch_info(const cast_batch *b, int *n_steps, uint64_t *total_items, double *state_bytes) {
    if (!b) return fail(CAST_EINVAL, "batch is NULL");
    if (n_steps) *n_steps = b->nsteps;
    if (total_items) *total_items = b->total_items;
    if (state_bytes) {
        double s = 0;
        for (auto &ip : b->inst) s += 2.0 * std::ldexp(1.0, ip.n) * (double)amp_bytes(b->dt);
        *state_bytes = s;
    }
    return CAST_OK;
}

cast_status batch_segments(int n, const cast_gate *gates, size_t n_gates, cast_dtype dt, int reverse,
                           size_t *n_segments, int *order, int *segment_of) {
    if (!n_segments) return fail(CAST_EINVAL, "n_segments is NULL");
    if (n_gates && !gates) return fail(CAST_EINVAL, "gates is NULL");
    if (dt != CAST_C64 && dt != CAST_C128) return fail(CAST_EINVAL, "bad dtype");
    if (n < 3 || n > kMaxQubits) return fail(CAST_EINVAL, "qubit count must be in [3, 34]");
    std::vector<uint64_t> gmask(n_gates, 0);
    std::vector<char> gdiag(n_gates, 0);
    for (size_t l = 0; l < n_gates; ++l) {
        const cast_gate &g = gates[l];
        if (g.k < 1 || g.k > 2) return fail(CAST_EUNSUPPORTED, "batched programs take 1- and 2-qubit gates");
        for (int a = 0; a < g.k; ++a) {
            if (g.qubits[a] < 0 || g.qubits[a] >= n) return fail(CAST_EINVAL, "gate qubit out of range");
            gmask[l] |= 1ull << g.qubits[a];
        }
        bool diag = true;
        if (g.param_id >= 0) {
            for (int a = 0; a < g.k; ++a) {
                const int letter = (g.generator >> (2 * a)) & 3;
                if (letter == 1 || letter == 2) diag = false;
            }
        } else {
            if (!g.matrix) return fail(CAST_EINVAL, "fixed gate without a matrix");
            const int D = 1 << g.k;
            for (int r = 0; r < D; ++r)
                for (int c = 0; c < D; ++c)
                    if (r != c && (g.matrix[2 * (r * D + c)] != 0.0 || g.matrix[2 * (r * D + c) + 1] != 0.0)) diag = false;
        }
        gdiag[l] = diag;
    }
    const std::vector<std::vector<int>> segs =
        segment_gates(gmask, gdiag, std::min(n, batch_tile_bits(dt)), reverse != 0, batch_reorder(),
                      batch_min_window(dt, std::min(n, batch_tile_bits(dt))));
    *n_segments = segs.size();
    size_t i = 0;
    for (size_t sgi = 0; sgi < segs.size(); ++sgi)
        for (int l : segs[sgi]) {
            if (order) order[i] = l;
            if (segment_of) segment_of[i] = (int)sgi;
            ++i;
        }
    return CAST_OK;
}

cast_status batch_traffic(const cast_batch *b, double *alg_bytes, uint64_t *state_passes) {
    if (!b) return fail(CAST_EINVAL, "batch is NULL");
    double bytes = 0;
    uint64_t passes = 0;
    for (auto &ip : b->inst) {
        const double S = std::ldexp(1.0, ip.n) * (double)amp_bytes(b->dt);
        bytes += S;                           // initial state written
        for (auto &op : ip.ops) {
            if (op.kind == BK_ADJ) {          // psi and lambda read and written
                bytes += 4 * S;
                passes += 2;
            } else {                          // FWD: psi read and written; HPSI: psi read, lambda written
                bytes += 2 * S;
                passes += 1;
            }
        }
    }
    if (alg_bytes) *alg_bytes = bytes;
    if (state_passes) *state_passes = passes;
    return CAST_OK;
}

}  // extern "C"
