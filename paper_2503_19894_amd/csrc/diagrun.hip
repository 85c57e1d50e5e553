// Diagonal runs: consecutive diagonal fused gates applied in one elementwise
// pass over the state.
//
// A product of diagonal gates is diagonal, and applying it costs one complex
// multiply per amplitude whatever the number of qubits involved, so fusing
// diagonals is never limited by arithmetic the way dense fusion is (Sec.
// III-C prices a pass by its operation count; a diagonal's does not grow with
// its size).  The host multiplies a run of consecutive diagonal fused gates,
// in FP64, into at most kRunMaxTables phase tables over at most 8 qubits
// each; entries within the one-tolerance of 1 are snapped to exactly 1.  The
// kernel multiplies each amplitude by the product of its table entries; an
// amplitude is touched only where some table entry differs from 1.  Identity
// phases are skipped as in the single-gate diagonal kernel: a 128-byte line
// none of whose amplitudes is touched is neither loaded nor stored, and tiles whose selecting high bits give no
// active amplitude are never visited.  Besides the saved passes, this removes
// the partly active lines that a diagonal on low qubits leaves behind: in a
// run, lines idle in one gate are mostly active in another.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.hpp"

namespace cast {

struct DiagRunArgs {
    uint64_t nchunks;        // 16-byte chunks in the state
    uint64_t ntiles;         // active tiles = npat << rest_bits (0: state smaller than a tile)
    uint64_t hlowmask[6];    // per selecting bit (ascending): tile-index bits below it
    int kh;                  // selecting bits
    int rest_bits;
    int pattern_major;
    int spread;
    uint32_t npat;
    uint32_t patoff[64];     // tile-index bits of each active pattern
    int ntab;
    int tk[kRunMaxTables];   // qubits of table g
    int tq[kRunMaxTables][kRunMaxQ];
    uint64_t amask[kRunMaxTables][4];   // bit j of table g: entry j differs from 1
};

namespace {

template <typename R> struct RunAmp;
template <> struct RunAmp<double> { using T = double2; };
template <> struct RunAmp<float> { using T = float2; };
typedef unsigned int run_u4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint64_t run_deposit(uint64_t g, const uint64_t *lowmask, int k) {
    for (int i = 0; i < k; ++i) {
        const uint64_t lm = lowmask[i];
        g = ((g & ~lm) << 1) | (g & lm);
    }
    return g;
}

// Tile number -> XCD: workgroups are dealt to the 8 XCDs round-robin; XOR of
// the 3-bit digits spreads any few-bit pattern of tile numbers evenly.
__device__ __forceinline__ uint64_t run_xcd_spread(uint64_t it) {
    const uint64_t r = it >> 3;
    uint64_t f = 0;
    for (uint64_t y = r; y; y >>= 3) f ^= y;
    return (r << 3) | ((it ^ f) & 7);
}

// Bit j (< 256) of a table's activity mask (four words, kernel arguments).
__device__ __forceinline__ bool run_active(const uint64_t *m, uint32_t j) {
    const uint64_t w = (j & 128u) ? ((j & 64u) ? m[3] : m[2]) : ((j & 64u) ? m[1] : m[0]);
    return (w >> (j & 63u)) & 1ull;
}

template <typename V>
__device__ __forceinline__ V run_cmul(const V &a, const V &b) {
    V r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}

// Tables at entry offsets g * 256 (each table <= 256 entries), so a per-lane
// index part that includes the offset can be OR-ed with a uniform part below
// 2^tk.  LDS_TAB: the tables are staged in LDS once per workgroup; otherwise
// they are read from global memory, where the few KiB they take stay in the
// L1 cache, and a workgroup needs no set-up (so it can take a single tile).
template <typename R, int U, int G, bool LDS_TAB>
__global__ void __launch_bounds__(256) k_diag_run(R *__restrict__ psi_r, const R *__restrict__ tables,
                                                  DiagRunArgs a) {
    using V = typename RunAmp<R>::T;
    constexpr int S = sizeof(V) == 16 ? 0 : 1;   // log2(amplitudes per 16-byte chunk)
    constexpr int A = 1 << S;
    __shared__ V tab_lds[LDS_TAB ? G * 256 : 1];
    const V *tab = LDS_TAB ? tab_lds : reinterpret_cast<const V *>(tables);
    if (LDS_TAB) {
        for (int j = threadIdx.x; j < G * 256; j += 256) {
            V t;
            t.x = tables[2 * j];
            t.y = tables[2 * j + 1];
            tab_lds[j] = t;
        }
        __syncthreads();
    }
    run_u4 *p16 = reinterpret_cast<run_u4 *>(psi_r);
    const int line0 = (int)(threadIdx.x & 56);   // first lane of this lane's 128-byte line
    auto jof = [&](int g, uint64_t x) {
        uint32_t j = 0;
        for (int i = 0; i < a.tk[g]; ++i) j |= (uint32_t)((x >> a.tq[g][i]) & 1u) << i;
        return j;
    };
    // amplitude index = (uniform chunk base << S) + (lane << S) + h with the
    // base a multiple of 256 << S, so each table index splits into a per-lane
    // part (computed once, offset included) and a wave-uniform part
    uint32_t jl[G][A];
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
        for (int h = 0; h < A; ++h) jl[g][h] = ((uint32_t)g << 8) | jof(g, ((uint64_t)threadIdx.x << S) | (uint64_t)h);
    constexpr uint64_t per = 256ull * U;
    const bool spread = a.spread && (a.ntiles & 7) == 0 && (gridDim.x & 7) == 0;
    // Two tiles in flight per workgroup: the loads of the next tile are
    // issued before the current one's table lookups and multiplies, so the
    // lookups (G per amplitude) overlap memory latency instead of adding to
    // it.  A tile's loads depend only on the activity masks (no memory).
    struct Stage {
        run_u4 w[U];
        bool act[U];
        uint32_t hact[U];
        uint32_t ju[U][G];
        uint64_t tile;
    };
    auto issue = [&](uint64_t it, Stage &st) {
        const uint32_t t = (uint32_t)(spread ? run_xcd_spread(it) : it);   // ntiles <= 2^26
        uint32_t rest, pat;
        if (a.pattern_major) {
            rest = t & ((1u << a.rest_bits) - 1);
            pat = t >> a.rest_bits;
        } else {
            rest = t / a.npat;
            pat = t - rest * a.npat;
        }
        st.tile = run_deposit(rest, a.hlowmask, a.kh) | a.patoff[pat];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t c0 = st.tile * per + (uint64_t)u * 256;   // uniform
#pragma unroll
            for (int g = 0; g < G; ++g) st.ju[u][g] = jof(g, c0 << S);
            uint32_t m = 0;
#pragma unroll
            for (int h = 0; h < A; ++h) {
                bool on = false;
#pragma unroll
                for (int g = 0; g < G; ++g) on |= run_active(a.amask[g], (jl[g][h] & 255u) | st.ju[u][g]);
                m |= (uint32_t)on << h;
            }
            st.hact[u] = m;
            st.act[u] = ((__ballot(m != 0) >> line0) & 0xffull) != 0;
            if (st.act[u]) st.w[u] = __builtin_nontemporal_load(p16 + c0 + threadIdx.x);
        }
    };
    // Every amplitude of an active line is multiplied by its phase product:
    // where all entries are 1 the product is exactly 1 and so is the
    // multiply, which saves a divergent branch per amplitude.  With two
    // amplitudes per chunk (complex64) a table without qubit 0 gives both
    // the same entry, read once.
    auto finish = [&](Stage &st) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!st.act[u]) continue;
            V *v = reinterpret_cast<V *>(&st.w[u]);
            V p[A];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                V e[A];
                e[0] = tab[jl[g][0] | st.ju[u][g]];
#pragma unroll
                for (int h = 1; h < A; ++h) {
                    if (a.tq[g][0] != 0) e[h] = e[0];
                    else e[h] = tab[jl[g][h] | st.ju[u][g]];
                }
#pragma unroll
                for (int h = 0; h < A; ++h) p[h] = g ? run_cmul(p[h], e[h]) : e[h];
            }
#pragma unroll
            for (int h = 0; h < A; ++h) v[h] = run_cmul(v[h], p[h]);
            __builtin_nontemporal_store(st.w[u], p16 + st.tile * per + (uint64_t)u * 256 + threadIdx.x);
        }
    };
    uint64_t it = blockIdx.x;
    if (it < a.ntiles) {
        Stage s0, s1;
        issue(it, s0);
        for (;;) {
            const uint64_t i1 = it + gridDim.x;
            const bool more1 = i1 < a.ntiles;   // uniform
            if (more1) issue(i1, s1);
            finish(s0);
            if (!more1) break;
            const uint64_t i2 = i1 + gridDim.x;
            const bool more2 = i2 < a.ntiles;
            if (more2) issue(i2, s0);
            finish(s1);
            if (!more2) break;
            it = i2;
        }
    }
    // a state smaller than one tile: one chunk per lane (8-lane groups are
    // still whole lines)
    if (a.ntiles) return;
    for (uint64_t c = (uint64_t)blockIdx.x * 256 + threadIdx.x; c < a.nchunks; c += (uint64_t)gridDim.x * 256) {
        V p[A];
        uint32_t m = 0;
#pragma unroll
        for (int h = 0; h < A; ++h) {
            const uint64_t x = (c << S) | (uint64_t)h;
            V q = tab[jof(0, x)];
            bool on = q.x != (R)1 || q.y != (R)0;
#pragma unroll
            for (int g = 1; g < G; ++g) {
                const V e = tab[((uint32_t)g << 8) | jof(g, x)];
                on |= e.x != (R)1 || e.y != (R)0;
                q = run_cmul(q, e);
            }
            p[h] = q;
            m |= (uint32_t)on << h;
        }
        if (((__ballot(m != 0) >> line0) & 0xffull) == 0) continue;
        run_u4 wv = p16[c];
        V *v = reinterpret_cast<V *>(&wv);
#pragma unroll
        for (int h = 0; h < A; ++h)
            if ((m >> h) & 1u) v[h] = run_cmul(v[h], p[h]);
        p16[c] = wv;
    }
}

// Phase reuse.  The high amplitude-index bits (above a lane's chunk) split
// into D, the bits some table depends on, and F, the bits no table touches.
// Amplitudes that differ only in F bits get the same phase, so a work unit
// takes one pattern of the D bits and 2^c patterns of the F bits: each lane
// looks its phase product up once (G table reads) and then streams 2^c
// chunks, one complex multiply per amplitude.  Line-level skipping is as
// above (the activity of a line does not depend on F bits either).
struct DiagReuseArgs {
    uint64_t nunits;        // D patterns x blocks of 2^c F patterns
    int nd, nf, c;          // dependent and free high bits; log2 F patterns per unit
    int dpos[40];           // amplitude-index positions of the D bits (ascending)
    int fpos[40];           // amplitude-index positions of the F bits (ascending)
    int ntab;
    int tk[kRunMaxTables];
    int tq[kRunMaxTables][kRunMaxQ];
    int rot, it_bits;       // units visited in an order rotated left by rot of it_bits bits (0: in order)
};

template <typename R, int G, bool LDS_TAB, int UI>
__global__ void __launch_bounds__(256) k_diag_run_reuse(R *__restrict__ psi_r, const R *__restrict__ tables,
                                                        DiagReuseArgs a) {
    using V = typename RunAmp<R>::T;
    constexpr int S = sizeof(V) == 16 ? 0 : 1;   // log2(amplitudes per 16-byte chunk)
    constexpr int A = 1 << S;
    __shared__ V tab_lds[LDS_TAB ? G * 256 : 1];
    const V *tab = LDS_TAB ? tab_lds : reinterpret_cast<const V *>(tables);
    if (LDS_TAB) {
        for (int j = threadIdx.x; j < G * 256; j += 256) {
            V t;
            t.x = tables[2 * j];
            t.y = tables[2 * j + 1];
            tab_lds[j] = t;
        }
        __syncthreads();
    }
    run_u4 *p16 = reinterpret_cast<run_u4 *>(psi_r);
    const int line0 = (int)(threadIdx.x & 56);
    auto jof = [&](int g, uint64_t x) {
        uint32_t j = 0;
        for (int i = 0; i < a.tk[g]; ++i) j |= (uint32_t)((x >> a.tq[g][i]) & 1u) << i;
        return j;
    };
    uint32_t jl[G][A];
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
        for (int h = 0; h < A; ++h) jl[g][h] = ((uint32_t)g << 8) | jof(g, ((uint64_t)threadIdx.x << S) | (uint64_t)h);
    const uint32_t nin = 1u << a.c;
    const int bshift = a.nf - a.c;
    for (uint64_t unit0 = blockIdx.x; unit0 < a.nunits; unit0 += gridDim.x) {
        // nunits is 2^it_bits when rot > 0
        const uint64_t unit =
            a.rot ? (((unit0 << a.rot) | (unit0 >> (a.it_bits - a.rot))) & (a.nunits - 1)) : unit0;
        const uint64_t o = unit >> bshift, b = unit & ((1ull << bshift) - 1);
        uint64_t xo = 0, xb = 0;   // uniform
        for (int i = 0; i < a.nd; ++i) xo |= ((o >> i) & 1ull) << a.dpos[i];
        for (int i = a.c; i < a.nf; ++i) xb |= ((b >> (i - a.c)) & 1ull) << a.fpos[i];
        V p[A];
        bool on = false;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const uint32_t ju = jof(g, xo);
#pragma unroll
            for (int h = 0; h < A; ++h) {
                const V e = tab[jl[g][h] | ju];
                on |= e.x != (R)1 || e.y != (R)0;
                p[h] = g ? run_cmul(p[h], e) : e;
            }
        }
        const uint64_t bal = __ballot(on);
        if (!bal) continue;                                 // no active line in this wave
        const bool act = ((bal >> line0) & 0xffull) != 0;   // this lane's line
        const uint64_t cbase = ((xo | xb) >> S) + threadIdx.x;
        for (uint32_t j0 = 0; j0 < nin; j0 += UI) {
            run_u4 w[UI];
            uint64_t ci[UI];
#pragma unroll
            for (int u = 0; u < UI; ++u) {
                const uint32_t j = j0 + u;
                uint64_t xj = 0;
                for (int i = 0; i < a.c; ++i) xj |= (uint64_t)((j >> i) & 1u) << a.fpos[i];
                ci[u] = cbase + (xj >> S);
                if (j < nin && act) w[u] = __builtin_nontemporal_load(p16 + ci[u]);
            }
#pragma unroll
            for (int u = 0; u < UI; ++u) {
                if (j0 + u >= nin || !act) continue;
                V *v = reinterpret_cast<V *>(&w[u]);
#pragma unroll
                for (int h = 0; h < A; ++h) v[h] = run_cmul(v[h], p[h]);
                __builtin_nontemporal_store(w[u], p16 + ci[u]);
            }
        }
    }
}

template <typename R, int G, int UI>
hipError_t launch_reuse_g(bool lds, R *psi, const R *tabs, const DiagReuseArgs &a, int grid, hipStream_t s) {
    if (lds) hipLaunchKernelGGL((k_diag_run_reuse<R, G, true, UI>), dim3(grid), dim3(256), 0, s, psi, tabs, a);
    else hipLaunchKernelGGL((k_diag_run_reuse<R, G, false, UI>), dim3(grid), dim3(256), 0, s, psi, tabs, a);
    return hipGetLastError();
}

template <typename R, int UI>
hipError_t launch_reuse_u(int G, bool lds, R *psi, const R *tabs, const DiagReuseArgs &a, int grid, hipStream_t s) {
    switch (G) {
        case 1: return launch_reuse_g<R, 1, UI>(lds, psi, tabs, a, grid, s);
        case 2: return launch_reuse_g<R, 2, UI>(lds, psi, tabs, a, grid, s);
        case 3: return launch_reuse_g<R, 3, UI>(lds, psi, tabs, a, grid, s);
        case 4: return launch_reuse_g<R, 4, UI>(lds, psi, tabs, a, grid, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename R>
hipError_t launch_reuse(int UI, int G, bool lds, R *psi, const R *tabs, const DiagReuseArgs &a, int grid,
                        hipStream_t s) {
    switch (UI) {
        case 1: return launch_reuse_u<R, 1>(G, lds, psi, tabs, a, grid, s);
        case 2: return launch_reuse_u<R, 2>(G, lds, psi, tabs, a, grid, s);
        case 4: return launch_reuse_u<R, 4>(G, lds, psi, tabs, a, grid, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename R, int U, bool L>
hipError_t launch_run_u(int G, R *psi, const R *tabs, const DiagRunArgs &a, int grid, hipStream_t s) {
    switch (G) {
        case 1: hipLaunchKernelGGL((k_diag_run<R, U, 1, L>), dim3(grid), dim3(256), 0, s, psi, tabs, a); break;
        case 2: hipLaunchKernelGGL((k_diag_run<R, U, 2, L>), dim3(grid), dim3(256), 0, s, psi, tabs, a); break;
        case 3: hipLaunchKernelGGL((k_diag_run<R, U, 3, L>), dim3(grid), dim3(256), 0, s, psi, tabs, a); break;
        case 4: hipLaunchKernelGGL((k_diag_run<R, U, 4, L>), dim3(grid), dim3(256), 0, s, psi, tabs, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename R>
hipError_t launch_run(int U, bool lds, int G, R *psi, const R *tabs, const DiagRunArgs &a, int grid,
                      hipStream_t s) {
    switch (U * 2 + (lds ? 1 : 0)) {
        case 2: return launch_run_u<R, 1, false>(G, psi, tabs, a, grid, s);
        case 3: return launch_run_u<R, 1, true>(G, psi, tabs, a, grid, s);
        case 4: return launch_run_u<R, 2, false>(G, psi, tabs, a, grid, s);
        case 5: return launch_run_u<R, 2, true>(G, psi, tabs, a, grid, s);
        case 8: return launch_run_u<R, 4, false>(G, psi, tabs, a, grid, s);
        case 9: return launch_run_u<R, 4, true>(G, psi, tabs, a, grid, s);
        default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------------ host

bool snapped_one(const cplx &z) { return z == cplx(1.0, 0.0); }

cplx snap_one(cplx z, double tol) {
    if (std::fabs(z.real() - 1.0) <= tol && std::fabs(z.imag()) <= tol) return cplx(1.0, 0.0);
    return z;
}

// Bits of local index j over `from` (sorted qubits), placed at the positions
// those qubits have in `to` (sorted superset).
uint32_t move_bits(uint32_t j, const int *from, int kf, const int *to, int kt) {
    uint32_t o = 0;
    for (int i = 0; i < kf; ++i) {
        if (!((j >> i) & 1u)) continue;
        for (int t = 0; t < kt; ++t)
            if (to[t] == from[i]) o |= 1u << t;
    }
    return o;
}

// Diagonal of a plan as a table (bit i <-> sorted qubit p.q[i]).
PhaseTable table_of(const PassPlan &p) {
    PhaseTable t;
    t.k = p.k;
    for (int i = 0; i < p.k; ++i) t.q[i] = p.q[i];
    const size_t D = (size_t)1 << p.k;
    t.ph.resize(D);
    for (size_t j = 0; j < D; ++j) t.ph[j] = p.full[j * D + j];
    return t;
}

// Union of two sorted qubit lists.
int qubit_union(const int *a, int ka, const int *b, int kb, int *out) {
    int n = 0, i = 0, j = 0;
    while (i < ka || j < kb) {
        int v;
        if (j >= kb || (i < ka && a[i] < b[j])) v = a[i++];
        else if (i >= ka || b[j] < a[i]) v = b[j++];
        else v = a[i++], ++j;
        out[n++] = v;
    }
    return n;
}

PhaseTable combine(const PhaseTable &a, const PhaseTable &b, double tol) {
    PhaseTable t;
    int u[2 * kRunMaxQ];
    t.k = qubit_union(a.q, a.k, b.q, b.k, u);
    for (int i = 0; i < t.k; ++i) t.q[i] = u[i];
    const uint32_t D = 1u << t.k;
    t.ph.resize(D);
    for (uint32_t j = 0; j < D; ++j) {
        // bits of j at a's and b's qubits
        uint32_t ja = 0, jb = 0;
        for (int i = 0; i < a.k; ++i)
            for (int s = 0; s < t.k; ++s)
                if (t.q[s] == a.q[i] && ((j >> s) & 1u)) ja |= 1u << i;
        for (int i = 0; i < b.k; ++i)
            for (int s = 0; s < t.k; ++s)
                if (t.q[s] == b.q[i] && ((j >> s) & 1u)) jb |= 1u << i;
        t.ph[j] = snap_one(a.ph[ja] * b.ph[jb], tol);
    }
    return t;
}

// Qubits that lie in two or more of the tables.
std::vector<int> overlap_qubits(const std::vector<PhaseTable> &tabs) {
    std::vector<int> cnt(64, 0), o;
    for (auto &t : tabs)
        for (int i = 0; i < t.k; ++i) ++cnt[t.q[i]];
    for (int q = 0; q < 64; ++q)
        if (cnt[q] >= 2) o.push_back(q);
    return o;
}

constexpr int kRunMaxOverlap = 12;

// Amplitudes of a 2^n state at which some table has a phase other than 1.
// For each assignment of the shared qubits the tables are independent, so the
// idle count is a product of per-table counts: table t contributes the number
// of its idle entries that agree with the assignment on the shared qubits it
// holds (a histogram over those bits).
double active_amplitudes(const std::vector<PhaseTable> &tabs, int n) {
    const std::vector<int> o = overlap_qubits(tabs);
    const uint32_t no = 1u << o.size();
    int nu = 0;
    {
        std::vector<bool> in(64, false);
        for (auto &t : tabs)
            for (int i = 0; i < t.k; ++i) in[t.q[i]] = true;
        for (int q = 0; q < 64; ++q) nu += in[q];
    }
    std::vector<std::vector<double>> hist(tabs.size());
    std::vector<uint32_t> omask(tabs.size(), 0);
    for (size_t ti = 0; ti < tabs.size(); ++ti) {
        const PhaseTable &t = tabs[ti];
        int pos[kRunMaxQ * kRunMaxTables];
        for (size_t s = 0; s < o.size(); ++s) {
            pos[s] = -1;
            for (int i = 0; i < t.k; ++i)
                if (t.q[i] == o[s]) pos[s] = i, omask[ti] |= 1u << s;
        }
        hist[ti].assign(no, 0.0);
        for (uint32_t j = 0; j < (1u << t.k); ++j) {
            if (!snapped_one(t.ph[j])) continue;
            uint32_t key = 0;
            for (size_t s = 0; s < o.size(); ++s)
                if (pos[s] >= 0 && ((j >> pos[s]) & 1u)) key |= 1u << s;
            hist[ti][key] += 1;
        }
    }
    double idle = 0;
    for (uint32_t asg = 0; asg < no; ++asg) {
        double prod = 1;
        for (size_t ti = 0; ti < tabs.size() && prod != 0; ++ti) prod *= hist[ti][asg & omask[ti]];
        idle += prod;
    }
    return std::ldexp(1.0, n) - idle * std::ldexp(1.0, n - nu);
}

// Tile selection: tiles hold 2^tb amplitudes; up to six union qubits at or
// above tb (those in the most tables, then the highest) select tiles, and
// only patterns of them under which some table has an active entry are
// visited.
void select_tiles(const SchedPass &p, int n, int tb, int pattern_major, cast_dtype dt, DiagRunArgs *a) {
    std::vector<int> cnt(64, 0);
    for (auto &t : p.tabs)
        for (int i = 0; i < t.k; ++i)
            if (t.q[i] >= tb) ++cnt[t.q[i]];
    std::vector<int> cand;
    for (int q = 0; q < 64; ++q)
        if (cnt[q]) cand.push_back(q);
    std::sort(cand.begin(), cand.end(), [&](int x, int y) { return cnt[x] != cnt[y] ? cnt[x] > cnt[y] : x > y; });
    if (cand.size() > 6) cand.resize(6);
    std::sort(cand.begin(), cand.end());
    const int kh = (int)cand.size();
    // pattern ph (bit s <-> cand[s]) is active if some table has an active
    // entry agreeing with ph on the selecting qubits it contains
    std::vector<bool> act(1u << kh, false);
    for (auto &t : p.tabs) {
        uint32_t tmask = 0;   // selecting bits this table contains
        for (int s = 0; s < kh; ++s)
            for (int i = 0; i < t.k; ++i)
                if (t.q[i] == cand[s]) tmask |= 1u << s;
        std::vector<bool> key(1u << kh, false);
        for (uint32_t j = 0; j < (1u << t.k); ++j) {
            if (snapped_one(t.ph[j])) continue;
            uint32_t kk = 0;
            for (int s = 0; s < kh; ++s)
                for (int i = 0; i < t.k; ++i)
                    if (t.q[i] == cand[s] && ((j >> i) & 1u)) kk |= 1u << s;
            key[kk] = true;
        }
        for (uint32_t ph = 0; ph < (1u << kh); ++ph)
            if (key[ph & tmask]) act[ph] = true;
    }
    a->kh = kh;
    for (int s = 0; s < kh; ++s) a->hlowmask[s] = (1ull << (cand[s] - tb)) - 1;
    a->rest_bits = (n - tb) - kh;
    a->pattern_major = pattern_major;
    a->spread = tuning().diag_spread[dt];
    uint32_t npat = 0;
    for (uint32_t ph = 0; ph < (1u << kh); ++ph) {
        if (!act[ph]) continue;
        uint32_t off = 0;
        for (int s = 0; s < kh; ++s)
            if ((ph >> s) & 1u) off |= 1u << (cand[s] - tb);
        a->patoff[npat++] = off;
    }
    a->npat = npat;
    a->ntiles = (uint64_t)npat << a->rest_bits;
}

}  // namespace

bool diag_pass(int n, cast_dtype dt, const PassPlan &p) { return !p.identity() && pass_kernel_kind(n, dt, p) == 3; }

cast_status build_schedule(const std::vector<PassPlan> &plans, int n, cast_dtype dt, Schedule *out) {
    const Tuning &tu = tuning();
    const int G = tu.diag_run_tables[dt], Q = tu.diag_run_qubits[dt];
    out->n = n;
    out->dt = dt;
    out->run_tables = G;
    out->run_qubits = Q;
    out->use_diag = tu.use_diag[dt];
    out->passes.clear();
    const double tol = 1e-14;   // one-tolerance of the combined phases (same as the plans')
    size_t i = 0;
    while (i < plans.size()) {
        const PassPlan &p = plans[i];
        SchedPass sp;
        sp.first = i;
        sp.count = 1;
        if (G == 0 || !diag_pass(n, dt, p)) {
            sp.kind = p.identity() ? -1 : pass_kernel_kind(n, dt, p);
            out->passes.push_back(std::move(sp));
            ++i;
            continue;
        }
        // a run: extend while the next gate is diagonal (or the identity) and
        // fits the last table, or a new table within the limits
        sp.kind = 6;
        sp.count = 0;
        size_t last_diag = i;
        while (i < plans.size()) {
            const PassPlan &q = plans[i];
            if (q.identity()) {
                ++sp.count, ++i;
                continue;
            }
            if (!diag_pass(n, dt, q)) break;
            PhaseTable t = table_of(q);
            if (!sp.tabs.empty()) {
                int u[2 * kRunMaxQ];
                if (qubit_union(sp.tabs.back().q, sp.tabs.back().k, t.q, t.k, u) <= Q) {
                    sp.tabs.back() = combine(sp.tabs.back(), t, tol);
                    last_diag = i;
                    ++sp.count, ++i;
                    continue;
                }
                if ((int)sp.tabs.size() >= G) break;
                std::vector<PhaseTable> trial = sp.tabs;
                trial.push_back(t);
                if ((int)overlap_qubits(trial).size() > kRunMaxOverlap) break;
            }
            sp.tabs.push_back(std::move(t));
            last_diag = i;
            ++sp.count, ++i;
        }
        // trailing identities belong to the next pass
        const size_t end = last_diag + 1;
        i = end;
        size_t ndiag = 0;
        for (size_t g = sp.first; g < end; ++g) ndiag += !plans[g].identity();
        if (ndiag == 1) {
            // a lone diagonal gate keeps the single-gate diagonal kernel
            for (size_t g = sp.first; g < end; ++g) {
                SchedPass one;
                one.first = g;
                one.count = 1;
                one.kind = plans[g].identity() ? -1 : 3;
                out->passes.push_back(std::move(one));
            }
            continue;
        }
        sp.count = end - sp.first;
        sp.active_amps = active_amplitudes(sp.tabs, n);
        out->passes.push_back(std::move(sp));
    }
    return CAST_OK;
}

cast_status upload_schedule(Schedule *s) {
    std::vector<double> hd;
    std::vector<float> hf;
    size_t entries = 0;
    for (SchedPass &p : s->passes) {
        if (p.kind != 6) continue;
        p.tab_off = entries;
        entries += (size_t)p.tabs.size() * 256;
    }
    if (!entries) return CAST_OK;
    const bool c128 = s->dt == CAST_C128;
    if (c128) hd.assign(2 * entries, 0.0);
    else hf.assign(2 * entries, 0.0f);
    for (const SchedPass &p : s->passes) {
        if (p.kind != 6) continue;
        for (size_t g = 0; g < p.tabs.size(); ++g) {
            const PhaseTable &t = p.tabs[g];
            for (size_t j = 0; j < 256; ++j) {
                // unused entries of a table are never indexed; keep them at 1
                const cplx z = j < t.ph.size() ? t.ph[j] : cplx(1.0, 0.0);
                const size_t e = p.tab_off + g * 256 + j;
                if (c128) hd[2 * e] = z.real(), hd[2 * e + 1] = z.imag();
                else hf[2 * e] = (float)z.real(), hf[2 * e + 1] = (float)z.imag();
            }
        }
    }
    const size_t bytes = 2 * entries * (c128 ? sizeof(double) : sizeof(float));
    if (cast_status rc = dev_alloc(&s->dev.ptr, bytes)) return rc;
    s->dev.bytes = bytes;
    const hipError_t e = hipMemcpy(s->dev.ptr, c128 ? (const void *)hd.data() : (const void *)hf.data(), bytes,
                                   hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        dev_free(s->dev.ptr);
        s->dev.ptr = nullptr;
        return fail(CAST_EHIP, std::string("diagonal-run tables upload: ") + hipGetErrorString(e));
    }
    return CAST_OK;
}

cast_status launch_diag_run(void *psi, int n, cast_dtype dt, const SchedPass &p, const void *dtabs,
                            hipStream_t stream) {
    const Tuning &tu = tuning();
    DiagRunArgs a;
    memset(&a, 0, sizeof a);
    a.ntab = (int)p.tabs.size();
    if (a.ntab < 1 || a.ntab > kRunMaxTables) return fail(CAST_EINVAL, "diagonal run: bad table count");
    for (int g = 0; g < a.ntab; ++g) {
        a.tk[g] = p.tabs[g].k;
        for (int i = 0; i < p.tabs[g].k; ++i) a.tq[g][i] = p.tabs[g].q[i];
        for (size_t j = 0; j < p.tabs[g].ph.size(); ++j)
            if (!snapped_one(p.tabs[g].ph[j])) a.amask[g][j >> 6] |= 1ull << (j & 63);
    }
    const int Sb = dt == CAST_C128 ? 0 : 1;
    const int LB = 8 + Sb;   // amplitude-index bits inside one 256-lane tile
    if (tu.diag_run_reuse[dt] > 0 && n > LB) {
        DiagReuseArgs r;
        memset(&r, 0, sizeof r);
        r.ntab = a.ntab;
        uint64_t used = 0;
        for (int g = 0; g < a.ntab; ++g) {
            r.tk[g] = a.tk[g];
            for (int i = 0; i < a.tk[g]; ++i) r.tq[g][i] = a.tq[g][i], used |= 1ull << a.tq[g][i];
        }
        for (int q = LB; q < n; ++q) {
            if ((used >> q) & 1ull) r.dpos[r.nd++] = q;
            else r.fpos[r.nf++] = q;
        }
        r.c = std::min(r.nf, tu.diag_run_reuse[dt]);
        r.nunits = 1ull << (n - LB - r.c);
        // the pass's launch shape: units in rotated order
        if (p.shape.rot > 0 && p.shape.rot < n - LB - r.c) {
            r.rot = p.shape.rot;
            r.it_bits = n - LB - r.c;
        }
        uint64_t grid = std::min<uint64_t>(r.nunits, (uint64_t)tu.diag_run_grid[dt]);
        const size_t off = p.tab_off * 2;
        const bool lds = tu.diag_run_lds[dt] != 0;
        const int UI = tu.diag_run_unroll[dt];
        hipError_t e;
        if (dt == CAST_C128)
            e = launch_reuse<double>(UI, r.ntab, lds, (double *)psi, (const double *)dtabs + off, r, (int)grid, stream);
        else
            e = launch_reuse<float>(UI, r.ntab, lds, (float *)psi, (const float *)dtabs + off, r, (int)grid, stream);
        if (e != hipSuccess) return fail(CAST_EHIP, std::string("diagonal run launch: ") + hipGetErrorString(e));
        return CAST_OK;
    }
    a.nchunks = ((uint64_t)1 << n) * amp_bytes(dt) / 16;
    if (a.nchunks == 0) a.nchunks = 1;   // c64, n = 1
    const int U = tu.diag_run_unroll[dt];
    const uint64_t per = 256ull * U;
    uint64_t grid = (a.nchunks + per - 1) / per;
    if (a.nchunks >= per) {
        const int S = dt == CAST_C128 ? 0 : 1;
        int tb = S;
        while ((1ull << (tb - S)) < per) ++tb;
        select_tiles(p, n, tb, tu.diag_order[dt], dt, &a);
        grid = a.ntiles;
        if (grid == 0) return CAST_OK;   // every combined phase is 1
    }
    if (grid > (uint64_t)tu.diag_run_grid[dt]) grid = tu.diag_run_grid[dt];
    const size_t off = p.tab_off * 2;
    hipError_t e;
    const bool lds = tu.diag_run_lds[dt] != 0;
    if (dt == CAST_C128)
        e = launch_run<double>(U, lds, a.ntab, (double *)psi, (const double *)dtabs + off, a, (int)grid, stream);
    else
        e = launch_run<float>(U, lds, a.ntab, (float *)psi, (const float *)dtabs + off, a, (int)grid, stream);
    if (e != hipSuccess) return fail(CAST_EHIP, std::string("diagonal run launch: ") + hipGetErrorString(e));
    return CAST_OK;
}

void schedule_free(Schedule *s) {
    if (!s) return;
    dev_free(s->dev.ptr);
    delete s;
}

}  // namespace cast
