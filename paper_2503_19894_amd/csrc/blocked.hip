// Segment kernel of the cache-blocked executor: one workgroup per tile (see
// blocked.hpp).  The tile is staged through LDS with the same XOR swizzle as
// the single-gate tile kernel (16-byte chunk c at chunk c ^ hash(c / 16)), so
// coalesced load/store phases and power-of-two-strided group reads are both
// free of bank conflicts.
#include <hip/hip_runtime.h>

#include "blocked.hpp"
#include "internal.hpp"

namespace cast {
namespace {

template <typename R> struct Cx;
template <> struct Cx<double> { using T = double2; };
template <> struct Cx<float> { using T = float2; };
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t swz(uint32_t c) { return c ^ (((c >> 4) ^ (c >> 8)) & 15u); }

template <int S>   // S = log2(amplitudes per 16-byte chunk)
__device__ __forceinline__ uint32_t at(uint32_t y) {
    return (swz(y >> S) << S) | (y & ((1u << S) - 1));
}

// Inserts a zero bit at each position (1 << pos) - 1 = lowmask[i], ascending.
__device__ __forceinline__ uint64_t deposit_bits(uint64_t g, const uint64_t *lowmask, int k) {
    for (int i = 0; i < k; ++i) g = ((g & ~lowmask[i]) << 1) | (g & lowmask[i]);
    return g;
}

// Global index bits of tile position y (without the tile's base): window
// bits keep their place, tile bit w + i is high qubit i.  Like the coset
// enumeration, the L^-1 map and the LDS swizzle, this map is linear over
// GF(2), so the value at y = lane + uniform splits into a per-lane part
// computed once and a wave-uniform part computed on the scalar unit.
__device__ __forceinline__ uint64_t expand(uint32_t y, const BlkSeg &s) {
    uint64_t x = y & ((1u << s.w) - 1);
    const uint32_t hi = y >> s.w;
    for (int i = 0; i < s.nh; ++i)
        if ((hi >> i) & 1u) x |= 1ull << s.qh[i];
    return x;
}

// Virtual coordinates contributed by the in-tile targets of position y.
__device__ __forceinline__ uint32_t virt(uint32_t y, const BlkGate &g) {
    uint32_t u = 0;
#pragma unroll
    for (int s = 0; s < 6; ++s)
        if (s < g.k && g.tpos[s] >= 0 && ((y >> g.tpos[s]) & 1u)) u ^= g.colv[s];
    return u;
}

// Local index bits contributed by the in-tile targets of position y.
__device__ __forceinline__ uint32_t loc(uint32_t y, const BlkGate &g) {
    uint32_t j = 0;
#pragma unroll
    for (int s = 0; s < 6; ++s)
        if (s < g.k && g.tpos[s] >= 0) j |= ((y >> g.tpos[s]) & 1u) << s;
    return j;
}

// Staging of a gate area in two halves: the matrices (or a diagonal run's
// phase tables) are read from global memory into registers before the
// current gate is applied, so their latency hides behind it, and written to
// LDS afterwards, together with the slot table and this tile's iteration
// tables.
struct Prefetch {
    u4 m[kBlkMaxMatChunks / 256];
};

template <typename R, int NT>
__device__ __forceinline__ void prefetch(Prefetch &pf, const R *mats, const BlkGate *gates, uint32_t gi) {
    const BlkGate &g = gates[gi];
    // 16-byte chunks per phase-table stride: 2^tshift entries of 2 reals
    const uint32_t cshift = g.tshift + (sizeof(R) == 8 ? 0 : -1);
#pragma unroll
    for (int r = 0; r < (int)((kBlkMaxMatChunks + NT - 1) / NT); ++r) {
        const uint32_t i = threadIdx.x + r * NT;
        if (g.kind == 0) {
            const uint32_t t = i >> cshift, o = i & ((1u << cshift) - 1);
            if (t < (uint32_t)g.run) {
                const BlkGate &h = gates[gi + t];
                if (o < (h.mat_reals * (uint32_t)sizeof(R) + 15) / 16)
                    pf.m[r] = reinterpret_cast<const u4 *>(mats + h.mat)[o];
            }
        } else if (i < (g.mat_reals * (uint32_t)sizeof(R) + 15) / 16) {
            pf.m[r] = reinterpret_cast<const u4 *>(mats + g.mat)[i];   // 256-byte aligned
        }
    }
}

template <typename R, int S, int NT>
__device__ __forceinline__ void commit(char *area, const Prefetch &pf, const BlkGate *gates, uint32_t gi,
                                       uint64_t tbase, uint32_t tile_amps) {
    const BlkGate &g = gates[gi];
    u4 *dst = reinterpret_cast<u4 *>(area + kBlkAreaHead);
    uint2 *itab = reinterpret_cast<uint2 *>(area + kBlkIterOff);
    if (g.kind == 0) {
        const uint32_t cshift = g.tshift + (sizeof(R) == 8 ? 0 : -1);
#pragma unroll
        for (int r = 0; r < (int)((kBlkMaxMatChunks + NT - 1) / NT); ++r) {
            const uint32_t i = threadIdx.x + r * NT;
            const uint32_t t = i >> cshift, o = i & ((1u << cshift) - 1);
            if (t < (uint32_t)g.run && o < (gates[gi + t].mat_reals * (uint32_t)sizeof(R) + 15) / 16)
                dst[i] = pf.m[r];
        }
        // per (gate t of the run, iteration i): uniform part of its local index
        const uint32_t iters = tile_amps / NT;
        if (threadIdx.x < (uint32_t)g.run * iters) {
            const uint32_t t = threadIdx.x / iters, i = threadIdx.x % iters;
            const BlkGate &h = gates[gi + t];
            uint32_t juni = 0;
#pragma unroll
            for (int q = 0; q < 6; ++q)
                if (q < h.k && h.tpos[q] < 0 && ((tbase >> h.q[q]) & 1u)) juni |= 1u << q;
            reinterpret_cast<uint32_t *>(area + kBlkJOff)[t * kBlkMaxIters + i] = juni ^ loc(i * NT, h);
            if (t == 0) itab[i] = make_uint2(0u, at<S>(i * NT));
        }
        return;
    }
    if (threadIdx.x < 32) reinterpret_cast<int8_t *>(area)[threadIdx.x] = g.slot[threadIdx.x];
    const uint32_t n16 = (g.mat_reals * (uint32_t)sizeof(R) + 15) / 16;
#pragma unroll
    for (int r = 0; r < (int)((kBlkMaxMatChunks + NT - 1) / NT); ++r) {
        const uint32_t i = threadIdx.x + r * NT;
        if (i < n16) dst[i] = pf.m[r];
    }
    // iteration i covers cosets i*NT + lane; its uniform part is coset i*NT
    const uint32_t items = tile_amps >> g.d;
    if (threadIdx.x < (items + NT - 1) / NT) {
        uint32_t uuni = 0;   // targets outside the tile, fixed by the tile
#pragma unroll
        for (int q = 0; q < 6; ++q)
            if (q < g.k && g.tpos[q] < 0 && ((tbase >> g.q[q]) & 1u)) uuni ^= g.colv[q];
        uint32_t y = threadIdx.x * NT;
        for (int i = 0; i < g.d; ++i) y = ((y & ~g.pivlow[i]) << 1) | (y & g.pivlow[i]);
        itab[threadIdx.x] = make_uint2(uuni ^ virt(y, g), at<S>(y));
    }
}

// A run of M diagonal gates: amplitude y is read once, multiplied by each
// gate's phase D_t[j_t(y)] in order (identity phases are exactly 1), and
// written once.  Instantiated per run length so the phase loop is straight
// code.
template <typename R, int S, int NT, int M>
__device__ __forceinline__ void diag_run_m(typename Cx<R>::T *tile, const char *area, const BlkGate *gates,
                                           uint32_t gi, uint32_t tile_amps) {
    using V = typename Cx<R>::T;
    const int ts = gates[gi].tshift;
    const V *tabs = reinterpret_cast<const V *>(area + kBlkAreaHead);
    const uint2 *itab = reinterpret_cast<const uint2 *>(area + kBlkIterOff);
    const uint32_t *jt = reinterpret_cast<const uint32_t *>(area + kBlkJOff);
    uint32_t jl[M];
#pragma unroll
    for (int t = 0; t < M; ++t) jl[t] = loc(threadIdx.x, gates[gi + t]) | ((uint32_t)t << ts);
    const uint32_t al = at<S>(threadIdx.x);
    const uint32_t iters = tile_amps / NT;
    for (uint32_t i = 0; i < iters; ++i) {
        const uint32_t a = al ^ itab[i].y;
        V x = tile[a];
#pragma unroll
        for (int t = 0; t < M; ++t) {
            const V ph = tabs[jl[t] ^ jt[t * kBlkMaxIters + i]];
            const R re = x.x * ph.x - x.y * ph.y;
            const R im = x.x * ph.y + x.y * ph.x;
            x.x = re;
            x.y = im;
        }
        tile[a] = x;
    }
}

template <typename R, int S, int NT>
__device__ __forceinline__ void diag_run(typename Cx<R>::T *tile, const char *area, const BlkGate *gates,
                                         uint32_t gi, uint32_t tile_amps) {
    switch (gates[gi].run) {
        case 1: diag_run_m<R, S, NT, 1>(tile, area, gates, gi, tile_amps); break;
        case 2: diag_run_m<R, S, NT, 2>(tile, area, gates, gi, tile_amps); break;
        case 3: diag_run_m<R, S, NT, 3>(tile, area, gates, gi, tile_amps); break;
        case 4: diag_run_m<R, S, NT, 4>(tile, area, gates, gi, tile_amps); break;
        case 5: diag_run_m<R, S, NT, 5>(tile, area, gates, gi, tile_amps); break;
        case 6: diag_run_m<R, S, NT, 6>(tile, area, gates, gi, tile_amps); break;
        case 7: diag_run_m<R, S, NT, 7>(tile, area, gates, gi, tile_amps); break;
        default: diag_run_m<R, S, NT, 8>(tile, area, gates, gi, tile_amps); break;
    }
}

// Block gate with 2^D x 2^D blocks: one work item per coset of the span.
// The item's virtual coordinates u = L^-1 j give its block (u >> D; identity
// blocks are skipped) and its place in the block (u mod 2^D), from which the
// block's first element follows.
template <int D, typename R, int S, int NT>
__device__ __forceinline__ void block_in_tile(typename Cx<R>::T *tile, const char *area, const BlkGate &g,
                                              uint32_t tile_amps) {
    using V = typename Cx<R>::T;
    constexpr int N = 1 << D;
    const int8_t *slot = reinterpret_cast<const int8_t *>(area);
    const uint2 *itab = reinterpret_cast<const uint2 *>(area + kBlkIterOff);
    const V *mt = reinterpret_cast<const V *>(area + kBlkAreaHead);
    uint32_t soff[N], sspan[D];
#pragma unroll
    for (int i = 0; i < D; ++i) sspan[i] = at<S>(g.span[i]);
#pragma unroll
    for (int c = 0; c < N; ++c) {
        uint32_t o = 0;
#pragma unroll
        for (int i = 0; i < D; ++i)
            if ((c >> i) & 1) o ^= sspan[i];
        soff[c] = o;
    }
    const uint32_t items = tile_amps >> D;
    uint32_t ylane = threadIdx.x;
#pragma unroll
    for (int i = 0; i < D; ++i) ylane = ((ylane & ~g.pivlow[i]) << 1) | (ylane & g.pivlow[i]);
    const uint32_t ul = virt(ylane, g);
    const uint32_t al = at<S>(ylane);
    const uint32_t iters = (items + NT - 1) / NT;
    for (uint32_t i = 0; i < iters; ++i) {
        if (i * NT + threadIdx.x >= items) break;
        const uint2 e = itab[i];
        const uint32_t u = ul ^ e.x;
        const int sl = slot[u >> D];
        if (sl < 0) continue;
        uint32_t a0 = al ^ e.y;
#pragma unroll
        for (int b = 0; b < D; ++b)
            if ((u >> b) & 1u) a0 ^= sspan[b];
        const V *m = mt + sl * N * N;
        V v[N];
#pragma unroll
        for (int c = 0; c < N; ++c) v[c] = tile[a0 ^ soff[c]];
#pragma unroll
        for (int r = 0; r < N; ++r) {
            R ar = 0, ai = 0;
#pragma unroll
            for (int c = 0; c < N; ++c) {
                const V x = m[r * N + c];
                ar = fma(x.x, v[c].x, ar);
                ar = fma(-x.y, v[c].y, ar);
                ai = fma(x.x, v[c].y, ai);
                ai = fma(x.y, v[c].x, ai);
            }
            V o;
            o.x = ar;
            o.y = ai;
            tile[a0 ^ soff[r]] = o;
        }
    }
}

// MAXD: the largest block dimension the instance handles (segments without
// 8 x 8 blocks use the MAXD = 2 instance, which needs fewer registers; the
// MAXD = 3 instance is held to 128 registers, four waves per SIMD, so that
// two workgroups still share a compute unit).
template <typename R, int NT, int MAXD>
__global__ void __launch_bounds__(NT, MAXD >= 3 ? 4 : 1) k_blocked(R *__restrict__ psi_r, const R *__restrict__ mats,
                                                const BlkGate *__restrict__ gates, BlkSeg s) {
    using V = typename Cx<R>::T;
    constexpr int S = sizeof(V) == 16 ? 0 : 1;
    constexpr int B = 8;                       // chunks in flight per lane
    extern __shared__ u4 lds16[];
    V *tile = reinterpret_cast<V *>(lds16);
    const uint32_t tile_amps = 1u << s.tb;
    char *area0 = reinterpret_cast<char *>(lds16) + (size_t)tile_amps * sizeof(V);
    u4 *p16 = reinterpret_cast<u4 *>(psi_r);
    const uint32_t chunks = tile_amps >> S;
    const uint64_t glane = expand(threadIdx.x << S, s) >> S;
    const uint32_t slane = swz(threadIdx.x);
    for (uint64_t t = blockIdx.x; t < s.ntiles; t += gridDim.x) {
        const uint64_t tbase = deposit_bits(t << s.w, s.hlowmask, s.nh);
        u4 *base16 = p16 + (tbase >> S) + glane;
        // ---- load (chunk c = c0 + lane)
        for (uint32_t c0 = 0; c0 < chunks; c0 += B * NT) {
            u4 buf[B];
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const uint32_t c = c0 + u * NT;
                if (c + threadIdx.x < chunks) buf[u] = __builtin_nontemporal_load(base16 + (expand(c << S, s) >> S));
            }
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const uint32_t c = c0 + u * NT;
                if (c + threadIdx.x < chunks) lds16[slane ^ swz(c)] = buf[u];
            }
        }
        Prefetch pf;
        prefetch<R, NT>(pf, mats, gates, s.g0);
        commit<R, S, NT>(area0, pf, gates, s.g0, tbase, tile_amps);
        __syncthreads();
        // ---- the segment's gates (a diagonal run counts as one), in order;
        // the next one is staged into the other area meanwhile
        uint32_t par = 0;
        for (uint32_t gi = s.g0; gi < s.g1;) {
            const BlkGate &g = gates[gi];
            const uint32_t gn = gi + (g.kind == 0 ? (uint32_t)g.run : 1u);
            char *area = area0 + par * s.area;
            const bool more = gn < s.g1;
            if (more) prefetch<R, NT>(pf, mats, gates, gn);
            if (g.kind == 0) {
                diag_run<R, S, NT>(tile, area, gates, gi, tile_amps);
            } else {
                switch (g.d) {
                    case 1: block_in_tile<1, R, S, NT>(tile, area, g, tile_amps); break;
                    case 2: block_in_tile<2, R, S, NT>(tile, area, g, tile_amps); break;
                    default:
                        if (MAXD >= 3) block_in_tile<3, R, S, NT>(tile, area, g, tile_amps);
                        break;
                }
            }
            if (more) commit<R, S, NT>(area0 + (par ^ 1u) * s.area, pf, gates, gn, tbase, tile_amps);
            __syncthreads();
            gi = gn;
            par ^= 1u;
        }
        // ---- store
        for (uint32_t c0 = 0; c0 < chunks; c0 += B * NT) {
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const uint32_t c = c0 + u * NT;
                if (c + threadIdx.x < chunks)
                    __builtin_nontemporal_store(lds16[slane ^ swz(c)], base16 + (expand(c << S, s) >> S));
            }
        }
        __syncthreads();   // the next tile overwrites LDS
    }
}

template <typename R, int NT, int MAXD>
hipError_t launch_nt(R *psi, const R *mats, const BlkGate *gates, const BlkSeg &s, uint32_t grid, size_t lds,
                     hipStream_t stream) {
    static const hipError_t attr = hipFuncSetAttribute((const void *)k_blocked<R, NT, MAXD>,
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, 128 << 10);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL((k_blocked<R, NT, MAXD>), dim3(grid), dim3(NT), lds, stream, psi, mats, gates, s);
    return hipGetLastError();
}

template <typename R, int MAXD>
hipError_t launch_d(int nt, R *psi, const R *mats, const BlkGate *gates, const BlkSeg &s, uint32_t grid,
                    size_t lds, hipStream_t stream) {
    switch (nt) {
        case 256: return launch_nt<R, 256, MAXD>(psi, mats, gates, s, grid, lds, stream);
        case 512: return launch_nt<R, 512, MAXD>(psi, mats, gates, s, grid, lds, stream);
        default: return launch_nt<R, 1024, MAXD>(psi, mats, gates, s, grid, lds, stream);
    }
}

template <typename R>
hipError_t launch_r(int nt, R *psi, const R *mats, const BlkGate *gates, const BlkSeg &s, uint32_t grid,
                    size_t lds, hipStream_t stream) {
    if (s.maxd >= 3) return launch_d<R, 3>(nt, psi, mats, gates, s, grid, lds, stream);
    return launch_d<R, 2>(nt, psi, mats, gates, s, grid, lds, stream);
}

}  // namespace

cast_status launch_blocked(void *psi, cast_dtype dt, const void *mats, const BlkGate *gates, const BlkSeg &s,
                           hipStream_t stream) {
    const size_t tile = ((size_t)1 << s.tb) * amp_bytes(dt);
    const size_t lds = tile + 2 * (size_t)s.area;
    if (lds > (128u << 10)) return fail(CAST_EUNSUPPORTED, "blocked tile and gate areas exceed 128 KiB of LDS");
    int nt = tuning().blocked_threads[dt];
    while (nt > 256 && ((size_t)1 << s.tb) < (size_t)nt) nt >>= 1;   // at least one amplitude per thread
    uint64_t grid = s.ntiles;
    const uint64_t cap = (uint64_t)tuning().max_grid[dt];
    if (grid > cap) grid = cap;
    const hipError_t e = dt == CAST_C128
        ? launch_r<double>(nt, (double *)psi, (const double *)mats, gates, s, (uint32_t)grid, lds, stream)
        : launch_r<float>(nt, (float *)psi, (const float *)mats, gates, s, (uint32_t)grid, lds, stream);
    if (e != hipSuccess) return fail(CAST_EHIP, std::string("blocked pass launch: ") + hipGetErrorString(e));
    return CAST_OK;
}

}  // namespace cast
