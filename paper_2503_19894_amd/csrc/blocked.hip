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

// Global index of tile position y: window bits keep their place, tile bit
// w + i is high qubit i.
__device__ __forceinline__ uint64_t global_of(uint64_t tbase, uint32_t y, const BlkSeg &s) {
    uint64_t x = tbase | (y & ((1u << s.w) - 1));
    const uint32_t hi = y >> s.w;
    for (int i = 0; i < s.nh; ++i)
        if ((hi >> i) & 1u) x |= 1ull << s.qh[i];
    return x;
}

// Diagonal gate: amplitude y gets phase D[j], j = its bits at the targets.
// y = threadIdx.x + 256 i, so the targets on tile bits < 8 give a per-lane
// part of j and those on higher tile bits a part uniform per iteration.
template <typename R, int S>
__device__ __forceinline__ void diag_in_tile(typename Cx<R>::T *tile, const R *mats, const BlkGate &g,
                                             uint32_t juni, int tb) {
    using V = typename Cx<R>::T;
    uint32_t jl = juni, lane_bits = 0;
    for (int s = 0; s < g.k; ++s) {
        const int p = g.tpos[s];
        if (p >= 0 && p < 8) jl |= ((threadIdx.x >> p) & 1u) << s;
        if (p >= 8) lane_bits |= 1u << s;
    }
    const V *tab = reinterpret_cast<const V *>(mats + g.mat);
    const uint32_t iters = 1u << (tb - 8);
    for (uint32_t i = 0; i < iters; ++i) {
        uint32_t j = jl;
        if (lane_bits)
            for (int s = 0; s < g.k; ++s)
                if (g.tpos[s] >= 8) j |= ((i >> (g.tpos[s] - 8)) & 1u) << s;
        if (!((g.amask >> j) & 1u)) continue;
        const uint32_t y = threadIdx.x + (i << 8);
        V &a = tile[at<S>(y)];
        const V t = tab[j];
        const R re = a.x * t.x - a.y * t.y;
        const R im = a.x * t.y + a.y * t.x;
        a.x = re;
        a.y = im;
    }
}

// Block gate with 2^D x 2^D blocks: one work item per coset of the span
// (tile positions y with zeros at the pivot bits).  The item's virtual
// coordinates u = L^-1 j give the block (u >> D) and the item's place in it
// (u mod 2^D); identity blocks are skipped.
template <int D, typename R, int S>
__device__ __forceinline__ void block_in_tile(typename Cx<R>::T *tile, const R *mats, const BlkGate &g,
                                              uint32_t uuni, int tb) {
    using V = typename Cx<R>::T;
    constexpr int N = 1 << D;
    uint32_t off[N];
#pragma unroll
    for (int c = 0; c < N; ++c) {
        uint32_t o = 0;
#pragma unroll
        for (int i = 0; i < D; ++i)
            if ((c >> i) & 1) o ^= g.span[i];
        off[c] = o;
    }
    const uint32_t items = 1u << (tb - D);
    for (uint32_t it = threadIdx.x; it < items; it += 256) {
        uint32_t y = it;
#pragma unroll
        for (int i = 0; i < D; ++i) y = ((y & ~g.pivlow[i]) << 1) | (y & g.pivlow[i]);
        uint32_t u = uuni;
        for (int s = 0; s < g.k; ++s)
            if (g.tpos[s] >= 0 && ((y >> g.tpos[s]) & 1u)) u ^= g.colv[s];
        const int sl = g.slot[u >> D];
        if (sl < 0) continue;
        const uint32_t within = u & (N - 1);
        uint32_t b = y;
#pragma unroll
        for (int i = 0; i < D; ++i)
            if ((within >> i) & 1u) b ^= g.span[i];
        const R *m = mats + g.mat + (size_t)sl * (2 * N * N);
        V v[N];
#pragma unroll
        for (int c = 0; c < N; ++c) v[c] = tile[at<S>(b ^ off[c])];
#pragma unroll
        for (int r = 0; r < N; ++r) {
            R ar = 0, ai = 0;
#pragma unroll
            for (int c = 0; c < N; ++c) {
                const R mr = m[2 * (r * N + c)], mi = m[2 * (r * N + c) + 1];
                ar = fma(mr, v[c].x, ar);
                ar = fma(-mi, v[c].y, ar);
                ai = fma(mr, v[c].y, ai);
                ai = fma(mi, v[c].x, ai);
            }
            V o;
            o.x = ar;
            o.y = ai;
            tile[at<S>(b ^ off[r])] = o;
        }
    }
}

template <typename R>
__global__ void __launch_bounds__(256) k_blocked(R *__restrict__ psi_r, const R *__restrict__ mats,
                                                 const BlkGate *__restrict__ gates, BlkSeg s) {
    using V = typename Cx<R>::T;
    constexpr int S = sizeof(V) == 16 ? 0 : 1;
    extern __shared__ u4 lds16[];
    V *tile = reinterpret_cast<V *>(lds16);
    u4 *p16 = reinterpret_cast<u4 *>(psi_r);
    const uint32_t chunks = 1u << (s.tb - S);
    for (uint64_t t = blockIdx.x; t < s.ntiles; t += gridDim.x) {
        const uint64_t tbase = deposit_bits(t << s.w, s.hlowmask, s.nh);
        // ---- load: 8 chunks in flight per lane
        for (uint32_t c0 = threadIdx.x; c0 < chunks; c0 += 8 * 256) {
            u4 buf[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const uint32_t c = c0 + u * 256;
                if (c < chunks) buf[u] = __builtin_nontemporal_load(p16 + (global_of(tbase, c << S, s) >> S));
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const uint32_t c = c0 + u * 256;
                if (c < chunks) lds16[swz(c)] = buf[u];
            }
        }
        __syncthreads();
        // ---- the segment's gates, in order
        for (uint32_t gi = s.g0; gi < s.g1; ++gi) {
            const BlkGate &g = gates[gi];
            // contribution of the targets outside the tile (fixed by the tile)
            uint32_t juni = 0, uuni = 0;
            for (int q = 0; q < g.k; ++q)
                if (g.tpos[q] < 0 && ((tbase >> g.q[q]) & 1u)) juni |= 1u << q, uuni ^= g.colv[q];
            if (g.kind == 0) {
                diag_in_tile<R, S>(tile, mats, g, juni, s.tb);
            } else {
                switch (g.d) {
                    case 1: block_in_tile<1, R, S>(tile, mats, g, uuni, s.tb); break;
                    case 2: block_in_tile<2, R, S>(tile, mats, g, uuni, s.tb); break;
                    default: block_in_tile<3, R, S>(tile, mats, g, uuni, s.tb); break;
                }
            }
            __syncthreads();
        }
        // ---- store
        for (uint32_t c0 = threadIdx.x; c0 < chunks; c0 += 8 * 256) {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const uint32_t c = c0 + u * 256;
                if (c < chunks) __builtin_nontemporal_store(lds16[swz(c)], p16 + (global_of(tbase, c << S, s) >> S));
            }
        }
        __syncthreads();   // the next tile overwrites LDS
    }
}

template <typename R>
hipError_t allow_lds() {
    static hipError_t done = hipFuncSetAttribute((const void *)k_blocked<R>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, 128 << 10);
    return done;
}

}  // namespace

cast_status launch_blocked(void *psi, cast_dtype dt, const void *mats, const BlkGate *gates, const BlkSeg &s,
                           hipStream_t stream) {
    const size_t lds = ((size_t)1 << s.tb) * amp_bytes(dt);
    if (lds > (128u << 10)) return fail(CAST_EUNSUPPORTED, "blocked tile exceeds 128 KiB of LDS");
    const hipError_t ae = dt == CAST_C128 ? allow_lds<double>() : allow_lds<float>();
    if (ae != hipSuccess) return fail(CAST_EHIP, std::string("LDS attribute: ") + hipGetErrorString(ae));
    uint64_t grid = s.ntiles;
    const uint64_t cap = (uint64_t)tuning().max_grid[dt];
    if (grid > cap) grid = cap;
    if (dt == CAST_C128)
        hipLaunchKernelGGL(k_blocked<double>, dim3((uint32_t)grid), dim3(256), lds, stream, (double *)psi,
                           (const double *)mats, gates, s);
    else
        hipLaunchKernelGGL(k_blocked<float>, dim3((uint32_t)grid), dim3(256), lds, stream, (float *)psi,
                           (const float *)mats, gates, s);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(CAST_EHIP, std::string("blocked pass launch: ") + hipGetErrorString(e));
    return CAST_OK;
}

}  // namespace cast
