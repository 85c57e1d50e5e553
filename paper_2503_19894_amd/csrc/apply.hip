// Gate-pass kernels for gfx950: one in-place pass of a k-qubit gate over a
// 2^n state (Eq. 3).  Each group of 2^k amplitudes agreeing off the targets is
// multiplied by the gate matrix.
//
// The host plan (plan.cpp) relabels each group's local index by a GF(2)
// linear map L so that the matrix becomes block-diagonal with dense 2^d x 2^d
// blocks; a work item is one (group, block) pair, so only the blocks' entries
// are ever multiplied (all structural zeros are skipped) and identity blocks
// are never loaded or stored.  Block matrices are read with wave-uniform
// scalar loads whenever every lane of a wave works on the same block (the
// paper's GPU kernels take the matrix by pointer, Sec. IV-A).
//
// Two kernels:
//  * k_direct: every target is at or above a coalescing threshold, so lanes
//    with consecutive group indices touch consecutive amplitudes; amplitudes
//    go straight from HBM to registers and back.
//  * k_tile: some target is low.  A workgroup stages a tile (all amplitudes
//    whose bits outside the low window and the high targets are fixed: 2^kH
//    contiguous runs) through LDS with 16-byte coalesced loads, updates its
//    groups there, and writes the tile back (the GPU analogue of the paper's
//    shuffled loads for low targets, Sec. IV-A).
#include <hip/hip_runtime.h>

#include <cstring>

#include "internal.hpp"
#include "pass_args.hpp"

namespace cast {

template <typename R> struct Amp;
template <> struct Amp<double> { using T = double2; };
template <> struct Amp<float> { using T = float2; };

// Inserts a zero bit below each mask boundary (masks ascending): deposits the
// bits of g into the positions that are not targets (Eq. 4 with s = 0).
__device__ __forceinline__ uint64_t deposit(uint64_t g, const uint64_t *lowmask, int k) {
    for (int i = 0; i < k; ++i) {
        const uint64_t lm = lowmask[i];
        g = ((g & ~lm) << 1) | (g & lm);
    }
    return g;
}

template <int D>
__device__ __forceinline__ uint64_t off_lo(const uint64_t *off, int a) {
    uint64_t o = 0;
#pragma unroll
    for (int j = 0; j < D; ++j)
        if ((a >> j) & 1) o ^= off[j];
    return o;
}

template <typename V, typename R>
__device__ __forceinline__ void cmac(V &acc, R mre, R mim, const V &v) {
    acc.x = fma(mre, v.x, acc.x);
    acc.x = fma(-mim, v.y, acc.x);
    acc.y = fma(mre, v.y, acc.y);
    acc.y = fma(mim, v.x, acc.y);
}

// ------------------------------------------------------------------ direct
// IPT work items per thread per iteration, all loads issued before any
// store.  NT: non-temporal hint on the state's loads and stores (the state is
// streamed once per pass).
typedef double native_d2 __attribute__((ext_vector_type(2)));
typedef unsigned int native_u4 __attribute__((ext_vector_type(4)));
typedef float native_f2 __attribute__((ext_vector_type(2)));
template <typename V> struct Native;
template <> struct Native<double2> { using T = native_d2; };
template <> struct Native<float2> { using T = native_f2; };

template <bool NT, typename V>
__device__ __forceinline__ V ld(const V *p) {
    if (NT) {
        const auto x = __builtin_nontemporal_load(reinterpret_cast<const typename Native<V>::T *>(p));
        V v;
        v.x = x.x;
        v.y = x.y;
        return v;
    }
    return *p;
}
template <bool NT, typename V>
__device__ __forceinline__ void st(V *p, const V &v) {
    if (NT) {
        typename Native<V>::T x;
        x.x = v.x;
        x.y = v.y;
        __builtin_nontemporal_store(x, reinterpret_cast<typename Native<V>::T *>(p));
    } else {
        *p = v;
    }
}

// Item i of a block-decomposed pass: items are cut into runs of 2^cl
// consecutive groups of one block (cl >= 6, so a wave's 64 lanes share a
// block) and the block slot varies fastest across runs, so the blocks of the
// same groups are processed close together in time rather than in one sweep
// of the state per block.  Longer runs keep longer contiguous address ranges
// per block.  Needs 2^cl to divide ngroups; the run count stays below 2^28 for
// n <= 34.
__device__ __forceinline__ void direct_item(uint64_t i, uint32_t nblk, int cl, uint32_t &bs, uint64_t &g) {
    const uint32_t s = __builtin_amdgcn_readfirstlane((uint32_t)(i >> cl));
    const uint32_t gs = s / nblk;
    bs = s - gs * nblk;
    g = ((uint64_t)gs << cl) | (i & ((1ull << cl) - 1));
}

template <int D, typename R, int IPT, bool NT>
__global__ void __launch_bounds__(256) k_direct(R *__restrict__ psi_r, const R *__restrict__ mat,
                                                PassArgs a) {
    using V = typename Amp<R>::T;
    constexpr int N = 1 << D;
    V *psi = reinterpret_cast<V *>(psi_r);
    const uint64_t items = a.ngroups * a.nblk;
    constexpr uint64_t per_iter = 256ull * IPT;
    const uint64_t nfull = items / per_iter;
    for (uint64_t it0 = blockIdx.x; it0 < nfull; it0 += gridDim.x) {
        // iteration order: rotating the iteration index spreads the
        // workgroups in flight over more DRAM rows of each of the gate's
        // 2^d planes (nfull is then a power of two, 2^it_bits)
        const uint64_t it =
            a.rot ? (((it0 << a.rot) | (it0 >> (a.it_bits - a.rot))) & ((1ull << a.it_bits) - 1)) : it0;
        uint64_t base[IPT];
        const R *m[IPT];
        V v[IPT][N];
#pragma unroll
        for (int u = 0; u < IPT; ++u) {
            const uint64_t i = it * per_iter + (uint64_t)u * 256 + threadIdx.x;
            uint32_t bs;
            uint64_t g;
            direct_item(i, a.nblk, a.chunk_log, bs, g);
            const uint32_t bid = a.blk[bs];
            uint64_t b = deposit(g, a.lowmask, a.k);
            for (int j = 0; j < a.k - D; ++j)
                if ((bid >> j) & 1u) b ^= a.off[D + j];
            base[u] = b;
            // diagonal plans keep the full diagonal, indexed by block id
            m[u] = mat + (size_t)(D == 0 ? bid : bs) * (2 * N * N);
#pragma unroll
            for (int c = 0; c < N; ++c) v[u][c] = ld<NT>(psi + (b ^ off_lo<D>(a.off, c)));
        }
#pragma unroll
        for (int u = 0; u < IPT; ++u) {
#pragma unroll
            for (int r = 0; r < N; ++r) {
                V acc;
                acc.x = 0;
                acc.y = 0;
#pragma unroll
                for (int c = 0; c < N; ++c) cmac(acc, m[u][2 * (r * N + c)], m[u][2 * (r * N + c) + 1], v[u][c]);
                st<NT>(psi + (base[u] ^ off_lo<D>(a.off, r)), acc);
            }
        }
    }
    // tail: items not covered by full iterations, one per thread
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    for (uint64_t i = nfull * per_iter + (uint64_t)blockIdx.x * 256 + threadIdx.x; i < items; i += stride) {
        uint32_t bs;
        uint64_t g;
        direct_item(i, a.nblk, a.chunk_log, bs, g);
        const uint32_t bid = a.blk[bs];
        uint64_t b = deposit(g, a.lowmask, a.k);
        for (int j = 0; j < a.k - D; ++j)
            if ((bid >> j) & 1u) b ^= a.off[D + j];
        const R *mm = mat + (size_t)(D == 0 ? bid : bs) * (2 * N * N);
        V w[N];
#pragma unroll
        for (int c = 0; c < N; ++c) w[c] = psi[b ^ off_lo<D>(a.off, c)];
#pragma unroll
        for (int r = 0; r < N; ++r) {
            V acc;
            acc.x = 0;
            acc.y = 0;
#pragma unroll
            for (int c = 0; c < N; ++c) cmac(acc, mm[2 * (r * N + c)], mm[2 * (r * N + c) + 1], w[c]);
            psi[b ^ off_lo<D>(a.off, r)] = acc;
        }
    }
}

// ------------------------------------------------------------------ diagonal
// A diagonal gate (d = 0) multiplies amplitude x by D[j(x)], j(x) = the bits
// of x at the targets.  Lanes stream consecutive 16-byte chunks of the state
// whatever the targets are, so every access is coalesced.  Identity phases
// are skipped per 128-byte line: a line (8 consecutive lanes) none of whose
// amplitudes has D[j] != 1 is neither loaded nor stored, and a line with any
// such amplitude is loaded and stored whole, so HBM never sees a partial-line
// write (which it would have to complete by read-modify-write).
//
// Work is cut into tiles of 256 * U chunks, and a tile all of whose
// amplitudes have identity phases is never visited: the host lists the
// patterns of the high target bits that select an active tile, and the grid
// walks only those tiles.  Workgroups are dealt to the chip's 8 XCDs
// round-robin, so a plain tile = workgroup mapping can put the tiles of an
// address-bit pattern on a few XCDs; tile number t is given to the XCD equal
// to the XOR of its 3-bit digits, which spreads the tiles evenly.
__device__ __forceinline__ uint64_t xcd_spread(uint64_t it) {
    const uint64_t r = it >> 3;
    uint64_t f = 0;
    for (uint64_t y = r; y; y >>= 3) f ^= y;
    return (r << 3) | ((it ^ f) & 7);
}

template <typename R, int U, bool LDS_TABLE>
__global__ void __launch_bounds__(256) k_diag(R *__restrict__ psi_r, const R *__restrict__ table, DiagArgs a) {
    using V = typename Amp<R>::T;
    constexpr int S = sizeof(V) == 16 ? 0 : 1;   // log2(amplitudes per 16-byte chunk)
    constexpr int A = 1 << S;
    // phases: staged in LDS, or read straight from the (L1-resident) table
    __shared__ V tab_lds[LDS_TABLE ? 64 : 1];
    const V *tab = LDS_TABLE ? tab_lds : reinterpret_cast<const V *>(table);
    if (LDS_TABLE) {
        const int D = 1 << a.k;
        for (int j = threadIdx.x; j < D; j += 256) {
            V t;
            t.x = table[2 * j];
            t.y = table[2 * j + 1];
            tab_lds[j] = t;
        }
        __syncthreads();
    }
    native_u4 *p16 = reinterpret_cast<native_u4 *>(psi_r);
    const int line0 = (int)(threadIdx.x & 56);   // first lane of this lane's 128-byte line
    // j(x) = bits of amplitude x at the targets.  In the main loop a chunk's
    // amplitude index is (uniform tile base) + (threadIdx.x << S) + h with
    // the base a multiple of 256 << S, so j splits into a per-lane part
    // (computed once) and a wave-uniform part (one scalar pass per tile).
    auto jof = [&](uint64_t x) {
        uint32_t j = 0;
        for (int i = 0; i < a.k; ++i) j |= (uint32_t)((x >> a.q[i]) & 1u) << i;
        return j;
    };
    uint32_t jl[A];
#pragma unroll
    for (int h = 0; h < A; ++h) jl[h] = jof(((uint64_t)threadIdx.x << S) | (uint64_t)h);
    constexpr uint64_t per = 256ull * U;
    const bool spread = a.spread && (a.ntiles & 7) == 0 && (gridDim.x & 7) == 0;
    for (uint64_t it = blockIdx.x; it < a.ntiles; it += gridDim.x) {
        const uint32_t t = (uint32_t)(spread ? xcd_spread(it) : it);   // ntiles <= 2^24
        uint32_t rest, pat;
        if (a.pattern_major) {
            rest = t & ((1u << a.rest_bits) - 1);
            pat = t >> a.rest_bits;
        } else {
            rest = t / a.npat;
            pat = t - rest * a.npat;
        }
        if (a.rot) rest = ((rest << a.rot) | (rest >> (a.rest_bits - a.rot))) & ((1u << a.rest_bits) - 1);
        const uint64_t tile = deposit(rest, a.hlowmask, a.kh) | a.patoff[pat];
        native_u4 w[U];
        uint32_t ju[U];
        bool act[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t c0 = tile * per + (uint64_t)u * 256;     // uniform
            ju[u] = jof(c0 << S);
            bool any = false;
#pragma unroll
            for (int h = 0; h < A; ++h) any |= (a.amask >> (ju[u] | jl[h])) & 1u;
            act[u] = ((__ballot(any) >> line0) & 0xffull) != 0;
            if (act[u]) w[u] = __builtin_nontemporal_load(p16 + c0 + threadIdx.x);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!act[u]) continue;
            V *v = reinterpret_cast<V *>(&w[u]);
#pragma unroll
            for (int h = 0; h < A; ++h) {
                const uint32_t j = ju[u] | jl[h];
                if ((a.amask >> j) & 1u) {
                    const V t = tab[j];
                    const R re = v[h].x * t.x - v[h].y * t.y;
                    const R im = v[h].x * t.y + v[h].y * t.x;
                    v[h].x = re;
                    v[h].y = im;
                }
            }
            __builtin_nontemporal_store(w[u], p16 + tile * per + (uint64_t)u * 256 + threadIdx.x);
        }
    }
    // a state smaller than one tile: one chunk per lane (8-lane groups are
    // still whole lines)
    if (a.ntiles) return;
    for (uint64_t c = (uint64_t)blockIdx.x * 256 + threadIdx.x; c < a.nchunks; c += (uint64_t)gridDim.x * 256) {
        bool any = false;
        uint32_t js[A];
#pragma unroll
        for (int h = 0; h < A; ++h) {
            js[h] = jof((c << S) | (uint64_t)h);
            any |= (a.amask >> js[h]) & 1u;
        }
        if (((__ballot(any) >> line0) & 0xffull) == 0) continue;
        native_u4 w = p16[c];
        V *v = reinterpret_cast<V *>(&w);
#pragma unroll
        for (int h = 0; h < A; ++h) {
            if ((a.amask >> js[h]) & 1u) {
                const V t = tab[js[h]];
                const R re = v[h].x * t.x - v[h].y * t.y;
                const R im = v[h].x * t.y + v[h].y * t.x;
                v[h].x = re;
                v[h].y = im;
            }
        }
        p16[c] = w;
    }
}

// ------------------------------------------------------------------ tile
// LDS layout: 16-byte chunk c of the tile is stored at chunk swz(c), which
// XORs the chunk's column (c mod 16) with a hash of its row (c / 16).  Rows
// stay in place, so the coalesced tile load/store phases remain conflict-free,
// while group reads at power-of-two strides (consecutive groups skip the low
// target bits) spread over all banks.
__device__ __forceinline__ uint32_t swz(uint32_t c) { return c ^ (((c >> 4) ^ (c >> 8)) & 15u); }

template <int S>  // S = log2(amplitudes per 16-byte chunk)
__device__ __forceinline__ uint32_t lds_elem(uint32_t p) {
    return (swz(p >> S) << S) | (p & ((1u << S) - 1));
}

// Global 16-byte chunk index of tile chunk c.
__device__ __forceinline__ uint64_t tile_chunk_addr(uint32_t c, uint64_t tbase, uint32_t rcl, int apc_log,
                                                    const PassArgs &a) {
    const uint32_t r = c >> rcl;
    uint64_t x = tbase;
    for (int j = 0; j < a.khi; ++j)
        if ((r >> j) & 1u) x |= 1ull << a.qhi[j];
    return (x >> apc_log) + (c & ((1u << rcl) - 1));
}

// Tile position of global index bits: window bits [0, W) keep their place,
// high target j lands on bit W + j.  TWOBUF: the group's inputs are re-read
// from LDS for each output row and the results go to a second LDS tile (used
// when 2^d inputs do not fit in registers).
template <int D, typename R, bool UNI, bool TWOBUF>
__global__ void __launch_bounds__(256) k_tile(R *__restrict__ psi_r, const R *__restrict__ mat,
                                              PassArgs a) {
    using V = typename Amp<R>::T;
    constexpr int N = 1 << D;
    constexpr int S = sizeof(V) == 16 ? 0 : 1;   // log2(amplitudes per 16-byte chunk)
    extern __shared__ uint4 lds_raw[];
    V *tile = reinterpret_cast<V *>(lds_raw);
    const uint32_t tile_amps = 1u << a.tb;
    V *tout = TWOBUF ? tile + tile_amps : tile;
    uint4 *tile16 = lds_raw;
    uint4 *tout16 = reinterpret_cast<uint4 *>(tout);
    const uint4 *src16 = reinterpret_cast<const uint4 *>(psi_r);
    uint4 *dst16 = reinterpret_cast<uint4 *>(psi_r);

    const uint32_t chunks = tile_amps >> S;
    const uint32_t rcl = a.W - S;                     // log2(chunks per contiguous run)
    const uint32_t log_gt = a.tb - a.k;
    const uint32_t items = (1u << log_gt) * a.nblk;
    const bool batched = chunks >= 8 * 256;           // chunks is a power of two

    for (uint64_t t0 = blockIdx.x; t0 < a.ntiles; t0 += gridDim.x) {
        // tiles in an order rotated left by a.rot bits (ntiles = 2^it_bits then)
        const uint64_t t = a.rot ? (((t0 << a.rot) | (t0 >> (a.it_bits - a.rot))) & (a.ntiles - 1)) : t0;
        // global index of the tile's first amplitude: t above the window,
        // with zeros inserted at the high targets
        const uint64_t tbase = deposit(t << a.W, a.hilowmask, a.khi);
        // ---- load 2^kH runs of 2^W amplitudes, 16 bytes per lane
        if (batched) {
            for (uint32_t c0 = threadIdx.x; c0 < chunks; c0 += 8 * 256) {
                uint4 buf[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) buf[u] = src16[tile_chunk_addr(c0 + u * 256, tbase, rcl, S, a)];
#pragma unroll
                for (int u = 0; u < 8; ++u) tile16[swz(c0 + u * 256)] = buf[u];
            }
        } else {
            for (uint32_t c = threadIdx.x; c < chunks; c += 256) tile16[swz(c)] = src16[tile_chunk_addr(c, tbase, rcl, S, a)];
        }
        __syncthreads();
        // ---- update the tile's (group, block) items
        for (uint32_t it = threadIdx.x; it < items; it += 256) {
            uint32_t bs = it >> log_gt;
            if (UNI) bs = __builtin_amdgcn_readfirstlane(bs);
            const uint32_t gl = it & ((1u << log_gt) - 1);
            const uint32_t bid = a.blk[bs];
            uint32_t pos = gl;
            for (int i = 0; i < a.klo; ++i) {
                const uint32_t lm = a.tlowmask[i];
                pos = ((pos & ~lm) << 1) | (pos & lm);
            }
            for (int j = 0; j < a.k - D; ++j)
                if ((bid >> j) & 1u) pos ^= a.toff[D + j];
            uint32_t olo[N];
#pragma unroll
            for (int c = 0; c < N; ++c) {
                uint32_t o = 0;
#pragma unroll
                for (int j = 0; j < D; ++j)
                    if ((c >> j) & 1) o ^= a.toff[j];
                olo[c] = o;
            }
            const R *m = mat + (size_t)(D == 0 ? bid : bs) * (2 * N * N);
            if (!TWOBUF) {
                V v[N];
#pragma unroll
                for (int c = 0; c < N; ++c) v[c] = tile[lds_elem<S>(pos ^ olo[c])];
#pragma unroll
                for (int r = 0; r < N; ++r) {
                    V acc;
                    acc.x = 0;
                    acc.y = 0;
#pragma unroll
                    for (int c = 0; c < N; ++c) cmac(acc, m[2 * (r * N + c)], m[2 * (r * N + c) + 1], v[c]);
                    tile[lds_elem<S>(pos ^ olo[r])] = acc;
                }
            } else {
                constexpr int RC = 8;
#pragma unroll 1
                for (int r0 = 0; r0 < N; r0 += RC) {
                    V acc[RC];
#pragma unroll
                    for (int r = 0; r < RC; ++r) acc[r].x = acc[r].y = 0;
#pragma unroll
                    for (int c = 0; c < N; ++c) {
                        const V vc = tile[lds_elem<S>(pos ^ olo[c])];
#pragma unroll
                        for (int r = 0; r < RC; ++r)
                            cmac(acc[r], m[2 * ((r0 + r) * N + c)], m[2 * ((r0 + r) * N + c) + 1], vc);
                    }
#pragma unroll
                    for (int r = 0; r < RC; ++r) {
                        uint32_t o = 0;
                        const int rr = r0 + r;
#pragma unroll
                        for (int j = 0; j < D; ++j)
                            if ((rr >> j) & 1) o ^= a.toff[j];
                        tout[lds_elem<S>(pos ^ o)] = acc[r];
                    }
                }
            }
        }
        __syncthreads();
        // ---- store.  Identity blocks were never touched, so their tile copy is
        // the input.  (TWOBUF is used only for k = d = 6: one block, always active.)
        if (batched) {
            for (uint32_t c0 = threadIdx.x; c0 < chunks; c0 += 8 * 256) {
                uint4 buf[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) buf[u] = tout16[swz(c0 + u * 256)];
#pragma unroll
                for (int u = 0; u < 8; ++u) dst16[tile_chunk_addr(c0 + u * 256, tbase, rcl, S, a)] = buf[u];
            }
        } else {
            for (uint32_t c = threadIdx.x; c < chunks; c += 256) dst16[tile_chunk_addr(c, tbase, rcl, S, a)] = tout16[swz(c)];
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ MFMA
// Dense blocks (d >= 4) as complex GEMMs on the matrix cores: a wave takes 16
// groups of one block and computes all 2^d output rows as 16 x 16 tiles,
//   Yr += Ur Xr - Ui Xi,  Yi += Ur Xi + Ui Xr,
// four real 16x16x4 MFMAs per k-step (FP64 for complex128, FP32 for
// complex64).  Operand lane layouts (checked on gfx950): lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16]; result value v of lane l is
// D[row][l % 16] with row = l / 16 + 4 v (f64) or 4 (l / 16) + v (f32).
// The active blocks' matrices are staged transposed in LDS (lanes with
// consecutive rows read consecutive entries).  A wave reads all inputs of its
// 16 groups before writing any output, so updates are in place.
typedef double mf_v4d __attribute__((ext_vector_type(4)));
typedef float mf_v4f __attribute__((ext_vector_type(4)));

template <typename R> struct Mfma;
template <> struct Mfma<double> {
    using acc = mf_v4d;
    static __device__ __forceinline__ acc mma(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <> struct Mfma<float> {
    using acc = mf_v4f;
    static __device__ __forceinline__ acc mma(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

// Stages the active blocks' matrices transposed: mt[(b * N + c) * N + i] = M_b[i][c].
template <int D, typename V, typename R>
__device__ __forceinline__ void stage_blocks(V *mt, const R *mat, uint32_t nblk) {
    constexpr int N = 1 << D;
    for (uint32_t e = threadIdx.x; e < nblk * N * N; e += blockDim.x) {
        const uint32_t b = e / (N * N), rem = e % (N * N), i = rem / N, c = rem % N;
        V v;
        v.x = mat[2 * e];
        v.y = mat[2 * e + 1];
        mt[(b * N + c) * N + i] = v;
    }
}

// One unit: 16 groups of block slot bs.  load(c) returns X[c][group lane%16]
// (this lane's k-row c); store(row, value) writes Y[row][group lane%16].
// M3 = false: four real products per k-step, Yr += Ur Xr - Ui Xi and
// Yi += Ur Xi + Ui Xr.  M3 = true: the three-multiplication form of the
// complex product (Gauss; the "3M method" for complex matrix products):
// P = Ur Xr, Q = Ui Xi, S = (Ur + Ui)(Xr + Xi), then Yr = P - Q and
// Yi = S - P - Q, one matrix-core product fewer per k-step.
// PRE: the unit's 2^d / 4 input loads per lane are all issued before the
// first matrix-core product instead of one k-step ahead, so a wave waits on
// memory once per unit rather than repeatedly inside the product chain.
template <int D, typename R, bool M3, typename Load, typename Store, bool PRE = false>
__device__ __forceinline__ void mfma_unit(const typename Amp<R>::T *mt_blk, Load load, Store store) {
    using V = typename Amp<R>::T;
    using M = Mfma<R>;
    constexpr int N = 1 << D, T = N / 16;
    const int lane = threadIdx.x & 63, j = lane & 15, kk = lane >> 4;
    typename M::acc cr[T], ci[T], cs[M3 ? T : 1];
#pragma unroll
    for (int t = 0; t < T; ++t) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            cr[t][v] = ci[t][v] = 0;
            if (M3) cs[t][v] = 0;
        }
    }
    V xs[PRE ? N / 4 : 1];
    if (PRE) {
#pragma unroll
        for (int s = 0; s < N / 4; ++s) xs[PRE ? s : 0] = load(4 * s + kk);
    }
    constexpr int UNR = PRE ? N / 4 : 4;
#pragma unroll UNR
    for (int s = 0; s < N / 4; ++s) {
        const int c = 4 * s + kk;
        const V x = PRE ? xs[PRE ? s : 0] : load(c);
        const V *col = mt_blk + c * N + j;
        if (M3) {
            const R xs = x.x + x.y;
#pragma unroll
            for (int t = 0; t < T; ++t) {
                const V u = col[16 * t];
                cr[t] = M::mma(u.x, x.x, cr[t]);
                ci[t] = M::mma(u.y, x.y, ci[t]);
                cs[t] = M::mma(u.x + u.y, xs, cs[t]);
            }
        } else {
#pragma unroll
            for (int t = 0; t < T; ++t) {
                const V u = col[16 * t];
                cr[t] = M::mma(u.x, x.x, cr[t]);
                cr[t] = M::mma(-u.y, x.y, cr[t]);
                ci[t] = M::mma(u.x, x.y, ci[t]);
                ci[t] = M::mma(u.y, x.x, ci[t]);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < T; ++t) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            V y;
            if (M3) {
                y.x = cr[t][v] - ci[t][v];
                y.y = cs[t][v] - cr[t][v] - ci[t][v];
            } else {
                y.x = cr[t][v];
                y.y = ci[t][v];
            }
            store(16 * t + M::row(lane, v), y);
        }
    }
}

// The product of one unit from inputs already in registers: xs[s] is this
// lane's k-row 4s + lane / 16 of the unit's 16 groups.
template <int D, typename R, bool M3, typename Store>
__device__ __forceinline__ void mfma_core(const typename Amp<R>::T *mt_blk, const typename Amp<R>::T *xs, Store store) {
    using V = typename Amp<R>::T;
    using M = Mfma<R>;
    constexpr int N = 1 << D, T = N / 16;
    const int lane = threadIdx.x & 63, j = lane & 15, kk = lane >> 4;
    typename M::acc cr[T], ci[T], cs[M3 ? T : 1];
#pragma unroll
    for (int t = 0; t < T; ++t) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            cr[t][v] = ci[t][v] = 0;
            if (M3) cs[t][v] = 0;
        }
    }
#pragma unroll
    for (int s = 0; s < N / 4; ++s) {
        const int c = 4 * s + kk;
        const V x = xs[s];
        const V *col = mt_blk + c * N + j;
        if (M3) {
            const R xsum = x.x + x.y;
#pragma unroll
            for (int t = 0; t < T; ++t) {
                const V u = col[16 * t];
                cr[t] = M::mma(u.x, x.x, cr[t]);
                ci[t] = M::mma(u.y, x.y, ci[t]);
                cs[t] = M::mma(u.x + u.y, xsum, cs[t]);
            }
        } else {
#pragma unroll
            for (int t = 0; t < T; ++t) {
                const V u = col[16 * t];
                cr[t] = M::mma(u.x, x.x, cr[t]);
                cr[t] = M::mma(-u.y, x.y, cr[t]);
                ci[t] = M::mma(u.x, x.y, ci[t]);
                ci[t] = M::mma(u.y, x.x, ci[t]);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < T; ++t) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            V y;
            if (M3) {
                y.x = cr[t][v] - ci[t][v];
                y.y = cs[t][v] - cr[t][v] - ci[t][v];
            } else {
                y.x = cr[t][v];
                y.y = ci[t][v];
            }
            store(16 * t + M::row(lane, v), y);
        }
    }
}

template <int D>
__device__ __forceinline__ uint64_t off_of(const uint64_t *off, int c) {
    uint64_t o = 0;
#pragma unroll
    for (int b = 0; b < D; ++b)
        if ((c >> b) & 1) o ^= off[b];
    return o;
}

template <int D, typename R, bool M3, bool PRE>
__global__ void __launch_bounds__(256) k_mfma_direct(R *__restrict__ psi_r, const R *__restrict__ mat, PassArgs a) {
    using V = typename Amp<R>::T;
    constexpr int N = 1 << D;
    extern __shared__ uint4 lds_raw[];
    V *mt = reinterpret_cast<V *>(lds_raw);
    V *psi = reinterpret_cast<V *>(psi_r);
    stage_blocks<D>(mt, mat, a.nblk);
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, j = lane & 15;
    const uint64_t upb = a.ngroups >> 4;   // units per block
    const uint64_t units = upb * a.nblk;
    // the block slot varies fastest across units (as in the direct kernel);
    // units number below 2^26 for n <= 34
    for (uint64_t u = (uint64_t)blockIdx.x * 4 + wave; u < units; u += (uint64_t)gridDim.x * 4) {
        uint32_t uu = __builtin_amdgcn_readfirstlane((uint32_t)u);
        if (a.rot) {   // rotated order of the four-unit runs, as in k_mfma_direct_db
            uint32_t w = uu >> 2;
            w = ((w << a.rot) | (w >> (a.it_bits - a.rot))) & ((1u << a.it_bits) - 1);
            uu = (w << 2) | (uu & 3u);
        }
        const uint32_t gu = uu / a.nblk;
        const uint32_t bs = uu - gu * a.nblk;
        const uint64_t g = (uint64_t)gu * 16 + j;
        const uint32_t bid = a.blk[bs];
        uint64_t base = deposit(g, a.lowmask, a.k);
        for (int q = 0; q < a.k - D; ++q)
            if ((bid >> q) & 1u) base ^= a.off[D + q];
        auto ld = [&](int c) { return psi[base ^ off_of<D>(a.off, c)]; };
        auto st = [&](int row, const V &y) { psi[base ^ off_of<D>(a.off, row)] = y; };
        mfma_unit<D, R, M3, decltype(ld), decltype(st), PRE>(mt + (size_t)bs * N * N, ld, st);
    }
}

// k_mfma_direct with the inputs of a wave's next unit requested before the
// matrix-core products of the current one, so a wave's memory traffic
// overlaps its own products instead of alternating with them (the products
// of a 32-dimensional block take about as long as its loads).  The state is
// streamed with non-temporal loads and stores.  In both matrix-core direct
// kernels a.rot > 0 rotates the index of each run of four units (one
// workgroup's) left by a.rot bits within 2^a.it_bits runs, so the workgroups
// in flight spread over more DRAM rows of every plane; the host sets it only
// when the run count is 2^it_bits.
template <int D, typename R, bool M3>
__global__ void __launch_bounds__(256) k_mfma_direct_db(R *__restrict__ psi_r, const R *__restrict__ mat,
                                                        PassArgs a) {
    using V = typename Amp<R>::T;
    constexpr int N = 1 << D;
    extern __shared__ uint4 lds_raw[];
    V *mt = reinterpret_cast<V *>(lds_raw);
    V *psi = reinterpret_cast<V *>(psi_r);
    stage_blocks<D>(mt, mat, a.nblk);
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, j = lane & 15, kk = lane >> 4;
    const uint64_t units = (a.ngroups >> 4) * a.nblk;
    const uint64_t stride = (uint64_t)gridDim.x * 4;
    // group base and block slot of unit u
    auto locate = [&](uint64_t u, uint32_t &bs) {
        uint32_t uu = __builtin_amdgcn_readfirstlane((uint32_t)u);
        if (a.rot) {
            uint32_t w = uu >> 2;
            w = ((w << a.rot) | (w >> (a.it_bits - a.rot))) & ((1u << a.it_bits) - 1);
            uu = (w << 2) | (uu & 3u);
        }
        const uint32_t gu = uu / a.nblk;
        bs = uu - gu * a.nblk;
        const uint64_t g = (uint64_t)gu * 16 + j;
        const uint32_t bid = a.blk[bs];
        uint64_t base = deposit(g, a.lowmask, a.k);
        for (int q = 0; q < a.k - D; ++q)
            if ((bid >> q) & 1u) base ^= a.off[D + q];
        return base;
    };
    uint64_t u = (uint64_t)blockIdx.x * 4 + wave;
    if (u >= units) return;
    uint32_t bs;
    uint64_t base = locate(u, bs);
    V xs[N / 4];
#pragma unroll
    for (int s = 0; s < N / 4; ++s) xs[s] = ld<true>(psi + (base ^ off_of<D>(a.off, 4 * s + kk)));
    for (;;) {
        const uint64_t un = u + stride;
        const bool more = un < units;
        uint32_t bsn = 0;
        uint64_t basen = 0;
        V xn[N / 4];
        if (more) {
            basen = locate(un, bsn);
#pragma unroll
            for (int s = 0; s < N / 4; ++s) xn[s] = ld<true>(psi + (basen ^ off_of<D>(a.off, 4 * s + kk)));
        }
        auto sto = [&](int row, const V &y) { st<true>(psi + (base ^ off_of<D>(a.off, row)), y); };
        mfma_core<D, R, M3>(mt + (size_t)bs * N * N, xs, sto);
        if (!more) break;
        u = un;
        bs = bsn;
        base = basen;
#pragma unroll
        for (int s = 0; s < N / 4; ++s) xs[s] = xn[s];
    }
}

template <int D, typename R, bool M3>
__global__ void __launch_bounds__(256) k_mfma_tile(R *__restrict__ psi_r, const R *__restrict__ mat, PassArgs a) {
    using V = typename Amp<R>::T;
    constexpr int N = 1 << D;
    constexpr int S = sizeof(V) == 16 ? 0 : 1;
    extern __shared__ uint4 lds_raw[];
    V *mt = reinterpret_cast<V *>(lds_raw);
    const size_t mt_elems = (size_t)a.nblk * N * N;
    uint4 *tile16 = lds_raw + (mt_elems * sizeof(V)) / 16;
    V *tile = reinterpret_cast<V *>(tile16);
    const uint4 *src16 = reinterpret_cast<const uint4 *>(psi_r);
    uint4 *dst16 = reinterpret_cast<uint4 *>(psi_r);
    stage_blocks<D>(mt, mat, a.nblk);
    const uint32_t tile_amps = 1u << a.tb;
    const uint32_t chunks = tile_amps >> S;
    const uint32_t rcl = a.W - S;
    const uint32_t log_gt = a.tb - a.k;
    const uint32_t upb = (1u << log_gt) >> 4;   // units per block in a tile
    const uint32_t units = upb * a.nblk;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, j = lane & 15;
    for (uint64_t t0 = blockIdx.x; t0 < a.ntiles; t0 += gridDim.x) {
        // tiles in an order rotated left by a.rot bits, as in k_tile
        const uint64_t t = a.rot ? (((t0 << a.rot) | (t0 >> (a.it_bits - a.rot))) & (a.ntiles - 1)) : t0;
        const uint64_t tbase = deposit(t << a.W, a.hilowmask, a.khi);
        for (uint32_t c0 = threadIdx.x; c0 < chunks; c0 += 8 * 256) {
            uint4 buf[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) buf[u] = src16[tile_chunk_addr(c0 + u * 256, tbase, rcl, S, a)];
#pragma unroll
            for (int u = 0; u < 8; ++u) tile16[swz(c0 + u * 256)] = buf[u];
        }
        __syncthreads();
        for (uint32_t u = wave; u < units; u += 4) {
            const uint32_t bs = u / upb;
            const uint32_t gl = (u % upb) * 16 + j;
            const uint32_t bid = a.blk[bs];
            uint32_t pos = gl;
            for (int i = 0; i < a.klo; ++i) {
                const uint32_t lm = a.tlowmask[i];
                pos = ((pos & ~lm) << 1) | (pos & lm);
            }
            for (int q = 0; q < a.k - D; ++q)
                if ((bid >> q) & 1u) pos ^= a.toff[D + q];
            auto toff_of = [&](int c) {
                uint32_t o = 0;
#pragma unroll
                for (int b = 0; b < D; ++b)
                    if ((c >> b) & 1) o ^= a.toff[b];
                return o;
            };
            mfma_unit<D, R, M3>(
                mt + (size_t)bs * N * N, [&](int c) { return tile[lds_elem<S>(pos ^ toff_of(c))]; },
                [&](int row, const V &y) { tile[lds_elem<S>(pos ^ toff_of(row))] = y; });
        }
        __syncthreads();
        for (uint32_t c0 = threadIdx.x; c0 < chunks; c0 += 8 * 256) {
            uint4 buf[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) buf[u] = tile16[swz(c0 + u * 256)];
#pragma unroll
            for (int u = 0; u < 8; ++u) dst16[tile_chunk_addr(c0 + u * 256, tbase, rcl, S, a)] = buf[u];
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ dispatch
template <int DD, typename R, int IPT, bool NT>
static void launch_one(R *psi, const R *m, const PassArgs &a, int grid, hipStream_t s) {
    // several items per thread only pay (and only fit) for small blocks
    if constexpr (IPT == 1 || DD <= 3)
        hipLaunchKernelGGL((k_direct<DD, R, IPT, NT>), dim3(grid), dim3(256), 0, s, psi, m, a);
}

template <typename R, int IPT, bool NT>
static void launch_direct_t(int D, R *psi, const R *m, const PassArgs &a, int grid, hipStream_t s) {
#define CAST_DIRECT(DD) \
    case DD: launch_one<DD, R, IPT, NT>(psi, m, a, grid, s); break;
    switch (D) {
        CAST_DIRECT(0) CAST_DIRECT(1) CAST_DIRECT(2) CAST_DIRECT(3) CAST_DIRECT(4) CAST_DIRECT(5) CAST_DIRECT(6)
        default: break;
    }
#undef CAST_DIRECT
}

// Items per thread: enough loads in flight for small blocks, one item when a
// block already needs many registers.
static int direct_ipt(int D, cast_dtype dt) {
    const int amps_cap = dt == CAST_C128 ? 8 : 16;   // amplitudes a lane holds across its items
    int ipt = tuning().direct_ipt[dt];
    while (ipt > 1 && (ipt * (1 << D) > amps_cap || D > 3)) ipt >>= 1;
    return ipt;
}

template <typename R>
static hipError_t launch_direct(int D, cast_dtype dt, R *psi, const R *m, const PassArgs &a, hipStream_t s,
                                int rot_override) {
    const int ipt = direct_ipt(D, dt);
    const bool nt = tuning().direct_nt[dt] != 0;
    const uint64_t items = a.ngroups * a.nblk;
    uint64_t grid = (items + 256ull * ipt - 1) / (256ull * ipt);
    if (grid > (uint64_t)tuning().max_grid[dt]) grid = tuning().max_grid[dt];
    if (grid < 1) grid = 1;
    const int g = (int)grid;
    PassArgs b = a;
    b.rot = b.it_bits = 0;
    {
        // rotated iteration order for passes whose lowest target lies in
        // [direct_rot_lo, direct_rot_hi] (needs a power-of-two iteration count)
        // (a pass's own shape overrides the knobs)
        const Tuning &tu = tuning();
        const uint64_t nfull = items / (256ull * ipt);
        const int q0 = __builtin_ctzll(a.lowmask[0] + 1);   // lowest target
        const int rot = rot_override >= 0 ? rot_override
                        : (q0 >= tu.direct_rot_lo[dt] && q0 <= tu.direct_rot_hi[dt]) ? tu.direct_rot[dt]
                                                                                      : 0;
        if (rot > 0 && nfull > 1 && !(nfull & (nfull - 1))) {
            b.it_bits = __builtin_ctzll(nfull);
            b.rot = rot < b.it_bits ? rot : 0;
        }
    }
    switch (ipt * 2 + (nt ? 1 : 0)) {
        case 2: launch_direct_t<R, 1, false>(D, psi, m, b, g, s); break;
        case 3: launch_direct_t<R, 1, true>(D, psi, m, b, g, s); break;
        case 4: launch_direct_t<R, 2, false>(D, psi, m, b, g, s); break;
        case 5: launch_direct_t<R, 2, true>(D, psi, m, b, g, s); break;
        case 8: launch_direct_t<R, 4, false>(D, psi, m, b, g, s); break;
        case 9: launch_direct_t<R, 4, true>(D, psi, m, b, g, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename R>
static hipError_t launch_tile(int D, bool uni, bool twobuf, R *psi, const R *m, const PassArgs &a,
                              int grid, int wg, size_t lds, hipStream_t s) {
    if (lds > 65536) {
        // only the k = d = 6 two-buffer variants need more than 64 KiB
        static bool done[2][2] = {{false, false}, {false, false}};
        const int ri = sizeof(R) == 8;
        if (!done[ri][uni]) {
            hipError_t e = uni ? hipFuncSetAttribute((const void *)k_tile<6, R, true, true>,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)
                               : hipFuncSetAttribute((const void *)k_tile<6, R, false, true>,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
            done[ri][uni] = true;
        }
    }
#define CAST_TILE(DD)                                                                                      \
    case DD:                                                                                               \
        if (twobuf) {                                                                                      \
            if (uni) hipLaunchKernelGGL((k_tile<DD, R, true, true>), dim3(grid), dim3(wg), lds, s, psi, m, a); \
            else hipLaunchKernelGGL((k_tile<DD, R, false, true>), dim3(grid), dim3(wg), lds, s, psi, m, a);    \
        } else {                                                                                           \
            if (uni) hipLaunchKernelGGL((k_tile<DD, R, true, false>), dim3(grid), dim3(wg), lds, s, psi, m, a); \
            else hipLaunchKernelGGL((k_tile<DD, R, false, false>), dim3(grid), dim3(wg), lds, s, psi, m, a);    \
        }                                                                                                  \
        break;
    switch (D) {
        CAST_TILE(0) CAST_TILE(1) CAST_TILE(2) CAST_TILE(3) CAST_TILE(4) CAST_TILE(5) CAST_TILE(6)
        default: return hipErrorInvalidValue;
    }
#undef CAST_TILE
    return hipGetLastError();
}

template <typename R>
static hipError_t launch_diag(int U, bool lds_table, R *psi, const R *m, const DiagArgs &g, int grid, hipStream_t s) {
#define CAST_DIAG(UU)                                                                                     \
    case UU:                                                                                              \
        if (lds_table) hipLaunchKernelGGL((k_diag<R, UU, true>), dim3(grid), dim3(256), 0, s, psi, m, g);  \
        else hipLaunchKernelGGL((k_diag<R, UU, false>), dim3(grid), dim3(256), 0, s, psi, m, g);          \
        break;
    switch (U) {
        CAST_DIAG(1) CAST_DIAG(2) CAST_DIAG(4) CAST_DIAG(8)
        default: return hipErrorInvalidValue;
    }
#undef CAST_DIAG
    return hipGetLastError();
}

// Registers hold 2^d input amplitudes per lane; beyond this the kernel
// re-reads inputs from LDS (TWOBUF).
static int max_reg_d(cast_dtype dt) { return dt == CAST_C128 ? 5 : 5; }

static int mfma_tile_bits(int n, cast_dtype dt, const PassPlan &p);

// Targets at or above the MFMA tile's contiguous window: the smallest kH with
// #{targets >= tb - kH} == kH.
static int mfma_tile_khi(int n, cast_dtype dt, const PassPlan &p) {
    const int tb = mfma_tile_bits(n, dt, p);
    for (int khi = 0;; ++khi) {
        int cnt = 0;
        for (int i = 0; i < p.k; ++i) cnt += p.q[i] >= tb - khi;
        if (cnt == khi) return khi;
    }
}

// The direct MFMA gather puts 16 groups on the 16 lanes of a row; with a
// target below bit 4 those groups are not consecutive amplitudes, so each load
// collects scattered 16-byte pieces (more scattered still when the plan has
// several blocks, whose basis offsets are XOR combinations of the targets).
// The LDS tile reads runs of 2^(tb - kH) consecutive amplitudes instead, and
// wins for d <= 4 when at most one target lies above the window or the plan
// has several blocks.  At d = 5 a tile holds too few 32-amplitude groups to
// keep the matrix cores busy, and the direct gather stays ahead.
static bool mfma_prefer_tile(int n, cast_dtype dt, const PassPlan &p) {
    if (!tuning().mfma_low_tile[dt] || p.q[0] >= 4 || p.d > 4) return false;
    return p.blk.size() > 1 || mfma_tile_khi(n, dt, p) <= 1;
}

int pass_kernel_kind(int n, cast_dtype dt, const PassPlan &p) {
    const Tuning &tu = tuning();
    if (p.d == 0 && tu.use_diag[dt]) return 3;
    if (p.d >= tu.mfma_min_d[dt] && mfma_fits(n, dt, p)) {
        if (p.q[0] >= tu.mfma_direct_min_q[dt] && (n - p.k) >= 4 && !mfma_prefer_tile(n, dt, p)) return 4;
        return 5;
    }
    if (p.d > max_reg_d(dt)) return 2;
    if (p.q[0] >= tu.direct_min_q[dt] && (n - p.k) >= 6) return 0;
    return 1;
}

// LDS bytes of the staged block matrices, and the MFMA tile size.
static size_t mfma_mat_bytes(cast_dtype dt, const PassPlan &p) {
    return p.blk.size() * ((size_t)1 << (2 * p.d)) * amp_bytes(dt);
}
static int mfma_tile_bits(int n, cast_dtype dt, const PassPlan &p) {
    // tile + matrices within 128 KiB; a tile holds at least 16 groups
    int tb = tuning().tile_bits[dt];
    while (tb > p.k + 4 && ((size_t)1 << tb) * amp_bytes(dt) + mfma_mat_bytes(dt, p) > (128u << 10)) --tb;
    return tb > n ? n : tb;
}
bool mfma_fits(int n, cast_dtype dt, const PassPlan &p) {
    if (p.d < 4 || n - p.k < 4) return false;
    if (mfma_mat_bytes(dt, p) > (64u << 10)) return false;
    const int tb = mfma_tile_bits(n, dt, p);
    return tb >= p.k + 4 && ((size_t)1 << tb) * amp_bytes(dt) + mfma_mat_bytes(dt, p) <= (128u << 10) &&
           ((size_t)1 << tb) / (16 / amp_bytes(dt)) >= 8 * 256;
}

template <typename R>
static hipError_t launch_mfma(int D, bool tile, bool m3, int prefetch, R *psi, const R *m, const PassArgs &a, int grid,
                              size_t lds, hipStream_t s) {
    // prefetch 1: a unit's inputs all requested before its products; 2: the
    // next unit's inputs requested before the current unit's products
    // (the 64-dimensional blocks keep 1: two units of inputs would take
    // every register and leave one wave per SIMD)
    const bool pre2 = prefetch >= 2 && D < 6, pre = prefetch == 1 || (prefetch >= 2 && !pre2);
#define CAST_MFMA_K(KERN, ...)                                                                           \
    {                                                                                                    \
        static bool set = false;                                                                         \
        if (!set) {                                                                                      \
            hipError_t e = hipFuncSetAttribute((const void *)KERN<__VA_ARGS__>,                          \
                                               hipFuncAttributeMaxDynamicSharedMemorySize, 128 << 10);   \
            if (e != hipSuccess) return e;                                                               \
            set = true;                                                                                  \
        }                                                                                                \
        hipLaunchKernelGGL((KERN<__VA_ARGS__>), dim3(grid), dim3(256), lds, s, psi, m, a);               \
    }
#define CAST_MFMA(DD)                                                                                    \
    case DD:                                                                                             \
        if (tile) {                                                                                      \
            if (m3) CAST_MFMA_K(k_mfma_tile, DD, R, true) else CAST_MFMA_K(k_mfma_tile, DD, R, false)   \
        } else if (pre2) {                                                                               \
            if (m3) CAST_MFMA_K(k_mfma_direct_db, DD, R, true) else CAST_MFMA_K(k_mfma_direct_db, DD, R, false) \
        } else if (pre) {                                                                                \
            if (m3) CAST_MFMA_K(k_mfma_direct, DD, R, true, true)                                       \
            else CAST_MFMA_K(k_mfma_direct, DD, R, false, true)                                          \
        } else {                                                                                         \
            if (m3) CAST_MFMA_K(k_mfma_direct, DD, R, true, false)                                      \
            else CAST_MFMA_K(k_mfma_direct, DD, R, false, false)                                         \
        }                                                                                                \
        break;
    switch (D) {
        CAST_MFMA(4) CAST_MFMA(5) CAST_MFMA(6)
        default: return hipErrorInvalidValue;
    }
#undef CAST_MFMA_K
#undef CAST_MFMA
    return hipGetLastError();
}

cast_status launch_pass(void *psi, int n, cast_dtype dt, const PassPlan &p, const void *dmat,
                        hipStream_t stream, const PassShape *shape) {
    if (p.identity()) return CAST_OK;
    const Tuning &tu = tuning();
    const int k = p.k, D = p.d;
    PassArgs a;
    memset(&a, 0, sizeof a);
    a.k = k;
    a.nblk = (uint32_t)p.blk.size();
    for (size_t i = 0; i < p.blk.size(); ++i) a.blk[i] = p.blk[i];
    // physical offset of each virtual basis vector
    for (int i = 0; i < k; ++i) {
        uint64_t o = 0;
        for (int s = 0; s < k; ++s)
            if ((p.L[i] >> s) & 1u) o |= 1ull << p.q[s];
        a.off[i] = o;
    }
    const int kind = pass_kernel_kind(n, dt, p);
    const bool twobuf = kind == 2;
    const bool direct = kind == 0;
    hipError_t e;
    if (kind == 4 || kind == 5) {
        for (int i = 0; i < k; ++i) a.lowmask[i] = (1ull << p.q[i]) - 1;
        a.ngroups = 1ull << (n - k);
        size_t lds = mfma_mat_bytes(dt, p);
        uint64_t grid;
        if (kind == 4) {
            const uint64_t units = (a.ngroups >> 4) * a.nblk;
            grid = (units + 3) / 4;
            const uint64_t cap = (uint64_t)tu.mfma_grid_per_cu[dt] * 256;
            if (grid > cap) grid = cap;
            // rotated order of the four-unit runs
            const int rot = shape && shape->rot > 0 ? shape->rot : 0;
            if (rot > 0 && units % 4 == 0) {
                const uint64_t runs = units / 4;
                int bits = 0;
                while ((1ull << bits) < runs) ++bits;
                if ((1ull << bits) == runs && rot < bits) {
                    a.rot = rot;
                    a.it_bits = bits;
                }
            }
        } else {
            const int tb = mfma_tile_bits(n, dt, p);
            const int khi = mfma_tile_khi(n, dt, p);
            const int W = tb - khi;
            a.tb = tb;
            a.W = W;
            a.khi = khi;
            a.klo = k - khi;
            for (int j = 0; j < khi; ++j) {
                a.qhi[j] = p.q[a.klo + j];
                a.hilowmask[j] = (1ull << a.qhi[j]) - 1;
            }
            for (int i = 0; i < a.klo; ++i) a.tlowmask[i] = (1u << p.q[i]) - 1;
            for (int i = 0; i < k; ++i) {
                uint32_t o = 0;
                for (int s2 = 0; s2 < k; ++s2)
                    if ((p.L[i] >> s2) & 1u) o |= (s2 < a.klo) ? (1u << p.q[s2]) : (1u << (W + s2 - a.klo));
                a.toff[i] = o;
            }
            a.ntiles = 1ull << (n - tb);
            if (shape && shape->rot > 0 && shape->rot < n - tb) {   // rotated tile order
                a.rot = shape->rot;
                a.it_bits = n - tb;
            }
            grid = a.ntiles;
            if (grid > (uint64_t)tu.max_grid[dt]) grid = tu.max_grid[dt];
            lds += ((size_t)1 << tb) * amp_bytes(dt);
        }
        if (dt == CAST_C128)
            e = launch_mfma<double>(D, kind == 5, D >= tu.mfma_3m_min_d[dt], tu.mfma_prefetch[dt], (double *)psi,
                                    (const double *)dmat, a,
                                    (int)grid, lds, stream);
        else
            e = launch_mfma<float>(D, kind == 5, D >= tu.mfma_3m_min_d[dt], tu.mfma_prefetch[dt], (float *)psi,
                                   (const float *)dmat, a,
                                   (int)grid, lds, stream);
    } else if (kind == 3) {
        DiagArgs g;
        memset(&g, 0, sizeof g);
        g.k = k;
        for (int i = 0; i < k; ++i) g.q[i] = p.q[i];
        for (uint32_t b : p.blk) g.amask |= 1ull << b;
        g.nchunks = ((uint64_t)1 << n) * amp_bytes(dt) / 16;
        if (g.nchunks == 0) g.nchunks = 1;   // c64, n = 1: one chunk holds both amplitudes
        const int U = tu.diag_unroll[dt];
        const uint64_t per = 256ull * U;
        uint64_t grid = (g.nchunks + per - 1) / per;
        if (g.nchunks >= per) {
            // tile = 2^tb amplitudes; targets >= tb select tiles
            const int S = dt == CAST_C128 ? 0 : 1;   // log2(amplitudes per chunk)
            int tb = S;
            while ((1ull << (tb - S)) < per) ++tb;
            int kl = 0;
            while (kl < k && p.q[kl] < tb) ++kl;
            const int kha = k - kl;
            // does any amplitude of a tile whose high-target bits are ph have a phase != 1?
            const uint64_t lo = kl == 6 ? ~0ull : (1ull << (1u << kl)) - 1;
            auto active = [&](uint32_t ph) { return ((g.amask >> (ph << kl)) & lo) != 0; };
            // keep the high targets the activity depends on
            int rel[6], nrel = 0;
            for (int i = 0; i < kha; ++i) {
                bool matters = false;
                for (uint32_t ph = 0; ph < (1u << kha) && !matters; ++ph) matters = active(ph) != active(ph ^ (1u << i));
                if (matters) rel[nrel++] = i;
            }
            g.kh = nrel;
            for (int j = 0; j < nrel; ++j) g.hlowmask[j] = (1ull << (p.q[kl + rel[j]] - tb)) - 1;
            g.rest_bits = (n - tb) - nrel;
            g.pattern_major = tu.diag_order[dt];
            g.spread = tu.diag_spread[dt];
            int npat = 0;
            for (uint32_t pr = 0; pr < (1u << nrel); ++pr) {
                uint32_t ph = 0, off = 0;
                for (int j = 0; j < nrel; ++j)
                    if ((pr >> j) & 1u) ph |= 1u << rel[j], off |= 1u << (p.q[kl + rel[j]] - tb);
                if (active(ph)) g.patoff[npat++] = off;
            }
            g.npat = (uint32_t)npat;
            g.ntiles = (uint64_t)npat << g.rest_bits;
            if (shape && shape->rot > 0 && shape->rot < g.rest_bits) g.rot = shape->rot;
            grid = g.ntiles;
            if (grid == 0) return CAST_OK;   // every phase is 1
        }
        if (grid > (uint64_t)tu.diag_max_grid[dt]) grid = tu.diag_max_grid[dt];
        if (dt == CAST_C128) e = launch_diag<double>(U, tu.diag_lds_table[dt] != 0, (double *)psi, (const double *)dmat, g, (int)grid, stream);
        else e = launch_diag<float>(U, tu.diag_lds_table[dt] != 0, (float *)psi, (const float *)dmat, g, (int)grid, stream);
    } else if (direct) {
        for (int i = 0; i < k; ++i) a.lowmask[i] = (1ull << p.q[i]) - 1;
        a.ngroups = 1ull << (n - k);
        // ngroups >= 64 (n - k >= 6), so a run of 2^chunk_log items is one block's groups
        const int cl = shape && shape->chunk_log >= 0 ? shape->chunk_log : tu.direct_chunk_log[dt];
        a.chunk_log = cl < 6 ? 6 : cl;
        if (a.chunk_log > n - k) a.chunk_log = n - k;
        const int rot = shape ? shape->rot : -1;
        if (dt == CAST_C128)
            e = launch_direct<double>(D, dt, (double *)psi, (const double *)dmat, a, stream, rot);
        else
            e = launch_direct<float>(D, dt, (float *)psi, (const float *)dmat, a, stream, rot);
    } else {
        int tb = tu.tile_bits[dt];
        if (twobuf) tb = 12;
        if (tb > n) tb = n;
        // smallest kH with #{targets >= tb - kH} == kH
        int khi = 0;
        for (;; ++khi) {
            int cnt = 0;
            for (int i = 0; i < k; ++i) cnt += p.q[i] >= tb - khi;
            if (cnt == khi) break;
        }
        const int W = tb - khi;
        a.tb = tb;
        a.W = W;
        a.khi = khi;
        a.klo = k - khi;
        for (int j = 0; j < khi; ++j) {
            a.qhi[j] = p.q[a.klo + j];
            a.hilowmask[j] = (1ull << a.qhi[j]) - 1;
        }
        for (int i = 0; i < a.klo; ++i) a.tlowmask[i] = (1u << p.q[i]) - 1;
        for (int i = 0; i < k; ++i) {
            uint32_t o = 0;
            for (int s = 0; s < k; ++s)
                if ((p.L[i] >> s) & 1u) o |= (s < a.klo) ? (1u << p.q[s]) : (1u << (W + s - a.klo));
            a.toff[i] = o;
        }
        a.ntiles = 1ull << (n - tb);
        if (shape && shape->rot > 0 && shape->rot < n - tb) {   // rotated tile order
            a.rot = shape->rot;
            a.it_bits = n - tb;
        }
        const int wg = 256;
        uint64_t grid = a.ntiles;
        if (grid > (uint64_t)tu.max_grid[dt]) grid = tu.max_grid[dt];
        const bool uni = (tb - k) >= 6;
        const size_t lds = ((size_t)1 << tb) * amp_bytes(dt) * (twobuf ? 2 : 1);
        if (dt == CAST_C128)
            e = launch_tile<double>(D, uni, twobuf, (double *)psi, (const double *)dmat, a, (int)grid, wg,
                                    lds, stream);
        else
            e = launch_tile<float>(D, uni, twobuf, (float *)psi, (const float *)dmat, a, (int)grid, wg, lds,
                                   stream);
    }
    if (e != hipSuccess) return fail(CAST_EHIP, std::string("pass launch: ") + hipGetErrorString(e));
    return CAST_OK;
}

}  // namespace cast
