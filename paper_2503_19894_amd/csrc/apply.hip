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
template <int D, typename R, bool UNI>
__global__ void __launch_bounds__(256) k_direct(R *__restrict__ psi_r, const R *__restrict__ mat,
                                                PassArgs a) {
    using V = typename Amp<R>::T;
    constexpr int N = 1 << D;
    V *psi = reinterpret_cast<V *>(psi_r);
    const uint64_t items = a.ngroups * a.nblk;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < items; i += stride) {
        uint32_t bs = (uint32_t)(i >> a.log_ngroups);
        if (UNI) bs = __builtin_amdgcn_readfirstlane(bs);
        const uint64_t g = i & (a.ngroups - 1);
        const uint32_t bid = a.blk[bs];
        uint64_t base = deposit(g, a.lowmask, a.k);
        for (int j = 0; j < a.k - D; ++j)
            if ((bid >> j) & 1u) base ^= a.off[D + j];
        const R *m = mat + (size_t)bs * (2 * N * N);
        V v[N];
#pragma unroll
        for (int c = 0; c < N; ++c) v[c] = psi[base ^ off_lo<D>(a.off, c)];
#pragma unroll
        for (int r = 0; r < N; ++r) {
            V acc;
            acc.x = 0;
            acc.y = 0;
#pragma unroll
            for (int c = 0; c < N; ++c) cmac(acc, m[2 * (r * N + c)], m[2 * (r * N + c) + 1], v[c]);
            psi[base ^ off_lo<D>(a.off, r)] = acc;
        }
    }
}

// ------------------------------------------------------------------ tile
// Tile position of global index bits: window bits [0, W) keep their place,
// high target j lands on bit W + j.  TWOBUF: the group's inputs are re-read
// from LDS for each output row and the results go to a second LDS tile (used
// when 2^d inputs do not fit in registers).
template <int D, typename R, bool UNI, bool TWOBUF>
__global__ void __launch_bounds__(256) k_tile(R *__restrict__ psi_r, const R *__restrict__ mat,
                                              PassArgs a) {
    using V = typename Amp<R>::T;
    constexpr int N = 1 << D;
    extern __shared__ uint4 lds_raw[];
    V *tile = reinterpret_cast<V *>(lds_raw);
    V *tout = TWOBUF ? tile + ((size_t)1 << a.tb) : tile;
    uint4 *tile16 = lds_raw;
    uint4 *tout16 = reinterpret_cast<uint4 *>(tout);
    const uint4 *src16 = reinterpret_cast<const uint4 *>(psi_r);
    uint4 *dst16 = reinterpret_cast<uint4 *>(psi_r);
    V *psi = reinterpret_cast<V *>(psi_r);
    (void)psi;

    constexpr uint32_t APC = 16 / sizeof(V);           // amplitudes per 16-byte chunk
    const uint32_t chunks = (1u << a.tb) / APC;        // 16-byte chunks per tile
    const uint32_t run_chunks_log = a.W - (APC == 2 ? 1 : 0);
    const uint32_t items = (1u << (a.tb - a.k)) * a.nblk;
    const uint32_t log_gt = a.tb - a.k;

    for (uint64_t t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
        // global index of the tile's first amplitude: t above the window,
        // with zeros inserted at the high targets
        const uint64_t tbase = deposit(t << a.W, a.hilowmask, a.khi);
        // ---- load 2^kH runs of 2^W amplitudes, 16 bytes per lane
        for (uint32_t c0 = threadIdx.x; c0 < chunks; c0 += 8 * blockDim.x) {
            uint4 buf[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const uint32_t c = c0 + u * blockDim.x;
                if (c < chunks) {
                    const uint32_t r = c >> run_chunks_log;
                    const uint32_t w = c & ((1u << run_chunks_log) - 1);
                    uint64_t x = tbase;
                    for (int j = 0; j < a.khi; ++j)
                        if ((r >> j) & 1u) x |= 1ull << a.qhi[j];
                    buf[u] = src16[(x / APC) + w];
                }
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const uint32_t c = c0 + u * blockDim.x;
                if (c < chunks) tile16[c] = buf[u];
            }
        }
        __syncthreads();
        // ---- update the tile's (group, block) items
        for (uint32_t it = threadIdx.x; it < items; it += blockDim.x) {
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
            const R *m = mat + (size_t)bs * (2 * N * N);
            if (!TWOBUF) {
                V v[N];
#pragma unroll
                for (int c = 0; c < N; ++c) v[c] = tile[pos ^ olo[c]];
#pragma unroll
                for (int r = 0; r < N; ++r) {
                    V acc;
                    acc.x = 0;
                    acc.y = 0;
#pragma unroll
                    for (int c = 0; c < N; ++c) cmac(acc, m[2 * (r * N + c)], m[2 * (r * N + c) + 1], v[c]);
                    tile[pos ^ olo[r]] = acc;
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
                        const V vc = tile[pos ^ olo[c]];
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
                        tout[pos ^ o] = acc[r];
                    }
                }
            }
        }
        __syncthreads();
        // ---- store.  Identity blocks were never touched, so their tile copy is
        // the input.  (TWOBUF is used only for k = d = 6: one block, always active.)
        for (uint32_t c0 = threadIdx.x; c0 < chunks; c0 += 8 * blockDim.x) {
            uint4 buf[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const uint32_t c = c0 + u * blockDim.x;
                if (c < chunks) buf[u] = tout16[c];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const uint32_t c = c0 + u * blockDim.x;
                if (c < chunks) {
                    const uint32_t r = c >> run_chunks_log;
                    const uint32_t w = c & ((1u << run_chunks_log) - 1);
                    uint64_t x = tbase;
                    for (int j = 0; j < a.khi; ++j)
                        if ((r >> j) & 1u) x |= 1ull << a.qhi[j];
                    dst16[(x / APC) + w] = buf[u];
                }
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ dispatch
template <typename R>
static hipError_t launch_direct(int D, bool uni, R *psi, const R *m, const PassArgs &a, int grid,
                                int wg, hipStream_t s) {
#define CAST_DIRECT(DD)                                                                         \
    case DD:                                                                                    \
        if (uni) hipLaunchKernelGGL((k_direct<DD, R, true>), dim3(grid), dim3(wg), 0, s, psi, m, a); \
        else hipLaunchKernelGGL((k_direct<DD, R, false>), dim3(grid), dim3(wg), 0, s, psi, m, a);     \
        break;
    switch (D) {
        CAST_DIRECT(0) CAST_DIRECT(1) CAST_DIRECT(2) CAST_DIRECT(3) CAST_DIRECT(4) CAST_DIRECT(5)
        CAST_DIRECT(6)
        default: return hipErrorInvalidValue;
    }
#undef CAST_DIRECT
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

// Registers hold 2^d input amplitudes per lane; beyond this the kernel
// re-reads inputs from LDS (TWOBUF).
static int max_reg_d(cast_dtype dt) { return dt == CAST_C128 ? 5 : 6; }

cast_status launch_pass(void *psi, int n, cast_dtype dt, const PassPlan &p, const void *dmat,
                        hipStream_t stream) {
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
    const bool twobuf = D > max_reg_d(dt);
    const bool direct = !twobuf && p.q[0] >= tu.direct_min_q[dt] && (n - k) >= 6;
    hipError_t e;
    if (direct) {
        for (int i = 0; i < k; ++i) a.lowmask[i] = (1ull << p.q[i]) - 1;
        a.log_ngroups = n - k;
        a.ngroups = 1ull << (n - k);
        const uint64_t items = a.ngroups * a.nblk;
        const int wg = tu.wg_direct;
        uint64_t grid = (items + wg - 1) / wg;
        if (grid > (uint64_t)tu.max_grid) grid = tu.max_grid;
        const bool uni = true;  // ngroups >= 64 and a multiple of 64
        if (dt == CAST_C128)
            e = launch_direct<double>(D, uni, (double *)psi, (const double *)dmat, a, (int)grid, wg, stream);
        else
            e = launch_direct<float>(D, uni, (float *)psi, (const float *)dmat, a, (int)grid, wg, stream);
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
        const int wg = tu.wg_tile;
        uint64_t grid = a.ntiles;
        if (grid > (uint64_t)tu.max_grid) grid = tu.max_grid;
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
