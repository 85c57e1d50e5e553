// Kernels of the batched adjoint-gradient programs (batch.hpp).
//
// One work item = one workgroup's share (1 / wgs) of one op of one instance.
// The same item routine serves both launch modes: one launch per global step
// (all instances' op s side by side), or one persistent launch in which
// workgroups pull items in global order and wait, per instance, for the
// previous op to finish.
#include <hip/hip_runtime.h>

#include "batch.hpp"
#include "internal.hpp"

namespace cast {

extern __shared__ uint4 batch_lds[];

template <typename R> struct BAmp;
template <> struct BAmp<double> { using T = double2; };
template <> struct BAmp<float> { using T = float2; };

__device__ __forceinline__ uint64_t ins0(uint64_t g, int q) {
    const uint64_t lm = (1ull << q) - 1;
    return ((g & ~lm) << 1) | (g & lm);
}
__device__ __forceinline__ uint32_t ins0_32(uint32_t g, int q) {
    const uint32_t lm = (1u << q) - 1;
    return ((g & ~lm) << 1) | (g & lm);
}

// The read-only tables (gate matrices, gate and sweep records) are read
// through the constant address space.  Nothing in a kernel writes them, so
// their loads may use the scalar cache and land in SGPRs.  Through generic
// pointers the compiler must assume that the kernel's own stores to the
// states may alias them, and in a loop over work items (the persistent
// launch) every such load after the first item's stores became a vector load
// into VGPRs: 223 VGPRs instead of 119 for complex128.
template <typename T> using CPtr = const __attribute__((address_space(4))) T *;
template <typename T> __device__ __forceinline__ CPtr<T> cptr(const T *p) { return (CPtr<T>)p; }

template <typename V, typename R>
__device__ __forceinline__ V cmul_acc(V acc, R mr, R mi, V v) {
    acc.x = fma(mr, v.x, acc.x);
    acc.x = fma(-mi, v.y, acc.x);
    acc.y = fma(mr, v.y, acc.y);
    acc.y = fma(mi, v.x, acc.y);
    return acc;
}

// y = M x for a 2^K-vector held in registers (M row-major, uniform).
template <int K, typename V, typename R>
__device__ __forceinline__ void small_matvec(CPtr<R> m, const V *x, V *y) {
    constexpr int D = 1 << K;
#pragma unroll
    for (int r = 0; r < D; ++r) {
        V acc;
        acc.x = 0;
        acc.y = 0;
#pragma unroll
        for (int c = 0; c < D; ++c) acc = cmul_acc(acc, m[2 * (r * D + c)], m[2 * (r * D + c) + 1], x[c]);
        y[r] = acc;
    }
}

__device__ __forceinline__ double block_sum(double v, double *red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
    return s;
}

// Gates on a thread's 8 register amplitudes x[j], j over the sweep's three
// tile bits.  Bit positions are template parameters so every register index
// is a compile-time constant.
// The first eight reals of a gate's matrix entry, read ahead of the gate
// (every one-qubit form and the two-qubit diagonal need no more).
template <typename R> struct Coef8 {
    R c[8];
    __device__ __forceinline__ R operator[](int i) const { return c[i]; }
};
template <typename R>
__device__ __forceinline__ Coef8<R> load_coef(CPtr<R> m) {
    Coef8<R> k;
#pragma unroll
    for (int i = 0; i < 8; ++i) k.c[i] = m[i];
    return k;
}

template <int B, typename V, typename M>
__device__ __forceinline__ void reg_apply1(V *x, const M &m) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        if (j & (1 << B)) continue;
        const int j1 = j | (1 << B);
        const V a = x[j], b = x[j1];
        V y0, y1;
        y0.x = y0.y = y1.x = y1.y = 0;
        y0 = cmul_acc(y0, m[0], m[1], a);
        y0 = cmul_acc(y0, m[2], m[3], b);
        y1 = cmul_acc(y1, m[4], m[5], a);
        y1 = cmul_acc(y1, m[6], m[7], b);
        x[j] = y0;
        x[j1] = y1;
    }
}

template <int B0, int B1, typename V, typename R>
__device__ __forceinline__ void reg_apply2(V *x, CPtr<R> m) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        if (j & ((1 << B0) | (1 << B1))) continue;
        const int idx[4] = {j, j | (1 << B0), j | (1 << B1), j | (1 << B0) | (1 << B1)};
        V in[4], out[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) in[c] = x[idx[c]];
        small_matvec<2>(m, in, out);
#pragma unroll
        for (int r = 0; r < 4; ++r) x[idx[r]] = out[r];
    }
}

// Diagonal gate on sweep bits (B0, B1; B1 < 0 for one qubit): x[j] *= D[j's bits].
// A one-qubit diagonal is read from its 2 x 2 matrix (entries 0 and 3), a
// two-qubit one from its compact diagonal (the host stores its four entries
// first).
template <int B0, int B1, typename V, typename M>
__device__ __forceinline__ void reg_diag(V *x, const M &m) {
    constexpr int K = B1 < 0 ? 1 : 2;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int loc = ((j >> B0) & 1) | (B1 < 0 ? 0 : ((j >> (B1 < 0 ? 0 : B1)) & 1) << 1);
        const int e = K == 1 ? 3 * loc : loc;
        const auto dr = m[2 * e], di = m[2 * e + 1];
        const V a = x[j];
        x[j].x = dr * a.x - di * a.y;
        x[j].y = dr * a.y + di * a.x;
    }
}

// Sign pattern on sweep bits (B0, B1; B1 < 0 for one qubit): x[j] = -x[j]
// where the gate's diagonal entry for j's bits is -1 (`neg`, wave-uniform).
template <int B0, int B1, typename V>
__device__ __forceinline__ void reg_sign(V *x, uint32_t neg) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int loc = ((j >> B0) & 1) | (B1 < 0 ? 0 : ((j >> (B1 < 0 ? 0 : B1)) & 1) << 1);
        if ((neg >> loc) & 1u) {
            x[j].x = -x[j].x;
            x[j].y = -x[j].y;
        }
    }
}

// Pauli pair y_j = a x_j + b s(j) x_{j^X}, s(j) = (-1)^{popc(zl & (j ^ X))}
// (X over the sweep bits, compile time; zl wave-uniform): two complex
// products per amplitude where the dense two-qubit form takes four.
template <int X, typename V, typename R>
__device__ __forceinline__ void reg_pauli(V *x, const Coef8<R> &c, uint32_t zl) {
    const R ar = c[0], ai = c[1], br = c[2], bi = c[3];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int k = j ^ X;
        if (k < j) continue;   // each pair once
        const V xj = x[j], xk = x[k];
        V pj, pk;              // b x_k, b x_j
        pj.x = br * xk.x - bi * xk.y;
        pj.y = br * xk.y + bi * xk.x;
        pk.x = br * xj.x - bi * xj.y;
        pk.y = br * xj.y + bi * xj.x;
        if (__popc(zl & (uint32_t)k) & 1) pj.x = -pj.x, pj.y = -pj.y;
        if (__popc(zl & (uint32_t)j) & 1) pk.x = -pk.x, pk.y = -pk.y;
        x[j].x = ar * xj.x - ai * xj.y + pj.x;
        x[j].y = ar * xj.y + ai * xj.x + pj.y;
        x[k].x = ar * xk.x - ai * xk.y + pk.x;
        x[k].y = ar * xk.y + ai * xk.x + pk.y;
    }
}

// Real matrix: only the real parts of the entries are read (two multiplies per entry).
template <int B, typename V, typename M>
__device__ __forceinline__ void reg_real1(V *x, const M &m) {
    const auto m00 = m[0], m01 = m[2], m10 = m[4], m11 = m[6];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        if (j & (1 << B)) continue;
        const int j1 = j | (1 << B);
        const V a = x[j], b = x[j1];
        x[j].x = fma(m00, a.x, m01 * b.x);
        x[j].y = fma(m00, a.y, m01 * b.y);
        x[j1].x = fma(m10, a.x, m11 * b.x);
        x[j1].y = fma(m10, a.y, m11 * b.y);
    }
}

template <int B0, int B1, typename V, typename R>
__device__ __forceinline__ void reg_real2(V *x, CPtr<R> m) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        if (j & ((1 << B0) | (1 << B1))) continue;
        const int idx[4] = {j, j | (1 << B0), j | (1 << B1), j | (1 << B0) | (1 << B1)};
        V in[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) in[c] = x[idx[c]];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            R ar = 0, ai = 0;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                ar = fma(m[2 * (r * 4 + c)], in[c].x, ar);
                ai = fma(m[2 * (r * 4 + c)], in[c].y, ai);
            }
            x[idx[r]].x = ar;
            x[idx[r]].y = ai;
        }
    }
}

// Fields of a packed gate record (SegGate::info).
__device__ __forceinline__ int gi_k(uint32_t i) { return 1 + (int)(i & 1u); }
__device__ __forceinline__ int gi_t0(uint32_t i) { return (int)((i >> 1) & 3u); }
__device__ __forceinline__ int gi_t1(uint32_t i) { return (int)((i >> 3) & 3u); }
__device__ __forceinline__ int gi_form(uint32_t i) { return (int)((i >> 5) & 7u); }
__device__ __forceinline__ uint32_t gi_xl(uint32_t i) { return (i >> 8) & 7u; }
__device__ __forceinline__ uint32_t gi_zl(uint32_t i) { return (i >> 11) & 7u; }
__device__ __forceinline__ bool gi_param(uint32_t i) { return (i >> 14) & 1u; }

// One gate of a sweep: `c` holds the first eight reals of its matrix entry
// (read ahead), `m` points at the whole entry (two-qubit dense forms).
template <typename V, typename R>
__device__ __forceinline__ void reg_apply(uint32_t info, V *x, const Coef8<R> &c, CPtr<R> m) {
    const int k = gi_k(info), t0 = gi_t0(info), t1 = gi_t1(info), form = gi_form(info);
    if (form == BF_PAULI) {
        const uint32_t zl = gi_zl(info);
        switch (gi_xl(info)) {
            case 1: reg_pauli<1>(x, c, zl); break;
            case 2: reg_pauli<2>(x, c, zl); break;
            case 3: reg_pauli<3>(x, c, zl); break;
            case 4: reg_pauli<4>(x, c, zl); break;
            case 5: reg_pauli<5>(x, c, zl); break;
            case 6: reg_pauli<6>(x, c, zl); break;
            default: reg_pauli<7>(x, c, zl); break;
        }
        return;
    }
    if (form == BF_SIGN) {
        const uint32_t neg = (info >> 15) & 15u;
        if (k == 1) {
            switch (t0) {
                case 0: reg_sign<0, -1>(x, neg); break;
                case 1: reg_sign<1, -1>(x, neg); break;
                default: reg_sign<2, -1>(x, neg); break;
            }
        } else if (t0 == 0) {
            if (t1 == 1) reg_sign<0, 1>(x, neg);
            else reg_sign<0, 2>(x, neg);
        } else {
            reg_sign<1, 2>(x, neg);
        }
        return;
    }
    if (form == BF_DIAG) {
        if (k == 1) {
            switch (t0) {
                case 0: reg_diag<0, -1>(x, c); break;
                case 1: reg_diag<1, -1>(x, c); break;
                default: reg_diag<2, -1>(x, c); break;
            }
        } else if (t0 == 0) {
            if (t1 == 1) reg_diag<0, 1>(x, c);
            else reg_diag<0, 2>(x, c);
        } else {
            reg_diag<1, 2>(x, c);
        }
        return;
    }
    if (form == BF_REAL) {
        if (k == 1) {
            switch (t0) {
                case 0: reg_real1<0>(x, c); break;
                case 1: reg_real1<1>(x, c); break;
                default: reg_real1<2>(x, c); break;
            }
        } else if (t0 == 0) {
            if (t1 == 1) reg_real2<0, 1>(x, m);
            else reg_real2<0, 2>(x, m);
        } else {
            reg_real2<1, 2>(x, m);
        }
        return;
    }
    if (k == 1) {
        switch (t0) {
            case 0: reg_apply1<0>(x, c); break;
            case 1: reg_apply1<1>(x, c); break;
            default: reg_apply1<2>(x, c); break;
        }
    } else if (t0 == 0) {
        if (t1 == 1) reg_apply2<0, 1>(x, m);
        else reg_apply2<0, 2>(x, m);
    } else {
        reg_apply2<1, 2>(x, m);
    }
}

// sum_j conj(l[j ^ X]) (-1)^{|z & j|} x[j] over the 8 register amplitudes
template <int X, typename V>
__device__ __forceinline__ void reg_inner_x(const V *l, const V *x, uint32_t zl, double *re, double *im) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const V a = l[j ^ X];
        const double pr = (double)a.x * x[j].x + (double)a.y * x[j].y;
        const double pi = (double)a.x * x[j].y - (double)a.y * x[j].x;
        const bool neg = __popc(zl & (uint32_t)j) & 1;
        *re += neg ? -pr : pr;
        *im += neg ? -pi : pi;
    }
}

// The same sum with the generator's x and z masks known at compile time:
// signs and partner registers are fixed, so it is straight-line adds and
// subtracts.
template <int X, int Z, typename V>
__device__ __forceinline__ void reg_inner_xz(const V *l, const V *x, double *re, double *im) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const V a = l[j ^ X];
        const double pr = (double)a.x * x[j].x + (double)a.y * x[j].y;
        const double pi = (double)a.x * x[j].y - (double)a.y * x[j].x;
        if (__builtin_popcount(Z & j) & 1) {
            *re -= pr;
            *im -= pi;
        } else {
            *re += pr;
            *im += pi;
        }
    }
}

template <typename V>
__device__ __forceinline__ void reg_inner(const V *l, const V *x, uint32_t xl, uint32_t zl, double *re, double *im) {
    // one-qubit generators on a sweep bit b: Z (0, b), X (b, 0), Y (b, b)
    switch (xl * 8 + zl) {
        case 0 * 8 + 1: reg_inner_xz<0, 1>(l, x, re, im); return;
        case 0 * 8 + 2: reg_inner_xz<0, 2>(l, x, re, im); return;
        case 0 * 8 + 4: reg_inner_xz<0, 4>(l, x, re, im); return;
        case 1 * 8 + 0: reg_inner_xz<1, 0>(l, x, re, im); return;
        case 2 * 8 + 0: reg_inner_xz<2, 0>(l, x, re, im); return;
        case 4 * 8 + 0: reg_inner_xz<4, 0>(l, x, re, im); return;
        case 1 * 8 + 1: reg_inner_xz<1, 1>(l, x, re, im); return;
        case 2 * 8 + 2: reg_inner_xz<2, 2>(l, x, re, im); return;
        case 4 * 8 + 4: reg_inner_xz<4, 4>(l, x, re, im); return;
        default: break;
    }
    switch (xl) {
        case 0: reg_inner_x<0>(l, x, zl, re, im); break;
        case 1: reg_inner_x<1>(l, x, zl, re, im); break;
        case 2: reg_inner_x<2>(l, x, zl, re, im); break;
        case 3: reg_inner_x<3>(l, x, zl, re, im); break;
        case 4: reg_inner_x<4>(l, x, zl, re, im); break;
        case 5: reg_inner_x<5>(l, x, zl, re, im); break;
        case 6: reg_inner_x<6>(l, x, zl, re, im); break;
        default: reg_inner_x<7>(l, x, zl, re, im); break;
    }
}

// Sum over a wave's 64 lanes with DPP moves, which stay in the vector unit
// (cross-lane shuffles go through the LDS crossbar and wait on it): pairs and
// quads by quad permutations, rows of 16 by shifts right by 4 and 8 (lanes
// with no source add 0), then lane 15 of each row into the next row and
// lane 31 into the upper half.  Lane 63 ends with the total.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_move(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xf, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_total63(double v) {
    v += dpp_move<0xb1, 0xf>(v);    // quad_perm [1, 0, 3, 2]
    v += dpp_move<0x4e, 0xf>(v);    // quad_perm [2, 3, 0, 1]
    v += dpp_move<0x114, 0xf>(v);   // row_shr:4
    v += dpp_move<0x118, 0xf>(v);   // row_shr:8
    v += dpp_move<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
    v += dpp_move<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
    return v;
}

__device__ __forceinline__ SegSweep load_sweep(CPtr<SegSweep> p) {
    SegSweep w;
    w.b[0] = p->b[0];
    w.b[1] = p->b[1];
    w.b[2] = p->b[2];
    w.g0 = p->g0;
    w.g1 = p->g1;
    w.p0 = p->p0;
    return w;
}

struct GateOp {             // what the sweep loop reads of a gate record
    uint32_t info, mat;
};
__device__ __forceinline__ GateOp load_op(CPtr<SegGate> p) {
    GateOp o;
    o.info = p->info;
    o.mat = p->mat;
    return o;
}

__device__ __forceinline__ BatchInst load_inst(CPtr<BatchInst> p) {
    BatchInst b;
    b.psi = p->psi;
    b.lam = p->lam;
    b.n = p->n;
    b.nslots = p->nslots;
    b.wgs = p->wgs;
    b.ngroups = p->ngroups;
    b.part_off = p->part_off;
    b.res_off = p->res_off;
    b.tg_off = p->tg_off;
    b.tt_off = p->tt_off;
    b.init_kind = p->init_kind;
    b.pad = 0;
    b.init_src = p->init_src;
    return b;
}

// LDS position of tile amplitude e: 16-byte chunk c is stored at chunk
// c ^ hash(c / 16), which keeps the coalesced load/store phases conflict-free
// and spreads the sweeps' power-of-two-strided group reads over the banks.
__device__ __forceinline__ uint32_t bswz(uint32_t c) { return c ^ (((c >> 4) ^ (c >> 8)) & 15u); }
template <int S>
__device__ __forceinline__ uint32_t bat(uint32_t e) { return (bswz(e >> S) << S) | (e & ((1u << S) - 1)); }

// FWD / ADJ segment on tile w of an instance.  LDS layout: two 64-entry
// tables that deposit the 12 bits of a run index onto the tile's high qubits,
// per-gate, per-wave partial sums of the segment's inner products (at most
// kSegMaxGates gates), then the psi tile and (ADJ only) the lambda tile, 2^tb
// amplitudes each, swizzled as above.  A forward step's launch carries one
// tile's LDS, so more of its workgroups share a compute unit.  `pair` (FWD in
// the persistent launch, whose workgroups hold two tiles of LDS anyway):
// tiles w and w + 1 of psi go through the segment together in the two tile
// slots, the second one taking the lambda tile's place.
template <typename R>
__device__ void seg_item(const BatchDev &d, CPtr<BatchRec> rec, const BatchInst &in, uint32_t w, double *red,
                         typename BAmp<R>::T *lds, bool pair) {
    using V = typename BAmp<R>::T;
    constexpr int S = sizeof(V) == 16 ? 0 : 1;      // log2(amplitudes per 16-byte chunk)
    const bool adj = rec->kind == BK_ADJ;
    const bool two = adj || pair;                    // a second tile in the lambda slot
    const uint32_t T = 1u << rec->tb;
    uint64_t *hid = reinterpret_cast<uint64_t *>(lds);            // [2][64]
    double *gsum = reinterpret_cast<double *>(hid + 128);         // [kSegMaxGates][4 waves][2]
    V *tp = reinterpret_cast<V *>(reinterpret_cast<char *>(lds) + kSegLdsExtra), *tl = tp + T;
    V *psi = reinterpret_cast<V *>(in.psi);
    V *lam = reinterpret_cast<V *>(in.lam);
    uint64_t tbase = (uint64_t)w << rec->W, tbase2 = (uint64_t)(w + 1) << rec->W;
    for (int j = 0; j < rec->khi; ++j) tbase = ins0(tbase, rec->qhi[j]), tbase2 = ins0(tbase2, rec->qhi[j]);
    // the second tile: lambda's tile w, or psi's tile w + 1 (its amplitude
    // index differs from tile w's by the XOR of the two tile bases, which
    // lie above the tile's low window)
    V *sec = pair ? psi : lam;
    const uint64_t dsec = pair ? (tbase ^ tbase2) : 0;
    for (int i = threadIdx.x; i < kSegMaxGates * 4 * 2; i += blockDim.x) gsum[i] = 0.0;
    if (threadIdx.x < 128) {
        const uint32_t h = threadIdx.x >> 6, r = threadIdx.x & 63;
        uint64_t x = 0;
        for (int j = 0; j < 6; ++j) {
            const int bit = 6 * (int)h + j;
            if (bit < rec->khi && ((r >> j) & 1u)) x |= 1ull << rec->qhi[bit];
        }
        hid[threadIdx.x] = x;
    }
    __syncthreads();
    // 16-byte chunks of the tile (a run holds at least one chunk when W >= S)
    const bool chunked = rec->W >= S;
    const uint32_t nchunk = chunked ? (T >> S) : T;
    const uint32_t wmask = (1u << rec->W) - 1;
    auto addr = [&](uint32_t e) {
        const uint32_t r = e >> rec->W;
        return tbase | (e & wmask) | hid[r & 63] | hid[64 + (r >> 6)];
    };
    if (chunked) {
        // eight chunks of each state in flight per lane (a whole 2^11-amplitude
        // complex128 or 2^12-amplitude complex64 tile per 256 lanes): the item
        // waits on its loads once instead of twice
        constexpr int DEPTH = 8;
        typedef unsigned int nu4 __attribute__((ext_vector_type(4)));
        nu4 *t16p = reinterpret_cast<nu4 *>(tp), *t16l = reinterpret_cast<nu4 *>(tl);
        const nu4 *p16 = reinterpret_cast<const nu4 *>(psi), *l16 = reinterpret_cast<const nu4 *>(sec);
        for (uint32_t c0 = threadIdx.x; c0 < nchunk; c0 += DEPTH * blockDim.x) {
            nu4 bp[DEPTH], bl[DEPTH];
#pragma unroll
            for (int u = 0; u < DEPTH; ++u) {
                const uint32_t c = c0 + u * blockDim.x;
                if (c < nchunk) {
                    const uint64_t x = addr(c << S) >> S;
                    bp[u] = p16[x];
                    if (two) bl[u] = l16[x ^ (dsec >> S)];
                }
            }
#pragma unroll
            for (int u = 0; u < DEPTH; ++u) {
                const uint32_t c = c0 + u * blockDim.x;
                if (c < nchunk) {
                    t16p[bswz(c)] = bp[u];
                    if (two) t16l[bswz(c)] = bl[u];
                }
            }
        }
    } else {
        for (uint32_t e = threadIdx.x; e < T; e += blockDim.x) {
            const uint64_t x = addr(e);
            tp[bat<S>(e)] = psi[x];
            if (two) tl[bat<S>(e)] = sec[x ^ dsec];
        }
    }
    __syncthreads();
    CPtr<R> mats = cptr(reinterpret_cast<const R *>(d.mats));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int nred = 0;
    // sweeps: each thread loads 8-amplitude groups over the sweep's three
    // tile bits once, applies the sweep's gates in registers in order (taking
    // each inner product right before its gate), and writes the group back
    const uint32_t groups = 1u << (rec->tb - 3);
    char *tpb = reinterpret_cast<char *>(tp), *tlb = reinterpret_cast<char *>(tl);
    for (uint32_t sw = rec->sw0; sw < rec->sw1; ++sw) {
        const SegSweep SW = load_sweep(cptr(d.sweeps) + sw);
        // bat<S> is linear over GF(2) (shifts, masks and XORs) and a group's
        // base and the sweep offsets have disjoint bits, so the LDS slot of
        // base | off[j] is bat(base) ^ bat(off[j]): the eight swizzled
        // offsets are wave-uniform and each access costs one XOR
        // (byte offsets: the XOR of two multiples of sizeof(V) is one)
        uint32_t so[8];
#pragma unroll
        for (int j = 0; j < 8; ++j)
            so[j] = bat<S>(((j & 1) ? (1u << SW.b[0]) : 0u) | ((j & 2) ? (1u << SW.b[1]) : 0u) |
                           ((j & 4) ? (1u << SW.b[2]) : 0u)) * (uint32_t)sizeof(V);
        for (uint32_t g0 = 0; g0 < groups; g0 += blockDim.x) {
            const uint32_t g = g0 + threadIdx.x;
            const bool act = g < groups;
            uint32_t bb = 0;
            V x[8], l[8];
            if (act) {
                bb = bat<S>(ins0_32(ins0_32(ins0_32(g, SW.b[0]), SW.b[1]), SW.b[2])) * (uint32_t)sizeof(V);
#pragma unroll
                for (int j = 0; j < 8; ++j) x[j] = *reinterpret_cast<const V *>(tpb + (bb ^ so[j]));
                if (two) {
#pragma unroll
                    for (int j = 0; j < 8; ++j) l[j] = *reinterpret_cast<const V *>(tlb + (bb ^ so[j]));
                }
            }
            int p = SW.p0;
            // read ahead: the record two gates on and the coefficients of the
            // next gate are requested while this gate is applied, so the
            // scalar loads of a gate never wait on each other
            CPtr<SegGate> sg = cptr(d.segs);
            GateOp o0 = load_op(sg + SW.g0);
            GateOp o1 = SW.g0 + 1 < SW.g1 ? load_op(sg + SW.g0 + 1) : o0;
            Coef8<R> cn = load_coef(mats + 2 * (uint64_t)o0.mat);
            for (uint32_t gi = SW.g0; gi < SW.g1; ++gi) {
                const GateOp G = o0;
                const Coef8<R> c = cn;
                o0 = o1;
                if (gi + 2 < SW.g1) o1 = load_op(sg + gi + 2);
                if (gi + 1 < SW.g1) cn = load_coef(mats + 2 * (uint64_t)o0.mat);
                if (adj && gi_param(G.info)) {
                    double re = 0.0, im = 0.0;
                    if (act) reg_inner(l, x, gi_xl(G.info), gi_zl(G.info), &re, &im);
                    re = wave_total63(re);
                    im = wave_total63(im);
                    // one wave adds into its own slot, in program order
                    if (lane == 63) {
                        atomicAdd(&gsum[(p * 4 + wave) * 2], re);
                        atomicAdd(&gsum[(p * 4 + wave) * 2 + 1], im);
                    }
                    ++p;
                }
                if (act) {
                    CPtr<R> m = mats + 2 * (uint64_t)G.mat;
                    reg_apply(G.info, x, c, m);
                    if (two) reg_apply(G.info, l, c, m);
                }
            }
            if (act) {
#pragma unroll
                for (int j = 0; j < 8; ++j) *reinterpret_cast<V *>(tpb + (bb ^ so[j])) = x[j];
                if (two) {
#pragma unroll
                    for (int j = 0; j < 8; ++j) *reinterpret_cast<V *>(tlb + (bb ^ so[j])) = l[j];
                }
            }
        }
        __syncthreads();
    }
    for (uint32_t sg = rec->sg0; sg < rec->sg1; ++sg) nred += (adj && cptr(d.segs)[sg].slot >= 0);
    // one partial per inner product: its four waves in a fixed order
    if (adj && nred) {
        int idx = 0;
        for (uint32_t sg = rec->sg0; sg < rec->sg1; ++sg) {
            const int slot = cptr(d.segs)[sg].slot;
            if (slot < 0) continue;
            if ((int)threadIdx.x == (idx & 255)) {
                double sre = 0.0, sim = 0.0;
                for (int v = 0; v < 4; ++v) {
                    sre += gsum[(idx * 4 + v) * 2];
                    sim += gsum[(idx * 4 + v) * 2 + 1];
                }
                double *p = d.partials + in.part_off + 2 * ((uint64_t)slot * in.wgs + w);
                p[0] = sre;
                p[1] = sim;
            }
            ++idx;
        }
    }
    if (chunked) {
        const uint4 *t16p = reinterpret_cast<const uint4 *>(tp), *t16l = reinterpret_cast<const uint4 *>(tl);
        uint4 *p16 = reinterpret_cast<uint4 *>(psi), *l16 = reinterpret_cast<uint4 *>(sec);
        for (uint32_t c = threadIdx.x; c < nchunk; c += blockDim.x) {
            const uint64_t x = addr(c << S) >> S;
            p16[x] = t16p[bswz(c)];
            if (two) l16[x ^ (dsec >> S)] = t16l[bswz(c)];
        }
    } else {
        for (uint32_t e = threadIdx.x; e < T; e += blockDim.x) {
            const uint64_t x = addr(e);
            psi[x] = tp[bat<S>(e)];
            if (two) sec[x ^ dsec] = tl[bat<S>(e)];
        }
    }
    __syncthreads();   // the LDS tables and tiles are reused by the next item
}

// lambda[y] = (H psi)[y] for y in [y0, y1), and partial <psi|lambda>.
template <typename R>
__device__ void hpsi_range(const BatchInst &in, const PauliSumGroup *tg, const PauliSumTerm *tt, uint64_t y0,
                           uint64_t y1, double *pre, double *pim) {
    using V = typename BAmp<R>::T;
    const V *psi = reinterpret_cast<const V *>(in.psi);
    V *lam = reinterpret_cast<V *>(in.lam);
    CPtr<PauliSumGroup> groups = cptr(tg) + in.tg_off;
    CPtr<PauliSumTerm> terms = cptr(tt) + in.tt_off;
    double sre = 0.0, sim = 0.0;
    for (uint64_t y = y0 + threadIdx.x; y < y1; y += blockDim.x) {
        double ar = 0.0, ai = 0.0;
        for (uint32_t g = 0; g < in.ngroups; ++g) {
            const uint64_t src = y ^ groups[g].x;
            const V v = psi[src];
            double cr = 0.0, ci = 0.0;
            const int t1 = groups[g].first + groups[g].count;
            for (int t = groups[g].first; t < t1; ++t) {
                const bool neg = __popcll(terms[t].z & src) & 1;
                cr += neg ? -terms[t].cre : terms[t].cre;
                ci += neg ? -terms[t].cim : terms[t].cim;
            }
            ar += cr * (double)v.x - ci * (double)v.y;
            ai += cr * (double)v.y + ci * (double)v.x;
        }
        V o;
        o.x = (R)ar;
        o.y = (R)ai;
        lam[y] = o;
        const V p = psi[y];
        // <psi|lambda> with lambda as stored (rounded to the state dtype)
        sre += (double)p.x * (double)o.x + (double)p.y * (double)o.y;
        sim += (double)p.x * (double)o.y - (double)p.y * (double)o.x;
    }
    *pre = sre;
    *pim = sim;
}

// One work item: item w of record rec.
// One work item: item w of record rec (pair: items w and w + 1 of a FWD record).
template <typename R>
__device__ void run_item(const BatchDev &d, CPtr<BatchRec> rec, uint32_t w, double *red, bool pair = false) {
    using V = typename BAmp<R>::T;
    const BatchInst in = load_inst(cptr(d.insts) + rec->inst);
    if (rec->kind != BK_HPSI) {
        seg_item<R>(d, rec, in, w, red, reinterpret_cast<V *>(batch_lds), pair);
        return;
    }
    double re = 0.0, im = 0.0;
    {
        const uint64_t N = 1ull << in.n, per = N / rec->wgs;
        hpsi_range<R>(in, d.tg, d.tt, per * w, per * (w + 1), &re, &im);
    }
    if (rec->slot >= 0) {
        const double sre = block_sum(re, red);
        const double sim = block_sum(im, red);
        if (threadIdx.x == 0) {
            double *p = d.partials + in.part_off + 2 * ((uint64_t)rec->slot * in.wgs + w);
            p[0] = sre;
            p[1] = sim;
        }
    }
}

__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Largest r in [lo, hi) with recs[r].item0 <= x.
__device__ __forceinline__ uint64_t find_rec(CPtr<BatchRec> recs, uint64_t lo, uint64_t hi, uint64_t x) {
    while (hi - lo > 1) {
        const uint64_t mid = (lo + hi) / 2;
        if (recs[mid].item0 <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

template <typename R>
__global__ void __launch_bounds__(256) k_batch_step(BatchDev d, int s) {
    __shared__ double red[4];
    const uint64_t r = find_rec(cptr(d.recs), cptr(d.step_rec)[s], cptr(d.step_rec)[s + 1], blockIdx.x);
    CPtr<BatchRec> rec = cptr(d.recs) + r;   // by pointer: its qhi[] is indexed at run time
    run_item<R>(d, rec, blockIdx.x - rec->item0, red);
}

// counters[0]: next item; counters[1]: error flag; counters[2 + i]: items
// of instance i completed.  A workgroup claims `chunk` consecutive items per
// counter atomic and publishes its completions per run of items of one
// instance; before any wait it publishes what it holds, so it never waits on
// its own unpublished work.  Items are claimed in global order and every
// dependency is on an earlier item, so the earliest unfinished item can
// always proceed.
template <typename R>
__global__ void __launch_bounds__(256) k_batch_persistent(BatchDev d, uint64_t total, unsigned long long *counters,
                                                          uint32_t spin_limit, uint32_t chunk) {
    __shared__ double red[4];
    __shared__ unsigned long long base_sh;
    __shared__ int stop_sh;
    uint32_t pend_inst = 0;     // thread 0 only: completed, unpublished items
    unsigned long long pend = 0;
    for (;;) {
        if (threadIdx.x == 0) {
            base_sh = atomicAdd(&counters[0], (unsigned long long)chunk);
            stop_sh = __hip_atomic_load(&counters[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
        }
        __syncthreads();
        // values read from LDS are not known to be uniform; read through
        // readfirstlane they are, so everything derived stays scalar
        const uint64_t base = uniform64(base_sh);
        if (base >= total || __builtin_amdgcn_readfirstlane(stop_sh)) break;
        const uint64_t end = base + chunk < total ? base + chunk : total;
        for (uint64_t item = base; item < end; ++item) {
            uint64_t lo = 0, hi = (uint64_t)d.nsteps;
            while (hi - lo > 1) {
                const uint64_t mid = (lo + hi) / 2;
                if (cptr(d.step_item)[mid] <= item) lo = mid;
                else hi = mid;
            }
            const int s = (int)lo;
            const uint64_t x = item - cptr(d.step_item)[s];
            const uint64_t r = find_rec(cptr(d.recs), cptr(d.step_rec)[s], cptr(d.step_rec)[s + 1], x);
            CPtr<BatchRec> rec = cptr(d.recs) + r;   // by pointer: its qhi[] is indexed at run time
            if (threadIdx.x == 0) {
                unsigned long long *done = &counters[2 + rec->inst];
                if (pend && pend_inst != rec->inst) {
                    __hip_atomic_fetch_add(&counters[2 + pend_inst], pend, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                    pend = 0;
                }
                // poll with relaxed loads (an acquire per poll would invalidate the
                // caches under every other workgroup), then acquire once.  A
                // spin limit of 0 fails every item that has a dependency at all,
                // so the error path can be forced from the host.
                const bool force = spin_limit == 0 && rec->need != 0;
                if (force || __hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + pend < rec->need) {
                    if (pend) {
                        __hip_atomic_fetch_add(done, pend, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                        pend = 0;
                    }
                    uint32_t spins = 0;
                    while (force || __hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < rec->need) {
                        if (++spins > spin_limit ||
                            __hip_atomic_load(&counters[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                            atomicExch(&counters[1], 1ull);
                            stop_sh = 1;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(2);
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            __syncthreads();
            if (__builtin_amdgcn_readfirstlane(stop_sh)) break;
            // two forward items of one record claimed together run as a pair
            // (same gates, both tile slots of this workgroup's LDS)
            const uint32_t w = (uint32_t)(x - rec->item0);
            const bool pair = rec->kind == BK_FWD && item + 1 < end && w + 1 < rec->wgs;
            run_item<R>(d, rec, w, red, pair);
            // the barrier makes every wave's stores visible to the workgroup;
            // thread 0's agent-scope release later publishes them device-wide
            __syncthreads();
            if (threadIdx.x == 0) {
                pend_inst = rec->inst;
                pend += pair ? 2 : 1;
            }
            if (pair) ++item;
        }
        if (threadIdx.x == 0 && pend) {
            __hip_atomic_fetch_add(&counters[2 + pend_inst], pend, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            pend = 0;
        }
        __syncthreads();
        if (__builtin_amdgcn_readfirstlane(stop_sh)) break;
    }
}

__global__ void k_batch_zero(unsigned long long *p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

template <typename R>
__global__ void __launch_bounds__(256) k_batch_init(BatchDev d) {
    using V = typename BAmp<R>::T;
    const BatchInst in = d.insts[blockIdx.y];
    V *psi = reinterpret_cast<V *>(in.psi);
    const V *src = reinterpret_cast<const V *>(in.init_src);
    const uint64_t N = 1ull << in.n;
    const R amp = (R)exp2(-0.5 * in.n);
    for (uint64_t y = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; y < N; y += (uint64_t)gridDim.x * blockDim.x) {
        V v;
        if (in.init_kind == 2) {
            v = src[y];
        } else if (in.init_kind == 1) {
            v.x = amp;
            v.y = 0;
        } else {
            v.x = y == 0 ? (R)1 : (R)0;
            v.y = 0;
        }
        psi[y] = v;
    }
}

__global__ void k_batch_finish(BatchDev d) {
    const BatchInst in = d.insts[blockIdx.x];
    for (int v = threadIdx.x; v < 2 * in.nslots; v += blockDim.x) {
        const int slot = v >> 1, c = v & 1;
        double s = 0.0;
        for (uint32_t w = 0; w < in.wgs; ++w) s += d.partials[in.part_off + 2 * ((uint64_t)slot * in.wgs + w) + c];
        d.results[in.res_off + v] = s;
    }
}

static cast_status launched(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(CAST_EHIP, std::string(what) + ": " + hipGetErrorString(e));
    return CAST_OK;
}

// Raises the kernels' dynamic-LDS limit once (segment items use more than 64 KiB).
template <typename R>
static hipError_t allow_lds() {
    static hipError_t done = [] {
        hipError_t e = hipFuncSetAttribute((const void *)k_batch_step<R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           128 << 10);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void *)k_batch_persistent<R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    128 << 10);
        return e;
    }();
    return done;
}

cast_status batch_launch_step(const BatchDev &d, cast_dtype dt, int s, uint64_t nitems, size_t lds,
                              hipStream_t st) {
    if (lds > (128u << 10)) return fail(CAST_EUNSUPPORTED, "segment tiles exceed 128 KiB of LDS");
    const hipError_t ae = dt == CAST_C128 ? allow_lds<double>() : allow_lds<float>();
    if (ae != hipSuccess) return fail(CAST_EHIP, std::string("LDS attribute: ") + hipGetErrorString(ae));
    if (dt == CAST_C128) hipLaunchKernelGGL(k_batch_step<double>, dim3((uint32_t)nitems), dim3(256), lds, st, d, s);
    else hipLaunchKernelGGL(k_batch_step<float>, dim3((uint32_t)nitems), dim3(256), lds, st, d, s);
    return launched("batched step launch");
}

cast_status batch_launch_persistent(const BatchDev &d, cast_dtype dt, uint64_t total_items, int grid,
                                    unsigned long long *counters, uint32_t spin_limit, uint32_t chunk, size_t lds,
                                    hipStream_t st) {
    if (lds > (128u << 10)) return fail(CAST_EUNSUPPORTED, "segment tiles exceed 128 KiB of LDS");
    const hipError_t ae = dt == CAST_C128 ? allow_lds<double>() : allow_lds<float>();
    if (ae != hipSuccess) return fail(CAST_EHIP, std::string("LDS attribute: ") + hipGetErrorString(ae));
    if (dt == CAST_C128)
        hipLaunchKernelGGL(k_batch_persistent<double>, dim3(grid), dim3(256), lds, st, d, total_items, counters,
                           spin_limit, chunk);
    else
        hipLaunchKernelGGL(k_batch_persistent<float>, dim3(grid), dim3(256), lds, st, d, total_items, counters,
                           spin_limit, chunk);
    return launched("persistent batch launch");
}

cast_status batch_zero(unsigned long long *p, size_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_zero, dim3(1), dim3(256), 0, st, p, n);
    return launched("counter reset");
}

cast_status batch_init_states(const BatchDev &d, cast_dtype dt, hipStream_t st) {
    if (dt == CAST_C128) hipLaunchKernelGGL(k_batch_init<double>, dim3(1024, d.ninst), dim3(256), 0, st, d);
    else hipLaunchKernelGGL(k_batch_init<float>, dim3(1024, d.ninst), dim3(256), 0, st, d);
    return launched("batch init");
}

cast_status batch_finish(const BatchDev &d, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_finish, dim3(d.ninst), dim3(256), 0, st, d);
    return launched("batch finish");
}

}  // namespace cast
