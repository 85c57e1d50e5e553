// Pauli-string reductions and Pauli-sum application for gfx950.
//
// A Pauli string is P = i^{|x&z|} X^x Z^z (bit q of x/z gives qubit q's
// letter), so (P psi)[y ^ x] = i^{|x&z|} (-1)^{|z&y|} psi[y] and
//   <a|P|b> = i^{|x&z|} * S(x, z),  S(x, z) = sum_y conj(a[y^x]) (-1)^{|z&y|} b[y].
// k_pauli_inner computes S for up to 8 z-masks sharing one x-mask in a single
// pass over the two states, accumulating products in FP64 (complex64 inputs
// are promoted per product).  Reduction order is fixed (grid-stride partials,
// wave shuffles, LDS tree, then one finishing block), so results are bitwise
// reproducible for a given n.
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "reduce.hpp"

namespace cast {

template <typename R> struct AmpR;
template <> struct AmpR<double> { using T = double2; };
template <> struct AmpR<float> { using T = float2; };

constexpr int kRedThreads = 256;
constexpr int kRedMaxBlocks = 1024;

struct ZMasks {
    uint64_t z[kMaxZ];
};

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <typename R, int NZ>
__global__ void __launch_bounds__(kRedThreads) k_pauli_inner(const R *__restrict__ a_r, const R *__restrict__ b_r,
                                                            uint64_t N, uint64_t x, ZMasks zm, int nz,
                                                            double *__restrict__ partial) {
    using V = typename AmpR<R>::T;
    const V *a = reinterpret_cast<const V *>(a_r);
    const V *b = reinterpret_cast<const V *>(b_r);
    double acc[NZ][2];
#pragma unroll
    for (int j = 0; j < NZ; ++j) acc[j][0] = acc[j][1] = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t y = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; y < N; y += stride) {
        const V av = a[y ^ x];
        const V bv = b[y];
        const double ar = av.x, ai = av.y, br = bv.x, bi = bv.y;
        const double pr = ar * br + ai * bi;
        const double pi = ar * bi - ai * br;
#pragma unroll
        for (int j = 0; j < NZ; ++j) {
            if (j < nz) {
                const bool neg = __popcll(zm.z[j] & y) & 1;
                acc[j][0] += neg ? -pr : pr;
                acc[j][1] += neg ? -pi : pi;
            }
        }
    }
    __shared__ double red[kRedThreads / 64][2 * NZ];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < NZ; ++j) {
        const double s0 = wave_sum(acc[j][0]);
        const double s1 = wave_sum(acc[j][1]);
        if (lane == 0) {
            red[wave][2 * j] = s0;
            red[wave][2 * j + 1] = s1;
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * NZ) {
        double s = 0.0;
        for (int w = 0; w < kRedThreads / 64; ++w) s += red[w][threadIdx.x];
        partial[(size_t)blockIdx.x * (2 * NZ) + threadIdx.x] = s;
    }
}

// One block: out[v] = sum over blocks of partial[blk][v], fixed order.
__global__ void __launch_bounds__(kRedThreads) k_finish(const double *__restrict__ partial, int nblocks, int nvals,
                                                       int stride_vals, double *__restrict__ out) {
    __shared__ double red[kRedThreads];
    for (int v = 0; v < nvals; ++v) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += blockDim.x) s += partial[(size_t)b * stride_vals + v];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = blockDim.x / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[v] = red[0];
        __syncthreads();
    }
}

static int red_blocks(int n) {
    const uint64_t N = 1ull << n;
    uint64_t b = (N + kRedThreads * 4 - 1) / (kRedThreads * 4);
    if (b > kRedMaxBlocks) b = kRedMaxBlocks;
    if (b < 1) b = 1;
    return (int)b;
}

size_t reduce_scratch_doubles() { return (size_t)kRedMaxBlocks * 2 * kMaxZ; }

cast_status pauli_inner(const void *a, const void *b, int n, cast_dtype dt, uint64_t x, const uint64_t *z, int nz,
                        double *scratch, double *dev_out, hipStream_t s) {
    if (nz < 1 || nz > kMaxZ) return fail(CAST_EINVAL, "pauli_inner: 1..8 z-masks per call");
    ZMasks zm;
    for (int j = 0; j < kMaxZ; ++j) zm.z[j] = j < nz ? z[j] : 0;
    const int blocks = red_blocks(n);
    const uint64_t N = 1ull << n;
    if (nz == 1) {
        if (dt == CAST_C128)
            hipLaunchKernelGGL((k_pauli_inner<double, 1>), dim3(blocks), dim3(kRedThreads), 0, s, (const double *)a,
                               (const double *)b, N, x, zm, nz, scratch);
        else
            hipLaunchKernelGGL((k_pauli_inner<float, 1>), dim3(blocks), dim3(kRedThreads), 0, s, (const float *)a,
                               (const float *)b, N, x, zm, nz, scratch);
        hipLaunchKernelGGL(k_finish, dim3(1), dim3(kRedThreads), 0, s, scratch, blocks, 2, 2, dev_out);
    } else {
        if (dt == CAST_C128)
            hipLaunchKernelGGL((k_pauli_inner<double, kMaxZ>), dim3(blocks), dim3(kRedThreads), 0, s,
                               (const double *)a, (const double *)b, N, x, zm, nz, scratch);
        else
            hipLaunchKernelGGL((k_pauli_inner<float, kMaxZ>), dim3(blocks), dim3(kRedThreads), 0, s,
                               (const float *)a, (const float *)b, N, x, zm, nz, scratch);
        hipLaunchKernelGGL(k_finish, dim3(1), dim3(kRedThreads), 0, s, scratch, blocks, 2 * nz, 2 * kMaxZ, dev_out);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(CAST_EHIP, std::string("reduction launch: ") + hipGetErrorString(e));
    return CAST_OK;
}

// out[y] = sum_groups sum_{m in group} c_m (-1)^{|z_m & (y^x_g)|} psi[y ^ x_g]
// where c_m already includes i^{|x&z|}.  Term table layout (device):
//   groups: {x, first term, term count}, terms: {z, c_re, c_im}.
template <typename R>
__global__ void __launch_bounds__(256) k_apply_pauli_sum(const R *__restrict__ psi_r, R *__restrict__ out_r,
                                                        uint64_t N, const PauliSumGroup *__restrict__ groups,
                                                        int ngroups, const PauliSumTerm *__restrict__ terms) {
    using V = typename AmpR<R>::T;
    const V *psi = reinterpret_cast<const V *>(psi_r);
    V *out = reinterpret_cast<V *>(out_r);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t y = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; y < N; y += stride) {
        double accr = 0.0, acci = 0.0;
        for (int g = 0; g < ngroups; ++g) {
            const uint64_t x = groups[g].x;
            const uint64_t src = y ^ x;
            const V v = psi[src];
            double sr = 0.0, si = 0.0;
            const int t0 = groups[g].first, t1 = t0 + groups[g].count;
            for (int t = t0; t < t1; ++t) {
                const bool neg = __popcll(terms[t].z & src) & 1;
                sr += neg ? -terms[t].cre : terms[t].cre;
                si += neg ? -terms[t].cim : terms[t].cim;
            }
            const double vr = v.x, vi = v.y;
            accr += sr * vr - si * vi;
            acci += sr * vi + si * vr;
        }
        V o;
        o.x = (R)accr;
        o.y = (R)acci;
        out[y] = o;
    }
}

cast_status apply_pauli_sum(const void *psi, void *out, int n, cast_dtype dt, const PauliSumGroup *dgroups,
                            int ngroups, const PauliSumTerm *dterms, hipStream_t s) {
    const uint64_t N = 1ull << n;
    uint64_t grid = (N + 255) / 256;
    if (grid > 8192) grid = 8192;
    if (dt == CAST_C128)
        hipLaunchKernelGGL(k_apply_pauli_sum<double>, dim3(grid), dim3(256), 0, s, (const double *)psi,
                           (double *)out, N, dgroups, ngroups, dterms);
    else
        hipLaunchKernelGGL(k_apply_pauli_sum<float>, dim3(grid), dim3(256), 0, s, (const float *)psi, (float *)out,
                           N, dgroups, ngroups, dterms);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(CAST_EHIP, std::string("pauli-sum launch: ") + hipGetErrorString(e));
    return CAST_OK;
}

}  // namespace cast
