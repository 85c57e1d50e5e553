// Streaming reference kernel: an in-place scale of a buffer of doubles, the
// simplest pass that reads and writes every byte once.  It shares the access
// pattern of the elementwise gate kernels (16 bytes per lane, several chunks
// in flight per lane, non-temporal hints, grid-stride over tiles) and does no
// gate work, so its rate is the practical ceiling those kernels are measured
// against.
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace cast {

namespace {

typedef unsigned int st_u4 __attribute__((ext_vector_type(4)));
typedef double st_d2 __attribute__((ext_vector_type(2)));

template <int U>
__global__ void __launch_bounds__(256) k_stream_scale(st_u4 *__restrict__ p, uint64_t nchunks, double f) {
    constexpr uint64_t per = 256ull * U;
    const uint64_t ntiles = nchunks / per;
    for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        st_u4 w[U];
#pragma unroll
        for (int u = 0; u < U; ++u) w[u] = __builtin_nontemporal_load(p + t * per + (uint64_t)u * 256 + threadIdx.x);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            st_d2 v = *reinterpret_cast<st_d2 *>(&w[u]);
            v.x *= f;
            v.y *= f;
            __builtin_nontemporal_store(*reinterpret_cast<st_u4 *>(&v), p + t * per + (uint64_t)u * 256 + threadIdx.x);
        }
    }
    // chunks past the last whole tile
    for (uint64_t c = ntiles * per + (uint64_t)blockIdx.x * 256 + threadIdx.x; c < nchunks;
         c += (uint64_t)gridDim.x * 256) {
        st_d2 v = *reinterpret_cast<st_d2 *>(&p[c]);
        v.x *= f;
        v.y *= f;
        p[c] = *reinterpret_cast<st_u4 *>(&v);
    }
}

}  // namespace

}  // namespace cast

using namespace cast;

extern "C" {

cast_status stream_scale(void *data, size_t bytes, double factor, int chunks_per_lane, int grid, void *hip_stream) {
    if (!data) return fail(CAST_EINVAL, "data is NULL");
    if (bytes % 16 || ((uintptr_t)data & 15)) return fail(CAST_EINVAL, "stream_scale: 16-byte aligned whole chunks only");
    if (chunks_per_lane != 1 && chunks_per_lane != 2 && chunks_per_lane != 4 && chunks_per_lane != 8)
        return fail(CAST_EINVAL, "stream_scale: chunks_per_lane must be 1, 2, 4 or 8");
    if (grid < 0) return fail(CAST_EINVAL, "stream_scale: negative grid");
    const uint64_t nchunks = bytes / 16;
    if (!nchunks) return CAST_OK;
    const uint64_t per = 256ull * chunks_per_lane;
    uint64_t g = (nchunks + per - 1) / per;
    if (grid > 0 && (uint64_t)grid < g) g = (uint64_t)grid;
    if (g > 0x7fffffffull) g = 0x7fffffffull;
    hipStream_t s = (hipStream_t)hip_stream;
    st_u4 *p = (st_u4 *)data;
    switch (chunks_per_lane) {
        case 1: hipLaunchKernelGGL(k_stream_scale<1>, dim3((unsigned)g), dim3(256), 0, s, p, nchunks, factor); break;
        case 2: hipLaunchKernelGGL(k_stream_scale<2>, dim3((unsigned)g), dim3(256), 0, s, p, nchunks, factor); break;
        case 4: hipLaunchKernelGGL(k_stream_scale<4>, dim3((unsigned)g), dim3(256), 0, s, p, nchunks, factor); break;
        default: hipLaunchKernelGGL(k_stream_scale<8>, dim3((unsigned)g), dim3(256), 0, s, p, nchunks, factor); break;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(CAST_EHIP, std::string("stream_scale launch: ") + hipGetErrorString(e));
    return CAST_OK;
}

}  // extern "C"
