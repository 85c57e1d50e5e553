// Allocation-free variant of expval for callers that cannot allocate device
// memory (code under stream capture, tight serving loops, harnesses that
// forbid hipMalloc).
//
// expval needs device scratch for the reduction partials of k_pauli_inner
// and for the per-term results; expval takes it from the reuse pool.  Here it
// is one file-scope device array per GPU, whose device address is looked up
// once per device with hipGetSymbolAddress (in host code the array's name is
// not a device address) and passed to the same kernels expval uses.  Every
// call on a GPU uses that GPU's array, so calls that overlap on one GPU (from
// several threads, or queued on different streams) race.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <mutex>

#include "internal.hpp"
#include "reduce.hpp"

namespace cast {

namespace {

constexpr size_t kNoAllocPartials = 1024 * 2 * kMaxZ;   // reduce_scratch_doubles(), checked below
constexpr size_t kNoAllocDoubles = kNoAllocPartials + 2 * (size_t)CAST_EXPVAL_NOALLOC_MAX_TERMS;

static __device__ __align__(256) double scratch[kNoAllocDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_sym_mu;
double *g_sym_ptr[kMaxDevices] = {nullptr};

// Device address of `scratch` on the current device (looked up on the first
// call per device, with that device current).
cast_status scratch_ptr(double **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(CAST_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(CAST_EUNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> g(g_sym_mu);
    if (!g_sym_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(CAST_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_sym_ptr[dev] = (double *)p;
    }
    *out = g_sym_ptr[dev];
    return CAST_OK;
}

const std::complex<double> kIp[4] = {{1, 0}, {0, 1}, {-1, 0}, {0, -1}};

}  // namespace

}  // namespace cast

using namespace cast;

extern "C" {

cast_status expval_noalloc(const cast_sv *sv, const cast_pauli_term *terms, size_t n_terms, double *out) {
    if (!sv || !sv->data) return fail(CAST_EINVAL, "state is NULL");
    if (!out) return fail(CAST_EINVAL, "out is NULL");
    if (n_terms && !terms) return fail(CAST_EINVAL, "terms is NULL");
    if (n_terms > (size_t)CAST_EXPVAL_NOALLOC_MAX_TERMS)
        return fail(CAST_EINVAL, "expval_noalloc: more terms than the fixed scratch holds (" +
                                     std::to_string(CAST_EXPVAL_NOALLOC_MAX_TERMS) + ")");
    if (reduce_scratch_doubles() != kNoAllocPartials) return fail(CAST_EUNSUPPORTED, "reduction scratch size changed");
    const uint64_t full = sv->n >= 64 ? ~0ull : ((1ull << sv->n) - 1);
    for (size_t i = 0; i < n_terms; ++i)
        if ((terms[i].xmask | terms[i].zmask) & ~full) return fail(CAST_EINVAL, "Pauli term acts outside the state");
    out[0] = out[1] = 0.0;
    if (!n_terms) return CAST_OK;
    double *base = nullptr;
    if (cast_status rc = scratch_ptr(&base)) return rc;
    double *partials = base, *res = base + kNoAllocPartials;

    // Terms sharing an x mask go to one pass, up to kMaxZ z masks at a time;
    // results land in slot order, slot[i] = the term's place in that order.
    // Fixed-size host arrays: nothing is allocated, on the host either.
    uint16_t slot[CAST_EXPVAL_NOALLOC_MAX_TERMS];
    bool done[CAST_EXPVAL_NOALLOC_MAX_TERMS] = {false};
    uint32_t next = 0;
    for (size_t i = 0; i < n_terms; ++i) {
        if (done[i]) continue;
        const uint64_t x = terms[i].xmask;
        size_t j = i;
        while (j < n_terms) {
            uint64_t zs[kMaxZ];
            int nz = 0;
            const uint32_t first = next;
            for (; j < n_terms && nz < kMaxZ; ++j) {
                if (done[j] || terms[j].xmask != x) continue;
                done[j] = true;
                slot[j] = (uint16_t)next++;
                zs[nz++] = terms[j].zmask;
            }
            if (!nz) break;
            if (cast_status rc = pauli_inner(sv->data, sv->data, sv->n, sv->dt, x, zs, nz, partials, res + 2 * first,
                                             sv->stream))
                return rc;
        }
    }
    double h[2 * CAST_EXPVAL_NOALLOC_MAX_TERMS];
    CAST_HIP_TRY(hipMemcpyAsync(h, res, 2 * n_terms * sizeof(double), hipMemcpyDeviceToHost, sv->stream));
    CAST_HIP_TRY(hipStreamSynchronize(sv->stream));
    std::complex<double> e = 0;
    for (size_t i = 0; i < n_terms; ++i) {
        const std::complex<double> S(h[2 * slot[i]], h[2 * slot[i] + 1]);
        e += terms[i].coeff * kIp[__builtin_popcountll(terms[i].xmask & terms[i].zmask) & 3] * S;
    }
    out[0] = e.real();
    out[1] = e.imag();
    return CAST_OK;
}

}  // extern "C"
