// C ABI of libcast (declared in include/cast.h): argument validation, state
// objects, host->device matrix staging, and the host side of each entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>

#include "internal.hpp"

namespace cast {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

cast_status fail(cast_status code, const std::string &msg) {
    g_err = msg;
    return code;
}

Tuning &tuning() {
    static Tuning t = [] {
        Tuning x;
        // CAST_<KNOB> sets both dtypes, CAST_<KNOB>_C64 / _C128 one of them
        auto env = [](const char *name, int *v) {
            if (const char *s = std::getenv(name)) v[CAST_C64] = v[CAST_C128] = std::atoi(s);
            const std::string n64 = std::string(name) + "_C64", n128 = std::string(name) + "_C128";
            if (const char *s = std::getenv(n64.c_str())) v[CAST_C64] = std::atoi(s);
            if (const char *s = std::getenv(n128.c_str())) v[CAST_C128] = std::atoi(s);
        };
        env("CAST_DIRECT_MIN_Q", x.direct_min_q);
        env("CAST_TILE_BITS", x.tile_bits);
        env("CAST_DIRECT_IPT", x.direct_ipt);
        env("CAST_DIRECT_NT", x.direct_nt);
        env("CAST_DIRECT_CHUNK_LOG", x.direct_chunk_log);
        env("CAST_MAX_GRID", x.max_grid);
        env("CAST_USE_DIAG", x.use_diag);
        env("CAST_DIAG_UNROLL", x.diag_unroll);
        env("CAST_DIAG_MAX_GRID", x.diag_max_grid);
        env("CAST_DIAG_LDS_TABLE", x.diag_lds_table);
        env("CAST_DIAG_ORDER", x.diag_order);
        env("CAST_MFMA_MIN_D", x.mfma_min_d);
        env("CAST_MFMA_GRID_PER_CU", x.mfma_grid_per_cu);
        env("CAST_MFMA_DIRECT_MIN_Q", x.mfma_direct_min_q);
        env("CAST_MFMA_LOW_TILE", x.mfma_low_tile);
        env("CAST_MFMA_3M_MIN_D", x.mfma_3m_min_d);
        env("CAST_BLOCKED_TILE_BITS", x.blocked_tile_bits);
        env("CAST_BLOCKED_THREADS", x.blocked_threads);
        return x;
    }();
    return t;
}

// Pass-cost table (ms per 2^30 amplitudes), by dtype, k, d.  Initial values:
// every pass streams the state once at 5 TB/s, plus the FMA time at half of
// the FP peak for dense blocks.
static double g_cost[3][kMaxK + 1][kMaxK + 1];
static bool g_cost_init = [] {
    for (int dt = 1; dt <= 2; ++dt)
        for (int k = 1; k <= kMaxK; ++k)
            for (int d = 0; d <= k; ++d) {
                const double amp = dt == CAST_C128 ? 16.0 : 8.0;
                const double mem_ms = 2.0 * amp * 1073741824.0 / 5e12 * 1e3;
                const double peak = dt == CAST_C128 ? 78.6e12 : 157.3e12;
                const double fl_ms = 8.0 * std::ldexp(1.0, d) * 1073741824.0 / (0.5 * peak) * 1e3;
                g_cost[dt][k][d] = std::max(mem_ms, fl_ms);
            }
    return true;
}();

double pass_cost(cast_dtype dt, int k, int d) { return g_cost[dt][k][d]; }

// ----------------------------------------------------------------- memory
static std::mutex g_mem_mu;
static size_t g_mem_used = 0;

static size_t mem_cap() {
    static size_t cap = [] {
        const char *s = std::getenv("CAST_MAX_DEVICE_BYTES");
        return s ? (size_t)std::strtoull(s, nullptr, 10) : (size_t)0;
    }();
    return cap;
}

static std::mutex g_size_mu;
static std::vector<std::pair<void *, size_t>> g_sizes;

cast_status dev_alloc(void **ptr, size_t bytes) {
    *ptr = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mem_mu);
        if (mem_cap() && g_mem_used + bytes > mem_cap())
            return fail(CAST_ENOMEM, "allocation of " + std::to_string(bytes) +
                                         " bytes exceeds CAST_MAX_DEVICE_BYTES");
        g_mem_used += bytes;
    }
    hipError_t e = hipMalloc(ptr, bytes ? bytes : 16);
    if (e != hipSuccess) {
        std::lock_guard<std::mutex> lk(g_mem_mu);
        g_mem_used -= bytes;
        *ptr = nullptr;
        (void)hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? CAST_ENOMEM : CAST_EHIP,
                    std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    std::lock_guard<std::mutex> lk(g_size_mu);
    g_sizes.emplace_back(*ptr, bytes);
    return CAST_OK;
}

// Reuse pool for per-call scratch (expval, adjoint_grad): blocks are kept
// per device in power-of-two size classes and handed out again instead of
// being freed, so a call makes no hipMalloc/hipFree (each free synchronises
// the device) once the pool holds its sizes.  A block goes back only after
// its call has synchronised its stream.  At most kPoolKeep bytes stay pooled.
namespace {
struct PoolBlock {
    void *p;
    size_t bytes;
    int dev;
};
std::mutex g_pool_mu;
std::vector<PoolBlock> g_pool;
size_t g_pool_bytes = 0;
constexpr size_t kPoolKeep = size_t(8) << 30;
size_t pool_class(size_t bytes) {
    size_t c = 256;
    while (c < bytes) c <<= 1;
    return c;
}
}  // namespace

cast_status pool_alloc(void **ptr, size_t bytes, size_t *cls) {
    *cls = pool_class(bytes);
    int dev = 0;
    (void)hipGetDevice(&dev);
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        for (size_t i = 0; i < g_pool.size(); ++i)
            if (g_pool[i].bytes == *cls && g_pool[i].dev == dev) {
                *ptr = g_pool[i].p;
                g_pool_bytes -= g_pool[i].bytes;
                g_pool[i] = g_pool.back();
                g_pool.pop_back();
                return CAST_OK;
            }
    }
    return dev_alloc(ptr, *cls);
}

void pool_free(void *ptr, size_t cls) {
    if (!ptr) return;
    int dev = 0;
    (void)hipGetDevice(&dev);
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        if (g_pool_bytes + cls <= kPoolKeep) {
            g_pool.push_back(PoolBlock{ptr, cls, dev});
            g_pool_bytes += cls;
            return;
        }
    }
    dev_free(ptr);
}

void dev_free(void *ptr) {
    if (!ptr) return;
    size_t bytes = 0;
    {
        std::lock_guard<std::mutex> lk(g_size_mu);
        for (size_t i = 0; i < g_sizes.size(); ++i)
            if (g_sizes[i].first == ptr) {
                bytes = g_sizes[i].second;
                g_sizes[i] = g_sizes.back();
                g_sizes.pop_back();
                break;
            }
    }
    (void)hipFree(ptr);
    std::lock_guard<std::mutex> lk(g_mem_mu);
    g_mem_used -= bytes;
}

// ----------------------------------------------------------------- uploads
template <typename R>
static void pack(const PassPlan &p, std::vector<R> &dst) {
    pack_plan<R>(p, dst);
}

// Every plan's matrices, cast to the state dtype, one after another with each
// plan's start 256-byte aligned (for scalar loads); offsets in reals.
static size_t pack_all(const std::vector<PassPlan> &ps, cast_dtype dt, std::vector<double> &hd,
                       std::vector<float> &hf, std::vector<size_t> *offsets) {
    offsets->clear();
    size_t elems = 0;
    for (const PassPlan &p : ps) {
        offsets->push_back(elems);
        if (dt == CAST_C128) pack<double>(p, hd), elems = hd.size();
        else pack<float>(p, hf), elems = hf.size();
        const size_t align = 256 / (dt == CAST_C128 ? 8 : 4);
        while (elems % align) {
            if (dt == CAST_C128) hd.push_back(0); else hf.push_back(0);
            ++elems;
        }
    }
    return elems;
}

std::vector<size_t> plan_offsets(const std::vector<PassPlan> &ps, cast_dtype dt) {
    std::vector<double> hd;
    std::vector<float> hf;
    std::vector<size_t> off;
    pack_all(ps, dt, hd, hf, &off);
    return off;
}

cast_status upload_plans_pooled(const std::vector<PassPlan> &ps, cast_dtype dt, void **ptr, size_t *cls,
                                std::vector<size_t> *offsets) {
    std::vector<double> hd;
    std::vector<float> hf;
    const size_t elems = pack_all(ps, dt, hd, hf, offsets);
    const size_t bytes = elems * (dt == CAST_C128 ? 8 : 4);
    if (cast_status st = pool_alloc(ptr, bytes, cls)) return st;
    if (bytes) {
        const hipError_t e = hipMemcpy(*ptr, dt == CAST_C128 ? (void *)hd.data() : (void *)hf.data(), bytes,
                                       hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            pool_free(*ptr, *cls);
            *ptr = nullptr;
            return fail(CAST_EHIP, std::string("matrix upload: ") + hipGetErrorString(e));
        }
    }
    return CAST_OK;
}

cast_status upload_plans(const std::vector<PassPlan> &ps, cast_dtype dt, DeviceMatrix *out,
                         std::vector<size_t> *offsets) {
    std::vector<double> hd;
    std::vector<float> hf;
    const size_t elems = pack_all(ps, dt, hd, hf, offsets);
    const size_t bytes = elems * (dt == CAST_C128 ? 8 : 4);
    cast_status st = dev_alloc(&out->ptr, bytes);
    if (st) return st;
    out->bytes = bytes;
    if (bytes) {
        hipError_t e = hipMemcpy(out->ptr, dt == CAST_C128 ? (void *)hd.data() : (void *)hf.data(), bytes,
                                 hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            dev_free(out->ptr);
            out->ptr = nullptr;
            return fail(CAST_EHIP, std::string("matrix upload: ") + hipGetErrorString(e));
        }
    }
    return CAST_OK;
}

cast_status upload_plan(const PassPlan &p, cast_dtype dt, DeviceMatrix *out) {
    std::vector<size_t> off;
    return upload_plans(std::vector<PassPlan>{p}, dt, out, &off);
}

// Matrix buffers for apply_gate, shared by all host threads.  A slot is
// claimed under the lock (busy) and stays claimed until apply_gate has
// recorded its completion event after the launch that reads it; only then
// can another call take it, and only once the stream has passed that event.
// The copy itself runs outside the lock.  std::deque keeps slot addresses
// valid while new slots are appended.
struct Staging {
    void *ptr = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
    bool busy = false;
};
static std::mutex g_stage_mu;
static std::deque<Staging> g_stage;

static void release_slot(Staging *slot) {
    std::lock_guard<std::mutex> lk(g_stage_mu);
    slot->busy = false;
}

static cast_status stage_matrix(const PassPlan &p, cast_dtype dt, hipStream_t s, Staging **out) {
    std::vector<double> hd;
    std::vector<float> hf;
    size_t bytes;
    const void *src;
    if (dt == CAST_C128) { pack<double>(p, hd); bytes = hd.size() * 8; src = hd.data(); }
    else { pack<float>(p, hf); bytes = hf.size() * 4; src = hf.data(); }
    Staging *slot = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_stage_mu);
        for (Staging &st : g_stage)
            if (!st.busy && st.bytes >= bytes && hipEventQuery(st.done) == hipSuccess) { slot = &st; break; }
        if (!slot) {
            Staging st;
            st.bytes = std::max<size_t>(bytes, 4096);
            cast_status rc = dev_alloc(&st.ptr, st.bytes);
            if (rc) return rc;
            if (hipEventCreateWithFlags(&st.done, hipEventDisableTiming) != hipSuccess) {
                dev_free(st.ptr);
                return fail(CAST_EHIP, "hipEventCreate failed");
            }
            g_stage.push_back(st);
            slot = &g_stage.back();
        }
        slot->busy = true;
    }
    // stream-ordered copy from pageable memory; the synchronisation makes the
    // host buffer's lifetime irrelevant
    hipError_t e = hipMemcpyAsync(slot->ptr, src, bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        release_slot(slot);
        return fail(CAST_EHIP, std::string("matrix staging: ") + hipGetErrorString(e));
    }
    *out = slot;
    return CAST_OK;
}

static cast_status check_sv(const cast_sv *sv) {
    if (!sv) return fail(CAST_EINVAL, "state is NULL");
    if (!sv->data) return fail(CAST_ESTATE, "state has no device memory");
    return CAST_OK;
}

static cast_status check_qubits(int n, const int *qubits, int k) {
    if (k < 1 || k > kMaxK) return fail(CAST_EINVAL, "k must be in [1, 6], got " + std::to_string(k));
    if (!qubits) return fail(CAST_EINVAL, "qubits is NULL");
    if (k > n) return fail(CAST_EINVAL, "gate has more qubits than the state");
    for (int i = 0; i < k; ++i) {
        if (qubits[i] < 0 || qubits[i] >= n)
            return fail(CAST_EINVAL, "qubit " + std::to_string(qubits[i]) + " out of range");
        for (int j = 0; j < i; ++j)
            if (qubits[j] == qubits[i]) return fail(CAST_EINVAL, "duplicate qubit " + std::to_string(qubits[i]));
    }
    return CAST_OK;
}

static std::vector<cplx> read_matrix(int k, const double *m) {
    const size_t D = (size_t)1 << k;
    std::vector<cplx> out(D * D);
    for (size_t i = 0; i < D * D; ++i) out[i] = cplx(m[2 * i], m[2 * i + 1]);
    return out;
}

}  // namespace cast

using namespace cast;

extern "C" {

const char *cast_last_error(void) { return g_err.c_str(); }

void pool_trim(void) {
    std::vector<PoolBlock> blocks;
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        blocks.swap(g_pool);
        g_pool_bytes = 0;
    }
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (const PoolBlock &b : blocks) {
        (void)hipSetDevice(b.dev);
        dev_free(b.p);
    }
    (void)hipSetDevice(cur);
}

// ----------------------------------------------------------------- states
cast_status sv_create(int n, cast_dtype dt, void *hip_stream, cast_sv **out) {
    if (!out) return fail(CAST_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || n > kMaxQubits) return fail(CAST_EINVAL, "n must be in [1, 34]");
    if (dt != CAST_C64 && dt != CAST_C128) return fail(CAST_EINVAL, "dtype must be CAST_C64 or CAST_C128");
    const size_t bytes = ((size_t)1 << n) * amp_bytes(dt);
    void *p = nullptr;
    cast_status rc = dev_alloc(&p, bytes);
    if (rc) return rc;
    cast_sv *sv = new cast_sv;
    sv->data = p;
    sv->n = n;
    sv->dt = dt;
    sv->stream = (hipStream_t)hip_stream;
    sv->owns = true;
    rc = sv_set_basis(sv, 0);
    if (rc) {
        sv_destroy(sv);
        return rc;
    }
    *out = sv;
    return CAST_OK;
}

cast_status sv_wrap(void *dev_ptr, int n, cast_dtype dt, void *hip_stream, cast_sv **out) {
    if (!out) return fail(CAST_EINVAL, "out is NULL");
    *out = nullptr;
    if (!dev_ptr) return fail(CAST_EINVAL, "dev_ptr is NULL");
    if (((uintptr_t)dev_ptr) & 15) return fail(CAST_EINVAL, "dev_ptr must be 16-byte aligned");
    if (n < 1 || n > kMaxQubits) return fail(CAST_EINVAL, "n must be in [1, 34]");
    if (dt != CAST_C64 && dt != CAST_C128) return fail(CAST_EINVAL, "dtype must be CAST_C64 or CAST_C128");
    cast_sv *sv = new cast_sv;
    sv->data = dev_ptr;
    sv->n = n;
    sv->dt = dt;
    sv->stream = (hipStream_t)hip_stream;
    sv->owns = false;
    *out = sv;
    return CAST_OK;
}

void sv_destroy(cast_sv *sv) {
    if (!sv) return;
    if (sv->owns && sv->data) {
        (void)hipStreamSynchronize(sv->stream);
        dev_free(sv->data);
    }
    sv->data = nullptr;
    delete sv;
}

cast_status sv_copy_from_host(cast_sv *sv, const void *host, size_t bytes) {
    if (cast_status rc = check_sv(sv)) return rc;
    if (!host) return fail(CAST_EINVAL, "host is NULL");
    if (bytes != ((size_t)1 << sv->n) * amp_bytes(sv->dt)) return fail(CAST_EINVAL, "byte count mismatch");
    CAST_HIP_TRY(hipMemcpyAsync(sv->data, host, bytes, hipMemcpyHostToDevice, sv->stream));
    CAST_HIP_TRY(hipStreamSynchronize(sv->stream));
    return CAST_OK;
}

cast_status sv_copy_to_host(const cast_sv *sv, void *host, size_t bytes) {
    if (cast_status rc = check_sv(sv)) return rc;
    if (!host) return fail(CAST_EINVAL, "host is NULL");
    if (bytes != ((size_t)1 << sv->n) * amp_bytes(sv->dt)) return fail(CAST_EINVAL, "byte count mismatch");
    CAST_HIP_TRY(hipMemcpyAsync(host, sv->data, bytes, hipMemcpyDeviceToHost, sv->stream));
    CAST_HIP_TRY(hipStreamSynchronize(sv->stream));
    return CAST_OK;
}

cast_status sv_set_basis(cast_sv *sv, uint64_t index) {
    if (cast_status rc = check_sv(sv)) return rc;
    if (sv->n < 64 && index >= ((uint64_t)1 << sv->n)) return fail(CAST_EINVAL, "basis index out of range");
    const size_t ab = amp_bytes(sv->dt);
    CAST_HIP_TRY(hipMemsetAsync(sv->data, 0, ((size_t)1 << sv->n) * ab, sv->stream));
    static const double one_d[2] = {1.0, 0.0};
    static const float one_f[2] = {1.0f, 0.0f};
    CAST_HIP_TRY(hipMemcpyAsync((char *)sv->data + index * ab, sv->dt == CAST_C128 ? (const void *)one_d
                                                                                   : (const void *)one_f,
                                ab, hipMemcpyHostToDevice, sv->stream));
    CAST_HIP_TRY(hipStreamSynchronize(sv->stream));
    return CAST_OK;
}

cast_status sv_info(const cast_sv *sv, void **dev_ptr, int *n, cast_dtype *dt) {
    if (!sv) return fail(CAST_EINVAL, "state is NULL");
    if (dev_ptr) *dev_ptr = sv->data;
    if (n) *n = sv->n;
    if (dt) *dt = sv->dt;
    return CAST_OK;
}

// ----------------------------------------------------------------- gates
cast_status apply_gate(cast_sv *sv, const int *qubits, int k, const double *matrix) {
    if (cast_status rc = check_sv(sv)) return rc;
    if (cast_status rc = check_qubits(sv->n, qubits, k)) return rc;
    if (!matrix) return fail(CAST_EINVAL, "matrix is NULL");
    std::vector<cplx> m = read_matrix(k, matrix);
    PassPlan p;
    if (cast_status rc = make_plan(k, qubits, m.data(), 1e-14, 1e-14, &p)) return rc;
    if (p.identity()) return CAST_OK;
    Staging *slot = nullptr;
    if (cast_status rc = stage_matrix(p, sv->dt, sv->stream, &slot)) return rc;
    cast_status rc = launch_pass(sv->data, sv->n, sv->dt, p, slot->ptr, sv->stream);
    // a slot whose event could not be recorded is never handed out again
    CAST_HIP_TRY(hipEventRecord(slot->done, sv->stream));
    release_slot(slot);
    return rc;
}

cast_status gate_matrix(const char *name, const double *params, int *k, double *out) {
    if (!name || !k || !out) return fail(CAST_EINVAL, "NULL argument");
    static const double zeros[3] = {0, 0, 0};
    std::vector<cplx> m;
    if (!standard_gate(name, params ? params : zeros, k, &m))
        return fail(CAST_EINVAL, std::string("unknown gate ") + name);
    for (size_t i = 0; i < m.size(); ++i) {
        out[2 * i] = m[i].real();
        out[2 * i + 1] = m[i].imag();
    }
    return CAST_OK;
}

static int *tuning_field(const std::string &key, cast_dtype dt, int *lo, int *hi) {
    Tuning &t = tuning();
    const int i = dt == CAST_C64 ? CAST_C64 : CAST_C128;
    *lo = 0;
    *hi = 1 << 30;
    if (key == "direct_min_q") { *hi = 34; return &t.direct_min_q[i]; }
    if (key == "tile_bits") { *lo = 10; *hi = 13; return &t.tile_bits[i]; }
    if (key == "direct_ipt") { *lo = 1; *hi = 4; return &t.direct_ipt[i]; }
    if (key == "direct_nt") { *hi = 1; return &t.direct_nt[i]; }
    if (key == "direct_chunk_log") { *lo = 6; *hi = 16; return &t.direct_chunk_log[i]; }
    if (key == "max_grid") { *lo = 256; return &t.max_grid[i]; }
    if (key == "use_diag") { *hi = 1; return &t.use_diag[i]; }
    if (key == "diag_unroll") { *lo = 1; *hi = 8; return &t.diag_unroll[i]; }
    if (key == "diag_max_grid") { *lo = 256; return &t.diag_max_grid[i]; }
    if (key == "diag_lds_table") { *hi = 1; return &t.diag_lds_table[i]; }
    if (key == "diag_order") { *hi = 1; return &t.diag_order[i]; }
    if (key == "mfma_min_d") { *lo = 4; *hi = 7; return &t.mfma_min_d[i]; }
    if (key == "mfma_grid_per_cu") { *lo = 1; *hi = 16; return &t.mfma_grid_per_cu[i]; }
    if (key == "mfma_direct_min_q") { *hi = 34; return &t.mfma_direct_min_q[i]; }
    if (key == "mfma_low_tile") { *hi = 1; return &t.mfma_low_tile[i]; }
    if (key == "mfma_3m_min_d") { *lo = 4; *hi = 7; return &t.mfma_3m_min_d[i]; }
    if (key == "blocked_tile_bits") { *lo = 8; *hi = i == CAST_C64 ? 13 : 12; return &t.blocked_tile_bits[i]; }
    if (key == "blocked_threads") { *lo = 256; *hi = 1024; return &t.blocked_threads[i]; }
    if (key == "persistent_spin_limit") return &t.persistent_spin_limit[i];
    if (key == "diag_run_tables") { *hi = kRunMaxTables; return &t.diag_run_tables[i]; }
    if (key == "diag_run_qubits") { *lo = 4; *hi = kRunMaxQ; return &t.diag_run_qubits[i]; }
    if (key == "diag_run_unroll") { *lo = 1; *hi = 4; return &t.diag_run_unroll[i]; }
    if (key == "diag_run_grid") { *lo = 256; return &t.diag_run_grid[i]; }
    if (key == "diag_run_lds") { *hi = 1; return &t.diag_run_lds[i]; }
    if (key == "mfma_prefetch") { *hi = 2; return &t.mfma_prefetch[i]; }
    if (key == "diag_spread") { *hi = 1; return &t.diag_spread[i]; }
    if (key == "diag_run_reuse") { *hi = 12; return &t.diag_run_reuse[i]; }
    if (key == "direct_rot") { *hi = 16; return &t.direct_rot[i]; }
    if (key == "direct_rot_lo") { *hi = 34; return &t.direct_rot_lo[i]; }
    if (key == "direct_rot_hi") { *hi = 34; return &t.direct_rot_hi[i]; }
    if (key == "batch_tile_bits") { *lo = 4; *hi = 12; return &t.batch_tile_bits[i]; }
    if (key == "batch_min_window") { *hi = 10; return &t.batch_min_window[i]; }
    return nullptr;
}

cast_status tuning_set(const char *key, cast_dtype dt, int value) {
    if (!key) return fail(CAST_EINVAL, "key is NULL");
    int lo, hi;
    int *f = tuning_field(key, dt, &lo, &hi);
    if (!f) return fail(CAST_EINVAL, std::string("unknown tuning key ") + key);
    if (value < lo || value > hi || (std::string(key) == "direct_ipt" && value == 3) ||
        (std::string(key) == "diag_unroll" && (value & (value - 1))) ||
        (std::string(key) == "diag_run_unroll" && (value & (value - 1))) ||
        (std::string(key) == "blocked_threads" && (value & (value - 1))))
        return fail(CAST_EINVAL, std::string("value out of range for ") + key);
    *f = value;
    return CAST_OK;
}

cast_status tuning_get(const char *key, cast_dtype dt, int *value) {
    if (!key || !value) return fail(CAST_EINVAL, "NULL argument");
    int lo, hi;
    int *f = tuning_field(key, dt, &lo, &hi);
    if (!f) return fail(CAST_EINVAL, std::string("unknown tuning key ") + key);
    *value = *f;
    return CAST_OK;
}

cast_status cost_table_set(cast_dtype dt, int k, int d, double v) {
    if (dt != CAST_C64 && dt != CAST_C128) return fail(CAST_EINVAL, "bad dtype");
    if (k < 1 || k > kMaxK || d < 0 || d > k) return fail(CAST_EINVAL, "need 1 <= k <= 6, 0 <= d <= k");
    if (!(v > 0)) return fail(CAST_EINVAL, "cost must be positive");
    g_cost[dt][k][d] = v;
    return CAST_OK;
}

cast_status cost_table_get(cast_dtype dt, int k, int d, double *v) {
    if (dt != CAST_C64 && dt != CAST_C128) return fail(CAST_EINVAL, "bad dtype");
    if (k < 1 || k > kMaxK || d < 0 || d > k || !v) return fail(CAST_EINVAL, "bad argument");
    *v = g_cost[dt][k][d];
    return CAST_OK;
}

void fusion_opts_default(cast_fusion_opts *o) {
    if (!o) return;
    o->k_max = 5;
    o->opcount_cap = 0;
    o->zero_tol = 1e-14;
    o->one_tol = 1e-14;
    o->agglomerative = 1;
    o->multi_traversal = 1;
    o->cost_model = 0;
    o->cost_dtype = CAST_C128;
}

cast_status fuse_circuit(int n, const cast_gate *gates, size_t n_gates, const cast_fusion_opts *opts,
                         cast_fused **out) {
    if (!out) return fail(CAST_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || n > kMaxQubits) return fail(CAST_EINVAL, "n must be in [1, 34]");
    if (n_gates && !gates) return fail(CAST_EINVAL, "gates is NULL");
    cast_fusion_opts o;
    fusion_opts_default(&o);
    if (opts) o = *opts;
    if (o.k_max < 1 || o.k_max > kMaxK) return fail(CAST_EINVAL, "k_max must be in [1, 6]");
    if (o.cost_model < 0 || o.cost_model > 1) return fail(CAST_EINVAL, "cost_model must be 0 or 1");
    if (o.cost_dtype == 0) o.cost_dtype = CAST_C128;
    if (o.cost_dtype != CAST_C64 && o.cost_dtype != CAST_C128) return fail(CAST_EINVAL, "bad cost_dtype");
    auto t0 = std::chrono::steady_clock::now();
    std::vector<FusionGate> in;
    in.reserve(n_gates);
    for (size_t i = 0; i < n_gates; ++i) {
        const cast_gate &g = gates[i];
        if (cast_status rc = check_qubits(n, g.qubits, g.k)) return rc;
        if (g.param_id >= 0 || !g.matrix)
            return fail(CAST_EINVAL, "fuse_circuit takes fixed gates (matrix set, param_id = -1)");
        // sort the gate's qubits, permuting its matrix
        PassPlan p;
        std::vector<cplx> m = read_matrix(g.k, g.matrix);
        if (cast_status rc = make_plan(g.k, g.qubits, m.data(), 0.0, 0.0, &p)) return rc;
        FusionGate fg;
        fg.qubits.assign(p.q, p.q + g.k);
        fg.m = p.full;
        in.push_back(std::move(fg));
    }
    std::vector<FusionGate> fused;
    if (cast_status rc = fuse(n, std::move(in), o, &fused)) return rc;
    cast_fused *f = new cast_fused;
    f->n = n;
    for (const FusionGate &g : fused) {
        PassPlan p;
        if (cast_status rc = make_plan((int)g.qubits.size(), g.qubits.data(), g.m.data(), o.zero_tol,
                                       o.one_tol, &p)) {
            delete f;
            return rc;
        }
        f->plans.push_back(std::move(p));
    }
    f->fusion_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = f;
    return CAST_OK;
}

cast_status fused_info(const cast_fused *f, size_t *n_fused, double *total_opcount, double *fusion_ms) {
    if (!f) return fail(CAST_EINVAL, "fused list is NULL");
    if (n_fused) *n_fused = f->plans.size();
    if (total_opcount) {
        double s = 0;
        for (const PassPlan &p : f->plans) s += p.opcount;
        *total_opcount = s;
    }
    if (fusion_ms) *fusion_ms = f->fusion_ms;
    return CAST_OK;
}

cast_status fused_gate(const cast_fused *f, size_t i, int *k, int *qubits, double *opcount, int *subspace_dim,
                       int *active_blocks, double *matrix) {
    if (!f) return fail(CAST_EINVAL, "fused list is NULL");
    if (i >= f->plans.size()) return fail(CAST_EINVAL, "index out of range");
    const PassPlan &p = f->plans[i];
    if (k) *k = p.k;
    if (qubits)
        for (int j = 0; j < kMaxK; ++j) qubits[j] = j < p.k ? p.q[j] : -1;
    if (opcount) *opcount = p.opcount;
    if (subspace_dim) *subspace_dim = p.d;
    if (active_blocks) *active_blocks = (int)p.blk.size();
    if (matrix)
        for (size_t j = 0; j < p.full.size(); ++j) {
            matrix[2 * j] = p.full[j].real();
            matrix[2 * j + 1] = p.full[j].imag();
        }
    return CAST_OK;
}

}  // extern "C"

namespace cast {

// The pass schedule of a fused list for (n, dt), built with the current knobs
// and cached in the list; with `upload`, its run tables are on the device.
static cast_status get_schedule(cast_fused *f, int n, cast_dtype dt, bool upload, Schedule **out) {
    const Tuning &tu = tuning();
    Schedule *s = f->sched[dt];
    if (s && (s->n != n || s->run_tables != tu.diag_run_tables[dt] || s->run_qubits != tu.diag_run_qubits[dt] ||
              s->use_diag != tu.use_diag[dt])) {
        schedule_free(s);
        s = f->sched[dt] = nullptr;
    }
    if (!s) {
        s = new Schedule;
        if (cast_status rc = build_schedule(f->plans, n, dt, s)) {
            delete s;
            return rc;
        }
        f->sched[dt] = s;
    }
    if (upload && !s->dev.ptr)
        if (cast_status rc = upload_schedule(s)) return rc;
    *out = s;
    return CAST_OK;
}

static cast_status launch_sched_pass(cast_sv *sv, cast_fused *f, const Schedule &sc, const SchedPass &sp) {
    if (sp.kind == 6) return launch_diag_run(sv->data, sv->n, sv->dt, sp, sc.dev.ptr, sv->stream);
    const size_t rsz = sv->dt == CAST_C128 ? 8 : 4;
    const void *dm = (const char *)f->dev[sv->dt].ptr + f->dev_off[sv->dt][sp.first] * rsz;
    return launch_pass(sv->data, sv->n, sv->dt, f->plans[sp.first], dm, sv->stream, &sp.shape);
}

static cast_status prepare_circuit(cast_sv *sv, const cast_fused *fc, cast_fused **f, Schedule **sc) {
    if (cast_status rc = check_sv(sv)) return rc;
    if (!fc) return fail(CAST_EINVAL, "fused list is NULL");
    if (fc->n != sv->n) return fail(CAST_EINVAL, "fused list was built for a different qubit count");
    *f = const_cast<cast_fused *>(fc);
    const int dt = sv->dt;
    if (!(*f)->dev[dt].ptr && !(*f)->plans.empty())
        if (cast_status rc = upload_plans((*f)->plans, sv->dt, &(*f)->dev[dt], &(*f)->dev_off[dt])) return rc;
    return get_schedule(*f, sv->n, sv->dt, true, sc);
}

}  // namespace cast

extern "C" {

cast_status apply_circuit(cast_sv *sv, const cast_fused *fc) {
    cast_fused *f;
    Schedule *sc;
    if (cast_status rc = prepare_circuit(sv, fc, &f, &sc)) return rc;
    for (const SchedPass &sp : sc->passes)
        if (cast_status rc = launch_sched_pass(sv, f, *sc, sp)) return rc;
    return CAST_OK;
}

cast_status apply_circuit_timed(cast_sv *sv, const cast_fused *fc, float *pass_ms) {
    if (!pass_ms) return fail(CAST_EINVAL, "NULL argument");
    cast_fused *f;
    Schedule *sc;
    if (cast_status rc = prepare_circuit(sv, fc, &f, &sc)) return rc;
    const size_t np = sc->passes.size();
    std::vector<hipEvent_t> ev(np + 1);
    for (auto &e : ev) CAST_HIP_TRY(hipEventCreate(&e));
    cast_status rc = CAST_OK;
    CAST_HIP_TRY(hipEventRecord(ev[0], sv->stream));
    for (size_t i = 0; i < np && !rc; ++i) {
        rc = launch_sched_pass(sv, f, *sc, sc->passes[i]);
        if (!rc) CAST_HIP_TRY(hipEventRecord(ev[i + 1], sv->stream));
    }
    if (!rc) {
        CAST_HIP_TRY(hipEventSynchronize(ev[np]));
        for (size_t i = 0; i < np; ++i) CAST_HIP_TRY(hipEventElapsedTime(&pass_ms[i], ev[i], ev[i + 1]));
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    return rc;
}

cast_status circuit_pass_shape(const cast_fused *fc, int n, cast_dtype dt, size_t i, int *rot, int *chunk_log) {
    if (!fc) return fail(CAST_EINVAL, "fused list is NULL");
    if (dt != CAST_C64 && dt != CAST_C128) return fail(CAST_EINVAL, "bad dtype");
    if (n != fc->n) return fail(CAST_EINVAL, "n differs from the fused list's");
    Schedule *sc;
    if (cast_status rc = get_schedule(const_cast<cast_fused *>(fc), n, dt, false, &sc)) return rc;
    if (i >= sc->passes.size()) return fail(CAST_EINVAL, "pass index out of range");
    if (rot) *rot = sc->passes[i].shape.rot;
    if (chunk_log) *chunk_log = sc->passes[i].shape.chunk_log;
    return CAST_OK;
}

cast_status circuit_set_pass_shape(cast_fused *fc, int n, cast_dtype dt, size_t i, int rot, int chunk_log) {
    if (!fc) return fail(CAST_EINVAL, "fused list is NULL");
    if (dt != CAST_C64 && dt != CAST_C128) return fail(CAST_EINVAL, "bad dtype");
    if (n != fc->n) return fail(CAST_EINVAL, "n differs from the fused list's");
    if (rot < -1 || rot > 16) return fail(CAST_EINVAL, "rot must be -1..16");
    if (chunk_log != -1 && (chunk_log < 6 || chunk_log > 16)) return fail(CAST_EINVAL, "chunk_log must be -1 or 6..16");
    Schedule *sc;
    if (cast_status rc = get_schedule(fc, n, dt, false, &sc)) return rc;
    if (i >= sc->passes.size()) return fail(CAST_EINVAL, "pass index out of range");
    sc->passes[i].shape.rot = rot;
    sc->passes[i].shape.chunk_log = chunk_log;
    return CAST_OK;
}

cast_status circuit_tune(cast_sv *sv, cast_fused *fc, int reps, double *before_ms, double *after_ms) {
    if (reps < 1 || reps > 100) return fail(CAST_EINVAL, "reps must be 1..100");
    cast_fused *f;
    Schedule *sc;
    if (cast_status rc = prepare_circuit(sv, fc, &f, &sc)) return rc;
    const int n = sv->n;
    const cast_dtype dt = sv->dt;
    const Tuning &tu = tuning();
    std::vector<hipEvent_t> ev(2 * (size_t)reps);
    for (auto &e : ev) CAST_HIP_TRY(hipEventCreate(&e));
    cast_status rc = CAST_OK;
    // minimum over reps of one launch of pass sp with shape sh (ms)
    auto time_shape = [&](SchedPass &sp, const PassShape &sh, double *ms) -> cast_status {
        const PassShape keep = sp.shape;
        sp.shape = sh;
        cast_status r = CAST_OK;
        for (int j = 0; j < reps && !r; ++j) {
            if (hipEventRecord(ev[2 * j], sv->stream) != hipSuccess) r = fail(CAST_EHIP, "hipEventRecord");
            if (!r) r = launch_sched_pass(sv, f, *sc, sp);
            if (!r && hipEventRecord(ev[2 * j + 1], sv->stream) != hipSuccess) r = fail(CAST_EHIP, "hipEventRecord");
        }
        sp.shape = keep;
        if (r) return r;
        if (hipEventSynchronize(ev[2 * reps - 1]) != hipSuccess) return fail(CAST_EHIP, "hipEventSynchronize");
        double best = 1e30;
        for (int j = 0; j < reps; ++j) {
            float t = 0;
            if (hipEventElapsedTime(&t, ev[2 * j], ev[2 * j + 1]) != hipSuccess) return fail(CAST_EHIP, "hipEventElapsedTime");
            best = std::min(best, (double)t);
        }
        *ms = best;
        return CAST_OK;
    };
    double before = 0, after = 0;
    for (size_t i = 0; i < sc->passes.size() && !rc; ++i) {
        SchedPass &sp = sc->passes[i];
        // diagonal runs in the unit-reuse kernel: unit-order rotation only
        const bool drun = sp.kind == 6 && tu.diag_run_reuse[dt] > 0 && n > (dt == CAST_C128 ? 8 : 9);
        if ((sp.kind < 0 || sp.kind > 5) && !drun) continue;
        const PassPlan &pl = f->plans[sp.first];
        const int kind = drun ? 6 : pass_kernel_kind(n, dt, pl);
        // every kind but the direct one takes a unit- or tile-order rotation only
        const bool rot_only = kind != 0;
        const int k = pl.k;
        // the knobs' shape first, then run lengths (direct passes), then
        // rotations at the best run length (8 for rotation-only passes)
        const PassShape knob{-1, -1};
        double t_knob = 0;
        if ((rc = time_shape(sp, knob, &t_knob))) break;
        PassShape best = knob;
        double t_best = t_knob;
        int best_cl = rot_only ? -1 : std::min(std::max(tu.direct_chunk_log[dt], 6), n - k);
        for (int cl : {8, 10, 12}) {
            if (rot_only || cl > n - k || cl == best_cl) continue;
            double t = 0;
            if ((rc = time_shape(sp, PassShape{0, cl}, &t))) break;
            if (t < t_best) t_best = t, best = PassShape{0, cl}, best_cl = cl;
        }
        for (int rot : {2, 4, 6, 8}) {
            if (rc) break;
            if (rot == 8 && !rot_only) continue;
            double t = 0;
            if ((rc = time_shape(sp, PassShape{rot, best_cl}, &t))) break;
            if (t < t_best) t_best = t, best = PassShape{rot, best_cl};
        }
        if (rc) break;
        // a shape other than the knobs' must win by more than timing noise
        if (t_best > 0.99 * t_knob) best = knob, t_best = t_knob;
        sp.shape = best;
        before += t_knob;
        after += t_best;
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    if (rc) return rc;
    if (before_ms) *before_ms = before;
    if (after_ms) *after_ms = after;
    return CAST_OK;
}

cast_status circuit_passes(const cast_fused *fc, int n, cast_dtype dt, size_t *n_passes) {
    if (!fc || !n_passes) return fail(CAST_EINVAL, "NULL argument");
    if (dt != CAST_C64 && dt != CAST_C128) return fail(CAST_EINVAL, "bad dtype");
    if (n != fc->n) return fail(CAST_EINVAL, "n differs from the fused list's");
    Schedule *sc;
    if (cast_status rc = get_schedule(const_cast<cast_fused *>(fc), n, dt, false, &sc)) return rc;
    *n_passes = sc->passes.size();
    return CAST_OK;
}

cast_status circuit_pass_info(const cast_fused *fc, int n, cast_dtype dt, size_t i, size_t *first, size_t *count,
                              int *kernel, int *tables, double *alg_bytes, double *flops) {
    if (!fc) return fail(CAST_EINVAL, "fused list is NULL");
    if (dt != CAST_C64 && dt != CAST_C128) return fail(CAST_EINVAL, "bad dtype");
    if (n != fc->n) return fail(CAST_EINVAL, "n differs from the fused list's");
    Schedule *sc;
    if (cast_status rc = get_schedule(const_cast<cast_fused *>(fc), n, dt, false, &sc)) return rc;
    if (i >= sc->passes.size()) return fail(CAST_EINVAL, "pass index out of range");
    const SchedPass &sp = sc->passes[i];
    if (first) *first = sp.first;
    if (count) *count = sp.count;
    // a single gate's kernel follows the current knobs (the cached schedule
    // only keys on the knobs that change which gates form runs)
    if (kernel) *kernel = (sp.kind == 6 || sp.kind < 0) ? sp.kind : pass_kernel_kind(n, dt, fc->plans[sp.first]);
    if (tables) *tables = (int)sp.tabs.size();
    if (sp.kind == 6) {
        if (alg_bytes) *alg_bytes = 2.0 * (double)amp_bytes(dt) * sp.active_amps;
        if (flops) *flops = 8.0 * sp.active_amps;
        return CAST_OK;
    }
    return fused_pass_info(fc, sp.first, n, dt, nullptr, nullptr, alg_bytes, flops);
}

cast_status fused_pass_info(const cast_fused *f, size_t i, int n, cast_dtype dt, int *kernel, int *d,
                            double *alg_bytes, double *flops) {
    if (!f) return fail(CAST_EINVAL, "fused list is NULL");
    if (i >= f->plans.size()) return fail(CAST_EINVAL, "index out of range");
    if (dt != CAST_C64 && dt != CAST_C128) return fail(CAST_EINVAL, "bad dtype");
    if (n != f->n) return fail(CAST_EINVAL, "n differs from the fused list's");
    const PassPlan &p = f->plans[i];
    if (kernel) *kernel = p.identity() ? -1 : pass_kernel_kind(n, dt, p);
    if (d) *d = p.d;
    const double groups = std::ldexp(1.0, n - p.k), nb = (double)p.blk.size(), bd = std::ldexp(1.0, p.d);
    if (alg_bytes) *alg_bytes = 2.0 * (double)amp_bytes(dt) * groups * nb * bd;
    if (flops) *flops = 8.0 * groups * nb * bd * bd;
    return CAST_OK;
}

void fused_destroy(cast_fused *f) {
    if (!f) return;
    for (int d = 0; d < 3; ++d)
        dev_free(f->dev[d].ptr), blocked_free(f->blocked[d]), jit_free(f->jit[d]), schedule_free(f->sched[d]);
    delete f;
}

}  // extern "C"
