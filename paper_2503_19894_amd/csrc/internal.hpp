// Internal declarations shared by the host sources of libcast.
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "../../include/cast.h"

namespace cast {

using cplx = std::complex<double>;

// ----------------------------------------------------------------- errors
void set_error(const std::string &msg);
cast_status fail(cast_status code, const std::string &msg);

#define CAST_HIP_TRY(expr)                                                              \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return ::cast::fail(CAST_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ----------------------------------------------------------------- limits
constexpr int kMaxQubits = 34;
constexpr int kMaxK = 6;

inline size_t amp_bytes(cast_dtype dt) { return dt == CAST_C128 ? 16 : 8; }

// ----------------------------------------------------------------- pass plan
// One device pass of a k-qubit gate.  Targets are sorted; the local (group
// member) index j has bit i <-> q[i].  The matrix's nonzero pattern spans an
// XOR subspace V of local indices; `L` is an invertible GF(2) relabelling
// whose first d columns span V, so that in virtual coordinates u the matrix is
// block-diagonal with 2^(k-d) dense blocks of 2^d x 2^d.  Identity blocks are
// dropped from `blk`.
struct PassPlan {
    int k = 0;
    int q[kMaxK] = {0};
    int d = 0;
    uint32_t L[kMaxK] = {0};        // physical local index of virtual basis vector i
    std::vector<uint32_t> blk;      // active block ids b in [0, 2^(k-d))
    std::vector<cplx> mat;          // blk.size() x 2^d x 2^d, row-major per block
    std::vector<cplx> full;         // snapped FP64 matrix, bit i <-> q[i] (for reports)
    double opcount = 0;             // 2 x nonzero real scalars (Sec. III-C)
    bool identity() const { return blk.empty(); }
};

// Builds the plan of a gate given on (unsorted) qubits with bit i <-> qubits[i].
cast_status make_plan(int k, const int *qubits, const cplx *m, double zero_tol, double one_tol,
                      PassPlan *out);

// Operation count of Sec. III-C: two operations per nonzero real scalar.
double opcount_of(const std::vector<cplx> &m);

// ----------------------------------------------------------------- device side
struct DeviceMatrix {                // a plan's block matrices in the state dtype
    void *ptr = nullptr;
    size_t bytes = 0;
};

struct Tuning {                      // launch parameters, by dtype index (CAST_C64, CAST_C128)
    int direct_min_q[3] = {0, 4, 4}; // smallest target for the direct kernel
    int tile_bits[3] = {0, 12, 12};  // LDS tile size log2(amplitudes)
    int direct_ipt[3] = {0, 4, 4};   // work items per thread per iteration (capped by registers)
    int direct_nt[3] = {0, 1, 1};    // non-temporal loads/stores in the direct kernel
    int direct_chunk_log[3] = {0, 8, 8};  // direct kernel: log2(groups per block run), 6..16
    int max_grid[3] = {0, 1 << 20, 1 << 20};
    int use_diag[3] = {0, 1, 1};     // elementwise kernel for diagonal passes
    int diag_unroll[3] = {0, 4, 4};  // diagonal kernel: 16-byte chunks per thread per iteration
    int diag_max_grid[3] = {0, 1 << 20, 1 << 20};
    int diag_lds_table[3] = {0, 1, 1};   // diagonal kernel: phases staged in LDS (else read from L1)
    int diag_order[3] = {0, 1, 1};       // diagonal kernel: 0 pattern-fastest, 1 pattern-major tile order
    int mfma_min_d[3] = {0, 4, 4};   // smallest block dimension sent to the MFMA kernels
    int mfma_grid_per_cu[3] = {0, 4, 4};
    int mfma_direct_min_q[3] = {0, 4, 4};  // smallest target for the MFMA direct gather
    int mfma_low_tile[3] = {0, 1, 1};  // low-target d <= 4 MFMA passes on the LDS tile when its runs are long
    int mfma_3m_min_d[3] = {0, 6, 6};  // matrix cores: three-multiplication complex product from this d (7: never)
    int blocked_tile_bits[3] = {0, 13, 12};  // cache-blocked passes: log2(amplitudes per LDS tile)
    int blocked_threads[3] = {0, 512, 512};  // cache-blocked passes: threads per workgroup (256, 512, 1024)
    // persistent batch launch: polls before a dependency wait gives up; 0
    // makes every dependency fail at once (exercises the error path)
    int persistent_spin_limit[3] = {0, 1 << 24, 1 << 24};
    // diagonal runs: tables per merged elementwise pass (0: one pass per
    // fused gate), qubits per table, chunks per thread, workgroup cap
    int diag_run_tables[3] = {0, 4, 3};
    int diag_run_qubits[3] = {0, 8, 8};
    int diag_run_unroll[3] = {0, 2, 4};
    int diag_run_grid[3] = {0, 1 << 16, 1 << 16};
    int diag_run_lds[3] = {0, 1, 1};     // diagonal runs: phase tables in LDS (1) or read through L1 (0)
    int mfma_prefetch[3] = {0, 1, 1};    // matrix-core direct kernel: 1 all of a unit's loads before its
                                         // products, 2 also the next unit's (0: one k-step ahead)
    int diag_spread[3] = {0, 1, 1};      // diagonal kernels: tiles dealt to XCDs by a digit hash (else round-robin)
    // diagonal runs: log2 of the free-bit patterns one work unit streams with
    // one phase lookup per lane (phase reuse; 0: the tiled run kernel)
    int diag_run_reuse[3] = {0, 2, 2};
    // direct kernel: iteration order rotated left by direct_rot bits (0: in
    // order) for passes whose lowest target is in [direct_rot_lo, direct_rot_hi]
    int direct_rot[3] = {0, 0, 0};
    int direct_rot_lo[3] = {0, 18, 18};
    int direct_rot_hi[3] = {0, 25, 25};
    // batched programs: log2 amplitudes of a segment's LDS tile
    int batch_tile_bits[3] = {0, 11, 11};
    // batched programs: low bits every segment's tile keeps (runs of 2^w
    // consecutive amplitudes per tile load)
    int batch_min_window[3] = {0, 2, 3};
};
Tuning &tuning();
// Predicted ms per 2^30 amplitudes of a (k, d) pass, by dtype (cost_table_set).
double pass_cost(cast_dtype dt, int k, int d);
// Dimension of the XOR subspace spanned by a matrix's nonzero pattern.
int subspace_dim(int k, const std::vector<cplx> &m, double zero_tol);

// Kernel a pass uses: 0 direct, 1 LDS tile, 2 LDS tile with two buffers,
// 3 elementwise diagonal, 4 MFMA direct, 5 MFMA tile.
bool mfma_fits(int n, cast_dtype dt, const PassPlan &p);
// Device layout of a plan's matrices (reals of the state dtype): the active
// blocks, or for diagonal plans (d = 0) the full diagonal of 2^k entries.
template <typename R>
void pack_plan(const PassPlan &p, std::vector<R> &dst) {
    if (p.d == 0) {
        const size_t D = (size_t)1 << p.k;
        for (size_t j = 0; j < D; ++j) {
            dst.push_back((R)p.full[j * D + j].real());
            dst.push_back((R)p.full[j * D + j].imag());
        }
        return;
    }
    for (const cplx &z : p.mat) {
        dst.push_back((R)z.real());
        dst.push_back((R)z.imag());
    }
}
int pass_kernel_kind(int n, cast_dtype dt, const PassPlan &p);

// Launch shape of one direct pass, overriding the knobs (-1: the knob's
// value): rotation of the iteration order and log2 of the block run length.
struct PassShape {
    int rot = -1;
    int chunk_log = -1;
};

// Queues one pass on `stream`.  `dmat` holds the plan's blocks in dtype `dt`.
cast_status launch_pass(void *psi, int n, cast_dtype dt, const PassPlan &p, const void *dmat,
                        hipStream_t stream, const PassShape *shape = nullptr);

// Uploads a plan's matrices (cast to dt) into a new device buffer; the host
// staging is synchronous (the buffer is ready when this returns).
cast_status upload_plan(const PassPlan &p, cast_dtype dt, DeviceMatrix *out);
cast_status upload_plans(const std::vector<PassPlan> &ps, cast_dtype dt, DeviceMatrix *out,
                         std::vector<size_t> *offsets);
// The offsets (in reals) upload_plans gives each plan, computed on the host.
std::vector<size_t> plan_offsets(const std::vector<PassPlan> &ps, cast_dtype dt);

// ----------------------------------------------------------------- pass schedule
// The passes apply_circuit makes: one per fused gate, except that a run of
// consecutive diagonal fused gates is applied in one elementwise pass with
// its phases combined into at most kRunMaxTables tables of at most kRunMaxQ
// qubits (diagrun.hip).
constexpr int kRunMaxTables = 4;
constexpr int kRunMaxQ = 8;
struct PhaseTable {                  // phases over k sorted qubits, entry j: bit i <-> q[i]
    int k = 0;
    int q[kRunMaxQ] = {0};
    std::vector<cplx> ph;
};
struct SchedPass {
    size_t first = 0, count = 1;     // fused gates [first, first + count)
    int kind = 0;                    // pass_kernel_kind of a single gate, -1 identity, 6 diagonal run
    std::vector<PhaseTable> tabs;    // kind 6
    size_t tab_off = 0;              // kind 6: entry offset of its tables in the device buffer
    double active_amps = 0;          // kind 6: amplitudes at which some table differs from 1
    PassShape shape;                 // kinds 0 and 4: launch shape (circuit_tune)
};
struct Schedule {
    int n = 0;
    cast_dtype dt = CAST_C128;
    int run_tables = 0, run_qubits = 0, use_diag = 0;   // knobs it was built with
    std::vector<SchedPass> passes;
    DeviceMatrix dev;                // run tables in the state dtype, 256 entries per table
};
bool diag_pass(int n, cast_dtype dt, const PassPlan &p);
cast_status build_schedule(const std::vector<PassPlan> &plans, int n, cast_dtype dt, Schedule *out);
cast_status upload_schedule(Schedule *s);
cast_status launch_diag_run(void *psi, int n, cast_dtype dt, const SchedPass &p, const void *dtabs,
                            hipStream_t stream);
void schedule_free(Schedule *s);

// Device allocation with the CAST_MAX_DEVICE_BYTES cap.
cast_status dev_alloc(void **ptr, size_t bytes);
void dev_free(void *ptr);
// Pooled scratch: *cls receives the block's size class, which pool_free
// needs back.  Return a block only once the work using it has completed.
cast_status pool_alloc(void **ptr, size_t bytes, size_t *cls);
void pool_free(void *ptr, size_t cls);
// upload_plans into a pooled block (synchronous copy).
cast_status upload_plans_pooled(const std::vector<PassPlan> &ps, cast_dtype dt, void **ptr, size_t *cls,
                                std::vector<size_t> *offsets);

// ----------------------------------------------------------------- fusion
struct FusionGate {                  // a gate as fusion sees it
    std::vector<int> qubits;         // sorted
    std::vector<cplx> m;             // bit i <-> qubits[i]
};
cast_status fuse(int n, std::vector<FusionGate> gates, const cast_fusion_opts &o,
                 std::vector<FusionGate> *out);

// Builds the matrix of a standard gate; returns false for unknown names.
bool standard_gate(const std::string &name, const double *params, int *k, std::vector<cplx> *m);
// exp(-i a G / 2) for a Pauli string G (letters in 2-bit fields, see cast.h).
std::vector<cplx> rotation_matrix(int k, int generator, double angle);
std::vector<cplx> pauli_string_matrix(int k, int generator);

}  // namespace cast

struct cast_sv {
    void *data = nullptr;
    int n = 0;
    cast_dtype dt = CAST_C128;
    hipStream_t stream = nullptr;
    bool owns = false;
};

namespace cast {
struct BlockedPlan;                  // cache-blocked grouping of a fused list (blocked.cpp)
void blocked_free(BlockedPlan *b);
struct JitModule;                    // generated kernels of a fused list (jit.cpp)
void jit_free(JitModule *j);
}  // namespace cast

struct cast_fused {
    int n = 0;
    std::vector<cast::PassPlan> plans;
    double fusion_ms = 0;
    // device copies of the block matrices, per dtype (lazily uploaded)
    cast::DeviceMatrix dev[3];
    std::vector<size_t> dev_off[3];
    // cache-blocked grouping, per dtype (built on first use)
    cast::BlockedPlan *blocked[3] = {nullptr, nullptr, nullptr};
    // generated kernels, per dtype (compiled on first use)
    cast::JitModule *jit[3] = {nullptr, nullptr, nullptr};
    // pass schedule of apply_circuit, per dtype (built on first use)
    cast::Schedule *sched[3] = {nullptr, nullptr, nullptr};
};
