/*
 * cast.h -- C ABI of the MI355X (gfx950) fused-gate state-vector engine.
 *
 * The engine applies sequences of k-qubit gates (k = 1..6, 2^k x 2^k complex
 * matrices) to a 2^n-amplitude state held in device memory, after an optional
 * host-side agglomerative gate-fusion pass (Sec. III, Alg. 1).  It also
 * evaluates Pauli-sum expectation values and adjoint-method gradients of
 * parametrised circuits, one circuit or a batch of them per call.
 *
 * Conventions used by every entry point
 * -------------------------------------
 *  - State layout (Sec. II-A, Eq. 1): amplitude x (0 <= x < 2^n) is stored at
 *    element x, qubit q is bit q of x (little-endian).  Amplitudes are
 *    interleaved complex numbers: (re, im) as two doubles for CAST_C128 or two
 *    floats for CAST_C64 -- the memory layout of torch.complex128 / complex64.
 *  - Gate matrices are always passed as host FP64: 2^k x 2^k, row-major,
 *    interleaved (re, im), so 2 * 4^k doubles.  Bit i of a row/column index
 *    belongs to qubits[i]; qubit lists need not be sorted.  A k-qubit gate
 *    acts on the 2^{n-k} groups of amplitudes that agree off its qubits
 *    (Eq. 3).  Matrices are not checked for unitarity.
 *  - Errors: every function returns cast_status (0 = CAST_OK, < 0 = error)
 *    and never aborts or throws.  cast_last_error() returns a thread-local
 *    message for the last failing call on the calling thread.  Arguments are
 *    validated before any device work is queued; a failing call leaves its
 *    outputs untouched unless stated otherwise.
 *  - Streams: every state carries a HIP stream (NULL = the default stream).
 *    Device work is queued on it in call order.  Calls marked "synchronous"
 *    wait for the stream before returning; the others only queue work.
 *  - Host arrays passed in are copied (or fully consumed) before the call
 *    returns; the caller may free them immediately.
 */
#ifndef CAST_H
#define CAST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int cast_status;
enum {
    CAST_OK = 0,
    CAST_EINVAL = -1,       /* bad argument: range, NULL, duplicate qubit, size mismatch */
    CAST_ENOMEM = -2,       /* device (or the CAST_MAX_DEVICE_BYTES cap) cannot hold it */
    CAST_EHIP = -3,         /* a HIP runtime call failed; message has hipGetErrorString */
    CAST_EUNSUPPORTED = -4, /* valid request with no kernel for it */
    CAST_ESTATE = -5        /* object in the wrong state (e.g. destroyed state) */
};

typedef enum { CAST_C64 = 1, CAST_C128 = 2 } cast_dtype;

typedef struct cast_sv cast_sv;       /* opaque state vector (owning or borrowing) */
typedef struct cast_fused cast_fused; /* opaque fused-gate list, ready to apply */

/* Thread-local message of the last failing call ("" if none). */
const char *cast_last_error(void);

/* expval and adjoint_grad take their device scratch (reduction partials,
 * work states, matrices) from a reuse pool instead of allocating and freeing
 * it on every call; a block returns to the pool once its call has finished
 * its device work, and at most 8 GiB stay pooled (counted against
 * CAST_MAX_DEVICE_BYTES).  pool_trim frees everything pooled.  Not to be
 * called while those calls run on other threads. */
void pool_trim(void);

/* ------------------------------------------------------------------ states */

/* Allocates a 2^n state of dtype `dt` (1 <= n <= 34) on the current HIP
 * device and sets it to |0...0>.  `hip_stream` (hipStream_t or NULL) is used
 * for all work on this state.  The caller owns *out and frees it with
 * sv_destroy.  CAST_ENOMEM if the allocation fails or exceeds the byte cap in
 * the environment variable CAST_MAX_DEVICE_BYTES. */
cast_status sv_create(int n, cast_dtype dt, void *hip_stream, cast_sv **out);

/* Wraps existing device memory (2^n amplitudes of dtype `dt`, 16-byte
 * aligned) without copying or taking ownership: the caller keeps the memory
 * alive until sv_destroy.  Contents are left as they are. */
cast_status sv_wrap(void *dev_ptr, int n, cast_dtype dt, void *hip_stream, cast_sv **out);

/* Frees an owning state (or forgets a wrapped one).  NULL-safe. */
void sv_destroy(cast_sv *sv);

/* Copies `bytes` (= 2^n * amplitude size) of interleaved amplitudes from host
 * memory into the state.  Synchronous. */
cast_status sv_copy_from_host(cast_sv *sv, const void *host, size_t bytes);

/* Copies the whole state to host memory (`bytes` = 2^n * amplitude size).
 * Synchronous. */
cast_status sv_copy_to_host(const cast_sv *sv, void *host, size_t bytes);

/* Sets the state to the basis state |index>.  Queued on the state's stream. */
cast_status sv_set_basis(cast_sv *sv, uint64_t index);

/* Device pointer, qubit count and dtype of a state (any output may be NULL). */
cast_status sv_info(const cast_sv *sv, void **dev_ptr, int *n, cast_dtype *dt);

/* ------------------------------------------------------------------ gates */

/* Applies one k-qubit gate (1 <= k <= 6; Eq. 3) in place: each group of 2^k
 * amplitudes that agree off `qubits` is multiplied by `matrix`.  The matrix is
 * analysed on the host (zero/one snapping, XOR-subspace block structure) and
 * copied to the device in the state's dtype; zero blocks are skipped and
 * identity blocks are neither read nor written.  Queued on the state's stream
 * (the staging buffer is kept alive by the library until the work is done). */
cast_status apply_gate(cast_sv *sv, const int *qubits, int k, const double *matrix);

/* Fills `out` (2 * 4^k doubles) with the matrix of a standard gate, in the
 * index convention above.  Names: id h x y z s t p u3 rx ry rz rxx ryy rzz cx
 * cz cp swap.  `params` holds the gate's angles (u3: theta, phi, lambda;
 * rotations, p, cp: one angle; R(a) = exp(-i a G / 2)).  *k receives the
 * arity.  CAST_EINVAL for an unknown name. */
cast_status gate_matrix(const char *name, const double *params, int *k, double *out);

/* A gate in a circuit.  Fixed gates carry `matrix` (host FP64, layout above)
 * and param_id = -1.  Parametrised rotations carry matrix = NULL, param_id
 * >= 0 and `generator`: the Pauli letter of qubit i in bits 2i..2i+1
 * (1 = X, 2 = Y, 3 = Z); the gate is exp(-i * param_coeff * theta[param_id] *
 * G / 2). */
typedef struct {
    int k;
    int qubits[6];
    const double *matrix;
    int param_id;
    double param_coeff;
    int generator;
} cast_gate;

/* Options of the host fusion pass (Sec. III; Table 2 "Gate fusion"). */
typedef struct {
    int k_max;            /* largest fused gate, 1..6 (1 = no fusion) */
    double opcount_cap;   /* reject fusions whose op count exceeds it (<= 0: none) */
    double zero_tol;      /* |x| <= zero_tol snaps a real scalar to 0 */
    double one_tol;       /* |x -+ 1| <= one_tol snaps a real scalar to +-1 */
    int agglomerative;    /* grow the size limit 2 .. k_max (else k_max at once) */
    int multi_traversal;  /* repeat each traversal until nothing fuses */
    int cost_model;       /* 0: size-only; 1: adaptive (tuned cost table) */
    int cost_dtype;       /* dtype whose cost table the adaptive check uses (0 = CAST_C128) */
} cast_fusion_opts;

/* Default options: k_max 5, no cap, tolerances 1e-14, agglomerative and
 * multi-traversal on, size-only, complex128 cost table. */
void fusion_opts_default(cast_fusion_opts *opts);

/* Fuses a circuit of fixed gates (param_id must be -1; parametrised gates are
 * bound first by the caller) on n qubits into a list of gates of at most
 * k_max qubits whose product equals the circuit's unitary (Alg. 1 with the
 * agglomerative schedule of Sec. III-B).  Matrix products are FP64.  The
 * result is analysed for the device but holds no device memory until it is
 * first applied.  The caller owns *out (fused_destroy). */
cast_status fuse_circuit(int n, const cast_gate *gates, size_t n_gates,
                         const cast_fusion_opts *opts, cast_fused **out);

/* Summary of a fused list: number of fused gates, sum of their op counts
 * (2 per nonzero real matrix scalar, Sec. III-C), and host fusion time. */
cast_status fused_info(const cast_fused *f, size_t *n_fused, double *total_opcount,
                       double *fusion_ms);

/* Details of fused gate i: its k, sorted qubits (6 ints), op count, the
 * dimension d of the XOR subspace spanned by its nonzero pattern and the
 * number of non-identity blocks.  `matrix` (NULL or 2 * 4^k doubles) receives
 * its FP64 matrix with bit i <-> sorted qubit i.  For tests and reports. */
cast_status fused_gate(const cast_fused *f, size_t i, int *k, int *qubits, double *opcount,
                       int *subspace_dim, int *active_blocks, double *matrix);

/* Applies every fused gate, in order, to the state: one device pass per
 * fused gate, except that a run of consecutive diagonal fused gates is applied
 * in one elementwise pass.  A product of diagonal gates is diagonal and costs
 * one complex multiply per amplitude whatever its size (its operation count,
 * Sec. III-C, does not grow), so the host multiplies the run, in FP64, into
 * at most "diag_run_tables" phase tables of at most "diag_run_qubits" qubits
 * each, and the pass multiplies each amplitude by the product of its entries
 * (knob diag_run_tables = 0: one pass per fused gate).  The schedule is built
 * for the state's dtype with the knobs current at first use and cached in the
 * list (rebuilt when those knobs change).  The state's n must equal the n
 * given to fuse_circuit.  Queued on the state's stream. */
cast_status apply_circuit(cast_sv *sv, const cast_fused *f);

/* Same as apply_circuit, but records a HIP event pair around every pass on
 * the state's stream and returns each pass's device time in pass_ms (one
 * float per pass of circuit_passes, milliseconds).  Synchronous.  For
 * measurement. */
cast_status apply_circuit_timed(cast_sv *sv, const cast_fused *f, float *pass_ms);

/* Number of device passes apply_circuit makes for a 2^n state of dtype dt
 * with the current knobs (host only; builds and caches the schedule). */
cast_status circuit_passes(const cast_fused *f, int n, cast_dtype dt, size_t *n_passes);

/* Pass i of that schedule: the fused gates [first, first + count) it applies,
 * its kernel (as fused_pass_info, plus 6 = diagonal run and -1 = identity),
 * the number of phase tables of a diagonal run (0 otherwise), and its
 * algorithmic HBM bytes and flops: for a diagonal run, every amplitude at
 * which some phase table differs from 1 read and written once and one
 * complex multiply (8 flops) each.  Any output may be NULL.  CAST_EINVAL for i out of
 * range. */
cast_status circuit_pass_info(const cast_fused *f, int n, cast_dtype dt, size_t i, size_t *first, size_t *count,
                              int *kernel, int *tables, double *alg_bytes, double *flops);

/* Launch shapes of the passes (kernels 0 to 6).  A direct pass (0) walks
 * its (group, block) work items in runs of 2^chunk_log groups of one block
 * and visits its 2^it_bits iterations in an order rotated left by rot bits
 * (rot 0: address order; needs a power-of-two iteration count, else 0).  The
 * others take only rot (chunk_log is ignored): an LDS-tile pass (1, 2, 5)
 * rotates the order of its tiles, an elementwise diagonal pass (3) that of
 * the tiles of each active pattern, a matrix-core direct pass (4) that of its
 * runs of four 16-group units, and a diagonal run (6; on more than 8 qubits
 * for complex128, 9 for complex64, with diag_run_reuse > 0) that of its
 * units of one 4 KiB span repeated over 2^diag_run_reuse free high bits; a
 * rotation at or above the order's bit count is ignored.  Which rate a shape reaches depends on how the gate's planes
 * fall onto the DRAM channels and banks, so no one knob value suits every
 * pass (the paper's cost model is likewise measured, Sec. III-C).  The shape is kept
 * per pass in the list's schedule for (n, dt); -1 means the knob's value
 * (direct_rot / direct_chunk_log).  Every shape computes each amplitude with
 * the same operations, so results are bitwise the same whatever the shape.
 * A schedule rebuilt after a change of diag_run_tables, diag_run_qubits or
 * use_diag starts from -1 again.
 *
 * circuit_pass_shape reads pass i's shape (outputs may be NULL);
 * circuit_set_pass_shape sets it (rot -1..16, chunk_log -1 or 6..16; a
 * chunk_log above n - k acts as n - k), CAST_EINVAL for i out of range. */
cast_status circuit_pass_shape(const cast_fused *f, int n, cast_dtype dt, size_t i, int *rot, int *chunk_log);
cast_status circuit_set_pass_shape(cast_fused *f, int n, cast_dtype dt, size_t i, int rot, int chunk_log);

/* Chooses each shaped pass's launch shape by measurement on sv's device:
 * for a direct pass the knobs' shape, run lengths 2^8, 2^10 and 2^12 groups,
 * then rotations 2, 4 and 6 at the best run length; for the other shaped
 * kinds the knobs' shape and rotations 2, 4, 6 and 8; each
 * launched reps times (1..100; the minimum counts); a shape other than the
 * knobs' is kept only when it is more than 1 % faster.  The passes are applied to sv in place,
 * so its amplitudes change (they stay normalised: every pass is unitary).
 * *before_ms and *after_ms (may be NULL) receive the summed minimum times of
 * the tuned passes with the knobs' shapes and with the chosen ones.
 * Synchronous.  The shapes live in the list: do not tune a list while
 * another thread applies it (the same holds for circuit_set_pass_shape). */
cast_status circuit_tune(cast_sv *sv, cast_fused *f, int reps, double *before_ms, double *after_ms);

/* How fused gate i runs on a 2^n state of dtype dt: *kernel = 0 (direct
 * gather), 1 (LDS tile), 2 (LDS tile, two buffers), 3 (elementwise diagonal),
 * 4 (matrix-core direct gather), 5 (matrix-core LDS tile) or -1 (identity,
 * skipped), *d the block dimension,
 * and the pass's algorithmic HBM bytes (every amplitude of a non-identity
 * block read once and written once) and flops (8 per complex multiply-add
 * over the non-identity blocks). */
cast_status fused_pass_info(const cast_fused *f, size_t i, int n, cast_dtype dt, int *kernel, int *d,
                            double *alg_bytes, double *flops);

/* Streaming reference for the rooflines: multiplies `bytes` of device memory
 * (16-byte aligned, a multiple of 16, read as doubles) in place by `factor`,
 * each of 256 lanes per workgroup moving chunks_per_lane (1, 2, 4 or 8)
 * 16-byte chunks per tile with non-temporal loads and stores, on at most
 * `grid` workgroups (0: one per tile).  Every byte is read and written once
 * and no gate work is done, so its rate is the practical ceiling of the
 * elementwise gate kernels.  Queued on hip_stream (hipStream_t or NULL).
 * For measurement. */
cast_status stream_scale(void *data, size_t bytes, double factor, int chunks_per_lane, int grid, void *hip_stream);

/* ------------------------------------------------------------ cache-blocked passes */

/* Applies a fused list with several fused gates per HBM pass (cache
 * blocking).  Consecutive fused gates are grouped into segments: a segment
 * has a tile qubit set T = [0, w) plus up to tile_bits - w higher qubits
 * (w >= 4), every non-diagonal gate of the segment mixes only amplitudes that
 * differ on T (the qubits its non-identity blocks span; its other targets may
 * lie anywhere), and diagonal gates join any segment.  One workgroup loads
 * the 2^tile_bits amplitudes that agree off T into LDS, applies the segment's
 * gates in order and writes them back, so a segment costs one read and one
 * write of the state.  Gates with blocks larger than 8 x 8 (d >= 4) and
 * segments of one gate run as the ordinary passes of apply_circuit.  The
 * result equals apply_circuit's up to rounding.  The grouping is built on
 * first use for the state's dtype with the "blocked_tile_bits" knob
 * (log2 amplitudes per tile; 2^tile_bits amplitudes must fit 128 KiB) and
 * cached in the fused list; device memory for it is owned by the list.
 * Queued on the state's stream; not thread-safe on one fused list. */
cast_status apply_circuit_blocked(cast_sv *sv, const cast_fused *f);

/* Same, with a HIP event pair around every HBM pass; pass_ms receives one
 * float (ms) per pass (blocked_info's count).  Synchronous.  For measurement. */
cast_status apply_circuit_blocked_timed(cast_sv *sv, const cast_fused *f, float *pass_ms);

/* Number of HBM passes of the grouping for a 2^n state of dtype dt (builds
 * and caches the grouping, uploading the list's matrices if needed). */
cast_status blocked_info(const cast_fused *f, int n, cast_dtype dt, size_t *n_passes);

/* Pass i of that grouping: the fused gates [first, first + count) it covers,
 * and for a segment its tile_bits, window w and high tile qubits
 * (high_qubits: NULL or 10 ints, -1 past the last); tile_bits = window = 0
 * for an ordinary one-gate pass.  CAST_EINVAL for i out of range. */
cast_status blocked_pass_info(const cast_fused *f, int n, cast_dtype dt, size_t i, size_t *first, size_t *count,
                              int *tile_bits, int *window, int *high_qubits);

/* ------------------------------------------------------------ dynamic kernels */

/* Generated kernels (the paper's run-time generated, gate-specific kernels,
 * Sec. IV-A): one kernel per fused gate with block dimension d <= 4, written
 * from the gate's matrix cast to dt with every entry an immediate constant,
 * exact zeros dropped entry by entry, entries +-1 and +-i turned into
 * additions, and amplitudes that share a coefficient (up to sign) within an
 * output row summed before one multiplication; target masks and block
 * offsets are constants too.  All kernels of the list are compiled for
 * gfx950 with hipRTC in one program, on the host, and cached in the fused
 * list.  jit_compile compiles (no device needed) and reports the kernel
 * count and compile time (ms). */
cast_status jit_compile(const cast_fused *f, cast_dtype dt, int *n_kernels, double *compile_ms);

/* Applies the fused list with the generated kernels (compiling them first if
 * needed and loading them on the device at first use); gates with d > 4 run
 * with the library's kernels.  Same result as apply_circuit up to rounding.
 * Queued on the state's stream. */
cast_status apply_circuit_jit(cast_sv *sv, const cast_fused *f);

/* Same, with a HIP event pair around every pass (n_fused floats, ms).
 * Synchronous.  For measurement. */
cast_status apply_circuit_jit_timed(cast_sv *sv, const cast_fused *f, float *pass_ms);

/* Frees a fused list.  NULL-safe.  The caller must not destroy a list while
 * work that uses it is still queued (synchronise the stream first). */
void fused_destroy(cast_fused *f);

/* ------------------------------------------------------------ tuning */

/* Launch knobs of the pass kernels, per dtype (dt = CAST_C64 or CAST_C128).  Keys: "direct_min_q" (smallest
 * target for the direct gather), "tile_bits" (log2 amplitudes per LDS tile),
 * "direct_ipt" (work items per thread: 1, 2 or 4), "direct_nt" (non-temporal
 * hints 0/1), "direct_chunk_log" (direct kernel on a gate with several blocks:
 * log2 of the consecutive groups one block runs over before the next block
 * takes the same groups, 6..16), "max_grid" (workgroup cap), "use_diag" (elementwise diagonal
 * kernel 0/1), "mfma_min_d" (smallest block dimension for the matrix cores,
 * 4..7; 7 disables them), "mfma_grid_per_cu", "mfma_direct_min_q",
 * "diag_unroll" (diagonal kernel chunks per thread: 1, 2, 4, 8),
 * "diag_max_grid", "diag_lds_table" (phases in LDS 1 / read from L1 0),
 * "diag_order" (active tiles of the diagonal kernel visited pattern-fastest 0 /
 * pattern-major 1), "blocked_tile_bits" (log2 amplitudes per tile of the
 * cache-blocked passes, 8..12 for complex128, 8..13 for complex64: tiles of
 * at most 64 KiB, so two workgroups share a compute unit's LDS),
 * "blocked_threads" (their workgroup size: 256, 512 or 1024),
 * "mfma_3m_min_d" (matrix-core passes with blocks of d >= this value form
 * complex products with three real products instead of four; 4..7, 7 = never),
 * "mfma_low_tile" (1: a matrix-core pass with d <= 4 and a target below bit 4
 * runs on the LDS tile when at most one target lies above the tile's
 * contiguous window or the gate has several blocks; 0: the direct gather),
 * "diag_run_tables" (tables per diagonal-run pass, 0..4; 0 = no runs),
 * "diag_run_qubits" (qubits per diagonal-run table, 4..8), "diag_run_unroll"
 * (its chunks per thread: 1, 2, 4), "diag_run_grid" (its workgroup cap),
 * "persistent_spin_limit" (polls a persistent batch item makes before its
 * dependency wait gives up and the run fails with CAST_EHIP; read by
 * batch_create; 0 makes every item that has a dependency fail at once, which
 * exercises that error path from the host).
 * CAST_EINVAL for an unknown key or an out-of-range value.  Not thread-safe
 * against concurrent launches: set knobs before queuing work. */
cast_status tuning_set(const char *key, cast_dtype dt, int value);
cast_status tuning_get(const char *key, cast_dtype dt, int *value);

/* Predicted time of one pass of a k-qubit gate with block dimension d over
 * 2^n amplitudes, in milliseconds per 2^30 amplitudes, used by the adaptive
 * fusibility check (cost_model = 1): a fusion is accepted only if the fused
 * pass is predicted no slower than the two passes it replaces (Sec. III-C).
 * Entries start at an HBM-bound estimate and are replaced by the autotuner's
 * measurements. */
cast_status cost_table_set(cast_dtype dt, int k, int d, double ms_per_gamp);
cast_status cost_table_get(cast_dtype dt, int k, int d, double *ms_per_gamp);

/* ------------------------------------------------------------ path planner */

/* Measured rates the planner prices passes with, per dtype (Sec. III-C's
 * idea of a cost model measured on the target, applied to whole plans).
 * Keys: "bw0".."bw6" (GB/s of algorithmic bytes of a pass whose schedule
 * kernel kind, as circuit_pass_info reports it, is 0..6), "fl4".."fl6"
 * (GFLOP/s of the matrix-core passes by block dimension), "fl_vec" (GFLOP/s
 * of the other kernels), "launch_ms" (fixed cost of one pass), "seg_bw"
 * (GB/s of a cache-blocked segment's read and write of the state),
 * "seg_gate0".."seg_gate3" (ms per 2^30 amplitudes per fused gate applied
 * inside a segment, by block dimension; 0 = diagonal).  Values must be
 * positive and finite.  Not thread-safe against concurrent planning. */
cast_status path_cost_set(const char *key, cast_dtype dt, double value);
cast_status path_cost_get(const char *key, cast_dtype dt, double *value);

/* Predicted device time (ms) of applying f to a 2^n state of dtype dt with
 * apply_circuit (path 0: a launch plus max(algorithmic bytes / rate, flops /
 * rate) per pass) or apply_circuit_blocked (path 1: ordinary passes the same
 * way, a segment one read and write of the state plus its gates' in-tile
 * costs).  Host only. */
cast_status predict_ms(const cast_fused *f, int n, cast_dtype dt, int path, double *ms);

/* Fuses the circuit (fixed gates, as fuse_circuit) at every size limit
 * k_lo..k_hi, the other fusion options from opts (NULL: defaults), prices
 * each fused list on both paths with predict_ms, and returns the cheapest
 * pair: *out (caller owns; fused_destroy), *path (0: apply_circuit, 1:
 * apply_circuit_blocked), *k_max and, if not NULL, *predicted (ms).  Ties go
 * to the smaller k_max and to path 0.  Host only. */
cast_status plan_circuit(int n, const cast_gate *gates, size_t n_gates, cast_dtype dt, const cast_fusion_opts *opts,
                         int k_lo, int k_hi, cast_fused **out, int *path, int *k_max, double *predicted);

/* ------------------------------------------------------------ observables */

/* A Pauli term coeff * P with P = i^{|x & z|} X^x Z^z: bit q of xmask/zmask
 * gives qubit q's letter (x,z) = (1,0) X, (1,1) Y, (0,1) Z. */
typedef struct {
    double coeff;
    uint64_t xmask;
    uint64_t zmask;
} cast_pauli_term;

/* out[0] = sum_m coeff_m <psi|P_m|psi> (real part) and out[1] its imaginary
 * part (round-off for Hermitian sums), accumulated in FP64 for both dtypes
 * with a fixed reduction order.  Synchronous. */
cast_status expval(const cast_sv *sv, const cast_pauli_term *terms, size_t n_terms, double *out);

/* Most terms expval_noalloc takes. */
#define CAST_EXPVAL_NOALLOC_MAX_TERMS 4096

/* expval for callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result, bit for bit, from the same kernels, with the device scratch
 * (reduction partials and per-term results, 192 KiB) in a fixed array that
 * each GPU holds from the first call until the process ends.  Calls no
 * hipMalloc/hipFree; on success it allocates no host memory either (fixed
 * arrays on the stack).  n_terms above
 * CAST_EXPVAL_NOALLOC_MAX_TERMS is CAST_EINVAL.  The state must be on the
 * current HIP device.  All calls on one GPU share its array, so calls that
 * overlap on one GPU (other threads, or work queued on other streams) race;
 * the call is synchronous, so consecutive calls from one thread do not.
 * Synchronous. */
cast_status expval_noalloc(const cast_sv *sv, const cast_pauli_term *terms, size_t n_terms, double *out);

/* ------------------------------------------------------------ gradients */

/* Energy and adjoint-method gradient (Jones & Gacon 2020) of
 * E(theta) = <psi(theta)|H|psi(theta)>, psi(theta) = U_L ... U_1 |init>.
 * `init` is copied, not modified; the work uses the init state's dtype and
 * stream.  grad has n_params entries.  Synchronous. */
cast_status adjoint_grad(const cast_sv *init, const cast_gate *gates, size_t n_gates,
                         const double *theta, size_t n_params,
                         const cast_pauli_term *terms, size_t n_terms,
                         double *energy, double *grad);

/* ------------------------------------------------------ batched gradients */

/* Many parametrised circuits evaluated together on one GPU: the same
 * structure with different parameter sets (variational algorithms run the
 * same circuit thousands of times), or circuits of different qubit counts.
 * Each instance i has n_qubits[i] qubits (3..34), its own gate list
 * (1- and 2-qubit gates; parametrised gates as in cast_gate), n_params[i]
 * parameters and Pauli sum H_i, and starts from init_kind[i]:
 * CAST_INIT_ZERO |0...0>, CAST_INIT_PLUS |+...+>, or CAST_INIT_STATE a copy
 * of init_states[i] (a state of the same n and dtype that must stay alive
 * while the batch is used).  init_kind may be NULL (all |0...0>).
 *
 * Every instance runs: forward gates, lambda = H psi, energy <psi|lambda>,
 * and the reverse adjoint sweep; op s of every instance forms global step s.
 * mode CAST_BATCH_STEPS queues one launch per global step;
 * CAST_BATCH_STEPS_GRAPH captures those launches once in a hipGraph and
 * replays it; CAST_BATCH_PERSISTENT_GRAPH captures one persistent launch in
 * which workgroups take (step, instance, slice) items in order from a device
 * counter, each waiting (bounded) until its instance has finished the
 * previous op.  Results are identical in all modes (fixed reduction order).
 * The batch owns device states (psi and lambda per instance), a pinned
 * matrix buffer and its own stream; the caller owns *out (batch_destroy). */
enum { CAST_INIT_ZERO = 0, CAST_INIT_PLUS = 1, CAST_INIT_STATE = 2 };
enum { CAST_BATCH_STEPS = 0, CAST_BATCH_STEPS_GRAPH = 1, CAST_BATCH_PERSISTENT_GRAPH = 2 };

typedef struct cast_batch cast_batch;

cast_status batch_create(int n_inst, const int *n_qubits, cast_dtype dt, const cast_gate *const *circuits,
                         const size_t *n_gates, const size_t *n_params, const cast_pauli_term *const *hamiltonians,
                         const size_t *n_terms, const int *init_kind, const cast_sv *const *init_states, int mode,
                         cast_batch **out);

/* Binds theta[i] (n_params[i] doubles per instance; may be NULL for
 * instances without parameters), runs the whole batch and writes energies[i]
 * and grads[i][p] = dE_i/dtheta_i[p] (FP64).  Synchronous.  CAST_EHIP if a
 * persistent-mode dependency wait exceeded its bound (results invalid). */
cast_status batch_run(cast_batch *b, const double *const *theta, double *energies, double *const *grads);

/* Global steps, total work items of the persistent launch, and bytes of the
 * batch's device states (psi and lambda of every instance). */
cast_status batch_info(const cast_batch *b, int *n_steps, uint64_t *total_items, double *state_bytes);

/* Algorithmic HBM bytes of one batch_run as planned: every instance's
 * initial state written once (2^n amplitudes), each forward segment reading
 * and writing psi, the lambda = H psi op reading psi and writing lambda, and
 * each reverse segment reading and writing both psi and lambda.  Matrices,
 * partial sums and results are not counted.  *state_passes receives the
 * number of whole-state read+write passes those ops make (reverse segments
 * count two).  Either output may be NULL. */
cast_status batch_traffic(const cast_batch *b, double *alg_bytes, uint64_t *state_passes);

/* The segments batch_create cuts one instance's gate list into (host only,
 * no device work): gates whose qubits together fit one LDS tile of 2^tb
 * amplitudes (tb = min(n, batch_tile_bits), the tuning knob, 11 by default)
 * with at most tb - w of them at or above bit w (w = batch_min_window, 2 for
 * CAST_C128 and 3 for CAST_C64 by default, at most tb - 2), so that every
 * tile is read in runs of at least 2^w consecutive amplitudes, at
 * most 64 gates each, forward (reverse = 0) or for the reverse adjoint sweep
 * (reverse = 1).  Segments may take gates out of circuit order: two gates
 * that share a qubit keep their relative order unless both are diagonal;
 * gates on disjoint qubits commute (CAST_BATCH_REORDER=0 in the environment
 * keeps the circuit order).  *n_segments receives the count; if not NULL,
 * order[i] (n_gates entries) receives the i-th gate applied and
 * segment_of[i] its segment.  Gates are validated as in batch_create. */
cast_status batch_segments(int n, const cast_gate *gates, size_t n_gates, cast_dtype dt, int reverse,
                           size_t *n_segments, int *order, int *segment_of);

void batch_destroy(cast_batch *b);

/* batch_create + batch_run + batch_destroy in one call. */
cast_status adjoint_grad_batch(int n_inst, const int *n_qubits, cast_dtype dt, const cast_gate *const *circuits,
                               const size_t *n_gates, const double *const *theta, const size_t *n_params,
                               const cast_pauli_term *const *hamiltonians, const size_t *n_terms,
                               const int *init_kind, const cast_sv *const *init_states, int mode,
                               double *energies, double *const *grads);

#ifdef __cplusplus
}
#endif
#endif /* CAST_H */
