// Batched adjoint-gradient programs: many parametrised circuits (same or
// different qubit counts) evaluated together on one GPU.
//
// Each instance's program is a list of ops, op s of every instance forming
// global step s:
//   FWD  a segment of consecutive gates applied to psi
//   HPSI lambda <- H psi, partial sums of <psi|lambda>  (energy)
//   ADJ  a segment of gates in reverse order: for each, partial sums of
//        <lambda|G|psi>, then psi <- U^dag psi, lambda <- U^dag lambda
// A segment holds consecutive gates whose qubits together fit one LDS tile
// (the low window [0, W) plus the segment's qubits at or above W): a work
// item loads one tile of psi (and lambda), applies every gate of the segment
// in LDS in order, and writes the tile back, so one HBM pass serves many
// gates.  Every op of an instance has `wgs` items (tiles); partial sums of
// item w land in a fixed slot, and a final kernel adds them in a fixed order.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "reduce.hpp"

namespace cast {

enum BatchKind : uint32_t { BK_FWD = 0, BK_HPSI = 1, BK_ADJ = 2 };

constexpr int kSegMaxGates = 64;   // gates per segment (bounds the LDS reduction area)
// LDS of a segment item beyond its two tiles: address tables + partial sums
constexpr size_t kSegLdsExtra = 128 * sizeof(uint64_t) + (size_t)kSegMaxGates * 4 * 2 * sizeof(double);

struct SegGate {            // one gate of a sweep, in sweep coordinates
    // packed: bit 0 k - 1; bits 1-2 t0 and 3-4 t1, the sweep bits (0..2) of
    // the sorted targets (t1 unused for k = 1); bits 5-7 the matrix form for
    // every parameter value (BatchForm); bits 8-10 xl and 11-13 zl, the x / z
    // masks over the sweep bits of the generator (ADJ inner products) or of
    // a BF_PAULI gate's Pauli string; bit 14 set when the gate has a result
    // slot; bits 15-18 (BF_SIGN) the local indices whose diagonal entry is -1
    uint32_t info;
    uint32_t mat;           // offset (complex entries) of U (FWD) or U^dag (ADJ): its 2^k x 2^k
                            // entries, or for a two-qubit diagonal form its diagonal first
    int slot;               // ADJ: result slot, or -1
    int pad;
};
inline uint32_t seg_info(int k, int t0, int t1, int form, uint32_t xl, uint32_t zl, bool param, uint32_t neg) {
    return (uint32_t)(k - 1) | (uint32_t)t0 << 1 | (uint32_t)(t1 < 0 ? 0 : t1) << 3 | (uint32_t)form << 5 |
           xl << 8 | zl << 11 | (uint32_t)param << 14 | (neg & 15u) << 15;
}

// Matrix forms the register sweeps specialise (fewer multiplies): diagonal
// (e.g. RZ, RZZ, CZ) and real (e.g. RY).
// A fixed diagonal gate whose entries are all +1 or -1 (e.g. CZ) is a sign
// pattern: BF_SIGN, its -1 entries in info bits 14-17, no matrix read.
// A two-qubit gate a I + b' P with P one Pauli string that flips bits (e.g.
// RXX, RYY, or a fixed XX coupling) is BF_PAULI: y_r = a x_r + b s(r) x_{r^xm}
// with s(r) = (-1)^{popc(zm & (r ^ xm))}, the masks in the record's xl / zl
// fields and (a, b) the first two complex entries of its matrix slot.
enum BatchForm : int { BF_GENERAL = 0, BF_DIAG = 1, BF_REAL = 2, BF_SIGN = 3, BF_PAULI = 4 };

struct SegSweep {           // consecutive gates of a segment on at most three tile bits
    int b[3];               // the sweep's tile bits, ascending
    uint32_t g0, g1;        // its gates [g0, g1) of the SegGate table
    int p0;                 // index of its first inner product within the segment
};

struct BatchRec {           // op `s` of one instance
    uint32_t kind;
    uint32_t inst;
    uint32_t item0;         // first item of this record within its step
    uint32_t wgs;           // items (workgroups) of this record
    int slot;               // HPSI result slot
    uint32_t sg0, sg1;      // FWD/ADJ: gates [sg0, sg1) of the SegGate table
    uint32_t sw0, sw1;      // FWD/ADJ: sweeps [sw0, sw1) of the SegSweep table
    int tb, W, khi;         // tile: 2^tb amplitudes, window [0, W), khi high qubits
    uint8_t qhi[12];        // high qubits of the tile, ascending
    uint64_t need;          // persistent mode: items of this instance that must be done first
};

struct BatchInst {
    void *psi;
    void *lam;
    int n;
    int nslots;
    uint32_t wgs;
    uint32_t ngroups;       // Pauli-term groups of H
    uint64_t part_off;      // doubles: partial sums, nslots x wgs x 2
    uint64_t res_off;       // doubles: results, nslots x 2
    uint32_t tg_off;        // first PauliSumGroup of H
    uint32_t tt_off;        // first PauliSumTerm of H (groups' `first` are relative to it)
    int init_kind;          // 0 |0...0>, 1 |+...+>, 2 copy of init_src
    int pad;
    const void *init_src;
};

struct BatchDev {           // device pointers of one program
    const BatchRec *recs;   // all records, step-major
    const SegGate *segs;
    const SegSweep *sweeps;
    const uint64_t *step_rec;    // nsteps + 1: first record of each step
    const uint64_t *step_item;   // nsteps + 1: first global item of each step (persistent mode)
    const BatchInst *insts;
    const void *mats;
    const PauliSumGroup *tg;
    const PauliSumTerm *tt;
    double *partials;
    double *results;
    int nsteps;
    int ninst;
};

// Queues step s (one launch over all its records).
cast_status batch_launch_step(const BatchDev &d, cast_dtype dt, int s, uint64_t nitems, size_t lds,
                              hipStream_t st);
// Queues the whole program as one persistent launch: workgroups pull items
// in global order from a counter; an item waits until its instance has
// finished the previous op.  Waits are bounded by spin_limit polls; on
// overrun *err becomes nonzero and every workgroup exits.
cast_status batch_launch_persistent(const BatchDev &d, cast_dtype dt, uint64_t total_items, int grid,
                                    unsigned long long *counters, uint32_t spin_limit, uint32_t chunk, size_t lds,
                                    hipStream_t st);
// Zeroes `n` 64-bit counters with a kernel (graph-capture safe).
cast_status batch_zero(unsigned long long *p, size_t n, hipStream_t st);
// Sets every instance's psi to its initial state (BatchInst::init_kind).
cast_status batch_init_states(const BatchDev &d, cast_dtype dt, hipStream_t st);
// Adds each instance's partial sums into results (fixed order).
cast_status batch_finish(const BatchDev &d, hipStream_t st);

}  // namespace cast
