// Cache-blocked execution of a fused gate list: several fused gates per HBM
// pass.
//
// Consecutive fused gates are grouped into segments.  A segment has a tile
// qubit set T = [0, w) + H (w >= 4 low "window" qubits and up to tb - w higher
// qubits H, |T| = tb); every non-diagonal gate of the segment mixes only
// amplitudes that differ on T (its block span, the qubits touched by its first
// d virtual basis vectors, lies in T).  A tile is the 2^tb amplitudes that
// agree off T: 2^|H| contiguous runs of 2^w amplitudes.  One workgroup loads a
// tile into LDS, applies the segment's gates in order (block gates by coset of
// their span, diagonal gates elementwise, with the targets outside T read off
// the tile's base index), and writes it back, so a segment costs one read and
// one write of the state however many gates it holds.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cast {

constexpr int kBlkMaxHigh = 10;    // tile qubits above the window
constexpr int kBlkMaxD = 3;        // largest block dimension applied inside a tile
constexpr int kBlkMinWindow = 4;   // smallest window: runs of >= 16 amplitudes

struct BlkGate {             // one fused gate inside a tile
    int kind;                // 0 diagonal (d = 0), 1 blocks of 2^d x 2^d
    int k, d;
    int q[6];                // sorted targets
    int tpos[6];             // tile bit of each target, -1 when the target is outside the tile
    uint32_t colv[6];        // virtual coordinates of local index bit s (the columns of L^-1)
    uint32_t span[kBlkMaxD]; // tile offset of virtual basis vector i < d
    uint32_t pivlow[kBlkMaxD];   // coset enumeration: (1 << pivot) - 1 per pivot bit, ascending
    int8_t slot[32];         // block id -> index among the active blocks, -1: identity block
    uint64_t amask;          // diagonal: local indices whose phase is not 1
    uint64_t mat;            // offset (reals) of the gate's matrices in the fused list's buffer
    uint32_t mat_reals;      // their size: 2 * 2^k (diagonal) or 2 * blocks * 4^d
    int run;                 // diagonal: gates applied together from here (a run), 0 inside a run
    int tshift;              // first gate of a run: log2 of its phase-table stride (entries)
    int pad;
};

// LDS of a segment pass: the tile, then two gate areas (the gate or run of
// diagonal gates being applied and the next one, staged meanwhile).  An area
// holds the slot table (32 bytes); the iteration table (per loop iteration
// of the workgroup, the wave-uniform part of the virtual coordinates and of
// the LDS address; at most 32 iterations); for a run of diagonal gates the
// uniform part of each gate's local index per iteration; then the matrices,
// or the run's phase tables at a stride of 2^tshift entries.  The planner
// keeps tile + two areas within kBlkLdsBudget, so two workgroups share a
// compute unit's 160 KiB of LDS.
constexpr uint32_t kBlkIterOff = 64;
constexpr uint32_t kBlkMaxIters = 32;
constexpr uint32_t kBlkRunMax = 8;
constexpr uint32_t kBlkJOff = kBlkIterOff + kBlkMaxIters * 8;
constexpr uint32_t kBlkAreaHead = kBlkJOff + kBlkRunMax * kBlkMaxIters * 4;
constexpr uint32_t kBlkMaxMatChunks = 512;    // 16-byte chunks of one gate's matrices (<= 2 per thread)
constexpr uint32_t kBlkLdsBudget = 80u << 10;

struct BlkSeg {              // kernel arguments of one segment pass
    uint64_t ntiles;         // 2^(n - tb)
    uint64_t hlowmask[kBlkMaxHigh];  // per high tile qubit (ascending): global index bits below it
    int tb, w, nh;
    int qh[kBlkMaxHigh];     // high tile qubits, ascending
    uint32_t g0, g1;         // gates [g0, g1) of the gate table
    uint32_t area;           // bytes of one gate area (head + the largest matrices of the segment)
    int maxd;                // largest block dimension among the segment's gates (selects the kernel)
};

}  // namespace cast
