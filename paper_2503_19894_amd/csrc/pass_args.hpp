// Kernel argument block of one gate pass (passed by value).
#pragma once
#include <cstdint>

namespace cast {

struct PassArgs {
    uint64_t off[6];        // amplitude offset of each virtual basis vector
    uint64_t lowmask[6];    // direct: (1 << q_i) - 1 for the sorted targets
    uint64_t hilowmask[6];  // tile: (1 << qhi_j) - 1 for the high targets
    uint64_t ngroups;       // direct: 2^(n-k)
    uint64_t ntiles;        // tile: 2^(n-tb)
    uint32_t tlowmask[6];   // tile: (1 << q_i) - 1 for the low targets
    uint32_t toff[6];       // tile position of each virtual basis vector
    uint32_t blk[64];       // active block ids
    uint32_t nblk;
    int k;
    int chunk_log;          // direct: log2(items per block run), 6 <= chunk_log <= n - k
    int tb;                 // tile: log2(amplitudes per tile)
    int W;                  // tile: contiguous window bits
    int khi, klo;           // tile: targets at/above and below W
    int qhi[6];             // tile: high targets, ascending
    int rot, it_bits;       // direct (iterations) and matrix-core direct (four-unit runs): order rotated left by rot bits of it_bits (rot 0: in order)
};

// Kernel argument block of a diagonal pass (every block 1 x 1).
struct DiagArgs {
    uint64_t amask;         // bit j set: local index j has a phase != 1
    uint64_t nchunks;       // 16-byte chunks in the state
    int k;
    int q[6];               // sorted targets
    // Tiles of 256 * U chunks; only tiles whose high-target bits (targets at
    // or above the tile size on which the activity depends) form an active
    // pattern are visited.  Tile number a splits into a pattern and the other
    // tile bits, which are deposited around those targets: pattern-fastest
    // order (a mod npat, a / npat) keeps tiles of every pattern in flight at
    // once, pattern-major order (a >> rest_bits, a & (2^rest_bits - 1)) walks
    // one pattern's tiles in address order.  ntiles = 0: the state is smaller
    // than one tile and is walked chunk by chunk.
    uint64_t ntiles;        // active tiles = npat << rest_bits
    uint64_t hlowmask[6];   // per selecting target (ascending): bits of the tile index below it
    int kh;                 // selecting targets
    int rest_bits;
    int pattern_major;
    int spread;             // tile number -> XCD by the XOR of its 3-bit digits (else round-robin)
    int rot;                // the other tile bits rotated left by rot of rest_bits (0: in order)
    uint32_t npat;          // active patterns
    uint32_t patoff[64];    // tile-index bits of each active pattern
};

}  // namespace cast
