// Host gate fusion on the CircuitTile structure (Sec. III-A, III-B, Alg. 1).
//
// The tile is a sequence of rows, each an array with one cell per qubit that
// is empty or names the block occupying that qubit at that time step; rows
// are time-ordered and the blocks of one row act on disjoint qubits.  A new
// gate becomes a one-gate block in the uppermost row that keeps it after
// every earlier block on its qubits.  A traversal walks rows top to bottom:
//  * a block whose cells in the next row are all empty moves down one row
//    (no fusion; it may fuse with the block below when the walk reaches it);
//  * otherwise it is fused with the block right below it on each of its
//    qubits when the pair is fusible (consecutive fusion);
//  * neighbouring cells of one row holding different blocks are fused when
//    fusible (commuting fusion).
// A fused block replaces the pair in the lower row if its cells there are
// free, else in the upper row, else in a new row inserted between the two.
// After each traversal the tile is compacted.  The agglomerative schedule
// raises the size limit from 2 to k_max, repeating each traversal until it
// fuses nothing (multi-traversal).  Fused matrices are FP64 products.
#include <algorithm>
#include <cmath>

#include "internal.hpp"

namespace cast {
namespace {

struct Block {
    std::vector<int> qubits;  // sorted
    std::vector<cplx> m;      // bit i <-> qubits[i]
    double opcount = 0;
};

// Matrix of `b` on the sorted qubit set `U` (a superset of b.qubits).
std::vector<cplx> embed(const Block &b, const std::vector<int> &U) {
    const int ku = (int)U.size(), kb = (int)b.qubits.size();
    const int D = 1 << ku, Db = 1 << kb;
    int posb[kMaxK];
    uint32_t qmask = 0;
    for (int i = 0; i < kb; ++i) {
        posb[i] = (int)(std::find(U.begin(), U.end(), b.qubits[i]) - U.begin());
        qmask |= 1u << posb[i];
    }
    auto extract = [&](uint32_t x) {
        uint32_t o = 0;
        for (int i = 0; i < kb; ++i) o |= ((x >> posb[i]) & 1u) << i;
        return o;
    };
    std::vector<cplx> e((size_t)D * D, cplx(0, 0));
    for (uint32_t r = 0; r < (uint32_t)D; ++r)
        for (uint32_t c = 0; c < (uint32_t)D; ++c)
            if ((r & ~qmask) == (c & ~qmask)) e[(size_t)r * D + c] = b.m[(size_t)extract(r) * Db + extract(c)];
    return e;
}

// Block for "first a, then b" (a and b may commute; the product is b * a).
Block product(const Block &a, const Block &b) {
    Block f;
    f.qubits = a.qubits;
    f.qubits.insert(f.qubits.end(), b.qubits.begin(), b.qubits.end());
    std::sort(f.qubits.begin(), f.qubits.end());
    f.qubits.erase(std::unique(f.qubits.begin(), f.qubits.end()), f.qubits.end());
    const int D = 1 << f.qubits.size();
    std::vector<cplx> ea = embed(a, f.qubits), eb = embed(b, f.qubits);
    f.m.assign((size_t)D * D, cplx(0, 0));
    for (int r = 0; r < D; ++r)
        for (int t = 0; t < D; ++t) {
            const cplx x = eb[(size_t)r * D + t];
            if (x == cplx(0, 0)) continue;
            for (int c = 0; c < D; ++c) f.m[(size_t)r * D + c] += x * ea[(size_t)t * D + c];
        }
    return f;
}

class Tile {
  public:
    Tile(int n, const cast_fusion_opts &o) : n_(n), o_(o) {}

    void append(Block b) {
        int r = 0;
        for (int q : b.qubits) r = std::max(r, last_[q] + 1);
        const int id = (int)blocks_.size();
        b.opcount = snapped_opcount(b.m);
        blocks_.push_back(std::move(b));
        alive_.push_back(true);
        if (r == (int)rows_.size()) rows_.emplace_back(n_, -1);
        for (int q : blocks_[id].qubits) rows_[r][q] = id, last_[q] = r;
    }

    void init_last() { last_.assign(n_, -1); }

    // One traversal of the tile (Sec. III-B, Alg. 1): rows top to bottom;
    // in each row every occupied cell first lets its block settle (sink into
    // free space or take in the block under that cell), then blocks standing
    // side by side in the row are merged.  Returns whether anything fused.
    bool traverse(int k) {
        bool fused = false;
        for (size_t r = 0; r < rows_.size(); ++r) {
            // rows are only ever inserted below r, so a last row stays last
            if (r + 1 < rows_.size())
                for (int q = 0; q < n_; ++q) fused |= settle_cell(r, q, k);
            fused |= merge_neighbours(r, k);
        }
        return fused;
    }

    // The block at cell (r, q), if any, sinks one row when every cell it needs
    // in row r + 1 is empty -- a move, not a fusion: it meets the block below
    // when the walk reaches row r + 1 -- and otherwise absorbs the block right
    // under this cell when the pair is fusible (consecutive fusion).  A
    // multi-qubit block is settled once per cell, so it can absorb a block
    // under any of its qubits.
    bool settle_cell(size_t r, int q, int k) {
        const int upper = rows_[r][q];
        if (upper < 0) return false;
        if (cells_free(r + 1, blocks_[upper].qubits, -1)) {
            move(upper, r, r + 1);
            return false;
        }
        const int lower = rows_[r + 1][q];
        if (lower < 0 || lower == upper || !fusible(upper, lower, k)) return false;
        fuse_consecutive(upper, lower, r);
        return true;
    }

    // Neighbouring cells (q - 1, q) of row r holding different blocks: the
    // two act at the same step on disjoint qubits, so they commute, and they
    // are fused when fusible (commuting fusion).
    bool merge_neighbours(size_t r, int k) {
        bool fused = false;
        for (int q = 1; q < n_; ++q) {
            const int a = rows_[r][q - 1], b = rows_[r][q];
            if (a < 0 || b < 0 || a == b || !fusible(a, b, k)) continue;
            place(fuse_pair(a, b), r, r);
            fused = true;
        }
        return fused;
    }

    // Re-appends every block in time order: removes empty rows and lifts
    // blocks into vacant space above them.
    void compress() {
        std::vector<int> order;
        std::vector<bool> seen(blocks_.size(), false);
        for (auto &row : rows_)
            for (int q = 0; q < n_; ++q) {
                const int b = row[q];
                if (b >= 0 && !seen[b]) seen[b] = true, order.push_back(b);
            }
        rows_.clear();
        last_.assign(n_, -1);
        for (int b : order) {
            int r = 0;
            for (int q : blocks_[b].qubits) r = std::max(r, last_[q] + 1);
            if (r == (int)rows_.size()) rows_.emplace_back(n_, -1);
            for (int q : blocks_[b].qubits) rows_[r][q] = b, last_[q] = r;
        }
    }

    std::vector<FusionGate> result() const {
        std::vector<FusionGate> out;
        std::vector<bool> seen(blocks_.size(), false);
        for (auto &row : rows_)
            for (int q = 0; q < n_; ++q) {
                const int b = row[q];
                if (b >= 0 && !seen[b]) {
                    seen[b] = true;
                    out.push_back(FusionGate{blocks_[b].qubits, blocks_[b].m});
                }
            }
        return out;
    }

  private:
    double snapped_opcount(const std::vector<cplx> &m) const {
        double nnz = 0;
        for (const cplx &z : m) nnz += (std::fabs(z.real()) > o_.zero_tol) + (std::fabs(z.imag()) > o_.zero_tol);
        return 2.0 * nnz;
    }

    bool cells_free(size_t r, const std::vector<int> &qs, int except) const {
        for (int q : qs)
            if (rows_[r][q] >= 0 && rows_[r][q] != except) return false;
        return true;
    }

    void move(int b, size_t from, size_t to) {
        for (int q : blocks_[b].qubits) rows_[from][q] = -1, rows_[to][q] = b;
    }

    bool fusible(int a, int b, int k) {
        const Block &A = blocks_[a], &B = blocks_[b];
        int u = (int)A.qubits.size();
        for (int q : B.qubits)
            if (!std::binary_search(A.qubits.begin(), A.qubits.end(), q)) ++u;
        if (u > k) return false;
        if (o_.opcount_cap > 0 || o_.cost_model == 1) {
            Block f = product(A, B);
            if (o_.opcount_cap > 0 && snapped_opcount(f.m) > o_.opcount_cap) return false;
            if (o_.cost_model == 1) {
                // adaptive check (Sec. III-C): keep the fusion only if one pass of
                // the product is predicted no slower than the two passes it replaces
                const cast_dtype dt = (cast_dtype)o_.cost_dtype;
                const double tf = pass_cost(dt, (int)f.qubits.size(), subspace_dim((int)f.qubits.size(), f.m, o_.zero_tol));
                const double ta = pass_cost(dt, (int)A.qubits.size(), subspace_dim((int)A.qubits.size(), A.m, o_.zero_tol));
                const double tb = pass_cost(dt, (int)B.qubits.size(), subspace_dim((int)B.qubits.size(), B.m, o_.zero_tol));
                if (tf > ta + tb) return false;
            }
        }
        return true;
    }

    int fuse_pair(int first, int second) {
        Block f = product(blocks_[first], blocks_[second]);
        f.opcount = snapped_opcount(f.m);
        for (auto &row : rows_)
            for (int q = 0; q < n_; ++q)
                if (row[q] == first || row[q] == second) row[q] = -1;
        alive_[first] = alive_[second] = false;
        blocks_.push_back(std::move(f));
        alive_.push_back(true);
        return (int)blocks_.size() - 1;
    }

    void fuse_consecutive(int top, int bottom, size_t r) {
        const int f = fuse_pair(top, bottom);
        const std::vector<int> &qs = blocks_[f].qubits;
        if (cells_free(r + 1, qs, -1)) place(f, r + 1, r + 1);
        else if (cells_free(r, qs, -1)) place(f, r, r);
        else {
            rows_.insert(rows_.begin() + (long)(r + 1), std::vector<int>(n_, -1));
            place(f, r + 1, r + 1);
        }
    }

    void place(int b, size_t r, size_t) {
        for (int q : blocks_[b].qubits) rows_[r][q] = b;
    }

    int n_;
    cast_fusion_opts o_;
    std::vector<Block> blocks_;
    std::vector<bool> alive_;
    std::vector<std::vector<int>> rows_;
    std::vector<int> last_;
};

}  // namespace

cast_status fuse(int n, std::vector<FusionGate> gates, const cast_fusion_opts &o, std::vector<FusionGate> *out) {
    Tile t(n, o);
    t.init_last();
    for (FusionGate &g : gates) {
        Block b;
        b.qubits = std::move(g.qubits);
        b.m = std::move(g.m);
        t.append(std::move(b));
    }
    const int k_lo = o.agglomerative ? 2 : o.k_max;
    for (int k = k_lo; k <= o.k_max; ++k) {
        if (k < 2) continue;
        bool delta;
        do {
            delta = t.traverse(k);
            t.compress();
        } while (delta && o.multi_traversal);
    }
    *out = t.result();
    return CAST_OK;
}

}  // namespace cast
