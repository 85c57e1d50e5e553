// Host analysis of one gate before it becomes a device pass: qubit sorting,
// zero/one snapping (Table 2 "-zero-tolerance", "-one-tolerance"), the
// operation count of Sec. III-C, and the block structure that lets the kernels
// skip every structurally-zero entry (Sec. III overview: zero entries of the
// matrix are skipped).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.hpp"

namespace cast {

static double snap(double x, double zt, double ot) {
    if (std::fabs(x) <= zt) return 0.0;
    if (std::fabs(x - 1.0) <= ot) return 1.0;
    if (std::fabs(x + 1.0) <= ot) return -1.0;
    return x;
}

int subspace_dim(int k, const std::vector<cplx> &m, double zt) {
    const int D = 1 << k;
    bool seen[64] = {false};
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c) {
            const cplx z = m[(size_t)r * D + c];
            if (std::fabs(z.real()) > zt || std::fabs(z.imag()) > zt) seen[r ^ c] = true;
        }
    uint32_t basis[kMaxK];
    int piv[kMaxK], d = 0;
    for (uint32_t v0 = 1; v0 < (uint32_t)D; ++v0) {
        if (!seen[v0]) continue;
        uint32_t v = v0;
        for (int i = 0; i < d; ++i)
            if ((v >> piv[i]) & 1u) v ^= basis[i];
        if (!v) continue;
        const int pv = __builtin_ctz(v);
        for (int i = 0; i < d; ++i)
            if ((basis[i] >> pv) & 1u) basis[i] ^= v;
        basis[d] = v;
        piv[d] = pv;
        ++d;
    }
    return d;
}

double opcount_of(const std::vector<cplx> &m) {
    double nnz = 0;
    for (const cplx &z : m) nnz += (z.real() != 0.0) + (z.imag() != 0.0);
    return 2.0 * nnz;
}

static inline uint32_t apply_L(const uint32_t *L, int k, uint32_t u) {
    uint32_t j = 0;
    for (int i = 0; i < k; ++i)
        if ((u >> i) & 1u) j ^= L[i];
    return j;
}

cast_status make_plan(int k, const int *qubits, const cplx *m, double zt, double ot, PassPlan *out) {
    if (k < 1 || k > kMaxK) return fail(CAST_EINVAL, "gate size k must be in [1, 6]");
    const int D = 1 << k;
    PassPlan p;
    p.k = k;
    // sort targets; pos[i] = rank of qubits[i]
    int order[kMaxK];
    for (int i = 0; i < k; ++i) order[i] = i;
    std::sort(order, order + k, [&](int a, int b) { return qubits[a] < qubits[b]; });
    int pos[kMaxK];
    for (int r = 0; r < k; ++r) {
        p.q[r] = qubits[order[r]];
        pos[order[r]] = r;
    }
    auto perm = [&](uint32_t j) {
        uint32_t o = 0;
        for (int i = 0; i < k; ++i)
            if ((j >> i) & 1u) o |= 1u << pos[i];
        return o;
    };
    p.full.assign((size_t)D * D, cplx(0, 0));
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c) {
            cplx z = m[(size_t)r * D + c];
            p.full[(size_t)perm(r) * D + perm(c)] =
                cplx(snap(z.real(), zt, ot), snap(z.imag(), zt, ot));
        }
    p.opcount = opcount_of(p.full);

    // XOR subspace spanned by {r ^ c : M[r][c] != 0}, reduced echelon basis
    bool seen[64] = {false};
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c)
            if (p.full[(size_t)r * D + c] != cplx(0, 0)) seen[r ^ c] = true;
    uint32_t basis[kMaxK];
    int piv[kMaxK];
    int d = 0;
    for (uint32_t v0 = 1; v0 < (uint32_t)D; ++v0) {
        if (!seen[v0]) continue;
        uint32_t v = v0;
        for (int i = 0; i < d; ++i)
            if ((v >> piv[i]) & 1u) v ^= basis[i];
        if (!v) continue;
        int pv = __builtin_ctz(v);
        for (int i = 0; i < d; ++i)
            if ((basis[i] >> pv) & 1u) basis[i] ^= v;
        basis[d] = v;
        piv[d] = pv;
        ++d;
    }
    p.d = d;
    uint32_t pivmask = 0;
    for (int i = 0; i < d; ++i) {
        p.L[i] = basis[i];
        pivmask |= 1u << piv[i];
    }
    int nx = d;
    for (int b = 0; b < k; ++b)
        if (!((pivmask >> b) & 1u)) p.L[nx++] = 1u << b;

    // blocks in virtual coordinates
    const int bd = 1 << d, nblk = 1 << (k - d);
    for (int b = 0; b < nblk; ++b) {
        std::vector<cplx> blk((size_t)bd * bd);
        bool ident = true;
        for (int r = 0; r < bd; ++r)
            for (int c = 0; c < bd; ++c) {
                uint32_t jr = apply_L(p.L, k, ((uint32_t)b << d) | (uint32_t)r);
                uint32_t jc = apply_L(p.L, k, ((uint32_t)b << d) | (uint32_t)c);
                cplx z = p.full[(size_t)jr * D + jc];
                blk[(size_t)r * bd + c] = z;
                if (z != (r == c ? cplx(1, 0) : cplx(0, 0))) ident = false;
            }
        if (ident) continue;
        p.blk.push_back((uint32_t)b);
        p.mat.insert(p.mat.end(), blk.begin(), blk.end());
    }
    *out = std::move(p);
    return CAST_OK;
}

}  // namespace cast
