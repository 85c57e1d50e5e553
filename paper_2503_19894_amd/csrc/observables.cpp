// Host side of the observable entry points: Pauli-sum expectation values and
// adjoint-method gradients (Jones & Gacon 2020) of parametrised circuits.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>

#include "internal.hpp"
#include "reduce.hpp"

namespace cast {

static const cplx kIpow[4] = {cplx(1, 0), cplx(0, 1), cplx(-1, 0), cplx(0, -1)};

// Terms grouped by x mask, in first-appearance order of the x masks.
struct Grouped {
    std::vector<uint64_t> x;
    std::vector<std::vector<size_t>> idx;
};

static Grouped group_by_x(const cast_pauli_term *t, size_t n) {
    Grouped g;
    std::map<uint64_t, size_t> where;
    for (size_t i = 0; i < n; ++i) {
        auto it = where.find(t[i].xmask);
        if (it == where.end()) {
            where[t[i].xmask] = g.x.size();
            g.x.push_back(t[i].xmask);
            g.idx.emplace_back();
            g.idx.back().push_back(i);
        } else {
            g.idx[it->second].push_back(i);
        }
    }
    return g;
}

static cast_status check_terms(int n, const cast_pauli_term *t, size_t nt) {
    if (nt && !t) return fail(CAST_EINVAL, "terms is NULL");
    const uint64_t full = n >= 64 ? ~0ull : ((1ull << n) - 1);
    for (size_t i = 0; i < nt; ++i)
        if ((t[i].xmask | t[i].zmask) & ~full) return fail(CAST_EINVAL, "Pauli term acts outside the state");
    return CAST_OK;
}

// RAII device scratch from the reuse pool.  The block goes back only after
// its stream has drained (a no-op when the call already synchronised), so
// an early error return never hands out memory that queued work still uses.
struct DevBuf {
    void *p = nullptr;
    size_t cls = 0;
    hipStream_t s = nullptr;
    explicit DevBuf(hipStream_t stream) : s(stream) {}
    ~DevBuf() {
        if (!p) return;
        (void)hipStreamSynchronize(s);
        pool_free(p, cls);
    }
    cast_status alloc(size_t bytes) { return pool_alloc(&p, bytes, &cls); }
    template <typename T> T *as() const { return (T *)p; }
};

// Queues all z-groups of one x-mask; results (re, im per term) land in
// dev_out[2 * slot(term)].
static cast_status queue_pauli_inner(const void *a, const void *b, int n, cast_dtype dt, uint64_t x,
                                     const std::vector<uint64_t> &zs, double *scratch, double *dev_out,
                                     hipStream_t s) {
    for (size_t j0 = 0; j0 < zs.size(); j0 += kMaxZ) {
        const int nz = (int)std::min<size_t>(kMaxZ, zs.size() - j0);
        if (cast_status rc = pauli_inner(a, b, n, dt, x, zs.data() + j0, nz, scratch, dev_out + 2 * j0, s)) return rc;
    }
    return CAST_OK;
}

static void gen_masks(const int *qubits, int k, int generator, uint64_t *x, uint64_t *z) {
    *x = 0;
    *z = 0;
    for (int i = 0; i < k; ++i) {
        const int letter = (generator >> (2 * i)) & 3;
        if (letter == 1 || letter == 2) *x |= 1ull << qubits[i];
        if (letter == 2 || letter == 3) *z |= 1ull << qubits[i];
    }
}

}  // namespace cast

using namespace cast;

extern "C" {

cast_status expval(const cast_sv *sv, const cast_pauli_term *terms, size_t n_terms, double *out) {
    if (!sv || !sv->data) return fail(CAST_EINVAL, "state is NULL");
    if (!out) return fail(CAST_EINVAL, "out is NULL");
    if (cast_status rc = check_terms(sv->n, terms, n_terms)) return rc;
    out[0] = out[1] = 0.0;
    if (!n_terms) return CAST_OK;
    Grouped g = group_by_x(terms, n_terms);
    DevBuf scratch(sv->stream), res(sv->stream);
    if (cast_status rc = scratch.alloc(reduce_scratch_doubles() * sizeof(double))) return rc;
    if (cast_status rc = res.alloc(2 * n_terms * sizeof(double))) return rc;
    std::vector<size_t> slot_of(n_terms);
    size_t slot = 0;
    for (size_t gi = 0; gi < g.x.size(); ++gi) {
        std::vector<uint64_t> zs;
        for (size_t i : g.idx[gi]) {
            zs.push_back(terms[i].zmask);
            slot_of[i] = slot++;
        }
        const size_t first = slot_of[g.idx[gi][0]];
        if (cast_status rc = queue_pauli_inner(sv->data, sv->data, sv->n, sv->dt, g.x[gi], zs, scratch.as<double>(),
                                               res.as<double>() + 2 * first, sv->stream))
            return rc;
    }
    std::vector<double> h(2 * n_terms);
    CAST_HIP_TRY(hipMemcpyAsync(h.data(), res.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, sv->stream));
    CAST_HIP_TRY(hipStreamSynchronize(sv->stream));
    cplx e = 0;
    for (size_t i = 0; i < n_terms; ++i) {
        const size_t s = slot_of[i];
        const cplx S(h[2 * s], h[2 * s + 1]);
        e += terms[i].coeff * kIpow[__builtin_popcountll(terms[i].xmask & terms[i].zmask) & 3] * S;
    }
    out[0] = e.real();
    out[1] = e.imag();
    return CAST_OK;
}

cast_status adjoint_grad(const cast_sv *init, const cast_gate *gates, size_t n_gates, const double *theta,
                         size_t n_params, const cast_pauli_term *terms, size_t n_terms, double *energy,
                         double *grad) {
    if (!init || !init->data) return fail(CAST_EINVAL, "init state is NULL");
    if (n_gates && !gates) return fail(CAST_EINVAL, "gates is NULL");
    if (n_params && (!theta || !grad)) return fail(CAST_EINVAL, "theta/grad is NULL");
    if (!energy) return fail(CAST_EINVAL, "energy is NULL");
    if (cast_status rc = check_terms(init->n, terms, n_terms)) return rc;
    const int n = init->n;
    const cast_dtype dt = init->dt;
    hipStream_t s = init->stream;
    // ---- bind parameters, plan U_l and U_l^dag
    std::vector<PassPlan> plans;
    plans.reserve(2 * n_gates);
    std::vector<int> slot(n_gates, -1);
    int nslots = 0;
    for (size_t l = 0; l < n_gates; ++l) {
        const cast_gate &g = gates[l];
        if (g.k < 1 || g.k > kMaxK) return fail(CAST_EINVAL, "gate k out of range");
        for (int i = 0; i < g.k; ++i) {
            if (g.qubits[i] < 0 || g.qubits[i] >= n) return fail(CAST_EINVAL, "gate qubit out of range");
            for (int j = 0; j < i; ++j)
                if (g.qubits[i] == g.qubits[j]) return fail(CAST_EINVAL, "duplicate gate qubit");
        }
        std::vector<cplx> m;
        if (g.param_id >= 0) {
            if ((size_t)g.param_id >= n_params) return fail(CAST_EINVAL, "param_id out of range");
            if (g.generator <= 0 || g.generator >= (1 << (2 * g.k)))
                return fail(CAST_EINVAL, "parametrised gate needs a Pauli generator on its qubits");
            m = rotation_matrix(g.k, g.generator, g.param_coeff * theta[g.param_id]);
            slot[l] = nslots++;
        } else {
            if (!g.matrix) return fail(CAST_EINVAL, "fixed gate without a matrix");
            const size_t D = (size_t)1 << g.k;
            m.resize(D * D);
            for (size_t i = 0; i < D * D; ++i) m[i] = cplx(g.matrix[2 * i], g.matrix[2 * i + 1]);
        }
        const size_t D = (size_t)1 << g.k;
        std::vector<cplx> md(D * D);
        for (size_t r = 0; r < D; ++r)
            for (size_t c = 0; c < D; ++c) md[c * D + r] = std::conj(m[r * D + c]);
        PassPlan pf, pb;
        if (cast_status rc = make_plan(g.k, g.qubits, m.data(), 1e-14, 1e-14, &pf)) return rc;
        if (cast_status rc = make_plan(g.k, g.qubits, md.data(), 1e-14, 1e-14, &pb)) return rc;
        plans.push_back(std::move(pf));
        plans.push_back(std::move(pb));
    }
    std::vector<size_t> off;
    DevBuf mats(s);
    if (cast_status rc = upload_plans_pooled(plans, dt, &mats.p, &mats.cls, &off)) return rc;
    const size_t rsz = dt == CAST_C128 ? 8 : 4;
    auto mat_of = [&](size_t i) { return (const void *)((const char *)mats.p + off[i] * rsz); };

    const size_t sbytes = ((size_t)1 << n) * amp_bytes(dt);
    DevBuf psi(s), lam(s), scratch(s), res(s), tgroups(s), tterms(s);
    if (cast_status rc = psi.alloc(sbytes)) return rc;
    if (cast_status rc = lam.alloc(sbytes)) return rc;
    if (cast_status rc = scratch.alloc(reduce_scratch_doubles() * sizeof(double))) return rc;
    if (cast_status rc = res.alloc((2 + 2 * (size_t)nslots) * sizeof(double))) return rc;
    CAST_HIP_TRY(hipMemcpyAsync(psi.p, init->data, sbytes, hipMemcpyDeviceToDevice, s));
    // ---- forward
    for (size_t l = 0; l < n_gates; ++l)
        if (cast_status rc = launch_pass(psi.p, n, dt, plans[2 * l], mat_of(2 * l), s)) return rc;
    // ---- lambda = H psi, E = <psi|lambda>
    Grouped g = group_by_x(terms, n_terms);
    std::vector<PauliSumGroup> hg;
    std::vector<PauliSumTerm> ht;
    for (size_t gi = 0; gi < g.x.size(); ++gi) {
        hg.push_back(PauliSumGroup{g.x[gi], (int)ht.size(), (int)g.idx[gi].size()});
        for (size_t i : g.idx[gi]) {
            const cplx c = terms[i].coeff * kIpow[__builtin_popcountll(terms[i].xmask & terms[i].zmask) & 3];
            ht.push_back(PauliSumTerm{terms[i].zmask, c.real(), c.imag()});
        }
    }
    if (n_terms) {
        if (cast_status rc = tgroups.alloc(hg.size() * sizeof(PauliSumGroup))) return rc;
        if (cast_status rc = tterms.alloc(ht.size() * sizeof(PauliSumTerm))) return rc;
        CAST_HIP_TRY(hipMemcpyAsync(tgroups.p, hg.data(), hg.size() * sizeof(PauliSumGroup), hipMemcpyHostToDevice, s));
        CAST_HIP_TRY(hipMemcpyAsync(tterms.p, ht.data(), ht.size() * sizeof(PauliSumTerm), hipMemcpyHostToDevice, s));
        if (cast_status rc = apply_pauli_sum(psi.p, lam.p, n, dt, tgroups.as<PauliSumGroup>(), (int)hg.size(),
                                             tterms.as<PauliSumTerm>(), s))
            return rc;
    } else {
        CAST_HIP_TRY(hipMemsetAsync(lam.p, 0, sbytes, s));
    }
    const uint64_t z0 = 0;
    if (cast_status rc = pauli_inner(psi.p, lam.p, n, dt, 0, &z0, 1, scratch.as<double>(), res.as<double>(), s))
        return rc;
    // ---- reverse sweep
    std::vector<uint64_t> gx(n_gates), gz(n_gates);
    for (size_t li = n_gates; li-- > 0;) {
        const cast_gate &gg = gates[li];
        if (slot[li] >= 0) {
            gen_masks(gg.qubits, gg.k, gg.generator, &gx[li], &gz[li]);
            if (cast_status rc = pauli_inner(lam.p, psi.p, n, dt, gx[li], &gz[li], 1, scratch.as<double>(),
                                             res.as<double>() + 2 + 2 * slot[li], s))
                return rc;
        }
        if (cast_status rc = launch_pass(psi.p, n, dt, plans[2 * li + 1], mat_of(2 * li + 1), s)) return rc;
        if (cast_status rc = launch_pass(lam.p, n, dt, plans[2 * li + 1], mat_of(2 * li + 1), s)) return rc;
    }
    std::vector<double> h(2 + 2 * (size_t)nslots);
    CAST_HIP_TRY(hipMemcpyAsync(h.data(), res.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    CAST_HIP_TRY(hipStreamSynchronize(s));
    *energy = h[0];
    for (size_t p = 0; p < n_params; ++p) grad[p] = 0.0;
    // d E / d theta_p += c_l Im(<lambda|G_l|psi>), <lambda|G|psi> = i^{|x&z|} S
    for (size_t li = n_gates; li-- > 0;) {
        if (slot[li] < 0) continue;
        const cplx S(h[2 + 2 * slot[li]], h[3 + 2 * slot[li]]);
        const cplx v = kIpow[__builtin_popcountll(gx[li] & gz[li]) & 3] * S;
        grad[gates[li].param_id] += gates[li].param_coeff * v.imag();
    }
    return CAST_OK;
}

}  // extern "C"
