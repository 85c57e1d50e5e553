// Exercises the host-only entry points of libcast (gate table, fusion,
// planning, pass schedules, cache-blocked grouping, tuning, argument
// validation) without a GPU, for runs under AddressSanitizer and
// UndefinedBehaviorSanitizer.  Exits nonzero if a call behaves unexpectedly.
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../include/cast.h"

using cplx = std::complex<double>;

static int failures = 0;
#define EXPECT(cond)                                                        \
    do {                                                                    \
        if (!(cond)) {                                                      \
            std::fprintf(stderr, "FAILED %s:%d: %s\n", __FILE__, __LINE__, #cond); \
            ++failures;                                                     \
        }                                                                   \
    } while (0)

struct OwnedGate {
    cast_gate g;
    std::vector<double> m;
};

static std::vector<OwnedGate> random_circuit(int n, int count, std::mt19937_64 &rng) {
    std::vector<OwnedGate> out(count);
    std::uniform_real_distribution<double> u(-1.0, 1.0);
    for (auto &og : out) {
        const int kind = (int)(rng() % 4);
        const int k = 1 + (int)(rng() % (kind == 0 ? 6 : 3));
        std::vector<int> qs;
        while ((int)qs.size() < k) {
            const int q = (int)(rng() % n);
            bool dup = false;
            for (int x : qs) dup |= x == q;
            if (!dup) qs.push_back(q);
        }
        const int D = 1 << k;
        og.m.assign(2 * D * D, 0.0);
        for (int r = 0; r < D; ++r)
            for (int c = 0; c < D; ++c) {
                const bool nz = kind == 0 || (kind == 1 && r == c) || (kind == 2 && (r ^ c) == (D - 1)) ||
                                (kind == 3 && (r == c || (r ^ c) == 1));
                if (!nz) continue;
                og.m[2 * (r * D + c)] = (kind == 1 && (rng() % 3 == 0)) ? 1.0 : u(rng);
                og.m[2 * (r * D + c) + 1] = (kind == 1 && og.m[2 * (r * D + c)] == 1.0) ? 0.0 : u(rng);
            }
        og.g.k = k;
        for (int i = 0; i < 6; ++i) og.g.qubits[i] = i < k ? qs[i] : 0;
        og.g.param_id = -1;
        og.g.param_coeff = 1.0;
        og.g.generator = 0;
    }
    for (auto &og : out) og.g.matrix = og.m.data();
    return out;
}

static std::vector<OwnedGate> named_circuit(const std::vector<std::pair<const char *, std::vector<int>>> &spec,
                                            double angle) {
    std::vector<OwnedGate> out(spec.size());
    for (size_t i = 0; i < spec.size(); ++i) {
        int k = 0;
        out[i].m.assign(2 * 64 * 64, 0.0);
        const double params[3] = {angle * (double)(i + 1), 0.3, -0.2};
        EXPECT(gate_matrix(spec[i].first, params, &k, out[i].m.data()) == CAST_OK);
        EXPECT(k == (int)spec[i].second.size());
        out[i].g.k = k;
        for (int j = 0; j < 6; ++j) out[i].g.qubits[j] = j < k ? spec[i].second[j] : 0;
        out[i].g.param_id = -1;
        out[i].g.param_coeff = 1.0;
        out[i].g.generator = 0;
    }
    for (auto &og : out) og.g.matrix = og.m.data();
    return out;
}

static std::vector<cast_gate> view(const std::vector<OwnedGate> &v) {
    std::vector<cast_gate> g;
    for (auto &og : v) g.push_back(og.g);
    return g;
}

static void inspect(cast_fused *f, int n) {
    size_t nf = 0;
    double oc = 0, ms = 0;
    EXPECT(fused_info(f, &nf, &oc, &ms) == CAST_OK);
    std::vector<double> mat(2 * 64 * 64);
    for (size_t i = 0; i < nf; ++i) {
        int k, qs[6], d, nb;
        double op;
        EXPECT(fused_gate(f, i, &k, qs, &op, &d, &nb, mat.data()) == CAST_OK);
        for (cast_dtype dt : {CAST_C64, CAST_C128}) {
            int kern, dd;
            double b, fl;
            EXPECT(fused_pass_info(f, i, n, dt, &kern, &dd, &b, &fl) == CAST_OK);
        }
    }
    EXPECT(fused_gate(f, nf, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == CAST_EINVAL);
    for (cast_dtype dt : {CAST_C64, CAST_C128}) {
        for (int tables : {0, 1, 2, 4}) {
            EXPECT(tuning_set("diag_run_tables", dt, tables) == CAST_OK);
            for (int q : {4, 8}) {
                EXPECT(tuning_set("diag_run_qubits", dt, q) == CAST_OK);
                size_t np = 0;
                EXPECT(circuit_passes(f, n, dt, &np) == CAST_OK);
                size_t covered = 0;
                for (size_t i = 0; i < np; ++i) {
                    size_t first, count;
                    int kern, tabs;
                    double b, fl;
                    EXPECT(circuit_pass_info(f, n, dt, i, &first, &count, &kern, &tabs, &b, &fl) == CAST_OK);
                    EXPECT(first == covered);
                    covered += count;
                }
                EXPECT(covered == nf);
                EXPECT(circuit_pass_info(f, n, dt, np, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) ==
                       CAST_EINVAL);
            }
        }
        EXPECT(tuning_set("diag_run_tables", dt, 4) == CAST_OK);
        EXPECT(tuning_set("diag_run_qubits", dt, 8) == CAST_OK);
    }
}

int main() {
    std::mt19937_64 rng(12345);
    // gate table
    for (const char *name : {"id", "h", "x", "y", "z", "s", "t", "p", "u3", "rx", "ry", "rz", "rxx", "ryy", "rzz",
                             "cx", "cz", "cp", "swap"}) {
        int k = 0;
        std::vector<double> out(2 * 16);
        const double params[3] = {0.4, -1.1, 2.0};
        EXPECT(gate_matrix(name, params, &k, out.data()) == CAST_OK);
    }
    {
        int k;
        double out[32];
        EXPECT(gate_matrix("nope", nullptr, &k, out) == CAST_EINVAL);
    }
    // fusion and planning on random and structured circuits
    cast_fusion_opts o;
    for (int n : {6, 12, 20}) {
        auto circ = random_circuit(n, 60, rng);
        auto gv = view(circ);
        for (int kmax = 1; kmax <= 6; ++kmax)
            for (int cost = 0; cost <= 1; ++cost)
                for (int agg = 0; agg <= 1; ++agg) {
                    fusion_opts_default(&o);
                    o.k_max = kmax;
                    o.cost_model = cost;
                    o.agglomerative = agg;
                    o.opcount_cap = (kmax == 4) ? 1024 : 0;
                    cast_fused *f = nullptr;
                    EXPECT(fuse_circuit(n, gv.data(), gv.size(), &o, &f) == CAST_OK);
                    if (f) {
                        inspect(f, n);
                        size_t np = 0;
                        if (blocked_info(f, n, CAST_C128, &np) == CAST_OK) {
                            for (size_t i = 0; i < np; ++i) {
                                size_t first, count;
                                int tb, w, hq[10];
                                EXPECT(blocked_pass_info(f, n, CAST_C128, i, &first, &count, &tb, &w, hq) == CAST_OK);
                            }
                        }
                        fused_destroy(f);
                    }
                }
    }
    {
        // QFT-like structure at 30 qubits: controlled phases and swaps
        std::vector<std::pair<const char *, std::vector<int>>> spec;
        const int n = 30;
        for (int j = n - 1; j >= 0; --j) {
            spec.push_back({"h", {j}});
            for (int m = j - 1; m >= 0; --m) spec.push_back({"cp", {m, j}});
        }
        for (int i = 0; i < n / 2; ++i) spec.push_back({"swap", {i, n - 1 - i}});
        auto circ = named_circuit(spec, 0.01);
        auto gv = view(circ);
        fusion_opts_default(&o);
        cast_fused *f = nullptr;
        EXPECT(fuse_circuit(n, gv.data(), gv.size(), &o, &f) == CAST_OK);
        if (f) {
            inspect(f, n);
            fused_destroy(f);
        }
    }
    // path planner: pricing and plan choice over k_max 1..6
    {
        auto circ = random_circuit(16, 80, rng);
        auto gv = view(circ);
        for (cast_dtype dt : {CAST_C64, CAST_C128}) {
            cast_fused *f = nullptr;
            int path = -1, k = -1;
            double ms = 0;
            EXPECT(plan_circuit(16, gv.data(), gv.size(), dt, nullptr, 1, 6, &f, &path, &k, &ms) == CAST_OK);
            EXPECT(f != nullptr && (path == 0 || path == 1) && k >= 1 && k <= 6 && ms > 0);
            double p0 = 0, p1 = 0;
            EXPECT(predict_ms(f, 16, dt, 0, &p0) == CAST_OK);
            EXPECT(predict_ms(f, 16, dt, 1, &p1) == CAST_OK);
            EXPECT(predict_ms(f, 16, dt, 2, &p1) == CAST_EINVAL);
            fused_destroy(f);
            double v = 0;
            EXPECT(path_cost_get("seg_gate2", dt, &v) == CAST_OK && v > 0);
            EXPECT(path_cost_set("seg_gate2", dt, v) == CAST_OK);
            EXPECT(path_cost_set("bw7", dt, 1.0) == CAST_EINVAL);
        }
        cast_fused *f = nullptr;
        int path, k;
        EXPECT(plan_circuit(16, gv.data(), gv.size(), CAST_C128, nullptr, 3, 2, &f, &path, &k, nullptr) == CAST_EINVAL);
    }
    // validation paths
    {
        fusion_opts_default(&o);
        o.k_max = 7;
        cast_fused *f = nullptr;
        auto circ = random_circuit(8, 4, rng);
        auto gv = view(circ);
        EXPECT(fuse_circuit(8, gv.data(), gv.size(), &o, &f) == CAST_EINVAL);
        fusion_opts_default(&o);
        gv[0].qubits[0] = 9;
        EXPECT(fuse_circuit(8, gv.data(), gv.size(), &o, &f) == CAST_EINVAL);
        gv[0].qubits[0] = 0;
        gv[1].param_id = 0;
        EXPECT(fuse_circuit(8, gv.data(), gv.size(), &o, &f) == CAST_EINVAL);
        EXPECT(fuse_circuit(8, nullptr, 3, &o, &f) == CAST_EINVAL);
    }
    {
        cast_sv *sv = nullptr;
        EXPECT(sv_create(0, CAST_C128, nullptr, &sv) == CAST_EINVAL);
        EXPECT(sv_wrap((void *)0x1008, 4, CAST_C128, nullptr, &sv) == CAST_EINVAL);
        EXPECT(sv_wrap((void *)0x100000, 4, CAST_C128, nullptr, &sv) == CAST_OK);
        const int dup[2] = {1, 1};
        double m[32] = {1, 0};
        EXPECT(apply_gate(sv, dup, 2, m) == CAST_EINVAL);
        cast_pauli_term t = {1.0, 1u << 4, 0};
        double out[2];
        EXPECT(expval(sv, &t, 1, out) == CAST_EINVAL);
        sv_destroy(sv);
        sv_destroy(nullptr);
        fused_destroy(nullptr);
    }
    // tuning and cost table
    int v = 0;
    EXPECT(tuning_get("diag_unroll", CAST_C128, &v) == CAST_OK);
    EXPECT(tuning_set("diag_unroll", CAST_C128, 3) == CAST_EINVAL);
    EXPECT(tuning_set("no_such_key", CAST_C128, 1) == CAST_EINVAL);
    EXPECT(tuning_set("diag_unroll", CAST_C128, v) == CAST_OK);
    double c = 0;
    EXPECT(cost_table_get(CAST_C128, 3, 1, &c) == CAST_OK);
    EXPECT(cost_table_set(CAST_C128, 3, 1, c) == CAST_OK);
    EXPECT(cost_table_set(CAST_C128, 9, 1, c) == CAST_EINVAL);
    std::printf("host driver: %d failures\n", failures);
    return failures ? 1 : 0;
}
