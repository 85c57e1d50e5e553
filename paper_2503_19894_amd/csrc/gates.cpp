// Standard gate matrices for the library (FP64).  Index convention: bit i of
// a row/column index belongs to the i-th listed qubit (Sec. II-A, Eq. 1 puts
// qubit q at index bit q).
#include <cmath>

#include "internal.hpp"

namespace cast {

static const cplx I1(0.0, 1.0);

static void pauli2(int letter, cplx out[4]) {
    // row-major 2x2
    switch (letter) {
        case 1: out[0] = 0; out[1] = 1; out[2] = 1; out[3] = 0; break;              // X
        case 2: out[0] = 0; out[1] = -I1; out[2] = I1; out[3] = 0; break;           // Y
        case 3: out[0] = 1; out[1] = 0; out[2] = 0; out[3] = -1.0; break;           // Z
        default: out[0] = 1; out[1] = 0; out[2] = 0; out[3] = 1; break;             // I
    }
}

std::vector<cplx> pauli_string_matrix(int k, int generator) {
    const int D = 1 << k;
    std::vector<cplx> m((size_t)D * D);
    cplx f[kMaxK][4];
    for (int i = 0; i < k; ++i) pauli2((generator >> (2 * i)) & 3, f[i]);
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c) {
            cplx v = 1.0;
            for (int i = 0; i < k; ++i) v *= f[i][(((r >> i) & 1) << 1) | ((c >> i) & 1)];
            m[(size_t)r * D + c] = v;
        }
    return m;
}

std::vector<cplx> rotation_matrix(int k, int generator, double angle) {
    // P^2 = I, so exp(-i a P / 2) = cos(a/2) I - i sin(a/2) P
    std::vector<cplx> m = pauli_string_matrix(k, generator);
    const int D = 1 << k;
    const double c = std::cos(angle / 2), s = std::sin(angle / 2);
    for (int r = 0; r < D; ++r)
        for (int cc = 0; cc < D; ++cc) {
            cplx &z = m[(size_t)r * D + cc];
            z = -I1 * s * z + (r == cc ? cplx(c, 0) : cplx(0, 0));
        }
    return m;
}

bool standard_gate(const std::string &name, const double *p, int *k, std::vector<cplx> *m) {
    auto diag = [&](std::initializer_list<cplx> d) {
        const int D = (int)d.size();
        m->assign((size_t)D * D, 0.0);
        int i = 0;
        for (cplx z : d) (*m)[(size_t)i * D + i] = z, ++i;
    };
    if (name == "id") { *k = 1; diag({1, 1}); return true; }
    if (name == "x") { *k = 1; *m = pauli_string_matrix(1, 1); return true; }
    if (name == "y") { *k = 1; *m = pauli_string_matrix(1, 2); return true; }
    if (name == "z") { *k = 1; *m = pauli_string_matrix(1, 3); return true; }
    if (name == "h") {
        *k = 1;
        const double r = 1.0 / std::sqrt(2.0);
        *m = {r, r, r, -r};
        return true;
    }
    if (name == "s") { *k = 1; diag({1, I1}); return true; }
    if (name == "t") { *k = 1; diag({1, std::exp(I1 * (M_PI / 4))}); return true; }
    if (name == "p") { *k = 1; diag({1, std::exp(I1 * p[0])}); return true; }
    if (name == "u3") {
        *k = 1;
        const double c = std::cos(p[0] / 2), s = std::sin(p[0] / 2);
        *m = {c, -std::exp(I1 * p[2]) * s, std::exp(I1 * p[1]) * s, std::exp(I1 * (p[1] + p[2])) * c};
        return true;
    }
    if (name == "rx") { *k = 1; *m = rotation_matrix(1, 1, p[0]); return true; }
    if (name == "ry") { *k = 1; *m = rotation_matrix(1, 2, p[0]); return true; }
    if (name == "rz") { *k = 1; *m = rotation_matrix(1, 3, p[0]); return true; }
    if (name == "rxx") { *k = 2; *m = rotation_matrix(2, 1 | (1 << 2), p[0]); return true; }
    if (name == "ryy") { *k = 2; *m = rotation_matrix(2, 2 | (2 << 2), p[0]); return true; }
    if (name == "rzz") { *k = 2; *m = rotation_matrix(2, 3 | (3 << 2), p[0]); return true; }
    if (name == "cz") { *k = 2; diag({1, 1, 1, -1.0}); return true; }
    if (name == "cp") { *k = 2; diag({1, 1, 1, std::exp(I1 * p[0])}); return true; }
    if (name == "cx") {
        // bit 0 = control, bit 1 = target: |c=1,t> -> |c=1,1-t>
        *k = 2;
        m->assign(16, 0.0);
        for (int j = 0; j < 4; ++j) (*m)[(size_t)((j & 1) ? (j ^ 2) : j) * 4 + j] = 1.0;
        return true;
    }
    if (name == "swap") {
        *k = 2;
        m->assign(16, 0.0);
        for (int j = 0; j < 4; ++j) (*m)[(size_t)(((j & 1) << 1) | (j >> 1)) * 4 + j] = 1.0;
        return true;
    }
    return false;
}

}  // namespace cast
