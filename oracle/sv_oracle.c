/*
 * Plain CPU FP64 state-vector oracle.  TEST INFRASTRUCTURE ONLY: this file is
 * compiled into oracle/liboracle.so, which only the test-suite, the smoke check
 * and the CPU-baseline leg of the benchmark load.  It shares no code with the
 * GPU library.
 *
 * State layout (Sec. II-A, Eq. 1): an n-qubit state is 2^n complex amplitudes
 * stored interleaved (re, im) as doubles; qubit q is bit q of the amplitude
 * index (the factor I^{(n-k-1)} (x) U (x) I^{(k)} acts on index bit k).
 *
 * oracle_apply_gate is Eq. 3 written out: a k-qubit gate U (2^k x 2^k,
 * row-major, interleaved complex) acts on 2^{n-k} independent groups of 2^k
 * amplitudes.  Group t collects the indices whose non-target bits spell t (t's
 * bits deposited, lowest first, into the non-target positions); member j of
 * the group sets target qubits[i] to bit i of j.  No zero skipping, no fusion,
 * no special cases.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_MAX_K 12

/* Deposit the bits of t, lowest first, into the positions of [0, n) that are
 * not in `is_target`. */
static uint64_t deposit_nontarget(uint64_t t, int n, const unsigned char *is_target)
{
    uint64_t x = 0;
    int src = 0;
    for (int pos = 0; pos < n; ++pos) {
        if (is_target[pos]) continue;
        if ((t >> src) & 1u) x |= (uint64_t)1 << pos;
        ++src;
    }
    return x;
}

/* Returns 0 on success, -1 on bad arguments (k out of range, a qubit out of
 * range or repeated). psi is updated in place. */
int oracle_apply_gate(double *psi, int n, int k, const int *qubits, const double *U)
{
    if (n < 1 || n > 40 || k < 1 || k > ORACLE_MAX_K || k > n) return -1;
    unsigned char is_target[64];
    memset(is_target, 0, sizeof is_target);
    for (int i = 0; i < k; ++i) {
        if (qubits[i] < 0 || qubits[i] >= n || is_target[qubits[i]]) return -1;
        is_target[qubits[i]] = 1;
    }
    const int64_t ngroups = (int64_t)1 << (n - k);
    const int dim = 1 << k;

#pragma omp parallel
    {
        int64_t idx[1 << ORACLE_MAX_K];
        double vre[1 << ORACLE_MAX_K], vim[1 << ORACLE_MAX_K];
#pragma omp for schedule(static)
        for (int64_t t = 0; t < ngroups; ++t) {
            uint64_t base = deposit_nontarget((uint64_t)t, n, is_target);
            for (int j = 0; j < dim; ++j) {
                uint64_t x = base;
                for (int i = 0; i < k; ++i)
                    if ((j >> i) & 1) x |= (uint64_t)1 << qubits[i];
                idx[j] = (int64_t)x;
                vre[j] = psi[2 * x];
                vim[j] = psi[2 * x + 1];
            }
            for (int r = 0; r < dim; ++r) {
                double accre = 0.0, accim = 0.0;
                for (int c = 0; c < dim; ++c) {
                    double ure = U[2 * (r * dim + c)], uim = U[2 * (r * dim + c) + 1];
                    accre += ure * vre[c] - uim * vim[c];
                    accim += ure * vim[c] + uim * vre[c];
                }
                psi[2 * idx[r]] = accre;
                psi[2 * idx[r] + 1] = accim;
            }
        }
    }
    return 0;
}

/* <a|b> = sum_x conj(a[x]) b[x] over 2^n amplitudes, plain FP64 sums. */
void oracle_inner(const double *a, const double *b, int n, double *out_re, double *out_im)
{
    const int64_t N = (int64_t)1 << n;
    double sre = 0.0, sim = 0.0;
#pragma omp parallel for reduction(+ : sre, sim) schedule(static)
    for (int64_t x = 0; x < N; ++x) {
        double ar = a[2 * x], ai = a[2 * x + 1], br = b[2 * x], bi = b[2 * x + 1];
        sre += ar * br + ai * bi;
        sim += ar * bi - ai * br;
    }
    *out_re = sre;
    *out_im = sim;
}

/* Applies the gate to selected groups only: for each listed group index t,
 * reads the group's 2^k amplitudes from `src` (a full 2^n state) and writes the
 * 2^k results, in member order j, to out[t_i * 2^k + j]. Used to check one
 * pass of a very large state on a sample of groups. */
int oracle_apply_gate_groups(const double *src, int n, int k, const int *qubits, const double *U,
                             const int64_t *groups, int64_t ngroups, double *out)
{
    if (n < 1 || n > 40 || k < 1 || k > ORACLE_MAX_K || k > n) return -1;
    unsigned char is_target[64];
    memset(is_target, 0, sizeof is_target);
    for (int i = 0; i < k; ++i) {
        if (qubits[i] < 0 || qubits[i] >= n || is_target[qubits[i]]) return -1;
        is_target[qubits[i]] = 1;
    }
    const int dim = 1 << k;
#pragma omp parallel
    {
        double vre[1 << ORACLE_MAX_K], vim[1 << ORACLE_MAX_K];
#pragma omp for schedule(static)
        for (int64_t g = 0; g < ngroups; ++g) {
            uint64_t base = deposit_nontarget((uint64_t)groups[g], n, is_target);
            for (int j = 0; j < dim; ++j) {
                uint64_t x = base;
                for (int i = 0; i < k; ++i)
                    if ((j >> i) & 1) x |= (uint64_t)1 << qubits[i];
                vre[j] = src[2 * x];
                vim[j] = src[2 * x + 1];
            }
            for (int r = 0; r < dim; ++r) {
                double accre = 0.0, accim = 0.0;
                for (int c = 0; c < dim; ++c) {
                    double ure = U[2 * (r * dim + c)], uim = U[2 * (r * dim + c) + 1];
                    accre += ure * vre[c] - uim * vim[c];
                    accim += ure * vim[c] + uim * vre[c];
                }
                out[2 * (g * dim + r)] = accre;
                out[2 * (g * dim + r) + 1] = accim;
            }
        }
    }
    return 0;
}

/* Index of member j of group t (same deposit rule as above); lets a caller
 * locate where a group lives in a full state. */
int64_t oracle_group_index(int n, int k, const int *qubits, int64_t t, int j)
{
    unsigned char is_target[64];
    memset(is_target, 0, sizeof is_target);
    for (int i = 0; i < k; ++i) is_target[qubits[i]] = 1;
    uint64_t x = deposit_nontarget((uint64_t)t, n, is_target);
    for (int i = 0; i < k; ++i)
        if ((j >> i) & 1) x |= (uint64_t)1 << qubits[i];
    return (int64_t)x;
}
