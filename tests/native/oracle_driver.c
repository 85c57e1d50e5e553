/* Exercises the C oracle (oracle/sv_oracle.c) for runs under AddressSanitizer
 * and UndefinedBehaviorSanitizer: random gates on small states, the sampled
 * group form against the full application, the group-index rule, inner
 * products and argument rejection.  Exits nonzero on any mismatch. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_apply_gate(double *psi, int n, int k, const int *qubits, const double *U);
void oracle_inner(const double *a, const double *b, int n, double *out_re, double *out_im);
int oracle_apply_gate_groups(const double *src, int n, int k, const int *qubits, const double *U,
                             const int64_t *groups, int64_t ngroups, double *out);
int64_t oracle_group_index(int n, int k, const int *qubits, int64_t t, int j);

static uint64_t st = 88172645463325252ull;
static uint64_t rnd(void) { st ^= st << 13; st ^= st >> 7; st ^= st << 17; return st; }
static double urand(void) { return (double)(rnd() >> 11) / 9007199254740992.0 * 2.0 - 1.0; }

int main(void)
{
    int fails = 0;
    for (int trial = 0; trial < 200; ++trial) {
        const int n = 1 + (int)(rnd() % 10);
        const int k = 1 + (int)(rnd() % (n < 6 ? n : 6));
        int q[6];
        for (int i = 0; i < k;) {
            const int c = (int)(rnd() % n);
            int dup = 0;
            for (int j = 0; j < i; ++j) dup |= q[j] == c;
            if (!dup) q[i++] = c;
        }
        const int D = 1 << k;
        const int64_t N = (int64_t)1 << n;
        double *U = malloc(sizeof(double) * 2 * D * D);
        double *psi = malloc(sizeof(double) * 2 * N);
        double *src = malloc(sizeof(double) * 2 * N);
        for (int i = 0; i < 2 * D * D; ++i) U[i] = urand();
        for (int64_t i = 0; i < 2 * N; ++i) psi[i] = src[i] = urand();
        if (oracle_apply_gate(psi, n, k, q, U) != 0) ++fails;
        const int64_t ng = (int64_t)1 << (n - k);
        int64_t *groups = malloc(sizeof(int64_t) * ng);
        for (int64_t t = 0; t < ng; ++t) groups[t] = t;
        double *out = malloc(sizeof(double) * 2 * ng * D);
        if (oracle_apply_gate_groups(src, n, k, q, U, groups, ng, out) != 0) ++fails;
        for (int64_t t = 0; t < ng; ++t)
            for (int j = 0; j < D; ++j) {
                const int64_t x = oracle_group_index(n, k, q, t, j);
                if (x < 0 || x >= N) { ++fails; continue; }
                if (out[2 * (t * D + j)] != psi[2 * x] || out[2 * (t * D + j) + 1] != psi[2 * x + 1]) ++fails;
            }
        double re, im;
        oracle_inner(psi, psi, n, &re, &im);
        if (!(re > 0) || fabs(im) > 1e-9 * re) ++fails;
        free(U); free(psi); free(src); free(groups); free(out);
    }
    {
        double psi[8] = {1, 0, 0, 0, 0, 0, 0, 0}, U[8] = {1, 0, 0, 0, 0, 0, 1, 0};
        int bad[2] = {0, 0}, oob[1] = {2};
        if (oracle_apply_gate(psi, 2, 2, bad, U) != -1) ++fails;
        if (oracle_apply_gate(psi, 2, 1, oob, U) != -1) ++fails;
        if (oracle_apply_gate(psi, 2, 3, bad, U) != -1) ++fails;
    }
    printf("oracle driver: %d failures\n", fails);
    return fails ? 1 : 0;
}
