// Host interface of the reduction kernels (reduce.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/cast.h"

namespace cast {

constexpr int kMaxZ = 8;  // z-masks evaluated per pass of k_pauli_inner

struct PauliSumGroup {
    uint64_t x;
    int first, count;
};
struct PauliSumTerm {
    uint64_t z;
    double cre, cim;  // coefficient times i^{|x&z|}
};

// Doubles of device scratch pauli_inner needs.
size_t reduce_scratch_doubles();

// dev_out[2j], dev_out[2j+1] = re, im of S(x, z_j) = sum_y conj(a[y^x]) (-1)^{|z_j & y|} b[y]
// for j < nz (1 <= nz <= 8), FP64, fixed reduction order.  Stream-ordered.
cast_status pauli_inner(const void *a, const void *b, int n, cast_dtype dt, uint64_t x, const uint64_t *z, int nz,
                        double *scratch, double *dev_out, hipStream_t s);

// out = (sum of Pauli terms) psi; term tables in device memory.  out != psi.
cast_status apply_pauli_sum(const void *psi, void *out, int n, cast_dtype dt, const PauliSumGroup *dgroups,
                            int ngroups, const PauliSumTerm *dterms, hipStream_t s);

}  // namespace cast
