"""The vectorised group-member helper agrees with the oracle's scalar rule."""
import numpy as np

import oracle
from tests.group_members import member_indices


def test_member_indices_match_oracle():
    rng = np.random.default_rng(77)
    for n, qubits in ((32, (27, 3, 14, 0, 31, 9)), (32, (5, 6, 30, 1, 17)), (10, (9,)), (12, (0, 1, 2))):
        k = len(qubits)
        groups = rng.integers(0, 1 << (n - k), 64)
        idx = member_indices(n, qubits, groups)
        for gi in range(len(groups)):
            for j in range(1 << k):
                assert idx[gi, j] == oracle.group_index(n, qubits, int(groups[gi]), j)
