"""Vectorised amplitude indices of sampled gate groups (Eq. 3-4): the bits of
each group number t are deposited, lowest first, into the non-target
positions, and member j sets target qubits[i] to bit i of j.  Used to gather a
sample of groups from a large device state; pinned against the oracle's
scalar rule in tests/test_group_members.py."""
import numpy as np


def member_indices(n, qubits, groups):
    """int64 array (len(groups), 2^k): index of member j of group t."""
    qubits = [int(q) for q in qubits]
    k = len(qubits)
    t = np.asarray(groups, dtype=np.uint64)
    base = np.zeros_like(t)
    src = 0
    for pos in range(n):
        if pos in qubits:
            continue
        base |= ((t >> np.uint64(src)) & np.uint64(1)) << np.uint64(pos)
        src += 1
    off = np.zeros(1 << k, dtype=np.uint64)
    for j in range(1 << k):
        for i, q in enumerate(qubits):
            if (j >> i) & 1:
                off[j] |= np.uint64(1) << np.uint64(q)
    return (base[:, None] | off[None, :]).astype(np.int64)
