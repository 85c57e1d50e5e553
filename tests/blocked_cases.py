"""Seeded circuits that exercise every in-tile gate kind of the cache-blocked
executor (input generation only; no simulation)."""
import math

import numpy as np

from circuits import Gate
from circuits.generators import haar_unitary


def mixed_circuit(n, seed, layers=5):
    """Per layer, on random qubits: Haar 1-, 2- and 3-qubit gates (blocks of
    2, 4 and 8), controlled Haar gates (identity blocks, controls anywhere),
    diagonal phases on up to 5 qubits (targets inside or outside a tile),
    SWAP and CX (blocks that mix two qubits at once), U3 and CZ."""
    rng = np.random.default_rng(seed)
    gates = []

    def qs(k):
        return tuple(int(q) for q in rng.permutation(n)[:k])

    for _ in range(layers):
        for _ in range(max(4, n // 2)):
            kind = int(rng.integers(8))
            if kind <= 2:
                k = kind + 1
                gates.append(Gate("unitary", qs(k), matrix=haar_unitary(1 << k, rng)))
            elif kind == 3:
                k = int(rng.integers(2, 4))
                m = np.eye(1 << k, dtype=np.complex128)
                c = (1 << (k - 1)) - 1
                hi = 1 << (k - 1)
                m[np.ix_([c, c | hi], [c, c | hi])] = haar_unitary(2, rng)
                gates.append(Gate("unitary", qs(k), matrix=m))
            elif kind == 4:
                k = int(rng.integers(1, 6))
                ph = np.exp(1j * rng.uniform(0, 2 * math.pi, 1 << k))
                ph[rng.random(1 << k) < 0.3] = 1.0
                gates.append(Gate("unitary", qs(k), matrix=np.diag(ph)))
            elif kind == 5:
                gates.append(Gate("swap", qs(2)))
            elif kind == 6:
                gates.append(Gate("cx", qs(2)))
            else:
                gates.append(Gate("u3", qs(1), tuple(float(a) for a in rng.uniform(0, 2 * math.pi, 3))))
                gates.append(Gate("cz", qs(2)))
    return gates
