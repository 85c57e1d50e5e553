"""Gate and Pauli-term records shared by the oracle, the GPU binding and the tests.

Conventions (Sec. II-A, Eq. 1): qubit q is bit q of the amplitude index.  A
gate's matrix is indexed so that bit i of the row/column index belongs to
``qubits[i]``; e.g. ``cx`` with ``qubits=(c, t)`` maps |c=1,t=0> to |c=1,t=1>.

Parametrised rotations (``param >= 0``) take the angle ``coeff * theta[param]``
and mean exp(-i * angle * G / 2) with G = X, Y, Z (1-qubit) or XX, YY, ZZ.
"""
from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np

#: gate name -> (number of qubits, number of fixed angles)
GATE_ARITY = {
    "id": (1, 0), "h": (1, 0), "x": (1, 0), "y": (1, 0), "z": (1, 0), "s": (1, 0), "t": (1, 0),
    "u3": (1, 3), "rx": (1, 1), "ry": (1, 1), "rz": (1, 1), "p": (1, 1),
    "cx": (2, 0), "cz": (2, 0), "cp": (2, 1), "swap": (2, 0),
    "rxx": (2, 1), "ryy": (2, 1), "rzz": (2, 1),
}

#: rotations that may carry ``param >= 0``
PARAMETRISABLE = ("rx", "ry", "rz", "rxx", "ryy", "rzz")


@dataclass(frozen=True)
class Gate:
    name: str
    qubits: Tuple[int, ...]
    params: Tuple[float, ...] = ()
    matrix: Optional[np.ndarray] = field(default=None, compare=False)  # name == "unitary"
    param: int = -1
    coeff: float = 1.0

    @property
    def k(self) -> int:
        return len(self.qubits)


@dataclass(frozen=True)
class PauliTerm:
    coeff: float
    ops: Tuple[Tuple[int, str], ...]  # ((qubit, "X" | "Y" | "Z"), ...), distinct qubits
