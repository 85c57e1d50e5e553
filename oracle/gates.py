"""Gate matrices for the oracle, in FP64 (numpy complex128).

The paper names H and U3 (Table 3) but defines no gate; these are the textbook
definitions.  Index convention (Sec. II-A, Eq. 1): bit i of a matrix row or
column index belongs to the i-th listed qubit, so ``cx`` on (control, target)
is [[1,0,0,0],[0,0,0,1],[0,0,1,0],[0,1,0,0]].
"""
import math

import numpy as np

I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / math.sqrt(2.0)
PAULI = {"I": I2, "X": X, "Y": Y, "Z": Z}
#: Pauli string generating each rotation: R(angle) = exp(-i angle G / 2)
GENERATOR = {"rx": "X", "ry": "Y", "rz": "Z", "rxx": "XX", "ryy": "YY", "rzz": "ZZ"}


def u3(theta, phi, lam):
    c, s = math.cos(theta / 2), math.sin(theta / 2)
    return np.array([[c, -np.exp(1j * lam) * s],
                     [np.exp(1j * phi) * s, np.exp(1j * (phi + lam)) * c]], dtype=np.complex128)


def pauli_string_matrix(letters):
    """Matrix of P_0 (x) ... on the listed qubits, letters[i] on matrix bit i
    (so letters[0] is the least-significant factor)."""
    m = np.ones((1, 1), dtype=np.complex128)
    for ch in letters:
        m = np.kron(PAULI[ch], m)
    return m


def rotation(letters, angle):
    """exp(-i angle P / 2) = cos(angle/2) I - i sin(angle/2) P, since P^2 = I."""
    p = pauli_string_matrix(letters)
    return math.cos(angle / 2) * np.eye(p.shape[0]) - 1j * math.sin(angle / 2) * p


def matrix(g, theta=None):
    """Matrix of a ``circuits.Gate`` (parametrised gates read ``theta``)."""
    name = g.name
    if g.param >= 0:
        return rotation(GENERATOR[name], g.coeff * float(theta[g.param]))
    if name == "unitary":
        return np.asarray(g.matrix, dtype=np.complex128)
    if name == "id":
        return I2.copy()
    if name == "h":
        return H.copy()
    if name == "x":
        return X.copy()
    if name == "y":
        return Y.copy()
    if name == "z":
        return Z.copy()
    if name == "s":
        return np.diag([1, 1j]).astype(np.complex128)
    if name == "t":
        return np.diag([1, np.exp(1j * math.pi / 4)]).astype(np.complex128)
    if name == "p":
        return np.diag([1, np.exp(1j * g.params[0])]).astype(np.complex128)
    if name == "u3":
        return u3(*g.params)
    if name == "rx":
        return rotation("X", g.params[0])
    if name == "ry":
        return rotation("Y", g.params[0])
    if name == "rz":
        return rotation("Z", g.params[0])
    if name == "rxx":
        return rotation("XX", g.params[0])
    if name == "ryy":
        return rotation("YY", g.params[0])
    if name == "rzz":
        return rotation("ZZ", g.params[0])
    if name == "cx":
        # bit 0 = control, bit 1 = target: flip bit 1 where bit 0 is set
        m = np.zeros((4, 4), dtype=np.complex128)
        for j in range(4):
            m[j ^ 2 if j & 1 else j, j] = 1
        return m
    if name == "cz":
        return np.diag([1, 1, 1, -1]).astype(np.complex128)
    if name == "cp":
        return np.diag([1, 1, 1, np.exp(1j * g.params[0])]).astype(np.complex128)
    if name == "swap":
        m = np.zeros((4, 4), dtype=np.complex128)
        for j in range(4):
            m[((j & 1) << 1) | (j >> 1), j] = 1
        return m
    raise ValueError(f"unknown gate {name}")
