"""FP64 oracle: unfused, gate-by-gate simulation on the CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Gate application is the
C routine in ``sv_oracle.c`` (Eq. 3 written out); everything here is plain
numpy orchestration in the order the definitions give.
"""
import ctypes
import math
import os

import numpy as np

from . import gates as G

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None


def _load():
    global _lib
    if _lib is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from .build import build
            build(force=False)
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.oracle_apply_gate.argtypes = [dp, ctypes.c_int, ctypes.c_int, ip, dp]
        lib.oracle_apply_gate.restype = ctypes.c_int
        lib.oracle_inner.argtypes = [dp, dp, ctypes.c_int, dp, dp]
        lib.oracle_inner.restype = None
        lib.oracle_apply_gate_groups.argtypes = [dp, ctypes.c_int, ctypes.c_int, ip, dp,
                                                 ctypes.POINTER(ctypes.c_int64), ctypes.c_int64, dp]
        lib.oracle_apply_gate_groups.restype = ctypes.c_int
        lib.oracle_group_index.argtypes = [ctypes.c_int, ctypes.c_int, ip, ctypes.c_int64, ctypes.c_int]
        lib.oracle_group_index.restype = ctypes.c_int64
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _nqubits(psi):
    n = int(psi.size).bit_length() - 1
    if psi.size != (1 << n):
        raise ValueError("state length is not a power of two")
    return n


def apply_gate(psi, qubits, U):
    """In place: psi <- (U on `qubits`) psi, Eq. 3.  psi: complex128 C-contiguous."""
    assert psi.dtype == np.complex128 and psi.flags.c_contiguous
    U = np.ascontiguousarray(U, dtype=np.complex128)
    k = len(qubits)
    assert U.shape == (1 << k, 1 << k)
    q = (ctypes.c_int * k)(*[int(x) for x in qubits])
    rc = _load().oracle_apply_gate(_dp(psi.view(np.float64)), _nqubits(psi), k, q,
                                   _dp(U.view(np.float64)))
    if rc != 0:
        raise ValueError(f"oracle_apply_gate rejected qubits={qubits}")
    return psi


def apply_gate_groups(src, qubits, U, groups):
    """Outputs of the gate on the listed groups only (Eq. 3 restricted to
    those t), shape (len(groups), 2^k), member order j; src is not modified."""
    U = np.ascontiguousarray(U, dtype=np.complex128)
    k = len(qubits)
    groups = np.ascontiguousarray(groups, dtype=np.int64)
    out = np.empty((groups.size, 1 << k), dtype=np.complex128)
    q = (ctypes.c_int * k)(*[int(x) for x in qubits])
    rc = _load().oracle_apply_gate_groups(
        _dp(src.view(np.float64)), _nqubits(src), k, q, _dp(U.view(np.float64)),
        groups.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), groups.size, _dp(out.view(np.float64)))
    if rc != 0:
        raise ValueError("bad gate")
    return out


def group_index(n, qubits, t, j):
    """Amplitude index of member j of group t for a gate on `qubits`."""
    k = len(qubits)
    q = (ctypes.c_int * k)(*[int(x) for x in qubits])
    return int(_load().oracle_group_index(n, k, q, int(t), int(j)))


def inner(a, b):
    """<a|b> in FP64."""
    re, im = ctypes.c_double(), ctypes.c_double()
    _load().oracle_inner(_dp(a.view(np.float64)), _dp(b.view(np.float64)), _nqubits(a),
                         ctypes.byref(re), ctypes.byref(im))
    return complex(re.value, im.value)


def run_circuit(n, gates, psi0=None, theta=None):
    """Applies every gate of the list, unfused, in order; returns the state.
    psi0=None means |0...0>."""
    if psi0 is None:
        psi = np.zeros(1 << n, dtype=np.complex128)
        psi[0] = 1.0
    else:
        psi = np.array(psi0, dtype=np.complex128, copy=True)
        assert psi.size == 1 << n
    for g in gates:
        apply_gate(psi, g.qubits, G.matrix(g, theta))
    return psi


def _apply_pauli_term(psi, term):
    phi = psi.copy()
    for q, p in term.ops:
        apply_gate(phi, (q,), G.PAULI[p])
    return phi


def expval(psi, terms):
    """E = sum_m c_m <psi|P_m psi>: each Pauli factor applied as a 1-qubit gate,
    then an FP64 inner product.  Returns a complex number (imaginary part is
    round-off for Hermitian sums)."""
    e = 0.0 + 0.0j
    for t in terms:
        e += t.coeff * inner(psi, _apply_pauli_term(psi, t))
    return e


def energy(n, gates, theta, terms, psi0=None):
    return expval(run_circuit(n, gates, psi0, theta), terms).real


def adjoint_grad(n, gates, theta, terms, psi0=None):
    """Adjoint-method gradient (Jones & Gacon 2020, arXiv:2009.02823).

    Gates with param >= 0 are U_l = exp(-i c_l theta_p G_l / 2).  Forward to
    psi_L; lambda = H psi_L; E = Re<psi_L|lambda>.  Walking l = L..1, before
    uncomputing gate l: dE/dtheta_p += c_l Im<lambda|G_l|psi>; then
    psi <- U_l^dag psi and lambda <- U_l^dag lambda."""
    psi = run_circuit(n, gates, psi0, theta)
    lam = np.zeros_like(psi)
    for t in terms:
        lam += t.coeff * _apply_pauli_term(psi, t)
    e = inner(psi, lam).real
    grad = np.zeros(len(theta), dtype=np.float64)
    for g in reversed(gates):
        if g.param >= 0:
            gpsi = psi.copy()
            apply_gate(gpsi, g.qubits, G.pauli_string_matrix(G.GENERATOR[g.name]))
            grad[g.param] += g.coeff * inner(lam, gpsi).imag
        udag = G.matrix(g, theta).conj().T
        apply_gate(psi, g.qubits, udag)
        apply_gate(lam, g.qubits, udag)
    return e, grad


def finite_diff_grad(n, gates, theta, terms, psi0=None, h=1e-4, params=None):
    """Central differences [E(theta + h e_p) - E(theta - h e_p)] / (2h)."""
    theta = np.asarray(theta, dtype=np.float64)
    params = range(len(theta)) if params is None else params
    out = {}
    for p in params:
        tp, tm = theta.copy(), theta.copy()
        tp[p] += h
        tm[p] -= h
        out[p] = (energy(n, gates, tp, terms, psi0) - energy(n, gates, tm, terms, psi0)) / (2 * h)
    return out


def param_shift_grad(n, gates, theta, terms, psi0=None, params=None):
    """[E(theta + pi/2 e_p) - E(theta - pi/2 e_p)] / 2: exact for a parameter
    used by a single rotation with coefficient 1."""
    theta = np.asarray(theta, dtype=np.float64)
    params = range(len(theta)) if params is None else params
    out = {}
    for p in params:
        tp, tm = theta.copy(), theta.copy()
        tp[p] += math.pi / 2
        tm[p] -= math.pi / 2
        out[p] = (energy(n, gates, tp, terms, psi0) - energy(n, gates, tm, terms, psi0)) / 2
    return out
