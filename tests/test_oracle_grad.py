"""Pins for the oracle's expectation values and gradients.

Closed forms (GHZ, |+...+>, single-qubit rotations), Pauli strings built by
numpy kron straight from Eq. 1, the parameter-shift rule (exact for a
parameter used once with coefficient 1), central finite differences, and the
global-flip symmetry of the textbook transverse-field Ising convention."""
import math

import numpy as np
import pytest

import oracle
from oracle import gates as OG
from circuits import (Gate, PauliTerm, hea_vqa, random_state, tfim_fields, tfim_trotter,
                      vqa_hamiltonian, vqa_thetas)


def _kron_pauli(n, ops):
    m = np.ones((1, 1), dtype=np.complex128)
    d = dict(ops)
    for q in range(n - 1, -1, -1):          # most significant qubit first (Eq. 1)
        m = np.kron(m, OG.PAULI[d.get(q, "I")])
    return m


def test_expval_ghz_closed_forms():
    n = 6
    psi = oracle.run_circuit(n, [Gate("h", (0,))] + [Gate("cx", (0, i)) for i in range(1, n)])
    for i in range(n):
        assert abs(oracle.expval(psi, [PauliTerm(1.0, ((i, "Z"),))])) < 1e-15
        for j in range(i + 1, n):
            assert abs(oracle.expval(psi, [PauliTerm(1.0, ((i, "Z"), (j, "Z")))]) - 1) < 1e-15
    xall = PauliTerm(1.0, tuple((q, "X") for q in range(n)))
    assert abs(oracle.expval(psi, [xall]) - 1) < 1e-15


def test_expval_plus_state_and_y():
    n = 5
    psi = np.full(1 << n, 2 ** (-n / 2), dtype=np.complex128)
    for q in range(n):
        assert abs(oracle.expval(psi, [PauliTerm(1.0, ((q, "X"),))]) - 1) < 1e-15
    for th in (0.3, 1.7, -2.2):
        psi = oracle.run_circuit(1, [Gate("rx", (0,), (th,))])
        assert abs(oracle.expval(psi, [PauliTerm(1.0, ((0, "Y"),))]) - (-math.sin(th))) < 1e-15
        assert abs(oracle.expval(psi, [PauliTerm(1.0, ((0, "Z"),))]) - math.cos(th)) < 1e-15


def test_expval_matches_kron_pauli_strings():
    n = 6
    rng = np.random.default_rng(3)
    psi = random_state(n, seed=5, workload=9)
    for _ in range(10):
        qs = rng.permutation(n)[: rng.integers(1, n + 1)]
        ops = tuple((int(q), "XYZ"[rng.integers(3)]) for q in qs)
        c = float(rng.normal())
        want = c * np.vdot(psi, _kron_pauli(n, ops) @ psi)
        got = oracle.expval(psi, [PauliTerm(c, ops)])
        assert abs(got - want) < 1e-14


def test_adjoint_single_qubit_closed_form():
    for th in (0.1, 1.0, 2.5, -1.3):
        e, g = oracle.adjoint_grad(1, [Gate("ry", (0,), param=0)], np.array([th]),
                                   [PauliTerm(1.0, ((0, "Z"),))])
        assert abs(e - math.cos(th)) < 1e-15
        assert abs(g[0] + math.sin(th)) < 1e-15
    # coefficient: RX(c*theta), <Z> = cos(c theta) -> d/dtheta = -c sin(c theta)
    c, th = -0.7, 0.9
    e, g = oracle.adjoint_grad(1, [Gate("rx", (0,), param=0, coeff=c)], np.array([th]),
                               [PauliTerm(1.0, ((0, "Z"),))])
    assert abs(e - math.cos(c * th)) < 1e-15
    assert abs(g[0] + c * math.sin(c * th)) < 1e-15


def test_adjoint_matches_parameter_shift_hea():
    n = 5
    gates, P = hea_vqa(n=n, layers=2)
    theta = vqa_thetas(P, 1, seed=1)[0]
    H = vqa_hamiltonian(n)
    e, g = oracle.adjoint_grad(n, gates, theta, H)
    ps = oracle.param_shift_grad(n, gates, theta, H)
    for p in range(P):
        assert abs(g[p] - ps[p]) < 1e-12, p
    assert abs(e - oracle.energy(n, gates, theta, H)) < 1e-13


def test_adjoint_matches_finite_differences_two_qubit_generators():
    n = 4
    rng = np.random.default_rng(8)
    gates = []
    for layer in range(3):
        for q in range(n):
            gates.append(Gate("ry", (q,), param=len(gates)))
        for q in range(n - 1):
            gates.append(Gate(["rxx", "ryy", "rzz"][layer], (q, q + 1), param=len(gates), coeff=0.5))
    P = len(gates)
    theta = rng.uniform(-math.pi, math.pi, P)
    H = [PauliTerm(0.8, ((0, "X"), (2, "Y"))), PauliTerm(-0.3, ((1, "Z"),)), PauliTerm(1.1, ((3, "Y"),))]
    e, g = oracle.adjoint_grad(n, gates, theta, H)
    fd = oracle.finite_diff_grad(n, gates, theta, H, h=1e-4)
    for p in range(P):
        assert abs(g[p] - fd[p]) < 1e-7, (p, g[p], fd[p])


def test_adjoint_shared_parameter_chain_rule_tfim():
    n = 4
    h = tfim_fields(n, seed=0)
    gates = tfim_trotter(n, steps=3, dt=0.05)
    psi0 = np.full(1 << n, 2 ** (-n / 2), dtype=np.complex128)
    obs = [PauliTerm(1.0, ((0, "Z"),))]
    e, g = oracle.adjoint_grad(n, gates, h, obs, psi0)
    fd = oracle.finite_diff_grad(n, gates, h, obs, psi0, h=1e-4)
    for p in range(n):
        assert abs(g[p] - fd[p]) < 1e-8


def test_tfim_textbook_convention_symmetry_zero():
    """With H = -J sum ZZ - sum h X from |+...+>, every Trotter gate commutes
    with the global flip prod X_i, of which |+...+> is a +1 eigenstate, so
    <Z_0> and all its gradients vanish."""
    n = 6
    h = tfim_fields(n, seed=1)
    gates = tfim_trotter(n, steps=5, dt=0.05, convention="zz")
    psi0 = np.full(1 << n, 2 ** (-n / 2), dtype=np.complex128)
    e, g = oracle.adjoint_grad(n, gates, h, [PauliTerm(1.0, ((0, "Z"),))], psi0)
    assert abs(e) < 1e-14 and np.max(np.abs(g)) < 1e-14
    e2, g2 = oracle.adjoint_grad(n, tfim_trotter(n, steps=5, dt=0.05), h,
                                 [PauliTerm(1.0, ((0, "Z"),))], psi0)
    assert abs(e2) > 0.05 and np.max(np.abs(g2)) > 1e-3
