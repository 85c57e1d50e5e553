"""Pins for the oracle's gate application (Eq. 1-3) and gate matrices.

Each check is independent of the oracle's own code path: numpy kron built
straight from Eq. 1, a tensor contraction (einsum) on the [2]*n reshaped
state, exact index permutations, and closed forms (GHZ, product states, QFT
phases, numpy's inverse FFT)."""
import math

import numpy as np
import pytest

import oracle
from oracle import gates as OG
from circuits import Gate, qft, random_state, rqc_u3_cx, dense_haar_layers
from circuits.generators import haar_unitary


def _rand_state(n, seed):
    return random_state(n, seed=seed, workload=9)


def _eq1_full(n, k_lo, U):
    """Eq. 1: I^{(n-k-1)} (x) U (x) I^{(k)} for a gate on adjacent ascending
    qubits k_lo, k_lo+1, ... (matrix bit i <-> qubit k_lo + i)."""
    d = U.shape[0]
    kk = d.bit_length() - 1
    return np.kron(np.kron(np.eye(1 << (n - k_lo - kk)), U), np.eye(1 << k_lo))


def _einsum_apply(psi, qubits, U):
    """Tensor contraction on the state reshaped to [2]*n (axis a <-> qubit n-1-a)."""
    n = psi.size.bit_length() - 1
    k = len(qubits)
    T = psi.reshape([2] * n)
    # U as a tensor: out bits (k-1..0) then in bits (k-1..0), bit i <-> qubits[i]
    Ut = U.reshape([2] * (2 * k))
    axes_in = [n - 1 - qubits[i] for i in range(k - 1, -1, -1)]
    res = np.tensordot(Ut, T, axes=(list(range(k, 2 * k)), axes_in))
    # res axes: k output axes (for qubits[k-1..0]) followed by the remaining axes in order
    rest = [a for a in range(n) if a not in axes_in]
    order = axes_in + rest
    inv = np.argsort(order)
    return np.transpose(res, inv).reshape(-1)


@pytest.mark.parametrize("n", [1, 3, 6, 8])
def test_single_qubit_matches_eq1_kron(n):
    rng = np.random.default_rng(n)
    for q in range(n):
        U = haar_unitary(2, rng)
        psi = _rand_state(n, q)
        want = _eq1_full(n, q, U) @ psi
        got = oracle.apply_gate(psi.copy(), (q,), U)
        np.testing.assert_allclose(got, want, atol=1e-14, rtol=0)


@pytest.mark.parametrize("n", [2, 5, 8])
def test_adjacent_two_qubit_matches_eq1_kron(n):
    rng = np.random.default_rng(10 + n)
    for q in range(n - 1):
        U = haar_unitary(4, rng)
        psi = _rand_state(n, q)
        want = _eq1_full(n, q, U) @ psi
        got = oracle.apply_gate(psi.copy(), (q, q + 1), U)
        np.testing.assert_allclose(got, want, atol=1e-14, rtol=0)


@pytest.mark.parametrize("n,k", [(4, 3), (6, 2), (7, 4), (8, 5), (8, 6), (8, 1)])
def test_arbitrary_targets_match_tensor_contraction(n, k):
    rng = np.random.default_rng(100 * n + k)
    for trial in range(4):
        qs = tuple(int(x) for x in rng.permutation(n)[:k])   # unsorted on purpose
        U = haar_unitary(1 << k, rng)
        psi = _rand_state(n, trial)
        want = _einsum_apply(psi, qs, U)
        got = oracle.apply_gate(psi.copy(), qs, U)
        np.testing.assert_allclose(got, want, atol=1e-13, rtol=0)


def test_brute_force_full_matrix_n6():
    """Full 2^n x 2^n operator of a whole random circuit, built from Eq. 1
    krons and SWAP-free permutations, against the oracle's run."""
    n = 6
    gates = rqc_u3_cx(n=n, layers=3, seed=3)
    M = np.eye(1 << n, dtype=np.complex128)
    for g in gates:
        U = OG.matrix(g)
        if g.k == 1:
            F = _eq1_full(n, g.qubits[0], U)
        else:
            c, t = g.qubits
            assert t == c + 1
            F = _eq1_full(n, c, U)
        M = F @ M
    psi0 = _rand_state(n, 7)
    got = oracle.run_circuit(n, gates, psi0)
    np.testing.assert_allclose(got, M @ psi0, atol=1e-13, rtol=0)


@pytest.mark.parametrize("n", [3, 7])
def test_permutation_and_sign_gates_bit_exact(n):
    psi = _rand_state(n, 1)
    idx = np.arange(1 << n)
    for q in range(n):
        got = oracle.apply_gate(psi.copy(), (q,), OG.X)
        assert np.array_equal(got, psi[idx ^ (1 << q)])
        sign = np.where((idx >> q) & 1, -1.0, 1.0)
        got = oracle.apply_gate(psi.copy(), (q,), OG.Z)
        assert np.array_equal(got, psi * sign)
    for a in range(n):
        for b in range(n):
            if a == b:
                continue
            got = oracle.apply_gate(psi.copy(), (a, b), OG.matrix(Gate("cx", (a, b))))
            src = np.where((idx >> a) & 1, idx ^ (1 << b), idx)
            assert np.array_equal(got, psi[src])
            got = oracle.apply_gate(psi.copy(), (a, b), OG.matrix(Gate("swap", (a, b))))
            ba, bb = (idx >> a) & 1, (idx >> b) & 1
            src = idx & ~((1 << a) | (1 << b)) | (ba << b) | (bb << a)
            assert np.array_equal(got, psi[src])
            got = oracle.apply_gate(psi.copy(), (a, b), OG.matrix(Gate("cz", (a, b))))
            sign = np.where(((idx >> a) & (idx >> b) & 1) == 1, -1.0, 1.0)
            assert np.array_equal(got, psi * sign)


def test_cx_orientation():
    psi = np.zeros(4, dtype=np.complex128)
    psi[1] = 1.0                      # |c=1 (qubit 0), t=0 (qubit 1)>
    got = oracle.apply_gate(psi, (0, 1), OG.matrix(Gate("cx", (0, 1))))
    assert got[3] == 1.0 and np.count_nonzero(got) == 1


@pytest.mark.parametrize("n", [2, 5, 10])
def test_ghz(n):
    gates = [Gate("h", (0,))] + [Gate("cx", (0, i)) for i in range(1, n)]
    psi = oracle.run_circuit(n, gates)
    want = np.zeros(1 << n, dtype=np.complex128)
    want[0] = want[-1] = 1 / math.sqrt(2)
    np.testing.assert_allclose(psi, want, atol=1e-15, rtol=0)


def test_product_layer_closed_form():
    n = 7
    rng = np.random.default_rng(5)
    gates = [Gate("u3", (q,), tuple(rng.uniform(0, 2 * math.pi, 3))) for q in range(n)]
    psi = oracle.run_circuit(n, gates)
    cols = [OG.u3(*g.params)[:, 0] for g in gates]
    for x in range(1 << n):
        want = np.prod([cols[q][(x >> q) & 1] for q in range(n)])
        assert abs(psi[x] - want) < 1e-15


@pytest.mark.parametrize("n", [1, 4, 9])
def test_qft_basis_states_closed_form(n):
    N = 1 << n
    for x in sorted({0, 1, N // 3, N - 1}):
        psi0 = np.zeros(N, dtype=np.complex128)
        psi0[x] = 1.0
        got = oracle.run_circuit(n, qft(n), psi0)
        y = np.arange(N)
        want = np.exp(2j * np.pi * x * y / N) / math.sqrt(N)
        np.testing.assert_allclose(got, want, atol=1e-13, rtol=0)


@pytest.mark.parametrize("n", [6, 12])
def test_qft_random_state_is_scaled_ifft(n):
    psi0 = _rand_state(n, 2)
    got = oracle.run_circuit(n, qft(n), psi0)
    want = np.fft.ifft(psi0) * math.sqrt(1 << n)
    np.testing.assert_allclose(got, want, atol=1e-13, rtol=0)


def test_norm_and_inverse():
    gates = dense_haar_layers(n=11, depth=2, seed=1)
    n = 11
    psi0 = _rand_state(n, 4)
    psi = oracle.run_circuit(n, gates, psi0)
    assert abs(np.vdot(psi, psi).real - 1.0) < 1e-13
    inv = [Gate("unitary", g.qubits, matrix=OG.matrix(g).conj().T) for g in reversed(gates)]
    back = oracle.run_circuit(n, inv, psi)
    np.testing.assert_allclose(back, psi0, atol=1e-12, rtol=0)


def test_rqc_config_norm_and_inverse():
    n = 12
    gates = rqc_u3_cx(n, 10, seed=0)
    assert len(gates) == 175
    psi = oracle.run_circuit(n, gates)
    assert abs(np.vdot(psi, psi).real - 1.0) < 1e-13
    inv = [Gate("unitary", g.qubits, matrix=OG.matrix(g).conj().T) for g in reversed(gates)]
    back = oracle.run_circuit(n, inv, psi)
    want = np.zeros(1 << n); want[0] = 1
    np.testing.assert_allclose(back, want, atol=1e-12, rtol=0)


def test_group_outputs_match_full_apply():
    n, qs = 9, (7, 2, 4)
    rng = np.random.default_rng(0)
    U = haar_unitary(8, rng)
    psi = _rand_state(n, 3)
    full = oracle.apply_gate(psi.copy(), qs, U)
    groups = np.array([0, 5, 17, 63], dtype=np.int64)
    out = oracle.apply_gate_groups(psi, qs, U, groups)
    for gi, t in enumerate(groups):
        for j in range(8):
            assert out[gi, j] == full[oracle.group_index(n, qs, t, j)]


def test_rejects_bad_qubits():
    psi = _rand_state(3, 0)
    with pytest.raises(ValueError):
        oracle.apply_gate(psi, (0, 0), np.eye(4))
    with pytest.raises(ValueError):
        oracle.apply_gate(psi, (3,), np.eye(2))


def test_gate_matrices_unitary_and_textbook():
    from circuits import GATE_ARITY
    rng = np.random.default_rng(1)
    for name, (k, npar) in GATE_ARITY.items():
        g = Gate(name, tuple(range(k)), tuple(rng.uniform(-3, 3, npar)))
        U = OG.matrix(g)
        np.testing.assert_allclose(U.conj().T @ U, np.eye(1 << k), atol=1e-14)
    # textbook identities that a sign or transpose slip would break
    np.testing.assert_allclose(OG.matrix(Gate("u3", (0,), (math.pi / 2, 0, math.pi))), OG.H, atol=1e-15)
    np.testing.assert_allclose(OG.matrix(Gate("rx", (0,), (math.pi,))), -1j * OG.X, atol=1e-15)
    np.testing.assert_allclose(OG.matrix(Gate("ry", (0,), (math.pi,))), -1j * OG.Y, atol=1e-15)
    np.testing.assert_allclose(OG.matrix(Gate("rz", (0,), (math.pi,))), -1j * OG.Z, atol=1e-15)
    np.testing.assert_allclose(OG.Y, 1j * OG.X @ OG.Z, atol=0)
    th = 0.37
    rxx = OG.matrix(Gate("rxx", (0, 1), (th,)))
    np.testing.assert_allclose(rxx, math.cos(th / 2) * np.eye(4) - 1j * math.sin(th / 2) * np.kron(OG.X, OG.X), atol=1e-15)
    rzz = OG.matrix(Gate("rzz", (0, 1), (th,)))
    np.testing.assert_allclose(np.diag(rzz), np.exp(-1j * th / 2 * np.array([1, -1, -1, 1])), atol=1e-15)
