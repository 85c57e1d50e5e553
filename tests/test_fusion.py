"""Host gate fusion (Sec. III, Alg. 1), checked on the CPU.

The fused list is replayed by the oracle (each fused gate as one k-qubit gate,
Eq. 3) and compared with the oracle's unfused run; fused sizes respect k_max;
operation counts match the values the paper fixes."""
import math
import os

import numpy as np
import pytest

import oracle
import paper_2503_19894_amd as cast
from circuits import (Gate, dense_haar_layers, gate_sweep, hea_vqa, qft, random_state, rqc_u3_cx,
                      tfim_trotter, tfim_fields, vqa_thetas)
from circuits.generators import haar_unitary

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_opcounts.txt")


def replay(fc, n, psi0):
    psi = psi0.copy()
    for i in range(len(fc)):
        g = fc.gate(i, with_matrix=True)
        oracle.apply_gate(psi, g["qubits"], g["matrix"])
    return psi


def bind(gates, theta):
    """Parametrised rotations -> fixed rotations with the bound angle."""
    return [Gate(g.name, g.qubits, (g.coeff * theta[g.param],)) if g.param >= 0 else g for g in gates]


CASES = {
    "rqc12": (12, lambda: rqc_u3_cx(12, 10, seed=0)),
    "qft10": (10, lambda: qft(10)),
    "haar11": (11, lambda: dense_haar_layers(11, depth=3, seed=2)),
    "hea8": (8, lambda: bind(hea_vqa(8, 2)[0], vqa_thetas(32, 1, seed=3)[0])),
    "tfim6": (6, lambda: bind(tfim_trotter(6, steps=3), tfim_fields(6, 0))),
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("k_max", [1, 2, 3, 4, 5, 6])
def test_fused_list_reproduces_circuit(case, k_max):
    n, mk = CASES[case]
    gates = mk()
    psi0 = random_state(n, seed=11, workload=9)
    want = oracle.run_circuit(n, gates, psi0)
    fc = cast.FusedCircuit(n, gates, k_max=max(k_max, max(g.k for g in gates)))
    got = replay(fc, n, psi0)
    np.testing.assert_allclose(got, want, atol=1e-12, rtol=0)
    info = fc.info()
    assert info["n_fused"] <= len(gates)
    for i in range(info["n_fused"]):
        g = fc.gate(i)
        assert g["k"] <= max(k_max, max(x.k for x in gates))
        assert list(g["qubits"]) == sorted(g["qubits"])


@pytest.mark.parametrize("agg,multi", [(True, True), (False, True), (True, False), (False, False)])
def test_schedule_options_preserve_unitary(agg, multi):
    n = 9
    gates = qft(n)
    psi0 = random_state(n, seed=1, workload=9)
    want = oracle.run_circuit(n, gates, psi0)
    fc = cast.FusedCircuit(n, gates, k_max=4, agglomerative=agg, multi_traversal=multi)
    np.testing.assert_allclose(replay(fc, n, psi0), want, atol=1e-12, rtol=0)


def test_fusion_compresses_qft():
    n = 12
    counts = [len(cast.FusedCircuit(n, qft(n), k_max=k)) for k in range(1, 6)]
    assert counts[0] == len(qft(n))            # k_max = 1 leaves the QFT unfused
    assert all(a >= b for a, b in zip(counts, counts[1:])), counts
    assert counts[4] < counts[0] / 4, counts


def test_opcount_cap_respected():
    n = 10
    gates = rqc_u3_cx(n, 6, seed=4)
    fc = cast.FusedCircuit(n, gates, k_max=6, opcount_cap=256)
    for i in range(len(fc)):
        assert fc.gate(i)["opcount"] <= 256 or fc.gate(i)["k"] == 1
    psi0 = random_state(n, seed=2, workload=9)
    np.testing.assert_allclose(replay(fc, n, psi0), oracle.run_circuit(n, gates, psi0), atol=1e-12, rtol=0)


def _golden():
    rows = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        name, nnz, ops = line.split()
        rows[name] = (int(nnz), int(ops))
    return rows


def test_opcounts_match_paper_values():
    g = _golden()
    rng = np.random.default_rng(0)
    for k in range(1, 7):
        fc = cast.FusedCircuit(k, [Gate("unitary", tuple(range(k)), matrix=haar_unitary(1 << k, rng))], k_max=k)
        assert fc.gate(0)["opcount"] == g[f"dense_k{k}"][1]
        assert fc.gate(0)["opcount"] == 2 * g[f"dense_k{k}"][0]
        assert g[f"dense_k{k}"][1] == 2 ** (2 * k + 2)
    assert g["dense_k5"][1] == 4096
    for p in "xyz":
        fc = cast.FusedCircuit(1, [Gate(p, (0,))], k_max=1)
        assert fc.gate(0)["opcount"] == g[f"pauli_{p}"][1]


def test_block_structure_of_standard_patterns():
    """Subspace dimension d (dense 2^d x 2^d blocks) and active blocks."""
    def one(gates, n, k):
        fc = cast.FusedCircuit(n, gates, k_max=k)
        assert len(fc) == 1
        return fc.gate(0)
    g = one(gate_sweep("h", 3, (0, 1, 2)), 3, 3)
    assert (g["d"], g["active_blocks"]) == (3, 1)
    g = one(gate_sweep("diag", 4, (0, 1, 2, 3)), 4, 4)
    assert (g["d"], g["active_blocks"]) == (0, 16)
    g = one(gate_sweep("x", 3, (0, 1, 2)), 3, 3)
    assert (g["d"], g["active_blocks"]) == (1, 4)
    g = one(gate_sweep("ctrl", 3, (0, 1, 2)), 3, 3)
    assert (g["d"], g["active_blocks"]) == (1, 1)       # only the all-controls block moves
    g = one([Gate("cz", (0, 1))], 2, 2)
    assert (g["d"], g["active_blocks"]) == (0, 1)
    g = one([Gate("swap", (0, 1))], 2, 2)
    assert (g["d"], g["active_blocks"]) == (1, 1)


def test_unsorted_qubits_and_permuted_matrix():
    n = 7
    rng = np.random.default_rng(9)
    gates = [Gate("unitary", (5, 1, 3), matrix=haar_unitary(8, rng)), Gate("cx", (4, 0)),
             Gate("unitary", (6, 2), matrix=haar_unitary(4, rng))]
    psi0 = random_state(n, seed=3, workload=9)
    for k in (2, 3, 5):
        fc = cast.FusedCircuit(n, gates, k_max=max(k, 3))
        np.testing.assert_allclose(replay(fc, n, psi0), oracle.run_circuit(n, gates, psi0), atol=1e-13, rtol=0)


def test_adaptive_cost_model_reproduces_circuit_and_uses_table():
    n = 8
    gates = rqc_u3_cx(n, 4, seed=5)
    psi0 = random_state(n, seed=6, workload=9)
    want = oracle.run_circuit(n, gates, psi0)
    fc = cast.FusedCircuit(n, gates, k_max=5, cost_model=1)
    np.testing.assert_allclose(replay(fc, n, psi0), want, atol=1e-12, rtol=0)
    # a table that makes dense 2-qubit passes prohibitively slow blocks every
    # fusion that would produce one
    import ctypes
    old = ctypes.c_double()
    cast.cost_table_get(cast.C128, 2, 2, ctypes.byref(old))
    try:
        cast.cost_table_set(cast.C128, 2, 2, 1e9)
        fc2 = cast.FusedCircuit(n, gates, k_max=2, cost_model=1)
        assert all(not (g["k"] == 2 and g["d"] == 2) for g in (fc2.gate(i) for i in range(len(fc2))))
        np.testing.assert_allclose(replay(fc2, n, psi0), want, atol=1e-12, rtol=0)
        fc3 = cast.FusedCircuit(n, gates, k_max=2, cost_model=0)
        assert any(g["k"] == 2 and g["d"] == 2 for g in (fc3.gate(i) for i in range(len(fc3))))
    finally:
        cast.cost_table_set(cast.C128, 2, 2, old.value)


def test_tuning_knobs_roundtrip_and_validation():
    import torch
    for key in cast.TUNING_KEYS:
        v = cast.get_tuning(key, torch.complex64)
        cast.set_tuning(key, v, torch.complex64)
        assert cast.get_tuning(key, torch.complex64) == v
    with pytest.raises(cast.CastError):
        cast.set_tuning("no_such_knob", 1)
    with pytest.raises(cast.CastError):
        cast.set_tuning("direct_ipt", 3)
    with pytest.raises(cast.CastError):
        cast.cost_table_set(cast.C128, 7, 1, 1.0)
