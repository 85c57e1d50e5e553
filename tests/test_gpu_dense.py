"""Dense random circuits (Haar gates on 6- and 5-qubit random subsets, the
MFMA path): full oracle comparison at 22 qubits with the same generator, and
at 32 qubits (complex128, 64 GiB) the product-state closed form after the
first layer plus the circuit-inverse round trip, and one k = 6 and one k = 5
pass checked against the oracle on 2^20 sampled groups."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402
import paper_2503_19894_amd as cast  # noqa: E402
from circuits import Gate, dense_haar_layers, random_state  # noqa: E402


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-12), (torch.complex64, 1e-5)], ids=["c128", "c64"])
def test_dense_haar_22_vs_oracle(dtype, tol):
    n = 22
    gates = dense_haar_layers(n, depth=4, seed=1)
    psi0 = random_state(n, seed=1, workload=3)
    want = oracle.run_circuit(n, gates, psi0)
    sv = cast.StateVector(n, tensor=torch.tensor(psi0, dtype=dtype, device="cuda"))
    fc = cast.FusedCircuit(n, gates, k_max=6)
    kinds = {fc.pass_info(i, dtype)["kernel"] for i in range(len(fc))}
    print(f"dense22 {dtype}: kernels {sorted(kinds)}", flush=True)
    assert kinds & {4, 5}, "expected the MFMA kernels"
    sv.apply_circuit(fc)
    err = float(np.max(np.abs(sv.numpy().astype(np.complex128) - want)))
    print(f"  max |d amp| = {err:.2e}", flush=True)
    assert err <= tol


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-12), (torch.complex64, 1e-5)], ids=["c128", "c64"])
@pytest.mark.parametrize("m3_min_d", [4, 7], ids=["3m_from_d4", "4m_only"])
@pytest.mark.parametrize("prefetch", [0, 1, 2], ids=["stepwise_loads", "prefetch", "next_unit_prefetch"])
def test_dense_mfma_product_forms(dtype, tol, m3_min_d, prefetch):
    """The matrix-core passes with the three-multiplication complex product
    at every block size (d >= 4) and with the four-product form only, on
    direct and LDS-tile placements (the 4-qubit gate on 0, 2, 5, 9 goes to
    the tile kernel), with the direct kernel's inputs loaded one k-step
    ahead, all before the first product, or the next unit's before this
    unit's products, against the oracle."""
    n = 16
    gates = dense_haar_layers(n, depth=2, seed=3)
    gates.append(Gate("unitary", (0, 2, 5, 9), matrix=_haar(16, 5)))
    psi0 = random_state(n, seed=2, workload=3)
    want = oracle.run_circuit(n, gates, psi0)
    old = cast.get_tuning("mfma_3m_min_d", dtype)
    old_pre = cast.get_tuning("mfma_prefetch", dtype)
    cast.set_tuning("mfma_3m_min_d", m3_min_d, dtype)
    cast.set_tuning("mfma_prefetch", prefetch, dtype)
    try:
        sv = cast.StateVector(n, tensor=torch.tensor(psi0, dtype=dtype, device="cuda"))
        fc = cast.FusedCircuit(n, gates, k_max=6)
        kinds = {fc.pass_info(i, dtype)["kernel"] for i in range(len(fc))}
        assert kinds & {4, 5}
        sv.apply_circuit(fc)
        err = float(np.max(np.abs(sv.numpy().astype(np.complex128) - want)))
    finally:
        cast.set_tuning("mfma_3m_min_d", old, dtype)
        cast.set_tuning("mfma_prefetch", old_pre, dtype)
    print(f"dense16 {dtype} 3M from d={m3_min_d} prefetch {prefetch}: kernels {sorted(kinds)} err {err:.2e}", flush=True)
    assert err <= tol


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-12), (torch.complex64, 1e-5)], ids=["c128", "c64"])
@pytest.mark.parametrize("low_tile", [0, 1], ids=["direct", "tile"])
def test_low_target_mfma_placement(dtype, tol, low_tile):
    """Matrix-core passes with a target below bit 4: two 5-qubit gates made
    of two 16-dimensional blocks (Haar on four targets times a phase on the
    fifth; contiguous low targets, and low targets plus two high ones) and a
    single-block 4-qubit gate, on the direct gather (mfma_low_tile 0) and on
    the LDS tile (1), against the oracle."""
    n = 18
    rng = np.random.default_rng(11)
    ph = np.exp(1j * rng.uniform(0, 2 * np.pi, 2))
    two_blocks = np.kron(np.diag(ph), _haar(16, 12))
    gates = [Gate("unitary", (0, 1, 2, 3, 4), matrix=two_blocks),
             Gate("unitary", (0, 1, 2, 16, 17), matrix=np.kron(np.diag(ph[::-1]), _haar(16, 13))),
             Gate("unitary", (1, 2, 3, 6), matrix=_haar(16, 14))]
    psi0 = random_state(n, seed=4, workload=3)
    want = oracle.run_circuit(n, gates, psi0)
    old = cast.get_tuning("mfma_low_tile", dtype)
    cast.set_tuning("mfma_low_tile", low_tile, dtype)
    try:
        fc = cast.FusedCircuit(n, gates, k_max=1)   # each gate its own pass
        info = [(fc.gate(i)["d"], fc.gate(i)["active_blocks"], fc.pass_info(i, dtype)["kernel"]) for i in range(len(fc))]
        sv = cast.StateVector(n, tensor=torch.tensor(psi0, dtype=dtype, device="cuda"))
        sv.apply_circuit(fc)
        err = float(np.max(np.abs(sv.numpy().astype(np.complex128) - want)))
    finally:
        cast.set_tuning("mfma_low_tile", old, dtype)
    print(f"low-target mfma {dtype} low_tile={low_tile}: (d, blocks, kernel) {info} err {err:.2e}", flush=True)
    assert [i[:2] for i in info] == [(4, 2), (4, 2), (4, 1)]
    assert {i[2] for i in info} == ({5} if low_tile else {4})
    assert err <= tol


def _haar(dim, seed):
    from circuits import haar_unitary
    return haar_unitary(dim, np.random.default_rng(seed))


def _column0(g):
    return np.asarray(g.matrix, dtype=np.complex128)[:, 0]


def test_dense_haar_32_first_layer_and_inverse():
    n = 32
    gates = dense_haar_layers(n, depth=20, seed=0)
    first = gates[:6]
    assert sorted(q for g in first for q in g.qubits) == list(range(n))
    psi = torch.zeros(1 << n, dtype=torch.complex128, device="cuda")
    psi[0] = 1
    sv = cast.StateVector(n, tensor=psi)
    print("dense32: first layer", flush=True)
    sv.apply_circuit(cast.FusedCircuit(n, first, k_max=6))
    torch.cuda.synchronize()
    # product state: amp(x) = prod over gates of U_g[j_g(x)][0], j_g(x) = bits of x on the gate's qubits
    rng = np.random.default_rng(32)
    xs = [0, (1 << n) - 1] + [int(v) for v in rng.integers(0, 1 << n, 30)]
    got = psi[torch.tensor(xs, device="cuda")].cpu().numpy()
    for x, a in zip(xs, got):
        want = 1.0 + 0j
        for g in first:
            j = sum(((x >> q) & 1) << i for i, q in enumerate(g.qubits))
            want *= _column0(g)[j]
        assert abs(a - want) <= 1e-13, (x, a, want)
    print("dense32: remaining layers and the inverse", flush=True)
    sv.apply_circuit(cast.FusedCircuit(n, gates[6:], k_max=6))
    inv = [Gate("unitary", g.qubits, matrix=np.asarray(g.matrix).conj().T) for g in reversed(gates)]
    sv.apply_circuit(cast.FusedCircuit(n, inv, k_max=6))
    torch.cuda.synchronize()
    err0 = abs(complex(psi[0].item()) - 1.0)
    psi[0] = 0
    rest = float(psi.abs().max())
    print(f"  |psi[0] - 1| = {err0:.2e}, max |other| = {rest:.2e}", flush=True)
    assert err0 <= 1e-12 and rest <= 1e-12


@pytest.mark.timeout(900)
def test_dense_haar_32_sampled_groups_vs_oracle():
    """One k = 6 and one k = 5 Haar pass of the 32-qubit dense circuit (the
    matrix-core kernels at the benchmarked size, 64 GiB complex128), each
    applied to the same seeded random input state; 2^20 random groups of the
    output are compared with the oracle's Eq. 3 on those groups, computed in
    FP64 on the host from a copy of the input."""
    from circuits import random_state_torch
    from tests.group_members import member_indices

    n = 32
    gates = dense_haar_layers(n, depth=20, seed=0)
    layer = gates[18:24]
    picks = [next(g for g in layer if len(g.qubits) == 6), next(g for g in layer if len(g.qubits) == 5)]
    rng = np.random.default_rng(3232)
    host = None
    for g in picks:
        k = len(g.qubits)
        print(f"dense32 sampled: k={k} on {g.qubits}: seeded input", flush=True)
        psi = random_state_torch(n, seed=7, device="cuda", dtype=torch.complex128, workload=3)
        if host is None:
            print("  copying the input to the host", flush=True)
            host = psi.cpu().numpy()
        fc = cast.FusedCircuit(n, [g], k_max=1)
        assert len(fc) == 1
        kind = fc.pass_info(0, torch.complex128)["kernel"]
        assert kind in (4, 5), kind
        cast.StateVector(n, tensor=psi).apply_circuit(fc)
        torch.cuda.synchronize()
        groups = rng.integers(0, 1 << (n - k), 1 << 20)
        idx = member_indices(n, g.qubits, groups)
        got = psi[torch.from_numpy(idx.reshape(-1)).to("cuda")].cpu().numpy().reshape(idx.shape)
        del psi
        want = oracle.apply_gate_groups(host, g.qubits, np.asarray(g.matrix), groups)
        err = float(np.max(np.abs(got - want)))
        print(f"  kernel {kind}: max |d amp| over {groups.size} groups: {err:.2e}", flush=True)
        assert err <= 1e-12
