"""Batched adjoint gradients (many parameter sets, mixed qubit counts) on the
GPU against the oracle's adjoint gradient, per instance."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402
import paper_2503_19894_amd as cast  # noqa: E402
from circuits import PauliTerm, hea_vqa, tfim_fields, tfim_trotter, vqa_hamiltonian, vqa_thetas  # noqa: E402

MODES = [cast.BATCH_STEPS, cast.BATCH_STEPS_GRAPH, cast.BATCH_PERSISTENT_GRAPH]
TOL = {torch.complex128: 1e-10, torch.complex64: 5e-4}


def vqa_case(n=8, layers=3, sets=5, seed=0):
    gates, P = hea_vqa(n, layers)
    return gates, P, vqa_thetas(P, sets, seed=seed), vqa_hamiltonian(n)


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64], ids=["c128", "c64"])
@pytest.mark.parametrize("mode", MODES, ids=["steps", "graph", "persistent"])
def test_vqa_batch_vs_oracle(dtype, mode):
    n = 8
    gates, P, th, H = vqa_case(n)
    B = th.shape[0]
    print(f"vqa batch n={n} B={B} mode={mode} {dtype}", flush=True)
    b = cast.Batch([gates] * B, [n] * B, [P] * B, [H] * B, dtype=dtype, mode=mode)
    e, g = b.run(list(th))
    for i in range(B):
        ew, gw = oracle.adjoint_grad(n, gates, th[i], H)
        assert abs(e[i] - ew) <= TOL[dtype], (i, e[i], ew)
        assert np.max(np.abs(g[i] - gw)) <= TOL[dtype]


def test_modes_bitwise_identical_and_replay():
    n = 9
    gates, P, th, H = vqa_case(n, layers=2, sets=4, seed=1)
    B = th.shape[0]
    outs = []
    for mode in MODES:
        b = cast.Batch([gates] * B, [n] * B, [P] * B, [H] * B, mode=mode)
        outs.append(b.run(list(th)))
        # replay with other parameters, then the original ones again
        b.run(list(vqa_thetas(P, B, seed=7)))
        e2, g2 = b.run(list(th))
        assert np.array_equal(e2, outs[-1][0])
        assert all(np.array_equal(x, y) for x, y in zip(g2, outs[-1][1]))
    for e, g in outs[1:]:
        assert np.array_equal(e, outs[0][0])
        assert all(np.array_equal(x, y) for x, y in zip(g, outs[0][1]))


@pytest.mark.parametrize("mode", MODES, ids=["steps", "graph", "persistent"])
def test_mixed_sizes_tfim(mode):
    ns = [4, 4, 6, 6, 8, 9]
    circs, fields, obs = [], [], [PauliTerm(1.0, ((0, "Z"),))]
    for i, n in enumerate(ns):
        circs.append(tfim_trotter(n, steps=4, dt=0.05))
        fields.append(tfim_fields(n, seed=i))
    print(f"mixed tfim mode={mode}", flush=True)
    b = cast.Batch(circs, ns, ns, [obs] * len(ns), init=["plus"] * len(ns), mode=mode)
    e, g = b.run(fields)
    for i, n in enumerate(ns):
        psi0 = np.full(1 << n, 2 ** (-n / 2), dtype=np.complex128)
        ew, gw = oracle.adjoint_grad(n, circs[i], fields[i], obs, psi0)
        assert abs(e[i] - ew) <= 1e-11
        assert np.max(np.abs(g[i] - gw)) <= 1e-11


def test_batch_larger_states_cross_workgroups():
    """n above the single-workgroup size: an op spans several work items."""
    n = 16
    gates, P = hea_vqa(n, 1)
    th = vqa_thetas(P, 2, seed=3)
    H = vqa_hamiltonian(n)
    for mode in MODES:
        b = cast.Batch([gates] * 2, [n] * 2, [P] * 2, [H] * 2, mode=mode)
        e, g = b.run(list(th))
        for i in range(2):
            ew, gw = oracle.adjoint_grad(n, gates, th[i], H)
            assert abs(e[i] - ew) <= 1e-10
            assert np.max(np.abs(g[i] - gw)) <= 1e-10


def test_persistent_pairs_bitwise_and_vs_oracle():
    """Paired forward items of the persistent launch (two tiles of one record
    in one workgroup), with records that start at odd item offsets (a
    one-item instance before each large one) and claims that end between
    the two items of a would-be pair: bitwise equal to the per-step launch
    (which never pairs) and within the bar of the oracle."""
    ns = [4, 14, 5, 14]
    obs = [PauliTerm(1.0, ((0, "Z"),)), PauliTerm(0.5, ((1, "X"),))]
    circs = [tfim_trotter(n, steps=3, dt=0.07) for n in ns]
    fields = [tfim_fields(n, seed=20 + i) for i, n in enumerate(ns)]
    outs = {}
    for mode in (cast.BATCH_STEPS, cast.BATCH_PERSISTENT_GRAPH):
        b = cast.Batch(circs, ns, ns, [obs] * len(ns), init=["plus"] * len(ns), mode=mode)
        outs[mode] = b.run(fields)
    e0, g0 = outs[cast.BATCH_STEPS]
    e1, g1 = outs[cast.BATCH_PERSISTENT_GRAPH]
    assert np.array_equal(e0, e1)
    assert all(np.array_equal(x, y) for x, y in zip(g0, g1))
    for i, n in enumerate(ns):
        psi0 = np.full(1 << n, 2 ** (-n / 2), dtype=np.complex128)
        ew, gw = oracle.adjoint_grad(n, circs[i], fields[i], obs, psi0)
        assert abs(e1[i] - ew) <= 1e-10
        assert np.max(np.abs(g1[i] - gw)) <= 1e-10


def test_init_state_copy():
    n = 7
    gates, P, th, H = vqa_case(n, layers=1, sets=2)
    rng = np.random.default_rng(0)
    psi0 = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi0 /= np.linalg.norm(psi0)
    sv = cast.StateVector(n, tensor=torch.tensor(psi0, device="cuda"))
    b = cast.Batch([gates] * 2, [n] * 2, [P] * 2, [H] * 2, init=[sv, "zero"])
    e, g = b.run(list(th))
    ew, gw = oracle.adjoint_grad(n, gates, th[0], H, psi0)
    assert abs(e[0] - ew) <= 1e-10 and np.max(np.abs(g[0] - gw)) <= 1e-10
    ew, gw = oracle.adjoint_grad(n, gates, th[1], H)
    assert abs(e[1] - ew) <= 1e-10 and np.max(np.abs(g[1] - gw)) <= 1e-10


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64], ids=["c128", "c64"])
def test_two_qubit_generators_unsorted_and_high_qubits(dtype):
    """Parametrised XX / YY / ZZ rotations (Y phases, two-letter generators),
    unsorted qubit lists and gates reaching the top qubits, across several
    segments and sweeps."""
    from circuits import Gate
    n = 13
    rng = np.random.default_rng(11)
    gates = []
    for layer in range(3):
        for q in rng.permutation(n):
            gates.append(Gate(["rx", "ry", "rz"][int(rng.integers(3))], (int(q),), param=len(gates),
                              coeff=float(rng.uniform(0.5, 1.5))))
        for i in range(n):
            a, b = int(rng.integers(n)), int(rng.integers(n))
            if a == b:
                continue
            gates.append(Gate(["rxx", "ryy", "rzz"][(i + layer) % 3], (a, b), param=len(gates), coeff=-0.7))
        gates.append(Gate("cz", (n - 1, 2)))
        gates.append(Gate("cx", (n - 2, 0)))
    P = len(gates)
    thetas = [rng.uniform(-np.pi, np.pi, P) for _ in range(3)]
    H = [PauliTerm(0.9, ((0, "Y"), (n - 1, "X"))), PauliTerm(-0.4, ((5, "Z"), (7, "Z"))), PauliTerm(0.3, ((11, "Y"),))]
    tol = TOL[dtype]
    for mode in MODES:
        b = cast.Batch([gates] * 3, [n] * 3, [P] * 3, [H] * 3, dtype=dtype, mode=mode)
        e, g = b.run(thetas)
        for i in range(3):
            ew, gw = oracle.adjoint_grad(n, gates, thetas[i], H)
            assert abs(e[i] - ew) <= tol, (mode, i)
            assert np.max(np.abs(g[i] - gw)) <= tol, (mode, i, np.max(np.abs(g[i] - gw)))


def test_persistent_wait_bound_error_path():
    """The persistent launch's bounded dependency wait, forced to give up from
    the host (spin limit 0: every item with a dependency fails at once): the
    run returns CAST_EHIP with its message, every workgroup exits, and a batch
    built afterwards with the normal limit runs and matches the oracle."""
    n = 6
    gates, P, th, H = vqa_case(n, layers=2, sets=3, seed=5)
    B = th.shape[0]
    dt = torch.complex128
    old = cast.get_tuning("persistent_spin_limit", dt)
    cast.set_tuning("persistent_spin_limit", 0, dt)
    try:
        b = cast.Batch([gates] * B, [n] * B, [P] * B, [H] * B, dtype=dt, mode=cast.BATCH_PERSISTENT_GRAPH)
        with pytest.raises(cast.CastError) as ei:
            b.run(list(th))
        print(f"forced wait failure: code {ei.value.code}, {cast.last_error()}", flush=True)
        assert ei.value.code == -3 and "exceeded its bound" in cast.last_error()
        del b
    finally:
        cast.set_tuning("persistent_spin_limit", old, dt)
    torch.cuda.synchronize()
    b = cast.Batch([gates] * B, [n] * B, [P] * B, [H] * B, dtype=dt, mode=cast.BATCH_PERSISTENT_GRAPH)
    e, g = b.run(list(th))
    for i in range(B):
        ew, gw = oracle.adjoint_grad(n, gates, th[i], H)
        assert abs(e[i] - ew) <= TOL[dt]
        assert np.max(np.abs(g[i] - gw)) <= TOL[dt]
