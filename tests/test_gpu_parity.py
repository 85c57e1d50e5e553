"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle,
element by element, on the same seeded inputs.

Bars: max |d amp| <= 1e-12 for complex128 and <= 1e-5 for complex64."""
import math
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

import oracle  # noqa: E402
import paper_2503_19894_amd as cast  # noqa: E402
from circuits import (Gate, PauliTerm, dense_haar_layers, gate_sweep, haar_unitary, hea_vqa, qft,  # noqa: E402
                      random_state, rqc_u3_cx, tfim_fields, tfim_trotter, vqa_hamiltonian, vqa_thetas)

TOL = {torch.complex128: 1e-12, torch.complex64: 1e-5}
DTYPES = [torch.complex128, torch.complex64]


def note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_gpu(n, gates, psi0, dtype, k_max):
    sv = cast.StateVector(n, tensor=torch.tensor(psi0, dtype=dtype, device="cuda"))
    fc = cast.FusedCircuit(n, gates, k_max=k_max)
    sv.apply_circuit(fc)
    return sv.numpy(), fc


def maxerr(a, b):
    return float(np.max(np.abs(np.asarray(a, dtype=np.complex128) - b)))


@pytest.mark.parametrize("dtype", DTYPES, ids=["c128", "c64"])
def test_config1_rqc12_unfused(dtype):
    n = 12
    gates = rqc_u3_cx(n, 10, seed=0)
    want = oracle.run_circuit(n, gates)
    psi0 = np.zeros(1 << n, dtype=np.complex128)
    psi0[0] = 1
    note("rqc12", dtype)
    got, fc = run_gpu(n, gates, psi0, dtype, k_max=1)
    assert len(fc) == 175
    err = maxerr(got, want)
    note("rqc12 err", err)
    assert err <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES, ids=["c128", "c64"])
def test_config1_apply_gate_one_by_one(dtype):
    n = 12
    gates = rqc_u3_cx(n, 10, seed=1)
    want = oracle.run_circuit(n, gates)
    sv = cast.StateVector(n, dtype=dtype)
    for g in gates:
        # the library's own gate table, not the oracle's matrices
        m = cast.std_matrix(g.name, g.params)
        sv.apply_gate(g.qubits, m[..., 0] + 1j * m[..., 1])
    assert maxerr(sv.numpy(), want) <= TOL[dtype]


PLACEMENTS = {
    "low": lambda n, k, rng: tuple(range(k)),
    "high": lambda n, k, rng: tuple(range(n - k, n)),
    "straddle": lambda n, k, rng: tuple(sorted(set([0, 3] + list(range(n - k + 2, n))))[:k]),
    "random": lambda n, k, rng: tuple(int(x) for x in rng.permutation(n)[:k]),
    "window": lambda n, k, rng: tuple(range(5, 5 + k)),
}


@pytest.mark.parametrize("dtype", DTYPES, ids=["c128", "c64"])
@pytest.mark.parametrize("kind", ["haar", "diag", "x", "ctrl", "h", "u3"])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_single_pass_patterns(dtype, kind, k):
    n = 17
    rng = np.random.default_rng(100 * k + len(kind))
    psi0 = random_state(n, seed=k, workload=9)
    for pname, place in PLACEMENTS.items():
        qs = place(n, k, rng)
        if len(set(qs)) != k:
            continue
        gates = gate_sweep(kind, k, qs, seed=k)
        note(f"pattern {kind} k={k} {pname} qubits={qs} {dtype}")
        want = oracle.run_circuit(n, gates, psi0)
        got, fc = run_gpu(n, gates, psi0, dtype, k_max=k)
        # Alg. 1 fuses commuting blocks only in neighbouring qubit cells, so
        # k one-qubit gates on scattered targets may stay several passes
        assert 1 <= len(fc) <= len(gates)
        err = maxerr(got, want)
        assert err <= TOL[dtype], (pname, qs, err)


@pytest.mark.parametrize("dtype", DTYPES, ids=["c128", "c64"])
@pytest.mark.parametrize("n", [1, 2, 3, 5, 6, 7, 9, 11])
def test_small_states(dtype, n):
    gates = rqc_u3_cx(n, 3, seed=n) + qft(n)
    psi0 = random_state(n, seed=n, workload=9)
    want = oracle.run_circuit(n, gates, psi0)
    for k in sorted({1, min(n, 3), min(n, 6)}):
        note(f"small n={n} k_max={k} {dtype}")
        got, _ = run_gpu(n, gates, psi0, dtype, k_max=max(k, 2 if n >= 2 else 1))
        assert maxerr(got, want) <= TOL[dtype]


FUSED = {
    "qft16": (16, lambda: qft(16)),
    "haar16": (16, lambda: dense_haar_layers(16, depth=3, seed=0)),
    "rqc15": (15, lambda: rqc_u3_cx(15, 8, seed=2)),
}


@pytest.mark.parametrize("dtype", DTYPES, ids=["c128", "c64"])
@pytest.mark.parametrize("case", sorted(FUSED))
@pytest.mark.parametrize("k_max", [2, 3, 4, 5, 6])
def test_fused_circuits(dtype, case, k_max):
    n, mk = FUSED[case]
    gates = mk()
    k_max = max(k_max, max(g.k for g in gates))
    psi0 = random_state(n, seed=5, workload=9)
    want = oracle.run_circuit(n, gates, psi0)
    note(f"fused {case} k_max={k_max} {dtype}")
    got, fc = run_gpu(n, gates, psi0, dtype, k_max)
    err = maxerr(got, want)
    note(f"  passes={len(fc)} err={err:.2e}")
    assert err <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES, ids=["c128", "c64"])
@pytest.mark.parametrize("chunk_log", [6, 8, 16])
def test_direct_block_runs(dtype, chunk_log):
    """Direct-kernel passes of gates with several blocks (d = 1, 2, 3 on
    targets at bit 4 and above) under every block-run length, including
    runs clamped to the group count, against the oracle."""
    n = 17
    rng = np.random.default_rng(21)
    gates = []
    for qs, d in (((4, 6, 9, 12, 16), 1), ((5, 7, 8, 15), 2), ((4, 10, 11, 13, 14, 16), 3)):
        k = len(qs)
        u = haar_unitary(1 << d, rng)
        ph = np.exp(1j * rng.uniform(0.1, 6.0, 1 << (k - d)))
        gates.append(Gate("unitary", qs, matrix=np.kron(np.diag(ph), u)))
    psi0 = random_state(n, seed=5, workload=3)
    want = oracle.run_circuit(n, gates, psi0)
    old = cast.get_tuning("direct_chunk_log", dtype)
    cast.set_tuning("direct_chunk_log", chunk_log, dtype)
    try:
        fc = cast.FusedCircuit(n, gates, k_max=1)
        info = [(fc.gate(i)["d"], fc.gate(i)["active_blocks"], fc.pass_info(i, dtype)["kernel"]) for i in range(len(fc))]
        sv = cast.StateVector(n, tensor=torch.tensor(psi0, dtype=dtype, device="cuda"))
        sv.apply_circuit(fc)
        err = float(np.max(np.abs(sv.numpy().astype(np.complex128) - want)))
    finally:
        cast.set_tuning("direct_chunk_log", old, dtype)
    note(f"direct block runs 2^{chunk_log} {dtype}: (d, blocks, kernel) {info} err {err:.2e}")
    assert info == [(1, 16, 0), (2, 4, 0), (3, 8, 0)]
    assert err <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES, ids=["c128", "c64"])
@pytest.mark.parametrize("rot", [1, 3, 7])
def test_direct_rotated_order(dtype, rot):
    """The direct kernel with its iteration order rotated (every target
    height, so small iteration counts clamp the rotation too): fused QFT and
    several-block gates against the oracle."""
    n = 17
    rng = np.random.default_rng(23)
    gates = qft(n)
    for qs, d in (((4, 6, 9, 12, 16), 1), ((5, 7, 8, 15), 2), ((10, 11, 13), 3)):
        k = len(qs)
        u = haar_unitary(1 << d, rng)
        ph = np.exp(1j * rng.uniform(0.1, 6.0, 1 << (k - d)))
        gates.append(Gate("unitary", qs, matrix=np.kron(np.diag(ph), u)))
    psi0 = random_state(n, seed=6, workload=3)
    want = oracle.run_circuit(n, gates, psi0)
    keys = ("direct_rot", "direct_rot_lo", "direct_rot_hi")
    old = {key: cast.get_tuning(key, dtype) for key in keys}
    for key, v in zip(keys, (rot, 0, 34)):
        cast.set_tuning(key, v, dtype)
    try:
        fc = cast.FusedCircuit(n, gates, k_max=4)
        kinds = [p["kernel"] for p in fc.schedule(dtype)]
        sv = cast.StateVector(n, tensor=torch.tensor(psi0, dtype=dtype, device="cuda"))
        sv.apply_circuit(fc)
        err = float(np.max(np.abs(sv.numpy().astype(np.complex128) - want)))
    finally:
        for key, v in old.items():
            cast.set_tuning(key, v, dtype)
    note(f"direct rotation {rot} {dtype}: kernels {kinds} err {err:.2e}")
    assert 0 in kinds
    assert err <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES, ids=["c128", "c64"])
def test_pass_shapes_and_tuner(dtype):
    """Per-pass launch shapes set by hand on every direct pass (rotation,
    block-run length) and every LDS-tile, diagonal and diagonal-run pass
    (rotation, including rotations the host must ignore), and the shapes the
    tuner picks: the same circuit gives bitwise the same state as with the
    knobs' shapes, and matches the oracle."""
    n = 17
    rng = np.random.default_rng(29)
    gates = qft(n)
    for qs, d in (((4, 6, 9, 12, 16), 1), ((5, 7, 8, 15), 2), ((10, 11, 13), 3)):
        k = len(qs)
        u = haar_unitary(1 << d, rng)
        ph = np.exp(1j * rng.uniform(0.1, 6.0, 1 << (k - d)))
        gates.append(Gate("unitary", qs, matrix=np.kron(np.diag(ph), u)))
    psi0 = random_state(n, seed=8, workload=3)
    want = oracle.run_circuit(n, gates, psi0)
    fc = cast.FusedCircuit(n, gates, k_max=4)
    sched = fc.schedule(dtype)
    direct = [i for i, p in enumerate(sched) if p["kernel"] == 0]
    runs = [i for i, p in enumerate(sched) if p["kernel"] in (1, 2, 3, 5, 6)]   # tiles and diagonals
    assert direct and all(any(sched[i]["kernel"] == kk for i in runs) for kk in (1, 3, 6))
    sv = cast.StateVector(n, tensor=torch.tensor(psi0, dtype=dtype, device="cuda"))
    sv.apply_circuit(fc)
    ref = sv.tensor.clone()
    shapes = [(1, 6), (2, 9), (5, 12), (3, 16), (0, 7)]
    for j, i in enumerate(direct):
        fc.set_pass_shape(dtype, i, *shapes[j % len(shapes)])
    assert fc.pass_shape(dtype, direct[0]) == shapes[0]
    run_rots = [1, 3, 6, 7, 12, 4, 2]
    for j, i in enumerate(runs):
        fc.set_pass_shape(dtype, i, run_rots[j % len(run_rots)], -1)
    sv.tensor.copy_(torch.tensor(psi0, dtype=dtype, device="cuda"))
    sv.apply_circuit(fc)
    torch.cuda.synchronize()
    assert torch.equal(sv.tensor, ref)
    # the tuner applies passes to the state it is given; then start again
    for i in direct + runs:
        fc.set_pass_shape(dtype, i, -1, -1)
    before, after = sv.tune_circuit(fc, reps=2)
    chosen = [fc.pass_shape(dtype, i) for i in direct]
    chosen_runs = [fc.pass_shape(dtype, i)[0] for i in runs]
    assert all(r in (-1, 2, 4, 6, 8) for r in chosen_runs), chosen_runs
    sv.tensor.copy_(torch.tensor(psi0, dtype=dtype, device="cuda"))
    sv.apply_circuit(fc)
    torch.cuda.synchronize()
    note(f"pass shapes {dtype}: direct passes {direct}, tuned {chosen}, tiles and diagonals {runs}, tuned {chosen_runs}, "
         f"ms {before:.4f} -> {after:.4f}")
    assert 0 < after <= before
    assert torch.equal(sv.tensor, ref)
    err = float(np.max(np.abs(sv.numpy().astype(np.complex128) - want)))
    assert err <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES, ids=["c128", "c64"])
def test_mfma_pass_rotation(dtype):
    """Rotated unit order of the matrix-core direct passes, in every input
    load mode: shapes set by hand, including rotations the host must ignore
    (at or above the run count's bits), and the shapes the tuner picks give
    bitwise the same state as the knobs' order and match the oracle."""
    n = 17
    rng = np.random.default_rng(37)
    gates = [Gate("unitary", (0, 3, 8, 12, 16), matrix=haar_unitary(32, rng)),
             Gate("unitary", (1, 4, 7, 10, 14, 11),
                  matrix=np.kron(np.diag(np.exp(1j * rng.uniform(0.1, 6.0, 2))), haar_unitary(32, rng))),
             Gate("unitary", (2, 5, 9, 13, 15), matrix=haar_unitary(32, rng)),
             Gate("unitary", (6, 12, 15, 16), matrix=haar_unitary(16, rng)),
             Gate("unitary", (0, 5, 8, 10, 13, 16), matrix=haar_unitary(64, rng))]
    psi0 = random_state(n, seed=9, workload=3)
    want = oracle.run_circuit(n, gates, psi0)
    keep = cast.get_tuning("mfma_prefetch", dtype)
    try:
        for pre in (0, 1, 2):
            cast.set_tuning("mfma_prefetch", pre, dtype)
            fc = cast.FusedCircuit(n, gates, k_max=6)
            sched = fc.schedule(dtype)
            mf = [i for i, p in enumerate(sched) if p["kernel"] == 4]
            assert len(mf) >= 2, sched
            sv = cast.StateVector(n, tensor=torch.tensor(psi0, dtype=dtype, device="cuda"))
            sv.apply_circuit(fc)
            ref = sv.tensor.clone()
            for rots in ((1, 3, 5, 2), (6, 9, 16, 4)):
                for j, i in enumerate(mf):
                    fc.set_pass_shape(dtype, i, rots[j % len(rots)], -1)
                sv.tensor.copy_(torch.tensor(psi0, dtype=dtype, device="cuda"))
                sv.apply_circuit(fc)
                torch.cuda.synchronize()
                assert torch.equal(sv.tensor, ref), rots
            for i in mf:
                fc.set_pass_shape(dtype, i, -1, -1)
            before, after = sv.tune_circuit(fc, reps=2)
            chosen = [fc.pass_shape(dtype, i) for i in mf]
            assert all(c[0] in (-1, 2, 4, 6, 8) for c in chosen), chosen
            sv.tensor.copy_(torch.tensor(psi0, dtype=dtype, device="cuda"))
            sv.apply_circuit(fc)
            torch.cuda.synchronize()
            note(f"matrix-core rotation {dtype} prefetch {pre}: passes {mf}, tuned {chosen}, ms {before:.4f} -> {after:.4f}")
            assert 0 < after <= before
            assert torch.equal(sv.tensor, ref)
            err = float(np.max(np.abs(sv.numpy().astype(np.complex128) - want)))
            assert err <= TOL[dtype]
    finally:
        cast.set_tuning("mfma_prefetch", keep, dtype)


@pytest.mark.parametrize("dtype", DTYPES, ids=["c128", "c64"])
def test_tile_idle_runs_skipped(dtype):
    """LDS-tile passes whose identity blocks are selected by high targets
    (controlled gates with a low target and high controls, a low-target
    block chosen by a high qubit): the tile holds runs of identity blocks
    too, which must come back unchanged; the result matches the oracle."""
    n = 17
    rng = np.random.default_rng(31)
    gates = [gate_sweep("ctrl", 2, (15, 0), seed=1)[0], gate_sweep("ctrl", 3, (12, 16, 1), seed=2)[0],
             Gate("unitary", (0, 1, 13), matrix=np.kron(np.diag([1.0, np.exp(0.7j)]), haar_unitary(4, rng))),
             Gate("unitary", (2, 3, 14, 15), matrix=np.kron(np.diag([1, 1, 1, np.exp(0.3j)]), haar_unitary(4, rng)))]
    psi0 = random_state(n, seed=8, workload=3)
    want = oracle.run_circuit(n, gates, psi0)
    fc = cast.FusedCircuit(n, gates, k_max=1)
    kinds = [fc.pass_info(i, dtype)["kernel"] for i in range(len(fc))]
    sv = cast.StateVector(n, tensor=torch.tensor(psi0, dtype=dtype, device="cuda"))
    sv.apply_circuit(fc)
    err = float(np.max(np.abs(sv.numpy().astype(np.complex128) - want)))
    note(f"tile idle runs {dtype}: kernels {kinds} err {err:.2e}")
    assert set(kinds) == {1}
    assert err <= TOL[dtype]


def test_qft_closed_form_via_fft():
    n = 20
    psi0 = random_state(n, seed=3, workload=2)
    want = np.fft.ifft(psi0) * math.sqrt(1 << n)
    for dtype in DTYPES:
        for k in (1, 3, 5):
            note(f"qft20 k_max={k} {dtype}")
            got, _ = run_gpu(n, qft(n), psi0, dtype, k)
            assert maxerr(got, want) <= TOL[dtype]


def test_bitwise_deterministic():
    n = 18
    psi0 = random_state(n, seed=1, workload=9)
    gates = dense_haar_layers(17, depth=2, seed=1) + qft(17)
    outs = []
    for _ in range(2):
        got, _ = run_gpu(17, gates, psi0[: 1 << 17] / np.linalg.norm(psi0[: 1 << 17]), torch.complex128, 5)
        outs.append(got)
    assert np.array_equal(outs[0], outs[1])


def test_guard_region_untouched():
    n = 16
    buf = torch.full((3 << n,), 7.0 + 3.0j, dtype=torch.complex128, device="cuda")
    psi0 = random_state(n, seed=2, workload=9)
    mid = buf[1 << n: 2 << n]
    mid.copy_(torch.tensor(psi0))
    sv = cast.StateVector(n, tensor=mid)
    fc = cast.FusedCircuit(n, dense_haar_layers(16, 2, seed=3), k_max=6)
    sv.apply_circuit(fc)
    torch.cuda.synchronize()
    h = buf.cpu().numpy()
    assert np.all(h[: 1 << n] == 7.0 + 3.0j) and np.all(h[2 << n:] == 7.0 + 3.0j)


@pytest.mark.parametrize("dtype", DTYPES, ids=["c128", "c64"])
def test_expval(dtype):
    n = 14
    psi0 = random_state(n, seed=4, workload=9)
    rng = np.random.default_rng(4)
    terms = vqa_hamiltonian(n)
    for _ in range(12):
        qs = rng.permutation(n)[: rng.integers(1, 5)]
        terms.append(PauliTerm(float(rng.normal()), tuple((int(q), "XYZ"[rng.integers(3)]) for q in qs)))
    want = oracle.expval(psi0, terms)
    sv = cast.StateVector(n, tensor=torch.tensor(psi0, dtype=dtype, device="cuda"))
    got = sv.expval(terms)
    tol = 1e-12 if dtype == torch.complex128 else 1e-5 * sum(abs(t.coeff) for t in terms)
    assert abs(got - want) <= tol, (got, want)


@pytest.mark.parametrize("dtype", DTYPES, ids=["c128", "c64"])
def test_adjoint_vs_oracle(dtype):
    n = 8
    gates, P = hea_vqa(n, 3)
    theta = vqa_thetas(P, 2, seed=0)[1]
    H = vqa_hamiltonian(n)
    e_want, g_want = oracle.adjoint_grad(n, gates, theta, H)
    init = cast.StateVector(n, dtype=dtype)
    e, g = cast.adjoint(init, gates, theta, H)
    tol = 1e-10 if dtype == torch.complex128 else 5e-4
    note(f"adjoint {dtype}: dE={abs(e - e_want):.2e} dg={np.max(np.abs(g - g_want)):.2e}")
    assert abs(e - e_want) <= tol
    assert np.max(np.abs(g - g_want)) <= tol


def test_adjoint_tfim_shared_params_and_symmetry():
    n = 6
    h = tfim_fields(n, seed=0)
    psi0 = np.full(1 << n, 2 ** (-n / 2), dtype=np.complex128)
    obs = [PauliTerm(1.0, ((0, "Z"),))]
    for conv in ("xx", "zz"):
        gates = tfim_trotter(n, steps=5, dt=0.05, convention=conv)
        e_want, g_want = oracle.adjoint_grad(n, gates, h, obs, psi0)
        init = cast.StateVector(n, tensor=torch.tensor(psi0, device="cuda"))
        e, g = cast.adjoint(init, gates, h, obs)
        assert abs(e - e_want) <= 1e-12 and np.max(np.abs(g - g_want)) <= 1e-12
        if conv == "zz":
            assert abs(e) <= 1e-12 and np.max(np.abs(g)) <= 1e-12


def test_autograd_function():
    n = 6
    gates, P = hea_vqa(n, 2)
    H = vqa_hamiltonian(n)
    theta = torch.tensor(vqa_thetas(P, 3, seed=2), requires_grad=True)
    E = cast.CircuitEnergy.apply(theta, n, gates, H)
    w = torch.tensor([1.0, -2.0, 0.5], dtype=torch.float64)
    (E.cpu() * w).sum().backward()
    for b in range(3):
        e_want, g_want = oracle.adjoint_grad(n, gates, theta[b].detach().numpy(), H)
        assert abs(float(E[b]) - e_want) <= 1e-10
        np.testing.assert_allclose(theta.grad[b].numpy(), w[b].item() * g_want, atol=1e-10)


@pytest.mark.parametrize("sets", [1, 3])
def test_autograd_function_cuda_theta(sets):
    """theta on the GPU: forward and backward keep every tensor on theta's
    device, and theta.grad matches the oracle's adjoint gradient (one set:
    the per-instance path; three sets: the batched program)."""
    n = 6
    gates, P = hea_vqa(n, 2)
    H = vqa_hamiltonian(n)
    th = vqa_thetas(P, sets, seed=4)
    theta = torch.tensor(th if sets > 1 else th[0], device="cuda", requires_grad=True)
    E = cast.CircuitEnergy.apply(theta, n, gates, H)
    assert E.device == theta.device
    w = torch.linspace(1.0, -1.0, max(sets, 1), dtype=torch.float64, device="cuda")[:sets]
    (E * (w if sets > 1 else w[0])).sum().backward()
    assert theta.grad.device == theta.device
    grad = theta.grad.cpu().numpy().reshape(sets, P)
    for b in range(sets):
        e_want, g_want = oracle.adjoint_grad(n, gates, th[b], H)
        got_e = float(E.reshape(-1)[b])
        print(f"autograd cuda theta set {b}: dE {abs(got_e - e_want):.2e}", flush=True)
        assert abs(got_e - e_want) <= 1e-10
        np.testing.assert_allclose(grad[b], float(w[b]) * g_want, atol=1e-10)


def test_apply_gate_concurrent_host_threads():
    """Four host threads, each with its own stream and state, call apply_gate
    at the same time (ctypes releases the GIL): the shared matrix staging
    slots must never hand one thread's buffer to another while its pass is
    pending.  Each state is checked against the oracle."""
    import threading

    n, T, G = 12, 4, 60
    results = [None] * T
    errors = []

    def work(i):
        try:
            rng = np.random.default_rng(900 + i)
            gates = []
            for _ in range(G):
                k = int(rng.integers(1, 4))
                qs = tuple(int(q) for q in rng.permutation(n)[:k])
                gates.append(Gate("unitary", qs, matrix=haar_unitary(1 << k, rng)))
            psi0 = random_state(n, seed=i, workload=8)
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                sv = cast.StateVector(n, tensor=torch.tensor(psi0, device="cuda"))
                for g in gates:
                    sv.apply_gate(g.qubits, g.matrix)
                results[i] = (gates, psi0, sv.numpy())
        except Exception as e:  # reported below, on the main thread
            errors.append(e)

    th = [threading.Thread(target=work, args=(i,)) for i in range(T)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors, errors
    for i, (gates, psi0, got) in enumerate(results):
        err = float(np.max(np.abs(got - oracle.run_circuit(n, gates, psi0))))
        print(f"thread {i}: max |d amp| {err:.2e}", flush=True)
        assert err <= 1e-12


def test_device_byte_cap_accounting():
    """With CAST_MAX_DEVICE_BYTES set (in a child process, since the cap is
    read once), a second state that would exceed the cap fails with
    CAST_ENOMEM, and freeing the first makes room again."""
    import subprocess
    code = ("import ctypes, paper_2503_19894_amd as c\n"
            "a, b = ctypes.c_void_p(), ctypes.c_void_p()\n"
            "c.sv_create(20, c.C128, None, ctypes.byref(a))\n"
            "try:\n"
            "    c.sv_create(20, c.C128, None, ctypes.byref(b))\n"
            "    print('second created')\n"
            "except c.CastError as e:\n"
            "    print('second', e.code)\n"
            "c.sv_destroy(a)\n"
            "c.sv_create(20, c.C128, None, ctypes.byref(b))\n"
            "c.sv_destroy(b)\n"
            "print('third ok')\n")
    env = dict(os.environ, CAST_MAX_DEVICE_BYTES=str(24 << 20))
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    print(r.stdout, r.stderr[-2000:], flush=True)
    assert r.returncode == 0
    assert "second -2" in r.stdout and "third ok" in r.stdout


@pytest.mark.parametrize("dtype", DTYPES, ids=["c128", "c64"])
def test_pooled_scratch_reuse(dtype):
    """adjoint_grad and expval take their scratch from the reuse pool: calls
    that reuse pooled blocks (and calls after pool_trim) give bit-identical
    results, on different state sizes in turn."""
    outs = {}
    for rep in range(3):
        for n in (7, 10):
            gates, P = hea_vqa(n, 2)
            H = vqa_hamiltonian(n)
            th = vqa_thetas(P, 1, seed=n)[0]
            init = cast.StateVector(n, dtype=dtype)
            e, g = cast.adjoint(init, gates, th, H)
            ev = init.expval(H)
            key = (n,)
            if key in outs:
                assert outs[key][0] == e and np.array_equal(outs[key][1], g) and outs[key][2] == ev
            else:
                outs[key] = (e, g.copy(), ev)
        if rep == 1:
            cast.pool_trim()
    for n in (7, 10):
        gates, P = hea_vqa(n, 2)
        ew, gw = oracle.adjoint_grad(n, gates, vqa_thetas(P, 1, seed=n)[0], vqa_hamiltonian(n))
        tol = 1e-10 if dtype == torch.complex128 else 5e-4
        assert abs(outs[(n,)][0] - ew) <= tol and np.max(np.abs(outs[(n,)][1] - gw)) <= tol
