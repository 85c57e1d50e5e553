"""Diagonal runs on the GPU against the oracle: apply_circuit merges runs of
consecutive diagonal fused gates into one elementwise pass.  Sweeps the
run knobs (tables per pass, qubits per table, chunks per thread, grid cap)
over circuits rich in diagonals, state sizes below, at and above one tile,
and both dtypes; the oracle applies the unfused gates one by one."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402
import paper_2503_19894_amd as cast  # noqa: E402
from circuits import Gate, iqp, qft, random_state  # noqa: E402

TOL = {torch.complex128: 1e-12, torch.complex64: 1e-5}
KEYS = ("diag_run_tables", "diag_run_qubits", "diag_run_unroll", "diag_run_grid", "diag_run_lds", "diag_run_reuse")


@pytest.fixture
def knobs():
    old = {(k, d): cast.get_tuning(k, d) for k in KEYS for d in (torch.complex128, torch.complex64)}
    yield
    for (k, d), v in old.items():
        cast.set_tuning(k, v, d)


def _mixed(n, seed):
    """Layers of H on a few qubits, then many controlled phases and random
    diagonals on scattered qubits (entries exactly 1 included)."""
    rng = np.random.default_rng(seed)
    gates = []
    for _ in range(3):
        gates += [Gate("h", (int(q),)) for q in rng.permutation(n)[:3]]
        for _ in range(12):
            a, b = (int(q) for q in rng.permutation(n)[:2])
            gates.append(Gate("cp", (a, b), (float(rng.uniform(0, 2 * np.pi)),)))
        for _ in range(4):
            k = int(rng.integers(1, 4))
            qs = tuple(int(q) for q in rng.permutation(n)[:k])
            ph = np.exp(1j * rng.uniform(0, 2 * np.pi, 1 << k))
            ph[rng.permutation(1 << k)[:1]] = 1.0
            gates.append(Gate("unitary", qs, matrix=np.diag(ph)))
    return gates


CIRCUITS = {"qft": lambda n: qft(n), "iqp": lambda n: iqp(n, seed=3), "mixed": lambda n: _mixed(n, 5)}


def _run(n, gates, dtype, k_max):
    psi0 = random_state(n, seed=n, workload=8)
    want = oracle.run_circuit(n, gates, psi0)
    fc = cast.FusedCircuit(n, gates, k_max=k_max)
    sched = fc.schedule(dtype)
    sv = cast.StateVector(n, tensor=torch.tensor(psi0, dtype=dtype, device="cuda"))
    sv.apply_circuit(fc)
    err = float(np.max(np.abs(sv.numpy().astype(np.complex128) - want)))
    return err, sched, len(fc)


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64], ids=["c128", "c64"])
@pytest.mark.parametrize("circ", sorted(CIRCUITS))
@pytest.mark.parametrize("n", [3, 7, 11, 16])
def test_runs_vs_oracle(knobs, dtype, circ, n):
    gates = CIRCUITS[circ](n)
    err, sched, nf = _run(n, gates, dtype, k_max=3)
    runs = sum(p["kernel"] == 6 for p in sched)
    print(f"{circ} n={n} {dtype}: {nf} fused -> {len(sched)} passes ({runs} runs), max |d amp| {err:.2e}",
          flush=True)
    assert err <= TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64], ids=["c128", "c64"])
@pytest.mark.parametrize("tables,qubits,unroll,grid,lds,reuse", [
    (1, 8, 1, 256, 1, 0), (2, 4, 2, 4096, 1, 0), (2, 8, 4, 256, 0, 0), (3, 6, 1, 1 << 20, 0, 0),
    (4, 8, 2, 4096, 0, 0), (4, 5, 4, 1 << 20, 1, 0), (3, 8, 1, 1 << 24, 0, 0), (4, 8, 2, 1 << 24, 1, 0),
    (1, 8, 1, 256, 1, 1), (2, 4, 2, 4096, 0, 2), (3, 8, 4, 1 << 16, 1, 4), (4, 8, 1, 1 << 20, 0, 4),
    (4, 6, 2, 256, 1, 12), (2, 8, 4, 1 << 24, 0, 12)])
def test_run_knobs_vs_oracle(knobs, dtype, tables, qubits, unroll, grid, lds, reuse):
    """Each knob setting against the oracle; reuse = 0 is the tiled run
    kernel, reuse > 0 the phase-reuse kernel (F patterns per unit)."""
    for key, v in zip(KEYS, (tables, qubits, unroll, grid, lds, reuse)):
        cast.set_tuning(key, v, dtype)
    runs = 0
    for circ in sorted(CIRCUITS):
        for n in (9, 17):
            gates = CIRCUITS[circ](n)
            err, sched, nf = _run(n, gates, dtype, k_max=4)
            runs += sum(p["kernel"] == 6 for p in sched)
            assert max(p["tables"] for p in sched) <= tables
            print(f"knobs {tables}/{qubits}/{unroll}/{grid}/{lds}/{reuse} {circ} n={n} {dtype}: {len(sched)} passes, "
                  f"max |d amp| {err:.2e}", flush=True)
            assert err <= TOL[dtype]
    assert runs > 0


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64], ids=["c128", "c64"])
def test_runs_on_and_off_agree(knobs, dtype):
    """The same fused list with runs and with one pass per fused gate."""
    n = 18
    gates = qft(n) + _mixed(n, 9)
    fc = cast.FusedCircuit(n, gates, k_max=5)
    psi0 = torch.tensor(random_state(n, seed=1, workload=8), dtype=dtype, device="cuda")
    outs = []
    for tables in (0, 4):
        cast.set_tuning("diag_run_tables", tables, dtype)
        x = psi0.clone()
        cast.StateVector(n, tensor=x).apply_circuit(fc)
        torch.cuda.synchronize()
        outs.append(x)
    d = float((outs[0] - outs[1]).abs().max())
    print(f"runs on/off {dtype}: max |d amp| {d:.2e}", flush=True)
    assert d <= TOL[dtype]
