"""Cache-blocked execution (several fused gates per HBM pass, one LDS tile
per workgroup) on the GPU against the FP64 oracle's unfused run, element by
element, and against the one-pass-per-gate path.

Bars: max |d amp| <= 1e-12 for complex128 and <= 1e-5 for complex64."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402
import paper_2503_19894_amd as cast  # noqa: E402
from circuits import dense_haar_layers, qft, random_state, rqc_u3_cx  # noqa: E402
from tests.blocked_cases import mixed_circuit  # noqa: E402

TOL = {torch.complex128: 1e-12, torch.complex64: 1e-5}
DTYPES = [torch.complex128, torch.complex64]


def note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


class tile_bits:
    """Sets the blocked tile size for one dtype, restoring it afterwards."""

    def __init__(self, dtype, bits):
        self.dtype, self.bits = dtype, bits

    def __enter__(self):
        self.old = cast.get_tuning("blocked_tile_bits", self.dtype)
        if self.bits:
            cast.set_tuning("blocked_tile_bits", self.bits, self.dtype)

    def __exit__(self, *exc):
        cast.set_tuning("blocked_tile_bits", self.old, self.dtype)


def run_blocked(n, fc, psi0, dtype):
    sv = cast.StateVector(n, tensor=torch.tensor(psi0, dtype=dtype, device="cuda"))
    sv.apply_circuit_blocked(fc)
    return sv.numpy()


def maxerr(a, b):
    return float(np.max(np.abs(np.asarray(a, dtype=np.complex128) - b)))


CASES = {
    "qft16": (16, lambda: qft(16)),
    "rqc15": (15, lambda: rqc_u3_cx(15, 6, seed=3)),
    "mixed16": (16, lambda: mixed_circuit(16, seed=4)),
    "mixed13": (13, lambda: mixed_circuit(13, seed=5)),
    "haar16": (16, lambda: dense_haar_layers(16, depth=2, seed=1)),
}


@pytest.mark.parametrize("dtype", DTYPES, ids=["c128", "c64"])
@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("k_max", [2, 3, 5])
@pytest.mark.parametrize("bits", [8, 10, 0], ids=["tb8", "tb10", "tbdefault"])
def test_blocked_vs_oracle(dtype, case, k_max, bits):
    n, mk = CASES[case]
    gates = mk()
    k_max = max(k_max, max(g.k for g in gates))
    psi0 = random_state(n, seed=7, workload=9)
    want = oracle.run_circuit(n, gates, psi0)
    fc = cast.FusedCircuit(n, gates, k_max=k_max)
    with tile_bits(dtype, bits):
        passes = fc.blocked_passes(dtype)
        note(f"blocked {case} k_max={k_max} tb={bits or 'default'} {dtype}: {len(fc)} fused -> {len(passes)} passes")
        got = run_blocked(n, fc, psi0, dtype)
    err = maxerr(got, want)
    note(f"  err={err:.2e}")
    assert err <= TOL[dtype]
    assert len(passes) <= len(fc)


@pytest.mark.parametrize("dtype", DTYPES, ids=["c128", "c64"])
def test_blocked_matches_per_pass_path(dtype):
    n = 17
    gates = qft(n) + mixed_circuit(n, seed=8)
    psi0 = random_state(n, seed=9, workload=9)
    fc = cast.FusedCircuit(n, gates, k_max=4)
    a = cast.StateVector(n, tensor=torch.tensor(psi0, dtype=dtype, device="cuda"))
    a.apply_circuit(fc)
    b = run_blocked(n, fc, psi0, dtype)
    assert maxerr(a.numpy(), b) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES, ids=["c128", "c64"])
@pytest.mark.parametrize("n", [9, 12, 13, 14])
def test_blocked_single_tile_and_small_states(dtype, n):
    """n below the tile size (every pass ordinary), equal to it (one tile)
    and just above it."""
    gates = qft(n) + mixed_circuit(n, seed=n)
    psi0 = random_state(n, seed=n, workload=9)
    want = oracle.run_circuit(n, gates, psi0)
    fc = cast.FusedCircuit(n, gates, k_max=3)
    note(f"blocked small n={n} {dtype}: {len(fc.blocked_passes(dtype))} passes")
    assert maxerr(run_blocked(n, fc, psi0, dtype), want) <= TOL[dtype]


def test_blocked_replay_and_timed():
    """Applying twice equals the oracle's circuit twice; the timed variant
    gives one positive time per pass and the same state."""
    n, dtype = 16, torch.complex128
    gates = mixed_circuit(n, seed=11)
    psi0 = random_state(n, seed=12, workload=9)
    want = oracle.run_circuit(n, gates + gates, psi0)
    fc = cast.FusedCircuit(n, gates, k_max=3)
    sv = cast.StateVector(n, tensor=torch.tensor(psi0, dtype=dtype, device="cuda"))
    sv.apply_circuit_blocked(fc)
    ms = sv.apply_circuit_blocked_timed(fc)
    assert len(ms) == len(fc.blocked_passes(dtype)) and np.all(ms > 0)
    assert maxerr(sv.numpy(), want) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES, ids=["c128", "c64"])
@pytest.mark.parametrize("threads", [256, 1024])
def test_blocked_workgroup_sizes(dtype, threads):
    """The segment kernel's 256- and 1024-thread instances (both block-size
    instances: the circuit has 3-qubit Haar gates) against the oracle."""
    n = 15
    gates = mixed_circuit(n, seed=13)
    psi0 = random_state(n, seed=14, workload=9)
    want = oracle.run_circuit(n, gates, psi0)
    fc = cast.FusedCircuit(n, gates, k_max=3)
    assert any(fc.gate(i)["d"] == 3 for i in range(len(fc)))
    old = cast.get_tuning("blocked_threads", dtype)
    cast.set_tuning("blocked_threads", threads, dtype)
    try:
        got = run_blocked(n, fc, psi0, dtype)
    finally:
        cast.set_tuning("blocked_threads", old, dtype)
    assert maxerr(got, want) <= TOL[dtype]
