"""Generated (immediate-valued) kernels on the GPU against the FP64 oracle's
unfused run.  Bars: max |d amp| <= 1e-12 (complex128), <= 1e-5 (complex64)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402
import paper_2503_19894_amd as cast  # noqa: E402
from circuits import dense_haar_layers, gate_sweep, qft, random_state, rqc_u3_cx  # noqa: E402
from tests.blocked_cases import mixed_circuit  # noqa: E402

TOL = {torch.complex128: 1e-12, torch.complex64: 1e-5}
CASES = {
    "qft16": (16, lambda: qft(16)),
    "rqc15": (15, lambda: rqc_u3_cx(15, 5, seed=4)),
    "mixed15": (15, lambda: mixed_circuit(15, seed=6)),
    "haar16": (16, lambda: dense_haar_layers(16, depth=2, seed=2)),
    "h3": (15, lambda: gate_sweep("h", 3, (1, 7, 12))),
    "ctrl4": (15, lambda: gate_sweep("ctrl", 4, (0, 5, 9, 14), seed=3)),
}


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64], ids=["c128", "c64"])
@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("k_max", [2, 4, 6])
def test_jit_vs_oracle(dtype, case, k_max):
    n, mk = CASES[case]
    gates = mk()
    k_max = max(k_max, max(g.k for g in gates))
    psi0 = random_state(n, seed=31, workload=9)
    want = oracle.run_circuit(n, gates, psi0)
    fc = cast.FusedCircuit(n, gates, k_max=k_max)
    sv = cast.StateVector(n, tensor=torch.tensor(psi0, dtype=dtype, device="cuda"))
    sv.apply_circuit_jit(fc)
    err = float(np.max(np.abs(sv.numpy().astype(np.complex128) - want)))
    print(f"jit {case} k_max={k_max} {dtype}: {len(fc)} fused, err {err:.2e}", flush=True)
    assert err <= TOL[dtype]


def test_jit_timed_matches_and_replays():
    n, dtype = 15, torch.complex128
    gates = mixed_circuit(n, seed=9)
    psi0 = random_state(n, seed=32, workload=9)
    want = oracle.run_circuit(n, gates + gates, psi0)
    fc = cast.FusedCircuit(n, gates, k_max=3)
    sv = cast.StateVector(n, tensor=torch.tensor(psi0, dtype=dtype, device="cuda"))
    sv.apply_circuit_jit(fc)
    ms = sv.apply_circuit_jit_timed(fc)
    assert len(ms) == len(fc) and np.all(ms >= 0)
    assert float(np.max(np.abs(sv.numpy() - want))) <= TOL[dtype]
