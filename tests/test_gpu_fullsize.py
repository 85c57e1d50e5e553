"""Parity at the benchmarked size: QFT on 30 qubits, fused with k_max = 5,
in the launch configuration bench.py times.

The full state is far too large for the oracle's replay, so the checks are
(1) sampled outputs against the DFT closed form (a property of the QFT at any
size, pinned against numpy.fft in tests/test_dft_helper.py), (2) the fused
inverse QFT returning the input, amplitude by amplitude, and (3) the whole
output state against sqrt(N) times a library inverse FFT of the input."""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2503_19894_amd as cast  # noqa: E402
from circuits import Gate, qft, random_state_torch  # noqa: E402
from tests.dft_closed_form import qft_output  # noqa: E402

N_QUBITS = 30


def inverse_qft(n):
    inv = []
    for g in reversed(qft(n)):
        inv.append(Gate(g.name, g.qubits, tuple(-p for p in g.params)))
    return inv


@pytest.mark.parametrize("mode", ["per_pass", "blocked"])
@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-12), (torch.complex64, 1e-5)], ids=["c128", "c64"])
def test_qft30_closed_form_and_inverse(dtype, tol, mode):
    n = N_QUBITS
    print(f"qft{n} {dtype} {mode}: generating input", flush=True)
    psi = random_state_torch(n, seed=0, device="cuda", dtype=dtype)
    psi0 = psi.cpu().numpy().astype(np.complex128)
    sv = cast.StateVector(n, tensor=psi)
    fc = cast.FusedCircuit(n, qft(n), k_max=5)
    apply = sv.apply_circuit if mode == "per_pass" else sv.apply_circuit_blocked
    print(f"  {len(fc)} fused gates; applying", flush=True)
    apply(fc)
    torch.cuda.synchronize()
    rng = np.random.default_rng(30)
    ys = [0, 1, (1 << n) - 1] + [int(y) for y in rng.integers(0, 1 << n, 2)]
    got = psi[torch.tensor(ys, device="cuda")].cpu().numpy().astype(np.complex128)
    for y, g in zip(ys, got):
        want = qft_output(psi0, y)
        print(f"  y={y}: |d| = {abs(g - want):.2e}", flush=True)
        assert abs(g - want) <= tol
    print("  inverse", flush=True)
    inv = cast.FusedCircuit(n, inverse_qft(n), k_max=5)
    apply(inv)
    torch.cuda.synchronize()
    err = float((psi.to(torch.complex128) - torch.from_numpy(psi0).to("cuda")).abs().max())
    print(f"  max |d amp| after QFT^-1 QFT: {err:.2e}", flush=True)
    assert err <= tol
    nrm = float(torch.linalg.vector_norm(psi.to(torch.complex128)))
    assert abs(nrm - 1.0) <= tol


@pytest.mark.timeout(900)
@pytest.mark.parametrize("mode", ["per_pass", "blocked"])
@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-12), (torch.complex64, 1e-5)], ids=["c128", "c64"])
def test_qft30_full_state_vs_fft(dtype, tol, mode):
    """Every one of the 2^30 outputs against the DFT closed form: with the gate
    order used here the QFT maps psi to sqrt(N) * ifft(psi) (a library FFT,
    independent of this library), evaluated in FP64 on the device."""
    n = N_QUBITS
    N = 1 << n
    print(f"qft{n} full state {dtype} {mode}: input and FP64 FFT", flush=True)
    psi = random_state_torch(n, seed=3, device="cuda", dtype=dtype)
    ref = torch.fft.ifft(psi.to(torch.complex128))
    ref.mul_(math.sqrt(N))
    torch.cuda.synchronize()
    sv = cast.StateVector(n, tensor=psi)
    fc = cast.FusedCircuit(n, qft(n), k_max=5)
    print(f"  {len(fc)} fused gates; applying", flush=True)
    (sv.apply_circuit if mode == "per_pass" else sv.apply_circuit_blocked)(fc)
    torch.cuda.synchronize()
    err = 0.0
    chunk = 1 << 26
    for s in range(0, N, chunk):
        err = max(err, float((psi[s:s + chunk].to(torch.complex128) - ref[s:s + chunk]).abs().max()))
    print(f"  max |d amp| over all {N} outputs: {err:.2e}", flush=True)
    assert err <= tol
