"""Parity of the batched programs at the benchmarked sizes, in the launch
modes the benchmark times: the 20-qubit, 320-parameter VQA with 256 parameter
sets (sampled sets against the oracle's adjoint gradient), and the mixed-size
TFIM batch (n = 16, 16, 20, 20, 24, 26; its 16-qubit instances against the
oracle, all instances' <Z_0> finite and within [-1, 1])."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402
import paper_2503_19894_amd as cast  # noqa: E402
from circuits import PauliTerm, hea_vqa, tfim_fields, tfim_trotter, vqa_hamiltonian, vqa_thetas  # noqa: E402

TOL = {torch.complex128: 1e-10, torch.complex64: 5e-4}


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64], ids=["c128", "c64"])
def test_vqa_256_sets_sampled_vs_oracle(dtype):
    n, sets = 20, 256
    gates, P = hea_vqa(n, 8)
    H = vqa_hamiltonian(n)
    th = vqa_thetas(P, sets, seed=0)
    b = cast.Batch([gates] * sets, [n] * sets, [P] * sets, [H] * sets, dtype=dtype, mode=cast.BATCH_STEPS_GRAPH)
    e, g = b.run(list(th))
    for i in (0, 137, 255):
        ew, gw = oracle.adjoint_grad(n, gates, th[i], H)
        print(f"vqa20 set {i} {dtype}: dE {abs(e[i] - ew):.2e} dg {np.max(np.abs(g[i] - gw)):.2e}", flush=True)
        assert abs(e[i] - ew) <= TOL[dtype]
        assert np.max(np.abs(g[i] - gw)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64], ids=["c128", "c64"])
def test_tfim_mixed_batch_vs_oracle(dtype):
    ns = (16, 16, 20, 20, 24, 26)
    circs = [tfim_trotter(n, steps=50, dt=0.05) for n in ns]
    fields = [tfim_fields(n, seed=i) for i, n in enumerate(ns)]
    obs = [PauliTerm(1.0, ((0, "Z"),))]
    b = cast.Batch(circs, list(ns), list(ns), [obs] * len(ns), dtype=dtype, init=["plus"] * len(ns),
                   mode=cast.BATCH_PERSISTENT_GRAPH)
    e, g = b.run(fields)
    assert all(np.isfinite(e)) and all(abs(x) <= 1 + 1e-6 for x in e)
    for i in (0, 1):
        n = ns[i]
        psi0 = np.full(1 << n, 2.0 ** (-n / 2), dtype=np.complex128)
        ew, gw = oracle.adjoint_grad(n, circs[i], fields[i], obs, psi0=psi0)
        print(f"tfim16 instance {i} {dtype}: dE {abs(e[i] - ew):.2e} dg {np.max(np.abs(g[i] - gw)):.2e}", flush=True)
        assert abs(e[i] - ew) <= TOL[dtype]
        assert np.max(np.abs(g[i] - gw)) <= TOL[dtype]
