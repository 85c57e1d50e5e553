"""Parity of the batched programs at the benchmarked sizes, in the launch
modes the benchmark times: the 20-qubit, 320-parameter VQA with 256 parameter
sets (sampled sets against the oracle's adjoint gradient), and the mixed-size
TFIM batch (n = 16, 16, 20, 20, 24, 26): its 16- and 20-qubit instances
against the oracle in the graph and persistent modes, and every instance,
24 and 26 qubits included, against two symmetries that hold at any size."""
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


TFIM_NS = (16, 16, 20, 20, 24, 26)
_ORACLE = {}


def _tfim_oracle(i, circs, fields, obs):
    """The oracle's energy and gradient of instance i (cached: the 20-qubit
    instance takes about a minute on the host)."""
    if i not in _ORACLE:
        n = TFIM_NS[i]
        psi0 = np.full(1 << n, 2.0 ** (-n / 2), dtype=np.complex128)
        _ORACLE[i] = oracle.adjoint_grad(n, circs[i], fields[i], obs, psi0=psi0)
    return _ORACLE[i]


@pytest.mark.timeout(900)
@pytest.mark.parametrize("mode", [cast.BATCH_STEPS_GRAPH, cast.BATCH_PERSISTENT_GRAPH], ids=["graph", "persistent"])
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64], ids=["c128", "c64"])
def test_tfim_mixed_batch_vs_oracle(dtype, mode):
    """The benchmarked mixed-size batch in both captured launch modes: the
    16-qubit instances and the first 20-qubit instance (a separate cache
    group at this size) against the oracle's adjoint gradient."""
    ns = TFIM_NS
    circs = [tfim_trotter(n, steps=50, dt=0.05) for n in ns]
    fields = [tfim_fields(n, seed=i) for i, n in enumerate(ns)]
    obs = [PauliTerm(1.0, ((0, "Z"),))]
    b = cast.Batch(circs, list(ns), list(ns), [obs] * len(ns), dtype=dtype, init=["plus"] * len(ns), mode=mode)
    e, g = b.run(fields)
    assert all(np.isfinite(e)) and all(abs(x) <= 1 + 1e-6 for x in e)
    for i in (0, 1, 2):
        print(f"tfim instance {i} (n={ns[i]}) {dtype} mode {mode}: oracle", flush=True)
        ew, gw = _tfim_oracle(i, circs, fields, obs)
        print(f"  dE {abs(e[i] - ew):.2e} dg {np.max(np.abs(g[i] - gw)):.2e}", flush=True)
        assert abs(e[i] - ew) <= TOL[dtype]
        assert np.max(np.abs(g[i] - gw)) <= TOL[dtype]


# the symmetry zero holds bit for bit in the amplitudes (x and its complement
# go through identical arithmetic) and the reductions are FP64, so it gets
# the tight bar; the reflection maps gates to a different order, so its
# asymmetry is bounded by the gradient bars
ZERO_TOL = {torch.complex128: 1e-12, torch.complex64: 1e-6}


@pytest.mark.parametrize("mode", [cast.BATCH_STEPS_GRAPH, cast.BATCH_PERSISTENT_GRAPH], ids=["graph", "persistent"])
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64], ids=["c128", "c64"])
def test_tfim_mixed_batch_symmetries(dtype, mode):
    """Properties that hold at every size, for all six instances including
    n = 24 and 26 (too large for the oracle's adjoint):
    (1) reflection i -> -i mod n: the Strang step's field terms commute with
    each other and so do its XX couplings, so with fields symmetric under the
    reflection the circuit, |+...+> and Z_0 are all invariant, and
    dE/dh_i = dE/dh_{n-i};
    (2) the textbook convention (RX fields, RZZ couplings) commutes with the
    global flip prod X_i, of which |+...+> is an eigenstate while Z_0 changes
    sign, so <Z_0> and every gradient entry vanish."""
    ns = TFIM_NS
    obs = [PauliTerm(1.0, ((0, "Z"),))]
    fields = []
    for i, n in enumerate(ns):
        f = tfim_fields(n, seed=10 + i)
        fields.append(np.array([f[min(j, n - j)] for j in range(n)]))
    for conv in ("xx", "zz"):
        circs = [tfim_trotter(n, steps=50, dt=0.05, convention=conv) for n in ns]
        b = cast.Batch(circs, list(ns), list(ns), [obs] * len(ns), dtype=dtype, init=["plus"] * len(ns), mode=mode)
        e, g = b.run(fields)
        for i, n in enumerate(ns):
            if conv == "xx":
                asym = max(abs(g[i][j] - g[i][(n - j) % n]) for j in range(n))
                print(f"tfim n={n} {dtype} mode {mode}: <Z0> {e[i]:.6f}, reflection asymmetry {asym:.2e}", flush=True)
                assert abs(e[i]) > 1e-3
                assert asym <= TOL[dtype]
            else:
                zero = max(abs(e[i]), float(np.max(np.abs(g[i]))))
                print(f"tfim n={n} {dtype} mode {mode}: textbook convention max |<Z0>|, |grad| {zero:.2e}", flush=True)
                assert zero <= ZERO_TOL[dtype]
