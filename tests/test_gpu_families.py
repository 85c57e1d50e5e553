"""The synthetic circuit families (QFT, IQP, ALA, QVC, RQC, HES) through both
execution paths and every fusion setting, against the FP64 oracle's unfused
run.  Bars: max |d amp| <= 1e-12 (complex128), <= 1e-5 (complex64)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402
import paper_2503_19894_amd as cast  # noqa: E402
from circuits import FAMILIES, random_state  # noqa: E402

TOL = {torch.complex128: 1e-12, torch.complex64: 1e-5}
MODES = {"none": dict(k_max=1), "size": dict(k_max=5), "adaptive": dict(k_max=5, cost_model=1)}


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64], ids=["c128", "c64"])
@pytest.mark.parametrize("family", sorted(FAMILIES))
def test_family_all_paths(dtype, family):
    n = 14
    gates = FAMILIES[family](n)
    psi0 = random_state(n, seed=21, workload=9)
    want = oracle.run_circuit(n, gates, psi0)
    for mode, opts in MODES.items():
        fc = cast.FusedCircuit(n, gates, cost_dtype=dtype, **opts)
        for path in ("apply_circuit", "apply_circuit_blocked"):
            t = torch.tensor(psi0, dtype=dtype, device="cuda")
            sv = cast.StateVector(n, tensor=t)
            getattr(sv, path)(fc)
            err = float(np.max(np.abs(sv.numpy().astype(np.complex128) - want)))
            print(f"{family} {mode} {path} {dtype}: {len(fc)} fused, err {err:.2e}", flush=True)
            assert err <= TOL[dtype], (mode, path, err)
