"""Generated kernels compile for gfx950 on the host (no GPU): one kernel per
non-identity fused gate with blocks up to 16 x 16, for both dtypes."""
import torch

import paper_2503_19894_amd as cast
from circuits import dense_haar_layers, qft, rqc_u3_cx
from tests.blocked_cases import mixed_circuit


def test_jit_compiles_one_kernel_per_small_gate():
    for n, gates, km in ((12, qft(12), 5), (13, rqc_u3_cx(13, 3, seed=2), 4), (12, mixed_circuit(12, seed=3), 3),
                         (16, dense_haar_layers(16, 1, seed=0), 6)):
        fc = cast.FusedCircuit(n, gates, k_max=km)
        want = sum(1 for i in range(len(fc)) if fc.gate(i)["active_blocks"] > 0 and fc.gate(i)["d"] <= 4)
        for dt in (torch.complex128, torch.complex64):
            nk, ms = fc.jit_compile(dt)
            assert nk == want and ms > 0
            assert fc.jit_compile(dt) == (nk, ms)      # cached
