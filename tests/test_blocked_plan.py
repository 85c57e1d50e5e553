"""Host grouping of the cache-blocked executor (no GPU needed): passes cover
the fused list in order, tile geometry is well formed, and every gate run
inside a tile mixes only amplitudes that differ on the tile's qubits, the
mixed qubits read off the gate's FP64 matrix independently of the planner."""
import numpy as np
import pytest
import torch

import paper_2503_19894_amd as cast
from circuits import dense_haar_layers, qft, rqc_u3_cx
from tests.blocked_cases import mixed_circuit


def mixed_qubits(g):
    """Qubits on which some nonzero entry's row and column differ."""
    m = g["matrix"]
    r, c = np.nonzero(np.abs(m) > 1e-14)
    diff = np.bitwise_or.reduce(r ^ c) if len(r) else 0
    return {q for i, q in enumerate(g["qubits"]) if (diff >> i) & 1}


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64], ids=["c128", "c64"])
@pytest.mark.parametrize("case,n,k_max", [("qft", 30, 5), ("qft", 20, 3), ("rqc", 18, 4), ("mixed", 22, 3),
                                          ("mixed", 16, 5), ("haar", 16, 6)])
@pytest.mark.parametrize("bits", [8, 11, 0])
def test_grouping_invariants(dtype, case, n, k_max, bits):
    gates = {"qft": lambda: qft(n), "rqc": lambda: rqc_u3_cx(n, 5, seed=1),
             "mixed": lambda: mixed_circuit(n, seed=2), "haar": lambda: dense_haar_layers(n, 2, seed=0)}[case]()
    fc = cast.FusedCircuit(n, gates, k_max=max(k_max, max(g.k for g in gates)))
    old = cast.get_tuning("blocked_tile_bits", dtype)
    try:
        if bits:
            cast.set_tuning("blocked_tile_bits", bits, dtype)
        tb = cast.get_tuning("blocked_tile_bits", dtype)
        passes = fc.blocked_passes(dtype)
    finally:
        cast.set_tuning("blocked_tile_bits", old, dtype)
    nxt = 0
    for p in passes:
        assert p["first"] >= nxt and p["count"] >= 1
        members = [fc.gate(i, with_matrix=True) for i in range(p["first"], p["first"] + p["count"])]
        live = [g for g in members if g["active_blocks"] > 0]
        # only identity gates are left out between passes
        for i in range(nxt, p["first"]):
            assert fc.gate(i)["active_blocks"] == 0
        nxt = p["first"] + p["count"]
        if p["tile_bits"] == 0:
            assert len(live) == 1
            continue
        assert p["tile_bits"] == tb and len(live) >= 2
        w, hq = p["window"], p["high_qubits"]
        assert 4 <= w <= tb and len(hq) == tb - w and list(hq) == sorted(hq) and all(q >= w for q in hq)
        tile_qubits = set(range(w)) | set(hq)
        for g in live:
            assert g["d"] <= 3
            assert mixed_qubits(g) <= tile_qubits, (g["qubits"], w, hq)
    for i in range(nxt, len(fc)):
        assert fc.gate(i)["active_blocks"] == 0
    if n < tb:
        assert all(p["tile_bits"] == 0 for p in passes)


def test_qft30_grouping_is_compact():
    """QFT-30 fused with k_max = 5: 112 fused gates in at most 8 HBM passes."""
    fc = cast.FusedCircuit(30, qft(30), k_max=5)
    for dt in (torch.complex128, torch.complex64):
        assert len(fc) == 112
        assert len(fc.blocked_passes(dt)) <= 8


def test_bad_tile_bits_rejected():
    with pytest.raises(cast.CastError):
        cast.set_tuning("blocked_tile_bits", 13, torch.complex128)   # 128 KiB of LDS
    with pytest.raises(cast.CastError):
        cast.set_tuning("blocked_tile_bits", 7, torch.complex64)
