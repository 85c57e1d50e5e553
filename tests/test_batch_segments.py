"""Segments of the batched programs (host planning, no GPU): every segment
fits one LDS tile that keeps its low window (batch_min_window) and at most
64 gates, the segments cover every gate once,
gates that share a qubit keep their circuit order unless both are diagonal,
and the reordered circuit is the same operator (checked by the oracle on
small instances).  On the layered ansatz and the Trotter circuit the
commutation-aware cut needs far fewer segments than the circuit-order cut."""
import os

import numpy as np
import pytest
import torch

import oracle
import paper_2503_19894_amd as cast
from circuits import hea_vqa, tfim_trotter, random_state, vqa_thetas, tfim_fields

TB = {dt: cast.get_tuning("batch_tile_bits", dt) for dt in (torch.complex128, torch.complex64)}


def _qubits(g):
    return set(int(q) for q in g.qubits)


def _is_diag(g):
    if getattr(g, "param", -1) >= 0:
        return g.name in ("rz", "rzz")
    return g.name in ("cz", "z", "s", "t", "p", "cp", "rz") or (
        g.name == "unitary" and np.allclose(np.asarray(g.matrix) - np.diag(np.diag(np.asarray(g.matrix))), 0))


def _check(n, gates, dtype, reverse):
    segs = cast.segments(n, gates, dtype, reverse=reverse)
    flat = [l for s in segs for l in s]
    assert sorted(flat) == list(range(len(gates)))
    tb = min(n, TB[dtype])
    w = max(0, min(cast.get_tuning("batch_min_window", dtype), tb - 2))
    for s in segs:
        assert 1 <= len(s) <= 64
        qs = set().union(*(_qubits(gates[l]) for l in s))
        assert len(qs) <= tb
        # the tile keeps a low window of w bits: at most tb - w qubits at or above bit w
        assert len([q for q in qs if q >= w]) <= tb - w
    pos = {l: i for i, l in enumerate(flat)}
    for a in range(len(gates)):
        for b in range(a + 1, len(gates)):
            if not (_qubits(gates[a]) & _qubits(gates[b])):
                continue
            if _is_diag(gates[a]) and _is_diag(gates[b]):
                continue
            # the pair keeps its relative order (reversed for the adjoint sweep)
            assert (pos[a] < pos[b]) != reverse, (a, b)
    return segs


def _circuit_order_count(n, gates, dtype, reverse):
    old = os.environ.get("CAST_BATCH_REORDER")
    os.environ["CAST_BATCH_REORDER"] = "0"
    try:
        return len(cast.segments(n, gates, dtype, reverse=reverse))
    finally:
        if old is None:
            del os.environ["CAST_BATCH_REORDER"]
        else:
            os.environ["CAST_BATCH_REORDER"] = old


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64], ids=["c128", "c64"])
@pytest.mark.parametrize("reverse", [False, True], ids=["fwd", "adj"])
def test_vqa_ansatz_segments(dtype, reverse):
    n = 20
    gates, _ = hea_vqa(n, 8)
    segs = _check(n, gates, dtype, reverse)
    base = _circuit_order_count(n, gates, dtype, reverse)
    print(f"hea20x8 {dtype} {'adj' if reverse else 'fwd'}: {len(segs)} segments (circuit order {base})", flush=True)
    assert len(segs) * 3 <= base * 2


@pytest.mark.parametrize("reverse", [False, True], ids=["fwd", "adj"])
def test_tfim_trotter_segments(reverse):
    n = 16
    gates = tfim_trotter(n, steps=6, dt=0.05)
    segs = _check(n, gates, torch.complex128, reverse)
    base = _circuit_order_count(n, gates, torch.complex128, reverse)
    print(f"tfim16x6: {len(segs)} segments (circuit order {base})", flush=True)
    assert len(segs) <= base


@pytest.mark.parametrize("which", ["hea", "tfim"])
def test_reordered_circuit_is_the_same_operator(which):
    """The oracle applies the gates in circuit order and in the segments'
    order (parameters bound); the states agree to rounding."""
    n = 8
    if which == "hea":
        gates, P = hea_vqa(n, 3)
        theta = vqa_thetas(P, 1, seed=5)[0]
    else:
        gates = tfim_trotter(n, steps=3, dt=0.1)
        theta = tfim_fields(n, seed=5)
    psi0 = random_state(n, seed=9, workload=12)
    want = oracle.run_circuit(n, gates, psi0, theta)
    for dtype in (torch.complex128, torch.complex64):
        old = os.environ.get("CAST_BATCH_TILE_BITS")
        os.environ["CAST_BATCH_TILE_BITS"] = "4"   # small tiles: many segments, much reordering
        try:
            flat = [l for s in cast.segments(n, gates, dtype) for l in s]
        finally:
            if old is None:
                del os.environ["CAST_BATCH_TILE_BITS"]
            else:
                os.environ["CAST_BATCH_TILE_BITS"] = old
        assert flat != list(range(len(gates)))
        got = oracle.run_circuit(n, [gates[l] for l in flat], psi0, theta)
        assert np.max(np.abs(got - want)) <= 1e-12
