"""Host-side kernel selection (no GPU needed: pass_info only plans).  Pins
the placement rules of the pass kernels on 30 qubits: diagonal passes go to
the elementwise kernel, d <= 3 to the direct gather when no target is below
bit 4 and to the LDS tile otherwise, and matrix-core passes (d >= 4) to the
direct gather unless a target is below bit 4, d = 4 and either at most one
target lies above the tile's window or the gate has several blocks
(mfma_low_tile), in which case they go to the LDS tile."""
import numpy as np
import pytest
import torch

import paper_2503_19894_amd as cast
from circuits import Gate, haar_unitary

DIAG, DIRECT, TILE, MFMA_DIRECT, MFMA_TILE = 3, 0, 1, 4, 5


def _two_block(seed):
    rng = np.random.default_rng(seed)
    ph = np.exp(1j * rng.uniform(0.1, 6.0, 2))
    return np.kron(np.diag(ph), haar_unitary(16, rng))   # Haar on the first four targets


def _kind(qubits, matrix, dtype, n=30):
    fc = cast.FusedCircuit(n, [Gate("unitary", qubits, matrix=matrix)], k_max=len(qubits))
    assert len(fc) == 1
    g = fc.gate(0)
    return g["d"], g["active_blocks"], fc.pass_info(0, dtype)["kernel"]


@pytest.fixture
def knobs():
    saved = {(k, dt): cast.get_tuning(k, dt) for k in ("mfma_low_tile", "mfma_direct_min_q", "direct_min_q")
             for dt in (torch.complex128, torch.complex64)}
    for dt in (torch.complex128, torch.complex64):
        cast.set_tuning("mfma_direct_min_q", 0, dt)
        cast.set_tuning("direct_min_q", 4, dt)
        cast.set_tuning("mfma_low_tile", 1, dt)
    yield
    for (k, dt), v in saved.items():
        cast.set_tuning(k, v, dt)


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64], ids=["c128", "c64"])
def test_matrix_core_placement(knobs, dtype):
    rng = np.random.default_rng(5)
    h32, h16 = haar_unitary(32, rng), haar_unitary(16, rng)
    # two blocks, low targets: the tile, whatever the high targets
    assert _kind((0, 1, 2, 3, 4), _two_block(1), dtype) == (4, 2, MFMA_TILE)
    assert _kind((0, 1, 2, 28, 29), _two_block(2), dtype) == (4, 2, MFMA_TILE)
    assert _kind((0, 14, 15, 16, 17), _two_block(3), dtype) == (4, 2, MFMA_TILE)
    # one block, d = 4: the tile only with at most one target above the window
    assert _kind((1, 2, 3, 6), h16, dtype) == (4, 1, MFMA_TILE)
    assert _kind((0, 3, 7, 21), h16, dtype) == (4, 1, MFMA_TILE)
    assert _kind((1, 7, 24, 27), h16, dtype) == (4, 1, MFMA_DIRECT)
    # d = 5 stays on the direct gather; no target below bit 4 as well
    assert _kind((0, 1, 2, 3, 4), h32, dtype) == (5, 1, MFMA_DIRECT)
    assert _kind((4, 5, 6, 7, 8), _two_block(4), dtype) == (4, 2, MFMA_DIRECT)
    # the knob switches the low-target rule off
    cast.set_tuning("mfma_low_tile", 0, dtype)
    assert _kind((0, 1, 2, 3, 4), _two_block(1), dtype) == (4, 2, MFMA_DIRECT)
    assert _kind((1, 2, 3, 6), h16, dtype) == (4, 1, MFMA_DIRECT)


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64], ids=["c128", "c64"])
def test_small_block_placement(knobs, dtype):
    rng = np.random.default_rng(6)
    assert _kind((3, 9), np.diag(np.exp(1j * rng.uniform(0.1, 6.0, 4))), dtype)[2] == DIAG
    h4 = haar_unitary(4, rng)
    assert _kind((4, 20), h4, dtype) == (2, 1, DIRECT)
    assert _kind((3, 20), h4, dtype) == (2, 1, TILE)
