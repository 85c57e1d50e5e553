"""Seeded generators for the synthetic workloads.

The paper evaluates on circuit families (QFT, ALA, RQC, QVC, IQP, HES) whose
files it does not publish (Sec. V-A); the generators below stand in for them at
the shapes of the five measured workloads.  Every random draw comes from
``numpy.random.default_rng(1000 * workload + seed)`` (PCG64), or, for
multi-GiB input states that are built directly in device memory, from torch's
Philox generator seeded the same way.
"""
import math
from typing import List, Sequence, Tuple

import numpy as np

from .spec import Gate, PauliTerm


def _rng(workload: int, seed: int) -> np.random.Generator:
    return np.random.default_rng(1000 * workload + seed)


# --------------------------------------------------------------------------- states
def random_state(n: int, seed: int = 0, workload: int = 2) -> np.ndarray:
    """i.i.d. complex Gaussian amplitudes divided by their FP64 2-norm."""
    rng = _rng(workload, seed)
    N = 1 << n
    a = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    a /= np.sqrt(np.vdot(a, a).real)
    return a.astype(np.complex128)


def random_state_torch(n: int, seed: int = 0, device="cuda", dtype=None, workload: int = 2):
    """Same distribution as :func:`random_state`, drawn by torch's generator on
    ``device`` (used for states too large to stage through host memory).
    Returns a complex128 (default) or complex64 tensor of 2^n amplitudes."""
    import torch

    dtype = dtype or torch.complex128
    real = torch.float64 if dtype == torch.complex128 else torch.float32
    g = torch.Generator(device=device)
    g.manual_seed(1000 * workload + seed)
    N = 1 << n
    out = torch.empty(N, dtype=dtype, device=device)
    view = torch.view_as_real(out)
    chunk = 1 << 26
    nrm = 0.0
    for s in range(0, N, chunk):
        e = min(N, s + chunk)
        view[s:e].normal_(generator=g)
        nrm += float(view[s:e].double().square().sum())
    view.mul_(1.0 / math.sqrt(nrm))
    return out


def plus_state_amp(n: int) -> float:
    """Amplitude of every basis state in |+...+>."""
    return 2.0 ** (-n / 2)


# --------------------------------------------------------------------------- gates
def haar_unitary(dim: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-random unitary by Mezzadri's recipe ("How to generate random
    matrices from the classical compact groups", 2007): QR of a complex
    Gaussian matrix, columns rephased by R's diagonal."""
    z = (rng.standard_normal((dim, dim)) + 1j * rng.standard_normal((dim, dim))) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r)
    return (q * (d / np.abs(d))[None, :]).astype(np.complex128)


def rqc_u3_cx(n: int = 12, layers: int = 10, seed: int = 0) -> List[Gate]:
    """Random circuit (RQC stand-in): each layer is U3 on every qubit with
    angles uniform in [0, 2pi), then CX on brick-pattern neighbour pairs:
    (0,1),(2,3),... on even layers, (1,2),(3,4),... on odd layers; control is
    the lower qubit."""
    rng = _rng(1, seed)
    gates: List[Gate] = []
    for layer in range(layers):
        for q in range(n):
            th, ph, la = rng.uniform(0.0, 2.0 * math.pi, 3)
            gates.append(Gate("u3", (q,), (float(th), float(ph), float(la))))
        for c in range(layer % 2, n - 1, 2):
            gates.append(Gate("cx", (c, c + 1)))
    return gates


def qft(n: int) -> List[Gate]:
    """QFT: for j = n-1 .. 0, H on j then CP(2pi / 2^(j-m+1)) on (m, j) for
    m = j-1 .. 0; finally SWAP(i, n-1-i).  With qubit q = index bit q this maps
    psi to y -> 2^(-n/2) sum_x exp(+2 pi i x y / 2^n) psi[x]."""
    gates: List[Gate] = []
    for j in range(n - 1, -1, -1):
        gates.append(Gate("h", (j,)))
        for m in range(j - 1, -1, -1):
            gates.append(Gate("cp", (m, j), (2.0 * math.pi / 2.0 ** (j - m + 1),)))
    for i in range(n // 2):
        gates.append(Gate("swap", (i, n - 1 - i)))
    return gates


def partition_sizes(n: int) -> List[int]:
    """Block sizes 6a + 5b = n with a, b >= 1 and the most 6-qubit blocks;
    falls back to a or b = 0 when no such split exists."""
    best = None
    for a in range(n // 6, -1, -1):
        if (n - 6 * a) % 5 == 0:
            b = (n - 6 * a) // 5
            if a >= 1 and b >= 1:
                return [6] * a + [5] * b
            if best is None:
                best = [6] * a + [5] * b
    if best is None:
        raise ValueError(f"no 5/6-qubit partition of {n}")
    return best


def dense_haar_layers(n: int = 32, depth: int = 20, seed: int = 0) -> List[Gate]:
    """Dense random circuit (QVC/RQC stand-in): each layer cuts a random
    permutation of the qubits into blocks of 6 and 5 (shuffled order) and puts
    an independent Haar unitary on each block.  Qubit lists are left in the
    permutation's order (not sorted)."""
    rng = _rng(3, seed)
    sizes = partition_sizes(n)
    gates: List[Gate] = []
    for _ in range(depth):
        perm = rng.permutation(n)
        order = list(rng.permutation(len(sizes)))
        pos = 0
        for bi in order:
            k = sizes[bi]
            qs = tuple(int(q) for q in perm[pos:pos + k])
            pos += k
            gates.append(Gate("unitary", qs, matrix=haar_unitary(1 << k, rng)))
    return gates


def hea_vqa(n: int = 20, layers: int = 8) -> Tuple[List[Gate], int]:
    """Hardware-efficient ansatz (ALA stand-in): per layer RY(theta) on every
    qubit, RZ(theta) on every qubit, then CZ on the ring (i, i+1 mod n).
    Returns (gates, number of parameters)."""
    gates: List[Gate] = []
    p = 0
    for _ in range(layers):
        for q in range(n):
            gates.append(Gate("ry", (q,), param=p)); p += 1
        for q in range(n):
            gates.append(Gate("rz", (q,), param=p)); p += 1
        for q in range(n):
            gates.append(Gate("cz", (q, (q + 1) % n)))
    return gates, p


def vqa_thetas(n_params: int, n_sets: int, seed: int = 0) -> np.ndarray:
    return _rng(4, seed).uniform(-math.pi, math.pi, (n_sets, n_params))


def vqa_hamiltonian(n: int = 20) -> List[PauliTerm]:
    """H = sum_i Z_i Z_{i+1 mod n} + 0.5 sum_i X_i."""
    terms = [PauliTerm(1.0, ((i, "Z"), ((i + 1) % n, "Z"))) for i in range(n)]
    terms += [PauliTerm(0.5, ((i, "X"),)) for i in range(n)]
    return terms


def tfim_fields(n: int, seed: int = 0) -> np.ndarray:
    return _rng(5, seed).uniform(0.5, 1.5, n)


def tfim_trotter(n: int, steps: int = 50, dt: float = 0.05, J: float = 1.0,
                 convention: str = "xx") -> List[Gate]:
    """Second-order (Strang) Trotter circuit of a transverse-field Ising ring.

    convention "xx": H = -J sum X_i X_{i+1} - sum h_i Z_i.  Per step: field
    half-steps RZ(-h_i dt), couplings RXX(-2 J dt), field half-steps again.
    convention "zz": H = -J sum Z_i Z_{i+1} - sum h_i X_i with RX / RZZ.
    Field gates are parametrised: param i with coeff -dt, so theta = h."""
    field, coup = ("rz", "rxx") if convention == "xx" else ("rx", "rzz")
    gates: List[Gate] = []
    for _ in range(steps):
        for i in range(n):
            gates.append(Gate(field, (i,), param=i, coeff=-dt))
        for i in range(n):
            gates.append(Gate(coup, (i, (i + 1) % n), (-2.0 * J * dt,)))
        for i in range(n):
            gates.append(Gate(field, (i,), param=i, coeff=-dt))
    return gates


def gate_sweep(kind: str, k: int, targets: Sequence[int], seed: int = 0) -> List[Gate]:
    """Single-pass workloads: a k-qubit pattern on ``targets``.

    kinds: "h" (k Hadamards), "u3" (k random U3), "x" (k Pauli-X), "haar"
    (one dense Haar unitary), "diag" (one diagonal of random phases),
    "ctrl" (Haar 1-qubit U on targets[-1] controlled by the others)."""
    rng = _rng(6, seed)
    t = tuple(int(q) for q in targets)
    assert len(t) == k
    if kind == "h":
        return [Gate("h", (q,)) for q in t]
    if kind == "x":
        return [Gate("x", (q,)) for q in t]
    if kind == "u3":
        return [Gate("u3", (q,), tuple(float(a) for a in rng.uniform(0, 2 * math.pi, 3))) for q in t]
    if kind == "haar":
        return [Gate("unitary", t, matrix=haar_unitary(1 << k, rng))]
    if kind == "diag":
        ph = rng.uniform(0, 2 * math.pi, 1 << k)
        return [Gate("unitary", t, matrix=np.diag(np.exp(1j * ph)))]
    if kind == "ctrl":
        m = np.eye(1 << k, dtype=np.complex128)
        u = haar_unitary(2, rng)
        c = (1 << (k - 1)) - 1          # all controls (bits 0..k-2) set
        hi = 1 << (k - 1)               # bit of targets[-1]
        m[np.ix_([c, c | hi], [c, c | hi])] = u
        return [Gate("unitary", t, matrix=m)]
    raise ValueError(kind)


# ----------------------------------------------------------- benchmark families
# Synthetic stand-ins for the paper's circuit families (Sec. V; the circuit
# files themselves are not available): seeded, with the families' gate mix.

def iqp(n: int, seed: int = 0, density: float = 0.3) -> List[Gate]:
    """IQP: H on every qubit, a diagonal layer (RZ on every qubit and CP with
    random angles on a random subset of all pairs), H on every qubit."""
    rng = _rng(11, seed)
    gates = [Gate("h", (q,)) for q in range(n)]
    gates += [Gate("rz", (q,), (float(rng.uniform(0, 2 * math.pi)),)) for q in range(n)]
    for i in range(n):
        for j in range(i + 1, n):
            if rng.random() < density:
                gates.append(Gate("cp", (i, j), (float(rng.uniform(0, 2 * math.pi)),)))
    gates += [Gate("h", (q,)) for q in range(n)]
    return gates


def ala(n: int, layers: int = 10, seed: int = 0) -> List[Gate]:
    """Alternating layered ansatz: per layer RY on every qubit, then CZ on the
    brick pairs (i, i+1) starting at 0 on even and 1 on odd layers."""
    rng = _rng(12, seed)
    gates: List[Gate] = []
    for layer in range(layers):
        gates += [Gate("ry", (q,), (float(rng.uniform(0, 2 * math.pi)),)) for q in range(n)]
        gates += [Gate("cz", (c, c + 1)) for c in range(layer % 2, n - 1, 2)]
    return gates


def qvc(n: int, depth: int = 10, seed: int = 0) -> List[Gate]:
    """Quantum-volume circuit: per layer a random pairing of the qubits, a
    Haar-random two-qubit unitary on each pair."""
    rng = _rng(13, seed)
    gates: List[Gate] = []
    for _ in range(depth):
        perm = rng.permutation(n)
        for i in range(0, n - 1, 2):
            gates.append(Gate("unitary", (int(perm[i]), int(perm[i + 1])), matrix=haar_unitary(4, rng)))
    return gates


def hes(n: int, steps: int = 10, dt: float = 0.05, seed: int = 0) -> List[Gate]:
    """Hamiltonian simulation: Strang-Trotter steps of a transverse-field Ising
    ring (RZ field half-steps with random fields, RXX couplings), fixed angles."""
    h = _rng(14, seed).uniform(0.5, 1.5, n)
    gates: List[Gate] = []
    for _ in range(steps):
        gates += [Gate("rz", (i,), (float(-h[i] * dt),)) for i in range(n)]
        gates += [Gate("rxx", (i, (i + 1) % n), (-2.0 * dt,)) for i in range(n)]
        gates += [Gate("rz", (i,), (float(-h[i] * dt),)) for i in range(n)]
    return gates


FAMILIES = {
    "qft": lambda n: qft(n),
    "iqp": lambda n: iqp(n),
    "ala": lambda n: ala(n),
    "qvc": lambda n: qvc(n),
    "rqc": lambda n: rqc_u3_cx(n, 10, seed=0),
    "hes": lambda n: hes(n),
}
