"""Host side of the diagonal runs (no GPU: the schedule is planned on the
host).  apply_circuit applies a run of consecutive diagonal fused gates in one
elementwise pass; these tests pin the schedule's structure and its
algorithmic byte count against a brute-force count over the amplitudes."""
import numpy as np
import pytest
import torch

import paper_2503_19894_amd as cast
from circuits import Gate, qft

DT = torch.complex128


@pytest.fixture
def knobs():
    keys = ("diag_run_tables", "diag_run_qubits")
    old = {(k, d): cast.get_tuning(k, d) for k in keys for d in (torch.complex128, torch.complex64)}
    yield
    for (k, d), v in old.items():
        cast.set_tuning(k, v, d)


def _diag_gate(qubits, rng, ones):
    """Diagonal gate with random phases, `ones` of its entries exactly 1."""
    D = 1 << len(qubits)
    ph = np.exp(1j * rng.uniform(0.1, 6.0, D))
    ph[rng.permutation(D)[:ones]] = 1.0
    return Gate("unitary", tuple(qubits), matrix=np.diag(ph))


def _touched_bruteforce(n, gates):
    """Amplitudes at which some gate has a phase other than 1."""
    x = np.arange(1 << n)
    hit = np.zeros(1 << n, dtype=bool)
    for g in gates:
        d = np.diag(np.asarray(g.matrix))
        j = np.zeros(1 << n, dtype=np.int64)
        for i, q in enumerate(g.qubits):
            j |= ((x >> q) & 1) << i
        hit |= d[j] != 1.0
    return int(hit.sum())


def test_schedule_covers_fused_list_in_order(knobs):
    n = 30
    fc = cast.FusedCircuit(n, qft(n), k_max=5)
    for tables in (0, 1, 2, 4):
        cast.set_tuning("diag_run_tables", tables, DT)
        sched = fc.schedule(DT)
        assert sum(p["count"] for p in sched) == len(fc)
        nxt = 0
        for p in sched:
            assert p["first"] == nxt
            nxt += p["count"]
            if p["kernel"] == 6:
                assert 1 <= p["tables"] <= max(tables, 1) and p["count"] >= 2
                assert all(fc.pass_info(i, DT)["kernel"] in (3, -1) for i in range(p["first"], p["first"] + p["count"]))
        if tables == 0:
            assert len(sched) == len(fc) and all(p["kernel"] != 6 for p in sched)
        else:
            assert any(p["kernel"] == 6 for p in sched)
    cast.set_tuning("diag_run_tables", 4, DT)
    sched = fc.schedule(DT)
    print(f"qft30: {len(fc)} fused gates -> {len(sched)} passes", flush=True)
    assert len(sched) < 0.6 * len(fc)


@pytest.mark.parametrize("tables,qubits", [(1, 8), (2, 4), (2, 8), (3, 6), (4, 8)])
def test_run_alg_bytes_match_bruteforce(knobs, tables, qubits):
    """Random diagonals (generic phases, some entries exactly 1) on scattered
    qubits: each run's algorithmic bytes are 2 x 16 B per amplitude at which
    some member gate's phase differs from 1 (generic phases never multiply
    to exactly 1, so this equals the kernel's criterion)."""
    cast.set_tuning("diag_run_tables", tables, DT)
    cast.set_tuning("diag_run_qubits", qubits, DT)
    n = 12
    rng = np.random.default_rng(tables * 10 + qubits)
    gates = []
    for _ in range(14):
        k = int(rng.integers(1, 5))
        qs = sorted(int(q) for q in rng.permutation(n)[:k])
        gates.append(_diag_gate(qs, rng, ones=int(rng.integers(0, (1 << k) - 1))))
    gates.append(Gate("h", (3,)))
    gates += [_diag_gate(sorted(int(q) for q in rng.permutation(n)[:3]), rng, ones=5) for _ in range(5)]
    fc = cast.FusedCircuit(n, gates, k_max=1)    # every gate its own fused gate
    sched = fc.schedule(DT)
    runs = [p for p in sched if p["kernel"] == 6]
    assert runs
    for p in runs:
        # the fused list's own gates (fusion orders gates by tile rows)
        members = []
        for i in range(p["first"], p["first"] + p["count"]):
            g = fc.gate(i, with_matrix=True)
            members.append(Gate("unitary", tuple(g["qubits"][:g["k"]]), matrix=g["matrix"]))
        want = 2 * 16 * _touched_bruteforce(n, members)
        assert p["alg_bytes"] == want, (p, want)
