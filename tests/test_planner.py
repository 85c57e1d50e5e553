"""The path planner (no GPU: fusion, schedules and the blocked grouping are
planned on the host).  With the path costs fixed, the plan it picks follows
from the pricing rule: a Trotter circuit (HES) whose 5-qubit fused gates are
dense matrix-core passes is cheaper as 3-qubit fused gates in cache-blocked
segments, a choice that size-only fusion at k_max 5 does not make; with
in-tile costs raised it falls back to k_max 5 per pass."""
import pytest
import torch

import paper_2503_19894_amd as cast
from circuits import FAMILIES

DT = torch.complex128
FIXED = {"bw0": 5200, "bw1": 4800, "bw2": 4000, "bw3": 5260, "bw4": 4840, "bw5": 4500, "bw6": 5400,
         "fl4": 38000, "fl5": 38700, "fl6": 51900, "fl_vec": 60000, "launch_ms": 0.005, "seg_bw": 5000,
         "seg_gate0": 0.25, "seg_gate1": 0.5, "seg_gate2": 0.5, "seg_gate3": 0.6}


@pytest.fixture
def fixed_costs():
    old = {k: cast.get_path_cost(k, DT) for k in cast.PATH_COST_KEYS}
    for k, v in FIXED.items():
        cast.set_path_cost(k, v, DT)
    yield
    for k, v in old.items():
        cast.set_path_cost(k, v, DT)


def test_hes_plan_differs_from_size_only(fixed_costs):
    n = 30
    gates = FAMILIES["hes"](n)
    fc, path, k, pred = cast.plan(n, gates, DT, k_range=(2, 6))
    size_only = cast.FusedCircuit(n, gates, k_max=5)
    print(f"hes30: plan k_max {k} path {path} {pred:.1f} ms; size-only per pass "
          f"{size_only.predict_ms(DT, 0):.1f} ms", flush=True)
    assert (k, path) == (3, 1)
    assert pred < size_only.predict_ms(DT, 0)
    assert len(fc) == len(cast.FusedCircuit(n, gates, k_max=3))


def test_expensive_tiles_fall_back_to_per_pass(fixed_costs):
    n = 30
    gates = FAMILIES["hes"](n)
    for d in range(4):
        cast.set_path_cost(f"seg_gate{d}", 50.0, DT)
    fc, path, k, pred = cast.plan(n, gates, DT, k_range=(2, 6))
    assert path == 0 and k >= 5


def test_prediction_prices_every_pass(fixed_costs):
    """Per-pass prediction = sum over the schedule of a launch plus
    max(bytes / rate, flops / rate), recomputed here from the schedule."""
    n = 24
    fc = cast.FusedCircuit(n, FAMILIES["qvc"](n), k_max=5)
    want = 0.0
    for p in fc.schedule(DT):
        if p["kernel"] < 0:
            continue
        d = fc.gate(p["first"])["d"] if p["kernel"] != 6 else 0
        rate = FIXED[f"fl{max(d, 4)}"] if p["kernel"] in (4, 5) else FIXED["fl_vec"]
        want += FIXED["launch_ms"] + max(p["alg_bytes"] / (FIXED[f"bw{p['kernel']}"] * 1e6), p["flops"] / (rate * 1e6))
    assert abs(fc.predict_ms(DT, 0) - want) <= 1e-9 * want


def test_path_cost_validation():
    with pytest.raises(cast.CastError):
        cast.set_path_cost("bw9", 1.0)
    with pytest.raises(cast.CastError):
        cast.set_path_cost("seg_bw", -1.0)
    with pytest.raises(cast.CastError):
        cast.plan(10, FAMILIES["qft"](10), DT, k_range=(4, 2))
