"""The committed autotuner result loads, names only known knobs, and every
value is accepted by the library (applied at import)."""
import json
import os

import paper_2503_19894_amd as cast


def test_tuning_file_is_applied_and_valid():
    data = json.load(open(cast.TUNING_FILE))
    assert set(data["knobs"]) == {"c64", "c128"}
    for dname, knobs in data["knobs"].items():
        assert set(knobs) <= set(cast.TUNING_KEYS)
    assert cast.apply_tuning_file() or os.environ.get("CAST_NO_TUNING_FILE")
    import torch
    for key, value in data["knobs"]["c128"].items():
        env = cast._ENV_OF.get(key, "")
        if not (os.environ.get(env) or os.environ.get(env + "_C128")):
            assert cast.get_tuning(key, torch.complex128) == value
    for dname in ("c64", "c128"):
        ks = {(e["k"], e["d"]) for e in data["cost"][dname]}
        assert ks == {(k, d) for k in range(1, 7) for d in range(k + 1)}
        assert all(e["ms_per_gamp"] > 0 for e in data["cost"][dname])
