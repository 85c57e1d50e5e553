"""Autotuner for libcast on the current GPU.

Measures (1) the launch knobs of the pass kernels by coordinate descent on a
representative suite of passes, and (2) the pass-cost table that the adaptive
fusion check uses (one pass of a k-qubit gate whose nonzero pattern spans a
d-dimensional XOR subspace), then writes both to tuning_gfx950.json next to
the library, which the binding applies at import.

    python paper_2503_19894_amd/autotune.py [--n 30] [--out PATH]

The cost table follows the paper's CostModel idea (Sec. III-C): time gates of
varied size and sparsity on the target and let fusion consult the table.
"""
import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import numpy as np  # noqa: E402
import torch  # noqa: E402

import paper_2503_19894_amd as cast  # noqa: E402
from circuits import Gate, gate_sweep, haar_unitary, qft  # noqa: E402

KNOB_CHOICES = [
    ("direct_min_q", [3, 4, 5, 6]),
    ("tile_bits", [11, 12, 13]),
    ("direct_ipt", [1, 2, 4]),
    ("direct_nt", [0, 1]),
    ("mfma_direct_min_q", [0, 2, 4]),
    ("mfma_grid_per_cu", [2, 4, 8]),
    ("max_grid", [1 << 18, 1 << 20]),
    ("diag_unroll", [2, 4, 8]),
    ("diag_max_grid", [1 << 14, 1 << 16, 1 << 18, 1 << 20]),
    ("diag_lds_table", [0, 1]),
    ("diag_order", [0, 1]),
    ("mfma_3m_min_d", [4, 5, 6, 7]),
    ("mfma_low_tile", [0, 1]),
    ("direct_chunk_log", [6, 8, 10, 12]),
    ("diag_run_unroll", [1, 2, 4]),
    ("diag_run_grid", [1 << 12, 1 << 16, 1 << 20]),
    ("diag_run_lds", [0, 1]),
    ("mfma_prefetch", [0, 1, 2]),
    ("diag_run_reuse", [0, 2, 4, 6]),
    ("direct_rot", [0, 1, 2, 3]),
]


def structured_unitary(k, d, rng):
    """A k-qubit unitary whose nonzero pattern spans exactly the XOR subspace
    of its first d qubits: (Haar on d qubits) x (random diagonal phases on
    the other k - d), every block active."""
    u = haar_unitary(1 << d, rng) if d else np.ones((1, 1), dtype=np.complex128)
    ph = np.exp(1j * rng.uniform(0.1, 2 * math.pi - 0.1, 1 << (k - d)))
    return np.kron(np.diag(ph), u)   # bit i < d: the Haar factor (least significant)


def suite(n, dtype):
    """Fused circuits whose passes cover every kernel class."""
    rng = np.random.default_rng(0)
    items = [cast.FusedCircuit(n, qft(n), k_max=5)]
    for k, qs in ((4, (0, 1, 2, 3)), (5, (n - 5, n - 4, n - 3, n - 2, n - 1)), (6, (1, 7, 12, 18, 23, n - 1)),
                  (3, (2, 9, 20)), (2, (0, 15))):
        items.append(cast.FusedCircuit(n, [Gate("unitary", qs, matrix=haar_unitary(1 << k, rng))], k_max=k))
    items.append(cast.FusedCircuit(n, gate_sweep("x", 3, (0, 1, 2)), k_max=3))
    # low targets, two 16-dimensional blocks (the Ising-chain shape)
    items.append(cast.FusedCircuit(n, [Gate("unitary", (0, 1, 2, 3, 4), matrix=structured_unitary(5, 4, rng))],
                                   k_max=5))
    return items


def time_suite(sv, items, reps=3):
    best = []
    for fc in items:
        sv.apply_circuit(fc)
        ts = [float(sv.apply_circuit_timed(fc).sum()) for _ in range(reps)]
        best.append(min(ts))
    return float(sum(best))


def tune_knobs(n, dtype, log):
    psi = torch.zeros(1 << n, dtype=dtype, device="cuda")
    psi[0] = 1
    sv = cast.StateVector(n, tensor=psi)
    items = suite(n, dtype)
    chosen = {}
    base = time_suite(sv, items)
    log(f"  start: {base:.2f} ms")
    for key, values in KNOB_CHOICES:
        cur = cast.get_tuning(key, dtype)
        results = {}
        for v in values:
            cast.set_tuning(key, v, dtype)
            results[v] = time_suite(sv, items)
        best = min(results, key=results.get)
        # keep the current value unless another is clearly better (> 1 %)
        if results.get(cur, float("inf")) <= results[best] * 1.01:
            best = cur
        cast.set_tuning(key, best, dtype)
        chosen[key] = best
        log(f"  {key}: " + ", ".join(f"{v}: {t:.2f}" for v, t in results.items()) + f" -> {best}")
    del sv, psi
    torch.cuda.empty_cache()
    return chosen


def cost_table(n, dtype, log):
    psi = torch.zeros(1 << n, dtype=dtype, device="cuda")
    psi[0] = 1
    sv = cast.StateVector(n, tensor=psi)
    rng = np.random.default_rng(1)
    spread = [0, 7, 13, 19, 23, n - 1]
    out = []
    for k in range(1, 7):
        qs = tuple(spread[:k])
        for d in range(0, k + 1):
            fc = cast.FusedCircuit(n, [Gate("unitary", qs, matrix=structured_unitary(k, d, rng))], k_max=k)
            assert fc.gate(0)["d"] == d
            sv.apply_circuit(fc)
            ms = min(float(sv.apply_circuit_timed(fc)[0]) for _ in range(3))
            out.append({"k": k, "d": d, "ms_per_gamp": ms * 2.0 ** (30 - n)})
        log(f"  k={k}: " + " ".join(f"d{e['d']}={e['ms_per_gamp']:.2f}" for e in out if e["k"] == k))
    del sv, psi
    torch.cuda.empty_cache()
    return out


def _timed_passes(sv, fc, reps=3):
    """Best-of-reps device time of each pass of fc's schedule (ms)."""
    sv.apply_circuit(fc)
    return np.min([sv.apply_circuit_timed(fc) for _ in range(reps)], axis=0)


def stream_rate(buf, nbytes, reps=5):
    """Read + write GB/s of the library's streaming kernel over `buf`
    (in-place scale by 1), best of reps."""
    import ctypes
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    run = lambda: cast.stream_scale(ctypes.c_void_p(buf.data_ptr()), nbytes, 1.0, 1, 0, stream)  # noqa: E731
    run()
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        run()
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b))
    return 2.0 * nbytes / (best * 1e-3) / 1e9


def path_costs(n, dtype, log):
    """Rates the path planner prices plans with (measured on 2^n states):
    algorithmic GB/s of each pass kernel, the matrix cores' GFLOP/s by block
    dimension, the fixed cost of a pass, and for cache-blocked segments the
    state read/write rate and the in-tile cost per gate by block dimension
    (a linear fit over segments of different lengths)."""
    rng = np.random.default_rng(2)
    psi = torch.zeros(1 << n, dtype=dtype, device="cuda")
    psi[0] = 1
    sv = cast.StateVector(n, tensor=psi)
    rates = {}   # kind -> [GB/s]
    fl = {}
    cases = []
    for k in (2, 3):
        cases += [gate_sweep("haar", k, tuple(range(n - k, n)), seed=k), gate_sweep("haar", k, tuple(range(k)), seed=k),
                  gate_sweep("diag", k, tuple(sorted(rng.permutation(n)[:k])), seed=k)]
    for k in (4, 5, 6):
        cases += [gate_sweep("haar", k, tuple(range(n - k, n)), seed=k), gate_sweep("haar", k, tuple(range(k)), seed=k)]
    for gates in cases:
        k = max(len(g.qubits) for g in gates)
        fc = cast.FusedCircuit(n, gates, k_max=k)
        inf = fc.schedule(dtype)[0]
        t = float(_timed_passes(sv, fc)[0])
        rates.setdefault(inf["kernel"], []).append(inf["alg_bytes"] / (t * 1e-3) / 1e9)
        if inf["kernel"] in (4, 5):
            d = fc.gate(0)["d"]
            fl.setdefault(d, []).append(inf["flops"] / (t * 1e-3) / 1e9)
    fc = cast.FusedCircuit(n, qft(n), k_max=5)
    sched = fc.schedule(dtype)
    ts = _timed_passes(sv, fc)
    for inf, t in zip(sched, ts):
        if inf["kernel"] >= 0 and inf["alg_bytes"] > 0:
            rates.setdefault(inf["kernel"], []).append(inf["alg_bytes"] / (t * 1e-3) / 1e9)
    out = {f"bw{kind}": float(np.median(v)) for kind, v in rates.items()}
    out.update({f"fl{d}": float(np.median(v)) for d, v in fl.items()})
    # fixed cost: passes on a small state
    small = cast.StateVector(12, dtype=dtype)
    fc = cast.FusedCircuit(12, gate_sweep("haar", 2, (10, 11), seed=1) * 1, k_max=2)
    out["launch_ms"] = float(np.median(_timed_passes(small, fc, reps=7)))
    # segments: m gates of block dimension d on the low qubits, one segment
    seg = {}
    for d in (0, 1, 2, 3):
        pts = []
        for m in (4, 24):
            gates = []
            for i in range(m):
                qs = tuple(sorted(rng.permutation(8)[:max(d, 1) + (1 if d == 0 else 0)]))
                if d == 0:
                    gates.append(Gate("unitary", qs, matrix=np.diag(np.exp(1j * rng.uniform(0.1, 6, 1 << len(qs))))))
                else:
                    gates.append(Gate("unitary", qs, matrix=haar_unitary(1 << d, rng)))
            fc = cast.FusedCircuit(n, gates, k_max=1)
            bp = fc.blocked_passes(dtype)
            if len(bp) != 1 or not bp[0]["tile_bits"]:
                continue
            sv.apply_circuit_blocked(fc)
            t = min(float(sv.apply_circuit_blocked_timed(fc)[0]) for _ in range(3))
            pts.append((len(fc), t))
        if len(pts) == 2 and pts[1][0] > pts[0][0]:
            (m0, t0), (m1, t1) = pts
            b = (t1 - t0) / (m1 - m0)
            seg[d] = (max(b, 1e-4) * 2.0 ** (30 - n), t0 - b * m0)
    for d, (per_gate, _) in seg.items():
        out[f"seg_gate{d}"] = per_gate
    base = [a for _, a in seg.values() if a > 0]
    S = (1 << n) * (16 if dtype == torch.complex128 else 8)
    stream = stream_rate(psi, S)
    if base:
        # a segment's state read and write cannot beat the streaming kernel
        fit = 2.0 * S / (max(float(np.median(base)) - out["launch_ms"], 1e-3) * 1e-3) / 1e9
        out["seg_bw"] = min(fit, stream)
    del sv, psi, small
    torch.cuda.empty_cache()
    log("  " + ", ".join(f"{k}={v:.4g}" for k, v in sorted(out.items())))
    return {k: v for k, v in out.items() if v > 0 and np.isfinite(v)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=30)
    ap.add_argument("--out", default=os.path.join(HERE, "tuning_gfx950.json"))
    ap.add_argument("--path-costs-only", action="store_true",
                    help="keep the knobs and cost table of the existing file; measure only the path costs")
    args = ap.parse_args()
    if not torch.cuda.is_available():
        sys.exit("autotune needs a GPU")

    def log(msg):
        print(msg, flush=True)

    t0 = time.time()
    if args.path_costs_only:
        result = json.load(open(args.out))
        result["path_cost"] = {}
        for dname, dtype in (("c128", torch.complex128), ("c64", torch.complex64)):
            log(f"{dname}: path costs")
            result["path_cost"][dname] = path_costs(args.n, dtype, log)
        result["seconds_path_cost"] = round(time.time() - t0, 1)
        with open(args.out, "w") as f:
            json.dump(result, f, indent=1)
        log(f"wrote {args.out}")
        return
    result = {"device": torch.cuda.get_device_properties(0).gcnArchName, "n_qubits": args.n,
              "knobs": {}, "cost": {}}
    for dname, dtype in (("c128", torch.complex128), ("c64", torch.complex64)):
        log(f"{dname}: knobs")
        result["knobs"][dname] = tune_knobs(args.n, dtype, log)
        # the batched programs' tile size is measured on the batch workloads
        # (bench.py --vqa-only / --tfim-only), not on this suite: carried over
        result["knobs"][dname]["batch_tile_bits"] = cast.get_tuning("batch_tile_bits", dtype)
        result["knobs"][dname]["batch_min_window"] = cast.get_tuning("batch_min_window", dtype)
        log(f"{dname}: cost table (ms per 2^30 amplitudes)")
        result["cost"][dname] = cost_table(args.n, dtype, log)
        log(f"{dname}: path costs")
        result.setdefault("path_cost", {})[dname] = path_costs(args.n, dtype, log)
        for key, v in result["path_cost"][dname].items():
            cast.set_path_cost(key, v, dtype)
    result["seconds"] = round(time.time() - t0, 1)
    with open(args.out, "w") as f:
        json.dump(result, f, indent=1)
    log(f"wrote {args.out} in {result['seconds']} s")


if __name__ == "__main__":
    main()
