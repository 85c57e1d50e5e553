#!/usr/bin/env python3
"""Benchmark of the fused-gate hot path on one MI355X.

Workload: 30-qubit QFT (30 H + 435 controlled-phase + 15 SWAP gates) applied
to a random normalised state with i.i.d. complex Gaussian amplitudes, after
host fusion with k_max = 5.  One step = one application of the whole fused
circuit (every fused gate = one in-place pass over the 2^30 amplitudes), with
the state already resident in HBM.  Before the warmup the passes' launch
shapes are measured on the state (circuit_tune, extras.<dtype>.tune),
which is then drawn again from its seed; marker dispatches bracket the timed
steps so that kernel traces can be cut to them (--summarize-kernel-trace on a
per-dispatch trace).

Headline value: effective HBM GB/s per fused-gate pass = the passes'
algorithmic bytes (every amplitude of a non-identity block read and written
once; amplitudes whose phase is 1 in a diagonal pass are not counted) summed
over the fused list / wall time of the timed steps.  The dense-equivalent rate
(every pass counted as a full read and write of the state) is reported as
extras.c128.dense_equivalent_gbs.  The line also carries:
  roofline     -- the dominant kernel's algorithmic bytes (amplitudes of
                  non-identity blocks, read + written) over its average launch
                  duration from HIP events on the state's stream, vs 8 TB/s;
  cpu_baseline -- the FP64 CPU oracle timed on a bounded sample of the same
                  workload (the first unfused QFT gates on the same 2^30
                  state), in the same unit;
  vqa_grads_per_s -- batched adjoint VQA gradients/s (20 qubits, 320
                  parameters, 256 sets) against the plain per-instance
                  adjoint, both dtypes (details under extras.vqa);
  blocked      -- the same fused QFT cache-blocked (several fused gates per
                  HBM pass, apply_circuit_blocked): ms per step and HBM passes
                  for both dtypes (details under extras.<dtype>.blocked);
  extras       -- the complex64 run and per-kernel breakdowns.
"""
import argparse
import json
import math
import os
import sys
import time

HBM_PEAK_GBS = 8000.0



def kernel_label(info, dtype_name):
    """Name of the kernel template instance a pass launches, as the profiler
    prints it (without the argument list), from the library's active knobs.
    `info` is a schedule entry (FusedCircuit.schedule) with the fused gate's
    block dimension "d" added for single-gate passes."""
    import torch

    import paper_2503_19894_amd as cast

    dt = torch.complex128 if dtype_name == "c128" else torch.complex64
    kind, d = info["kernel"], info.get("d", 0)
    r = "double" if dtype_name == "c128" else "float"
    if kind == 6:
        lds = "true" if cast.get_tuning("diag_run_lds", dt) else "false"
        u = cast.get_tuning("diag_run_unroll", dt)
        tile_bits = 8 if dtype_name == "c128" else 9   # amplitude-index bits inside one 256-lane tile
        if cast.get_tuning("diag_run_reuse", dt) > 0 and info.get("n", 30) > tile_bits:
            return f"k_diag_run_reuse<{r}, {info['tables']}, {lds}, {u}>"
        return f"k_diag_run<{r}, {u}, {info['tables']}, {lds}>"
    if kind == 3:
        lds = "true" if cast.get_tuning("diag_lds_table", dt) else "false"
        return f"k_diag<{r}, {cast.get_tuning('diag_unroll', dt)}, {lds}>"
    if kind == 0:
        ipt, cap = cast.get_tuning("direct_ipt", dt), 8 if dtype_name == "c128" else 16
        while ipt > 1 and (ipt * (1 << d) > cap or d > 3):
            ipt >>= 1
        nt = "true" if cast.get_tuning("direct_nt", dt) else "false"
        return f"k_direct<{d}, {r}, {ipt}, {nt}>"
    m3 = "true" if d >= cast.get_tuning("mfma_3m_min_d", dt) else "false"
    if kind == 4:
        pre = cast.get_tuning("mfma_prefetch", dt)
        if pre >= 2 and d < 6:
            return f"k_mfma_direct_db<{d}, {r}, {m3}>"
        return f"k_mfma_direct<{d}, {r}, {m3}, {'true' if pre else 'false'}>"
    if kind == 5:
        return f"k_mfma_tile<{d}, {r}, {m3}>"
    two = "true" if kind == 2 else "false"
    return f"k_tile<{d}, {r}, true, {two}>"


def region_marker():
    """Queues the marker dispatch that brackets a timed region in kernel
    traces: the streaming reference kernel on one 16-byte chunk (one
    workgroup of 256 lanes, a grid no other launch here has)."""
    import ctypes

    import torch

    import paper_2503_19894_amd as cast

    buf = getattr(region_marker, "buf", None)
    if buf is None:
        buf = region_marker.buf = torch.ones(2, dtype=torch.float64, device="cuda")
    cast.stream_scale(ctypes.c_void_p(buf.data_ptr()), 16, 1.0, 1, 1,
                      ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


def run_gpu(n, k_max, dtype_name, steps, warmup, seed=0, tune_reps=3):
    import numpy as np
    import torch

    import paper_2503_19894_amd as cast
    from circuits import qft, random_state_torch

    dtype = torch.complex128 if dtype_name == "c128" else torch.complex64
    amp = 16 if dtype_name == "c128" else 8
    gates = qft(n)
    t0 = time.perf_counter()
    fc = cast.FusedCircuit(n, gates, k_max=k_max)
    host_fusion_ms = (time.perf_counter() - t0) * 1e3
    infos = schedule_infos(fc, dtype)
    npass = len(infos)
    psi = random_state_torch(n, seed=seed, device="cuda", dtype=dtype)
    sv = cast.StateVector(n, tensor=psi)
    tune = None
    if tune_reps > 0:
        # launch shapes of the direct, matrix-core and diagonal-run passes,
        # measured on this state (which the tuner changes), then the input again
        t0 = time.perf_counter()
        before, after = sv.tune_circuit(fc, reps=tune_reps)
        tune = {"reps": tune_reps, "s": round(time.perf_counter() - t0, 3), "tuned_ms_before": round(before, 4),
                "tuned_ms_after": round(after, 4),
                "shapes": {i: list(fc.pass_shape(dtype, i)) for i, inf in enumerate(infos) if inf["kernel"] in (0, 4, 6)}}
        psi.copy_(random_state_torch(n, seed=seed, device="cuda", dtype=dtype))
    for _ in range(warmup):
        sv.apply_circuit(fc)
    torch.cuda.synchronize()
    per_pass = np.zeros(npass)
    region_marker()
    t0 = time.perf_counter()
    for _ in range(steps):
        per_pass += sv.apply_circuit_timed(fc)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    region_marker()
    per_pass /= steps
    state_bytes = (1 << n) * amp
    alg_bytes_per_step = float(sum(i["alg_bytes"] for i in infos))
    alg_gbs = alg_bytes_per_step * steps / wall / 1e9
    dense_equiv_gbs = npass * 2 * state_bytes * steps / wall / 1e9
    # per-kernel totals from the HIP events
    kern = {}
    for inf, ms in zip(infos, per_pass):
        if inf["kernel"] < 0:
            continue
        lab = kernel_label(inf, dtype_name)
        k = kern.setdefault(lab, {"launches_per_step": 0, "ms_per_step": 0.0, "alg_bytes_per_step": 0.0,
                                  "flops_per_step": 0.0})
        k["launches_per_step"] += 1
        k["ms_per_step"] += float(ms)
        k["alg_bytes_per_step"] += inf["alg_bytes"]
        k["flops_per_step"] += inf["flops"]
    for k in kern.values():
        k["avg_launch_ms"] = k["ms_per_step"] / k["launches_per_step"]
        k["alg_bytes_per_launch"] = k["alg_bytes_per_step"] / k["launches_per_step"]
        k["achieved_gbs"] = k["alg_bytes_per_step"] / (k["ms_per_step"] * 1e-3) / 1e9
    dominant = max(kern, key=lambda x: kern[x]["ms_per_step"])
    out = {
        "passes": npass, "fused_gates": len(fc), "diag_run_passes": sum(i["kernel"] == 6 for i in infos),
        "host_fusion_ms": round(host_fusion_ms, 2), "wall_s": wall,
        "ms_per_step": wall / steps * 1e3, "alg_bytes_per_step": alg_bytes_per_step, "alg_gbs": alg_gbs,
        "dense_equivalent_gbs": dense_equiv_gbs,
        "paper_gibps_per_pass": state_bytes / (per_pass.sum() / npass * 1e-3) / 2**30,
        "event_ms_per_step": float(per_pass.sum()),
        "kernels": kern, "dominant": dominant, "tune": tune,
    }
    out["blocked"] = run_blocked(sv, psi, fc, n, dtype, state_bytes, steps, warmup, out["ms_per_step"])
    del sv, psi
    torch.cuda.empty_cache()
    return out


def schedule_infos(fc, dtype):
    """The passes apply_circuit makes (diagonal runs merged), each with the
    block dimension of its fused gate for single-gate passes."""
    infos = fc.schedule(dtype)
    for inf in infos:
        inf["n"] = fc.n
        if inf["kernel"] != 6 and inf["kernel"] >= 0:
            inf["d"] = fc.pass_info(inf["first"], dtype)["d"]
    return infos


def qft_c64_error(n, k_max, seed=5):
    """Largest amplitude difference between the complex64 and the complex128
    result of the fused QFT on the same input (the complex128 input rounded
    to complex64), and the complex128 result's own norm error."""
    import torch

    import paper_2503_19894_amd as cast
    from circuits import qft, random_state_torch

    fc = cast.FusedCircuit(n, qft(n), k_max=k_max)
    a = random_state_torch(n, seed=seed, device="cuda", dtype=torch.complex128)
    b = a.to(torch.complex64)
    cast.StateVector(n, tensor=a).apply_circuit(fc)
    cast.StateVector(n, tensor=b).apply_circuit(fc)
    torch.cuda.synchronize()
    err, chunk = 0.0, 1 << 26
    for s in range(0, a.numel(), chunk):
        err = max(err, float((b[s:s + chunk].to(torch.complex128) - a[s:s + chunk]).abs().max()))
    nrm = float(torch.linalg.vector_norm(a))
    del a, b
    torch.cuda.empty_cache()
    return {"c64_max_abs_diff_vs_c128": err, "c128_norm_error": abs(nrm - 1.0)}


def copy_bandwidth(gib=4, reps=5):
    """Streaming rate on this GPU (bytes read + written per second, HIP
    events): a device-to-device copy and an in-place scale of a `gib` GiB
    buffer by torch, and the library's streaming reference kernel
    (stream_scale: 16 bytes per lane, 1/2/4/8 chunks in flight per lane,
    non-temporal) on the same buffer; best of `reps` each.  Returns the best
    rate, its kind, and every rate measured."""
    import ctypes

    import torch

    import paper_2503_19894_amd as cast

    n = (gib << 30) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def kernel(u):
        return lambda: cast.stream_scale(ctypes.c_void_p(src.data_ptr()), n * 8, 1.0, u, 0, stream)

    ops = [("copy", lambda: dst.copy_(src)), ("in-place scale", lambda: src.mul_(1.0))]
    ops += [(f"stream kernel x{u}", kernel(u)) for u in (1, 2, 4, 8)]
    best = {}
    for kind, op in ops:
        op()
        t = float("inf")
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            op()
            b.record()
            b.synchronize()
            t = min(t, a.elapsed_time(b))
        best[kind] = round(2.0 * (gib << 30) / (t * 1e-3) / 1e9, 1)
    del src, dst
    torch.cuda.empty_cache()
    kind = max(best, key=best.get)
    return best[kind], kind, best


def run_families(n=30, dtype_names=("c128", "c64")):
    """Synthetic stand-ins of the paper's circuit families (QFT, IQP, ALA,
    QVC, RQC, HES) on n qubits from a random state: for each fusion setting
    (none = k_max 1, size-only k_max 5, adaptive k_max 5 with the measured
    cost table, and size-only k_max 2, 3, 4) the fused-gate count, host fusion
    time, one-pass-per-gate time and cache-blocked time (one warm-up
    application each, then one timed); then the path planner's choice of
    k_max in 2..6 and execution path, with its predicted and measured time."""
    import torch

    import paper_2503_19894_amd as cast
    from circuits import FAMILIES, random_state_torch

    modes = {"none": dict(k_max=1), "size": dict(k_max=5), "adaptive": dict(k_max=5, cost_model=1),
             "size_k2": dict(k_max=2), "size_k3": dict(k_max=3), "size_k4": dict(k_max=4)}
    out = {}
    for dname in dtype_names:
        dtype = torch.complex128 if dname == "c128" else torch.complex64
        psi = random_state_torch(n, seed=0, device="cuda", dtype=dtype)
        sv = cast.StateVector(n, tensor=psi)
        res = {}
        for fam, mk in FAMILIES.items():
            gates = mk(n)
            res[fam] = {"gates": len(gates)}
            for mode, opts in modes.items():
                print(f"[bench] families {dname} {fam} {mode}", file=sys.stderr, flush=True)
                t0 = time.perf_counter()
                fc = cast.FusedCircuit(n, gates, cost_dtype=dtype, **opts)
                fus = (time.perf_counter() - t0) * 1e3
                row = {"fused": len(fc), "host_fusion_ms": round(fus, 2)}
                for path, apply in (("per_pass", sv.apply_circuit), ("blocked", sv.apply_circuit_blocked)):
                    apply(fc)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    apply(fc)
                    torch.cuda.synchronize()
                    row[path + "_s"] = round(time.perf_counter() - t0, 4)
                row["hbm_passes_blocked"] = len(fc.blocked_passes(dtype))
                res[fam][mode] = row
                del fc
            # the path planner: fusion size and execution path chosen from the
            # measured path costs, then timed on the path it chose
            print(f"[bench] families {dname} {fam} planned", file=sys.stderr, flush=True)
            t0 = time.perf_counter()
            fc, path, k, pred = cast.plan(n, gates, dtype, k_range=(2, 6))
            plan_ms = (time.perf_counter() - t0) * 1e3
            apply = sv.apply_circuit_blocked if path == 1 else sv.apply_circuit
            apply(fc)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            apply(fc)
            torch.cuda.synchronize()
            res[fam]["planned"] = {"k_max": k, "path": "blocked" if path == 1 else "per_pass", "fused": len(fc),
                                   "predicted_s": round(pred / 1e3, 4), "s": round(time.perf_counter() - t0, 4),
                                   "planning_ms": round(plan_ms, 1)}
            del fc
        out[dname] = res
        del sv, psi
        torch.cuda.empty_cache()
    return out


def run_jit():
    """Generated (immediate-valued) kernels against the library kernels: the
    paper's single-gate table workload (H and U3 on 2 and 3 qubits, one fused
    pass, 28 qubits, high and low targets; GiBps counts the state once as the
    paper does) and QFT-30, both dtypes."""
    import numpy as np
    import torch

    import paper_2503_19894_amd as cast
    from circuits import gate_sweep, qft, random_state_torch

    out = {}
    for dname, dt in (("c128", torch.complex128), ("c64", torch.complex64)):
        amp = 16 if dname == "c128" else 8
        res = {}
        n = 30
        psi = random_state_torch(n, seed=0, device="cuda", dtype=dt)
        sv = cast.StateVector(n, tensor=psi)
        fc = cast.FusedCircuit(n, qft(n), k_max=5)
        nk, cms = fc.jit_compile(dt)
        sv.apply_circuit(fc)
        sv.apply_circuit_jit(fc)
        res["qft30"] = {"library_ms": min(float(sv.apply_circuit_timed(fc).sum()) for _ in range(2)),
                        "generated_ms": min(float(sv.apply_circuit_jit_timed(fc).sum()) for _ in range(2)),
                        "kernels": nk, "compile_ms": round(cms, 1)}
        del sv, psi
        torch.cuda.empty_cache()
        n = 28
        psi = random_state_torch(n, seed=1, device="cuda", dtype=dt)
        sv = cast.StateVector(n, tensor=psi)
        S = (1 << n) * amp
        for kind in ("h", "u3"):
            for k in (2, 3):
                for place, qs in (("high", tuple(range(n - k, n))), ("low", tuple(range(k)))):
                    fc = cast.FusedCircuit(n, gate_sweep(kind, k, qs, seed=k), k_max=k)
                    fc.jit_compile(dt)
                    sv.apply_circuit(fc)
                    sv.apply_circuit_jit(fc)
                    t1 = float(np.median([sv.apply_circuit_timed(fc).sum() for _ in range(5)]))
                    t2 = float(np.median([sv.apply_circuit_jit_timed(fc).sum() for _ in range(5)]))
                    res[f"{kind}x{k}_{place}"] = {"library_gibps": S / (t1 * 1e-3) / 2**30,
                                                  "generated_gibps": S / (t2 * 1e-3) / 2**30}
        del sv, psi
        torch.cuda.empty_cache()
        out[dname] = res
    return out


SWEEP_KINDS = ("haar", "diag", "x", "ctrl", "h", "u3")


def sweep_targets(n, k, place, rng):
    if place == "low":
        return tuple(range(k))
    if place == "high":
        return tuple(range(n - k, n))
    return tuple(int(q) for q in sorted(rng.permutation(n)[:k]))


def run_sweep(ns=(28, 30), reps=5):
    """Single fused-gate passes (the paper's single-gate table pattern,
    widened): k = 1..6 x {dense Haar, diagonal, X^k, controlled-U, H^k, U3^k}
    x targets {low, high, random} on 2^n states, both dtypes.  Each case is
    fused with k_max = k into one gate; its pass time is the median of `reps`
    HIP-event timings; the rate counts the pass's algorithmic bytes (every
    amplitude of a non-identity block read and written once)."""
    import numpy as np
    import torch

    import paper_2503_19894_amd as cast
    from circuits import gate_sweep, random_state_torch

    rows = []
    for dname, dt in (("c128", torch.complex128), ("c64", torch.complex64)):
        for n in ns:
            psi = random_state_torch(n, seed=4, device="cuda", dtype=dt)
            sv = cast.StateVector(n, tensor=psi)
            rng = np.random.default_rng(n)
            for k in range(1, 7):
                for kind in SWEEP_KINDS:
                    if kind == "ctrl" and k == 1:
                        continue
                    for place in ("low", "high", "random"):
                        qs = sweep_targets(n, k, place, rng)
                        fc = cast.FusedCircuit(n, gate_sweep(kind, k, qs, seed=k), k_max=k)
                        sched = schedule_infos(fc, dt)
                        if len(sched) != 1:
                            continue
                        inf = sched[0]
                        sv.apply_circuit(fc)
                        t = float(np.median([sv.apply_circuit_timed(fc)[0] for _ in range(reps)]))
                        gbs = inf["alg_bytes"] / (t * 1e-3) / 1e9
                        tfl = inf["flops"] / (t * 1e-3) / 1e12
                        peak_fl = 78.6 if dname == "c128" else 157.3
                        rows.append({"dtype": dname, "n": n, "k": k, "kind": kind, "place": place,
                                     "qubits": list(qs), "kernel": inf["kernel"], "d": inf.get("d", 0),
                                     "ms": round(t, 4), "alg_gbs": round(gbs, 1),
                                     "frac_hbm": round(gbs / HBM_PEAK_GBS, 4), "tflops": round(tfl, 2),
                                     "frac_fp": round(tfl / peak_fl, 4)})
                        print(f"[bench] sweep {dname} n={n} k={k} {kind} {place}: {t:.3f} ms "
                              f"{gbs:.0f} GB/s", file=sys.stderr, flush=True)
                        del fc
            del sv, psi
            torch.cuda.empty_cache()
    return rows


def run_blocked(sv, psi, fc, n, dtype, state_bytes, steps, warmup, per_pass_ms):
    """The same fused circuit cache-blocked (several fused gates per HBM
    pass): HBM passes, time per step, the passes' HBM rate (every pass reads
    and writes the whole state once), and the largest amplitude difference
    from the one-pass-per-gate path on the same input."""
    import numpy as np
    import torch

    import paper_2503_19894_amd as cast

    groups = fc.blocked_passes(dtype)
    hbm = len(groups)
    for _ in range(warmup):
        sv.apply_circuit_blocked(fc)
    torch.cuda.synchronize()
    per = np.zeros(hbm)
    t0 = time.perf_counter()
    for _ in range(steps):
        per += sv.apply_circuit_blocked_timed(fc)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per /= steps
    seg = [t for g, t in zip(groups, per) if g["tile_bits"]]
    # same input through both paths
    x = psi.clone()
    sv_x = cast.StateVector(n, tensor=x)
    sv_x.apply_circuit(fc)
    y = psi.clone()
    cast.StateVector(n, tensor=y).apply_circuit_blocked(fc)
    torch.cuda.synchronize()
    diff = float((x - y).abs().max())
    del x, y, sv_x
    torch.cuda.empty_cache()
    ms = wall / steps * 1e3
    return {
        "hbm_passes": hbm, "segments": len(seg), "fused_gates_per_pass": [g["count"] for g in groups],
        "ms_per_step": ms, "event_ms_per_step": float(per.sum()), "speedup_vs_per_pass": per_pass_ms / ms,
        "hbm_gbs": hbm * 2 * state_bytes / (per.sum() * 1e-3) / 1e9,
        "max_abs_diff_vs_per_pass": diff,
    }


def run_dense(n=32, depth=20, steps=1, warmup=1, tune_reps=2):
    """Dense random circuit (20 layers of Haar gates on 6- and 5-qubit random
    subsets, complex128, from |0...0>): per-pass kernel throughput; dense
    6-qubit passes are FP64-compute-bound, 5-qubit passes HBM-bound.  With
    tune_reps > 0 every pass's unit order is first chosen per pass by
    measurement (circuit_tune), then the state is reset."""
    import numpy as np
    import torch

    import paper_2503_19894_amd as cast
    from circuits import dense_haar_layers

    gates = dense_haar_layers(n, depth, seed=0)
    fc = cast.FusedCircuit(n, gates, k_max=6)
    infos = schedule_infos(fc, torch.complex128)
    psi = torch.zeros(1 << n, dtype=torch.complex128, device="cuda")
    psi[0] = 1
    sv = cast.StateVector(n, tensor=psi)
    tune = None
    if tune_reps > 0:
        t0 = time.perf_counter()
        before, after = sv.tune_circuit(fc, reps=tune_reps)
        rots = [fc.pass_shape(torch.complex128, i)[0] for i, inf in enumerate(infos) if inf["kernel"] == 4]
        tune = {"reps": tune_reps, "s": round(time.perf_counter() - t0, 3), "ms_before": round(before, 3),
                "ms_after": round(after, 3), "rot_counts": {str(r): rots.count(r) for r in sorted(set(rots))}}
        psi.zero_()
        psi[0] = 1
    for _ in range(warmup):
        sv.apply_circuit(fc)
    torch.cuda.synchronize()
    per = np.zeros(len(infos))
    region_marker()
    t0 = time.perf_counter()
    for _ in range(steps):
        per += sv.apply_circuit_timed(fc)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    region_marker()
    per /= steps
    kern = {}
    for inf, ms in zip(infos, per):
        if inf["kernel"] < 0:
            continue
        lab = kernel_label(inf, "c128")
        k = kern.setdefault(lab, {"launches": 0, "ms": 0.0, "alg_bytes": 0.0, "flops": 0.0})
        k["launches"] += 1
        k["ms"] += float(ms)
        k["alg_bytes"] += inf["alg_bytes"]
        k["flops"] += inf["flops"]
    for k in kern.values():
        k["achieved_gbs"] = k["alg_bytes"] / (k["ms"] * 1e-3) / 1e9
        k["achieved_tflops"] = k["flops"] / (k["ms"] * 1e-3) / 1e12
    nrm = float(torch.linalg.vector_norm(psi))
    del sv, psi
    torch.cuda.empty_cache()
    return {"n_qubits": n, "passes": len(fc), "s_per_circuit": wall / steps, "tune": tune,
            "event_s_per_circuit": float(per.sum()) / 1e3, "norm_after": nrm, "kernels": kern,
            "fp64_roof_s": sum(i["flops"] for i in infos) / 78.6e12,
            "hbm_roof_s": sum(i["alg_bytes"] for i in infos) / 8e12}


def run_tfim(ns=(16, 16, 20, 20, 24, 26), steps=50, dt=0.05, oracle_check=True):
    """Mixed-size batch: Strang-Trotter evolution of transverse-field Ising
    rings of different sizes from |+...+>, <Z_0> and its gradient w.r.t. every
    field h_i, all instances in one batch (graph and persistent launch) vs the
    plain per-instance adjoint."""
    import numpy as np
    import torch

    import paper_2503_19894_amd as cast
    from circuits import PauliTerm, tfim_fields, tfim_trotter

    circs = [tfim_trotter(n, steps=steps, dt=dt) for n in ns]
    fields = [tfim_fields(n, seed=i) for i, n in enumerate(ns)]
    obs = [PauliTerm(1.0, ((0, "Z"),))]
    out = {"n_qubits": list(ns), "trotter_steps": steps, "gates": [len(c) for c in circs]}
    ref = None
    for dname, dtype in (("c128", torch.complex128), ("c64", torch.complex64)):
        res = {}
        for mname, mode in (("graph", cast.BATCH_STEPS_GRAPH), ("persistent", cast.BATCH_PERSISTENT_GRAPH)):
            b = cast.Batch(circs, list(ns), list(ns), [obs] * len(ns), dtype=dtype, init=["plus"] * len(ns),
                           mode=mode)
            e, g = b.run(fields)        # warm-up (and the graph's first replay)
            t0 = time.perf_counter()
            e, g = b.run(fields)
            res[mname] = {"s_per_batch": time.perf_counter() - t0, **b.info()}
            del b
            torch.cuda.empty_cache()
        t0 = time.perf_counter()
        pe, pg = [], []
        for i, n in enumerate(ns):
            init = cast.StateVector(n, tensor=torch.full((1 << n,), 2.0 ** (-n / 2), dtype=dtype, device="cuda"))
            ei, gi = cast.adjoint(init, circs[i], fields[i], obs)
            pe.append(ei)
            pg.append(gi)
        res["plain"] = {"s_per_batch": time.perf_counter() - t0}
        best = min(res["graph"]["s_per_batch"], res["persistent"]["s_per_batch"])
        res["batched_vs_plain"] = res["plain"]["s_per_batch"] / best
        res["batched_plain_max_dgrad"] = float(max(np.max(np.abs(g[i] - pg[i])) for i in range(len(ns))))
        res["z0"] = [float(x) for x in e]
        if dname == "c128":
            ref = (e, g)
        else:
            res["error_vs_fp64"] = {"z0": float(np.max(np.abs(e - ref[0]))),
                                    "grad": float(max(np.max(np.abs(a - b)) for a, b in zip(g, ref[1])))}
        out[dname] = res
    if oracle_check:
        import oracle
        n = ns[0]
        psi0 = np.full(1 << n, 2.0 ** (-n / 2), dtype=np.complex128)
        ew, gw = oracle.adjoint_grad(n, circs[0], fields[0], obs, psi0)
        out["oracle_n%d" % n] = {"z0_err": abs(ref[0][0] - ew), "grad_err": float(np.max(np.abs(ref[1][0] - gw)))}
    return out


def run_vqa(sets=256, n=20, layers=8, steps=2, warmup=1, plain_sets=8, oracle_check=True):
    """Batched VQA gradients (hardware-efficient ansatz, H = sum Z_i Z_i+1 +
    0.5 sum X_i, parameter sets uniform in [-pi, pi]): grads/s of one batch
    of `sets` gradients vs the plain per-instance adjoint, both dtypes."""
    import numpy as np
    import torch

    import paper_2503_19894_amd as cast
    from circuits import hea_vqa, vqa_hamiltonian, vqa_thetas

    gates, P = hea_vqa(n, layers)
    H = vqa_hamiltonian(n)
    th = vqa_thetas(P, sets, seed=0)
    out = {"n_qubits": n, "layers": layers, "params": P, "sets": sets, "gates": len(gates)}
    ref = None
    for dname, dtype in (("c128", torch.complex128), ("c64", torch.complex64)):
        res = {}
        for mname, mode in (("graph", cast.BATCH_STEPS_GRAPH), ("persistent", cast.BATCH_PERSISTENT_GRAPH)):
            t0 = time.perf_counter()
            b = cast.Batch([gates] * sets, [n] * sets, [P] * sets, [H] * sets, dtype=dtype, mode=mode)
            create_s = time.perf_counter() - t0
            for _ in range(warmup):
                e, g = b.run(list(th))
            t0 = time.perf_counter()
            for _ in range(steps):
                e, g = b.run(list(th))
            wall = time.perf_counter() - t0
            info = b.info()
            tr = b.traffic()
            res[mname] = {"grads_per_s": sets * steps / wall, "s_per_batch": wall / steps,
                          "create_s": round(create_s, 3), "steps": info["steps"],
                          "state_bytes": info["state_bytes"], "alg_bytes_per_batch": tr["alg_bytes"],
                          "state_passes_per_batch": tr["state_passes"],
                          "alg_gbs": tr["alg_bytes"] / (wall / steps) / 1e9}
            del b
            torch.cuda.empty_cache()
        init = cast.StateVector(n, dtype=dtype)
        cast.adjoint(init, gates, th[0], H)          # warm-up
        t0 = time.perf_counter()
        pe, pg = [], []
        for i in range(plain_sets):
            ei, gi = cast.adjoint(init, gates, th[i], H)
            pe.append(ei)
            pg.append(gi)
        plain = plain_sets / (time.perf_counter() - t0)
        best = max(res.values(), key=lambda r: r["grads_per_s"])["grads_per_s"]
        res["plain"] = {"grads_per_s": plain, "sets_timed": plain_sets}
        res["batched_vs_plain"] = best / plain
        # batched and plain agree (different reduction orders)
        res["batched_plain_max_dgrad"] = float(max(np.max(np.abs(g[i] - pg[i])) for i in range(plain_sets)))
        if dname == "c128":
            ref = (e, g)
        else:
            res["error_vs_fp64"] = {"energy": float(np.max(np.abs(e - ref[0]))),
                                    "grad": float(max(np.max(np.abs(a - b)) for a, b in zip(g, ref[1])))}
        out[dname] = res
    if oracle_check:
        import oracle
        t0 = time.perf_counter()
        ew, gw = oracle.adjoint_grad(n, gates, th[0], H)
        out["oracle"] = {"s_per_grad": time.perf_counter() - t0,
                         "c128_energy_err": abs(ref[0][0] - ew), "c128_grad_err": float(np.max(np.abs(ref[1][0] - gw)))}
    return out


def run_vqa_profile(sets=256, n=20, layers=8):
    """One complex128 batch of the VQA workload in graph mode after one
    warm-up run: the command the batched kernels are profiled with."""
    import torch

    import paper_2503_19894_amd as cast
    from circuits import hea_vqa, vqa_hamiltonian, vqa_thetas

    gates, P = hea_vqa(n, layers)
    H = vqa_hamiltonian(n)
    th = vqa_thetas(P, sets, seed=0)
    b = cast.Batch([gates] * sets, [n] * sets, [P] * sets, [H] * sets, dtype=torch.complex128,
                   mode=cast.BATCH_STEPS_GRAPH)
    b.run(list(th))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run(list(th))
    wall = time.perf_counter() - t0
    return {"sets": sets, "s_per_batch": wall, "grads_per_s": sets / wall, **b.info(), **b.traffic()}


def vqa_summary(vqa):
    """Headline figures of the batched VQA measurement: grads/s batched (best
    mode) and plain, both dtypes, and the batched run's roofline: algorithmic
    bytes of one batch (from the batch plan) over its time, against 8 TB/s."""
    out = {}
    for d in ("c128", "c64"):
        r = vqa[d]
        mode = max(("graph", "persistent"), key=lambda m: r[m]["grads_per_s"])
        best = r[mode]
        out[f"batched_{d}"] = round(best["grads_per_s"], 2)
        out[f"plain_{d}"] = round(r["plain"]["grads_per_s"], 2)
        out[f"roofline_{d}"] = {"bound": "hbm", "mode": mode, "achieved": round(best["alg_gbs"], 1),
                                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                "frac": round(best["alg_gbs"] / HBM_PEAK_GBS, 4),
                                "alg_bytes_per_grad": best["alg_bytes_per_batch"] / vqa["sets"],
                                "state_passes_per_batch": best["state_passes_per_batch"]}
    if "error_vs_fp64" in vqa["c64"]:
        out["c64_error_vs_fp64"] = vqa["c64"]["error_vs_fp64"]
    return out


def cpu_baseline(n, target_s=15.0, max_gates=8, one_core=True):
    """The oracle (FP64, OpenMP over groups) on the first unfused QFT gates of
    a 2^n state; returns effective GB/s per pass in the same convention."""
    import numpy as np

    import oracle
    from circuits import qft

    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    N = 1 << n
    psi = np.empty(N, dtype=np.complex128)
    psi.real = 1.0 / math.sqrt(N)       # touch every page before timing
    psi.imag = 0.0
    gates = qft(n)
    done, t_total = 0, 0.0
    for g in gates[:max_gates]:
        U = oracle.gates.matrix(g)
        t0 = time.perf_counter()
        oracle.apply_gate(psi, g.qubits, U)
        t_total += time.perf_counter() - t0
        done += 1
        if t_total >= target_s:
            break
    gbs = done * 2 * N * 16 / t_total / 1e9
    del psi
    out = {"value": gbs, "unit": "GB/s", "cores": threads, "kind": "oracle",
           "sample": f"first {done} unfused QFT-{n} gates on a 2^{n} FP64 state, {t_total:.1f} s",
           "host": host_description()}
    if one_core:
        # the same oracle in a child process limited to one OpenMP thread
        import subprocess
        env = dict(os.environ, OMP_NUM_THREADS="1")
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-only", "--n", str(n),
                            "--cpu-target-s", "8", "--cpu-max-gates", "2"],
                           env=env, capture_output=True, text=True, timeout=600)
        if r.returncode == 0:
            one = json.loads(r.stdout.strip().splitlines()[-1])
            out["one_core"] = {"value": one["value"], "sample": one["sample"]}
    return out


def host_description():
    """CPU model, logical CPUs and memory of the host the oracle ran on."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
        mem = next(int(l.split()[1]) for l in open("/proc/meminfo") if l.startswith("MemTotal"))
    except (OSError, StopIteration):
        mem = 0
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "mem_total_gib": round(mem / 2**20, 1)}


PROFILES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles")
CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2503_19894_amd", "csrc")
# kernel name prefix -> the source file that defines it
KERNEL_FILES = (("k_diag_run", "diagrun.hip"), ("k_blocked", "blocked.hip"), ("k_batch", "batch_kernels.hip"),
                ("k_pauli", "reduce.hip"), ("k_apply_pauli", "reduce.hip"), ("k_finish", "reduce.hip"),
                ("k_stream", "stream.hip"), ("k_", "apply.hip"))


def kernel_source(kernel):
    """The csrc file that defines `kernel` (a profiler or label name)."""
    base = kernel.replace("void ", "").replace("cast::", "").replace("(anonymous namespace)::", "")
    for prefix, f in KERNEL_FILES:
        if base.startswith(prefix):
            return f
    return "apply.hip"


def source_digest(fname):
    import hashlib
    return hashlib.sha256(open(os.path.join(CSRC, fname), "rb").read()).hexdigest()[:16]


def digest_header():
    """One line with the digest of every kernel source, for the summaries."""
    files = sorted({f for _, f in KERNEL_FILES if os.path.exists(os.path.join(CSRC, f))})
    return "# kernel_sources_sha256_16: " + ", ".join(f"{f}={source_digest(f)}" for f in files)


def traffic_summary_path(kernel, workload="qft30_c128"):
    stem = kernel.split("<")[0].replace("void ", "").replace("cast::", "")
    return os.path.join(PROFILES, f"{stem}_{workload}_hbm_traffic.txt")


def recorded_traffic(kernel, workload="qft30_c128"):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when the summary is missing or the source that defines the kernel
    changed since the counters were taken."""
    try:
        lines = open(traffic_summary_path(kernel, workload)).read().splitlines()
    except OSError:
        return None
    digests = {}
    for l in lines:
        if l.startswith("# kernel_sources_sha256_16: "):
            digests = dict(x.split("=") for x in l.split(": ", 1)[1].split(", "))
    f = kernel_source(kernel)
    if digests.get(f) != source_digest(f):
        return None
    for l in lines:
        if l.startswith(kernel + " |"):
            return float(l.split("|")[4])
    return None


def timed_region_stats(trace_csv):
    """Per-kernel statistics of the dispatches in a rocprofv3 per-dispatch
    kernel trace that lie between the first two region markers (the first
    timed region of the run), in the layout of the --stats CSV."""
    import collections
    import csv
    rows = sorted(csv.DictReader(open(trace_csv)), key=lambda r: int(r["Dispatch_Id"]))
    marks = [i for i, r in enumerate(rows) if "k_stream_scale" in r["Kernel_Name"] and int(r["Grid_Size_X"]) == 256]
    if len(marks) < 2:
        raise SystemExit(f"{trace_csv}: fewer than two region markers")
    per = collections.defaultdict(list)
    for r in rows[marks[0] + 1:marks[1]]:
        per[r["Kernel_Name"]].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    total = sum(sum(v) for v in per.values())
    out = [{"Name": k, "Calls": len(v), "AverageNs": sum(v) / len(v), "TotalDurationNs": sum(v), "MinNs": min(v),
            "MaxNs": max(v), "Percentage": 100.0 * sum(v) / total} for k, v in per.items()]
    return sorted(out, key=lambda r: -r["TotalDurationNs"])


def summarize_kernel_trace(stats_csv, command, name_filter=None):
    """Top kernels of a rocprofv3 --stats CSV, or, given the per-dispatch
    kernel trace CSV, of the first timed region's dispatches only (with
    name_filter, only kernels whose name contains it), headed by the command
    and the digests of the kernel sources."""
    import csv
    region = "Dispatch_Id" in open(stats_csv).readline()
    rows = timed_region_stats(stats_csv) if region else list(csv.DictReader(open(stats_csv)))
    if name_filter:
        rows = [r for r in rows if name_filter in r["Name"]]
    out = [f"# rocprofv3 kernel-trace summary" + (f" (kernels matching {name_filter})" if name_filter else "") +
           (" of the first timed region (dispatches between its two marker dispatches)" if region else ""),
           f"# command: {command}", digest_header(),
           f"{'kernel':78s} {'calls':>6s} {'avg_ms':>9s} {'total_ms':>10s} {'min_ms':>8s} {'max_ms':>8s} {'pct':>6s}"]
    for r in rows[:16]:
        out.append(f"{r['Name'][:78]:78s} {int(r['Calls']):6d} {float(r['AverageNs'])/1e6:9.4f} "
                   f"{float(r['TotalDurationNs'])/1e6:10.1f} {float(r['MinNs'])/1e6:8.3f} {float(r['MaxNs'])/1e6:8.3f} "
                   f"{float(r['Percentage']):6.2f}")
    return "\n".join(out)


def summarize_traffic(fetch_csv, write_csv, command_fetch, command_write):
    """Per-kernel HBM bytes per launch from FETCH_SIZE / WRITE_SIZE (KiB per
    dispatch), each scaled by what the counter reads for the 1 GiB device copy
    that --calibrate-copy runs first."""
    import csv
    import collections

    def load(path, counter):
        per = collections.defaultdict(list)
        first_copy = None
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            if first_copy is None and "copyBuffer" in r["Kernel_Name"]:
                first_copy = float(r["Counter_Value"])
            per[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        return per, first_copy

    f, fcopy = load(fetch_csv, "FETCH_SIZE")
    w, wcopy = load(write_csv, "WRITE_SIZE")
    gib_kib = float(1 << 20)
    ff, wf = gib_kib / fcopy, gib_kib / wcopy
    out = ["# HBM traffic per launch from rocprofv3 PMC counters (two runs)",
           f"# command_fetch: {command_fetch}", f"# command_write: {command_write}",
           digest_header(),
           f"# calibration: 1 GiB device copy reads FETCH_SIZE {fcopy:.1f} KiB (factor {ff:.4f}), "
           f"WRITE_SIZE {wcopy:.1f} KiB (factor {wf:.4f})",
           "# columns: kernel | launches | fetch_KiB_avg | write_KiB_avg | scaled_bytes_per_launch"]
    names = sorted(set(f) | set(w), key=lambda k: -sum(f.get(k, [0])) / max(1, len(f.get(k, [1]))))
    for name in names:
        fv, wv = f.get(name, []), w.get(name, [])
        if not fv or not wv:
            continue
        fa, wa = sum(fv) / len(fv), sum(wv) / len(wv)
        label = name.replace("(anonymous namespace)::", "").split("(")[0].replace("void cast::", "")
        out.append(f"{label} | {len(fv)} | {fa:.1f} | {wa:.1f} | {(fa * ff + wa * wf) * 1024:.0f}")
    return "\n".join(out)


def summarize_counters(counter_csv, command, kernel_filter=None):
    """Per-kernel averages of every PMC counter in a rocprofv3 --pmc CSV
    (one column per counter), headed by the command and the source digests."""
    import csv
    import collections

    per = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in csv.DictReader(open(counter_csv)):
        name = r["Kernel_Name"]
        if kernel_filter and kernel_filter not in name:
            continue
        per[name][r["Counter_Name"]].append(float(r["Counter_Value"]))
    counters = sorted({c for v in per.values() for c in v})
    out = ["# rocprofv3 PMC counters, average per dispatch", f"# command: {command}", digest_header(),
           "# columns: kernel | dispatches | " + " | ".join(counters)]
    for name, v in sorted(per.items(), key=lambda kv: -len(next(iter(kv[1].values())))):
        label = name.replace("(anonymous namespace)::", "").split("(")[0].replace("void cast::", "")
        n = max(len(x) for x in v.values())
        out.append(f"{label} | {n} | " + " | ".join(f"{sum(v[c]) / len(v[c]):.1f}" if v.get(c) else "-"
                                                   for c in counters))
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=30)
    ap.add_argument("--k-max", type=int, default=5)
    ap.add_argument("--tune-reps", type=int, default=3,
                    help="launches per candidate shape when tuning the QFT's passes (0: knob shapes)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c64", action="store_true")
    ap.add_argument("--no-vqa", action="store_true")
    ap.add_argument("--vqa-only", action="store_true", help="only the batched VQA measurement")
    ap.add_argument("--vqa-profile", action="store_true",
                    help="only one complex128 VQA batch in graph mode (the profiled command)")
    ap.add_argument("--no-dense", action="store_true")
    ap.add_argument("--no-tfim", action="store_true")
    ap.add_argument("--tfim-only", action="store_true", help="only the mixed-size TFIM batch")
    ap.add_argument("--dense-only", action="store_true", help="only the 32-qubit dense circuit")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one device copy of exactly 1 GiB (reference for HBM byte counters)")
    ap.add_argument("--summarize-kernel-trace", nargs="+", metavar="STATS_CSV COMMAND [NAME_FILTER]")
    ap.add_argument("--jit", action="store_true",
                    help="only the generated-kernel comparison (paper's single-gate table workload, QFT-30)")
    ap.add_argument("--families", action="store_true",
                    help="only the circuit-family table (fusion none / size-only / adaptive, per pass and "
                         "cache-blocked); prints one JSON object")
    ap.add_argument("--summarize-counters", nargs="+", metavar="PMC_CSV COMMAND [KERNEL_FILTER]")
    ap.add_argument("--summarize-traffic", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "CMD_FETCH", "CMD_WRITE"))
    ap.add_argument("--sweep", action="store_true",
                    help="only the single-pass sweep (k = 1..6 x six gate kinds x three placements, 28 and 30 "
                         "qubits, both dtypes); prints one JSON object")
    ap.add_argument("--cpu-baseline-only", action="store_true",
                    help="only the oracle's CPU baseline (no GPU); prints one JSON object")
    ap.add_argument("--cpu-target-s", type=float, default=15.0)
    ap.add_argument("--cpu-max-gates", type=int, default=8)
    args = ap.parse_args()
    if args.cpu_baseline_only:
        print(json.dumps(cpu_baseline(args.n, args.cpu_target_s, args.cpu_max_gates, one_core=False)), flush=True)
        return
    if args.summarize_kernel_trace:
        print(summarize_kernel_trace(*args.summarize_kernel_trace))
        return
    if args.summarize_counters:
        print(summarize_counters(*args.summarize_counters))
        return
    if args.summarize_traffic:
        print(summarize_traffic(*args.summarize_traffic))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the state-vector path here is built and measured on a single "
              "MI355X; runs on more than one GPU are not supported.", file=sys.stderr)
        sys.exit(2)
    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        # one device copy of exactly 1 GiB: the reference the HBM byte
        # counters of the profiled kernels are scaled by
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.tfim_only:
        print(json.dumps(run_tfim(oracle_check=False)), flush=True)
        return
    if args.dense_only:
        print(json.dumps(run_dense()), flush=True)
        return
    if args.vqa_profile:
        print(json.dumps(run_vqa_profile()), flush=True)
        return
    if args.vqa_only:
        print(json.dumps(run_vqa(oracle_check=False)), flush=True)
        return
    if args.families:
        print(json.dumps(run_families(args.n)), flush=True)
        return
    if args.jit:
        print(json.dumps(run_jit()), flush=True)
        return
    if args.sweep:
        print(json.dumps({"sweep": run_sweep()}), flush=True)
        return
    def progress(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    progress("qft complex128")
    main_run = run_gpu(args.n, args.k_max, "c128", args.steps, args.warmup, tune_reps=args.tune_reps)
    extras = {}
    if not args.no_c64:
        progress("qft complex64")
        extras["c64"] = run_gpu(args.n, args.k_max, "c64", args.steps, args.warmup, tune_reps=args.tune_reps)
    progress("qft complex64 error against complex128")
    c64_err = None if args.no_c64 else qft_c64_error(args.n, args.k_max)
    dom = main_run["kernels"][main_run["dominant"]]
    traffic = recorded_traffic(main_run["dominant"])
    copy_gbs, copy_kind, copy_all = copy_bandwidth()
    roof = {"bound": "hbm", "kernel": main_run["dominant"], "achieved": round(dom["achieved_gbs"], 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(dom["achieved_gbs"] / HBM_PEAK_GBS, 4),
            "traffic": traffic, "avg_launch_ms": round(dom["avg_launch_ms"], 4),
            "alg_bytes_per_launch": dom["alg_bytes_per_launch"],
            "copy_gbs": round(copy_gbs, 1), "copy_kind": copy_kind, "streaming_rates_gbs": copy_all,
            "frac_of_copy": round(dom["achieved_gbs"] / copy_gbs, 4)}
    if traffic:
        # HBM bytes actually moved per launch over the launch time, against the copy rate
        roof["traffic_gbs"] = round(traffic / (dom["avg_launch_ms"] * 1e-3) / 1e9, 1)
        roof["traffic_frac_of_copy"] = round(roof["traffic_gbs"] / copy_gbs, 4)
    progress("batched vqa")
    vqa = None if args.no_vqa else run_vqa(oracle_check=not args.no_cpu_baseline)
    progress("dense 32-qubit circuit")
    dense = None if args.no_dense else run_dense()
    progress("mixed-size tfim batch")
    tfim = None if args.no_tfim else run_tfim(oracle_check=not args.no_cpu_baseline)
    progress("cpu baseline (oracle)")
    cpu = None if args.no_cpu_baseline else cpu_baseline(args.n)
    line = {
        "metric": "effective HBM GB/s per fused-gate pass at 30q",
        "value": round(main_run["alg_gbs"], 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_run["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"qft{args.n}_complex128_kmax{args.k_max}", "n_qubits": args.n,
                   "k_max": args.k_max, "fused_gates": main_run["fused_gates"], "passes": main_run["passes"],
                   "state_bytes": (1 << args.n) * 16},
        "roofline": roof,
        "c64_error_vs_fp64": c64_err,
        "cpu_baseline": cpu,
        "vqa_grads_per_s": None if vqa is None else vqa_summary(vqa),
        "blocked": {d: {"ms_per_step": round(r["blocked"]["ms_per_step"], 3), "hbm_passes": r["blocked"]["hbm_passes"],
                        "speedup_vs_per_pass": round(r["blocked"]["speedup_vs_per_pass"], 3)}
                    for d, r in (("c128", main_run), ("c64", extras.get("c64"))) if r},
        "extras": {"c128": main_run, **extras, "vqa": vqa, "dense32": dense, "tfim_mixed": tfim},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
