#!/usr/bin/env python3
"""Throughput of the sliced contraction hot path on one MI355X.

Workload: the 5x6-qubit (30 qubits), 14-cycle random lattice circuit
(sqrt-X/Y/W + fSim(pi/2, pi/6), ABCD couplers, seed 1001), 64 amplitudes
(qubits 24-29 open, the other 24 output bits fixed at random, seed 2001),
randomised-greedy path with the largest intermediate <= 2^26 entries and 8
sliced indices (256 slices).  One step = all 256 slices (the whole sliced
tree, FP64 cross-slice sum), inputs resident in HBM.

Two forms are timed on the same plan: complex64 (FP32 MFMA; the headline
`value`) and scaled complex FP16 (FP16 MFMA, FP32 accumulate, per-tensor
power-of-two exponents calibrated on slices 0-1), each with its amplitude
error against the oracle's values stored in tests/golden.  Prints one JSON
line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "slices/s + % MFMA peak, complex64 vs scaled complex-FP16 at stated amp error"
PEAK_FP32 = 157.3   # dense MFMA (and vector) TFLOP/s, FP32
PEAK_FP16 = 2500.0  # dense MFMA TFLOP/s, FP16
PEAK_HBM_GBS = 8000.0
CLASS_NAMES = ["small", "stem", "tile", "tall", "splitk", "stream", "section"]


def class_peak(label, cls):
    """Compute peak of the units a kernel class runs on: the FP16 form's tile
    and stream kernels use FP16 MFMA; everything else computes in FP32."""
    return PEAK_FP16 if label == "cf16" and cls in (2, 3, 4, 5) else PEAK_FP32
GOLDEN = os.path.join(ROOT, "tests", "golden", "config2_amplitudes.json")


def workload():
    import synth
    c = synth.lattice_circuit(5, 6, 14, seed=1001)
    spec = synth.output_spec(30, list(range(24, 30)), seed=2001)
    return c, spec


def golden_amplitudes():
    import numpy as np
    if not os.path.exists(GOLDEN):
        return None
    with open(GOLDEN) as f:
        g = json.load(f)
    return np.array([a + 1j * b for a, b in g["amplitudes"]])


def amp_error(got, ref):
    import oracle
    if ref is None:
        return None
    return {"rel_l2": oracle.rel_l2(got, ref), "overlap": oracle.overlap_fidelity(got, ref),
            "xeb_loss": abs(1.0 - oracle.xeb_ratio(got, ref)), "against": "FP64 oracle, all 64 amplitudes"}


TRAFFIC = os.path.join(ROOT, "profiles", "traffic.json")


def measured_traffic(label, kernel):
    """HBM bytes per launch of the dominant kernel from the committed
    FETCH_SIZE/WRITE_SIZE counters, or None when they do not apply: another
    kernel or form, or kernel sources changed since the counters were taken."""
    import hashlib
    if kernel != "stream" or not os.path.exists(TRAFFIC):
        return None
    with open(TRAFFIC) as f:
        rec = json.load(f)
    h = hashlib.sha256()
    for rel in ("paper_2504_09186_amd/csrc/kernels.hip", "paper_2504_09186_amd/csrc/step.hpp"):
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec.get("kernels_sha256"):
        return None
    return rec.get(f"stream_{label}_bytes_per_launch")


def run_form(net, precision, steps, warmup, label):
    import torch

    from paper_2504_09186_amd import tnc
    plan = tnc.Plan(net, precision=precision)
    st = plan.stats
    n_slices = plan.n_slices
    plan.upload()
    if precision != 0:
        plan.calibrate(0, 2)
    acc = plan.new_result()
    for _ in range(warmup):
        acc.zero_()
        plan.execute(acc)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        acc.zero_()
        plan.execute(acc)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    result = acc.cpu().numpy()
    # Kernel durations: the same steps again with a hipEvent pair around every
    # launch (the events add host-side launch cost, so `value` above is taken
    # without them).
    plan.timing(True)
    acc.zero_()
    plan.execute(acc)  # allocates the event pool
    torch.cuda.synchronize()
    plan.timing(True)
    for _ in range(steps):
        acc.zero_()
        plan.execute(acc)
    torch.cuda.synchronize()
    ms, launches, flops, nbytes = plan.timing_read()
    plan.timing(False)
    overflow = None
    if precision != 0:
        overflow = bool(float(plan.step_maxima().max()) >= 65504.0)
    nc = len(CLASS_NAMES)
    dom = int(max(range(nc), key=lambda k: ms[k]))
    # Bound of the dominant kernel: its arithmetic intensity against the
    # ridge point peak_flops / peak_bandwidth.
    peak = class_peak(label, dom)
    ai = flops[dom] / max(nbytes[dom], 1.0)
    if ai >= peak * 1e12 / (PEAK_HBM_GBS * 1e9):
        achieved = flops[dom] / (ms[dom] * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": None}
    else:
        achieved = nbytes[dom] / (ms[dom] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS, "traffic": None}
    roof["flop_per_byte"] = ai
    roof["kernel"] = CLASS_NAMES[dom]
    roof["algorithmic_bytes_per_launch"] = nbytes[dom] / max(1.0, launches[dom])
    roof["traffic"] = measured_traffic(label, CLASS_NAMES[dom])
    roof["launches"] = int(launches[dom])
    roof["avg_launch_ms"] = ms[dom] / max(1.0, launches[dom])
    total_flops = st.flops_reused_slice * n_slices * steps
    total_bytes = sum(nbytes[:nc])
    return {
        "value": n_slices * steps / el, "unit": "slices/s", "ms_per_step": el / steps * 1e3,
        "tflops": total_flops / el / 1e12, "hbm_gbs": total_bytes / el / 1e9,
        "mfma_frac": total_flops / el / 1e12 / (PEAK_FP16 if label == "cf16" else PEAK_FP32),
        "kernel_ms_by_class": {CLASS_NAMES[k]: ms[k] / steps for k in range(nc)},
        "roofline": roof, "n_slices": n_slices, "stats": st, "result": result, "fp16_overflow": overflow,
    }


def grad_timing(steps):
    """Differentiation form: 6x6 lattice, 8 cycles, 256 random bitstrings as a
    batch index (seeds 1003 / 2003 / 3003), intermediates <= 2^32 entries with
    the batch bits.  Times the forward over all slices and the backward (per
    slice: forward recompute, reverse pass, gate-gradient accumulation) with
    w = 1 / a, the holomorphic seed of L = sum log|a|^2."""
    import numpy as np
    import torch

    import synth
    from paper_2504_09186_amd import tnc
    c = synth.lattice_circuit(6, 6, 8, seed=1003)
    bits = synth.random_bitstrings(36, 256, seed=2003)
    spec = np.full(36, -2, dtype=np.int8)
    net = tnc.Network(c, spec, bits)
    net.path_search(seed=3003, trials=32, max_log2=32)
    plan = tnc.Plan(net, differentiable=True)
    plan.upload()
    acc = plan.new_result()
    plan.execute(acc)
    w = (1.0 / acc).contiguous()
    grad = torch.zeros(4 * plan.stats.n_grad_gates, dtype=torch.complex128, device=acc.device)
    plan.backward(w, grad)  # warmup
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        acc.zero_()
        plan.execute(acc)
    torch.cuda.synchronize()
    fwd = (time.perf_counter() - t0) / steps
    t0 = time.perf_counter()
    for _ in range(steps):
        grad.zero_()
        plan.backward(w, grad)
    torch.cuda.synchronize()
    bwd = (time.perf_counter() - t0) / steps
    st = plan.stats
    return {"workload": "rqc-6x6-8cyc-256bitstrings-grad", "slices": plan.n_slices,
            "forward_ms": fwd * 1e3, "backward_ms": bwd * 1e3, "backward_over_forward": bwd / fwd,
            "forward_flops": st.flops_full_slice * plan.n_slices,
            "reverse_flops": st.flops_reverse_slice * plan.n_slices, "n_grad_gates": st.n_grad_gates,
            "finite": bool(torch.isfinite(torch.view_as_real(grad)).all())}


def cpu_baseline(c, spec, path, sliced, seconds: float):
    """The FP64 oracle, as it stands, on the same path and slicing: slices
    0, 1, 2, ... until about `seconds` of host time are spent."""
    import oracle
    onet = oracle.build_network(c, spec)
    done = 0
    t0 = time.perf_counter()
    while True:
        oracle.contract_sliced(onet, path, sliced, slice_ids=[done])
        done += 1
        if time.perf_counter() - t0 >= seconds:
            break
    el = time.perf_counter() - t0
    try:
        from threadpoolctl import threadpool_info
        info = threadpool_info()
        cores = max(int(i.get("num_threads", 1)) for i in info) if info else 1
    except Exception:
        cores = os.cpu_count() or 1
    return {"value": done / el, "unit": "slices/s", "cores": cores, "kind": "oracle",
            "sample": f"slices 0..{done - 1} of the same 256-slice workload, same path and sliced "
                      f"indices, numpy complex128 ({el:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--trials", type=int, default=64, help="path-search trials")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp16", action="store_true")
    ap.add_argument("--grad", action="store_true",
                    help="only time the differentiation form (forward vs backward over all slices) and exit")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-MiB device buffer 3 times (reference for HBM byte counters) and exit")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        src = torch.ones(args.copy_probe << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_mib": args.copy_probe, "copies": 3}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(slices would be sharded by their outer sliced indices, one FP64 all-reduce at the end).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2504_09186_amd import tnc
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.grad:
        print(json.dumps(grad_timing(args.steps)), flush=True)
        return
    c, spec = workload()
    net = tnc.Network(c, spec)
    net.path_search(seed=3001, trials=args.trials, max_log2=26, min_sliced=8, max_sliced=8)
    ref = golden_amplitudes()

    r64 = run_form(net, 0, args.steps, args.warmup, "c64")
    st = r64["stats"]
    out = {
        "metric": METRIC, "value": r64["value"], "unit": "slices/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": "rqc-5x6-14cyc-64amp-256slices", "qubits": 30, "cycles": 14,
                   "open_qubits": 6, "slices_per_step": r64["n_slices"], "max_log2_elems": st.max_log2_elems,
                   "steps_per_slice": st.n_steps, "flops_per_slice": st.flops_reused_slice,
                   "precision": "complex64, FP32 MFMA (3M), FP64 cross-slice sum"},
        "tflops": r64["tflops"], "mfma_frac": r64["mfma_frac"], "hbm_gbs": r64["hbm_gbs"],
        "amp_error": amp_error(r64["result"], ref),
        "kernel_ms_by_class": r64["kernel_ms_by_class"],
        "roofline": r64["roofline"],
    }
    if not args.no_fp16:
        r16 = run_form(net, 1, args.steps, args.warmup, "cf16")
        out["cf16"] = {"value": r16["value"], "unit": "slices/s", "ms_per_step": r16["ms_per_step"],
                       "tflops": r16["tflops"], "mfma_frac": r16["mfma_frac"], "hbm_gbs": r16["hbm_gbs"],
                       "amp_error": amp_error(r16["result"], ref), "fp16_overflow": r16["fp16_overflow"],
                       "kernel_ms_by_class": r16["kernel_ms_by_class"], "roofline": r16["roofline"],
                       "precision": "complex FP16 storage, FP16 MFMA (4M) with FP32 accumulate, "
                                    "per-tensor 2^e scaling, FP64 cross-slice sum"}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(c, spec, net.path(), net.slicing(), args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
