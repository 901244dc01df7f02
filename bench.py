#!/usr/bin/env python3
"""Throughput of the sliced contraction hot path on one MI355X.

Workload: the 5x6-qubit (30 qubits), 14-cycle random lattice circuit
(sqrt-X/Y/W + fSim(pi/2, pi/6), ABCD couplers, seed 1001), 64 amplitudes
(qubits 24-29 open, the other 24 output bits fixed at random, seed 2001),
randomised-greedy path with the largest intermediate <= 2^26 entries and 8
sliced indices (256 slices), complex64 storage with FP32 MFMA arithmetic and
an FP64 cross-slice sum.  One step = all 256 slices (the whole sliced tree),
inputs resident in HBM.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "slices/s + % MFMA peak, complex64 vs scaled complex-FP16 at stated amp error"
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
CLASS_NAMES = ["small", "stem", "tile", "tall", "splitk"]
MFMA_CLASSES = (2, 3)


def workload():
    import synth
    c = synth.lattice_circuit(5, 6, 14, seed=1001)
    spec = synth.output_spec(30, list(range(24, 30)), seed=2001)
    return c, spec


def cpu_baseline(c, spec, path, sliced, seconds: float):
    """The FP64 oracle, as it stands, on the same path and slicing: slices
    0, 1, 2, ... until about `seconds` of host time are spent."""
    import numpy as np

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
        cores = max(int(i.get("num_threads", 1)) for i in threadpool_info()) if threadpool_info() else 1
    except Exception:
        cores = os.cpu_count() or 1
    del np
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
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(slices would be sharded by their outer sliced indices, one FP64 all-reduce at the end).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2504_09186_amd import tnc
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    c, spec = workload()
    net = tnc.Network(c, spec)
    net.path_search(seed=3001, trials=args.trials, max_log2=26, min_sliced=8, max_sliced=8)
    plan = tnc.Plan(net)
    st = plan.stats
    n_slices = plan.n_slices
    plan.upload()
    acc = plan.new_result()

    for _ in range(args.warmup):
        acc.zero_()
        plan.execute(acc)
    # one untimed step with event timing on allocates the event pool
    plan.timing(True)
    acc.zero_()
    plan.execute(acc)
    torch.cuda.synchronize()
    plan.timing(True)  # reset: record the timed region only

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        acc.zero_()
        plan.execute(acc)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms, launches, flops, nbytes = plan.timing_read()
    plan.timing(False)

    slices_per_s = n_slices * args.steps / el
    dom = int(max(range(5), key=lambda k: ms[k]))
    if dom in MFMA_CLASSES:
        achieved = flops[dom] / (ms[dom] * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_MFMA_TFLOPS, "traffic": None}
    else:
        achieved = nbytes[dom] / (ms[dom] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS, "traffic": None}
    roof["kernel"] = CLASS_NAMES[dom]
    roof["launches"] = int(launches[dom])
    roof["avg_launch_ms"] = ms[dom] / max(1.0, launches[dom])
    total_flops = st.flops_reused_slice * n_slices * args.steps
    out = {
        "metric": METRIC, "value": slices_per_s, "unit": "slices/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": "rqc-5x6-14cyc-64amp-256slices", "qubits": 30, "cycles": 14,
                   "open_qubits": 6, "slices_per_step": n_slices, "max_log2_elems": st.max_log2_elems,
                   "steps_per_slice": st.n_steps, "flops_per_slice": st.flops_reused_slice,
                   "precision": "complex64, FP32 MFMA, FP64 cross-slice sum"},
        "tflops": total_flops / el / 1e12,
        "mfma_frac": total_flops / el / 1e12 / PEAK_FP32_MFMA_TFLOPS,
        "kernel_ms_by_class": {CLASS_NAMES[k]: ms[k] / args.steps for k in range(5)},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(c, spec, net.path(), net.slicing(), args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
