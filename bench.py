#!/usr/bin/env python3
"""Throughput of the sliced contraction hot path on one MI355X.

Headline workload (the metric's configuration): a 7x8-qubit (56 qubits),
20-cycle random lattice circuit (sqrt-X/Y/W + fSim(pi/2, pi/6), ABCD couplers,
seed 1004), qubits 44-55 open (2^12 amplitudes), the other 44 output bits
fixed at random (seed 2004); the library's recursive-bisection path search
(seed 3004) with every intermediate <= 2^30 entries; one GPU's share of 256
slices (the 8 innermost sliced indices vary, the outer ones are 0).  One step
= those 256 slices (shared-prefix reuse across them, FP64 cross-slice sum),
inputs resident in HBM.

Two forms run on the same path and slicing: complex64 (FP32 MFMA; the
headline `value`) and scaled complex FP16 (FP16 MFMA, FP32 accumulate,
per-tensor power-of-two exponents calibrated on slices 0-1, re-run on an
exponent miss).  Errors are reported against the FP64 oracle's stored
sub-slice results (the oracle's own 60-index slicing of the same network,
computed by tests/golden/make_golden_config4.py) and, for the FP16 form,
against the complex64 result of the 256 slices.  Also reported: the 5x6-qubit
14-cycle workload (64 amplitudes, 256 slices) and the differentiation form
(forward vs backward time).  Prints one JSON line.
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
CLASS_NAMES = ["small", "stem", "tile", "tall", "splitk", "stream", "section", "merge"]


def class_peak(label, cls):
    """Compute peak of the units a kernel class runs on: the FP16 form's tile
    and stream kernels use FP16 MFMA; everything else computes in FP32."""
    return PEAK_FP16 if label == "cf16" and cls in (2, 3, 4, 5) else PEAK_FP32


def executed_fraction(label, cls):
    """Real flops the MFMA executes per flop of the 4M count (8 M K N): the
    complex64 tile, tall and stream kernels run the 3M split (three real
    products instead of four); the FP16/BF16 kernels run the 4M split as one
    real GEMM."""
    return 0.75 if label == "c64" and cls in (2, 3, 5) else 1.0
GOLDEN2 = os.path.join(ROOT, "tests", "golden", "config2_amplitudes.json")
GOLDEN4 = os.path.join(ROOT, "tests", "golden", "config4_subslices.json")
# Stored path and slicing of the headline network (written by
# paper_2504_09186_amd/paths/make_paths.py: recursive-bisection search, 1024
# trials, 48 sliced indices, ranked by the flops of all slices dealt in
# 256-slice shares, then branch exchange; its plans merge the 8 inner
# slice-id bits where nested).
PATH4 = os.path.join(ROOT, "paper_2504_09186_amd", "paths", "rqc_7x8_20.json")
# The same network with fewer, larger slices (1024 trials; 44 sliced indices).
PATH4_S44 = os.path.join(ROOT, "paper_2504_09186_amd", "paths", "rqc_7x8_20_s44.json")
WORKLOAD4 = "rqc-7x8-20cyc-4096amp-256slice-share"
WORKLOAD2 = "rqc-5x6-14cyc-64amp-256slices"


def workload4():
    import synth
    c = synth.lattice_circuit(7, 8, 20, seed=1004)
    spec = synth.output_spec(56, list(range(44, 56)), seed=2004)
    return c, spec


def workload2():
    import synth
    c = synth.lattice_circuit(5, 6, 14, seed=1001)
    spec = synth.output_spec(30, list(range(24, 30)), seed=2001)
    return c, spec


def load_json(path):
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def to_complex(v):
    import numpy as np
    return np.array([a + 1j * b for a, b in v])


def error_metrics(got, ref, against):
    import oracle
    return {"rel_l2": oracle.rel_l2(got, ref), "overlap": oracle.overlap_fidelity(got, ref),
            "xeb_loss": abs(1.0 - oracle.xeb_ratio(got, ref)), "against": against}


TRAFFIC = os.path.join(ROOT, "profiles", "traffic.json")


def measured_traffic(workload, label, kernel):
    """HBM bytes per launch of the dominant kernel from the committed
    FETCH_SIZE/WRITE_SIZE counters, or None when they do not apply: another
    workload, kernel or form, or kernel sources changed since the counters
    were taken."""
    import hashlib
    rec = load_json(TRAFFIC)
    if rec is None:
        return None
    h = hashlib.sha256()
    for rel in ("paper_2504_09186_amd/csrc/kernels.hip", "paper_2504_09186_amd/csrc/step.hpp"):
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec.get("kernels_sha256"):
        return None
    return rec.get(f"{workload}:{kernel}:{label}")


def run_form(plan, steps, warmup, label, workload, s0=0, s1=None):
    """Times `steps` executions of slices [s0, s1) after `warmup` untimed
    ones, then repeats them with per-launch event timing for the kernel
    classes.  Returns the throughput record and the last result."""
    import torch
    st = plan.stats
    s1 = plan.n_slices if s1 is None else s1
    n_slices = s1 - s0
    acc = plan.new_result()
    for _ in range(warmup):
        acc.zero_()
        plan.execute(acc, s0, s1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        acc.zero_()
        plan.execute(acc, s0, s1)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    result = acc.cpu().numpy()
    # Kernel durations: the same steps again with a hipEvent pair around every
    # launch (the events add host-side launch cost, so `value` is taken
    # without them).
    plan.timing(True)
    acc.zero_()
    plan.execute(acc, s0, s1)  # allocates the event pool
    torch.cuda.synchronize()
    plan.timing(True)
    for _ in range(steps):
        acc.zero_()
        plan.execute(acc, s0, s1)
    torch.cuda.synchronize()
    ms, launches, flops, nbytes = plan.timing_read()
    plan.timing(False)
    nc = len(CLASS_NAMES)
    dom = int(max(range(nc), key=lambda k: ms[k]))
    # Bound of the dominant kernel: its arithmetic intensity against the
    # ridge point peak_flops / peak_bandwidth.
    peak = class_peak(label, dom)
    ai = flops[dom] / max(nbytes[dom], 1.0)
    if ai >= peak * 1e12 / (PEAK_HBM_GBS * 1e9):
        # executed MFMA flops against the dense peak of their type
        achieved = flops[dom] * executed_fraction(label, dom) / (ms[dom] * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": None, "achieved_4m_count": flops[dom] / (ms[dom] * 1e-3) / 1e12}
    else:
        achieved = nbytes[dom] / (ms[dom] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS, "traffic": None}
    roof["flop_per_byte"] = ai
    roof["kernel"] = CLASS_NAMES[dom]
    roof["algorithmic_bytes_per_launch"] = nbytes[dom] / max(1.0, launches[dom])
    roof["algorithmic_flops_per_launch"] = flops[dom] / max(1.0, launches[dom])
    roof["traffic"] = measured_traffic(workload, label, CLASS_NAMES[dom])
    roof["launches"] = int(launches[dom])
    roof["avg_launch_ms"] = ms[dom] / max(1.0, launches[dom])
    # algorithmic contraction flops of one step's launches (the merge
    # additions are not contractions)
    step_flops = float(sum(flops[k] for k in range(nc) if CLASS_NAMES[k] != "merge")) / steps
    total_bytes = sum(nbytes[:nc])
    overflow = None
    if plan.stats is not None and label != "c64":
        overflow = bool(float(plan.step_maxima().max()) >= 65504.0)
    rec = {
        "value": n_slices * steps / el, "unit": "slices/s", "ms_per_step": el / steps * 1e3,
        "tflops": step_flops * steps / el / 1e12, "hbm_gbs": total_bytes / el / 1e9,
        "flops_per_step": step_flops,
        "kernel_ms_by_class": {CLASS_NAMES[k]: ms[k] / steps for k in range(nc)},
        "kernel_tflops_by_class": {CLASS_NAMES[k]: (flops[k] / (ms[k] * 1e-3) / 1e12 if ms[k] > 0 else 0.0)
                                   for k in range(nc)},
        "roofline": roof, "n_slices": n_slices, "fp16_overflow": overflow,
        "exponent_reruns": plan.exponents()[1] if label != "c64" else None,
    }
    return rec, result


def grad_config3(steps, n_slices=32):
    """Differentiation form on the gradient configuration itself: 6x6
    lattice, 16 cycles, 256 random bitstrings as a batch index (seeds 1003 /
    2003 / 3003), intermediates <= 2^30 entries with the batch bits
    (bisection search, 16 trials: 13 sliced indices, 8192 slices; the
    differentiable plan keeps every node, about 70 GiB).  A sub-batch of the
    slices is timed: slices 0 .. n_slices-1, forward over the range (with
    shared-prefix reuse) and backward over the same range, seeded with
    w = 1 / (the range's partial amplitudes); the full gradient sums every
    range."""
    import numpy as np
    import torch

    import synth
    from paper_2504_09186_amd import tnc
    c = synth.lattice_circuit(6, 6, 16, seed=1003)
    bits = synth.random_bitstrings(36, 256, seed=2003)
    spec = np.full(36, -2, dtype=np.int8)
    net = tnc.Network(c, spec, bits)
    net.path_search(seed=3003, trials=16, max_log2=30, method=1, max_sliced=30)
    plan = tnc.Plan(net, differentiable=True)
    plan.upload()
    acc = plan.new_result()
    n = min(n_slices, plan.n_slices)
    plan.execute(acc, 0, n)
    w = (1.0 / acc).contiguous()
    grad = torch.zeros(4 * plan.stats.n_grad_gates, dtype=torch.complex128, device=acc.device)
    plan.backward(w, grad, 0, n)  # warmup
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        acc.zero_()
        plan.execute(acc, 0, n)
    torch.cuda.synchronize()
    fwd = (time.perf_counter() - t0) / steps
    t0 = time.perf_counter()
    for _ in range(steps):
        grad.zero_()
        plan.backward(w, grad, 0, n)
    torch.cuda.synchronize()
    bwd = (time.perf_counter() - t0) / steps
    st = plan.stats
    out = {"workload": "rqc-6x6-16cyc-256bitstrings-grad-cap30", "slices_total": plan.n_slices,
           "slices_timed": n, "n_sliced": st.n_sliced, "max_log2_elems": st.max_log2_elems,
           "workspace_gib": st.workspace_bytes / 2 ** 30,
           "forward_ms": fwd * 1e3, "backward_ms": bwd * 1e3, "backward_over_forward": bwd / fwd,
           "reverse_flops_per_slice": st.flops_reverse_slice, "forward_flops_per_slice_reused": st.flops_reused_slice,
           "n_grad_gates": st.n_grad_gates, "finite": bool(torch.isfinite(torch.view_as_real(grad)).all())}
    del plan
    torch.cuda.empty_cache()
    return out


def alt_path_timing(c, spec, steps, warmup):
    """Complex64 share of the 56-qubit network on the stored 44-index path:
    slices/s and the projected time of all its slices on one GPU, against
    which the headline path's projection compares (slices/s alone does not:
    slice sizes differ between paths)."""
    import torch

    from paper_2504_09186_amd import tnc
    stored = load_json(PATH4_S44)
    if stored is None:
        return None
    net = tnc.Network(c, spec)
    net.set_path([tuple(x) for x in stored["path"]])
    net.set_slicing(stored["slicing"])
    plan = tnc.Plan(net, precision=0, merge_bits=stored.get("merge_bits", 0))
    plan.upload()
    r, _ = run_form(plan, steps, warmup, "c64", WORKLOAD4, 0, 256)
    S = plan.stats.n_sliced
    out = {"path": "stored: recursive bisection, 1024 trials, sliced indices as the 2^30 cap needs, then branch "
                   "exchange", "n_sliced": S,
           "value": r["value"], "unit": "slices/s", "ms_per_step": r["ms_per_step"],
           "job_seconds_projected": r["ms_per_step"] * 1e-3 * 2.0 ** (S - 8),
           "job_flops": r["flops_per_step"] * 2.0 ** (S - 8), "roofline": r["roofline"],
           "kernel_ms_by_class": r["kernel_ms_by_class"]}
    del plan
    torch.cuda.empty_cache()
    return out


def subslice_check(c, spec, g, precision):
    """The oracle's stored sub-slices (its own slicing of the same network),
    recomputed with the library's path for that slicing."""
    import numpy as np
    import torch

    from paper_2504_09186_amd import tnc
    net = tnc.Network(c, spec)
    lab = g["oracle_sliced_labels"]
    net.set_slicing(lab)
    net.path_search(seed=3004, trials=8, max_log2=30, min_sliced=len(lab), max_sliced=62, keep_slicing=True,
                    method=1)
    extra = len(net.slicing()) - len(lab)
    plan = tnc.Plan(net, precision=precision)
    plan.upload()
    gots, refs = [], []
    for sid in g["sub_slice_ids"]:
        s0, s1 = sid << extra, (sid + 1) << extra
        if precision:
            plan.calibrate(s0, min(s1, s0 + 2))
        acc = plan.new_result()
        plan.execute(acc, s0, s1)
        torch.cuda.synchronize()
        gots.append(acc.cpu().numpy())
        refs.append(to_complex(g["sub_slice_results"][str(sid)]))
    del plan
    torch.cuda.empty_cache()
    # metrics per sub-slice (each its own result set of 2^12 amplitudes); the worst is reported
    per = [error_metrics(a, b, "") for a, b in zip(gots, refs)]
    worst = {k: max(p[k] for p in per) for k in ("rel_l2", "xeb_loss")}
    worst["overlap"] = min(p["overlap"] for p in per)
    worst["against"] = (f"FP64 oracle, worst of {len(gots)} sub-slices of its own {len(lab)}-index slicing "
                        f"(2^12 amplitudes each)")
    return worst


def grad_timing(steps, cap=28):
    """Differentiation form: 6x6 lattice, 8 cycles, 256 random bitstrings as a
    batch index (seeds 1003 / 2003 / 3003), intermediates <= 2^28 entries with
    the batch bits (greedy and bisection search; the path found needs no
    sliced index at this cap).  Times the forward over all slices and the
    backward (per slice: forward recompute unless the workspace still holds
    that slice's values, reverse pass, gate-gradient accumulation) with
    w = 1 / a, the holomorphic seed of L = sum log|a|^2."""
    import numpy as np
    import torch

    import synth
    from paper_2504_09186_amd import tnc
    c = synth.lattice_circuit(6, 6, 8, seed=1003)
    bits = synth.random_bitstrings(36, 256, seed=2003)
    spec = np.full(36, -2, dtype=np.int8)
    net = tnc.Network(c, spec, bits)
    net.path_search(seed=3003, trials=16, max_log2=cap, method=2)
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
    return {"workload": f"rqc-6x6-8cyc-256bitstrings-grad-cap{cap}", "slices": plan.n_slices,
            "max_log2_elems": st.max_log2_elems,
            "forward_ms": fwd * 1e3, "backward_ms": bwd * 1e3, "backward_over_forward": bwd / fwd,
            "forward_flops": st.flops_full_slice * plan.n_slices,
            "reverse_flops": st.flops_reverse_slice * plan.n_slices, "n_grad_gates": st.n_grad_gates,
            "finite": bool(torch.isfinite(torch.view_as_real(grad)).all())}


def cpu_baseline_subslice(c, spec, g, gpu_flops_per_slice):
    """The FP64 oracle, as it stands, on a bounded sample of the same
    network: one sub-slice of its own 62-index slicing (stored path), timed
    on the host's cores; its flop rate is converted to slices/s of the GPU
    plan's executed flops per slice."""
    import oracle
    onet = oracle.build_network(c, spec)
    path = [tuple(p) for p in g["oracle_path"]]
    sl = g["cpu_sample_sliced_labels"]
    t0 = time.perf_counter()
    oracle.contract_sliced(onet, path, sl, slice_ids=[0])
    el = time.perf_counter() - t0
    rate = g["cpu_sample_flops"] / el
    return {"value": rate / gpu_flops_per_slice, "unit": "slices/s", "cores": _host_threads(), "kind": "oracle",
            "sample": f"one sub-slice of the oracle's own {len(sl)}-index slicing of the same 56-qubit network "
                      f"({g['cpu_sample_flops']:.3e} flops in {el:.1f} s = {rate / 1e9:.1f} GFLOP/s, numpy "
                      f"complex128), converted at the GPU plan's {gpu_flops_per_slice:.3e} executed flops per "
                      f"slice", "host": _host_info()}


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
    return {"value": done / el, "unit": "slices/s", "cores": _host_threads(), "kind": "oracle",
            "sample": f"slices 0..{done - 1} of the same 256-slice workload, same path and sliced "
                      f"indices, numpy complex128 ({el:.1f} s)", "host": _host_info()}


def _host_threads():
    try:
        from threadpoolctl import threadpool_info
        info = threadpool_info()
        return max(int(i.get("num_threads", 1)) for i in info) if info else 1
    except Exception:
        return os.cpu_count() or 1


def _host_info():
    model, mem = None, None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as f:
            mem = int(f.readline().split()[1]) / 2 ** 20
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu": model, "ram_gib": mem}


def share_flops(plan, s0, s1):
    """Flops the plan's launch list executes for slices s0 .. s1-1."""
    import numpy as np
    sch = plan.schedule(s0, s1)
    runs = np.bincount(sch[:, 1], minlength=plan.stats.n_steps)
    return float((plan.steps()[:, 6] * runs).sum()), int(len(sch))


def spindle_report(net, merge_bits, s0, s1, before=None):
    """Flops of one share with pre-lifetime reuse only (same path) and with
    the post-lifetime merge on top (Sec. III-B), host-side from the launch
    lists; before = (what, flops of the share on the earlier plan) adds the
    total cut against that plan."""
    from paper_2504_09186_amd import tnc
    pre, n_pre = share_flops(tnc.Plan(net, precision=0), s0, s1)
    p = tnc.Plan(net, precision=0, merge_bits=merge_bits)
    spin, n_spin = share_flops(p, s0, s1)
    r = {"merge_bits": merge_bits, "n_merged": int(p.stats.n_merged), "share_flops_prelifetime": pre,
         "share_flops_spindle": spin, "merge_skipped_frac": 1.0 - spin / pre, "launches_prelifetime": n_pre,
         "launches_spindle": n_spin}
    if before is not None and before[1]:
        r["earlier_plan"] = before[0]
        r["share_flops_earlier_plan"] = before[1]
        r["total_skipped_frac"] = 1.0 - spin / before[1]
    return r


def config2_net(trials):
    """The 5x6-qubit network and its plan search: recursive-bisection and
    greedy trials ranked by the flops of one 256-slice share with the
    merge of the 8 sliced bits plus 2e8 flops per step launch (the
    workload is bound by launches), then branch exchange (Sec. III-B)."""
    from paper_2504_09186_amd import tnc
    c, spec = workload2()
    net = tnc.Network(c, spec)
    net.path_search(seed=3001, trials=trials, max_log2=26, min_sliced=8, max_sliced=8, method=2, window_bits=8,
                    merge_bits=8, branch_exchange=True, launch_cost_flops=2e8)
    return c, spec, net


def run_config2(steps, warmup, trials):
    """The 5x6-qubit workload: both forms on the greedy-search plan, errors
    against all 64 oracle amplitudes."""
    import torch

    from paper_2504_09186_amd import tnc
    c, spec, net = config2_net(trials)
    g = load_json(GOLDEN2)
    ref = to_complex(g["amplitudes"]) if g else None
    # the plan of a greedy search ranked by plain flops, for comparison
    net0 = tnc.Network(c, spec)
    net0.path_search(seed=3001, trials=trials, max_log2=26, min_sliced=8, max_sliced=8)
    before = ("greedy search ranked by plain flops, pre-lifetime reuse", share_flops(tnc.Plan(net0), 0, 256)[0])
    out = {"workload": WORKLOAD2, "spindle": spindle_report(net, 8, 0, 256, before)}
    for prec, label in ((0, "c64"), (1, "cf16")):
        plan = tnc.Plan(net, precision=prec, merge_bits=8)
        plan.upload()
        if prec:
            plan.calibrate(0, 2)
        rec, res = run_form(plan, steps, warmup, label, WORKLOAD2)
        rec["amp_error"] = error_metrics(res, ref, "FP64 oracle, all 64 amplitudes") if ref is not None else None
        out[label] = rec
        del plan
        torch.cuda.empty_cache()
    return out


MICRO = {
    # name: (m, n, k bits, kernel class or -1, description)
    "square": (15, 15, 13, -1, "MB-square: rank-28 x rank-28 tensors, 13 common indices (M = N = 2^15, K = 2^13)"),
    "stem": (25, 5, 5, -1, "MB-stem: rank-30 tensor x rank-10 tensor, 5 common (M = 2^25, K = N = 2^5)"),
    "gepdot": (3, 3, 27, -1, "MB-GEPDOT: rank-30 x rank-30, 27 common (M = N = 2^3, K = 2^27)"),
}


def micro(name, precision, reps):
    """Per-class microbenchmark: one pairwise contraction through the
    library's one-step entry point, seeded complex normal operands with
    random bit layouts (the permutation is part of the load), timed with
    events on the launching stream."""
    import numpy as np
    import torch

    from paper_2504_09186_amd import tnc
    mb, nb, kb, kern, desc = MICRO[name]
    rng = np.random.default_rng(5000 + len(name))
    M = [1000 + i for i in range(mb)]
    N = [2000 + i for i in range(nb)]
    K = [3000 + i for i in range(kb)]
    la = [int(x) for x in rng.permutation(M + K)]
    lb = [int(x) for x in rng.permutation(K + N)]
    lc = [int(x) for x in rng.permutation(M + N)]
    if name == "stem":
        # the planner's layout for a stem step: the new indices take the
        # address bits the contracted ones free ("in place")
        it = iter(N)
        lc = [next(it) if x in K else x for x in la]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5001)
    if precision == 0:
        a = torch.randn(1 << len(la), dtype=torch.complex64, device="cuda", generator=gen)
        b = torch.randn(1 << len(lb), dtype=torch.complex64, device="cuda", generator=gen)
        esz = 8
    else:
        a = torch.randn(2 << len(la), dtype=torch.float16, device="cuda", generator=gen).view(torch.int32)
        b = torch.randn(2 << len(lb), dtype=torch.float16, device="cuda", generator=gen).view(torch.int32)
        esz = 4
    out = torch.empty(1 << len(lc), dtype=torch.complex64 if precision == 0 else torch.int32, device="cuda")
    tnc.contract(a, la, b, lb, lc, kernel=kern, precision=precision, out=out)  # warmup
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        tnc.contract(a, la, b, lb, lc, kernel=kern, precision=precision, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    flops = 8.0 * 2.0 ** (mb + nb + kb)
    nbytes = esz * (2.0 ** len(la) + 2.0 ** len(lb) + 2.0 ** len(lc))
    # the complex64 tile and stream kernels run the 3M split; the split-K
    # kernels and the 16-bit forms run all four real products
    ex = 0.75 if precision == 0 and name in ("square", "stem") else 1.0
    peak = PEAK_FP32 if precision == 0 else PEAK_FP16
    return {"micro": name, "what": desc, "precision": "c64" if precision == 0 else "cf16", "ms": ms,
            "tflops_4m_count": flops / ms / 1e9, "tflops_executed": flops * ex / ms / 1e9,
            "mfma_frac": flops * ex / ms / 1e9 / peak, "gbs": nbytes / ms / 1e6, "hbm_frac": nbytes / ms / 1e6 / PEAK_HBM_GBS,
            "algorithmic_bytes": nbytes, "algorithmic_flops": flops, "reps": reps}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--trials", type=int, default=8, help="path-search trials (headline workload, with --search)")
    ap.add_argument("--search", action="store_true", help="search the headline path instead of loading the stored one")
    ap.add_argument("--only", choices=["c64", "cf16"], help="profiling runs: time one form only (no JSON line)")
    ap.add_argument("--no-check", action="store_true", help="skip the oracle sub-slice error check")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="headline workload only (no 5x6 workload, no differentiation form)")
    ap.add_argument("--workload", choices=["rqc7x8", "rqc5x6"], default="rqc7x8")
    ap.add_argument("--grad", action="store_true",
                    help="only time the differentiation form (forward vs backward over all slices) and exit")
    ap.add_argument("--micro", choices=sorted(MICRO), help="only run one per-class microbenchmark and exit")
    ap.add_argument("--micro-precision", type=int, default=0, help="0 complex64, 1 complex FP16")
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
        print(json.dumps({"grad": grad_timing(args.steps), "grad_sliced": grad_timing(args.steps, cap=22),
                          "grad_config3": grad_config3(args.steps)}), flush=True)
        return
    if args.micro:
        print(json.dumps(micro(args.micro, args.micro_precision, max(1, args.steps))), flush=True)
        return
    if args.workload == "rqc5x6":
        r = run_config2(args.steps, args.warmup, 64)
        c64 = r["c64"]
        out = {"metric": METRIC, "value": c64["value"], "unit": "slices/s", "n_gpus": 1, "steps": args.steps,
               "warmup": args.warmup, "ms_per_step": c64["ms_per_step"], "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": "c64", "data": "synthetic",
               "config": {"workload": WORKLOAD2}, "roofline": c64["roofline"], "detail": r}
        print(json.dumps(out), flush=True)
        return

    c, spec = workload4()
    net = tnc.Network(c, spec)
    stored = load_json(PATH4) if not args.search else None
    before_exchange = None
    if stored is not None and stored["n_leaves"] == net.n_leaves:
        net.set_path([tuple(x) for x in stored["path"]])
        net.set_slicing(stored["slicing"])
        search_s = stored["search"]["seconds"] + stored.get("branch_exchange", {}).get("seconds", 0.0)
        merge_bits = stored.get("merge_bits", 0)
        before_exchange = stored["search"].get("share_flops")
        path_source = (f"stored: recursive bisection, {stored['search']['trials']} trials, "
                       f"{stored['workload']['min_sliced']}-{stored['workload']['max_sliced']} sliced indices, "
                       f"ranked by job flops in 256-slice shares (merge, launch cost), then branch exchange")
    else:
        t0 = time.perf_counter()
        net.path_search(seed=3004, trials=args.trials, max_log2=30, min_sliced=8, max_sliced=62, method=1,
                        window_bits=8, merge_bits=8, branch_exchange=True)
        search_s = time.perf_counter() - t0
        merge_bits = 8
        path_source = f"searched here: recursive bisection, {args.trials} trials, then branch exchange"
    print(f"path {path_source} ({search_s:.1f} s), {len(net.slicing())} sliced indices", file=sys.stderr,
          flush=True)
    g4 = load_json(GOLDEN4)
    share = (0, 256)

    if args.only:
        # A profiling run: one form's share passes and nothing else, so that
        # kernel statistics of the run are those of the timed passes.
        prec = 0 if args.only == "c64" else 1
        plan = tnc.Plan(net, precision=prec, merge_bits=merge_bits)
        plan.upload()
        if prec:
            plan.calibrate(0, 2)
        r, _ = run_form(plan, args.steps, args.warmup, args.only, WORKLOAD4, *share)
        print(json.dumps({"only": args.only, "value": r["value"], "ms_per_step": r["ms_per_step"],
                          "roofline": r["roofline"], "kernel_ms_by_class": r["kernel_ms_by_class"]}), flush=True)
        return
    plan = tnc.Plan(net, precision=0, merge_bits=merge_bits)
    st = plan.stats
    plan.upload()
    r64, res64 = run_form(plan, args.steps, args.warmup, "c64", WORKLOAD4, *share)
    del plan
    torch.cuda.empty_cache()
    print(f"complex64: {r64['value']:.1f} slices/s", file=sys.stderr, flush=True)
    plan = tnc.Plan(net, precision=1, merge_bits=merge_bits)
    plan.upload()
    plan.calibrate(0, 2)
    r16, res16 = run_form(plan, args.steps, args.warmup, "cf16", WORKLOAD4, *share)
    del plan
    torch.cuda.empty_cache()
    print(f"complex FP16: {r16['value']:.1f} slices/s", file=sys.stderr, flush=True)
    r16["vs_complex64"] = error_metrics(res16, res64, "complex64 GPU result of the same 256 slices")
    if g4 is not None and not args.no_check:
        r64["amp_error"] = subslice_check(c, spec, g4, 0)
        r16["amp_error"] = subslice_check(c, spec, g4, 1)
    out = {
        "metric": METRIC, "value": r64["value"], "unit": "slices/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD4, "qubits": 56, "cycles": 20, "open_qubits": 12,
                   "slices_per_step": 256, "n_sliced": st.n_sliced, "max_log2_elems": st.max_log2_elems,
                   "steps_per_slice": st.n_steps, "flops_full_slice": st.flops_full_slice,
                   "path_search_s": search_s, "path": path_source, "merge_bits": merge_bits,
                   "n_merged": st.n_merged,
                   "job_flops": r64["flops_per_step"] * 2.0 ** (st.n_sliced - 8),
                   "job_seconds_projected": r64["ms_per_step"] * 1e-3 * 2.0 ** (st.n_sliced - 8),
                   "precision": "complex64, FP32 MFMA (3M), FP64 cross-slice sum"},
        "tflops": r64["tflops"],
        "hbm_gbs": r64["hbm_gbs"], "amp_error": r64.get("amp_error"),
        "kernel_ms_by_class": r64["kernel_ms_by_class"], "kernel_tflops_by_class": r64["kernel_tflops_by_class"],
        "roofline": r64["roofline"],
        "spindle": spindle_report(net, merge_bits, *share,
                                  ("same search before branch exchange, pre-lifetime reuse", before_exchange)),
        "cf16": dict(r16, precision="complex FP16 storage, FP16 MFMA (4M) with FP32 accumulate, per-tensor 2^e "
                                    "scaling, FP64 cross-slice sum"),
    }
    if not args.no_extras:
        out["alt_path"] = alt_path_timing(c, spec, args.steps, args.warmup)
        out["config2"] = run_config2(args.steps, args.warmup, 64)
        out["grad"] = grad_timing(args.steps)
        # the same with intermediates capped at 2^22 entries: 16 slices, each
        # recomputed per slice by the backward
        out["grad_sliced"] = grad_timing(args.steps, cap=22)
        out["grad_config3"] = grad_config3(args.steps)
    if not args.no_cpu_baseline and g4 is not None:
        out["cpu_baseline"] = cpu_baseline_subslice(c, spec, g4, r64["flops_per_step"] / 256)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
