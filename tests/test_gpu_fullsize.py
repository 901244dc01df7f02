"""Full-size parity: the bench workload (5x6 lattice, 14 cycles, 64
amplitudes, 256 slices, max intermediate <= 2^26) in the launch configuration
bench.py times, against values written by tests/golden/make_golden.py with the
oracle only.

* All 256 slices with the bench plan: the sum is the 64 amplitudes, which do
  not depend on the plan; compared within 1e-5 relative L2.
* Slices 0..15 of the oracle's own 8-index slicing, one by one: the library
  keeps that slicing and searches its own path for it.
"""
import json
import os

import numpy as np
import pytest

import synth
from helpers import require_gpu

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "config2_amplitudes.json")


def _golden():
    if not os.path.exists(GOLDEN):
        pytest.skip("golden file not generated")
    with open(GOLDEN) as f:
        g = json.load(f)
    to_c = lambda v: np.array([a + 1j * b for a, b in v])  # noqa: E731
    return g, to_c


def _workload():
    c = synth.lattice_circuit(5, 6, 14, seed=1001)
    spec = synth.output_spec(30, list(range(24, 30)), seed=2001)
    return c, spec


def _bench_net():
    """The benchmark's plan search for this network: bisection and greedy
    trials ranked with the merge of the 8 sliced bits and a cost per launch,
    then branch exchange (its plans merge where lifetimes nest)."""
    from paper_2504_09186_amd import tnc
    c, spec = _workload()
    net = tnc.Network(c, spec)
    net.path_search(seed=3001, trials=64, max_log2=26, min_sliced=8, max_sliced=8, method=2, window_bits=8,
                    merge_bits=8, branch_exchange=True, launch_cost_flops=2e8)
    return net


@pytest.mark.parametrize("fuse", [False, True])
def test_config2_all_slices_bench_plan(fuse):
    """All 256 slices, against the oracle's stored amplitudes: the benchmark
    plan (post-lifetime merge of all 8 sliced bits), and the plain greedy
    plan with the stem chains as fused sections (fused sections and merges
    are not combined)."""
    require_gpu()
    import torch
    from paper_2504_09186_amd import tnc
    g, to_c = _golden()
    if fuse:
        c, spec = _workload()
        net = tnc.Network(c, spec)
        net.path_search(seed=3001, trials=64, max_log2=26, min_sliced=8, max_sliced=8)
        plan = tnc.Plan(net, fuse_sections=True)
        assert any(plan.step_info(i)["section"] >= 0 for i in range(plan.stats.n_steps))
    else:
        plan = tnc.Plan(_bench_net(), merge_bits=8)
        assert plan.stats.n_merged >= 1
    assert plan.n_slices == 256
    plan.upload()
    acc = plan.new_result()
    print(f"config 2: all 256 slices, bench plan, fused sections {fuse}", flush=True)
    plan.execute(acc)
    torch.cuda.synchronize()
    got = acc.cpu().numpy()
    ref = to_c(g["amplitudes"])
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"rel-L2 {rel:.3e}")
    assert rel <= 1e-5


def test_config2_oracle_slicing_first_16_slices():
    require_gpu()
    import torch
    from paper_2504_09186_amd import tnc
    g, to_c = _golden()
    c, spec = _workload()
    net = tnc.Network(c, spec)
    net.set_slicing(g["oracle_sliced_labels"])
    net.path_search(seed=3001, trials=32, max_log2=28, min_sliced=8, max_sliced=8, keep_slicing=True)
    assert net.slicing() == g["oracle_sliced_labels"]
    plan = tnc.Plan(net)
    plan.upload()
    for s in range(16):
        acc = plan.new_result()
        print(f"config 2: oracle slicing, slice {s}", flush=True)
        plan.execute(acc, s, s + 1)
        torch.cuda.synchronize()
        got = acc.cpu().numpy()
        ref = to_c(g["slice_results"][str(s)])
        assert np.linalg.norm(got - ref) <= 1e-5 * max(np.linalg.norm(ref), 1e-30), f"slice {s}"


@pytest.mark.parametrize("prec,xeb_bound,rel_bound", [(1, 1e-3, 2e-2), (2, 1e-2, 1.5e-1)])
def test_config2_all_slices_half_precision(prec, xeb_bound, rel_bound):
    """Precision form at full size: all 256 slices of the benchmark plan (with
    merges) with complex FP16 (prec 1) or BF16 (prec 2) storage, FP32 accumulation and
    per-tensor exponents calibrated on slices 0-1, FP64 cross-slice sum.  The
    result is an approximation, pinned only by the error metrics against the
    FP64 oracle's amplitudes: linear-XEB fidelity loss <= 1e-3 (FP16) or
    <= 1e-2 (BF16, 8-bit significand) and relative L2 <= 2e-2 (FP16) or
    <= 1.5e-1 (BF16); no stored value may overflow."""
    require_gpu()
    import torch

    import oracle
    from paper_2504_09186_amd import tnc
    g, to_c = _golden()
    plan = tnc.Plan(_bench_net(), precision=prec, merge_bits=8)
    assert plan.stats.n_merged >= 1
    plan.upload()
    plan.calibrate(0, 2)
    acc = plan.new_result()
    print(f"config 2: all 256 slices, precision {prec}", flush=True)
    plan.execute(acc)
    torch.cuda.synchronize()
    got = acc.cpu().numpy()
    ref = to_c(g["amplitudes"])
    rel = oracle.rel_l2(got, ref)
    loss = abs(1.0 - oracle.xeb_ratio(got, ref))
    mx = float(plan.step_maxima().max())
    print(f"rel-L2 {rel:.3e}, XEB loss {loss:.3e}, largest stored {mx:.1f}")
    assert np.all(np.isfinite(got))
    assert mx < 65504.0
    assert loss <= xeb_bound
    assert rel <= rel_bound


GOLDEN4 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "config4_subslices.json")


def _config4_subslice_plan(prec, exchange=False):
    """The 7x8-qubit, 20-cycle network (qubits 44-55 open) with the oracle's
    sliced indices kept (outermost, in its order) and the library's own
    path; extra inner indices only if its path needs them for 2^30."""
    from paper_2504_09186_amd import tnc
    if not os.path.exists(GOLDEN4):
        pytest.skip("golden file not generated")
    with open(GOLDEN4) as f:
        g = json.load(f)
    c = synth.lattice_circuit(7, 8, 20, seed=1004)
    spec = synth.output_spec(56, list(range(44, 56)), seed=2004)
    net = tnc.Network(c, spec)
    lab = g["oracle_sliced_labels"]
    net.set_slicing(lab)
    net.path_search(seed=3004, trials=8, max_log2=30, min_sliced=len(lab), max_sliced=62, keep_slicing=True,
                    method=1)
    assert net.slicing()[:len(lab)] == lab
    extra = len(net.slicing()) - len(lab)
    if exchange:
        before, after = net.branch_exchange(window_bits=extra, merge_bits=extra, max_log2=30)
        assert after < before
    plan = tnc.Plan(net, precision=prec, merge_bits=extra)
    return g, plan, extra


@pytest.mark.parametrize("exchange", [False, True])
@pytest.mark.parametrize("prec", [0, 1])
def test_config4_oracle_subslices(prec, exchange):
    """Full-size 56-qubit network, sub-slices of the oracle's 60-index slicing
    (each a partial sum over the sliced indices' other values, about 4e12
    flops for the oracle): complex64 within 1e-5 relative L2 of the FP64
    oracle; complex FP16 (exponents calibrated on the first checked
    sub-slice) within 2e-2 relative L2 and an XEB fidelity loss <= 1e-3 over
    the 2^12 open amplitudes of each sub-slice.  Also on the path after
    branch exchange (Sec. III-B), which must not change the values."""
    require_gpu()
    import torch

    import oracle
    g, plan, extra = _config4_subslice_plan(prec, exchange)
    to_c = lambda v: np.array([a + 1j * b for a, b in v])  # noqa: E731
    plan.upload()
    for sid in g["sub_slice_ids"]:
        s0, s1 = sid << extra, (sid + 1) << extra
        if prec:
            plan.calibrate(s0, min(s1, s0 + 2))
        acc = plan.new_result()
        print(f"config 4: sub-slice {sid} (library slices {s0}..{s1 - 1}), precision {prec}, exchange {exchange}",
              flush=True)
        plan.execute(acc, s0, s1)
        torch.cuda.synchronize()
        got = acc.cpu().numpy()
        ref = to_c(g["sub_slice_results"][str(sid)])
        rel = oracle.rel_l2(got, ref)
        print(f"rel-L2 {rel:.3e}")
        if prec == 0:
            assert rel <= 1e-5
        else:
            assert rel <= 2e-2
            assert abs(1.0 - oracle.xeb_ratio(got, ref)) <= 1e-3
