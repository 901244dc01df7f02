"""Whole sliced contractions on the GPU against the FP64 oracle.

Slicing labels are chosen by the test (canonical wire labels) and set in both
the library and the oracle; each side plans its own contraction order, which
does not change the value.  Tolerance: complex64 within 1e-5 relative L2.
"""
import numpy as np
import pytest

import oracle
import synth
from helpers import require_gpu

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _lib_net(circ, spec, bits=None):
    from paper_2504_09186_amd import tnc
    return tnc.Network(circ, spec, bits)


def _run(net, s0=0, s1=None, reuse=True, force=-1):
    import torch
    from paper_2504_09186_amd import tnc
    plan = tnc.Plan(net, reuse=reuse, force_kernel=force)
    plan.upload()
    acc = plan.new_result()
    plan.execute(acc, s0, plan.n_slices if s1 is None else s1)
    torch.cuda.synchronize()
    return acc.cpu().numpy(), plan


def test_config1_against_statevector():
    """3x4 lattice, 8 cycles, greedy path, 2 sliced indices, one amplitude."""
    require_gpu()
    c = synth.lattice_circuit(3, 4, 8, seed=1000)
    spec = synth.output_spec(12, [], seed=2000)
    net = _lib_net(c, spec)
    net.path_search(seed=3000, trials=8, max_log2=30, min_sliced=2, max_sliced=2)
    assert len(net.slicing()) == 2
    got, plan = _run(net)
    assert plan.n_slices == 4
    ref = oracle.sv_amplitudes(c, spec)
    assert abs(got[0] - ref) / abs(ref) < TOL


@pytest.mark.parametrize("rows,cols,cycles,nopen,nsl,seed", [
    (2, 3, 5, 2, 2, 1), (3, 3, 6, 3, 3, 2), (3, 4, 8, 4, 3, 3), (2, 4, 10, 0, 4, 4), (4, 4, 8, 6, 4, 5)])
def test_per_slice_partial_sums(rows, cols, cycles, nopen, nsl, seed):
    require_gpu()
    c = synth.lattice_circuit(rows, cols, cycles, seed=seed)
    n = c.n_qubits
    spec = synth.output_spec(n, list(range(n - nopen, n)), seed=seed + 50)
    onet = oracle.build_network(c, spec)
    rng = np.random.default_rng(seed + 99)
    sliced = [int(x) for x in rng.choice(onet.closed_labels(), size=nsl, replace=False)]
    opath = oracle.greedy_path(onet)
    total, parts = oracle.contract_sliced(onet, opath, sliced, per_slice=True)
    net = _lib_net(c, spec)
    net.path_search(seed=seed, trials=4, max_log2=30)
    net.set_slicing(sliced)
    print(f"partial sums case {rows}x{cols}x{cycles} sliced {sliced}", flush=True)
    for s in range(1 << nsl):
        got, _ = _run(net, s, s + 1)
        ref = np.asarray(parts[s]).reshape(-1)
        assert np.linalg.norm(got - ref) <= TOL * max(np.linalg.norm(ref), 1e-12), f"slice {s}"
    got, _ = _run(net)
    ref = np.asarray(total).reshape(-1)
    assert np.linalg.norm(got - ref) <= TOL * np.linalg.norm(ref)
    assert np.linalg.norm(got - oracle.sv_amplitudes(c, spec).reshape(-1)) <= TOL * np.linalg.norm(ref)


def test_reuse_and_ranges_consistent():
    """Cross-slice reuse and any split of the slice range give the same sum."""
    require_gpu()
    c = synth.lattice_circuit(4, 4, 10, seed=7)
    spec = synth.output_spec(16, [13, 14, 15], seed=8)
    net = _lib_net(c, spec)
    net.path_search(seed=9, trials=8, max_log2=11, min_sliced=5)
    full_reuse, plan = _run(net, reuse=True)
    full_plain, _ = _run(net, reuse=False)
    n = plan.n_slices
    a, _ = _run(net, 0, 5)
    b, _ = _run(net, 5, n)
    ref = oracle.sv_amplitudes(c, spec).reshape(-1)
    for x in (full_reuse, full_plain, a + b):
        assert np.linalg.norm(x - ref) <= TOL * np.linalg.norm(ref)


def test_batched_bitstrings():
    require_gpu()
    c = synth.lattice_circuit(3, 3, 6, seed=21)
    bits = synth.random_bitstrings(9, 16, seed=22)
    spec = np.full(9, -2, dtype=np.int8)
    net = _lib_net(c, spec, bits)
    net.path_search(seed=23, trials=8, max_log2=30, min_sliced=2)
    got, _ = _run(net)
    ref = oracle.sv_amplitudes(c, spec, bits).reshape(-1)
    assert np.linalg.norm(got - ref) <= TOL * np.linalg.norm(ref)


@pytest.mark.parametrize("force", [0, 2, 3, 4])
def test_forced_kernel_class(force):
    """Every step on one kernel class (any shape must be handled correctly)."""
    require_gpu()
    c = synth.lattice_circuit(3, 4, 6, seed=31)
    spec = synth.output_spec(12, [10, 11], seed=32)
    net = _lib_net(c, spec)
    net.path_search(seed=33, trials=4, max_log2=30, min_sliced=2)
    got, _ = _run(net, force=force)
    ref = oracle.sv_amplitudes(c, spec).reshape(-1)
    assert np.linalg.norm(got - ref) <= TOL * np.linalg.norm(ref)


@pytest.mark.parametrize("prec", [1, 2])
def test_precision_form_circuit(prec):
    """Scaled complex FP16 / BF16 form on a 4x4 lattice (16 open amplitudes):
    calibrated on slices 0-1, all slices summed in FP64.  Reported and bounded:
    relative L2 error and linear-XEB fidelity loss against the FP64 oracle.
    FP16 (11-bit significand) is held to the 1e-3 XEB-loss target; BF16
    (8-bit significand, about 8x coarser) to 1e-2."""
    require_gpu()
    import torch
    from paper_2504_09186_amd import tnc
    c = synth.lattice_circuit(4, 4, 10, seed=81)
    spec = synth.output_spec(16, [12, 13, 14, 15], seed=82)
    net = _lib_net(c, spec)
    net.path_search(seed=83, trials=8, max_log2=10, min_sliced=4)
    plan = tnc.Plan(net, precision=prec)
    plan.upload()
    plan.calibrate(0, 2)
    acc = plan.new_result()
    plan.execute(acc)
    torch.cuda.synchronize()
    got = acc.cpu().numpy()
    mx = plan.step_maxima()
    ref = oracle.sv_amplitudes(c, spec).reshape(-1)
    rel = oracle.rel_l2(got, ref)
    xeb_loss = abs(1.0 - oracle.xeb_ratio(got, ref))
    print(f"precision {prec}: rel-L2 {rel:.3e}, XEB loss {xeb_loss:.3e}, max stored {mx.max():.3e}")
    assert np.all(np.isfinite(mx)) and mx.max() < 65504
    assert rel < (5e-3 if prec == 1 else 5e-2)
    assert xeb_loss < (1e-3 if prec == 1 else 1e-2)


@pytest.mark.parametrize("force", [2, 3, 4])
def test_precision_form_forced_tiles(force):
    """FP16 plans whose every step runs on one MFMA tile class: the complex64
    calibration slice uses tiles of the complex64 geometry, the FP16 run its
    own (regression for a calibration launched with FP16 tile descriptors)."""
    require_gpu()
    import torch
    from paper_2504_09186_amd import tnc
    c = synth.lattice_circuit(4, 4, 8, seed=91)
    spec = synth.output_spec(16, [14, 15], seed=92)
    net = _lib_net(c, spec)
    net.path_search(seed=93, trials=4, max_log2=30, min_sliced=3)
    plan = tnc.Plan(net, precision=1, force_kernel=force)
    plan.upload()
    plan.calibrate(0, 1)
    acc = plan.new_result()
    plan.execute(acc)
    torch.cuda.synchronize()
    ref = oracle.sv_amplitudes(c, spec).reshape(-1)
    assert oracle.rel_l2(acc.cpu().numpy(), ref) < 5e-3


@pytest.mark.parametrize("prec", [0, 1])
def test_fused_sections(prec):
    """4x5 lattice, 12 cycles, intermediates <= 2^17, 4 sliced indices: the
    stem chain runs as fused sections (Sec. IV).  complex64: fused, unfused
    and every slice range agree with the state vector to 1e-5; FP16: the
    fused plan's XEB loss stays below 1e-3."""
    require_gpu()
    import torch
    from paper_2504_09186_amd import tnc
    c = synth.lattice_circuit(4, 5, 12, seed=12)
    spec = synth.output_spec(20, [17, 18, 19], seed=13)
    net = _lib_net(c, spec)
    net.path_search(seed=12, trials=8, max_log2=17, min_sliced=4, max_sliced=4)
    ref = oracle.sv_amplitudes(c, spec).reshape(-1)
    print(f"fused sections case prec {prec}", flush=True)
    plan = tnc.Plan(net, precision=prec, fuse_sections=True)
    assert any(plan.step_info(i)["section"] >= 0 for i in range(plan.stats.n_steps))
    plan.upload()
    if prec:
        plan.calibrate(0, 2)
    acc = plan.new_result()
    plan.execute(acc)
    torch.cuda.synchronize()
    got = acc.cpu().numpy()
    if prec == 0:
        assert np.linalg.norm(got - ref) <= TOL * np.linalg.norm(ref)
        plain, _ = _run_opts(net, fuse_sections=False)
        assert np.linalg.norm(plain - ref) <= TOL * np.linalg.norm(ref)
        a = plan.new_result()
        plan.execute(a, 0, 3)
        plan.execute(a, 3, plan.n_slices)
        torch.cuda.synchronize()
        assert np.linalg.norm(a.cpu().numpy() - ref) <= TOL * np.linalg.norm(ref)
    else:
        assert oracle.rel_l2(got, ref) < 2e-2
        assert abs(1.0 - oracle.xeb_ratio(got, ref)) < 1e-3


def _run_opts(net, **kw):
    import torch
    from paper_2504_09186_amd import tnc
    plan = tnc.Plan(net, **kw)
    plan.upload()
    acc = plan.new_result()
    plan.execute(acc)
    torch.cuda.synchronize()
    return acc.cpu().numpy(), plan


@pytest.mark.parametrize("case", ["demote", "merge"])
def test_cache_budget_demotion(case):
    """Shared-prefix reuse under a byte budget for kept tensors (Sec. III-B
    dynamic tuning).  "demote": with a budget of 4 KiB the largest kept nodes
    are demoted (recomputed as often as their parent: more flops per slice);
    "merge": a plan whose four sliced bits are all merged keeps its merge
    accumulators under the same budget.  The sums over all slices and over
    two ranges (one, when a merge group spans all slices) equal the state
    vector."""
    require_gpu()
    import torch
    from helpers import nested_chain
    from paper_2504_09186_amd import tnc
    if case == "demote":
        c = synth.lattice_circuit(4, 4, 10, seed=7)
        spec = synth.output_spec(16, [13, 14, 15], seed=8)
        net = _lib_net(c, spec)
        net.path_search(seed=9, trials=8, max_log2=11, min_sliced=5, max_sliced=5)
        kw = {}
    else:
        c = synth.lattice_circuit(4, 4, 10, seed=5)
        spec = synth.output_spec(16, [15], seed=6)
        onet = oracle.build_network(c, spec)
        path = oracle.greedy_path(onet)
        net = _lib_net(c, spec)
        net.set_path(path)
        net.set_slicing(nested_chain(onet, path, 4)[::-1])
        kw = {"merge_bits": 4, "no_hoist": True}
    ref = oracle.sv_amplitudes(c, spec).reshape(-1)
    full = tnc.Plan(net, **kw)
    plan = tnc.Plan(net, cache_budget_bytes=4096, **kw)
    if case == "demote":
        assert plan.stats.flops_reused_slice > full.stats.flops_reused_slice
    else:
        assert plan.stats.n_merged == 4
    print(f"cache budget, {case}: flops/slice {full.stats.flops_reused_slice:.3e} -> "
          f"{plan.stats.flops_reused_slice:.3e}", flush=True)
    plan.upload()
    acc = plan.new_result()
    plan.execute(acc)
    # two ranges, each a whole number of merge groups when there are merges
    half = max(1 << plan.stats.merge_align_bits, plan.n_slices // 2)
    acc2 = plan.new_result()
    for s0, s1 in ((0, half), (half, plan.n_slices)):
        if s0 < s1:
            plan.execute(acc2, s0, s1)
    torch.cuda.synchronize()
    for got in (acc.cpu().numpy(), acc2.cpu().numpy()):
        assert np.linalg.norm(got - ref) <= TOL * np.linalg.norm(ref)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("pb", [0, 3])
def test_range_prologue(prec, pb):
    """The range prologue on the GPU: steps computed once per slice range run
    first, SMALL ones batched per dependency level (prologue_bits 0: no
    sliced index; 3: sliced indices at bits >= 3, ranges within aligned
    blocks of 8 slices).  Sums over the blocks equal the state vector
    (complex64 1e-5; FP16 5e-3 relative L2)."""
    require_gpu()
    import torch
    from paper_2504_09186_amd import tnc
    c = synth.lattice_circuit(4, 4, 10, seed=7)
    spec = synth.output_spec(16, [13, 14, 15], seed=8)
    net = _lib_net(c, spec)
    net.path_search(seed=9, trials=8, max_log2=11, min_sliced=5, max_sliced=5)
    ref = oracle.sv_amplitudes(c, spec).reshape(-1)
    plan = tnc.Plan(net, precision=prec, prologue_bits=pb)
    assert plan.stats.n_batched_small >= 2
    print(f"range prologue, precision {prec}, prologue_bits {pb}: {plan.stats.n_batched_small} steps in "
          f"{plan.stats.n_batched_launches} batched launches", flush=True)
    plan.upload()
    step = 8 if pb else plan.n_slices
    if prec:
        plan.calibrate(0, 2)
    acc = plan.new_result()
    for s0 in range(0, plan.n_slices, step):
        plan.execute(acc, s0, s0 + step)
    torch.cuda.synchronize()
    got = acc.cpu().numpy()
    assert np.linalg.norm(got - ref) <= (TOL if prec == 0 else 5e-3) * np.linalg.norm(ref)
