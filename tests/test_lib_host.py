"""Host-side checks of libmitnc (no GPU): exported symbols, planner arithmetic
against the oracle's counted flops, validation of paths and slicing."""
import os
import re

import numpy as np
import pytest

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2504_09186_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2504_09186_amd import build
        build.build()
    return _lib.load()


def test_exports_every_header_symbol(lib):
    from paper_2504_09186_amd import _lib
    text = open(os.path.join(ROOT, "include", "mitnc.h")).read()
    declared = set(re.findall(r"\b(mitnc_[a-z_0-9]+)\s*\(", text))
    assert declared, "no declarations found"
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(_lib.EXPORTED)


def _nets(rows=2, cols=3, cycles=5, seed=31, nopen=1):
    from paper_2504_09186_amd import tnc
    c = synth.lattice_circuit(rows, cols, cycles, seed=seed)
    n = c.n_qubits
    spec = synth.output_spec(n, list(range(n - nopen, n)), seed=seed + 1)
    onet = oracle.build_network(c, spec)
    return c, spec, onet, tnc.Network(c, spec)


def test_leaf_count_and_canonical_order(lib):
    c, spec, onet, net = _nets()
    assert net.n_leaves == onet.n_leaves


def test_planner_flops_match_counted_flops(lib):
    """The oracle's path and a slicing chosen by the test are set in the
    library; its per-slice flop count must equal the flops counted while the
    oracle actually contracts one subtask (8 real flops per complex MAC)."""
    from paper_2504_09186_amd import tnc
    c, spec, onet, net = _nets(3, 3, 6, seed=41, nopen=2)
    path = oracle.greedy_path(onet)
    net.set_path(path)
    for sliced in ([], onet.closed_labels()[5:7]):
        net.set_slicing(sliced)
        plan = tnc.Plan(net)
        counted = oracle.count_contraction_flops(onet, path, sliced)
        assert plan.stats.flops_full_slice == pytest.approx(counted, rel=1e-12)
        assert plan.stats.n_sliced == len(sliced)


def test_index_overhead_eq1(lib):
    c, spec, onet, net = _nets(3, 3, 6, seed=51, nopen=2)
    path = oracle.greedy_path(onet)
    net.set_path(path)
    for a in onet.closed_labels()[:8]:
        want = 2.0 * oracle.count_contraction_flops(onet, path, [a], 1) / oracle.count_contraction_flops(onet, path)
        assert net.index_overhead(a) == pytest.approx(want, rel=1e-12)


def test_path_search_structure(lib):
    c, spec, onet, net = _nets(4, 4, 8, seed=61, nopen=3)
    net.path_search(seed=1, trials=8, max_log2=9, min_sliced=3)
    p = net.path()
    n = net.n_leaves
    assert len(p) == n - 1
    used = set()
    for t, (i, j) in enumerate(p):
        assert i != j and i < n + t and j < n + t and i not in used and j not in used
        used |= {i, j}
    sl = net.slicing()
    assert len(sl) >= 3
    assert set(sl) <= set(onet.closed_labels())
    from paper_2504_09186_amd import tnc
    plan = tnc.Plan(net)
    assert plan.stats.max_log2_elems <= 9
    assert plan.stats.flops_reused_slice <= plan.stats.flops_full_slice + 1e-9
    info = plan.steps()
    assert info.shape == (n - 1, 12)
    assert info[-1, 11] == 1 and info[:-1, 11].sum() == 0


def test_path_search_window_ranking(lib):
    """Ranking trials by the reuse-aware flops of aligned slice windows
    (window_bits) returns a valid path and slicing under the cap; a negative
    window is refused."""
    from paper_2504_09186_amd import _lib
    c, spec, onet, net = _nets(4, 4, 8, seed=62, nopen=3)
    net.path_search(seed=5, trials=6, max_log2=9, min_sliced=3, method=1, window_bits=2)
    p = net.path()
    assert len(p) == net.n_leaves - 1
    assert len(net.slicing()) >= 3
    from paper_2504_09186_amd import tnc
    assert tnc.Plan(net).stats.max_log2_elems <= 9
    with pytest.raises(_lib.MitncError):
        net.path_search(seed=5, trials=2, max_log2=9, min_sliced=3, method=1, window_bits=-1)


def test_validation_errors(lib):
    from paper_2504_09186_amd import _lib
    c, spec, onet, net = _nets()
    n = net.n_leaves
    with pytest.raises(_lib.MitncError):
        net.set_path([(0, 0)] * (n - 1))
    with pytest.raises(_lib.MitncError):
        net.set_path([(0, 1)])
    open_label = onet.output[0]
    with pytest.raises(_lib.MitncError):
        net.set_slicing([open_label])
    with pytest.raises(_lib.MitncError):
        net.set_slicing([12345678])
    good = onet.closed_labels()[0]
    with pytest.raises(_lib.MitncError):
        net.set_slicing([good, good])


def test_plan_workspace_and_reuse_levels(lib):
    from paper_2504_09186_amd import tnc
    c, spec, onet, net = _nets(4, 4, 10, seed=71, nopen=2)
    net.path_search(seed=3, trials=4, max_log2=10, min_sliced=4)
    p1 = tnc.Plan(net, reuse=True)
    p0 = tnc.Plan(net, reuse=False)
    assert p1.stats.workspace_bytes >= p0.stats.workspace_bytes * 0  # both positive
    assert p1.stats.workspace_bytes > 0 and p0.stats.workspace_bytes > 0
    assert p0.stats.flops_reused_slice == pytest.approx(p0.stats.flops_full_slice)
    assert p1.stats.flops_reused_slice < p1.stats.flops_full_slice
    # budget 0 bytes of cache except unavoidable: still plans
    p2 = tnc.Plan(net, reuse=True, cache_budget_bytes=256)
    assert p2.stats.flops_reused_slice >= p1.stats.flops_reused_slice - 1e-9


def test_stream_class_rejects_unsupported_shapes():
    """The stream kernel class refuses shapes outside its limits (more than
    2^10 batch indices, fewer than 2^8 rows, N > 64, too many B entries per lane) when the step
    is built, before any device work."""
    import torch
    from paper_2504_09186_amd import tnc
    from paper_2504_09186_amd._lib import MitncError
    for mb, nb, kb, bb in [(12, 6, 6, 0), (7, 2, 2, 0), (8, 2, 2, 11), (12, 7, 2, 0)]:
        M = [1000 + i for i in range(mb)]
        N = [2000 + i for i in range(nb)]
        K = [3000 + i for i in range(kb)]
        Bt = [-1 - i for i in range(bb)]
        a = torch.zeros(1 << (mb + kb + bb), dtype=torch.complex64)
        b = torch.zeros(1 << (kb + nb + bb), dtype=torch.complex64)
        with pytest.raises(MitncError, match="stream kernel"):
            tnc.contract(a, M + K + Bt, b, K + N + Bt, M + N + Bt, kernel=5)
    # Row indices past the four lowest out of A's order in C.
    M = [1000 + i for i in range(10)]
    a = torch.zeros(1 << 12, dtype=torch.complex64)
    b = torch.zeros(1 << 4, dtype=torch.complex64)
    lc = M[:5] + [M[6], M[5]] + M[7:] + [2000, 2001]
    with pytest.raises(MitncError, match="C row bits in order"):
        tnc.contract(a, M + [3000, 3001], b, [3000, 3001, 2000, 2001], lc, kernel=5)


# ---------------------------------------------------------------- plan replay
# The plan's schedule re-executed on the host from its address maps
# (tests/plan_replay.py) against the oracle: per slice, over ranges, with and
# without cross-slice reuse and hoisting.
@pytest.mark.parametrize("rows,cols,cycles,nopen,nsl,seed", [
    (2, 3, 5, 2, 2, 1), (3, 3, 6, 3, 3, 2), (3, 4, 8, 4, 3, 3), (2, 4, 10, 0, 4, 4)])
def test_plan_replay_per_slice(lib, rows, cols, cycles, nopen, nsl, seed):
    from plan_replay import PlanReplay
    from paper_2504_09186_amd import tnc
    c = synth.lattice_circuit(rows, cols, cycles, seed=seed)
    n = c.n_qubits
    spec = synth.output_spec(n, list(range(n - nopen, n)), seed=seed + 50)
    onet = oracle.build_network(c, spec)
    rng = np.random.default_rng(seed + 99)
    sliced = [int(x) for x in rng.choice(onet.closed_labels(), size=nsl, replace=False)]
    total, parts = oracle.contract_sliced(onet, oracle.greedy_path(onet), sliced, per_slice=True)
    net = tnc.Network(c, spec)
    net.path_search(seed=seed, trials=4, max_log2=30)
    net.set_slicing(sliced)
    for reuse in (True, False):
        plan = tnc.Plan(net, reuse=reuse)
        for s in range(1 << nsl):
            got = PlanReplay(plan).run(s, s + 1)
            ref = np.asarray(parts[s]).reshape(-1)
            assert np.linalg.norm(got - ref) <= 1e-5 * max(np.linalg.norm(ref), 1e-12), (reuse, s)
        got = PlanReplay(plan).run(0, 1 << nsl)
        assert np.linalg.norm(got - np.asarray(total).reshape(-1)) <= 1e-5 * np.linalg.norm(total)


def test_plan_replay_reuse_and_hoisting(lib):
    """4x4 lattice, 10 cycles, 5 sliced indices: hoisted subtrees exist, run
    once per range, and the replayed sums over any split of the range equal
    the state-vector amplitudes; reuse and hoisting execute fewer steps."""
    from plan_replay import PlanReplay
    from paper_2504_09186_amd import tnc
    c = synth.lattice_circuit(4, 4, 10, seed=7)
    spec = synth.output_spec(16, [13, 14, 15], seed=8)
    net = tnc.Network(c, spec)
    net.path_search(seed=9, trials=8, max_log2=11, min_sliced=5)
    ref = oracle.sv_amplitudes(c, spec).reshape(-1)
    plan = tnc.Plan(net, reuse=True)
    n = plan.n_slices
    hoisted = [i for i in range(plan.stats.n_steps + net.n_leaves) if plan.node_info(i)["hoisted"]]
    assert hoisted, "expected hoisted subtrees"
    for i in hoisted:
        assert plan.node_info(i)["level"] == -1
    r = PlanReplay(plan)
    full = r.run(0, n)
    split = PlanReplay(plan).run(0, 5) + PlanReplay(plan).run(5, n)
    plain = PlanReplay(tnc.Plan(net, reuse=False))
    full_plain = plain.run(0, n)
    budget = PlanReplay(tnc.Plan(net, reuse=True, cache_budget_bytes=256)).run(0, n)  # cached nodes demoted
    for x in (full, split, full_plain, budget):
        assert np.linalg.norm(x - ref) <= 1e-5 * np.linalg.norm(ref)
    assert r.executed < plain.executed


def test_plan_replay_batched_bitstrings(lib):
    from plan_replay import PlanReplay
    from paper_2504_09186_amd import tnc
    c = synth.lattice_circuit(3, 3, 6, seed=21)
    bits = synth.random_bitstrings(9, 16, seed=22)
    spec = np.full(9, -2, dtype=np.int8)
    net = tnc.Network(c, spec, bits)
    net.path_search(seed=23, trials=8, max_log2=30, min_sliced=2)
    plan = tnc.Plan(net)
    got = PlanReplay(plan).run(0, plan.n_slices)
    ref = oracle.sv_amplitudes(c, spec, bits).reshape(-1)
    assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref)


def _sections(plan):
    out = {}
    for i in range(plan.stats.n_steps):
        si = plan.step_info(i)
        if si["section"] >= 0:
            out.setdefault(si["section"], []).append(i)
    return out


def test_plan_replay_fused_sections(lib):
    """4x5 lattice, 12 cycles, intermediates <= 2^17, 4 sliced indices: the
    stem chain forms a fused section (Sec. IV); replayed with only the
    section's last output stored, the sum equals the state vector, and the
    unfused plan gives the same.  Every section is a chain: each step's A is
    the previous step's output."""
    from plan_replay import PlanReplay
    from paper_2504_09186_amd import tnc
    c = synth.lattice_circuit(4, 5, 12, seed=12)
    spec = synth.output_spec(20, [17, 18, 19], seed=13)
    net = tnc.Network(c, spec)
    net.path_search(seed=12, trials=8, max_log2=17, min_sliced=4, max_sliced=4)
    plan = tnc.Plan(net, fuse_sections=True)
    secs = _sections(plan)
    assert secs and max(len(v) for v in secs.values()) >= 2
    for steps in secs.values():
        for u, v in zip(steps, steps[1:]):
            assert plan.step_info(v)["a"] == plan.step_info(u)["out"]
    ref = oracle.sv_amplitudes(c, spec).reshape(-1)
    fused = PlanReplay(plan).run(0, plan.n_slices)
    plain = PlanReplay(tnc.Plan(net, fuse_sections=False)).run(0, plan.n_slices)
    for x in (fused, plain):
        assert np.linalg.norm(x - ref) <= 1e-5 * np.linalg.norm(ref)
    assert not _sections(tnc.Plan(net, fuse_sections=False))


@pytest.mark.parametrize("rows,cols,cycles,nbits,nsl,seed", [(3, 3, 6, 16, 2, 41), (2, 4, 8, 4, 3, 42)])
def test_reverse_schedule_levels(lib, rows, cols, cycles, nbits, nsl, seed):
    """The backward runs level by level: execution order never goes back a
    level, every adjoint is written once, and an op reads the root's adjoint
    (the seed) or one written at an earlier level.  SMALL ops of a level
    share one batched launch, so none of them may read an adjoint written at
    its own level.  Every step with a single-qubit gate below it contributes
    its adjoint ops (pruning removes only gradient-free subtrees)."""
    from paper_2504_09186_amd import tnc
    c = synth.lattice_circuit(rows, cols, cycles, seed=seed)
    n = c.n_qubits
    bits = synth.random_bitstrings(n, nbits, seed=seed + 1)
    spec = np.full(n, -2, dtype=np.int8)
    net = tnc.Network(c, spec, bits)
    net.path_search(seed=seed + 2, trials=8, max_log2=30, min_sliced=nsl)
    plan = tnc.Plan(net, differentiable=True)
    n_ops = plan.reverse_info()
    assert n_ops > 0
    ops = [plan.reverse_info(i) for i in range(n_ops)]
    steps = [plan.step_info(i) for i in range(plan.stats.n_steps)]
    root = max(s["out"] for s in steps)
    written = {}
    last_level = 0
    for op in ops:
        assert op["level"] >= last_level
        last_level = op["level"]
        assert op["out"] not in written, "adjoint written twice"
        if op["a"] != root:
            assert op["a"] in written, "adjoint read before it is written"
            assert written[op["a"]] < op["level"]
        else:
            assert op["level"] == 0
        written[op["out"]] = op["level"]
    # every single-qubit gate leaf gets its adjoint
    assert n_ops == plan.stats.n_reverse_ops
    n_1q = sum(1 for g in c.gates if len(g.qubits) == 1)
    assert n_1q == plan.stats.n_grad_gates
    assert sum(1 for x in written if x < net.n_leaves) == n_1q
    with pytest.raises(Exception):
        plan.reverse_info(n_ops)


# ------------------------------------------- post-lifetime merge (Sec. III-B)
def _counts(plan, s0, s1):
    sch = plan.schedule(s0, s1)
    return np.bincount(sch[:, 1], minlength=plan.stats.n_steps), sch


def test_schedule_matches_level_rule(lib):
    """Without merges the launch list is the pre-lifetime rule: step t runs in
    slice s iff s is the first of the range or ctz(s) >= its node's level
    (level -1: first slice only); without reuse every step runs in every
    slice.  The steps of the range prologue (batched SMALL steps computed
    once per range) come first, so the list is compared per slice as a set,
    and checked to be in dependency order."""
    from paper_2504_09186_amd import tnc
    c = synth.lattice_circuit(4, 4, 10, seed=7)
    spec = synth.output_spec(16, [13, 14, 15], seed=8)
    net = tnc.Network(c, spec)
    net.path_search(seed=9, trials=8, max_log2=11, min_sliced=5)
    for reuse in (True, False):
        plan = tnc.Plan(net, reuse=reuse)
        levels = [plan.node_info(plan.step_info(t)["out"])["level"] for t in range(plan.stats.n_steps)]
        steps_ = [plan.step_info(t) for t in range(plan.stats.n_steps)]
        out_step = {st["out"]: t for t, st in enumerate(steps_)}
        for s0, s1 in ((0, plan.n_slices), (5, 19)):
            want = []
            for s in range(s0, s1):
                for t, lv in enumerate(levels):
                    if s == s0 or (lv >= 0 and (s & -s).bit_length() - 1 >= lv):
                        want.append((s, t, 1))
            got = [tuple(int(v) for v in r) for r in plan.schedule(s0, s1)]
            assert sorted(got) == sorted(want), (reuse, s0, s1)
            produced = {}  # node -> position of its last computation
            for pos, (s, t, _) in enumerate(got):
                for o in (steps_[t]["a"], steps_[t]["b"]):
                    if o in out_step:
                        assert o in produced, "operand used before it is computed"
                produced[steps_[t]["out"]] = pos


@pytest.mark.parametrize("rows,cols,cycles,seed", [(4, 4, 10, 5), (3, 4, 10, 6), (4, 4, 8, 7)])
def test_merge_nested_counts_equal_lifetimes(lib, rows, cols, cycles, seed):
    """Strictly nested lifetimes (the spindle's condition): with every sliced
    bit merged, each step runs exactly 2^(sliced indices alive at it) times
    over all slices, the count of distinct values it has (the oracle's
    lifetimes), so no calculation is repeated; without merges it runs
    2^(S - lowest bit below it) times (pre-lifetime reuse).  The replayed
    sums equal the state vector both ways."""
    from plan_replay import PlanReplay
    from paper_2504_09186_amd import tnc
    c = synth.lattice_circuit(rows, cols, cycles, seed=seed)
    n = c.n_qubits
    spec = synth.output_spec(n, [n - 1], seed=seed + 1)
    onet = oracle.build_network(c, spec)
    path = oracle.greedy_path(onet)
    from helpers import nested_chain
    chain = nested_chain(onet, path, 4)
    assert chain is not None
    net = tnc.Network(c, spec)
    net.set_path(path)
    net.set_slicing(chain[::-1])  # outer -> inner: the innermost is bit 0
    below, alive = oracle.sliced_lifetimes(onet, path, chain)
    bit = {x: i for i, x in enumerate(chain)}
    S = len(chain)
    merged = tnc.Plan(net, merge_bits=S, no_hoist=True)
    plain = tnc.Plan(net, no_hoist=True)
    assert merged.stats.n_merged == S and merged.stats.merge_align_bits == S
    cm, sch = _counts(merged, 0, 1 << S)
    cp, _ = _counts(plain, 0, 1 << S)
    for t in range(len(path)):
        assert cm[t] == 2 ** len(alive[t]), t
        lo = min((bit[x] for x in below[t]), default=None)
        assert cp[t] == (1 if lo is None else 2 ** (S - lo)), t
    assert cm.sum() < cp.sum() and (sch[:, 2] == 2).any()
    ref = oracle.sv_amplitudes(c, spec).reshape(-1)
    for p in (merged, plain):
        got = PlanReplay(p).run(0, 1 << S)
        assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref)
    # flops of the launch list = the plan's analytic count
    fl = merged.steps()[:, 6]
    assert (fl * cm).sum() / (1 << S) == pytest.approx(merged.stats.flops_reused_slice, rel=1e-12)


@pytest.mark.parametrize("rows,cols,cycles,nsl,seed", [(3, 4, 8, 4, 3), (4, 4, 10, 5, 9), (3, 5, 9, 6, 11)])
def test_merge_random_slicing_replay(lib, rows, cols, cycles, nsl, seed):
    """Random slicings (lifetimes not nested in general; hoisting on): only
    the bits the nesting rule allows are merged.  The replayed launch list
    sums to the state vector over the whole range and over aligned
    sub-ranges; no step runs more often than without merges; the plan's
    analytic flops equal the launch list's; unaligned ranges are refused."""
    from plan_replay import PlanReplay
    from paper_2504_09186_amd import tnc
    from paper_2504_09186_amd._lib import MitncError
    c = synth.lattice_circuit(rows, cols, cycles, seed=seed)
    n = c.n_qubits
    spec = synth.output_spec(n, [n - 2, n - 1], seed=seed + 1)
    onet = oracle.build_network(c, spec)
    ref = oracle.sv_amplitudes(c, spec).reshape(-1)
    rng = np.random.default_rng(seed)
    net = tnc.Network(c, spec)
    net.set_path(oracle.greedy_path(onet))
    seen_merge = False
    for trial in range(6):
        net.set_slicing([int(x) for x in rng.choice(onet.closed_labels(), size=nsl, replace=False)])
        merged = tnc.Plan(net, merge_bits=nsl)
        plain = tnc.Plan(net)
        N = merged.n_slices
        cm, sch = _counts(merged, 0, N)
        cp, _ = _counts(plain, 0, N)
        assert (cm <= cp).all()
        fl = merged.steps()[:, 6]
        assert (fl * cm).sum() / N == pytest.approx(merged.stats.flops_reused_slice, rel=1e-12)
        got = PlanReplay(merged).run(0, N)
        assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref)
        al = merged.stats.merge_align_bits
        if al:
            seen_merge = True
            step = 1 << al
            if step < N:
                parts = sum(PlanReplay(merged).run(s, s + step) for s in range(0, N, step))
                assert np.linalg.norm(parts - ref) <= 1e-5 * np.linalg.norm(ref)
            with pytest.raises(MitncError, match="multiple"):
                merged.schedule(1, N)
    assert seen_merge


def test_merge_options_validated(lib):
    from paper_2504_09186_amd import tnc
    from paper_2504_09186_amd._lib import MitncError
    c, spec, onet, net = _nets(3, 4, 8, seed=3, nopen=2)
    net.set_path(oracle.greedy_path(onet))
    net.set_slicing([2, 589831, 131074, 458759])
    with pytest.raises(MitncError, match="merge_bits"):
        tnc.Plan(net, merge_bits=13)
    assert tnc.Plan(net, merge_bits=4).stats.n_merged > 0
    with pytest.raises(MitncError, match="post-lifetime merge"):
        tnc.Plan(net, merge_bits=4, differentiable=True)


def test_branch_exchange_keeps_result_and_lowers_flops(lib):
    """Branch exchange (Sec. III-B) on a greedy path with sliced indices:
    the reported flops never rise, the path stays a valid SSA path with the
    same amplitudes, and the plan's executed flops (merge-aware, no
    hoisting) after the exchange equal the reported count."""
    from plan_replay import PlanReplay
    from paper_2504_09186_amd import tnc
    c = synth.lattice_circuit(4, 4, 10, seed=5)
    spec = synth.output_spec(16, [15], seed=6)
    onet = oracle.build_network(c, spec)
    path = oracle.greedy_path(onet)
    ref = oracle.sv_amplitudes(c, spec).reshape(-1)
    rng = np.random.default_rng(12)
    improved = 0
    for trial in range(4):
        net = tnc.Network(c, spec)
        net.set_path(path)
        sl = [int(x) for x in rng.choice(onet.closed_labels(), size=5, replace=False)]
        net.set_slicing(sl)
        before, after = net.branch_exchange(window_bits=0, merge_bits=5, max_log2=30)
        assert after <= before
        improved += after < before
        plan = tnc.Plan(net, merge_bits=5, no_hoist=True)
        assert plan.stats.flops_reused_slice * plan.n_slices == pytest.approx(after, rel=1e-12)
        got = PlanReplay(plan).run(0, plan.n_slices)
        assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref)
    assert improved > 0


def test_reverse_groups_structure(lib):
    """Grouped reverse pass (every kept node deferred): each deferral root is
    a kept node (its sliced bits all at or above a level its parent's are
    not), so a nested root has a strictly larger level than the one above
    it; the plan's workspace grows by one term buffer per root; with
    deferral off there are no groups."""
    from paper_2504_09186_amd import tnc
    c = synth.lattice_circuit(4, 5, 10, seed=31)
    bits = synth.random_bitstrings(20, 16, seed=32)
    spec = np.full(20, -2, dtype=np.int8)
    net = tnc.Network(c, spec, bits)
    net.path_search(seed=31, trials=8, max_log2=30)
    rng = np.random.default_rng(33)
    onet = oracle.build_network(c, spec, bits)
    net.set_slicing([int(x) for x in rng.choice(onet.closed_labels(), size=4, replace=False)])
    off = tnc.Plan(net, differentiable=True, reverse_defer=-1)
    allg = tnc.Plan(net, differentiable=True, reverse_defer=1)
    model = tnc.Plan(net, differentiable=True, reverse_defer=0)
    assert off.stats.n_reverse_groups == 0
    assert allg.stats.n_reverse_groups > 0
    assert 0 <= model.stats.n_reverse_groups <= allg.stats.n_reverse_groups
    assert allg.stats.workspace_bytes > off.stats.workspace_bytes
    # kept nodes: level strictly above the parent's (level -1 = never recomputed)
    steps = [allg.step_info(i) for i in range(allg.stats.n_steps)]
    parent = {}
    for st in steps:
        parent[st["a"]] = st["out"]
        parent[st["b"]] = st["out"]
    lv = lambda v: 10 ** 6 if allg.node_info(v)["level"] < 0 else allg.node_info(v)["level"]  # noqa: E731
    kept = [st["out"] for st in steps if not st["root"] and lv(st["out"]) > lv(parent[st["out"]])]
    assert len(kept) >= allg.stats.n_reverse_groups
    # the reverse schedule itself (levels, each adjoint written once) is unchanged by grouping
    assert off.reverse_info() == allg.reverse_info()


@pytest.mark.parametrize("merge", [0, 4])
def test_range_prologue_replay(lib, merge):
    """The range prologue (steps a slice range computes once, batched by
    dependency level): with prologue_bits 0 and 3 the host replay of the
    library's launch list (prologue first) sums to the state vector over
    whole ranges and aligned blocks, with and without merges; a range that
    crosses a 2^3 block is refused when prologue_bits is 3."""
    from plan_replay import PlanReplay
    from paper_2504_09186_amd import tnc
    from paper_2504_09186_amd._lib import MitncError
    c = synth.lattice_circuit(4, 4, 10, seed=7)
    spec = synth.output_spec(16, [13, 14, 15], seed=8)
    net = tnc.Network(c, spec)
    net.path_search(seed=9, trials=8, max_log2=11, min_sliced=5, max_sliced=5)
    ref = oracle.sv_amplitudes(c, spec).reshape(-1)
    for pb in (0, 3):
        plan = tnc.Plan(net, merge_bits=merge, prologue_bits=pb)
        assert plan.stats.n_batched_small >= 2
        step = 1 << max(pb, plan.stats.merge_align_bits, 0) if pb else plan.n_slices
        got = sum(PlanReplay(plan).run(s0, s0 + step) for s0 in range(0, plan.n_slices, step))
        assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref), (pb, merge)
        if pb:
            with pytest.raises(MitncError, match="aligned block"):
                plan.schedule(0, 16)
