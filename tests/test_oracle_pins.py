"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test fixes the oracle by an independent route: closed forms, unitarity,
brute-force state vectors, explicit loops over index values, normalisation,
invariance under contraction order and slicing, finite differences.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth
from oracle.contract import contract_pair, slice_values
from synth.circuits import Circuit, Gate


# ---------------------------------------------------------------- gates
@pytest.mark.parametrize("name", ["sqrt_x", "sqrt_y", "sqrt_w", "fsim"])
def test_gate_unitary(name):
    u = synth.gate_matrix(name)
    eye = np.eye(u.shape[0])
    assert np.max(np.abs(u.conj().T @ u - eye)) <= 1e-14


def test_sqrt_gates_square_to_paulis():
    x = np.array([[0, 1], [1, 0]], dtype=complex)
    y = np.array([[0, -1j], [1j, 0]], dtype=complex)
    w = np.array([[0, np.exp(-1j * np.pi / 4)], [np.exp(1j * np.pi / 4), 0]])
    assert np.allclose(synth.sqrt_x() @ synth.sqrt_x(), x, atol=1e-15)
    assert np.allclose(synth.sqrt_y() @ synth.sqrt_y(), y, atol=1e-15)
    assert np.allclose(synth.sqrt_w() @ synth.sqrt_w(), w, atol=1e-15)


def test_fsim_action():
    f = synth.fsim()
    e = np.eye(4)
    assert np.allclose(f @ e[0], e[0])
    assert np.allclose(f @ e[1], -1j * e[2])  # |01> -> -i|10>
    assert np.allclose(f @ e[2], -1j * e[1])
    assert np.allclose(f @ e[3], np.exp(-1j * np.pi / 6) * e[3])


def test_generator_no_repeat_and_patterns():
    c = synth.lattice_circuit(3, 4, 8, seed=1000)
    last = {}
    for g in c.gates:
        if g.arity == 1:
            (q,) = g.qubits
            assert last.get(q) != g.name
            last[q] = g.name
    # every cycle touches each qubit with one single-qubit gate
    assert sum(1 for g in c.gates if g.arity == 1) == 12 * 8
    # pattern pairs are disjoint within a cycle and are lattice neighbours
    for pat in "ABCD":
        pairs = synth.circuits.couplers(3, 4, pat)
        qs = [q for p in pairs for q in p]
        assert len(qs) == len(set(qs))
        for a, b in pairs:
            ra, ca = divmod(a, 4)
            rb, cb = divmod(b, 4)
            assert abs(ra - rb) + abs(ca - cb) == 1
    assert synth.lattice_circuit(3, 4, 8, seed=1000).gates == c.gates


# ---------------------------------------------------------------- pairwise contraction
def _loop_contract(a, la, b, lb, out_labels):
    """Einstein summation written as explicit loops over every label value."""
    labels = sorted(set(la) | set(lb))
    dims = {}
    for x, d in zip(la, a.shape):
        dims[x] = d
    for x, d in zip(lb, b.shape):
        dims[x] = d
    c = np.zeros([dims[x] for x in out_labels], dtype=complex)
    for vals in itertools.product(*[range(dims[x]) for x in labels]):
        v = dict(zip(labels, vals))
        c[tuple(v[x] for x in out_labels)] += a[tuple(v[x] for x in la)] * b[tuple(v[x] for x in lb)]
    return c


@pytest.mark.parametrize("seed", range(6))
def test_contract_pair_matches_loops(seed):
    rng = np.random.default_rng(seed)
    # labels 0..6; pick A and B label sets with common, free and batch labels
    la = list(rng.permutation([0, 1, 2, 3, 4])[: rng.integers(2, 5)])
    lb = list(rng.permutation([2, 3, 4, 5, 6])[: rng.integers(2, 5)])
    common = [x for x in la if x in lb]
    keep_batch = set(common[:1]) if (common and seed % 2) else set()
    keep = set(x for x in la + lb if x not in common) | keep_batch
    a = synth.complex_normal([2] * len(la), seed=10 + seed)
    b = synth.complex_normal([2] * len(lb), seed=20 + seed)
    c, lc = contract_pair(a, la, b, lb, keep)
    ref = _loop_contract(a, la, b, lb, list(lc))
    assert np.max(np.abs(c - ref)) < 1e-13


# ---------------------------------------------------------------- TN vs state vector
@pytest.mark.parametrize("rows,cols,cycles,seed", [
    (3, 4, 8, 1000), (2, 2, 0, 1), (2, 2, 3, 2), (2, 3, 5, 3), (3, 3, 6, 4), (1, 4, 7, 5)])
def test_tn_matches_statevector_open(rows, cols, cycles, seed):
    c = synth.lattice_circuit(rows, cols, cycles, seed=seed)
    n = c.n_qubits
    spec = synth.output_spec(n, list(range(max(0, n - 4), n)), seed=seed + 7)
    net = oracle.build_network(c, spec)
    a = oracle.contract_network(net, oracle.greedy_path(net))
    ref = oracle.sv_amplitudes(c, spec)
    assert np.max(np.abs(a - ref)) < 1e-13


def test_config1_single_amplitude_and_slices():
    """3x4 lattice, 8 cycles, 2 sliced indices, one random bitstring."""
    c = synth.lattice_circuit(3, 4, 8, seed=1000)
    spec = synth.output_spec(12, [], seed=2000)
    net = oracle.build_network(c, spec)
    path = oracle.greedy_path(net)
    sliced = oracle.choose_slices(net, path, cap_log2=7, min_sliced=2)[:2]
    assert len(sliced) == 2
    total, parts = oracle.contract_sliced(net, path, sliced, per_slice=True)
    assert len(parts) == 4
    ref = oracle.sv_amplitudes(c, spec)
    assert abs(total - ref) < 1e-14
    assert abs(oracle.contract_network(net, path) - ref) < 1e-14


def test_normalisation_all_open():
    c = synth.lattice_circuit(3, 4, 8, seed=1000)
    spec = np.full(12, -1, dtype=np.int8)
    net = oracle.build_network(c, spec)
    amps = oracle.contract_network(net, oracle.greedy_path(net))
    assert amps.shape == (2,) * 12
    assert abs(np.sum(np.abs(amps) ** 2) - 1.0) < 1e-12
    # qubit 0 is the most significant bit: compare with the flat state vector
    assert np.max(np.abs(amps.reshape(-1) - oracle.sv_state(c).reshape(-1))) < 1e-13


def test_invariance_paths_and_slicing():
    c = synth.lattice_circuit(3, 3, 6, seed=11)
    spec = synth.output_spec(9, [7, 8], seed=12)
    net = oracle.build_network(c, spec)
    ref = oracle.contract_network(net, oracle.greedy_path(net))
    for s in range(5):
        p = oracle.random_greedy_path(net, seed=s, jitter=1.0)
        assert np.max(np.abs(oracle.contract_network(net, p) - ref)) < 1e-13
    closed = net.closed_labels()
    rng = np.random.default_rng(5)
    p = oracle.greedy_path(net)
    for ns in (1, 2, 3):
        sl = list(rng.choice(closed, size=ns, replace=False))
        assert np.max(np.abs(oracle.contract_sliced(net, p, sl) - ref)) < 1e-13


def test_slice_id_bit_order():
    # last listed sliced index is the least significant bit of the slice id
    assert slice_values(1, 3) == [0, 0, 1]
    assert slice_values(4, 3) == [1, 0, 0]
    assert slice_values(6, 3) == [1, 1, 0]


# ---------------------------------------------------------------- closed-form special cases
def test_depth_zero_delta():
    c = Circuit(n_qubits=3, gates=[])
    for x in range(8):
        bits = [(x >> (2 - q)) & 1 for q in range(3)]
        spec = np.array(bits, dtype=np.int8)
        net = oracle.build_network(c, spec)
        a = oracle.contract_network(net, oracle.greedy_path(net))
        assert abs(a - (1.0 if x == 0 else 0.0)) < 1e-15


def test_single_qubit_only_product():
    rng = np.random.default_rng(3)
    names = ["sqrt_x", "sqrt_y", "sqrt_w"]
    gates = []
    prod_u = [np.eye(2, dtype=complex) for _ in range(4)]
    for layer in range(3):
        for q in range(4):
            nm = names[rng.integers(0, 3)]
            u = synth.gate_matrix(nm)
            gates.append(Gate(nm, (q,), u))
            prod_u[q] = u @ prod_u[q]
    c = Circuit(n_qubits=4, gates=gates)
    for x in (0, 5, 11, 15):
        bits = [(x >> (3 - q)) & 1 for q in range(4)]
        net = oracle.build_network(c, np.array(bits, dtype=np.int8))
        a = oracle.contract_network(net, oracle.greedy_path(net))
        expect = np.prod([prod_u[q][bits[q], 0] for q in range(4)])
        assert abs(a - expect) < 1e-15


def test_fsim_only_keeps_zero_state():
    gates = []
    for cyc in range(4):
        for a, b in synth.circuits.couplers(2, 3, "ABCD"[cyc]):
            gates.append(Gate("fsim", (a, b), synth.fsim()))
    c = Circuit(n_qubits=6, gates=gates)
    net = oracle.build_network(c, np.zeros(6, dtype=np.int8))
    assert abs(oracle.contract_network(net, oracle.greedy_path(net)) - 1.0) < 1e-15


def test_batched_equals_fixed():
    c = synth.lattice_circuit(2, 3, 4, seed=21)
    bits = synth.random_bitstrings(6, 8, seed=22)
    spec = np.full(6, -2, dtype=np.int8)
    net = oracle.build_network(c, spec, bits)
    amps = oracle.contract_network(net, oracle.greedy_path(net))
    for b in range(8):
        netb = oracle.build_network(c, bits[b].astype(np.int8))
        ab = oracle.contract_network(netb, oracle.greedy_path(netb))
        assert abs(amps[b] - ab) < 1e-14
    assert np.max(np.abs(amps - oracle.sv_amplitudes(c, spec, bits))) < 1e-14


# ---------------------------------------------------------------- Eq. (1) index overhead
def test_index_overhead_matches_counted_flops():
    c = synth.lattice_circuit(2, 3, 5, seed=31)
    spec = synth.output_spec(6, [5], seed=32)
    net = oracle.build_network(c, spec)
    path = oracle.greedy_path(net)
    c_ori = oracle.count_contraction_flops(net, path)
    for a in net.closed_labels()[:6]:
        c_a = oracle.count_contraction_flops(net, path, [a], slice_id=1)
        assert oracle.index_overhead(net, path, a) == pytest.approx(2.0 * c_a / c_ori, rel=1e-12)
        assert oracle.index_overhead(net, path, a) >= 1.0 - 1e-12


# ---------------------------------------------------------------- gradients
def _fd_gate_grad(c, spec, bits, gate_index, h=1e-6):
    """Central finite differences of L = sum log|a|^2 w.r.t. Re and Im of each
    entry of one gate matrix, via the state vector."""
    out = np.zeros((2, 2), dtype=complex)
    for i in range(2):
        for j in range(2):
            vals = []
            for step in (h, -h, 1j * h, -1j * h):
                gates = list(c.gates)
                g = gates[gate_index]
                m = g.matrix.copy()
                m[i, j] += step
                gates[gate_index] = Gate(g.name, g.qubits, m)
                c2 = Circuit(n_qubits=c.n_qubits, gates=gates)
                vals.append(oracle.loss_log_abs2(oracle.sv_amplitudes(c2, spec, bits)))
            out[i, j] = (vals[0] - vals[1]) / (2 * h) + 1j * (vals[2] - vals[3]) / (2 * h)
    return out


def test_sv_gradient_matches_finite_differences():
    c = synth.lattice_circuit(2, 2, 3, seed=41)
    bits = synth.random_bitstrings(4, 4, seed=42)
    spec = np.full(4, -2, dtype=np.int8)
    amps = oracle.sv_amplitudes(c, spec, bits)
    j = oracle.sv_gate_gradients(c, spec, 1.0 / amps, bits)
    for gi in c.one_qubit_gate_ids()[:5]:
        fd = _fd_gate_grad(c, spec, bits, gi)
        assert np.max(np.abs(oracle.torch_convention_grad(j[gi]) - fd)) < 1e-6


@pytest.mark.parametrize("nsliced", [0, 2])
def test_tn_gradient_matches_sv_environment(nsliced):
    c = synth.lattice_circuit(2, 3, 4, seed=51)
    bits = synth.random_bitstrings(6, 4, seed=52)
    spec = np.full(6, -2, dtype=np.int8)
    net = oracle.build_network(c, spec, bits)
    path = oracle.greedy_path(net)
    amps = oracle.contract_network(net, path)
    w = 1.0 / amps
    sliced = net.closed_labels()[3:3 + nsliced]
    jt = oracle.tn_gate_gradients(net, path, w, sliced=sliced)
    js = oracle.sv_gate_gradients(c, spec, w, bits)
    assert set(jt) == set(c.one_qubit_gate_ids())
    for g in jt:
        assert np.max(np.abs(jt[g] - js[g])) < 1e-12


def test_tn_gradient_open_outputs():
    c = synth.lattice_circuit(2, 2, 4, seed=61)
    spec = synth.output_spec(4, [2, 3], seed=62)
    net = oracle.build_network(c, spec)
    path = oracle.greedy_path(net)
    w = synth.complex_normal((2, 2), seed=63)
    jt = oracle.tn_gate_gradients(net, path, w)
    js = oracle.sv_gate_gradients(c, spec, w)
    for g in jt:
        assert np.max(np.abs(jt[g] - js[g])) < 1e-13


# ---------------------------------------------------------------- metrics
def test_metrics_closed_forms():
    a = synth.complex_normal(64, seed=71)
    assert oracle.rel_l2(a, a) == 0.0
    assert oracle.overlap_fidelity(a * (2 - 1j), a) == pytest.approx(1.0, abs=1e-14)
    assert oracle.xeb_ratio(a * 3.0, a) == pytest.approx(1.0, abs=1e-12)
    b = a + 1e-3 * synth.complex_normal(64, seed=72)
    assert 0 < oracle.rel_l2(b, a) < 2e-3


def _from_probs(p, scale, seed):
    """Amplitudes with |x|^2 proportional to p, arbitrary norm and phases."""
    rng = np.random.default_rng(seed)
    ph = np.exp(2j * np.pi * rng.random(len(p)))
    return scale * np.sqrt(np.asarray(p, dtype=np.float64)) * ph


def test_xeb_ratio_hand_values():
    """Linear XEB ratio (|B| sum p q - 1) / (|B| sum p^2 - 1) worked by hand on
    non-identical distributions; p (reference) and q (approximation) enter
    asymmetrically, so exchanging them in the denominator, dropping the
    normalisation or the -1 terms fails one of the cases."""
    p = [0.4, 0.3, 0.2, 0.1]          # sum p^2 = 0.30
    # q = (0.5, 0.5, 0, 0): sum p q = 0.35 -> (1.4 - 1) / (1.2 - 1) = 2
    # (with q in the denominator: sum q^2 = 0.5 -> 0.4 / 1.0 = 0.4)
    ref = _from_probs(p, 3e-5, 1)
    got = _from_probs([0.5, 0.5, 0.0, 0.0], 7.0, 2)
    assert oracle.xeb_ratio(got, ref) == pytest.approx(2.0, rel=1e-12)
    # q uniform: sum p q = 1/4 -> (1 - 1) / 0.2 = 0
    assert abs(oracle.xeb_ratio(_from_probs([1, 1, 1, 1], 0.1, 3), ref)) < 1e-12
    # q reversed: sum p q = 0.2 -> (0.8 - 1) / 0.2 = -1
    assert oracle.xeb_ratio(_from_probs(p[::-1], 2.0, 4), ref) == pytest.approx(-1.0, rel=1e-12)
    # |B| = 2: p = (1/4, 3/4), q = (1/2, 1/2): sum p q = 1/2 -> (1 - 1) / (2 * 5/8 - 1) = 0
    assert abs(oracle.xeb_ratio(np.array([1.0, 1j]), np.array([1.0, np.sqrt(3.0)]))) < 1e-12
    # |B| = 2: p = (1/4, 3/4), q = (3/4, 1/4): (2 * 3/8 - 1) / (2 * 5/8 - 1) = -1
    assert oracle.xeb_ratio(np.array([np.sqrt(3.0), 1.0]), np.array([1.0, 1j * np.sqrt(3.0)])) == \
        pytest.approx(-1.0, rel=1e-12)


def test_overlap_fidelity_hand_values():
    """|<a, b>|^2 / (|a|^2 |b|^2) with the conjugate on the reference."""
    # <(1, i), (1, -i)> = 1 + (-i)(-i) = 0; without the conjugate it would be 2 -> 1
    assert oracle.overlap_fidelity(np.array([1.0, -1j]), np.array([1.0, 1j])) == pytest.approx(0.0, abs=1e-15)
    # <(1, 0), (1, 1)> = 1, norms 1 and 2 -> 1/2
    assert oracle.overlap_fidelity(np.array([1.0, 1.0]), np.array([1.0, 0.0])) == pytest.approx(0.5, rel=1e-14)
    # <(1, i, 0), (2, 0, 2i)> = 2, norms 2 and 8 -> 4 / 16
    assert oracle.overlap_fidelity(np.array([2.0, 0.0, 2j]), np.array([1.0, 1j, 0.0])) == \
        pytest.approx(0.25, rel=1e-14)


def test_rel_l2_hand_values():
    """||b - a|| / ||a|| with the reference norm in the denominator."""
    # a = (3, 4), b = (3, 4 + 5i): ||b - a|| = 5, ||a|| = 5 (||b|| = sqrt 50)
    assert oracle.rel_l2(np.array([3.0, 4.0 + 5j]), np.array([3.0, 4.0])) == pytest.approx(1.0, rel=1e-15)
    # a = (1, 1, 1, 1), b = (1, 1, 1, 2i - 1): ||b - a|| = |2i - 2| = sqrt 8, ||a|| = 2
    assert oracle.rel_l2(np.array([1, 1, 1, 2j - 1]), np.ones(4)) == pytest.approx(np.sqrt(2.0), rel=1e-15)


# ---------------------------------------------------------------- oracle planning for large networks
def _is_valid_path(n, path):
    alive = set(range(n))
    for t, (i, j) in enumerate(path):
        if i == j or i not in alive or j not in alive:
            return False
        alive -= {i, j}
        alive.add(n + t)
    return len(path) == n - 1


@pytest.mark.parametrize("seed,imb", [(0, 0.1), (1, 0.5), (2, 0.7)])
def test_bisection_path_valid_and_same_amplitudes(seed, imb):
    """The recursive-bisection path is a valid SSA path (every tensor used
    once) and contracts to the state-vector amplitudes, sliced or not."""
    from oracle import planning
    c = synth.lattice_circuit(3, 4, 8, seed=70 + seed)
    spec = synth.output_spec(12, [9, 10, 11], seed=71)
    net = oracle.build_network(c, spec)
    path = planning.bisection_path(net, imbalance=imb, seed=seed, cutoff=4)
    assert _is_valid_path(net.n_leaves, path)
    ref = oracle.sv_amplitudes(c, spec).reshape(-1)
    got = oracle.contract_network(net, path).reshape(-1)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-14)
    sl = net.closed_labels()[5:8]
    assert np.allclose(oracle.contract_sliced(net, path, sl).reshape(-1), ref, rtol=1e-12, atol=1e-14)


def test_bitset_stats_match_path_stats():
    """The bitset statistics (C = A xor B plus shared outputs) give the same
    largest intermediate and flops as the set-based path_stats, with and
    without sliced labels."""
    from oracle import planning
    c = synth.lattice_circuit(4, 4, 10, seed=80)
    spec = synth.output_spec(16, [13, 14, 15], seed=81)
    net = oracle.build_network(c, spec)
    path = planning.bisection_path(net, seed=3)
    masks, out, labels = planning._bitsets(net)
    for sl in ([], net.closed_labels()[::17]):
        cut = sum(1 << labels.index(x) for x in sl)
        big, flops = planning._bit_stats(masks, out, path, cut)
        st = planning.path_stats(net, path, sl)
        assert big == max(s[0] for s in st)
        assert np.isclose(flops, sum(s[1] for s in st), rtol=1e-12)


def test_choose_slices_eval_follows_the_rule():
    """Slicing with evaluations reaches the cap, and each chosen label is
    the best (largest intermediate, then flops, then label) among the closed
    labels of the largest intermediates at that point: checked by brute
    force with path_stats."""
    from oracle import planning
    c = synth.lattice_circuit(3, 4, 10, seed=90)
    spec = synth.output_spec(12, [10, 11], seed=91)
    net = oracle.build_network(c, spec)
    path = planning.bisection_path(net, seed=1)
    cap = max(s[0] for s in planning.path_stats(net, path)) - 3
    chosen = planning.choose_slices_eval(net, path, cap)
    assert max(s[0] for s in planning.path_stats(net, path, chosen)) <= cap
    closed = net.closed_labels()
    for i, x in enumerate(chosen):
        before = chosen[:i]
        st = planning.path_stats(net, path, before)
        big = max(s[0] for s in st)
        keys = []
        for y in closed:
            if y in before:
                continue
            s2 = planning.path_stats(net, path, before + [y])
            keys.append((max(s[0] for s in s2), sum(s[1] for s in s2), y))
        best = min(keys)
        mine = [k for k in keys if k[2] == x][0]
        assert mine[:2] == best[:2]


# ------------------------------------------------------- lifetimes (Sec. III-B)
def _chain_net():
    """T0(a,b) T1(b,c) T2(c,d) T3(d,e), labels a..e = 1..5, open a and e."""
    rng = np.random.default_rng(77)
    arrs = [rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2)) for _ in range(4)]
    labels = [(1, 2), (2, 3), (3, 4), (4, 5)]
    net = oracle.Network(n_qubits=0, arrays=arrs, labels=labels, output=(1, 5), dims={x: 2 for x in range(1, 6)})
    return net, [(0, 1), (4, 2), (5, 3)]


def test_sliced_lifetimes_hand_chain():
    """Worked by hand: b ends at step 0; c starts at step 0 and ends at step
    1; d starts at step 1 and ends at step 2; b is below steps 1 and 2 but no
    longer alive there, and d is not below step 0."""
    net, path = _chain_net()
    below, alive = oracle.sliced_lifetimes(net, path, [2, 3, 4])
    assert below == [{2, 3}, {2, 3, 4}, {2, 3, 4}]
    assert alive == [{2, 3}, {3, 4}, {4}]


def test_sliced_lifetimes_count_distinct_partial_sums():
    """Brute force over the 8 slices of the chain: a step's output summed over
    the sliced labels that ended strictly below it takes exactly 2^|alive|
    distinct values (generic random tensors), which is the number of times
    the spindle must compute it."""
    net, path = _chain_net()
    t0, t1, t2, t3 = net.arrays
    below, alive = oracle.sliced_lifetimes(net, path, [2, 3, 4])
    vals = {}  # step -> {(b, c, d): vector over the open labels}
    for b in (0, 1):
        for c in (0, 1):
            for d in (0, 1):
                x = t0[:, b] * t1[b, c]           # step 0: open a
                y = x * t2[c, d]                  # step 1: open a
                z = np.outer(y * 1.0, t3[d, :])   # step 2: open a, e
                for t, v in enumerate((x, y, z)):
                    vals.setdefault(t, {})[(b, c, d)] = np.asarray(v).reshape(-1)
    name = {2: 0, 3: 1, 4: 2}
    for t in range(3):
        ended = below[t] - alive[t]
        groups = {}
        for key, v in vals[t].items():
            keep = tuple(key[name[x]] for x in sorted(alive[t]))
            groups[keep] = groups.get(keep, 0) + v
        # the partial sums differ between groups and the group count is 2^|alive|
        distinct = {tuple(np.round(g, 9)) for g in groups.values()}
        assert len(groups) == len(distinct) == 2 ** len(alive[t]), (t, ended)
        # summing over fewer labels than `ended` would leave more distinct values
        if ended:
            assert len({tuple(np.round(v, 9)) for v in vals[t].values()}) > 2 ** len(alive[t])
