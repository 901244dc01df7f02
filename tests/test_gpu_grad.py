"""Differentiation form on the GPU: gradients of L = sum_b log|a_b|^2 with
respect to every single-qubit gate matrix, through torch.autograd, against
the oracle's reverse-mode gradient (itself pinned to the state-vector
environment formula and finite differences in test_oracle_pins.py), and
against central finite differences of the GPU forward.

Tolerance: complex64 forward and reverse contractions, gradient compared in
relative L2 over all entries <= 1e-4.
"""
import numpy as np
import pytest

import oracle
import synth
from helpers import require_gpu

pytestmark = pytest.mark.gpu


def _setup(rows, cols, cycles, nbits, nsl, seed, batched=True, open_q=()):
    from paper_2504_09186_amd import tnc
    c = synth.lattice_circuit(rows, cols, cycles, seed=seed)
    n = c.n_qubits
    if batched:
        bits = synth.random_bitstrings(n, nbits, seed=seed + 1)
        spec = np.full(n, -2, dtype=np.int8)
    else:
        bits = None
        spec = synth.output_spec(n, list(open_q), seed=seed + 1)
    net = tnc.Network(c, spec, bits)
    onet = oracle.build_network(c, spec, bits)
    rng = np.random.default_rng(seed + 2)
    sliced = [int(x) for x in rng.choice(onet.closed_labels(), size=nsl, replace=False)] if nsl else []
    net.path_search(seed=seed, trials=8, max_log2=30)
    net.set_slicing(sliced)
    return c, spec, bits, net, onet, sliced


def _gpu_grad(net, c, defer=0):
    import torch
    from paper_2504_09186_amd import tnc
    plan = tnc.Plan(net, differentiable=True, reverse_defer=defer)
    plan.upload()
    mats = np.stack([g.matrix for g in c.gates if g.arity == 1])
    gates = torch.tensor(mats, dtype=torch.complex128, requires_grad=True)
    amps = tnc.AmplitudeFn().apply(gates, plan)
    loss = torch.sum(torch.log(torch.abs(amps) ** 2))
    loss.backward()
    torch.cuda.synchronize()
    return amps.detach().cpu().numpy(), gates.grad.numpy(), plan, float(loss)


@pytest.mark.parametrize("defer", [0, 1, -1])
@pytest.mark.parametrize("rows,cols,cycles,nbits,nsl,seed", [
    (2, 3, 5, 8, 0, 1), (3, 3, 6, 16, 2, 2), (3, 4, 8, 4, 3, 3), (2, 4, 6, 32, 1, 4)])
def test_gradient_matches_oracle(rows, cols, cycles, nbits, nsl, seed, defer):
    """defer: grouped reverse pass at the kept nodes the cost model picks
    (0), at every kept node (1: adjoints summed over runs of slices, nested
    groups), or not at all (-1)."""
    require_gpu()
    c, spec, bits, net, onet, sliced = _setup(rows, cols, cycles, nbits, nsl, seed)
    print(f"gradient case {rows}x{cols}x{cycles}, {nbits} bitstrings, sliced {sliced}, defer {defer}", flush=True)
    amps, grad, plan, _ = _gpu_grad(net, c, defer)
    if defer == 1 and nsl >= 2:
        assert plan.stats.n_reverse_groups > 0
    ref_amps = oracle.sv_amplitudes(c, spec, bits).reshape(-1)
    assert oracle.rel_l2(amps, ref_amps) < 1e-5
    opath = oracle.greedy_path(onet)
    j = oracle.tn_gate_gradients(onet, opath, 1.0 / ref_amps, sliced=sliced)
    ids = c.one_qubit_gate_ids()
    ref = np.stack([oracle.torch_convention_grad(j[g]) for g in ids])
    assert np.linalg.norm(grad - ref) <= 1e-4 * np.linalg.norm(ref)


def test_gradient_open_outputs_weighted():
    """Open outputs instead of a batch: the VJP weights come from a random
    real-valued loss L = sum_o c_o |a_o|^2."""
    require_gpu()
    import torch
    from paper_2504_09186_amd import tnc
    c, spec, bits, net, onet, sliced = _setup(3, 3, 6, 0, 2, 11, batched=False, open_q=(6, 7, 8))
    plan = tnc.Plan(net, differentiable=True)
    plan.upload()
    mats = np.stack([g.matrix for g in c.gates if g.arity == 1])
    gates = torch.tensor(mats, dtype=torch.complex128, requires_grad=True)
    amps = tnc.AmplitudeFn().apply(gates, plan)
    coef = torch.tensor(np.random.default_rng(12).uniform(0.5, 2.0, amps.numel()), dtype=torch.float64,
                        device=amps.device)
    loss = torch.sum(coef * torch.abs(amps) ** 2)
    loss.backward()
    a = oracle.sv_amplitudes(c, spec).reshape(-1)
    # dL/dz* for L = sum c |a|^2 gives the holomorphic weights w = c * conj(a)
    w = coef.cpu().numpy() * np.conj(a)
    js = oracle.sv_gate_gradients(c, spec, w)
    ref = np.stack([2.0 * np.conj(js[g]) for g in c.one_qubit_gate_ids()])
    assert np.linalg.norm(gates.grad.numpy() - ref) <= 1e-4 * np.linalg.norm(ref)


def test_gradient_finite_differences_gpu():
    """Central differences (h = 1e-3) of the GPU loss on 20 random gate
    entries (re and im) against the GPU gradient; the step is chosen so that
    truncation (~h^2) and complex64 rounding (~1e-7 |L| / h) stay small."""
    require_gpu()
    import torch
    from paper_2504_09186_amd import tnc
    c, spec, bits, net, onet, sliced = _setup(3, 4, 8, 16, 2, 21)
    amps, grad, plan, _ = _gpu_grad(net, c)
    mats = np.stack([g.matrix for g in c.gates if g.arity == 1])
    rng = np.random.default_rng(4003)
    h = 1e-3

    def loss_of(m):
        plan.set_gates(m)
        acc = plan.new_result()
        plan.execute(acc)
        torch.cuda.synchronize()
        # FP64 loss of the complex64-computed amplitudes
        return float(np.sum(np.log(np.abs(acc.cpu().numpy()) ** 2)))

    picks = [(int(rng.integers(len(mats))), int(rng.integers(2)), int(rng.integers(2))) for _ in range(20)]
    fd, gv = [], []
    for g, i, j in picks:
        for delta, part in ((h, 0), (1j * h, 1)):
            mp = mats.copy()
            mm = mats.copy()
            mp[g, i, j] += delta
            mm[g, i, j] -= delta
            fd.append((loss_of(mp) - loss_of(mm)) / (2 * h))
            gv.append(grad[g, i, j].real if part == 0 else grad[g, i, j].imag)
    fd, gv = np.array(fd), np.array(gv)
    assert np.linalg.norm(fd - gv) <= 1e-3 * np.linalg.norm(gv)


@pytest.mark.parametrize("defer", [0, 1])
def test_gradient_20_qubits_sliced(defer):
    """A 4x5 lattice (20 qubits), 10 cycles, 16 random bitstrings as a batch
    index, 4 sliced indices (16 slices, each recomputed by the backward):
    GPU gradient of L = sum log|a|^2 against the oracle's reverse-mode
    gradient on the same slicing, relative L2 <= 1e-4; with the grouped
    reverse pass where the cost model picks it and at every kept node."""
    require_gpu()
    c, spec, bits, net, onet, sliced = _setup(4, 5, 10, 16, 4, 31)
    print(f"gradient case 4x5x10, 16 bitstrings, sliced {sliced}, defer {defer}", flush=True)
    amps, grad, plan, _ = _gpu_grad(net, c, defer)
    if defer == 1:
        assert plan.stats.n_reverse_groups > 0
    assert plan.n_slices == 16
    opath = oracle.greedy_path(onet)
    ref_amps = oracle.contract_sliced(onet, opath, sliced).reshape(-1)
    assert oracle.rel_l2(amps, ref_amps) < 1e-5
    j = oracle.tn_gate_gradients(onet, opath, 1.0 / ref_amps, sliced=sliced)
    ref = np.stack([oracle.torch_convention_grad(j[g]) for g in c.one_qubit_gate_ids()])
    assert np.linalg.norm(grad - ref) <= 1e-4 * np.linalg.norm(ref)


def test_two_forwards_before_backward():
    """loss = f(G1) + f(G2) with two forwards on one plan before the backward:
    each backward differentiates at its own forward's gate matrices (the
    plan's gate leaves were replaced by the second forward)."""
    require_gpu()
    import torch
    from paper_2504_09186_amd import tnc
    c, spec, bits, net, onet, sliced = _setup(3, 3, 6, 8, 2, 41)
    plan = tnc.Plan(net, differentiable=True)
    plan.upload()
    m1 = np.stack([g.matrix for g in c.gates if g.arity == 1])
    rng = np.random.default_rng(42)
    m2 = m1 + 0.05 * (rng.standard_normal(m1.shape) + 1j * rng.standard_normal(m1.shape))
    g1 = torch.tensor(m1, dtype=torch.complex128, requires_grad=True)
    g2 = torch.tensor(m2, dtype=torch.complex128, requires_grad=True)
    f = tnc.AmplitudeFn()
    loss = torch.sum(torch.log(torch.abs(f.apply(g1, plan)) ** 2)) + \
        torch.sum(torch.log(torch.abs(f.apply(g2, plan)) ** 2))
    loss.backward()
    opath = oracle.greedy_path(onet)
    ids = c.one_qubit_gate_ids()
    for g, m in ((g1, m1), (g2, m2)):
        c2 = synth.Circuit(c.n_qubits, [synth.Gate(gt.name, gt.qubits, m[ids.index(i)] if gt.arity == 1
                                                   else gt.matrix) for i, gt in enumerate(c.gates)])
        on2 = oracle.build_network(c2, spec, bits)
        a = oracle.contract_network(on2, opath).reshape(-1)
        j = oracle.tn_gate_gradients(on2, opath, 1.0 / a)
        ref = np.stack([oracle.torch_convention_grad(j[k]) for k in ids])
        assert np.linalg.norm(g.grad.numpy() - ref) <= 1e-4 * np.linalg.norm(ref)
