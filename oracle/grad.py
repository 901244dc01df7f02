"""Reverse-mode contraction for gate-tensor gradients (oracle side).

Not in the paper; this is the problem definition of the differentiation form:
loss L = sum_b log|a_b|^2 over a batch of amplitudes, gradients with respect to
every single-qubit gate tensor, each gate instance an independent complex
parameter.

Rule: for a step C = contract(A, B), the adjoint of A is the contraction of
the adjoint of C with B onto A's labels, and symmetrically for B (this is the
same pairwise contraction, with the batch labels of the step kept).  The
adjoint of a sliced leaf is added into the full leaf's adjoint at the sliced
values.  The holomorphic VJP J = sum_b w_b da_b/dG is returned; for the loss,
w_b = 1/a_b and the torch-convention gradient (dL/dRe + i dL/dIm) is
2 * conj(J).
Parity: pinned in tests against the state-vector environment formula and
central finite differences.
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Tuple

import numpy as np

from .contract import contract_pair, slice_leaves, slice_values
from .network import Network


def loss_log_abs2(amps: np.ndarray) -> float:
    a = np.asarray(amps).reshape(-1)
    return float(np.sum(np.log(np.abs(a) ** 2)))


def torch_convention_grad(j: np.ndarray) -> np.ndarray:
    return 2.0 * np.conj(j)


def _forward_store(arrays, labels, output, path):
    n = len(arrays)
    nodes: Dict[int, Tuple[np.ndarray, Tuple[int, ...]]] = {i: (arrays[i], labels[i]) for i in range(n)}
    count: Dict[int, int] = {}
    for lab in labels:
        for x in lab:
            count[x] = count.get(x, 0) + 1
    out = set(output)
    alive = set(range(n))
    for t, (i, j) in enumerate(path):
        a, la = nodes[i]
        b, lb = nodes[j]
        alive.discard(i)
        alive.discard(j)
        for x in la:
            count[x] -= 1
        for x in lb:
            count[x] -= 1
        keep = {x for x in set(la) | set(lb) if count.get(x, 0) > 0 or x in out}
        c, lc = contract_pair(a, la, b, lb, keep)
        for x in lc:
            count[x] = count.get(x, 0) + 1
        nodes[n + t] = (c, lc)
        alive.add(n + t)
    return nodes


def tn_gate_gradients(net: Network, path: Sequence[Tuple[int, int]], weights: np.ndarray,
                      sliced: Sequence[int] = (), slice_ids=None) -> Dict[int, np.ndarray]:
    """Holomorphic VJP sum_o w_o da_o/dG_l for every single-qubit gate leaf l,
    summed over the given slices (default all).  {circuit gate index: 2x2}."""
    n = net.n_leaves
    s = len(sliced)
    if slice_ids is None:
        slice_ids = range(1 << s)
    leaf_to_gate = {leaf: g for g, leaf in net.gate_leaf.items()
                    if net.arrays[leaf].shape == (2, 2)}
    # which nodes have a single-qubit gate leaf below them
    has_grad = {i: (i in leaf_to_gate) for i in range(n)}
    for t, (i, j) in enumerate(path):
        has_grad[n + t] = has_grad[i] or has_grad[j]
    grads = {g: np.zeros((2, 2), dtype=np.complex128) for g in leaf_to_gate.values()}
    w = np.asarray(weights, dtype=np.complex128)
    for sid in slice_ids:
        vals = slice_values(sid, s)
        arrays, labels = slice_leaves(net, sliced, vals)
        nodes = _forward_store(arrays, labels, net.output, path)
        root = n + len(path) - 1
        rc, rl = nodes[root]
        # seed in the root's own label order
        seed = np.transpose(w.reshape([net.dims[x] for x in net.output]),
                            [net.output.index(x) for x in rl])
        adj: Dict[int, np.ndarray] = {root: seed}
        for t in range(len(path) - 1, -1, -1):
            cid = n + t
            if cid not in adj:
                continue
            cbar = adj.pop(cid)
            lc = nodes[cid][1]
            i, j = path[t]
            for mine, other in ((i, j), (j, i)):
                if not has_grad[mine]:
                    continue
                b, lb = nodes[other]
                la = nodes[mine][1]
                abar, labs = contract_pair(cbar, lc, b, lb, keep=set(la))
                abar = np.transpose(abar, [labs.index(x) for x in la])
                adj[mine] = adj[mine] + abar if mine in adj else abar
        for leaf, g in leaf_to_gate.items():
            if leaf not in adj:
                continue
            a = adj[leaf]
            full_labels = list(net.labels[leaf])
            idx: List = []
            k = 0
            for x in full_labels:
                if x in sliced:
                    idx.append(vals[list(sliced).index(x)])
                else:
                    idx.append(slice(None))
                    k += 1
            grads[g][tuple(idx)] += a
    return grads
