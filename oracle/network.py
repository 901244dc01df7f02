"""Circuit -> tensor network (oracle side).

Paper, Sec. II-A: a circuit is represented as a tensor network whose nodes are
tensors and whose edges are shared indices; contracting eliminates shared edges
until one tensor remains.  Here every gate instance is a leaf tensor, the
initial |0> of each qubit is a [1, 0] leaf, each fixed output bit b is an e_b
leaf, open output qubits keep their last wire segment as an open index, and
batched output qubits share one batch hyperindex (dimension = number of
bitstrings) through projector leaves P[x, j] = [bits[j, q] == x].

Edge labels are canonical (they identify the same edge on any implementation):
the wire segment of qubit q that follows its t-th gate (t = 0 is the segment
after the initial state) has label ``q * 65536 + t``.  The batch hyperindex
has label ``BATCH`` (-1).

Canonical leaf order: gate instances in circuit order, then the initial-state
leaves for qubits 0..n-1, then the output projector leaves for every fixed or
batched qubit in increasing qubit order.

Output labels: the batch label first (if any), then the final segments of the
open qubits in increasing qubit order, so that qubit order is most-significant
first.  Parity: pinned by the state-vector comparison in tests.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np

BATCH = -1


def wire_label(q: int, t: int) -> int:
    return q * 65536 + t


@dataclass
class Network:
    n_qubits: int
    arrays: List[np.ndarray]
    labels: List[Tuple[int, ...]]
    output: Tuple[int, ...]
    dims: Dict[int, int]
    gate_leaf: Dict[int, int] = field(default_factory=dict)  # circuit gate index -> leaf id
    n_batch: int = 0

    @property
    def n_leaves(self) -> int:
        return len(self.arrays)

    def closed_labels(self) -> List[int]:
        """Binary edges shared by exactly two leaves and not in the output."""
        count: Dict[int, int] = {}
        for lab in self.labels:
            for x in lab:
                count[x] = count.get(x, 0) + 1
        out = set(self.output)
        return sorted(x for x, c in count.items() if c == 2 and x not in out and x != BATCH)


def build_network(circuit, spec: np.ndarray, batch_bits: Optional[np.ndarray] = None) -> Network:
    """Build the network of <x|U|0...0> for the request ``spec``.

    spec[q]: 0/1 fixed output bit, -1 open, -2 batched (bit taken from
    ``batch_bits[:, q_rank]`` where q_rank counts batched qubits in order).
    """
    n = circuit.n_qubits
    spec = np.asarray(spec)
    seg = [0] * n  # current segment index per qubit
    arrays: List[np.ndarray] = []
    labels: List[Tuple[int, ...]] = []
    gate_leaf: Dict[int, int] = {}
    for gi, g in enumerate(circuit.gates):
        if g.arity == 1:
            (q,) = g.qubits
            lin = wire_label(q, seg[q])
            seg[q] += 1
            lout = wire_label(q, seg[q])
            arrays.append(np.array(g.matrix, dtype=np.complex128))
            labels.append((lout, lin))
        else:
            q0, q1 = g.qubits
            i0, i1 = wire_label(q0, seg[q0]), wire_label(q1, seg[q1])
            seg[q0] += 1
            seg[q1] += 1
            o0, o1 = wire_label(q0, seg[q0]), wire_label(q1, seg[q1])
            arrays.append(np.array(g.matrix, dtype=np.complex128).reshape(2, 2, 2, 2))
            labels.append((o0, o1, i0, i1))
        gate_leaf[gi] = len(arrays) - 1
    for q in range(n):
        arrays.append(np.array([1.0, 0.0], dtype=np.complex128))
        labels.append((wire_label(q, 0),))
    batched = [q for q in range(n) if spec[q] == -2]
    n_batch = 0
    if batched:
        if batch_bits is None:
            raise ValueError("batched qubits need batch_bits")
        batch_bits = np.asarray(batch_bits, dtype=np.uint8)
        n_batch = batch_bits.shape[0]
        if batch_bits.shape[1] != len(batched):
            raise ValueError("batch_bits must have one column per batched qubit")
    dims: Dict[int, int] = {}
    for q in range(n):
        last = wire_label(q, seg[q])
        if spec[q] in (0, 1):
            e = np.zeros(2, dtype=np.complex128)
            e[int(spec[q])] = 1.0
            arrays.append(e)
            labels.append((last,))
        elif spec[q] == -2:
            col = batched.index(q)
            p = np.zeros((2, n_batch), dtype=np.complex128)
            p[batch_bits[:, col], np.arange(n_batch)] = 1.0
            arrays.append(p)
            labels.append((last, BATCH))
        elif spec[q] != -1:
            raise ValueError(f"bad output spec {spec[q]} for qubit {q}")
    out = []
    if batched:
        out.append(BATCH)
    out += [wire_label(q, seg[q]) for q in range(n) if spec[q] == -1]
    for lab in labels:
        for x in lab:
            dims[x] = 2
    if batched:
        dims[BATCH] = n_batch
    return Network(n_qubits=n, arrays=arrays, labels=labels, output=tuple(out), dims=dims,
                   gate_leaf=gate_leaf, n_batch=n_batch)
