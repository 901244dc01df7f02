"""Brute-force state-vector amplitudes and gradients (small circuits only).

Not in the paper (which contrasts tensor networks with state vectors in its
Introduction); used as the independent pin of the tensor-network oracle:
amp(x) = <x| U_L ... U_1 |0...0>, with the gate conventions of ``synth``.

``sv_gate_gradients`` evaluates, for every single-qubit gate instance l, the
environment formula
    d(sum_o w_o a_o)/dG_l[i, j] = sum_rest phi_l[q=i, rest] psi_l[q=j, rest],
with psi_l = U_{<l} |0> (state just before gate l) and phi_l = U_{>l}^T c
(c[x] = sum of the weights w_o of the outputs o that select basis state x).
Parity: pinned against finite differences and closed forms in tests.
"""
from __future__ import annotations

from typing import Dict, Optional

import numpy as np


def _apply(state: np.ndarray, mat: np.ndarray, qubits) -> np.ndarray:
    if len(qubits) == 1:
        (q,) = qubits
        st = np.tensordot(mat, state, axes=([1], [q]))
        return np.moveaxis(st, 0, q)
    q0, q1 = qubits
    u = mat.reshape(2, 2, 2, 2)
    st = np.tensordot(u, state, axes=([2, 3], [q0, q1]))
    return np.moveaxis(st, [0, 1], [q0, q1])


def _apply_transpose(state: np.ndarray, mat: np.ndarray, qubits) -> np.ndarray:
    """Apply U^T (plain transpose, no conjugation)."""
    if len(qubits) == 1:
        return _apply(state, mat.T, qubits)
    u = mat.reshape(2, 2, 2, 2).transpose(2, 3, 0, 1).reshape(4, 4)
    return _apply(state, u, qubits)


def sv_state(circuit) -> np.ndarray:
    n = circuit.n_qubits
    state = np.zeros((2,) * n, dtype=np.complex128)
    state[(0,) * n] = 1.0
    for g in circuit.gates:
        state = _apply(state, g.matrix, g.qubits)
    return state


def _output_index_list(n: int, spec, batch_bits=None):
    """Basis-state index tuple for every entry of the requested result, in the
    result's own order (batch first, then open qubits, most significant first)."""
    spec = np.asarray(spec)
    open_q = [q for q in range(n) if spec[q] == -1]
    batched = [q for q in range(n) if spec[q] == -2]
    nb = batch_bits.shape[0] if batched else 1
    entries = []
    for b in range(nb):
        for o in range(1 << len(open_q)):
            x = [int(spec[q]) if spec[q] >= 0 else 0 for q in range(n)]
            for k, q in enumerate(open_q):
                x[q] = (o >> (len(open_q) - 1 - k)) & 1
            for k, q in enumerate(batched):
                x[q] = int(batch_bits[b, k])
            entries.append(tuple(x))
    shape = ([nb] if batched else []) + [2] * len(open_q)
    return entries, shape


def sv_amplitudes(circuit, spec, batch_bits=None) -> np.ndarray:
    """Requested amplitudes from the full state vector (shape as the TN result)."""
    state = sv_state(circuit)
    entries, shape = _output_index_list(circuit.n_qubits, spec, batch_bits)
    vals = np.array([state[x] for x in entries], dtype=np.complex128)
    return vals.reshape(shape) if shape else vals.reshape(())


def sv_gate_gradients(circuit, spec, weights: np.ndarray, batch_bits=None) -> Dict[int, np.ndarray]:
    """Holomorphic VJP sum_o w_o d a_o / d G_l for every single-qubit gate l.

    Returns {circuit gate index: 2x2 complex array J[i, j]}.
    """
    n = circuit.n_qubits
    entries, _ = _output_index_list(n, spec, batch_bits)
    w = np.asarray(weights, dtype=np.complex128).reshape(-1)
    c = np.zeros((2,) * n, dtype=np.complex128)
    for x, wo in zip(entries, w):
        c[x] += wo
    # forward states before each gate
    psi = []
    state = np.zeros((2,) * n, dtype=np.complex128)
    state[(0,) * n] = 1.0
    for g in circuit.gates:
        psi.append(state)
        state = _apply(state, g.matrix, g.qubits)
    grads: Dict[int, np.ndarray] = {}
    phi = c
    for l in range(len(circuit.gates) - 1, -1, -1):
        g = circuit.gates[l]
        # phi currently = U_{>l}^T c
        if g.arity == 1:
            (q,) = g.qubits
            a = np.moveaxis(phi, q, 0).reshape(2, -1)
            b = np.moveaxis(psi[l], q, 0).reshape(2, -1)
            grads[l] = a @ b.T
        phi = _apply_transpose(phi, g.matrix, g.qubits)
    return grads
