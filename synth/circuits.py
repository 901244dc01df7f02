"""Random lattice circuits: the synthetic stand-in for the paper's RQC workloads.

The paper evaluates on Zuchongzhi-56/60 circuits (Evaluation section); their gate
files are not available, so circuits of the same family are generated here:
an R x C qubit grid, and per cycle one layer of random single-qubit gates drawn
from {sqrt(X), sqrt(Y), sqrt(W)} (never the same gate twice in a row on a
qubit) followed by fSim(pi/2, pi/6) on one of four disjoint coupler patterns.

Conventions (the paper is silent on all of them):
  * qubit q = r * cols + c;
  * a gate matrix is U[out, in]; for a two-qubit gate on (q0, q1) the row and
    column index is (bit of q0) * 2 + (bit of q1);
  * coupler patterns: A = horizontal pairs starting at an even column,
    B = horizontal pairs starting at an odd column, C = vertical pairs starting
    at an even row, D = vertical pairs starting at an odd row; cycle k uses
    pattern ``pattern[k % len(pattern)]`` (default "ABCD");
  * the initial state is |0...0>; in an amplitude index qubit 0 is the most
    significant bit.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

_X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
_Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
_W = (_X + _Y) / np.sqrt(2.0)
_I2 = np.eye(2, dtype=np.complex128)


def _sqrt_involution(p: np.ndarray) -> np.ndarray:
    """Principal square root of an involution P (P @ P = I).

    ((1+i)/2) I + ((1-i)/2) P squares to I * ((1+i)^2 + (1-i)^2)/4 + P * 2(1+i)(1-i)/4
    = 0 * I + 1 * P.
    """
    return 0.5 * (1 + 1j) * _I2 + 0.5 * (1 - 1j) * p


def sqrt_x() -> np.ndarray:
    return _sqrt_involution(_X)


def sqrt_y() -> np.ndarray:
    return _sqrt_involution(_Y)


def sqrt_w() -> np.ndarray:
    return _sqrt_involution(_W)


def fsim(theta: float = np.pi / 2, phi: float = np.pi / 6) -> np.ndarray:
    """fSim(theta, phi) in the basis |00>, |01>, |10>, |11>."""
    c, s = np.cos(theta), np.sin(theta)
    return np.array(
        [[1, 0, 0, 0],
         [0, c, -1j * s, 0],
         [0, -1j * s, c, 0],
         [0, 0, 0, np.exp(-1j * phi)]], dtype=np.complex128)


_ONE_QUBIT = ("sqrt_x", "sqrt_y", "sqrt_w")


def gate_matrix(name: str) -> np.ndarray:
    if name == "sqrt_x":
        return sqrt_x()
    if name == "sqrt_y":
        return sqrt_y()
    if name == "sqrt_w":
        return sqrt_w()
    if name == "fsim":
        return fsim()
    raise ValueError(f"unknown gate {name!r}")


@dataclass(frozen=True)
class Gate:
    name: str
    qubits: Tuple[int, ...]
    matrix: np.ndarray = field(compare=False, repr=False)

    @property
    def arity(self) -> int:
        return len(self.qubits)


@dataclass
class Circuit:
    n_qubits: int
    gates: List[Gate]
    rows: int = 0
    cols: int = 0
    cycles: int = 0
    seed: int = 0

    def one_qubit_gate_ids(self) -> List[int]:
        return [i for i, g in enumerate(self.gates) if g.arity == 1]


def couplers(rows: int, cols: int, pattern: str) -> List[Tuple[int, int]]:
    out = []
    if pattern in "AB":
        start = 0 if pattern == "A" else 1
        for r in range(rows):
            for c in range(start, cols - 1, 2):
                out.append((r * cols + c, r * cols + c + 1))
    elif pattern in "CD":
        start = 0 if pattern == "C" else 1
        for r in range(start, rows - 1, 2):
            for c in range(cols):
                out.append((r * cols + c, (r + 1) * cols + c))
    else:
        raise ValueError(pattern)
    return out


def lattice_circuit(rows: int, cols: int, cycles: int, seed: int,
                    pattern: str = "ABCD", final_1q: bool = False) -> Circuit:
    """Seeded random lattice circuit (see module docstring for conventions).

    Single-qubit choice: cycle 0 draws uniformly from the three gates; later
    cycles draw uniformly from the two gates that differ from the previous
    single-qubit gate on the same qubit.  ``final_1q`` appends one more
    single-qubit layer after the last cycle.
    """
    rng = np.random.default_rng(seed)
    n = rows * cols
    prev = [-1] * n
    mats = {name: gate_matrix(name) for name in _ONE_QUBIT + ("fsim",)}
    gates: List[Gate] = []

    def one_qubit_layer():
        for q in range(n):
            if prev[q] < 0:
                k = int(rng.integers(0, 3))
            else:
                choices = [j for j in range(3) if j != prev[q]]
                k = choices[int(rng.integers(0, 2))]
            prev[q] = k
            name = _ONE_QUBIT[k]
            gates.append(Gate(name, (q,), mats[name]))

    for k in range(cycles):
        one_qubit_layer()
        for (a, b) in couplers(rows, cols, pattern[k % len(pattern)]):
            gates.append(Gate("fsim", (a, b), mats["fsim"]))
    if final_1q:
        one_qubit_layer()
    return Circuit(n_qubits=n, gates=gates, rows=rows, cols=cols, cycles=cycles, seed=seed)


def random_fixed_bits(n_qubits: int, seed: int) -> np.ndarray:
    """Uniform random bit per qubit (uint8), from ``default_rng(seed)``."""
    return np.random.default_rng(seed).integers(0, 2, size=n_qubits).astype(np.uint8)


def random_bitstrings(n_qubits: int, count: int, seed: int) -> np.ndarray:
    """``count`` uniform random bitstrings, shape (count, n_qubits), uint8.

    Duplicates are allowed.
    """
    return np.random.default_rng(seed).integers(0, 2, size=(count, n_qubits)).astype(np.uint8)


def output_spec(n_qubits: int, open_qubits: Sequence[int], seed: int,
                batched: Sequence[int] = ()) -> np.ndarray:
    """Per-qubit output request: 0/1 fixed bit, -1 open, -2 batched.

    Qubits not listed as open or batched get a fixed bit from
    ``random_fixed_bits(n_qubits, seed)``.
    """
    spec = random_fixed_bits(n_qubits, seed).astype(np.int8)
    for q in open_qubits:
        spec[q] = -1
    for q in batched:
        spec[q] = -2
    return spec
