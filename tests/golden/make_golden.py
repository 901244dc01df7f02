"""Writes the stored expected values of the full-size parity tests.

Only the oracle (and the shared input generator) is called: the 64
amplitudes of the 5x6-qubit, 14-cycle circuit (qubits 24-29 open, the other
output bits random) by the oracle's own path and slicing, and the individual
results of slices 0..15 of an 8-index slicing chosen by the oracle.

Usage: python tests/golden/make_golden.py   (about 10 minutes on 8 cores)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402


def best_path(net, trials, seed):
    best = None
    for t in range(trials):
        p = oracle.greedy_path(net, jitter=0.25, seed=seed + t)
        f = oracle.planning.total_flops(net, p)
        if best is None or f < best[0]:
            best = (f, p)
    return best[1]


def cplx(a):
    a = np.asarray(a, dtype=np.complex128).reshape(-1)
    return [[float(x.real), float(x.imag)] for x in a]


def main():
    rows, cols, cycles = 5, 6, 14
    circ = synth.lattice_circuit(rows, cols, cycles, seed=1001)
    spec = synth.output_spec(30, list(range(24, 30)), seed=2001)
    net = oracle.build_network(circ, spec)
    path = best_path(net, 60, 3001)
    sliced = oracle.choose_slices(net, path, cap_log2=26, min_sliced=8)
    assert len(sliced) == 8
    t0 = time.time()
    total, parts = oracle.contract_sliced(net, path, sliced, per_slice=True)
    el = time.time() - t0
    out = {
        "what": "oracle results for the 5x6 lattice, 14 cycles, seed 1001, output spec seed 2001, "
                "qubits 24-29 open",
        "circuit": {"rows": rows, "cols": cols, "cycles": cycles, "seed": 1001},
        "spec_seed": 2001, "open_qubits": list(range(24, 30)),
        "oracle_sliced_labels": [int(x) for x in sliced],
        "amplitudes": cplx(total),
        "slice_results": {str(s): cplx(parts[s]) for s in range(16)},
        "oracle_seconds": el,
    }
    with open(os.path.join(HERE, "config2_amplitudes.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote config2_amplitudes.json ({el:.0f} s of contraction)")


if __name__ == "__main__":
    main()
