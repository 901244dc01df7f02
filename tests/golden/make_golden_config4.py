"""Writes the stored expected values of the 7x8-qubit, 20-cycle sub-slice
parity checks.

Only the oracle (and the shared input generator) is called.  The full
network (56 qubits, qubits 44-55 open: 2^12 amplitudes, the other 44 output
bits random) is far beyond a brute-force or unsliced evaluation, so the
oracle takes its own recursive-bisection path, slices it with its own greedy
rule until every intermediate has at most 2^29 entries, and contracts a few
of those sub-slices one by one (each a partial sum of the amplitudes over the
sliced indices' other values).  A GPU run keeps the same sliced indices and
computes the same sub-slices with its own path.

Usage: python tests/golden/make_golden_config4.py   (a few minutes on 8 cores,
about 40 GiB of host memory)
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
from oracle import planning  # noqa: E402

ROWS, COLS, CYCLES, OPEN = 7, 8, 20, list(range(44, 56))
CAP, MAX_SLICED = 29, 60


def cplx(a):
    a = np.asarray(a, dtype=np.complex128).reshape(-1)
    return [[float(x.real), float(x.imag)] for x in a]


def main():
    circ = synth.lattice_circuit(ROWS, COLS, CYCLES, seed=1004)
    spec = synth.output_spec(ROWS * COLS, OPEN, seed=2004)
    net = oracle.build_network(circ, spec)
    masks, out, labels = planning._bitsets(net)
    best = None
    t0 = time.time()
    for seed in range(24):
        for imb in (0.5, 0.7):
            p = planning.bisection_path(net, imbalance=imb, seed=seed)
            f = planning._bit_stats(masks, out, p, 0)[1]
            if best is None or f < best[0]:
                best = (f, p)
    path = best[1]
    sliced = planning.choose_slices_eval(net, path, CAP, max_sliced=MAX_SLICED)
    st = planning.path_stats(net, path, sliced)
    width = max(s[0] for s in st)
    flops = sum(s[1] for s in st)
    print(f"path search {time.time() - t0:.0f} s: {len(sliced)} sliced, width {width}, "
          f"{flops:.3e} flops per sub-slice", flush=True)
    assert width <= CAP, width
    rng = np.random.default_rng(4004)
    ids = [0, int(rng.integers(1 << len(sliced)))]
    results = {}
    secs = []
    for sid in ids:
        t1 = time.time()
        r = oracle.contract_sliced(net, path, sliced, slice_ids=[sid])
        secs.append(time.time() - t1)
        results[str(sid)] = cplx(r)
        print(f"sub-slice {sid}: {secs[-1]:.0f} s, |r| = {np.linalg.norm(r):.3e}", flush=True)
    # a bounded sample for timing the oracle: the same slicing with two more
    # indices chosen by the same rule, one sub-slice of it
    sample = planning.choose_slices_eval(net, path, 0, max_sliced=MAX_SLICED + 2, start=sliced)
    sample_flops = sum(s[1] for s in planning.path_stats(net, path, sample))
    rec = {
        "what": "oracle sub-slice partial sums for the 7x8 lattice, 20 cycles, seed 1004, output spec "
                "seed 2004, qubits 44-55 open (result order: open qubits, lower qubit more significant)",
        "circuit": {"rows": ROWS, "cols": COLS, "cycles": CYCLES, "seed": 1004},
        "spec_seed": 2004, "open_qubits": OPEN,
        "oracle_sliced_labels": [int(x) for x in sliced],
        "oracle_path_flops_per_subslice": flops, "oracle_width": width,
        "sub_slice_ids": ids, "sub_slice_results": results, "oracle_seconds": secs,
        "oracle_path": [[int(a), int(b)] for a, b in path],
        "cpu_sample_sliced_labels": [int(x) for x in sample], "cpu_sample_flops": sample_flops,
    }
    with open(os.path.join(HERE, "config4_subslices.json"), "w") as f:
        json.dump(rec, f, indent=1)
    print("wrote config4_subslices.json")


if __name__ == "__main__":
    main()
