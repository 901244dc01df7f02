"""Writes the stored contraction paths of the benchmark workloads.

A path search is not part of the contraction itself (the paper takes its
path from a separate search); the benchmark loads the stored result so that
its run does not repeat a minutes-long search.  Each file holds the SSA path
pairs and the sliced labels (outer to inner) of one network, with the search
parameters and the resulting costs.

Usage: python -m paper_2504_09186_amd.paths.make_paths [--trials N] [--out FILE]

rqc_7x8_20.json: the defaults (1024 trials, exactly 48 sliced indices, launch
cost 5e8); rqc_7x8_20_s44.json: --trials 1024 --launch-cost 0 --min-sliced 8
--max-sliced 62 (the size cap decides the count: 44 sliced indices).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))

# 7x8 lattice, 20 cycles, last 12 qubits open: the headline workload.
RQC_7X8_20 = dict(rows=7, cols=8, cycles=20, circuit_seed=1004, open_qubits=list(range(44, 56)), spec_seed=2004,
                  max_log2=30, min_sliced=8, max_sliced=62, window_bits=8, merge_bits=8)
# flops charged per step launch in the ranking (about 5 us at 100 TFLOP/s)
LAUNCH_COST = 5e8


def share_flops(plan, window_bits):
    """Flops the plan's launch list executes for the first 2^window_bits
    slices (shared-prefix reuse, and the post-lifetime merge if the plan
    merges)."""
    import numpy as np
    sch = plan.schedule(0, 1 << window_bits)
    runs = np.bincount(sch[:, 1], minlength=plan.stats.n_steps)
    return float((plan.steps()[:, 6] * runs).sum())


def make_rqc_7x8_20(trials: int, seed: int, launch_cost: float = LAUNCH_COST, min_sliced: int = 48,
                    max_sliced: int = 48) -> dict:
    """Recursive-bisection search ranked by the flops of all slices dealt in
    256-slice shares with the merge of the 8 inner slice-id bits and
    launch_cost flops per step launch, then branch exchange ranked the same
    way.  With min_sliced = max_sliced the slicing goes on past the size cap
    to that many indices (smaller slices: each 256-slice share is a fixed
    2^-(S-8) of the job)."""
    sys.path.insert(0, ROOT)
    import synth
    from paper_2504_09186_amd import tnc
    w = dict(RQC_7X8_20, min_sliced=min_sliced, max_sliced=max_sliced)
    c = synth.lattice_circuit(w["rows"], w["cols"], w["cycles"], seed=w["circuit_seed"])
    spec = synth.output_spec(w["rows"] * w["cols"], w["open_qubits"], seed=w["spec_seed"])
    net = tnc.Network(c, spec)
    t0 = time.perf_counter()
    net.path_search(seed=seed, trials=trials, max_log2=w["max_log2"], min_sliced=w["min_sliced"],
                    max_sliced=w["max_sliced"], method=1, window_bits=w["window_bits"],
                    merge_bits=w["merge_bits"] if launch_cost else 0, launch_cost_flops=launch_cost)
    search_s = time.perf_counter() - t0
    sf_search = share_flops(tnc.Plan(net, precision=0), w["window_bits"])
    t0 = time.perf_counter()
    before, after = net.branch_exchange(window_bits=w["window_bits"], merge_bits=w["merge_bits"],
                                        max_log2=w["max_log2"], passes=8, launch_cost_flops=launch_cost)
    exchange_s = time.perf_counter() - t0
    plan = tnc.Plan(net, precision=0, merge_bits=w["merge_bits"])
    sl = [int(x) for x in net.slicing()]
    sf = share_flops(plan, w["window_bits"])
    return dict(workload=w, n_leaves=net.n_leaves,
                search=dict(method=1, trials=trials, seed=seed, seconds=round(search_s, 1),
                            share_flops=sf_search, launch_cost_flops=launch_cost),
                branch_exchange=dict(passes=8, seconds=round(exchange_s, 1), job_flops_before=before,
                                     job_flops_after=after),
                path=[[int(a), int(b)] for a, b in net.path()], slicing=sl, n_sliced=len(sl),
                max_log2_elems=int(plan.stats.max_log2_elems), merge_bits=w["merge_bits"],
                n_merged=int(plan.stats.n_merged), share_flops=sf,
                job_flops=sf * 2.0 ** (len(sl) - w["window_bits"]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trials", type=int, default=1024)
    ap.add_argument("--seed", type=int, default=3004)
    ap.add_argument("--out", default="rqc_7x8_20.json")
    ap.add_argument("--launch-cost", type=float, default=LAUNCH_COST)
    ap.add_argument("--min-sliced", type=int, default=48)
    ap.add_argument("--max-sliced", type=int, default=48)
    args = ap.parse_args()
    out = make_rqc_7x8_20(args.trials, args.seed, args.launch_cost, args.min_sliced, args.max_sliced)
    path = os.path.join(HERE, os.path.basename(args.out))
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print(f"wrote {path}: {out['n_sliced']} sliced, share flops {out['search']['share_flops']:.3e} after the "
          f"search, {out['share_flops']:.3e} after branch exchange and merge, job flops {out['job_flops']:.3e} "
          f"({out['search']['seconds']} s search, {out['branch_exchange']['seconds']} s exchange)")


if __name__ == "__main__":
    main()
