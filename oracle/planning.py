"""Contraction order and slicing choice used by the oracle for its own runs.

The paper obtains paths from an external hyper-optimised search (Evaluation
section) and chooses sliced indices with the index overhead of Eq. (1) as the
key indicator (Sec. III-A).  The result of a contraction does not depend on the
path or the sliced set (distributivity), so these helpers only need to yield
valid, affordable plans for the oracle; they are independent of the GPU
library's own planner.

  * ``greedy_path``: repeatedly contract the connected pair minimising
    size(out) - size(a) - size(b), ties broken by the lowest ids; optional
    Gaussian jitter of the log-sizes gives alternative valid paths.
  * ``path_stats``: per-step output log2 size and real flops (8 M K N batch).
  * ``choose_slices``: greedily slice the index that minimises the largest
    intermediate, then the per-subtask flops.
  * ``index_overhead``: Eq. (1), O(a) = 2 C_a / C_ori.
"""
from __future__ import annotations

import heapq
import math
from typing import Dict, FrozenSet, List, Optional, Sequence, Set, Tuple

import numpy as np

from .network import Network


def _logdims(net: Network) -> Dict[int, float]:
    return {x: math.log2(d) for x, d in net.dims.items()}


def _out_labels(la: FrozenSet[int], lb: FrozenSet[int], count: Dict[int, int],
                out: Set[int]) -> FrozenSet[int]:
    res = set()
    for x in la | lb:
        held = (x in la) + (x in lb)
        if count[x] - held > 0 or x in out:
            res.add(x)
    return frozenset(res)


def _size(ls, ld) -> float:
    return sum(ld[x] for x in ls)


def greedy_path(net: Network, sliced: Sequence[int] = (), jitter: float = 0.0,
                seed: Optional[int] = None) -> List[Tuple[int, int]]:
    """Greedy SSA path (see module docstring)."""
    rng = np.random.default_rng(seed)
    ld = _logdims(net)
    sl = set(sliced)
    out = set(net.output)
    n = net.n_leaves
    tens: Dict[int, FrozenSet[int]] = {i: frozenset(x for x in lab if x not in sl)
                                       for i, lab in enumerate(net.labels)}
    holders: Dict[int, Set[int]] = {}
    count: Dict[int, int] = {}
    for i, lab in tens.items():
        for x in lab:
            holders.setdefault(x, set()).add(i)
            count[x] = count.get(x, 0) + 1
    heap: List[Tuple[float, int, int]] = []

    def jit(v):
        return v + (rng.normal(0.0, jitter) if jitter > 0 else 0.0)

    def push(i, j):
        if i > j:
            i, j = j, i
        lc = _out_labels(tens[i], tens[j], count, out)
        cost = 2.0 ** jit(_size(lc, ld)) - 2.0 ** jit(_size(tens[i], ld)) - 2.0 ** jit(_size(tens[j], ld))
        heapq.heappush(heap, (cost, i, j))

    for x, hs in holders.items():
        hs = sorted(hs)
        for a in range(len(hs)):
            for b in range(a + 1, len(hs)):
                push(hs[a], hs[b])
    path: List[Tuple[int, int]] = []
    nxt = n
    while len(tens) > 1:
        pair = None
        while heap:
            _, i, j = heapq.heappop(heap)
            if i in tens and j in tens:
                pair = (i, j)
                break
        if pair is None:  # disconnected: join the two smallest tensors
            ids = sorted(tens, key=lambda t: (_size(tens[t], ld), t))
            pair = (min(ids[0], ids[1]), max(ids[0], ids[1]))
        i, j = pair
        lc = _out_labels(tens[i], tens[j], count, out)
        for x in tens[i] | tens[j]:
            held = (x in tens[i]) + (x in tens[j])
            count[x] -= held
            holders[x].discard(i)
            holders[x].discard(j)
        del tens[i]
        del tens[j]
        tens[nxt] = lc
        nb = set()
        for x in lc:
            count[x] = count.get(x, 0) + 1
            holders.setdefault(x, set()).add(nxt)
            nb |= holders[x]
        nb.discard(nxt)
        for m in sorted(nb):
            push(m, nxt)
        path.append((i, j))
        nxt += 1
    return path


def random_greedy_path(net: Network, seed: int, jitter: float = 1.0) -> List[Tuple[int, int]]:
    return greedy_path(net, jitter=jitter, seed=seed)


def path_stats(net: Network, path: Sequence[Tuple[int, int]], sliced: Sequence[int] = ()):
    """Per-step (log2 |C|, real flops) for one subtask of the sliced network."""
    ld = _logdims(net)
    sl = set(sliced)
    out = set(net.output)
    n = net.n_leaves
    tens: Dict[int, FrozenSet[int]] = {i: frozenset(x for x in lab if x not in sl)
                                       for i, lab in enumerate(net.labels)}
    count: Dict[int, int] = {}
    for lab in tens.values():
        for x in lab:
            count[x] = count.get(x, 0) + 1
    steps = []
    for t, (i, j) in enumerate(path):
        la, lb = tens.pop(i), tens.pop(j)
        lc = _out_labels(la, lb, count, out)
        contracted = (la & lb) - lc
        for x in la:
            count[x] -= 1
        for x in lb:
            count[x] -= 1
        for x in lc:
            count[x] += 1
        tens[n + t] = lc
        logc = _size(lc, ld)
        flops = 8.0 * 2.0 ** (logc + _size(contracted, ld))
        steps.append((logc, flops))
    return steps


def max_log_size(net, path, sliced=()) -> float:
    return max(s[0] for s in path_stats(net, path, sliced))


def total_flops(net, path, sliced=()) -> float:
    return sum(s[1] for s in path_stats(net, path, sliced))


def choose_slices(net: Network, path: Sequence[Tuple[int, int]], cap_log2: float,
                  min_sliced: int = 0, max_sliced: int = 64) -> List[int]:
    """Greedy slicing until the largest intermediate is <= 2^cap_log2 and at
    least ``min_sliced`` indices are sliced.  Returned outer -> inner in the
    order chosen (first chosen = outermost)."""
    closed = set(net.closed_labels())
    sliced: List[int] = []
    while len(sliced) < max_sliced:
        stats = path_stats(net, path, sliced)
        big = max(s[0] for s in stats)
        if big <= cap_log2 and len(sliced) >= min_sliced:
            break
        # candidates: closed labels present in some intermediate of maximal size
        ld = _logdims(net)
        cand = set()
        sl = set(sliced)
        out = set(net.output)
        tens = {i: frozenset(x for x in lab if x not in sl) for i, lab in enumerate(net.labels)}
        count: Dict[int, int] = {}
        for lab in tens.values():
            for x in lab:
                count[x] = count.get(x, 0) + 1
        for t, (i, j) in enumerate(path):
            la, lb = tens.pop(i), tens.pop(j)
            lc = _out_labels(la, lb, count, out)
            for x in la:
                count[x] -= 1
            for x in lb:
                count[x] -= 1
            for x in lc:
                count[x] += 1
            tens[net.n_leaves + t] = lc
            if _size(lc, ld) >= big - 1e-9:
                cand |= (lc & closed)
        if not cand:
            cand = closed - sl
        best = None
        for x in sorted(cand - sl):
            st = path_stats(net, path, sliced + [x])
            key = (max(s[0] for s in st), sum(s[1] for s in st), x)
            if best is None or key < best:
                best = key
        if best is None:
            break
        sliced.append(best[2])
    return sliced


def index_overhead(net: Network, path: Sequence[Tuple[int, int]], a: int,
                   sliced: Sequence[int] = ()) -> float:
    """Eq. (1): O(a) = 2 C_a / C_ori, with C_ori the per-subtask complexity
    before slicing ``a`` and C_a the complexity of one of the two subtasks
    after slicing it (flop counts of the given path)."""
    c_ori = total_flops(net, path, sliced)
    c_a = total_flops(net, path, list(sliced) + [a])
    return 2.0 * c_a / c_ori
