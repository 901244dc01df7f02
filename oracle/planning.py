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
  * ``sliced_lifetimes``: per step, the sliced indices its subtree carries and
    those alive at it (Sec. III-B: an index's lifetime runs from the first
    step that holds one of its tensors to the step that joins both).
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


def _fm_improve(side: np.ndarray, nets: List[List[int]], lo: int, hi: int, passes: int = 6,
                vw: Optional[np.ndarray] = None) -> None:
    """Fiduccia-Mattheyses refinement of a bisection in place: nets are lists
    of vertices (a net is cut when it has vertices on both sides); each pass
    moves every vertex once, largest gain first within the bounds on the
    weight of side 1 (vertex weights ``vw``, default 1), and keeps the best
    prefix of the moves."""
    m = len(side)
    if vw is None:
        vw = np.ones(m, dtype=np.int64)
    vnets: List[List[int]] = [[] for _ in range(m)]
    nets = [n for n in nets if len(n) > 1]
    for e, pins in enumerate(nets):
        for v in pins:
            vnets[v].append(e)
    for _ in range(passes):
        cnt = np.zeros((len(nets), 2), dtype=np.int64)
        for e, pins in enumerate(nets):
            for v in pins:
                cnt[e, side[v]] += 1

        def gain(v):
            s0 = side[v]
            g = 0
            for e in vnets[v]:
                if cnt[e, s0] == 1 and cnt[e, 1 - s0] > 0:
                    g += 1
                elif cnt[e, 1 - s0] == 0 and cnt[e, s0] > 1:
                    g -= 1
            return g

        gains = np.array([gain(v) for v in range(m)], dtype=np.float64)
        locked = np.zeros(m, dtype=bool)
        w1 = int(vw[side == 1].sum())
        moves, cum, best, best_len = [], 0, 0, 0
        for _step in range(m):
            cand = np.where(~locked)[0]
            after = w1 + np.where(side[cand] == 0, vw[cand], -vw[cand])
            cand = cand[(after >= lo) & (after <= hi)]
            if cand.size == 0:
                break
            v = int(cand[np.argmax(gains[cand])])
            s0 = side[v]
            for e in vnets[v]:
                cnt[e, s0] -= 1
                cnt[e, 1 - s0] += 1
            side[v] = 1 - s0
            w1 += int(vw[v]) if s0 == 0 else -int(vw[v])
            locked[v] = True
            cum += gains[v]
            moves.append(v)
            for e in vnets[v]:
                for u in nets[e]:
                    if not locked[u]:
                        gains[u] = gain(u)
            if cum > best:
                best, best_len = cum, len(moves)
        for v in moves[best_len:][::-1]:
            side[v] = 1 - side[v]
        if best_len == 0:
            break


def _coarsen(m: int, nets: List[List[int]], vw: np.ndarray, rng, max_vw: int):
    """Heavy-net matching: in random order each unmatched vertex pairs with
    the unmatched neighbour it shares the most net weight with (a net of p
    vertices gives 1 / (p - 1) to each pair), per unit of combined vertex
    weight.  Returns (coarse vertex count, coarse nets, coarse weights,
    fine -> coarse map)."""
    nbr: List[Dict[int, float]] = [dict() for _ in range(m)]
    for pins in nets:
        w = 1.0 / (len(pins) - 1)
        for a in pins:
            for b in pins:
                if a != b:
                    nbr[a][b] = nbr[a].get(b, 0.0) + w
    match = np.full(m, -1, dtype=np.int64)
    for v in rng.permutation(m):
        if match[v] >= 0:
            continue
        best, bv = -1, 0.0
        for u, w in nbr[v].items():
            if match[u] < 0 and vw[u] + vw[v] <= max_vw:
                sc = w / float(vw[u] + vw[v])
                if sc > bv or (sc == bv and u < best):
                    best, bv = u, sc
        match[v] = best if best >= 0 else v
        if best >= 0:
            match[best] = v
    cmap = np.full(m, -1, dtype=np.int64)
    cvw = []
    for v in range(m):
        if cmap[v] >= 0:
            continue
        cmap[v] = len(cvw)
        if match[v] != v:
            cmap[match[v]] = len(cvw)
        cvw.append(int(vw[v]) + (int(vw[match[v]]) if match[v] != v else 0))
    cnets = []
    for pins in nets:
        cp = sorted({int(cmap[v]) for v in pins})
        if len(cp) > 1:
            cnets.append(cp)
    return len(cvw), cnets, np.array(cvw, dtype=np.int64), cmap


def _grow(m: int, nets: List[List[int]], vw: np.ndarray, target: int, rng) -> np.ndarray:
    """Side 1 grown breadth-first from a random vertex to weight >= target."""
    adj: List[List[int]] = [[] for _ in range(m)]
    for pins in nets:
        for a in pins:
            adj[a].extend(b for b in pins if b != a)
    side = np.zeros(m, dtype=np.int64)
    queue = [int(rng.integers(m))]
    w = 0
    while w < target:
        if not queue:
            rest = np.where(side == 0)[0]
            if rest.size == 0:
                break
            queue = [int(rest[0])]
        v = queue.pop(0)
        if side[v]:
            continue
        side[v] = 1
        w += int(vw[v])
        queue.extend(u for u in adj[v] if not side[u])
    return side


def _multilevel_bisect(m: int, nets: List[List[int]], imbalance: float, starts: int, rng) -> np.ndarray:
    """Bisection of m unit-weight vertices: coarsen by heavy-net matching to
    at most 40 vertices, keep the best of ``starts`` grown and refined parts
    there, then project back, refining at every level."""
    W = m
    lo = max(1, int(np.floor(W / 2 * (1 - imbalance))))
    hi = min(W - 1, int(np.ceil(W / 2 * (1 + imbalance))))
    levels = [(m, nets, np.ones(m, dtype=np.int64))]
    maps = []
    while levels[-1][0] > 40:
        cm, cnets, cvw, cmap = _coarsen(*levels[-1], rng, max(2, W // 8))
        if cm > 0.9 * levels[-1][0]:
            break
        levels.append((cm, cnets, cvw))
        maps.append(cmap)
    cm, cnets, cvw = levels[-1]
    best, best_cut = None, None
    for _ in range(starts):
        side = _grow(cm, cnets, cvw, int(rng.integers(lo, hi + 1)), rng)
        _fm_improve(side, cnets, lo, hi, vw=cvw)
        w1 = int(cvw[side == 1].sum())
        if not lo <= w1 <= hi:
            continue
        cut = sum(1 for ks in cnets if 0 < side[ks].sum() < len(ks))
        if best_cut is None or cut < best_cut:
            best, best_cut = side.copy(), cut
    if best is None:
        best = _grow(m, nets, np.ones(m, dtype=np.int64), (lo + hi) // 2, rng)
        _fm_improve(best, nets, lo, hi)
        return best
    for L in range(len(levels) - 2, -1, -1):
        best = best[maps[L]]
        _fm_improve(best, levels[L][1], lo, hi, vw=levels[L][2])
    return best


def bisection_path(net: Network, sliced: Sequence[int] = (), cutoff: int = 8, imbalance: float = 0.1,
                   starts: int = 4, seed: int = 0) -> List[Tuple[int, int]]:
    """SSA path by recursive bisection (sliced labels removed).

    First every tensor with at most two labels (single-qubit gates, initial
    and projector vectors) is contracted into the lowest-id neighbour it
    shares a label with, repeatedly.  Then a set of tensors is split in two
    (``_multilevel_bisect``: coarsening by heavy-net matching; at the
    coarsest level ``starts`` parts grown breadth-first from random tensors
    to random sizes within (1 +- imbalance) / 2, each improved by
    Fiduccia-Mattheyses passes on the number of cut labels, the best kept;
    refinement at every level back up); the parts are split recursively and
    joined last.  Sets of at most
    ``cutoff`` tensors are contracted with the greedy rule of
    ``greedy_path`` restricted to them.  Only the cost of the path depends on
    these choices; any valid path gives the same contraction value.  The
    index set of a subtree follows from its leaves: a label stays while a
    leaf outside holds it or it is an output."""
    rng = np.random.default_rng(seed)
    sl = set(sliced)
    out = set(net.output)
    ld = _logdims(net)
    n = net.n_leaves
    labs = [frozenset(x for x in lab if x not in sl) for lab in net.labels]
    count: Dict[int, int] = {}
    for lab in labs:
        for x in lab:
            count[x] = count.get(x, 0) + 1
    tens: Dict[int, FrozenSet[int]] = dict(enumerate(labs))
    path: List[Tuple[int, int]] = []

    def join(i, j):
        lc = _out_labels(tens[i], tens[j], count, out)
        for x in tens[i]:
            count[x] -= 1
        for x in tens[j]:
            count[x] -= 1
        for x in lc:
            count[x] += 1
        del tens[i], tens[j]
        k = n + len(path)
        tens[k] = lc
        path.append((min(i, j), max(i, j)))
        return k

    def greedy(ids: List[int]) -> int:
        ids = list(ids)
        while len(ids) > 1:
            best = None
            for a in range(len(ids)):
                for b in range(a + 1, len(ids)):
                    i, j = ids[a], ids[b]
                    shared = bool(tens[i] & tens[j])
                    lc = _out_labels(tens[i], tens[j], count, out)
                    cost = (0 if shared else 1,
                            2.0 ** _size(lc, ld) - 2.0 ** _size(tens[i], ld) - 2.0 ** _size(tens[j], ld), i, j)
                    if best is None or cost < best:
                        best = cost
            _, _, i, j = best
            ids.remove(i)
            ids.remove(j)
            ids.append(join(i, j))
        return ids[0]

    def split(ids: List[int]) -> int:
        m = len(ids)
        if m <= cutoff:
            return greedy(ids)
        pos = {v: k for k, v in enumerate(ids)}
        by_label: Dict[int, List[int]] = {}
        for v in ids:
            for x in tens[v]:
                by_label.setdefault(x, []).append(pos[v])
        nets = [ks for ks in by_label.values() if len(ks) > 1]
        best_side = _multilevel_bisect(m, nets, imbalance, starts, rng)
        left = sorted(ids[k] for k in range(m) if best_side[k] == 0)
        right = sorted(ids[k] for k in range(m) if best_side[k] == 1)
        if not left or not right:
            return greedy(ids)
        a = split(left)
        b = split(right)
        return join(a, b)

    changed = True
    while changed:
        changed = False
        for i in sorted(tens):
            if i not in tens or len(tens[i]) > 2:
                continue
            nbrs = sorted(j for j in tens if j != i and tens[j] & tens[i])
            if nbrs:
                join(i, nbrs[0])
                changed = True
    split(sorted(tens))
    return path


def _bitsets(net: Network):
    """Leaf label sets as Python-int bitsets (label -> bit) for networks whose
    labels each join at most two leaves; (leaf masks, output mask, label list)."""
    labels = sorted({x for lab in net.labels for x in lab})
    bit = {x: k for k, x in enumerate(labels)}
    masks = []
    holders: Dict[int, int] = {}
    for lab in net.labels:
        m = 0
        for x in lab:
            m |= 1 << bit[x]
            holders[x] = holders.get(x, 0) + 1
        masks.append(m)
    if any(h > 2 for h in holders.values()):
        raise ValueError("bitset statistics need labels shared by at most two leaves")
    out = 0
    for x in net.output:
        out |= 1 << bit[x]
    return masks, out, labels


def _bit_stats(masks, out, path, cut_mask):
    """(largest log2 size, total flops) of a path with the labels in cut_mask
    sliced; a label joining two tensors is summed when both are contracted
    together, so C = (A xor B) plus the shared output labels."""
    keep = ~cut_mask
    t = [m & keep for m in masks]
    big, flops = 0, 0.0
    for i, j in path:
        a, b = t[i], t[j]
        both = a & b
        c = (a ^ b) | (both & out)
        k = (both & ~out).bit_count()
        cb = c.bit_count()
        t.append(c)
        big = max(big, cb)
        flops += 8.0 * 2.0 ** (cb + k)
    return big, flops


def choose_slices_eval(net: Network, path: Sequence[Tuple[int, int]], cap_log2: int,
                       max_sliced: int = 64, min_sliced: int = 0, start: Sequence[int] = ()) -> List[int]:
    """Greedy slicing with trial evaluations (the rule of ``choose_slices``:
    the largest intermediate first, then the per-subtask flops, then the
    lowest label), for networks whose labels join at most two leaves, using
    bitset statistics; ``start`` labels are sliced first.  Returned in the
    order chosen (``start`` first)."""
    masks, out, labels = _bitsets(net)
    closed = set(net.closed_labels())
    bit = {x: k for k, x in enumerate(labels)}
    chosen: List[int] = list(start)
    cut = 0
    for x in chosen:
        cut |= 1 << bit[x]
    while len(chosen) < max_sliced:
        big, _ = _bit_stats(masks, out, path, cut)
        if big <= cap_log2 and len(chosen) >= min_sliced:
            break
        # candidates: closed labels of the intermediates of the largest size
        keep = ~cut
        t = [m & keep for m in masks]
        cand = 0
        for i, j in path:
            a, b = t[i], t[j]
            c = (a ^ b) | (a & b & out)
            t.append(c)
            if c.bit_count() == big:
                cand |= c
        best = None
        for x in sorted(closed):
            if x in chosen or not (cand >> bit[x]) & 1:
                continue
            key = _bit_stats(masks, out, path, cut | (1 << bit[x])) + (x,)
            if best is None or key < best:
                best = key
        if best is None:
            break
        chosen.append(best[2])
        cut |= 1 << bit[best[2]]
    return chosen


def sliced_lifetimes(net: Network, path: Sequence[Tuple[int, int]], sliced: Sequence[int]):
    """For every step t of an SSA path, two sets of sliced labels (Sec. III-B,
    lifetimes of sliced indices):

      * ``below[t]``: labels carried by some leaf of the step's subtree (its
        value depends on them);
      * ``alive[t]``: labels whose lifetime covers the step: carried by a leaf
        of its subtree and by a leaf outside it (started, not ended), or
        carried by a leaf under each of its two operands (ended here).

    A step whose alive set holds j of the sliced labels has 2^j distinct
    values over all slices; executing it exactly that often is the spindle's
    aim of removing every repeated calculation.  Plain definition: leaves
    below each node by explicit set union."""
    sl = set(sliced)
    n = net.n_leaves
    holders: Dict[int, Set[int]] = {x: set() for x in sl}
    for i, lab in enumerate(net.labels):
        for x in lab:
            if x in sl:
                holders[x].add(i)
    leaves_of: Dict[int, Set[int]] = {i: {i} for i in range(n)}
    below, alive = [], []
    for t, (i, j) in enumerate(path):
        li, lj = leaves_of[i], leaves_of[j]
        lv = li | lj
        leaves_of[n + t] = lv
        b, a = set(), set()
        for x, hs in holders.items():
            inside = hs & lv
            if not inside:
                continue
            b.add(x)
            if inside != hs or (hs & li and hs & lj):
                a.add(x)
        below.append(b)
        alive.append(a)
    return below, alive
