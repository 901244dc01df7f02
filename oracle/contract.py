"""Pairwise contraction, contraction along a path, and slicing (oracle side).

Paper, Sec. II-A: a pairwise contraction is organised as an M x K x N matrix
product after the common indices are permuted into K (transpose, reshape,
GEMM).  Paper, Sec. II-A and III-A: slicing fixes chosen indices; each of the
2^s assignments is an independent subtask and the subtask results sum to the
unsliced contraction (distributivity).

Plain definitions only: no blocking, no fusion, no reuse across slices.
Parity: pinned in tests against brute-force state vectors, normalisation,
path/slicing invariance and closed-form special cases.
"""
from __future__ import annotations

from typing import Dict, Iterable, List, Optional, Sequence, Tuple

import numpy as np

from .network import Network


def contract_pair(a: np.ndarray, la: Sequence[int], b: np.ndarray, lb: Sequence[int],
                  keep: Iterable[int]) -> Tuple[np.ndarray, Tuple[int, ...]]:
    """Contract two tensors.

    Labels shared by both operands are summed unless they are in ``keep`` (then
    they are batch labels carried to the output, i.e. a hyperedge still in use).
    A label of only one operand that is not in ``keep`` is summed over that
    operand alone.  Output labels: batch labels, then A's free labels, then
    B's free labels, each in operand order.
    """
    keep = set(keep)
    la, lb = list(la), list(lb)
    # sum out dangling labels first
    for lab_list, arr_name in ((la, "a"), (lb, "b")):
        other = lb if arr_name == "a" else la
        drop = [i for i, x in enumerate(lab_list) if x not in other and x not in keep]
        if drop:
            if arr_name == "a":
                a = a.sum(axis=tuple(drop))
            else:
                b = b.sum(axis=tuple(drop))
            for i in reversed(drop):
                del lab_list[i]
    common = [x for x in la if x in lb]
    batch = [x for x in common if x in keep]
    contr = [x for x in common if x not in keep]
    fa = [x for x in la if x not in lb]
    fb = [x for x in lb if x not in la]
    dim = {}
    for x, d in zip(la, a.shape):
        dim[x] = d
    for x, d in zip(lb, b.shape):
        if x in dim and dim[x] != d:
            raise ValueError(f"dimension mismatch on label {x}")
        dim[x] = d

    def prod(ls):
        p = 1
        for x in ls:
            p *= dim[x]
        return p

    at = np.transpose(a, [la.index(x) for x in batch + fa + contr])
    bt = np.transpose(b, [lb.index(x) for x in batch + contr + fb])
    nb, m, k, n = prod(batch), prod(fa), prod(contr), prod(fb)
    c = np.matmul(at.reshape(nb, m, k), bt.reshape(nb, k, n))
    out_labels = tuple(batch + fa + fb)
    return c.reshape([dim[x] for x in out_labels]), out_labels


def slice_leaves(net: Network, sliced: Sequence[int], values: Sequence[int]):
    """Fix each sliced label to its value in every leaf holding it (np.take)."""
    val = dict(zip(sliced, values))
    arrays, labels = [], []
    for arr, lab in zip(net.arrays, net.labels):
        lab = list(lab)
        for x in list(lab):
            if x in val:
                ax = lab.index(x)
                arr = np.take(arr, val[x], axis=ax)
                lab.pop(ax)
        arrays.append(arr)
        labels.append(tuple(lab))
    return arrays, labels


def _run_path(arrays: List[np.ndarray], labels: List[Tuple[int, ...]], output: Tuple[int, ...],
              path: Sequence[Tuple[int, int]], flop_counter: Optional[List[int]] = None):
    n_leaves = len(arrays)
    if len(path) != n_leaves - 1:
        raise ValueError(f"path has {len(path)} steps, need {n_leaves - 1}")
    pool: Dict[int, Tuple[np.ndarray, Tuple[int, ...]]] = {
        i: (arrays[i], labels[i]) for i in range(n_leaves)}
    count: Dict[int, int] = {}
    for lab in labels:
        for x in lab:
            count[x] = count.get(x, 0) + 1
    out_set = set(output)
    for step, (i, j) in enumerate(path):
        if i not in pool or j not in pool or i == j:
            raise ValueError(f"invalid path step {step}: ({i}, {j})")
        a, la = pool.pop(i)
        b, lb = pool.pop(j)
        for x in la:
            count[x] -= 1
        for x in lb:
            count[x] -= 1
        keep = {x for x in set(la) | set(lb) if count.get(x, 0) > 0 or x in out_set}
        c, lc = contract_pair(a, la, b, lb, keep)
        if flop_counter is not None:
            contracted = [x for x in la if x in lb and x not in keep]
            k = 1
            for x in contracted:
                k *= a.shape[la.index(x)]
            flop_counter.append(8 * c.size * k)
        for x in lc:
            count[x] = count.get(x, 0) + 1
        pool[n_leaves + step] = (c, lc)
    (c, lc), = pool.values()
    if set(lc) != out_set:
        raise ValueError(f"final labels {lc} != output {output}")
    return np.transpose(c, [lc.index(x) for x in output])


def contract_network(net: Network, path: Sequence[Tuple[int, int]]) -> np.ndarray:
    """Contract the whole (unsliced) network along an SSA path.

    Path step t contracts tensors i and j (leaf ids, or n_leaves + t' for the
    result of step t') into tensor n_leaves + t.  Result axes follow
    ``net.output``.
    """
    return _run_path(net.arrays, net.labels, net.output, path)


def slice_values(slice_id: int, n_sliced: int) -> List[int]:
    """Value of each sliced index for a slice id: the last listed index is the
    least significant bit of the slice id (outer -> inner order)."""
    return [(slice_id >> (n_sliced - 1 - j)) & 1 for j in range(n_sliced)]


def contract_sliced(net: Network, path: Sequence[Tuple[int, int]], sliced: Sequence[int],
                    slice_ids: Optional[Iterable[int]] = None, per_slice: bool = False):
    """Sum of the sliced sub-network contractions over ``slice_ids``
    (default: all 2^s slices), summed in complex128 in the given order.

    With ``per_slice`` the list of individual slice results is returned too.
    """
    s = len(sliced)
    if slice_ids is None:
        slice_ids = range(1 << s)
    total = None
    parts = []
    for sid in slice_ids:
        arrays, labels = slice_leaves(net, sliced, slice_values(sid, s))
        r = _run_path(arrays, labels, net.output, path)
        parts.append(r)
        total = r.copy() if total is None else total + r
    if per_slice:
        return total, parts
    return total


def count_contraction_flops(net: Network, path: Sequence[Tuple[int, int]],
                            sliced: Sequence[int] = (), slice_id: int = 0) -> int:
    """Real flops (8 per complex multiply-add) of one subtask, counted from the
    array shapes met while actually contracting it."""
    counter: List[int] = []
    arrays, labels = slice_leaves(net, sliced, slice_values(slice_id, len(sliced)))
    _run_path(arrays, labels, net.output, path, flop_counter=counter)
    return int(sum(counter))


def amplitudes(circuit, spec, batch_bits=None, path=None, sliced: Sequence[int] = (),
               slice_ids=None):
    """Requested amplitudes by tensor-network contraction (own greedy path if
    none is given)."""
    from .network import build_network
    from .planning import greedy_path
    net = build_network(circuit, spec, batch_bits)
    if path is None:
        path = greedy_path(net)
    if sliced:
        return contract_sliced(net, path, sliced, slice_ids)
    return contract_network(net, path)
