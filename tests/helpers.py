"""Shared test helpers: LSB-first label layouts <-> numpy axes, GPU gating."""
import os

import numpy as np
import pytest

import oracle


def lib_built() -> bool:
    from paper_2504_09186_amd import _lib
    return os.path.exists(_lib.LIB_PATH)


def have_gpu() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def require_gpu():
    if not have_gpu():
        pytest.skip("no GPU")
    if not lib_built():
        raise RuntimeError("libmitnc.so not built: the GPU path has no fallback")


def np_from_flat(flat: np.ndarray, labels_lsb):
    """Flat array whose address bit i carries labels_lsb[i] -> (array, numpy labels)."""
    r = len(labels_lsb)
    return np.asarray(flat).reshape((2,) * r) if r else np.asarray(flat).reshape(()), list(reversed(labels_lsb))


def flat_from_np(arr: np.ndarray, np_labels, labels_lsb):
    """numpy array with axis labels np_labels -> flat array in LSB-first layout labels_lsb."""
    want = list(reversed(labels_lsb))
    return np.transpose(arr, [list(np_labels).index(x) for x in want]).reshape(-1)


def ref_contract(a_flat, la, b_flat, lb, lc, absval=False):
    """FP64 oracle contraction of flat LSB-first tensors to layout lc."""
    a, nla = np_from_flat(np.asarray(a_flat, dtype=np.complex128), la)
    b, nlb = np_from_flat(np.asarray(b_flat, dtype=np.complex128), lb)
    if absval:
        a, b = np.abs(a).astype(np.complex128), np.abs(b).astype(np.complex128)
    c, lab = oracle.contract_pair(a, nla, b, nlb, keep=set(lc))
    return flat_from_np(c, lab, lc)


def gamma(n: int, u: float = 2.0 ** -24) -> float:
    return n * u / (1 - n * u)


def nested_chain(onet, path, k):
    """k closed labels whose lifetimes (oracle.sliced_lifetimes) are strictly
    nested, the innermost ending before the root; innermost first (None if
    the path has no such family)."""
    closed = onet.closed_labels()
    below, alive = oracle.sliced_lifetimes(onet, path, closed)
    life = {x: frozenset(t for t in range(len(path)) if x in alive[t]) for x in closed}
    labs = sorted(closed, key=lambda x: (len(life[x]), x))
    for x in labs:
        if len(path) - 1 in life[x]:
            continue
        ch = [x]
        for y in labs:
            if len(ch) < k and life[ch[-1]] < life[y]:
                ch.append(y)
        if len(ch) == k:
            return ch
    return None
