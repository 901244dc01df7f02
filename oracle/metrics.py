"""Error metrics of an approximate result a~ against the FP64 reference a.

Not in the paper.  Readings used (result set B = all entries compared):
  rel-L2          = ||a~ - a||_2 / ||a||_2
  overlap         = |<a, a~>|^2 / (||a||^2 ||a~||^2)
  linear XEB ratio = (|B| sum p_x q_x - 1) / (|B| sum p_x^2 - 1),
                    p = |a|^2 / sum_B |a|^2, q = |a~|^2 / sum_B |a~|^2
The XEB fidelity loss is |1 - ratio|.
"""
from __future__ import annotations

import numpy as np


def rel_l2(approx, ref) -> float:
    a = np.asarray(ref, dtype=np.complex128).reshape(-1)
    b = np.asarray(approx, dtype=np.complex128).reshape(-1)
    return float(np.linalg.norm(b - a) / np.linalg.norm(a))


def overlap_fidelity(approx, ref) -> float:
    a = np.asarray(ref, dtype=np.complex128).reshape(-1)
    b = np.asarray(approx, dtype=np.complex128).reshape(-1)
    return float(abs(np.vdot(a, b)) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real))


def xeb_ratio(approx, ref) -> float:
    a = np.asarray(ref, dtype=np.complex128).reshape(-1)
    b = np.asarray(approx, dtype=np.complex128).reshape(-1)
    p = np.abs(a) ** 2
    p = p / p.sum()
    q = np.abs(b) ** 2
    q = q / q.sum()
    nb = a.size
    return float((nb * np.sum(p * q) - 1.0) / (nb * np.sum(p * p) - 1.0))
