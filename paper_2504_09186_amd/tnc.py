"""Python front end of libmitnc: networks, plans and amplitude evaluation.

Argument marshalling only: every contraction runs in the library's HIP
kernels; torch provides device memory and the stream.
"""
from __future__ import annotations

import ctypes as C
from typing import List, Optional, Sequence, Tuple

import numpy as np

from . import _lib
from ._lib import call, mitnc_gate, mitnc_plan_opts, mitnc_plan_stats, mitnc_search_opts


def _stream_handle(stream=None) -> C.c_void_p:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Network:
    """Tensor network of <x|U|0...0> for a gate list (objects with ``qubits``
    and ``matrix`` attributes, matrix U[out, in])."""

    def __init__(self, circuit, spec: Sequence[int], batch_bits: Optional[np.ndarray] = None):
        lib = _lib.load()
        n = int(circuit.n_qubits)
        gates = list(circuit.gates)
        self._mats = []
        arr = (mitnc_gate * max(1, len(gates)))()
        for i, g in enumerate(gates):
            m = np.ascontiguousarray(np.asarray(g.matrix, dtype=np.complex128)).view(np.float64)
            self._mats.append(m)
            q = tuple(g.qubits)
            arr[i].arity = len(q)
            arr[i].q0 = q[0]
            arr[i].q1 = q[1] if len(q) > 1 else -1
            arr[i].mat = m.ctypes.data_as(C.POINTER(C.c_double))
        h = C.c_void_p()
        call("mitnc_network_from_circuit", n, len(gates), arr, C.byref(h))
        self.h = h
        self._lib = lib
        spec = np.ascontiguousarray(np.asarray(spec, dtype=np.int8))
        if batch_bits is not None:
            bb = np.ascontiguousarray(np.asarray(batch_bits, dtype=np.uint8))
            nb = bb.shape[0]
            bptr = bb.ctypes.data_as(C.POINTER(C.c_uint8))
        else:
            nb, bptr = 0, None
        call("mitnc_network_set_output", h, spec.ctypes.data_as(C.POINTER(C.c_int8)), nb, bptr)
        nl = C.c_int32()
        call("mitnc_network_info", h, C.byref(nl), None)
        self.n_leaves = nl.value
        self.n_qubits = n

    def __del__(self):
        if getattr(self, "h", None):
            self._lib.mitnc_network_destroy(self.h)
            self.h = None

    def path_search(self, seed: int = 0, trials: int = 32, max_log2: int = 30, min_sliced: int = 0,
                    max_sliced: int = 40) -> None:
        o = mitnc_search_opts(seed, trials, max_log2, min_sliced, max_sliced)
        call("mitnc_path_search", self.h, C.byref(o))

    def path(self) -> List[Tuple[int, int]]:
        buf = (C.c_int32 * (2 * (self.n_leaves - 1)))()
        call("mitnc_get_path", self.h, buf)
        return [(buf[2 * i], buf[2 * i + 1]) for i in range(self.n_leaves - 1)]

    def set_path(self, path: Sequence[Tuple[int, int]]) -> None:
        flat = (C.c_int32 * (2 * len(path)))(*[x for p in path for x in p])
        call("mitnc_set_path", self.h, len(path), flat)

    def slicing(self) -> List[int]:
        n = C.c_int32()
        buf = (C.c_int64 * 64)()
        call("mitnc_get_slicing", self.h, C.byref(n), buf)
        return [int(buf[i]) for i in range(n.value)]

    def set_slicing(self, labels: Sequence[int]) -> None:
        buf = (C.c_int64 * max(1, len(labels)))(*[int(x) for x in labels])
        call("mitnc_set_slicing", self.h, len(labels), buf)

    def slice_greedy(self, max_log2: int, min_sliced: int = 0, max_sliced: int = 40) -> None:
        call("mitnc_slice_greedy", self.h, max_log2, min_sliced, max_sliced)

    def index_overhead(self, label: int) -> float:
        v = C.c_double()
        call("mitnc_index_overhead", self.h, int(label), C.byref(v))
        return v.value


class Plan:
    """Execution plan; owns nothing on the device."""

    def __init__(self, net: Network, precision: int = _lib.MITNC_C64, reuse: bool = True,
                 cache_budget_bytes: int = 0, force_kernel: int = -1):
        o = mitnc_plan_opts(precision, 1 if reuse else 0, cache_budget_bytes, force_kernel)
        h = C.c_void_p()
        call("mitnc_plan_create", net.h, C.byref(o), C.byref(h))
        self.h = h
        self._lib = net._lib
        st = mitnc_plan_stats()
        call("mitnc_plan_query", h, C.byref(st))
        self.stats = st
        self.n_slices = 1 << st.n_sliced
        self.workspace = None

    def __del__(self):
        if getattr(self, "h", None):
            self._lib.mitnc_plan_destroy(self.h)
            self.h = None

    def steps(self) -> np.ndarray:
        info = np.zeros((self.stats.n_steps, 12), dtype=np.float64)
        call("mitnc_plan_steps", self.h, info.ctypes.data_as(C.POINTER(C.c_double)))
        return info

    def upload(self, device="cuda", stream=None):
        import torch
        ws = torch.empty(max(256, int(self.stats.workspace_bytes)), dtype=torch.uint8, device=device)
        call("mitnc_plan_upload", self.h, C.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(stream))
        self.workspace = ws
        return ws

    def new_result(self, device="cuda"):
        import torch
        return torch.zeros(int(self.stats.result_elems), dtype=torch.complex128, device=device)

    def timing(self, enable: bool = True) -> None:
        """Start (or stop) per-launch event timing; discards recorded launches."""
        call("mitnc_plan_timing", self.h, 1 if enable else 0)

    def timing_read(self):
        """Per kernel class: (milliseconds, launches, flops, bytes) summed over
        the launches recorded since timing() was called."""
        arrs = [np.zeros(8) for _ in range(4)]
        ptrs = [a.ctypes.data_as(C.POINTER(C.c_double)) for a in arrs]
        call("mitnc_plan_timing_read", self.h, *ptrs)
        return tuple(arrs)

    def execute(self, acc, slice_begin: int = 0, slice_end: Optional[int] = None, stream=None):
        """acc += sum of slices [slice_begin, slice_end) (complex128 device tensor)."""
        import torch
        if self.workspace is None:
            raise RuntimeError("upload() the plan first")
        if acc.dtype != torch.complex128 or not acc.is_contiguous() or acc.numel() != self.stats.result_elems:
            raise ValueError("acc must be a contiguous complex128 tensor of result_elems entries")
        if slice_end is None:
            slice_end = self.n_slices
        call("mitnc_execute", self.h, C.c_void_p(self.workspace.data_ptr()), self.workspace.numel(),
             int(slice_begin), int(slice_end), C.c_void_p(acc.data_ptr()), _stream_handle(stream))
        return acc


def contract(a, la: Sequence[int], b, lb: Sequence[int], lc: Sequence[int], kernel: int = -1,
             stream=None):
    """One pairwise contraction on the GPU.  a, b: contiguous complex64 device
    tensors with 2^len(la) / 2^len(lb) entries; address bit i carries label
    la[i] (LSB first).  Returns C (complex64) with address bits lc."""
    import torch
    lib = _lib.load()
    la = (C.c_int64 * max(1, len(la)))(*la), len(la)
    lb = (C.c_int64 * max(1, len(lb)))(*lb), len(lb)
    lcv = (C.c_int64 * max(1, len(lc)))(*lc), len(lc)
    need = C.c_size_t()
    call("mitnc_contract", None, la[1], la[0], None, lb[1], lb[0], None, lcv[1], lcv[0], kernel, None, 0,
         C.byref(need), None)
    out = torch.empty(1 << lcv[1], dtype=torch.complex64, device=a.device)
    work = torch.empty(max(256, need.value), dtype=torch.uint8, device=a.device) if need.value else None
    if a.dtype != torch.complex64 or b.dtype != torch.complex64:
        raise ValueError("operands must be complex64")
    if a.numel() != (1 << la[1]) or b.numel() != (1 << lb[1]):
        raise ValueError("operand sizes do not match their labels")
    call("mitnc_contract", C.c_void_p(a.data_ptr()), la[1], la[0], C.c_void_p(b.data_ptr()), lb[1], lb[0],
         C.c_void_p(out.data_ptr()), lcv[1], lcv[0], kernel,
         C.c_void_p(work.data_ptr()) if work is not None else None, need.value, None,
         _stream_handle(stream))
    del lib
    return out


def amplitudes(circuit, spec, batch_bits=None, seed: int = 0, trials: int = 32, max_log2: int = 30,
               min_sliced: int = 0, slices: Optional[Tuple[int, int]] = None, reuse: bool = True,
               device="cuda"):
    """Requested amplitudes (complex128 device tensor in the canonical result
    order), or the partial sum over ``slices = (begin, end)``."""
    net = Network(circuit, spec, batch_bits)
    net.path_search(seed=seed, trials=trials, max_log2=max_log2, min_sliced=min_sliced)
    plan = Plan(net, reuse=reuse)
    plan.upload(device)
    acc = plan.new_result(device)
    s0, s1 = slices if slices is not None else (0, plan.n_slices)
    plan.execute(acc, s0, s1)
    return acc
