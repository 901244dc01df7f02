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
                    max_sliced: int = 40, keep_slicing: bool = False, method: int = 0,
                    window_bits: int = 0, merge_bits: int = 0, branch_exchange: bool = False,
                    launch_cost_flops: float = 0.0) -> None:
        """Path and slicing search (method 0 greedy, 1 recursive bisection, 2
        both).  Methods 1 and 2 rank trials by the reuse-aware flops of all
        slices, run in one sequence (window_bits 0) or dealt in aligned
        ranges of 2^window_bits slices that each start cold, counting the
        post-lifetime merge of the merge_bits innermost bits; branch_exchange
        then reorders absorptions with the same ranking; launch_cost_flops
        adds a per-launch cost to it."""
        o = mitnc_search_opts(seed, trials, max_log2, min_sliced, max_sliced, 1 if keep_slicing else 0, method,
                              window_bits, merge_bits, 1 if branch_exchange else 0, float(launch_cost_flops))
        call("mitnc_path_search", self.h, C.byref(o))

    def branch_exchange(self, window_bits: int = 0, merge_bits: int = 0, max_log2: int = 30,
                        passes: int = 8, launch_cost_flops: float = 0.0) -> Tuple[float, float]:
        """Swaps consecutive absorptions of the current path where that lowers
        the reuse- and merge-aware flops (mitnc_branch_exchange); returns the
        flops before and after."""
        b, a = C.c_double(), C.c_double()
        call("mitnc_branch_exchange", self.h, window_bits, merge_bits, max_log2, passes, C.c_double(launch_cost_flops),
             C.byref(b), C.byref(a))
        return b.value, a.value

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

    def slice_greedy(self, max_log2: int, min_sliced: int = 0, max_sliced: int = 40) -> List[int]:
        """Greedy slicing of the current path; returns the sliced labels, outer -> inner."""
        n = C.c_int32()
        buf = (C.c_int64 * 64)()
        call("mitnc_slice_greedy", self.h, max_log2, min_sliced, max_sliced, C.byref(n), buf)
        return [int(buf[i]) for i in range(n.value)]

    def index_overhead(self, label: int) -> float:
        v = C.c_double()
        call("mitnc_index_overhead", self.h, int(label), C.byref(v))
        return v.value


class Plan:
    """Execution plan; owns nothing on the device."""

    def __init__(self, net: Network, precision: int = _lib.MITNC_C64, reuse: bool = True,
                 cache_budget_bytes: int = 0, force_kernel: int = -1, differentiable: bool = False,
                 fuse_sections: bool = False, no_rerun: bool = False, splitk_max_mn_bits: int = 0,
                 splitk_target_bits: int = 0, merge_bits: int = 0, no_hoist: bool = False,
                 reverse_defer: int = 0, prologue_bits: int = 0):
        o = mitnc_plan_opts(precision, 1 if reuse else 0, cache_budget_bytes, force_kernel,
                            1 if differentiable else 0, 1 if fuse_sections else 0, 1 if no_rerun else 0,
                            splitk_max_mn_bits, splitk_target_bits, merge_bits, 1 if no_hoist else 0,
                            prologue_bits, reverse_defer)
        h = C.c_void_p()
        call("mitnc_plan_create", net.h, C.byref(o), C.byref(h))
        self.h = h
        self._lib = net._lib
        st = mitnc_plan_stats()
        call("mitnc_plan_query", h, C.byref(st))
        self.stats = st
        self._n_leaves = net.n_leaves
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

    def step_info(self, step: int) -> dict:
        """Address maps of one step (see mitnc_step_info)."""
        si = _lib.mitnc_step_info()
        call("mitnc_plan_step_info", self.h, step, C.byref(si))
        r = {f: int(getattr(si, f)) for f in ("a", "b", "out", "root", "kernel_class", "section", "section_pos",
                                              "section_len", "mb", "nb", "kb", "bb")}
        for f, cnt in (("am", "mb"), ("ak", "kb"), ("ab", "bb"), ("bk", "kb"), ("bn", "nb"), ("bbt", "bb"),
                       ("cm", "mb"), ("cn", "nb"), ("cb", "bb")):
            r[f] = list(getattr(si, f))[:r[cnt]]
        for f in ("tm", "tn", "tk", "vec_a", "vec_b"):
            r[f] = int(getattr(si, f))
        for f in ("a_tile", "b_tile", "lds_a_swz", "lds_b_swz", "lds_a_row", "lds_b_row", "lds_k_col"):
            r[f] = [int(x) for x in getattr(si, f)]
        return r

    def reverse_info(self, op: Optional[int] = None):
        """Number of adjoint contractions of the reverse pass (op None), or
        the description of one (see mitnc_plan_reverse_info; 'root' holds the
        reverse level)."""
        n = C.c_int32()
        if op is None:
            call("mitnc_plan_reverse_info", self.h, 0, None, C.byref(n))
            return n.value
        si = _lib.mitnc_step_info()
        call("mitnc_plan_reverse_info", self.h, op, C.byref(si), C.byref(n))
        r = {f: int(getattr(si, f)) for f in ("a", "b", "out", "root", "kernel_class", "mb", "nb", "kb", "bb")}
        r["level"] = r.pop("root")
        for f, cnt in (("am", "mb"), ("ak", "kb"), ("ab", "bb"), ("bk", "kb"), ("bn", "nb"), ("bbt", "bb"),
                       ("cm", "mb"), ("cn", "nb"), ("cb", "bb")):
            r[f] = list(getattr(si, f))[:r[cnt]]
        return r

    def node_info(self, node: int) -> dict:
        """Storage and schedule of one node (see mitnc_node_info)."""
        ni = _lib.mitnc_node_info()
        call("mitnc_plan_node_info", self.h, node, C.byref(ni))
        k = ni.n_slice_bits
        return {"is_leaf": bool(ni.is_leaf), "rank": ni.rank, "full_rank": ni.full_rank, "level": ni.level,
                "hoisted": bool(ni.hoisted), "slice_bits": list(zip(list(ni.slice_bit)[:k], list(ni.slice_pos)[:k])),
                "ws_offset": None if ni.ws_offset == 2 ** 64 - 1 else int(ni.ws_offset),
                "elig_mask": int(ni.elig_mask), "recompute_mask": int(ni.recompute_mask),
                "merge_mask": int(ni.merge_mask), "merge_tmp_offset": int(ni.merge_tmp_offset)}

    def schedule(self, slice_begin: int = 0, slice_end: Optional[int] = None) -> np.ndarray:
        """The launches mitnc_execute makes for a slice range: rows (slice,
        step, mode), mode 1 = store (root: accumulate), 2 = merge term."""
        if slice_end is None:
            slice_end = self.n_slices
        n = C.c_int64()
        call("mitnc_plan_schedule", self.h, slice_begin, slice_end, 0, None, C.byref(n))
        buf = np.zeros(3 * max(1, n.value), dtype=np.int64)
        call("mitnc_plan_schedule", self.h, slice_begin, slice_end, n.value,
             buf.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(n))
        return buf[:3 * n.value].reshape(-1, 3)

    def leaf_data(self, leaf: int) -> np.ndarray:
        """The complex64 entries the plan uploads for one leaf."""
        n = C.c_uint64()
        call("mitnc_plan_leaf_data", self.h, leaf, None, 0, C.byref(n))
        buf = np.zeros(n.value, dtype=np.float32)
        call("mitnc_plan_leaf_data", self.h, leaf, buf.ctypes.data_as(C.POINTER(C.c_float)), n.value, C.byref(n))
        return (buf[0::2] + 1j * buf[1::2]).astype(np.complex64)

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

    def calibrate(self, slice_begin: int = 0, slice_end: int = 1, stream=None) -> None:
        """FP16/BF16 plans: choose the per-tensor exponents from a complex64
        run of the given slices."""
        call("mitnc_calibrate", self.h, C.c_void_p(self.workspace.data_ptr()), self.workspace.numel(),
             int(slice_begin), int(slice_end), _stream_handle(stream))

    def step_maxima(self, reset: bool = False, stream=None) -> np.ndarray:
        """Largest stored |Re|, |Im| per step since the last reset (FP16/BF16)."""
        out = np.zeros(self.stats.n_steps, dtype=np.float32)
        call("mitnc_step_maxima", self.h, C.c_void_p(self.workspace.data_ptr()), self.workspace.numel(),
             out.ctypes.data_as(C.POINTER(C.c_float)), 1 if reset else 0, _stream_handle(stream))
        return out

    def exponents(self, new: Optional[Sequence[int]] = None):
        """(per-node exponents, exponent re-runs so far); with ``new`` the
        step outputs' exponents are replaced first (FP16/BF16 plans)."""
        nn = self.stats.n_steps + self._n_leaves
        out = np.zeros(nn, dtype=np.int32)
        rr = C.c_int32()
        inp = None
        if new is not None:
            arr = np.ascontiguousarray(np.asarray(new, dtype=np.int32))
            if arr.size != nn:
                raise ValueError("one exponent per node expected")
            inp = arr.ctypes.data_as(C.POINTER(C.c_int32))
        call("mitnc_plan_exponents", self.h, None, inp, None)
        call("mitnc_plan_exponents", self.h, out.ctypes.data_as(C.POINTER(C.c_int32)), None, C.byref(rr))
        return out, rr.value

    def set_gates(self, mats, stream=None) -> None:
        """Replace all single-qubit gate matrices (n_grad_gates x 2 x 2, U[out, in])."""
        m = np.ascontiguousarray(np.asarray(mats, dtype=np.complex128).reshape(-1)).view(np.float64)
        if m.size != 8 * self.stats.n_grad_gates:
            raise ValueError("expected n_grad_gates x 2 x 2 matrices")
        call("mitnc_plan_set_gates", self.h, C.c_void_p(self.workspace.data_ptr()), self.workspace.numel(),
             m.ctypes.data_as(C.POINTER(C.c_double)), _stream_handle(stream))
        self._gates = m.copy()

    def gates_equal(self, mats) -> bool:
        """True when the plan's single-qubit gate leaves were last set to mats."""
        cur = getattr(self, "_gates", None)
        m = np.ascontiguousarray(np.asarray(mats, dtype=np.complex128).reshape(-1)).view(np.float64)
        return cur is not None and cur.shape == m.shape and bool(np.array_equal(cur, m))

    def backward(self, w, grad, slice_begin: int = 0, slice_end: Optional[int] = None, stream=None):
        """grad += sum_r w[r] d result[r] / d U_g (holomorphic VJP; complex128
        device tensors: w with result_elems entries, grad with 4 n_grad_gates)."""
        import torch
        if w.dtype != torch.complex128 or not w.is_contiguous() or w.numel() != self.stats.result_elems:
            raise ValueError("w must be a contiguous complex128 tensor of result_elems entries")
        if grad.dtype != torch.complex128 or not grad.is_contiguous() or grad.numel() != 4 * self.stats.n_grad_gates:
            raise ValueError("grad must be a contiguous complex128 tensor of 4 n_grad_gates entries")
        if slice_end is None:
            slice_end = self.n_slices
        call("mitnc_backward", self.h, C.c_void_p(self.workspace.data_ptr()), self.workspace.numel(),
             int(slice_begin), int(slice_end), C.c_void_p(w.data_ptr()), C.c_void_p(grad.data_ptr()),
             _stream_handle(stream))
        return grad

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


_ELEM_BYTES = {_lib.MITNC_C64: 8, _lib.MITNC_CF16: 4, _lib.MITNC_CBF16: 4}


def contract_work_bytes(la: Sequence[int], lb: Sequence[int], lc: Sequence[int], kernel: int = -1,
                        precision: int = _lib.MITNC_C64) -> int:
    """Device bytes of split-K partials a contraction with these layouts
    needs (host-only size query)."""
    la_ = (C.c_int64 * max(1, len(la)))(*la)
    lb_ = (C.c_int64 * max(1, len(lb)))(*lb)
    lc_ = (C.c_int64 * max(1, len(lc)))(*lc)
    need = C.c_size_t()
    call("mitnc_contract", None, len(la), la_, None, len(lb), lb_, None, len(lc), lc_, precision,
         C.c_float(1.0), kernel, None, 0, C.byref(need), None)
    return int(need.value)


def contract(a, la: Sequence[int], b, lb: Sequence[int], lc: Sequence[int], kernel: int = -1,
             precision: int = _lib.MITNC_C64, out_scale: float = 1.0, stream=None, out=None,
             noalloc: bool = False):
    """One pairwise contraction on the GPU.  a, b: contiguous device tensors
    holding 2^len(la) / 2^len(lb) complex entries in the storage of
    `precision` (complex64, or interleaved FP16/BF16 halves in any 4-byte-per-
    entry dtype); address bit i carries label la[i] (LSB first).  Returns C
    with address bits lc (complex64 tensor, or int32 words of 16-bit pairs),
    scaled by out_scale.  ``out`` (optional) is a preallocated result of the
    right size; with ``noalloc`` the library's allocation-free entry point
    runs the contraction (split-K partials in its fixed device scratch)."""
    import torch
    eb = _ELEM_BYTES[precision]
    la_ = (C.c_int64 * max(1, len(la)))(*la)
    lb_ = (C.c_int64 * max(1, len(lb)))(*lb)
    lc_ = (C.c_int64 * max(1, len(lc)))(*lc)
    need = C.c_size_t()
    call("mitnc_contract", None, len(la), la_, None, len(lb), lb_, None, len(lc), lc_, precision,
         C.c_float(out_scale), kernel, None, 0, C.byref(need), None)
    for t, r in ((a, len(la)), (b, len(lb))):
        if not t.is_contiguous() or t.numel() * t.element_size() != (1 << r) * eb:
            raise ValueError("operand size does not match its labels and precision")
    dt = torch.complex64 if precision == _lib.MITNC_C64 else torch.int32
    if out is None:
        out = torch.empty(1 << len(lc), dtype=dt, device=a.device)
    elif out.dtype != dt or not out.is_contiguous() or out.numel() != (1 << len(lc)):
        raise ValueError("out does not match the output labels and precision")
    if noalloc:
        call("mitnc_contract_noalloc", C.c_void_p(a.data_ptr()), len(la), la_, C.c_void_p(b.data_ptr()), len(lb),
             lb_, C.c_void_p(out.data_ptr()), len(lc), lc_, precision, C.c_float(out_scale), kernel,
             _stream_handle(stream))
        return out
    work = torch.empty(max(256, need.value), dtype=torch.uint8, device=a.device) if need.value else None
    call("mitnc_contract", C.c_void_p(a.data_ptr()), len(la), la_, C.c_void_p(b.data_ptr()), len(lb), lb_,
         C.c_void_p(out.data_ptr()), len(lc), lc_, precision, C.c_float(out_scale), kernel,
         C.c_void_p(work.data_ptr()) if work is not None else None, need.value, None,
         _stream_handle(stream))
    return out


def amplitudes(circuit, spec, batch_bits=None, seed: int = 0, trials: int = 32, max_log2: int = 30,
               min_sliced: int = 0, slices: Optional[Tuple[int, int]] = None, reuse: bool = True,
               precision: int = _lib.MITNC_C64, device="cuda"):
    """Requested amplitudes (complex128 device tensor in the canonical result
    order), or the partial sum over ``slices = (begin, end)``."""
    net = Network(circuit, spec, batch_bits)
    net.path_search(seed=seed, trials=trials, max_log2=max_log2, min_sliced=min_sliced)
    plan = Plan(net, precision=precision, reuse=reuse)
    plan.upload(device)
    s0, s1 = slices if slices is not None else (0, plan.n_slices)
    if precision != _lib.MITNC_C64:
        plan.calibrate(s0, min(s1, s0 + 2))
    acc = plan.new_result(device)
    plan.execute(acc, s0, s1)
    return acc


def _amplitude_fn():
    import torch

    class AmplitudeFn(torch.autograd.Function):
        """amplitudes = AmplitudeFn.apply(gates, plan): the requested amplitudes
        (complex128, result order) as a function of the single-qubit gate
        matrices (complex128 tensor n_grad_gates x 2 x 2).  The backward pass
        runs the library's reverse contraction (recomputing each slice's
        forward) and returns conj of the holomorphic VJP with weights
        conj(grad_output), which is torch's convention for complex inputs."""

        @staticmethod
        def forward(ctx, gates, plan):
            mats = gates.detach().cpu().numpy().copy()
            plan.set_gates(mats)
            acc = plan.new_result(plan.workspace.device)
            plan.execute(acc)
            ctx.plan = plan
            # the plan's gate leaves may be replaced by another forward before
            # this backward runs: keep this call's matrices and restore them
            ctx.mats = mats
            ctx.gates_device = gates.device
            return acc

        @staticmethod
        def backward(ctx, grad_out):
            plan = ctx.plan
            if not plan.gates_equal(ctx.mats):
                plan.set_gates(ctx.mats)
            # conj_physical: a lazy conj() view would hand the library the
            # unconjugated bytes
            w = torch.conj_physical(grad_out.to(torch.complex128)).contiguous()
            grad = torch.zeros(4 * plan.stats.n_grad_gates, dtype=torch.complex128, device=w.device)
            plan.backward(w, grad)
            g = grad.conj().reshape(-1, 2, 2).to(ctx.gates_device)
            return g, None

    return AmplitudeFn


_AMPFN = None


def AmplitudeFn():
    """The torch.autograd.Function class (created on first use)."""
    global _AMPFN
    if _AMPFN is None:
        _AMPFN = _amplitude_fn()
    return _AMPFN
