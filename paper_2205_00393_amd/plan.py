"""Compiled plans and their execution on the GPU (marshalling only).

PyTorch supplies device memory (the workspace, outputs, gradients) and the
stream; every step of the contraction runs in libltn's HIP kernels.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

from . import _lib as L
from .network import (Network, path_search, slice_refine, tree_costs, SEARCH_ALPHAS, SEARCH_TAUS,
                      SEARCH_SEEDS)


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Plan:
    def __init__(self, net: Network, path, sliced: Sequence[int], max_rank: int = -1,
                 batch: int = 0, fat_threshold: int = 0, fuse_rank: int = 0):
        self.net = net
        self.path = [tuple(p) for p in path]
        self.sliced = [int(x) for x in sliced]
        flat = [int(x) for p in self.path for x in p]
        opt = L.Options(max_rank, batch, fat_threshold, fuse_rank)
        h = C.c_void_p()
        L.check(L.lib().ltn_plan_load(C.byref(net.view), L.i32_array(flat), len(self.sliced),
                                      L.i32_array(self.sliced), C.byref(opt), C.byref(h)))
        self._h = h
        self._ws = None
        self.grad_bound = False
        self.params_token = 0  # counts set_params calls

    def __del__(self):
        if getattr(self, "_h", None):
            try:
                L.lib().ltn_plan_free(self._h)
            except Exception:
                pass
            self._h = None

    # ---- host description ---------------------------------------------
    def info(self) -> dict:
        i = L.PlanInfo()
        L.check(L.lib().ltn_plan_describe(self._h, C.byref(i)))
        return dict(n_leaves=i.n_leaves, n_steps=i.n_steps, n_sliced=i.n_sliced, n_open=i.n_open,
                    n_open_unsliced=i.n_open_unsliced, n_params=i.n_params, batch=i.batch,
                    root_rank=i.root_rank, macs_per_slice=L.words_to_int(i.macs_words),
                    arena_bytes_per_slice=i.arena_bytes_per_slice,
                    grad_arena_bytes_per_slice=i.grad_arena_bytes_per_slice,
                    const_bytes=i.const_bytes,
                    sliced_ids=[i.sliced_ids[j] for j in range(i.n_sliced)])

    def step(self, k: int) -> dict:
        s = L.StepInfo()
        L.check(L.lib().ltn_plan_step(self._h, k, C.byref(s)))
        ka = s.m + s.k
        kb = s.n + s.k
        return dict(left=s.left, right=s.right, out=s.out, a_is_left=s.a_is_left, m=s.m, k=s.k,
                    n=s.n, kernel=s.kernel, a_idx=[s.a_idx[j] for j in range(ka)],
                    b_idx=[s.b_idx[j] for j in range(kb)],
                    c_idx=[s.c_idx[j] for j in range(s.m + s.n)], c_mask_a=s.c_mask_a,
                    arena_off=(s.arena_off_a, s.arena_off_b, s.arena_off_c))

    def groups(self) -> List[dict]:
        """Fused sub-paths: first step, number of steps, |Sigma|, working rank."""
        cap = max(1, self.info()["n_steps"])
        a, b, c, d = [(C.c_int32 * cap)() for _ in range(4)]
        n = C.c_int32()
        L.check(L.lib().ltn_plan_groups(self._h, a, b, c, d, cap, C.byref(n)))
        return [dict(first_step=a[g], n_steps=b[g], n_sigma=c[g], work_rank=d[g]) for g in range(n.value)]

    def set_fusion(self, enable: bool) -> None:
        L.check(L.lib().ltn_set_fusion(self._h, 1 if enable else 0))

    def steps(self) -> List[dict]:
        return [self.step(k) for k in range(self.info()["n_steps"])]

    def workspace_size(self, batch: int, grad: bool = False) -> int:
        n = C.c_size_t()
        L.check(L.lib().ltn_workspace_size(self._h, batch, 1 if grad else 0, C.byref(n)))
        return n.value

    # ---- device ---------------------------------------------------------
    def bind(self, batch: int = 0, grad: bool = False, budget_bytes: Optional[int] = None,
             device: str = "cuda", stream=None) -> int:
        """Allocate a workspace for ``batch`` slices per launch (0: as many
        as fit in ``budget_bytes``) and bind it; returns the batch size."""
        torch = _torch()
        if batch > 0:
            nbytes = self.workspace_size(batch, grad)
        else:
            if budget_bytes is None:
                free, _ = torch.cuda.mem_get_info()
                budget_bytes = int(free * 0.6)
            cap = min(4096, 1 << min(len(self.sliced), 12))
            nbytes = min(budget_bytes, self.workspace_size(cap, grad))
        self._ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self._stream = stream
        L.check(L.lib().ltn_bind(self._h, C.c_void_p(self._ws.data_ptr()), nbytes,
                                 1 if grad else 0, _stream_ptr(stream)))
        self.grad_bound = grad
        return self.info()["batch"]

    def new_output(self, device: str = "cuda"):
        torch = _torch()
        return torch.zeros(1 << self.info()["n_open"], dtype=torch.complex128, device=device)

    def execute(self, slice_ids, out=None, mode: str = "c64"):
        """Add the listed slices into ``out`` (complex128, 2^n_open)."""
        if out is None:
            out = self.new_output()
        ids = np.ascontiguousarray(np.asarray(slice_ids, dtype=np.uint64).reshape(-1))
        L.check(L.lib().ltn_execute(self._h, ids.ctypes.data_as(C.POINTER(C.c_uint64)), len(ids),
                                    L.MODES[mode], C.c_void_p(out.data_ptr())))
        return out

    def execute_range(self, begin: int, end: int, out=None, mode: str = "c64"):
        if out is None:
            out = self.new_output()
        L.check(L.lib().ltn_execute_range(self._h, begin, end, L.MODES[mode],
                                          C.c_void_p(out.data_ptr())))
        return out

    def execute_scratch(self, slice_ids, out=None, mode: str = "c64", stream=None):
        """Add the listed slices into ``out`` using the library's own device
        scratch (no workspace, no allocation by the library)."""
        if out is None:
            out = self.new_output()
        ids = np.ascontiguousarray(np.asarray(slice_ids, dtype=np.uint64).reshape(-1))
        L.check(L.lib().ltn_execute_scratch(self._h, ids.ctypes.data_as(C.POINTER(C.c_uint64)), len(ids),
                                            L.MODES[mode], C.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def set_params(self, angles):
        """angles: float64 CUDA tensor [n_params] laid out [gate][a, b, c]."""
        a = angles.contiguous()
        L.check(L.lib().ltn_set_params(self._h, C.c_void_p(a.data_ptr())))
        self._angles = a
        self.params_token += 1

    def execute_grad(self, slice_ids, cotangent, out=None, angle_grad=None, mode: str = "c64"):
        torch = _torch()
        ids = np.ascontiguousarray(np.asarray(slice_ids, dtype=np.uint64).reshape(-1))
        if angle_grad is None:
            angle_grad = torch.zeros(self.info()["n_params"], dtype=torch.float64,
                                     device=cotangent.device)
        cot = cotangent.contiguous()
        L.check(L.lib().ltn_execute_grad(self._h, ids.ctypes.data_as(C.POINTER(C.c_uint64)),
                                         len(ids), L.MODES[mode], C.c_void_p(cot.data_ptr()),
                                         C.c_void_p(out.data_ptr() if out is not None else 0),
                                         C.c_void_p(angle_grad.data_ptr())))
        return angle_grad

    def autotune(self, mode: str = "c64", cache: Optional[str] = None):
        L.check(L.lib().ltn_autotune(self._h, L.MODES[mode], cache.encode() if cache else None))

    def profile_steps(self, first: int = 0, mode: str = "c64") -> np.ndarray:
        n = self.info()["n_steps"]
        out = (C.c_float * max(1, n))()
        L.check(L.lib().ltn_profile_steps(self._h, first, L.MODES[mode], out))
        return np.asarray(out[:n], dtype=np.float64)

    def set_step_kernel(self, k: int, mode: str, kind: int, cfg: int = 0, swap: int = 0,
                        tk: int = 1) -> None:
        """Force the kernel of step k in a mode (kind 0 generic with tk, 1
        complex64 MFMA, 2 split MFMA, 3 narrow, 4 split sum for m, n <= 3)."""
        L.check(L.lib().ltn_set_step_kernel(self._h, k, L.MODES[mode], kind, cfg, swap, tk))

    def step_kernel(self, k: int, mode: str = "c64"):
        """(kind, cfg, swap, tk): kind 0 generic, 1 complex64 MFMA, 2 split MFMA,
        3 narrow, 4 split sum, 5 split-K complex64 MFMA."""
        kind, cfg, sw, tk = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        L.check(L.lib().ltn_step_kernel(self._h, k, L.MODES[mode], C.byref(kind), C.byref(cfg),
                                        C.byref(sw), C.byref(tk)))
        return kind.value, cfg.value, sw.value, tk.value

    def step_kernel_name(self, k: int, mode: str = "c64") -> str:
        """Name of the kernel choice of step k (ltn_kernel_name)."""
        kind, cfg, _, _ = self.step_kernel(k, mode)
        return kernel_name(kind, cfg, mode)


def kernel_name(kind: int, cfg: int, mode: str = "c64") -> str:
    """Name of a kernel choice (ltn_kernel_name); "?" if there is none."""
    return L.lib().ltn_kernel_name(kind, cfg, L.MODES[mode]).decode()


@dataclass
class Prepared:
    """A workload turned into a network, a path and a slicing set."""
    workload: object
    net: Network
    path: list
    sliced: list
    trial: int
    pre: list

    def plan(self, **kw) -> Plan:
        t = self.workload.max_rank
        return Plan(self.net, self.path, self.sliced, max_rank=t if t is not None else -1, **kw)

    def slice_of_bitstring(self, x: int) -> int:
        """Slice id of an output bitstring when the open indices are sliced
        (the pre-sliced open indices come first in S, last open qubit first)."""
        n_open = len(self.workload.open_qubits)
        s = 0
        for j in range(n_open):
            s |= ((x >> j) & 1) << j
        return s


def prepare(workload, alphas=SEARCH_ALPHAS, taus=SEARCH_TAUS, n_seeds=SEARCH_SEEDS,
            seed_base: int = 0, reconf_k: int = 0, reconf_sweeps: int = 4,
            refine_seeds: int = 0) -> Prepared:
    """Host planner for a workload: network (with absorption), randomised
    greedy path search (optionally with subtree reconfiguration) and
    lifetime-based slicing under its max rank; with refine_seeds > 0 the
    slicing set is then refined (Algorithms 2-4) with seeds 0..refine_seeds-1
    and the best result (C(B,S), |S|, seed) is kept."""
    w = workload
    net = Network.from_circuit(w.circuit, w.open_qubits, w.closed_bits)
    pre = []
    if w.slice_open:
        # every output bitstring is one slice: S starts with the open indices,
        # last open qubit first so that slice id == bitstring
        pre = list(reversed(net.open_ids))
    t = w.max_rank if w.max_rank is not None else -1
    path, S, trial = path_search(net, t, pre, alphas, taus, n_seeds, seed_base, reconf_k,
                                 reconf_sweeps)
    if refine_seeds > 0 and t >= 0:
        best = None
        for sd in range(refine_seeds):
            R, _ = slice_refine(net, path, t, S, n_fixed=len(pre), seed=sd)
            key = (tree_costs(net, path, R).sliced, len(R), sd)
            if best is None or key < best[0]:
                best = (key, R)
        S = best[1]
    return Prepared(w, net, path, S, trial, pre)


def permute(x, perm, out=None, stream=None):
    """Bit permutation of complex64 CUDA tensors: x has shape [batch, 2^rank]
    (or [2^rank]); out[b][y] = x[b][x_] with bit perm[j] of y = bit j of x_."""
    torch = _torch()
    rank = len(perm)
    xx = x.contiguous()
    batch = xx.numel() >> rank
    if out is None:
        out = torch.empty_like(xx)
    L.check(L.lib().ltn_permute(C.c_void_p(xx.data_ptr()), C.c_void_p(out.data_ptr()), rank,
                                L.i32_array(list(perm)), batch, _stream_ptr(stream)))
    return out
