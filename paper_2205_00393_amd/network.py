"""Tensor networks and the host planner, through libltn (marshalling only).

The planner steps (network construction and absorption, greedy path,
Eq. (1)/(4) costs, stem, Algorithm 1) all run inside the native library.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

from . import _lib as L

_KIND = {"sqrt_x": L.LTN_GATE_SQRT_X, "sqrt_y": L.LTN_GATE_SQRT_Y, "sqrt_w": L.LTN_GATE_SQRT_W,
         "fsim": L.LTN_GATE_FSIM, "u3": L.LTN_GATE_U3, "matrix": L.LTN_GATE_MATRIX}


def _gate_array(gates):
    arr = (L.Gate * max(1, len(gates)))()
    for i, g in enumerate(gates):
        e = arr[i]
        e.kind = _KIND[g.name]
        e.q0 = g.qubits[0]
        e.q1 = g.qubits[1] if len(g.qubits) > 1 else -1
        e.param_id = g.param_id
        if g.name == "matrix":
            flat = [complex(x) for x in g.params]
            for j, z in enumerate(flat):
                e.m[2 * j] = z.real
                e.m[2 * j + 1] = z.imag
        else:
            for j, v in enumerate(g.params[:3]):
                e.p[j] = float(v)
    return arr


class Network:
    """A network owned by libltn, or wrapped from Python arrays."""

    def __init__(self):
        self._nb = None
        self._keep = []
        self.view = L.Network()

    @classmethod
    def from_circuit(cls, circuit, open_qubits: Sequence[int], closed_bits: dict,
                     absorb: bool = True) -> "Network":
        self = cls()
        n = circuit.n_qubits
        cb = [-1 if q in set(open_qubits) else int(closed_bits[q]) for q in range(n)]
        nb = C.c_void_p()
        gates = _gate_array(circuit.gates)
        L.check(L.lib().ltn_network_build(n, gates, len(circuit.gates), L.i32_array(cb),
                                          1 if absorb else 0, C.byref(nb)))
        self._nb = nb
        L.check(L.lib().ltn_netbuf_view(nb, C.byref(self.view)))
        return self

    @classmethod
    def from_arrays(cls, indices: List[List[int]], data: List[np.ndarray], open_ids: List[int],
                    n_indices: int, param: Optional[List[int]] = None) -> "Network":
        self = cls()
        off = np.zeros(len(indices) + 1, dtype=np.int64)
        off[1:] = np.cumsum([len(ix) for ix in indices])
        ids = np.asarray([x for ix in indices for x in ix] or [0], dtype=np.int32)
        flat = np.concatenate([np.asarray(d, dtype=np.complex64).reshape(-1) for d in data])
        f32 = np.ascontiguousarray(flat.view(np.float32))
        opens = np.asarray(list(open_ids) or [0], dtype=np.int32)
        par = np.asarray(param if param is not None else [-1] * len(indices), dtype=np.int32)
        self._keep = [off, ids, f32, opens, par]
        v = self.view
        v.n_leaves = len(indices)
        v.leaf_off = off.ctypes.data_as(C.POINTER(C.c_int64))
        v.index_ids = ids.ctypes.data_as(C.POINTER(C.c_int32))
        v.leaf_data = f32.ctypes.data_as(C.POINTER(C.c_float))
        v.n_open = len(open_ids)
        v.open_ids = opens.ctypes.data_as(C.POINTER(C.c_int32))
        v.n_indices = n_indices
        v.param_leaf = par.ctypes.data_as(C.POINTER(C.c_int32))
        return self

    def __del__(self):
        if self._nb is not None:
            try:
                L.lib().ltn_netbuf_free(self._nb)
            except Exception:
                pass
            self._nb = None

    # ---- read-only views -------------------------------------------------
    @property
    def n_leaves(self) -> int:
        return self.view.n_leaves

    @property
    def n_indices(self) -> int:
        return self.view.n_indices

    @property
    def open_ids(self) -> List[int]:
        return [self.view.open_ids[j] for j in range(self.view.n_open)]

    @property
    def indices(self) -> List[List[int]]:
        v = self.view
        return [[v.index_ids[j] for j in range(v.leaf_off[i], v.leaf_off[i + 1])]
                for i in range(v.n_leaves)]

    @property
    def params(self) -> List[int]:
        return [self.view.param_leaf[i] for i in range(self.view.n_leaves)]

    def leaf_data(self, precision: str = "c64") -> List[np.ndarray]:
        v = self.view
        out = []
        off = 0
        if precision == "c128":
            assert self._nb is not None
            ptr = C.POINTER(C.c_double)()
            L.check(L.lib().ltn_netbuf_data128(self._nb, C.byref(ptr)))
        for i in range(v.n_leaves):
            r = v.leaf_off[i + 1] - v.leaf_off[i]
            n = 1 << r
            if precision == "c128":
                a = np.ctypeslib.as_array(ptr, shape=(2 * (off + n),))[2 * off:].view(np.complex128)
            else:
                a = np.ctypeslib.as_array(v.leaf_data, shape=(2 * (off + n),))[2 * off:].view(np.complex64)
            out.append(a.copy().reshape([2] * r))
            off += n
        return out


def _path_array(path):
    flat = [int(x) for p in path for x in p]
    return L.i32_array(flat)


def greedy_path(net: Network, alpha: float = 1.0, tau: float = 0.0, seed: int = 0,
                exclude: Sequence[int] = ()):
    out = (C.c_int32 * max(1, 2 * (net.n_leaves - 1)))()
    ex = list(exclude)
    L.check(L.lib().ltn_greedy_path(C.byref(net.view), L.i32_array(ex), len(ex), alpha, tau,
                                    seed, out))
    return [(out[2 * k], out[2 * k + 1]) for k in range(net.n_leaves - 1)]


@dataclass
class Costs:
    cost: int
    sliced: int
    log2_cost: float
    log2_sliced: float
    overhead: float
    space_log2: int
    space_log2_unsliced: int
    stem_len: int


def tree_costs(net: Network, path, S: Sequence[int]) -> Costs:
    c = L.Costs()
    L.check(L.lib().ltn_tree_costs(C.byref(net.view), _path_array(path), L.i32_array(list(S)),
                                   len(S), C.byref(c)))
    return Costs(L.words_to_int(c.cost_words), L.words_to_int(c.sliced_words), c.log2_cost,
                 c.log2_sliced, c.overhead, c.space_log2, c.space_log2_unsliced, c.stem_len)


def tree_stem(net: Network, path) -> List[int]:
    cap = 2 * net.n_leaves
    out = (C.c_int32 * cap)()
    n = C.c_int32()
    L.check(L.lib().ltn_tree_stem(C.byref(net.view), _path_array(path), out, cap, C.byref(n)))
    return list(out[: n.value])


def stem_profile(net: Network, path, S: Sequence[int] = ()) -> List[dict]:
    """One row per stem tensor, leaf to root (``ltn_stem_profile``): node id,
    rank, rank after S, and log2 of the Eq. (1) node cost without and with
    S (None for the leaf)."""
    cap = 2 * net.n_leaves
    rows = (L.StemRow * cap)()
    n = C.c_int32()
    L.check(L.lib().ltn_stem_profile(C.byref(net.view), _path_array(path), L.i32_array(list(S)), len(S),
                                     rows, cap, C.byref(n)))
    return [{"tensor": r.tensor, "rank": r.rank, "rank_sliced": r.rank_sliced,
             "log2_node_cost": None if r.node_bits < 0 else r.node_bits,
             "log2_node_cost_sliced": None if r.node_bits_sliced < 0 else r.node_bits_sliced}
            for r in rows[: n.value]]


def slice_finder(net: Network, path, t: int, pre: Sequence[int] = ()) -> List[int]:
    cap = net.n_indices + 1
    out = (C.c_int32 * cap)()
    n = C.c_int32()
    L.check(L.lib().ltn_slice_finder(C.byref(net.view), _path_array(path), t,
                                     L.i32_array(list(pre)), len(pre), out, cap, C.byref(n)))
    return list(out[: n.value])


def slice_refine(net: Network, path, t: int, S: Sequence[int], n_fixed: int = 0, t0: float = 1.0,
                 alpha: float = 0.98, tf: float = 1e-3, iters_per_temp: int = 1, seed: int = 0):
    """Slice refiner (Algorithms 2-4); returns (S, stats dict)."""
    o = L.RefineOpts(t0, alpha, tf, iters_per_temp, n_fixed, seed)
    out = (C.c_int32 * max(1, len(S)))()
    n = C.c_int32()
    st = L.RefineStats()
    L.check(L.lib().ltn_slice_refine(C.byref(net.view), _path_array(path), t, L.i32_array(list(S)),
                                     len(S), C.byref(o), out, C.byref(n), C.byref(st)))
    return list(out[: n.value]), {"iterations": st.iterations, "proposals": st.proposals,
                                  "accepted": st.accepted, "dropped": st.dropped}


def tree_reconfigure(net: Network, path, k: int = 8, sweeps: int = 1, S: Sequence[int] = (),
                     t: int = -1):
    """Subtree reconfiguration; returns the new SSA path."""
    out = (C.c_int32 * max(1, 2 * (net.n_leaves - 1)))()
    L.check(L.lib().ltn_tree_reconfigure(C.byref(net.view), _path_array(path), k, sweeps,
                                         L.i32_array(list(S)), len(S), t, out))
    return [(out[2 * j], out[2 * j + 1]) for j in range(net.n_leaves - 1)]


def slice_greedy_overhead(net: Network, path, t: int, pre: Sequence[int] = ()) -> List[int]:
    """Greedy least-overhead slicer (comparison baseline for Algorithm 1)."""
    cap = net.n_indices + 1
    out = (C.c_int32 * cap)()
    n = C.c_int32()
    L.check(L.lib().ltn_slice_greedy_overhead(C.byref(net.view), _path_array(path), t,
                                              L.i32_array(list(pre)), len(pre), out, cap,
                                              C.byref(n)))
    return list(out[: n.value])


def path_search(net: Network, t: int, pre: Sequence[int] = (), alphas=(1.0,), taus=(0.0,),
                n_seeds: int = 1, seed_base: int = 0, reconf_k: int = 0, reconf_sweeps: int = 4):
    """Randomised greedy trials (optionally improved by subtree
    reconfiguration) + slice finder; returns (path, S, best trial)."""
    a = (C.c_double * len(alphas))(*alphas)
    tt = (C.c_double * len(taus))(*taus)
    o = L.SearchOpts(len(alphas), a, len(taus), tt, n_seeds, seed_base, reconf_k, reconf_sweeps)
    path = (C.c_int32 * max(1, 2 * (net.n_leaves - 1)))()
    cap = net.n_indices + 1
    S = (C.c_int32 * cap)()
    n = C.c_int32()
    best = C.c_int32()
    L.check(L.lib().ltn_path_search(C.byref(net.view), t, L.i32_array(list(pre)), len(pre),
                                    C.byref(o), path, S, cap, C.byref(n), C.byref(best)))
    return ([(path[2 * k], path[2 * k + 1]) for k in range(net.n_leaves - 1)],
            list(S[: n.value]), best.value)


# default search grid of the randomised greedy (alpha-major, tau, seeds)
SEARCH_ALPHAS = (0.5, 1.0, 2.0)
SEARCH_TAUS = (0.0, 0.3, 1.0)
SEARCH_SEEDS = 16
