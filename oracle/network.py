"""Tensor network of a circuit, rank-1/2 absorption and plain contraction.

Notation follows the paper's Sec. 2.1.1: a network is a graph whose vertices
are tensors and whose edges are indices of size w(e) = 2; contracting two
vertices removes the edges they share and keeps the rest. Every index lies
in at most two tensors (supplement, Lemma 1 "Conservation").

Network conventions (the paper is silent; these are the build's readings):

* index ids in creation order: the initial wire of qubit q gets id q; then
  every gate, in circuit order, creates one new index per qubit it acts on
  (its output wire, in the gate's qubit order);
* tensors in order: |0> on each qubit (ascending q), one tensor per gate in
  circuit order with axes (out..., in...), then <b_q| on each closed qubit
  (ascending q); the final wires of open qubits are open indices, listed in
  ascending qubit order (first = most significant output bit);
* absorption (Sec. 2.1.2, "rank-1 and rank-2 tensors are absorbed"):
  repeatedly take the lowest-id tensor T that is not a u3 leaf, has rank <= 2
  and has a neighbour (a tensor sharing an index; any tensor if T is a
  scalar) that is not a u3 leaf; merge it into its lowest-id such neighbour
  N. The merged tensor keeps N's place, with axes = N's unshared axes then
  T's unshared axes. Afterwards tensors and indices are renumbered densely
  in ascending old id.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import numpy as np

from .gates import gate_matrix


@dataclass
class Network:
    indices: List[List[int]]          # per tensor, axis order (first slowest)
    data: List[np.ndarray]            # complex128, shape [2]*rank
    param: List[int]                  # u3 gate number or -1
    open_ids: List[int]               # output order, first = most significant
    n_indices: int
    meta: dict = field(default_factory=dict)

    def copy(self) -> "Network":
        return Network([list(i) for i in self.indices], [d.copy() for d in self.data],
                       list(self.param), list(self.open_ids), self.n_indices, dict(self.meta))


def circuit_network(circuit, open_qubits: Sequence[int], closed_bits: Dict[int, int]) -> Network:
    """Raw (unsimplified) network of <b| C |0> with ``open_qubits`` left open."""
    n = circuit.n_qubits
    wire = list(range(n))
    next_id = n
    indices, data, param = [], [], []
    for q in range(n):
        indices.append([q])
        data.append(np.array([1.0, 0.0], dtype=np.complex128))
        param.append(-1)
    for g in circuit.gates:
        k = len(g.qubits)
        outs = []
        for q in g.qubits:
            outs.append(next_id)
            next_id += 1
        ins = [wire[q] for q in g.qubits]
        for q, o in zip(g.qubits, outs):
            wire[q] = o
        indices.append(outs + ins)
        data.append(gate_matrix(g).reshape([2] * (2 * k)))
        param.append(g.param_id if g.name == "u3" else -1)
    open_set = set(open_qubits)
    for q in range(n):
        if q in open_set:
            continue
        v = np.zeros(2, dtype=np.complex128)
        v[closed_bits[q]] = 1.0
        indices.append([wire[q]])
        data.append(v)
        param.append(-1)
    open_ids = [wire[q] for q in sorted(open_set)]
    return Network(indices, data, param, open_ids, next_id)


def _merge(ni, nd, ti, td):
    """Contract tensor (ti, td) into (ni, nd) over their shared indices."""
    shared = [x for x in ni if x in ti]
    ax_n = [ni.index(x) for x in shared]
    ax_t = [ti.index(x) for x in shared]
    out = np.tensordot(nd, td, axes=(ax_n, ax_t))
    idx = [x for x in ni if x not in shared] + [x for x in ti if x not in shared]
    return idx, out


def absorb_small(net: Network) -> Network:
    """Absorb non-parameterised rank-1/rank-2 tensors (rule in module doc)."""
    idx = {i: list(v) for i, v in enumerate(net.indices)}
    dat = {i: v for i, v in enumerate(net.data)}
    par = {i: p for i, p in enumerate(net.param)}
    while True:
        chosen = None
        for t in sorted(idx):
            if par[t] >= 0 or len(idx[t]) > 2:
                continue
            if len(idx[t]) == 0:
                cands = [u for u in idx if u != t and par[u] < 0]
            else:
                ts = set(idx[t])
                cands = [u for u in idx if u != t and par[u] < 0 and ts & set(idx[u])]
            if cands:
                chosen = (t, min(cands))
                break
        if chosen is None:
            break
        t, nb = chosen
        idx[nb], dat[nb] = _merge(idx[nb], dat[nb], idx[t], dat[t])
        del idx[t], dat[t], par[t]
    keep = sorted(idx)
    used = sorted({x for t in keep for x in idx[t]})
    remap = {old: new for new, old in enumerate(used)}
    return Network([[remap[x] for x in idx[t]] for t in keep], [dat[t] for t in keep],
                   [par[t] for t in keep], [remap[x] for x in net.open_ids], len(used),
                   dict(net.meta, kept=keep))


def fix_indices(indices: List[int], data: np.ndarray, fixed: Dict[int, int]):
    """Slice a tensor: every index in ``fixed`` takes its given value."""
    sel = tuple(fixed[x] if x in fixed else slice(None) for x in indices)
    return [x for x in indices if x not in fixed], data[sel]


def contract_path(net: Network, path, fixed: Optional[Dict[int, int]] = None,
                  out_order: Optional[List[int]] = None) -> np.ndarray:
    """Contract pairwise along an SSA path (leaves 0..L-1, the k-th step
    makes L+k), with the indices in ``fixed`` sliced to their values.

    Returns the final tensor with axes in ``out_order`` (default: the open
    indices that are not fixed, in output order), flattened.
    """
    fixed = fixed or {}
    L = len(net.indices)
    tens = {}
    for i in range(L):
        tens[i] = fix_indices(net.indices[i], net.data[i], fixed)
    for k, (a, b) in enumerate(path):
        ia, da = tens.pop(a)
        ib, db = tens.pop(b)
        tens[L + k] = _merge(ia, da, ib, db)
    if len(tens) != 1:
        raise ValueError("path does not reduce the network to one tensor")
    (ix, d), = tens.values()
    if out_order is None:
        out_order = [x for x in net.open_ids if x not in fixed]
    if sorted(ix) != sorted(out_order):
        raise ValueError("final tensor's indices differ from the requested order")
    perm = [ix.index(x) for x in out_order]
    return np.transpose(d, perm).reshape(-1) if perm else d.reshape(-1)


def slice_values(S: Sequence[int], s: int) -> Dict[int, int]:
    """Slice id s -> index values: bit j (LSB first) of s is the value of S[j]."""
    return {x: (s >> j) & 1 for j, x in enumerate(S)}


def slice_output(net: Network, path, S: Sequence[int], s: int) -> np.ndarray:
    """Result of one slice (Sec. 2.1.1: one of the 2^|S| subtasks)."""
    return contract_path(net, path, slice_values(S, s))


def place(net: Network, S: Sequence[int], s: int, block: np.ndarray) -> tuple:
    """Output positions of a slice's block: open indices in S take their
    values from the slice id, the rest run over the block."""
    vals = slice_values(S, s)
    n_open = len(net.open_ids)
    free = [j for j, x in enumerate(net.open_ids) if x not in vals]
    pos = np.zeros(len(block), dtype=np.int64)
    base = 0
    for j, x in enumerate(net.open_ids):
        if x in vals:
            base |= vals[x] << (n_open - 1 - j)
    for e in range(len(block)):
        p = base
        for r, j in enumerate(free):
            bit = (e >> (len(free) - 1 - r)) & 1
            p |= bit << (n_open - 1 - j)
        pos[e] = p
    return pos


def sliced_sum(net: Network, path, S: Sequence[int], slice_ids=None) -> np.ndarray:
    """Sum (and placement of sliced open indices) over the given slices
    (default: all 2^|S|). Equals the unsliced contraction when all slices
    are taken (Sec. 2.1.1: results of the subtasks are accumulated)."""
    out = np.zeros(1 << len(net.open_ids), dtype=np.complex128)
    ids = range(1 << len(S)) if slice_ids is None else slice_ids
    for s in ids:
        blk = slice_output(net, path, S, int(s))
        out[place(net, S, int(s), blk)] += blk
    return out
