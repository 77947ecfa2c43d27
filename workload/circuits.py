"""Random quantum circuits on a 2-D grid, drawn from fixed seeds.

The paper simulates Sycamore-style random circuits (Introduction; Results,
"Sycamore RQC"). Its circuit files are not available, so the workloads here
are synthetic circuits of the same family:

* qubits on an R x C grid (optionally with sites removed), id = row-major
  rank among the kept sites;
* each cycle = one single-qubit layer on every qubit (ascending id), then one
  two-qubit layer on the couplers of pattern "ABCDCDAB"[cycle % 8];
* A / B = horizontal pairs (r,c)-(r,c+1) with c even / odd,
  C / D = vertical pairs (r,c)-(r+1,c) with r even / odd;
* single-qubit gates drawn from {sqrt_x, sqrt_y, sqrt_w}: uniform over the
  three in cycle 0, then uniform over the two that differ from the previous
  gate on the same qubit; draws are cycle-major, qubit-ascending, one
  ``rng.integers`` call per gate from ``numpy.random.default_rng(seed)``;
* two-qubit gates are fsim(theta=pi/2, phi=pi/6) on (q1 < q2);
* the gradient workload replaces every single-qubit gate by
  u3(a, b, c) with angles uniform in [0, 2*pi) drawn as one
  ``rng.uniform(0, 2*pi, size=(cycles, n_qubits, 3))`` array.

Only names, qubits and parameters are recorded here. Each consumer builds
its own matrices from the names.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

SINGLE_QUBIT_SET = ("sqrt_x", "sqrt_y", "sqrt_w")
FSIM_THETA = math.pi / 2
FSIM_PHI = math.pi / 6
DEFAULT_PATTERN = "ABCDCDAB"


@dataclass(frozen=True)
class Gate:
    """One gate: ``name`` in {sqrt_x, sqrt_y, sqrt_w, fsim, u3}.

    ``qubits`` is (q,) or (q1, q2) with q1 < q2; ``params`` is () for the
    fixed single-qubit gates, (theta, phi) for fsim and (a, b, c) for u3.
    ``param_id`` numbers the u3 gates 0.. in circuit order (-1 otherwise).
    """
    name: str
    qubits: Tuple[int, ...]
    params: Tuple[float, ...] = ()
    param_id: int = -1


@dataclass
class Circuit:
    rows: int
    cols: int
    cycles: int
    n_qubits: int
    removed: Tuple[Tuple[int, int], ...]
    pattern: str
    gates: List[Gate]

    def n_params(self) -> int:
        return 3 * sum(1 for g in self.gates if g.name == "u3")

    def angles(self) -> np.ndarray:
        """u3 angles as a flat float64 vector laid out [gate][a, b, c]."""
        out = [g.params for g in self.gates if g.name == "u3"]
        return np.asarray(out, dtype=np.float64).reshape(-1)


def grid_sites(rows: int, cols: int,
               removed: Sequence[Tuple[int, int]] = ()) -> Dict[Tuple[int, int], int]:
    """Map (r, c) -> qubit id, row-major over the kept sites."""
    rem = set(map(tuple, removed))
    sites = {}
    for r in range(rows):
        for c in range(cols):
            if (r, c) not in rem:
                sites[(r, c)] = len(sites)
    return sites


def coupler_pairs(rows: int, cols: int, letter: str,
                  removed: Sequence[Tuple[int, int]] = ()) -> List[Tuple[int, int]]:
    """Qubit pairs (q1 < q2) of coupler pattern A, B, C or D, sorted."""
    sites = grid_sites(rows, cols, removed)
    pairs = []
    for (r, c), q in sites.items():
        if letter in "AB":
            if c % 2 != (0 if letter == "A" else 1):
                continue
            other = (r, c + 1)
        elif letter in "CD":
            if r % 2 != (0 if letter == "C" else 1):
                continue
            other = (r + 1, c)
        else:
            raise ValueError(f"unknown coupler pattern {letter!r}")
        if other in sites:
            q2 = sites[other]
            pairs.append((min(q, q2), max(q, q2)))
    return sorted(pairs)


def make_rqc(rows: int, cols: int, cycles: int, seed: int = 0,
             removed: Sequence[Tuple[int, int]] = (),
             pattern: str = DEFAULT_PATTERN,
             u3_seed: Optional[int] = None) -> Circuit:
    """Draw one random circuit (see the module docstring for the rules)."""
    removed = tuple(tuple(x) for x in removed)
    sites = grid_sites(rows, cols, removed)
    n = len(sites)
    gates: List[Gate] = []
    if u3_seed is None:
        rng = np.random.default_rng(seed)
        prev = [-1] * n
    else:
        angles = np.random.default_rng(u3_seed).uniform(
            0.0, 2.0 * math.pi, size=(cycles, n, 3))
    pid = 0
    for cyc in range(cycles):
        for q in range(n):
            if u3_seed is None:
                if cyc == 0:
                    g = int(rng.integers(3))
                else:
                    choices = [x for x in range(3) if x != prev[q]]
                    g = choices[int(rng.integers(2))]
                prev[q] = g
                gates.append(Gate(SINGLE_QUBIT_SET[g], (q,)))
            else:
                a, b, c = (float(v) for v in angles[cyc, q])
                gates.append(Gate("u3", (q,), (a, b, c), pid))
                pid += 1
        letter = pattern[cyc % len(pattern)]
        for (q1, q2) in coupler_pairs(rows, cols, letter, removed):
            gates.append(Gate("fsim", (q1, q2), (FSIM_THETA, FSIM_PHI)))
    return Circuit(rows, cols, cycles, n, removed, pattern, gates)


def bits_of(x: int, n: int) -> List[int]:
    """Bits of basis index x, qubit 0 first (qubit 0 is the most significant)."""
    return [(x >> (n - 1 - q)) & 1 for q in range(n)]


def int_of_bits(bits: Sequence[int]) -> int:
    n = len(bits)
    return sum(int(b) << (n - 1 - q) for q, b in enumerate(bits))


def sample_bitstrings(n_bits: int, count: int, seed: int) -> np.ndarray:
    """``count`` distinct n-bit integers, uniform, without replacement."""
    rng = np.random.default_rng(seed)
    return np.asarray(rng.choice(1 << n_bits, size=count, replace=False),
                      dtype=np.int64)


def sample_slice_ids(n_sliced: int, count: int, seed: int) -> np.ndarray:
    """Sorted subset of slice ids in [0, 2**n_sliced); all ids if fewer.

    Slice ids are 64-bit: for more than 62 sliced indices the ids are drawn
    uniformly from [0, 2**62) (the higher sliced indices keep value 0)."""
    total = 1 << n_sliced
    if total <= count:
        return np.arange(total, dtype=np.uint64)
    rng = np.random.default_rng(seed)
    if n_sliced <= 62:
        ids = rng.choice(total, size=count, replace=False)
    else:
        ids = np.unique(rng.integers(0, 1 << 62, size=count, dtype=np.int64))
    return np.sort(np.asarray(ids, dtype=np.uint64))


@dataclass
class Workload:
    """A circuit plus what is asked of it.

    ``open_qubits``: qubits whose output index stays open (ascending; the
    first one is the most significant bit of the output vector).
    ``closed_bits``: dict qubit -> fixed output bit for the other qubits.
    ``slice_open``: the open indices are sliced too, one slice per output
    bitstring (used to evaluate a set of uncorrelated bitstrings).
    ``bitstrings``: for ``slice_open`` workloads, the requested bitstrings as
    integers over the open qubits (first open qubit most significant).
    ``max_rank``: target rank t of the slicing step (None = no cap).
    """
    name: str
    circuit: Circuit
    open_qubits: Tuple[int, ...]
    closed_bits: Dict[int, int]
    max_rank: Optional[int]
    slice_open: bool = False
    bitstrings: Optional[np.ndarray] = None
    slice_subset: Optional[int] = None
    slice_seed: int = 3
    meta: dict = field(default_factory=dict)


def _closed(n: int, open_qubits: Sequence[int], seed: int) -> Dict[int, int]:
    closed = [q for q in range(n) if q not in set(open_qubits)]
    bits = np.random.default_rng(seed).integers(0, 2, size=len(closed))
    return {q: int(b) for q, b in zip(closed, bits)}


def make_workload(name: str, **over) -> Workload:
    """Build one of the named workloads (keyword overrides for reduced sizes)."""
    spec = dict(WORKLOADS[name])
    spec.update(over)
    c = make_rqc(spec["rows"], spec["cols"], spec["cycles"],
                 seed=spec.get("seed", 0), removed=spec.get("removed", ()),
                 pattern=spec.get("pattern", DEFAULT_PATTERN),
                 u3_seed=spec.get("u3_seed"))
    n = c.n_qubits
    n_open = spec["n_open"]
    open_q = tuple(range(n - n_open, n))
    if spec.get("slice_open"):
        bs = sample_bitstrings(n_open, spec["n_bitstrings"], spec.get("bit_seed", 1))
        return Workload(name, c, open_q, {}, spec.get("max_rank"), True, bs)
    closed = _closed(n, open_q, spec.get("bit_seed", 1))
    return Workload(name, c, open_q, closed, spec.get("max_rank"),
                    slice_subset=spec.get("slice_subset"),
                    slice_seed=spec.get("slice_seed", 3))


# The five workloads (12-qubit parity case, 30-qubit throughput case and its
# split-precision twin, 20-qubit gradient case, 53-qubit Sycamore-shaped case).
WORKLOADS = {
    "rqc12": dict(rows=3, cols=4, cycles=8, n_open=0, max_rank=None),
    "rqc30": dict(rows=5, cols=6, cycles=14, n_open=6, max_rank=26),
    "rqc20_grad": dict(rows=4, cols=5, cycles=12, n_open=20, max_rank=None,
                       u3_seed=2, slice_open=True, n_bitstrings=256),
    "rqc53": dict(rows=6, cols=9, cycles=20, removed=((5, 8),), n_open=20,
                  max_rank=30, slice_subset=1024),
}
