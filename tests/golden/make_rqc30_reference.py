"""Write the complex128 reference amplitudes of the 30-qubit workload.

Calls only the oracle and the seeded workload generator: the oracle's own
path search (randomised greedy, same rule and grid as the library's
default), its slice finder at t = 26, and its plain tensordot contraction of
every slice, summed. Output: rqc30_amplitudes.npy (64 complex128 values,
first open qubit most significant) and rqc30_amplitudes.json (metadata).
Takes tens of minutes on 8 cores.
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import network as nw  # noqa: E402
from oracle import planner as pl  # noqa: E402
from workload import make_workload  # noqa: E402

ALPHAS, TAUS, SEEDS = (0.5, 1.0, 2.0), (0.0, 0.3, 1.0), 16


def main():
    w = make_workload("rqc30")
    net = nw.absorb_small(nw.circuit_network(w.circuit, w.open_qubits, w.closed_bits))
    t0 = time.time()
    path, S, trial = pl.path_search(net.indices, w.max_rank, (), ALPHAS, TAUS, SEEDS)
    tree = pl.Tree(net.indices, path)
    print(f"path search {time.time() - t0:.1f}s trial {trial} |S|={len(S)} "
          f"C(B,S)=2^{np.log2(float(tree.sliced_cost(S))):.2f}", flush=True)
    out = np.zeros(1 << len(net.open_ids), dtype=np.complex128)
    for s in range(1 << len(S)):
        t1 = time.time()
        blk = nw.slice_output(net, path, S, s)
        out[nw.place(net, S, s, blk)] += blk
        print(f"slice {s} {time.time() - t1:.1f}s", flush=True)
    np.save(os.path.join(HERE, "rqc30_amplitudes.npy"), out)
    meta = dict(workload="rqc30", trial=trial, sliced=[int(x) for x in S],
                path_sha256=hashlib.sha256(np.asarray(path, dtype=np.int32).tobytes()).hexdigest(),
                norm2=float(np.sum(np.abs(out) ** 2)), seconds=time.time() - t0)
    json.dump(meta, open(os.path.join(HERE, "rqc30_amplitudes.json"), "w"), indent=1)
    print(meta)


if __name__ == "__main__":
    main()
