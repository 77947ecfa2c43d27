"""Write oracle references for sampled slices of the 53-qubit workload.

Calls only the oracle and the seeded workload generator: the oracle's own
path search (randomised greedy, same rule and grid as the library's
default), its slice finder at t = 30, and, for each of the first N slice
ids of the seeded subset (seed 3), the plain tensordot contraction of that
slice in complex128, sub-sliced at t = 29 to fit host memory (the extra
sub-slice indices are summed over; sliced open indices are placed).
Stores, per slice, 2^16 amplitudes at seeded output positions (seed 5) and
the squared norm of the whole 2^20-amplitude block.

Usage: python tests/golden/make_rqc53_reference.py [N] [OUTDIR] [--reconf K] [--t-sub T]
At the default t = 29 for the sub-slices (16 sub-slices of the greedy
plan's slices) it needs ~40 GiB of host memory and ~20 minutes per slice
on 8 cores.

With --reconf K every greedy trial is improved by the oracle's subtree
reconfiguration (frontiers of K tensors, 4 sweeps) as in the library's
search, and the files are named rqc53_reconf_slices.*.
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
from workload import make_workload, sample_slice_ids  # noqa: E402

ALPHAS, TAUS, SEEDS = (0.5, 1.0, 2.0), (0.0, 0.3, 1.0), 16
T_SUB = 29
N_POS = 1 << 16


def main():
    args = [a for a in sys.argv[1:] if not a.startswith("--")]
    reconf, t_sub = 0, T_SUB
    if "--reconf" in sys.argv:
        reconf = int(sys.argv[sys.argv.index("--reconf") + 1])
        args = [a for a in args if a != str(reconf)]
    if "--t-sub" in sys.argv:
        t_sub = int(sys.argv[sys.argv.index("--t-sub") + 1])
        args = [a for a in args if a != str(t_sub)]
    n_slices = int(args[0]) if len(args) > 0 else 1
    outdir = args[1] if len(args) > 1 else HERE
    w = make_workload("rqc53")
    net = nw.absorb_small(nw.circuit_network(w.circuit, w.open_qubits, w.closed_bits))
    t0 = time.time()
    path, S, trial = pl.path_search(net.indices, w.max_rank, (), ALPHAS, TAUS, SEEDS,
                                    reconf_k=reconf, reconf_sweeps=4)
    tree = pl.Tree(net.indices, path)
    print(f"path search {time.time() - t0:.1f}s trial {trial} |S|={len(S)}", flush=True)
    S2 = pl.slice_finder(tree, t_sub, pre=S)
    extra = S2[len(S):]
    print(f"sub-slicing at t={t_sub}: {len(extra)} extra indices", flush=True)
    ids = [int(x) for x in sample_slice_ids(len(S), 1024, 3)[:n_slices]]
    pos = np.sort(np.random.default_rng(5).choice(1 << len(net.open_ids), N_POS, replace=False))
    rec = dict(workload="rqc53", trial=trial, sliced=[int(x) for x in S], extra=[int(x) for x in extra],
               t_sub=t_sub, path=[[int(a), int(b)] for a, b in path], path_sha256=hashlib.sha256(np.asarray(path, dtype=np.int32).tobytes()).hexdigest(),
               slices=[])
    amps = []
    for s in ids:
        out = np.zeros(1 << len(net.open_ids), dtype=np.complex128)
        t1 = time.time()
        for e in range(1 << len(extra)):
            s2 = s | (e << len(S))
            blk = nw.slice_output(net, path, S2, s2)
            out[nw.place(net, S2, s2, blk)] += blk
            print(f"slice {s} sub-slice {e} {time.time() - t1:.1f}s", flush=True)
        rec["slices"].append(dict(id=str(s), norm2=float(np.sum(np.abs(out) ** 2))))
        amps.append(out[pos])
    stem = "rqc53_reconf_slices" if reconf else "rqc53_slices"
    rec["reconf_k"] = reconf
    np.savez(os.path.join(outdir, stem + ".npz"), positions=pos, amplitudes=np.asarray(amps))
    json.dump(rec, open(os.path.join(outdir, stem + ".json"), "w"), indent=1)
    print(json.dumps(rec)[:400], flush=True)


if __name__ == "__main__":
    main()
