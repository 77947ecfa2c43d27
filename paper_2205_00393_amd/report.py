"""Host-side diagnostics of a contraction tree and its slicing sets: the
cost profile along the stem (the most computationally intensive root-to-leaf
path, Sec. 4.2) and the slicing overhead O(B,S) = C(B,S) / C(B) (Eq. 2) as a
function of the target rank t for the slice finder (Algorithm 1), the
finder followed by the refiner (Algorithms 2-4) and the greedy
least-overhead slicer. Everything is computed by libltn.

    python -m paper_2205_00393_amd.report rqc30 [--reconf 8] [--ts 22,24,26]
"""
from __future__ import annotations

import argparse
import json
from typing import Dict, List, Sequence

from .network import (Network, slice_finder, slice_greedy_overhead, slice_refine, stem_profile,
                      tree_costs)


def overhead_vs_t(net: Network, path, ts: Sequence[int], pre: Sequence[int] = (),
                  refine_seeds: int = 2) -> List[Dict]:
    """|S| and O(B,S) at each target t for three slicing strategies."""
    out = []
    for t in ts:
        row = {"t": t}
        S1 = slice_finder(net, path, t, pre)
        c1 = tree_costs(net, path, S1)
        row["alg1"] = {"n_sliced": len(S1), "overhead": c1.overhead, "log2_C_BS": c1.log2_sliced}
        best = None
        for sd in range(refine_seeds):
            R, _ = slice_refine(net, path, t, S1, n_fixed=len(pre), seed=sd)
            cr = tree_costs(net, path, R)
            if best is None or (cr.sliced, len(R)) < (best[0].sliced, len(best[1])):
                best = (cr, R)
        row["alg1_refined"] = {"n_sliced": len(best[1]), "overhead": best[0].overhead,
                               "log2_C_BS": best[0].log2_sliced}
        G = slice_greedy_overhead(net, path, t, pre)
        cg = tree_costs(net, path, G)
        row["greedy_overhead"] = {"n_sliced": len(G), "overhead": cg.overhead,
                                  "log2_C_BS": cg.log2_sliced}
        out.append(row)
    return out


def main(argv=None):
    from workload import make_workload
    from .plan import prepare
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("workload")
    ap.add_argument("--reconf", type=int, default=0, help="subtree reconfiguration k (0: off)")
    ap.add_argument("--ts", default="", help="comma list of target ranks (default: t-4..t+2)")
    ap.add_argument("--json", action="store_true")
    a = ap.parse_args(argv)
    w = make_workload(a.workload)
    pr = prepare(w, reconf_k=a.reconf)
    t0 = w.max_rank if w.max_rank is not None else max(len(ix) for ix in pr.net.indices) + 4
    ts = [int(x) for x in a.ts.split(",")] if a.ts else list(range(max(1, t0 - 4), t0 + 3))
    rep = {"workload": a.workload, "reconf_k": a.reconf, "sliced": len(pr.sliced),
           "costs": {"log2_C_B": tree_costs(pr.net, pr.path, []).log2_cost,
                     "log2_C_BS": tree_costs(pr.net, pr.path, pr.sliced).log2_sliced},
           "stem": stem_profile(pr.net, pr.path, pr.sliced),
           "overhead_vs_t": overhead_vs_t(pr.net, pr.path, ts, pr.pre)}
    if a.json:
        print(json.dumps(rep))
        return rep
    print(f"{a.workload}: |S| = {rep['sliced']}, log2 C(B) = {rep['costs']['log2_C_B']:.2f}, "
          f"log2 C(B,S) = {rep['costs']['log2_C_BS']:.2f}")
    print("stem (leaf -> root): tensor rank / rank after S / log2 node cost")
    for r in rep["stem"]:
        c = "-" if r["log2_node_cost"] is None else str(r["log2_node_cost"])
        print(f"  {r['tensor']:6d} {r['rank']:4d} {r['rank_sliced']:4d} {c:>5s}")
    print("overhead O(B,S) vs target rank t: |S| / O for Algorithm 1, + refiner, greedy slicer")
    for r in rep["overhead_vs_t"]:
        f = lambda k: f"{r[k]['n_sliced']:3d} / {r[k]['overhead']:.4g}"
        print(f"  t = {r['t']:3d}: {f('alg1'):>16s} {f('alg1_refined'):>16s} {f('greedy_overhead'):>16s}")
    return rep


if __name__ == "__main__":
    main()
