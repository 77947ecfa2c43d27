"""Host diagnostics (stem cost profile, overhead vs target rank) run through
libltn and stay consistent with the planner's own numbers."""
import paper_2205_00393_amd as P
from paper_2205_00393_amd import report


def test_report_rqc12_and_rqc30():
    rep = report.main(["rqc12", "--json", "--ts", "4,5,6"])
    stem = rep["stem"]
    assert stem[0]["log2_node_cost"] is None            # a leaf starts the stem
    assert all(r["log2_node_cost"] is not None for r in stem[1:])
    assert all(r["rank_sliced"] <= r["rank"] for r in stem)
    for row in rep["overhead_vs_t"]:
        assert row["alg1_refined"]["overhead"] <= row["alg1"]["overhead"] + 1e-12
        assert row["alg1_refined"]["n_sliced"] <= row["alg1"]["n_sliced"]
        assert row["alg1"]["overhead"] >= 1.0 - 1e-12 and row["greedy_overhead"]["overhead"] >= 1.0 - 1e-12
    rep = report.main(["rqc30", "--json", "--ts", "26", "--reconf", "6"])
    assert rep["overhead_vs_t"][0]["t"] == 26
    pr = P.prepare(__import__("workload").make_workload("rqc30"), reconf_k=6)
    assert abs(rep["costs"]["log2_C_BS"] - P.tree_costs(pr.net, pr.path, pr.sliced).log2_sliced) < 1e-12
    # the stem's largest sliced tensor respects the cap
    assert max(r["rank_sliced"] for r in rep["stem"]) <= 26
