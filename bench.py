"""Benchmark: sliced contraction of the 30-qubit random circuit on one GPU.

One step = the whole hot path over every slice of the workload (leaf
gather, all contraction steps, FP64 slice sum) into a zeroed output.
Prints one JSON line (see the keys below). Inputs are synthetic (seeded
circuit); the host planner runs before the timed region.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_MFMA_TFLOPS = 157.3   # MI355X dense FP32 matrix
PEAK_F16_MFMA_TFLOPS = 2516.6   # MI355X dense FP16 / BF16 matrix
PEAK_HBM_GBS = 8000.0
GOLDEN = os.path.join(ROOT, "tests", "golden", "rqc30_amplitudes.npy")


def counter_traffic(mode):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary, or None when the kernel source has changed
    since the counters were taken (or no summary exists for this mode)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"k_cgemm_{'c64' if mode == 'c64' else 'split'}__rqc30_{mode}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = open(os.path.join(ROOT, "paper_2205_00393_amd", "csrc", "k_mfma.hip"), "rb").read()
    if hashlib.sha256(src).hexdigest() != rec.get("source_sha256"):
        return None
    return rec["traffic_bytes_per_launch"]


def sig6(v):
    """Six significant digits (small errors stay visible)."""
    return float(f"{v:.6g}") if isinstance(v, float) else v


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(budget_s=30.0):
    """The oracle (numpy complex128 tensordot) contracting slice 0 of the
    same workload along its own path and slicing set."""
    from oracle import network as onw, planner as opl
    from workload import make_workload
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = len(os.sched_getaffinity(0))
    w = make_workload("rqc30")
    net = onw.absorb_small(onw.circuit_network(w.circuit, w.open_qubits, w.closed_bits))
    path, S, _ = opl.path_search(net.indices, w.max_rank, (), (0.5, 1.0, 2.0), (0.0, 0.3, 1.0), 16)
    tree = opl.Tree(net.indices, path)
    macs = tree.sliced_cost(S) >> len(S)
    t0 = time.perf_counter()
    onw.slice_output(net, path, S, 0)
    dt = time.perf_counter() - t0
    return {"value": 8.0 * macs / dt / 1e12, "unit": "TFLOP/s", "cores": int(threads),
            "kind": "oracle", "sec_per_slice": dt,
            "sample": f"1 of {1 << len(S)} slices of rqc30 (slice 0, {macs:.3e} complex MACs), "
                      "numpy complex128 tensordot along the oracle's own path"}


def gradient_leg(torch, P, args):
    """Forward + adjoint of the 20-qubit u3 workload (720 angles, loss over
    256 bitstrings, each one slice), timed with the same warm-up / step
    counts, checked against the stored oracle adjoint gradient."""
    from paper_2205_00393_amd.autograd import Amplitudes
    from workload import make_workload
    w = make_workload("rqc20_grad")
    pr = P.prepare(w, alphas=(0.5, 1.0), taus=(0.0, 0.3), n_seeds=3)
    plan = pr.plan()
    batch = plan.bind(batch=0, grad=True, budget_bytes=8 << 30)
    plan.autotune("c64", args.tune_cache)  # forward kernels (the adjoint follows fixed rules)
    ids = [pr.slice_of_bitstring(int(x)) for x in w.bitstrings]
    sel = torch.as_tensor(np.asarray(w.bitstrings), device="cuda")
    angles0 = torch.tensor(w.circuit.angles(), dtype=torch.float64, device="cuda")

    def step():
        angles = angles0.clone().requires_grad_(True)
        out = Amplitudes.apply(angles, plan, ids)
        loss = torch.sum(torch.log(torch.abs(out[sel]) ** 2))
        loss.backward()
        return angles.grad
    for _ in range(max(1, args.warmup)):
        g = step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    res = {"workload": "rqc20_grad: 4x5 grid, 12 cycles, u3 gates (720 angles), "
                       "loss over 256 bitstrings (one slice each)",
           "batch": batch, "ms_fwd_bwd": sig6(dt * 1e3),
           "ms_per_bitstring": sig6(dt * 1e3 / len(ids))}
    ref_path = os.path.join(ROOT, "tests", "golden", "rqc20_grad_reference.npz")
    if os.path.exists(ref_path):
        ref = np.load(ref_path)
        gg = g.detach().cpu().numpy()
        res["grad_rel_l2_error"] = sig6(float(np.linalg.norm(gg - ref["grad"]) / np.linalg.norm(ref["grad"])))
    log(f"gradient: {res['ms_fwd_bwd']:.2f} ms forward + backward, error {res.get('grad_rel_l2_error')}")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--modes", default="c64,split_f16,split_bf16",
                    help="comma list; the first is the headline value, the others are reported beside it")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--tune-cache", default=None, help="autotuner cache (JSON, keyed by mode and step shape)")
    ap.add_argument("--workload", default="rqc30", choices=["rqc30", "rqc53"],
                    help="rqc30: every slice per step; rqc53: a seeded sample of --slices slices")
    ap.add_argument("--slices", type=int, default=8, help="rqc53: sampled slices per step")
    ap.add_argument("--path", default="greedy", choices=["greedy", "reconf"],
                    help="path of the headline plan: randomised greedy (the workload's definition) "
                         "or greedy + subtree reconfiguration")
    ap.add_argument("--reconf-k", type=int, default=None,
                    help="subtree reconfiguration window (default: 10 for rqc30, 8 for rqc53)")
    ap.add_argument("--path-variant", default="c64,split_bf16",
                    help="modes to time on the reconfigured path as well ('' to skip)")
    ap.add_argument("--no-grad", action="store_true",
                    help="skip the gradient leg (20-qubit, 720 angles, 256 bitstrings)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration) and exit")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        n = args.copy_probe << 20
        x = torch.ones(n, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); slices are "
              "independent, so more GPUs would each take a share of the slice range.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2205_00393_amd as P
    from workload import make_workload

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    from workload import sample_slice_ids
    w = make_workload(args.workload)
    ref = np.load(GOLDEN) if os.path.exists(GOLDEN) else None

    def run_plan(pr, mode_list, tag, fuse_rank=0):
        """Bind a prepared plan and time each mode on it; returns (results,
        plan facts)."""
        t0 = time.perf_counter()
        plan = pr.plan(fuse_rank=fuse_rank)
        costs = P.tree_costs(pr.net, pr.path, pr.sliced)
        t_plan = time.perf_counter() - t0 + pr_seconds[tag]
        if args.workload == "rqc30":
            n_slices = 1 << len(pr.sliced)
            ids = None
        else:
            # the seeded subset of 2^10 slice ids, first --slices of them
            ids = sample_slice_ids(len(pr.sliced), 1024, 3)[: args.slices]
            n_slices = len(ids)
        info = plan.info()
        macs_slice = info["macs_per_slice"]
        flops_step = 8.0 * macs_slice * n_slices
        steps = plan.steps()
        log(f"[{tag}] planned in {t_plan:.2f}s: |S|={len(pr.sliced)} C(B,S)=2^{costs.log2_sliced:.2f} "
            f"overhead={costs.overhead:.4f} per-slice MACs={macs_slice:.3e}")
        batch = plan.bind(batch=n_slices) if plan.workspace_size(n_slices) < 0.7 * torch.cuda.mem_get_info()[0] \
            else plan.bind()
        log(f"[{tag}] bound: batch={batch}, workspace={plan.workspace_size(batch) / 2**30:.2f} GiB")

        def run_step(out, mode):
            if ids is None:
                plan.execute_range(0, n_slices, out, mode)
            else:
                plan.execute(ids, out, mode)

        def measure(mode):
            t0 = time.perf_counter()
            cache = args.tune_cache  # one file for all modes (keys carry the mode)
            plan.autotune(mode, cache)
            log(f"[{tag}/{mode}] autotuned in {time.perf_counter() - t0:.2f}s")
            out = plan.new_output()
            for _ in range(args.warmup):
                out.zero_()
                run_step(out, mode)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                out.zero_()
                run_step(out, mode)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            res = {"tflops": flops_step * args.steps / dt / 1e12, "ms_per_step": 1e3 * dt / args.steps,
                   "sec_per_slice": dt / args.steps / n_slices}
            if ref is not None and args.workload == "rqc30":
                got = out.cpu().numpy()
                res["rel_l2_error"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
            # the dominant kernel (the MFMA complex GEMM): live per-step HIP
            # events on the plan's stream (a replay of one batch outside the graph)
            ms = np.zeros(len(steps))
            reps = 3
            for _ in range(reps):
                ms += plan.profile_steps(0 if ids is None else int(ids[0]), mode)
            ms /= reps
            mf_flops, mf_ms, mf_launch, split_flops = 0.0, 0.0, 0, 0.0
            for k, st in enumerate(steps):
                kind, _, _, _ = plan.step_kernel(k, mode)
                if kind in (1, 2):
                    f = 8.0 * (1 << (st["m"] + st["k"] + st["n"])) * batch
                    mf_flops += f
                    mf_ms += ms[k]
                    mf_launch += 1
                    if kind == 2:
                        split_flops += f
            res["mfma_ms_per_batch"] = mf_ms
            res["step_ms_per_batch"] = float(ms.sum())
            res["mfma_launches_per_batch"] = mf_launch
            res["mfma_tflops"] = mf_flops / (mf_ms * 1e-3) / 1e12 if mf_ms > 0 else 0.0
            res["split_mac_fraction"] = split_flops / (8.0 * macs_slice * batch)
            log(f"[{tag}/{mode}] {res['ms_per_step']:.2f} ms/step, {res['tflops']:.2f} TFLOP/s, "
                f"MFMA {mf_ms:.2f} of {res['step_ms_per_batch']:.2f} ms per batch "
                f"({res['mfma_tflops']:.2f} TFLOP/s), err {res.get('rel_l2_error')}")
            return res

        results = {m: measure(m) for m in mode_list}
        facts = dict(n_slices=n_slices, batch=batch, costs=costs, macs_slice=macs_slice,
                     flops_step=flops_step, n_sliced=len(pr.sliced), plan_seconds=t_plan,
                     groups=plan.groups())
        del plan
        torch.cuda.empty_cache()
        return results, facts

    pr_seconds = {}
    reconf_k = args.reconf_k if args.reconf_k is not None else (10 if args.workload == "rqc30" else 8)
    t0 = time.perf_counter()
    pr = P.prepare(w, reconf_k=reconf_k if args.path == "reconf" else 0)
    pr_seconds[args.path] = time.perf_counter() - t0
    results, facts = run_plan(pr, args.modes.split(","), args.path)
    n_slices, batch, costs = facts["n_slices"], facts["batch"], facts["costs"]
    macs_slice, flops_step = facts["macs_slice"], facts["flops_step"]

    # the same workload on a better path: greedy trials improved by subtree
    # reconfiguration
    variant = None
    if args.path_variant and args.path == "greedy":
        t0 = time.perf_counter()
        prv = P.prepare(w, reconf_k=reconf_k)
        pr_seconds["reconf"] = time.perf_counter() - t0
        vres, vf = run_plan(prv, args.path_variant.split(","), "reconf")
        variant = {"path": f"randomised greedy + subtree reconfiguration (k={reconf_k})",
                   "plan_seconds": round(vf["plan_seconds"], 3),
                   "sliced_indices": vf["n_sliced"], "log2_C_BS": round(vf["costs"].log2_sliced, 4),
                   "overhead": round(vf["costs"].overhead, 5), "macs_per_slice": vf["macs_slice"],
                   "projected_seconds_all_slices": {m: r["sec_per_slice"] * 2.0 ** vf["n_sliced"]
                                                    for m, r in vres.items()},
                   "modes": {m: {k: sig6(v) for k, v in r.items()} for m, r in vres.items()}}
        if args.workload == "rqc30":
            # the same path with fused sub-paths (secondary slicing, working rank 10)
            pr_seconds["reconf+fused"] = pr_seconds["reconf"]
            fres, ff = run_plan(prv, ["c64"], "reconf+fused", fuse_rank=10)
            variant["fused_sub_paths"] = {
                "fuse_rank": 10, "groups": len(ff["groups"]),
                "steps_fused": sum(g["n_steps"] for g in ff["groups"]),
                "c64": {k: sig6(v) for k, v in fres["c64"].items()}}
        for m, r in vres.items():
            if m in results:
                variant["modes"][m]["time_to_solution_speedup_vs_greedy_path"] = round(
                    (results[m]["sec_per_slice"] * 2.0 ** len(pr.sliced)) /
                    (r["sec_per_slice"] * 2.0 ** vf["n_sliced"]), 3)

    main_mode = args.modes.split(",")[0]
    r0 = results[main_mode]
    tflops, ms_step, err = r0["tflops"], r0["ms_per_step"], r0.get("rel_l2_error")
    if main_mode == "c64":
        peak, achieved = PEAK_FP32_MFMA_TFLOPS, r0["mfma_tflops"]
    else:
        # split: three fp16/bf16 matrix products per real product; executed
        # matrix flops are 3x the algorithmic count
        peak, achieved = PEAK_F16_MFMA_TFLOPS, 3.0 * r0["mfma_tflops"]
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": counter_traffic(main_mode),
                "kernel": "k_cgemm_c64" if main_mode == "c64" else "k_cgemm_split",
                "launches_per_batch": r0["mfma_launches_per_batch"],
                "share_of_step_time": round(r0["mfma_ms_per_batch"] / r0["step_ms_per_batch"], 4)}
    modes = {}
    for m, r in results.items():
        modes[m] = {k: sig6(v) for k, v in r.items()}
        modes[m]["speedup_vs_c64"] = round(r["tflops"] / results["c64"]["tflops"], 4) if "c64" in results else None
        modes[m]["meets_tolerance"] = (r.get("rel_l2_error") is not None and
                                       r["rel_l2_error"] <= (1e-4 if m == "c64" else 5e-4))

    grad = None
    if not args.no_grad and args.workload == "rqc30":
        grad = gradient_leg(torch, P, args)

    cpu = None
    if not args.no_cpu and args.workload == "rqc30":
        log("timing the CPU oracle on one slice ...")
        cpu = cpu_baseline()
        log(f"oracle: {cpu['sec_per_slice']:.2f} s/slice, {cpu['value']:.4f} TFLOP/s on "
            f"{cpu['cores']} threads")

    line = {
        "metric": "contraction TFLOP/s + sec/slice on 1 GPU; split-FP16 vs complex64 at stated error",
        "value": round(tflops, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"c64": "c64", "split_f16": "f16x2", "split_bf16": "bf16x2"}[main_mode],
        "data": "synthetic",
        "config": {"workload": ("rqc30: 5x6 grid, 14 cycles, 6 open qubits (64 amplitudes), "
                                "max rank 26, all slices per step") if args.workload == "rqc30" else
                               (f"rqc53: 6x9 grid minus one site, 20 cycles, 20 open qubits (2^20 "
                                f"amplitudes), max rank 30, {n_slices} seeded slices per step"),
                   "projected_seconds_all_slices": r0["sec_per_slice"] * 2.0 ** len(pr.sliced),
                   "slices": n_slices, "sliced_indices": len(pr.sliced), "batch": batch,
                   "log2_C_BS": round(costs.log2_sliced, 4), "overhead": round(costs.overhead, 5),
                   "macs_per_slice": macs_slice, "flops_per_step": flops_step,
                   "mode": main_mode, "path": args.path},
        "sec_per_slice": r0["sec_per_slice"],
        "rel_l2_error": err,
        "modes": modes,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "path_variant": variant,
        "gradient": grad,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
