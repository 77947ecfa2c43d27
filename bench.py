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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mode", default="c64", choices=["c64", "split_f16", "split_bf16"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--tune-cache", default=None)
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
    w = make_workload("rqc30")
    t0 = time.perf_counter()
    pr = P.prepare(w)
    plan = pr.plan()
    costs = P.tree_costs(pr.net, pr.path, pr.sliced)
    t_plan = time.perf_counter() - t0
    n_slices = 1 << len(pr.sliced)
    info = plan.info()
    macs_slice = info["macs_per_slice"]
    flops_step = 8.0 * macs_slice * n_slices
    log(f"planned in {t_plan:.2f}s: |S|={len(pr.sliced)} C(B,S)=2^{costs.log2_sliced:.2f} "
        f"overhead={costs.overhead:.4f} per-slice MACs={macs_slice:.3e}")

    batch = plan.bind(batch=n_slices) if plan.workspace_size(n_slices) < 0.7 * torch.cuda.mem_get_info()[0] \
        else plan.bind()
    log(f"bound: batch={batch}, workspace={plan.workspace_size(batch) / 2**30:.2f} GiB")
    t0 = time.perf_counter()
    plan.autotune(args.mode, args.tune_cache)
    log(f"autotuned in {time.perf_counter() - t0:.2f}s")

    out = plan.new_output()
    for _ in range(args.warmup):
        out.zero_()
        plan.execute_range(0, n_slices, out, args.mode)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out.zero_()
        plan.execute_range(0, n_slices, out, args.mode)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = 1e3 * dt / args.steps
    tflops = flops_step * args.steps / dt / 1e12
    log(f"{args.steps} steps in {dt:.3f}s: {ms_step:.2f} ms/step, {tflops:.2f} TFLOP/s")

    err = None
    if os.path.exists(GOLDEN):
        ref = np.load(GOLDEN)
        got = out.cpu().numpy()
        err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        log(f"relative L2 error vs the oracle's complex128 amplitudes: {err:.3e}")

    # roofline of the dominant kernel (the MFMA complex GEMM), from live
    # per-step HIP events on the plan's stream (replay outside the graph)
    steps = plan.steps()
    ms = np.zeros(len(steps))
    reps = 3
    for _ in range(reps):
        ms += plan.profile_steps(0, args.mode)
    ms /= reps
    nb = batch
    mf_flops, mf_ms, mf_launch = 0.0, 0.0, 0
    for k, st in enumerate(steps):
        kind, _, _, _ = plan.step_kernel(k, args.mode)
        if kind > 0:
            mf_flops += 8.0 * (1 << (st["m"] + st["k"] + st["n"])) * nb
            mf_ms += ms[k]
            mf_launch += 1
    total_ms = float(ms.sum())
    peak = PEAK_FP32_MFMA_TFLOPS if args.mode == "c64" else PEAK_F16_MFMA_TFLOPS
    achieved = mf_flops / (mf_ms * 1e-3) / 1e12 if mf_ms > 0 else 0.0
    log(f"MFMA steps: {mf_launch} launches/batch, {mf_ms:.2f} of {total_ms:.2f} ms per batch, "
        f"{achieved:.2f} TFLOP/s")
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": counter_traffic(args.mode),
                "kernel": "k_cgemm_c64", "launches_per_batch": mf_launch,
                "share_of_step_time": round(mf_ms / total_ms, 4) if total_ms else None}

    cpu = None
    if not args.no_cpu:
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
        "dtype": "c64" if args.mode == "c64" else ("f16x2" if args.mode == "split_f16" else "bf16x2"),
        "data": "synthetic",
        "config": {"workload": "rqc30: 5x6 grid, 14 cycles, 6 open qubits (64 amplitudes), "
                               "max rank 26, all slices per step",
                   "slices": n_slices, "sliced_indices": len(pr.sliced), "batch": batch,
                   "log2_C_BS": round(costs.log2_sliced, 4), "overhead": round(costs.overhead, 5),
                   "macs_per_slice": macs_slice, "flops_per_step": flops_step,
                   "mode": args.mode},
        "sec_per_slice": dt / args.steps / n_slices,
        "rel_l2_error": err,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
