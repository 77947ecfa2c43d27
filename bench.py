"""Benchmark: sliced contraction of random quantum circuits on one GPU.

Headline workload (default): the 53-qubit circuit (6x9 grid minus one
site, 20 cycles, 2^20 open amplitudes) on its randomised greedy path,
sliced by Algorithm 1 under rank 30. One step = the whole hot path (leaf
gather, every contraction step, FP64 slice sum) over one batch of slices
taken in order from the seeded subset of 1024 slice ids; successive steps
walk the subset. complex64 is the headline; split fp16 and split bf16 are
timed beside it; each mode states its error on the stored oracle slices.

Extra keys: path_variant (the same circuit on the greedy trials improved
by subtree reconfiguration, errors on its own two stored oracle slices),
the 30-qubit workload (every slice per step, greedy and reconfigured
paths, fused sub-paths), the 20-qubit gradient workload, and CPU oracle
timings of each.

Prints one JSON line. Inputs are synthetic (seeded circuits); the host
planner runs before the timed regions.
"""
import argparse
import hashlib
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
GOLDEN = os.path.join(ROOT, "tests", "golden")
TOL = {"c64": 1e-4, "split_f16": 5e-4, "split_bf16": 5e-4}
WORKLOAD_TEXT = {
    "rqc53": "rqc53: 6x9 grid minus site (5,8), 20 cycles, 20 open qubits (2^20 amplitudes), max rank 30",
    "rqc30": "rqc30: 5x6 grid, 14 cycles, 6 open qubits (64 amplitudes), max rank 26",
}


# source file of each profiled kernel family (its hash marks the counters stale)
KERNEL_SOURCE = {"k_cgemm_c64": "k_mfma.hip", "k_cgemm_split": "k_mfma.hip", "k_narrow": "k_narrow.hip"}


def counter_traffic(workload, mode):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary for this workload and mode, or None when there
    is none or the kernel source has changed since the counters were taken."""
    kern = "k_cgemm_c64" if mode == "c64" else "k_cgemm_split"
    path = os.path.join(ROOT, "profiles", f"{kern}__{workload}_{mode}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = open(os.path.join(ROOT, "paper_2205_00393_amd", "csrc", "k_mfma.hip"), "rb").read()
    if hashlib.sha256(src).hexdigest() != rec.get("source_sha256"):
        return None
    return rec["traffic_bytes_per_launch"]


def step_roofline(kind, tile, m, k, n, batch):
    """Algorithmic flops, executed matrix flops, algorithmic bytes of one
    matrix-core step (kind 1/5 complex64 tiles, kind 2 split tiles) over a
    batch, and whether it is GEMM-bound: executed flops per algorithmic byte
    at or above the ridge of its matrix peak and the 8 TB/s HBM peak.
    Executed flops per complex MAC: 8 on direct complex64 tiles, 6 on the
    three-product ones (names with _3m_), 24 on split tiles."""
    f = 8.0 * (1 << (m + k + n)) * batch
    fx = f * (3.0 if kind == 2 else (0.75 if "_3m_" in tile else 1.0))
    by = 8.0 * ((1 << (m + k)) + (1 << (n + k)) + (1 << (m + n))) * batch
    peak = PEAK_F16_MFMA_TFLOPS if kind == 2 else PEAK_FP32_MFMA_TFLOPS
    return f, fx, by, fx / by >= peak / PEAK_HBM_GBS * 1e3


def sig6(v):
    """Six significant digits (small errors stay visible)."""
    return float(f"{v:.6g}") if isinstance(v, float) else v


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_cpu():
    """CPU model and the cores this process may run on."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    cores = len(os.sched_getaffinity(0))
    try:
        from threadpoolctl import threadpool_info
        blas = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        blas = None
    return model, cores, blas


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# ---------------------------------------------------------------- CPU oracle
def cpu_rqc53(S, t_cpu=27, budget_s=20.0):
    """The oracle contracting sub-slices of one sampled slice of the 53-qubit
    workload (complex128 tensordot), as many as fit in ``budget_s``, along
    the oracle's own path (its path search takes minutes in Python, so the
    path is the one the reference script stored, searched by the oracle).
    The slice is cut further at rank ``t_cpu`` so that one sub-slice takes
    seconds."""
    from oracle import network as onw, planner as opl
    from workload import make_workload
    meta_path = os.path.join(GOLDEN, "rqc53_slices.json")
    if not os.path.exists(meta_path):
        return None
    meta = json.load(open(meta_path))
    if "path" not in meta or list(S) != meta["sliced"]:
        log("cpu baseline: no stored oracle path for this slicing set; skipped")
        return None
    path = [tuple(p) for p in meta["path"]]
    w = make_workload("rqc53")
    net = onw.absorb_small(onw.circuit_network(w.circuit, w.open_qubits, w.closed_bits))
    tree = opl.Tree(net.indices, path)
    S2 = opl.slice_finder(tree, t_cpu, pre=meta["sliced"])
    n_sub = 1 << (len(S2) - len(S))
    macs_sub = tree.sliced_cost(S2) >> len(S2)
    macs_slice = tree.sliced_cost(S) >> len(S)
    s = int(meta["slices"][0]["id"])
    model, cores, blas = host_cpu()
    t0 = time.perf_counter()
    done = 0
    while done < n_sub and (done == 0 or time.perf_counter() - t0 < budget_s):
        onw.slice_output(net, path, S2, s | (done << len(S)))
        done += 1
    dt = time.perf_counter() - t0
    rate = 8.0 * macs_sub * done / dt
    return {"value": rate / 1e12, "unit": "TFLOP/s", "cores": cores,
            "blas_threads": blas, "cpu_model": model, "kind": "oracle",
            "sec_per_slice": 8.0 * macs_slice / rate,
            "sec_per_slice_as_subsliced": dt / done * n_sub,
            "sample": (f"{done} of the {n_sub} sub-slices (rank cap {t_cpu}) of slice {s} of rqc53, "
                       f"{macs_sub:.3e} complex MACs each, numpy complex128 tensordot along the "
                       f"oracle's path; sec_per_slice = one slice's {macs_slice:.3e} MACs at that "
                       "rate, sec_per_slice_as_subsliced = all sub-slices of the slice at that "
                       "rate (cutting at rank 27 adds work)")}


def cpu_rqc30(budget_s=30.0):
    """The oracle contracting slice 0 of the 30-qubit workload along its own
    path and slicing set."""
    from oracle import network as onw, planner as opl
    from workload import make_workload
    w = make_workload("rqc30")
    net = onw.absorb_small(onw.circuit_network(w.circuit, w.open_qubits, w.closed_bits))
    path, S, _ = opl.path_search(net.indices, w.max_rank, (), (0.5, 1.0, 2.0), (0.0, 0.3, 1.0), 16)
    tree = opl.Tree(net.indices, path)
    macs = tree.sliced_cost(S) >> len(S)
    model, cores, blas = host_cpu()
    t0 = time.perf_counter()
    onw.slice_output(net, path, S, 0)
    dt = time.perf_counter() - t0
    return {"value": 8.0 * macs / dt / 1e12, "unit": "TFLOP/s", "cores": cores, "blas_threads": blas,
            "cpu_model": model, "kind": "oracle", "sec_per_slice": dt,
            "sample": f"1 of {1 << len(S)} slices of rqc30 (slice 0, {macs:.3e} complex MACs), "
                      "numpy complex128 tensordot along the oracle's own path"}


def cpu_gradient():
    """The oracle's state-vector adjoint of the 20-qubit u3 workload: loss
    over 256 bitstrings and its gradient in all 720 angles."""
    from oracle import gradients as gr
    from workload import make_workload
    w = make_workload("rqc20_grad")
    model, cores, blas = host_cpu()
    t0 = time.perf_counter()
    gr.sv_adjoint(w.circuit, w.bitstrings)
    dt = time.perf_counter() - t0
    return {"ms_fwd_bwd": sig6(dt * 1e3), "cores": cores, "blas_threads": blas, "cpu_model": model,
            "kind": "oracle", "sample": "state-vector adjoint (complex128), all 720 angles"}


# ---------------------------------------------------------------- GPU legs
def time_plan(torch, P, pr, workload, modes, args, tag, fuse_rank=0, golden=None):
    """Bind a prepared plan and time each mode on it.

    rqc30: a step is every slice. rqc53: a step is one batch of slices from
    the seeded 1024-id subset, successive steps walking it. ``golden``
    (positions, per-slice amplitudes, slice ids, squared norms) gives each
    mode's error on those slices, run one at a time after the timed steps."""
    from workload import sample_slice_ids
    t0 = time.perf_counter()
    plan = pr.plan(fuse_rank=fuse_rank)
    costs = P.tree_costs(pr.net, pr.path, pr.sliced)
    info = plan.info()
    macs_slice = info["macs_per_slice"]
    steps = plan.steps()
    free = torch.cuda.mem_get_info()[0]
    if workload == "rqc30":
        ids = None
        batch = plan.bind(batch=1 << len(pr.sliced))
        per_step = 1 << len(pr.sliced)
    else:
        ids = np.asarray(sample_slice_ids(len(pr.sliced), 1024, 3), dtype=np.uint64)
        b = 1
        while b < len(ids) and plan.workspace_size(b + 1) < 0.75 * free:
            b += 1
        batch = plan.bind(batch=b)
        per_step = batch
    log(f"[{tag}] plan compiled and bound in {time.perf_counter() - t0:.2f}s: |S|={len(pr.sliced)} "
        f"C(B,S)=2^{costs.log2_sliced:.2f} per-slice MACs={macs_slice:.3e} batch={batch} "
        f"workspace={plan.workspace_size(batch) / 2**30:.2f} GiB")
    flops_step = 8.0 * macs_slice * per_step

    def batch_ids(j):
        lo = (j * per_step) % len(ids)
        sel = ids[lo:lo + per_step]
        if len(sel) < per_step:
            sel = np.concatenate([sel, ids[:per_step - len(sel)]])
        return sel

    def run_step(out, mode, j):
        if ids is None:
            plan.execute_range(0, per_step, out, mode)
        else:
            plan.execute(batch_ids(j), out, mode)

    def measure(mode):
        t0 = time.perf_counter()
        plan.autotune(mode, args.tune_cache)
        log(f"[{tag}/{mode}] autotuned in {time.perf_counter() - t0:.2f}s")
        out = plan.new_output()
        for j in range(args.warmup):
            out.zero_()
            run_step(out, mode, j)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for j in range(args.warmup, args.warmup + args.steps):
            out.zero_()
            run_step(out, mode, j)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res = {"tflops": flops_step * args.steps / dt / 1e12, "ms_per_step": 1e3 * dt / args.steps,
               "sec_per_slice": dt / args.steps / per_step}
        if golden is not None and ids is None:
            res["rel_l2_error"] = rel_l2(out.cpu().numpy(), golden["amplitudes"])
        elif golden is not None:
            errs, n2err = [], []
            for s, amp, n2 in zip(golden["ids"], golden["amplitudes"], golden["norm2"]):
                out.zero_()
                plan.execute([s], out, mode)
                got = out.cpu().numpy()
                errs.append(rel_l2(got[golden["positions"]], amp))
                n2err.append(abs(float(np.sum(np.abs(got) ** 2)) - n2) / n2)
            res["rel_l2_error"] = max(errs)
            res["rel_l2_error_per_slice"] = [sig6(e) for e in errs]
            res["norm2_rel_error_per_slice"] = [sig6(e) for e in n2err]
        # the dominant kernel (the MFMA complex GEMM): live per-step HIP
        # events on the plan's stream (a replay of one batch outside the graph)
        ms = np.zeros(len(steps))
        reps = 3
        first = 0 if ids is None else int(ids[0])
        for _ in range(reps):
            ms += plan.profile_steps(first, mode)
        ms /= reps
        # matrix-core steps: kinds 1 and 5 run k_cgemm_c64 (complex64, the
        # split-K form included), kind 2 runs k_cgemm_split; executed flops
        # and the GEMM-bound test per step come from step_roofline
        fam = {"k_cgemm_c64": (1, 5), "k_cgemm_split": (2,), "k_narrow": (3,)}
        kern = {name: {"launches": 0, "flops_per_batch": 0.0, "exec_flops_per_batch": 0.0,
                       "alg_bytes_per_batch": 0.0, "ms_per_batch": 0.0, "tiles": {}} for name in fam}
        for name in ("k_cgemm_c64", "k_cgemm_split"):
            kern[name]["steps"] = []
            kern[name]["gemm_bound"] = {"launches": 0, "exec_flops_per_batch": 0.0, "ms_per_batch": 0.0}
        mf_flops, mf_ms, mf_launch, split_flops = 0.0, 0.0, 0, 0.0
        for k, st in enumerate(steps):
            kind, _, _, _ = plan.step_kernel(k, mode)
            for name, kinds in fam.items():
                if kind in kinds:
                    tile = plan.step_kernel_name(k, mode)
                    f, fx, by, bound = step_roofline(kind, tile, st["m"], st["k"], st["n"], batch)
                    e = kern[name]
                    e["launches"] += 1
                    e["flops_per_batch"] += f
                    e["tiles"][tile] = e["tiles"].get(tile, 0) + 1
                    e["exec_flops_per_batch"] += fx
                    e["alg_bytes_per_batch"] += by
                    if "steps" in e:
                        e["steps"].append([k, st["m"], st["k"], st["n"], tile, round(float(ms[k]), 4), bound])
                        if bound:
                            g = e["gemm_bound"]
                            g["launches"] += 1
                            g["exec_flops_per_batch"] += fx
                            g["ms_per_batch"] += float(ms[k])
                    e["ms_per_batch"] += ms[k]
                    if name == "k_narrow":
                        continue
                    mf_flops += f
                    mf_ms += ms[k]
                    mf_launch += 1
                    if kind == 2:
                        split_flops += f
        for e in kern.values():
            e["alg_tflops"] = e["flops_per_batch"] / (e["ms_per_batch"] * 1e-3) / 1e12 if e["ms_per_batch"] > 0 else 0.0
            e["exec_tflops"] = e["exec_flops_per_batch"] / (e["ms_per_batch"] * 1e-3) / 1e12 if e["ms_per_batch"] > 0 else 0.0
            if "gemm_bound" in e:
                g = e["gemm_bound"]
                g["exec_tflops"] = g["exec_flops_per_batch"] / (g["ms_per_batch"] * 1e-3) / 1e12 if g["ms_per_batch"] > 0 else 0.0
            e["alg_gbs"] = e["alg_bytes_per_batch"] / (e["ms_per_batch"] * 1e-3) / 1e9 if e["ms_per_batch"] > 0 else 0.0
        res["kernels"] = kern
        res["mfma_ms_per_batch"] = mf_ms
        res["step_ms_per_batch"] = float(ms.sum())
        res["mfma_launches_per_batch"] = mf_launch
        res["mfma_tflops"] = mf_flops / (mf_ms * 1e-3) / 1e12 if mf_ms > 0 else 0.0
        res["split_mac_fraction"] = split_flops / (8.0 * macs_slice * batch)
        log(f"[{tag}/{mode}] {res['ms_per_step']:.2f} ms/step, {res['tflops']:.2f} TFLOP/s, "
            f"MFMA {mf_ms:.2f} of {res['step_ms_per_batch']:.2f} ms per batch "
            f"({res['mfma_tflops']:.2f} TFLOP/s), err {res.get('rel_l2_error')}")
        return res

    results = {m: measure(m) for m in modes}
    facts = dict(per_step=per_step, batch=batch, costs=costs, macs_slice=macs_slice,
                 flops_step=flops_step, n_sliced=len(pr.sliced), groups=plan.groups())
    del plan
    torch.cuda.empty_cache()
    return results, facts


def mode_table(results):
    out = {}
    for m, r in results.items():
        out[m] = {k: (sig6(v) if not isinstance(v, (list, dict)) else v) for k, v in r.items()}
        out[m]["speedup_vs_c64"] = round(r["tflops"] / results["c64"]["tflops"], 4) if "c64" in results else None
        out[m]["meets_tolerance"] = (r.get("rel_l2_error") is not None and r["rel_l2_error"] <= TOL[m])
    return out


def roofline_of(workload, mode, r):
    """The mode's dominant kernel over its own launches only: the complex64
    GEMM, whose achieved rate counts 8 algorithmic flops per complex MAC, or
    the split GEMM, whose achieved rate is what the matrix cores execute
    (three fp16/bf16 matrix products per real product: 3x the algorithmic
    count). The complex64 GEMM's three-product tiles execute 6 flops per
    complex MAC, so its algorithmic rate can pass the FP32 matrix peak (up
    to 4/3 of it); `executed` and `executed_frac` give what the matrix cores
    ran."""
    kernel = "k_cgemm_c64" if mode == "c64" else "k_cgemm_split"
    e = r["kernels"][kernel]
    if mode == "c64":
        peak, achieved = PEAK_FP32_MFMA_TFLOPS, e["alg_tflops"]
    else:
        peak, achieved = PEAK_F16_MFMA_TFLOPS, e["exec_tflops"]
    return {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4), "traffic": counter_traffic(workload, mode),
            "kernel": kernel, "executed": round(e["exec_tflops"], 3),
            "executed_frac": round(e["exec_tflops"] / peak, 4),
            "executed_flops_per_complex_mac": "6 on c64_3m/splitk_3m tiles, 8 on direct complex64 tiles"
            if mode == "c64" else "24 (three fp16/bf16 products of the 2x2 real form)",
            "gemm_bound_steps": {"launches": e["gemm_bound"]["launches"],
                                 "share_of_kernel_time": round(e["gemm_bound"]["ms_per_batch"] / e["ms_per_batch"], 4)
                                 if e["ms_per_batch"] > 0 else 0.0,
                                 "executed": round(e["gemm_bound"]["exec_tflops"], 3),
                                 "executed_frac": round(e["gemm_bound"]["exec_tflops"] / peak, 4)},
            "launches_per_batch": e["launches"],
            "share_of_step_time": round(e["ms_per_batch"] / r["step_ms_per_batch"], 4)}


def rqc53_golden(stem="rqc53_slices"):
    path = os.path.join(GOLDEN, stem + ".npz")
    if not os.path.exists(path):
        return None, None
    z = np.load(path)
    meta = json.load(open(os.path.join(GOLDEN, stem + ".json")))
    return {"positions": z["positions"], "amplitudes": list(z["amplitudes"]),
            "ids": [int(r["id"]) for r in meta["slices"]],
            "norm2": [r["norm2"] for r in meta["slices"]]}, meta


def rqc30_extra(torch, P, args):
    """The 30-qubit workload: every slice per step on the randomised greedy
    path (all modes), then the same circuit on the reconfigured path, with
    and without fused sub-paths."""
    from workload import make_workload
    w = make_workload("rqc30")
    ref_path = os.path.join(GOLDEN, "rqc30_amplitudes.npy")
    golden = {"amplitudes": np.load(ref_path)} if os.path.exists(ref_path) else None
    t0 = time.perf_counter()
    pr = P.prepare(w)
    t_plan = time.perf_counter() - t0
    res, f = time_plan(torch, P, pr, "rqc30", args.rqc30_modes.split(","), args, "rqc30", golden=golden)
    out = {"workload": WORKLOAD_TEXT["rqc30"] + ", all slices per step, randomised greedy path",
           "plan_seconds": round(t_plan, 3), "slices": f["per_step"], "sliced_indices": f["n_sliced"],
           "batch": f["batch"], "log2_C_BS": round(f["costs"].log2_sliced, 4),
           "overhead": round(f["costs"].overhead, 5), "macs_per_slice": f["macs_slice"],
           "modes": mode_table(res), "roofline": roofline_of("rqc30", "c64", res["c64"]) if "c64" in res else None}
    if args.path_variant:
        t0 = time.perf_counter()
        prv = P.prepare(w, reconf_k=10)
        t_plan = time.perf_counter() - t0
        vres, vf = time_plan(torch, P, prv, "rqc30", args.path_variant.split(","), args, "rqc30 reconf",
                             golden=golden)
        var = {"path": "randomised greedy + subtree reconfiguration (k=10)", "plan_seconds": round(t_plan, 3),
               "sliced_indices": vf["n_sliced"], "log2_C_BS": round(vf["costs"].log2_sliced, 4),
               "macs_per_slice": vf["macs_slice"],
               "modes": {m: {k: sig6(v) for k, v in r.items()} for m, r in vres.items()}}
        for m, r in vres.items():
            if m in res:
                var["modes"][m]["time_to_solution_speedup_vs_greedy_path"] = round(
                    res[m]["ms_per_step"] / r["ms_per_step"], 3)
        fres, ff = time_plan(torch, P, prv, "rqc30", ["c64"], args, "rqc30 reconf+fused", fuse_rank=10,
                             golden=golden)
        var["fused_sub_paths"] = {"fuse_rank": 10, "groups": len(ff["groups"]),
                                  "steps_fused": sum(g["n_steps"] for g in ff["groups"]),
                                  "c64": {k: sig6(v) for k, v in fres["c64"].items()}}
        out["path_variant"] = var
    return out


def gradient_leg(torch, P, args):
    """Forward + adjoint of the 20-qubit u3 workload (720 angles, loss over
    256 bitstrings, each one slice), timed with the same warm-up / step
    counts, checked against the stored oracle adjoint gradient."""
    from paper_2205_00393_amd.autograd import Amplitudes
    from workload import make_workload
    w = make_workload("rqc20_grad")
    pr = P.prepare(w, alphas=(0.5, 1.0), taus=(0.0, 0.3), n_seeds=3)
    plan = pr.plan()
    # 32 GiB of the 288 GB hold all 256 bitstring slices in one batch
    batch = plan.bind(batch=0, grad=True, budget_bytes=32 << 30)
    plan.autotune("c64", args.tune_cache)  # forward steps and the adjoint products
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
    ref_path = os.path.join(GOLDEN, "rqc20_grad_reference.npz")
    if os.path.exists(ref_path):
        ref = np.load(ref_path)
        gg = g.detach().cpu().numpy()
        res["grad_rel_l2_error"] = sig6(float(np.linalg.norm(gg - ref["grad"]) / np.linalg.norm(ref["grad"])))
    log(f"gradient: {res['ms_fwd_bwd']:.2f} ms forward + backward, error {res.get('grad_rel_l2_error')}")
    del plan
    torch.cuda.empty_cache()
    return res


# ------------------------------------------------------- profile summaries
def _csv_rows(d, suffix):
    import csv
    import glob
    rows = []
    for f in sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)):
        rows += [dict(r, _file=f) for r in csv.DictReader(open(f))]
    return rows


def _per_dispatch(d, counter, name_part=None, keep=None):
    """Counter value per dispatch (summed over the counter's dimensions),
    for kernels whose name contains name_part (all when None); with keep,
    only the last whole multiple of keep dispatches in dispatch order."""
    v = {}
    names = {}
    for r in _csv_rows(d, "counter_collection.csv"):
        if r["Counter_Name"] != counter or (name_part and name_part not in r["Kernel_Name"]):
            continue
        key = (r["_file"], int(r["Dispatch_Id"]))
        v[key] = v.get(key, 0.0) + float(r["Counter_Value"])
        names[key] = r["Kernel_Name"]
    if keep:
        order = sorted(v)
        order = order[len(order) - (len(order) // keep) * keep:]
        v = {k: v[k] for k in order}
    return v, names


def _durations(d, name_part, keep):
    """Durations (ns) of the dispatches of kernels containing name_part, the
    last whole multiple of keep in dispatch order (the launches of whole
    batches: the autotuner's forward pass over its default choices runs
    fewer of them before the first batch)."""
    rows = sorted((int(x["Dispatch_Id"]), int(x["End_Timestamp"]) - int(x["Start_Timestamp"]))
                  for x in _csv_rows(d, "kernel_trace.csv") if name_part in x["Kernel_Name"])
    rows = rows[len(rows) - (len(rows) // keep) * keep:]
    return [t for _, t in rows]


def summarize_main(argv):
    """Summarise the rocprofv3 runs of one kernel family into
    profiles/<stem>.json and .md (run from the repository root):

      python bench.py summarize --kernel k_cgemm_c64 --workload rqc53 --mode c64 \
          --bench BENCH_LINE.json --trace DIR --fetch DIR --write DIR \
          --copy-fetch DIR --copy-write DIR --copy-mib 1024 [--mfma DIR] \
          --commands FILE --out profiles/STEM

    The kernel trace gives the average launch duration; FETCH_SIZE and
    WRITE_SIZE (KiB per dispatch) are scaled by what they read for a plain
    device copy of --copy-mib MiB; the bench line of the same session gives
    the algorithmic flops and bytes per batch of the kernel family."""
    ap = argparse.ArgumentParser(prog="bench.py summarize")
    for a in ("--kernel", "--workload", "--mode", "--bench", "--trace", "--fetch", "--write",
              "--copy-fetch", "--copy-write", "--commands", "--out"):
        ap.add_argument(a, required=True)
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--mfma", default=None)
    ap.add_argument("--bound", default="mfma", choices=["mfma", "hbm"],
                    help="hbm: report achieved algorithmic GB/s against the 8 TB/s HBM peak")
    a = ap.parse_args(argv)
    line = json.loads(open(a.bench).read().strip().splitlines()[-1])
    r = line["modes"][a.mode] if a.workload in line["config"]["workload"] else \
        line[a.workload]["modes"][a.mode]
    batch = line["config"]["batch"] if a.workload in line["config"]["workload"] else line[a.workload]["batch"]
    e = r["kernels"][a.kernel]
    launches = e["launches"]
    flops_l = e["flops_per_batch"] / launches
    bytes_l = e["alg_bytes_per_batch"] / launches
    durs = _durations(a.trace, a.kernel, launches)
    avg_ms = sum(durs) / len(durs) / 1e6
    copy_bytes = a.copy_mib << 20
    cf, cfn = _per_dispatch(a.copy_fetch, "FETCH_SIZE")
    cw, cwn = _per_dispatch(a.copy_write, "WRITE_SIZE")
    kf = max(cf, key=cf.get)
    kw = max(cw, key=cw.get)
    fetch_scale = copy_bytes / (cf[kf] * 1024.0)
    write_scale = copy_bytes / (cw[kw] * 1024.0)
    f, _ = _per_dispatch(a.fetch, "FETCH_SIZE", a.kernel, launches)
    w, _ = _per_dispatch(a.write, "WRITE_SIZE", a.kernel, launches)
    fetch_l = sum(f.values()) / len(f) * 1024.0 * fetch_scale
    write_l = sum(w.values()) / len(w) * 1024.0 * write_scale
    split = a.mode != "c64" and a.kernel == "k_cgemm_split"
    peak = PEAK_F16_MFMA_TFLOPS if split else PEAK_FP32_MFMA_TFLOPS
    alg_tf = flops_l / (avg_ms * 1e-3) / 1e12
    # executed matrix flops: 3x the algorithmic count on split tiles, 3/4 of
    # it on the three-product complex64 tiles (the bench line counts them)
    exe_l = e["exec_flops_per_batch"] / launches if "exec_flops_per_batch" in e else \
        flops_l * (3.0 if split else 1.0)
    exe_tf = exe_l / (avg_ms * 1e-3) / 1e12
    alg_gbs = bytes_l / (avg_ms * 1e-3) / 1e9
    src_name = KERNEL_SOURCE.get(a.kernel, "k_mfma.hip")
    src = open(os.path.join(ROOT, "paper_2205_00393_amd", "csrc", src_name), "rb").read()
    rec = {"kernel": a.kernel, "workload": a.workload, "mode": a.mode, "batch": batch,
           "launches_per_batch": launches, "avg_launch_ms": avg_ms, "calls": len(durs),
           "alg_flops_per_launch": flops_l, "alg_bytes_per_launch": bytes_l,
           "achieved_alg_tflops": alg_tf, "executed_matrix_tflops": exe_tf, "peak_tflops": peak,
           "tiles_per_batch": e.get("tiles"), "alg_frac_of_peak": alg_tf / peak,
           "frac_of_peak": exe_tf / peak if a.bound == "mfma" else alg_gbs / PEAK_HBM_GBS,
           "bound": a.bound, "achieved_alg_gbs": alg_gbs, "peak_gbs": PEAK_HBM_GBS,
           "hbm_fetch_bytes_per_launch": fetch_l, "hbm_write_bytes_per_launch": write_l,
           "traffic_bytes_per_launch": fetch_l + write_l,
           "traffic_over_algorithmic": (fetch_l + write_l) / bytes_l,
           "fetch_scale": fetch_scale, "write_scale": write_scale,
           "copy_kernel": cfn[kf], "source": src_name, "source_sha256": hashlib.sha256(src).hexdigest(),
           "bench_tflops": line["value"] if a.workload in line["config"]["workload"] else None}
    md = [f"# {a.kernel} on the {a.workload} workload ({a.mode})", "",
          f"Workload: {line['config']['workload'] if a.workload in line['config']['workload'] else line[a.workload]['workload']}.",
          f"Batch of {batch} slices; tiles from the autotuner (cache written by the first command, "
          "in the same session).", "", "## Commands (repository root, `TMPDIR=/tmp`)", "", "```",
          open(a.commands).read().strip(), "```", ""]
    if a.mfma:
        inst, _ = _per_dispatch(a.mfma, "SQ_INSTS_MFMA", a.kernel, launches)
        busy, _ = _per_dispatch(a.mfma, "SQ_VALU_MFMA_BUSY_CYCLES", a.kernel, launches)
        n_inst = sum(inst.values())
        # flops per MFMA instruction: 32x32x2 FP32 = 4096, 32x32x16 f16/bf16 = 32768
        fpi = 32768 if split else 4096
        mc = {"dispatches": len(inst), "mfma_instructions": n_inst, "flops_per_instruction": fpi,
              "executed_flops": n_inst * fpi, "SQ_VALU_MFMA_BUSY_CYCLES": sum(busy.values())}
        # durations of the same dispatches from the counter run's own kernel trace
        md_durs = _durations(a.mfma, a.kernel, launches)
        if md_durs and len(md_durs) == len(inst):
            tf = n_inst * fpi / (sum(md_durs) * 1e-9) / 1e12
            mc.update(duration_ms_total=sum(md_durs) / 1e6, executed_tflops_from_counters=tf,
                      frac_of_peak_from_counters=tf / peak)
            # the GEMM-bound steps: the kept dispatches are whole batches, a
            # batch launching the family's steps in step order
            if e.get("steps") and len(e["steps"]) == launches:
                vals = [inst[key] for key in sorted(inst)]
                sel = [j for j in range(len(vals)) if e["steps"][j % launches][6]]
                if sel:
                    gtf = sum(vals[j] for j in sel) * fpi / (sum(md_durs[j] for j in sel) * 1e-9) / 1e12
                    mc.update(gemm_bound_dispatches=len(sel), gemm_bound_executed_tflops_from_counters=gtf,
                              gemm_bound_frac_of_peak_from_counters=gtf / peak)
        rec["mfma_counters"] = mc
    if a.bound == "mfma":
        first = (f"* {a.kernel}: {launches} launches per batch, average {avg_ms:.3f} ms per launch "
                 f"({len(durs)} launches traced); algorithmic flops per launch (8 per complex MAC) "
                 f"{flops_l:.4e} -> {alg_tf:.1f} TFLOP/s algorithmic ({100 * alg_tf / peak:.1f} % of the "
                 f"{peak} TFLOP/s dense peak), {exe_tf:.1f} TFLOP/s executed on the matrix cores "
                 f"({exe_l:.4e} flops per launch) = {100 * exe_tf / peak:.1f} % of peak.")
    else:
        first = (f"* {a.kernel}: {launches} launches per batch, average {avg_ms:.4f} ms per launch "
                 f"({len(durs)} launches traced); algorithmic bytes per launch (A + B + C once) "
                 f"{bytes_l:.4e} -> {alg_gbs:.0f} GB/s = {100 * alg_gbs / PEAK_HBM_GBS:.1f} % of the "
                 f"{PEAK_HBM_GBS:.0f} GB/s HBM peak (aggregate over the launches of a batch).")
    md += ["## Figures", "", first,
           f"* HBM traffic per launch: fetch {fetch_l:.4e} B + write {write_l:.4e} B = "
           f"{fetch_l + write_l:.4e} B against {bytes_l:.4e} B algorithmic (A + B + C once) = "
           f"{(fetch_l + write_l) / bytes_l:.2f} x.",
           f"* Counter scale from a {a.copy_mib} MiB device copy (`{cfn[kf][:60]}`): FETCH_SIZE x "
           f"{fetch_scale:.4f}, WRITE_SIZE x {write_scale:.4f}.",
           f"* {src_name} sha256 at measurement: `{rec['source_sha256']}`"]
    if e.get("tiles"):
        md.append("* Tiles per batch: " + ", ".join(f"{t} x {c}" for t, c in sorted(e["tiles"].items())) + ".")
    if e.get("gemm_bound") and e["gemm_bound"]["launches"]:
        g = e["gemm_bound"]
        rec["gemm_bound"] = {"launches_per_batch": g["launches"], "share_of_kernel_time": g["ms_per_batch"] / e["ms_per_batch"],
                             "executed_tflops_hip_events": g["exec_tflops"], "frac_of_peak": g["exec_tflops"] / peak}
        md.append(f"* GEMM-bound steps (executed flops per algorithmic byte at or above the ridge, {peak} TFLOP/s "
                  f"/ {PEAK_HBM_GBS:.0f} GB/s): {g['launches']} of {launches} launches per batch, "
                  f"{100 * g['ms_per_batch'] / e['ms_per_batch']:.1f} % of the kernel's time, executed "
                  f"{g['exec_tflops']:.1f} TFLOP/s = {100 * g['exec_tflops'] / peak:.1f} % of peak (HIP events in the "
                  f"bench run); the other steps are bound by HBM.")
    if "mfma_counters" in rec and "executed_tflops_from_counters" in rec["mfma_counters"]:
        mc = rec["mfma_counters"]
        md.append(f"* MFMA instruction counters: {mc['mfma_instructions']:.4e} instructions x "
                  f"{mc['flops_per_instruction']} flops in {mc['duration_ms_total']:.1f} ms of kernel time "
                  f"({mc['dispatches']} dispatches; counter runs serialise kernels) = "
                  f"{mc['executed_tflops_from_counters']:.1f} TFLOP/s = "
                  f"{100 * mc['frac_of_peak_from_counters']:.1f} % of peak"
                  + (f"; GEMM-bound steps alone ({mc['gemm_bound_dispatches']} dispatches) "
                     f"{mc['gemm_bound_executed_tflops_from_counters']:.1f} TFLOP/s = "
                     f"{100 * mc['gemm_bound_frac_of_peak_from_counters']:.1f} %."
                     if "gemm_bound_dispatches" in mc else "."))
    md.append("")
    stats = _csv_rows(a.trace, "kernel_stats.csv")
    if stats:
        md += ["## Kernel statistics (`--kernel-trace --stats`)", "",
               "| kernel | calls | total ms | avg us | % |", "|---|---|---|---|---|"]
        for x in stats[:20]:
            g = lambda *ks: next((x[k] for k in ks if k in x), "0")
            md.append(f"| {g('Name', 'KernelName')[:90]} | {g('Calls')} | "
                      f"{float(g('TotalDurationNs')) / 1e6:.3f} | {float(g('AverageNs')) / 1e3:.1f} | "
                      f"{float(g('Percentage')):.2f} |")
        md.append("")
    json.dump(rec, open(a.out + ".json", "w"), indent=1)
    open(a.out + ".md", "w").write("\n".join(md) + "\n")
    print(json.dumps(rec))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rqc53", choices=["rqc53", "rqc30"],
                    help="headline workload: rqc53 walks the seeded 1024-slice subset one batch "
                         "per step; rqc30 runs every slice per step")
    ap.add_argument("--modes", default="c64,split_f16,split_bf16",
                    help="comma list; the first is the headline value, the others are reported beside it")
    ap.add_argument("--extras", default="rqc30,grad",
                    help="comma list of extra legs: rqc30 (30-qubit workload), grad (20-qubit "
                         "gradient); '' for none")
    ap.add_argument("--rqc30-modes", default="c64,split_f16,split_bf16")
    ap.add_argument("--path-variant", default="c64,split_bf16",
                    help="modes to time on the reconfigured path as well, for the headline "
                         "workload and the rqc30 leg ('' to skip)")
    ap.add_argument("--reconf-k", type=int, default=0,
                    help="headline plan on the greedy trials improved by subtree reconfiguration with "
                         "this window (0: the randomised greedy path, the workloads' definition)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle legs")
    ap.add_argument("--no-golden", action="store_true",
                    help="skip the error checks on stored oracle slices (profiled runs: they launch "
                         "one-slice batches)")
    ap.add_argument("--tune-cache", default=None, help="autotuner cache (JSON, keyed by mode and step shape)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration) and exit")
    ap.add_argument("--gradient-only", action="store_true",
                    help="only run the gradient leg (profiling) and print its record")
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
    if args.gradient_only:
        print(json.dumps({"gradient": gradient_leg(torch, P, args)}), flush=True)
        return
    extras = [e for e in args.extras.split(",") if e]
    modes = args.modes.split(",")
    main_mode = modes[0]

    if args.workload == "rqc53":
        w = make_workload("rqc53")
        t0 = time.perf_counter()
        pr = P.prepare(w, reconf_k=args.reconf_k)
        t_plan = time.perf_counter() - t0
        log(f"[rqc53] host planner (randomised greedy search + Algorithm 1) {t_plan:.2f}s")
        golden, meta = rqc53_golden("rqc53_reconf_slices" if args.reconf_k else "rqc53_slices") \
            if not args.no_golden else (None, None)
        if meta is not None and meta["sliced"] != pr.sliced:
            log("[rqc53] the stored oracle slices belong to another slicing set; no error reported")
            golden = None
        results, f = time_plan(torch, P, pr, "rqc53", modes, args, "rqc53", golden=golden)
        walked = f["per_step"] * args.steps
        pathtxt = f"randomised greedy path + subtree reconfiguration (k={args.reconf_k})" if args.reconf_k \
            else "randomised greedy path"
        wl = (f"{WORKLOAD_TEXT['rqc53']}, {pathtxt}, |S|={f['n_sliced']}; one step = one "
              f"batch of {f['per_step']} slices walking the seeded subset of 1024 slice ids "
              f"(seed 3); {walked} slices timed")
        variant = None
        if args.path_variant and not args.reconf_k:
            # the same circuit on the greedy trials improved by subtree
            # reconfiguration (window 8): fewer sliced indices, less work per slice
            t0 = time.perf_counter()
            prv = P.prepare(w, reconf_k=8)
            t_planv = time.perf_counter() - t0
            gv, mv = rqc53_golden("rqc53_reconf_slices") if not args.no_golden else (None, None)
            if mv is not None and mv["sliced"] != prv.sliced:
                gv = None
            vres, vf = time_plan(torch, P, prv, "rqc53", args.path_variant.split(","), args, "rqc53 reconf",
                                 golden=gv)
            variant = {"path": "randomised greedy + subtree reconfiguration (k=8)",
                       "plan_seconds": round(t_planv, 3), "sliced_indices": vf["n_sliced"],
                       "log2_C_BS": round(vf["costs"].log2_sliced, 4), "macs_per_slice": vf["macs_slice"],
                       "batch": vf["batch"],
                       "projected_seconds_all_slices": {m: r["sec_per_slice"] * 2.0 ** vf["n_sliced"]
                                                        for m, r in vres.items()},
                       "modes": mode_table(vres)}
            for m, r in vres.items():
                if m in results:
                    variant["modes"][m]["time_to_solution_speedup_vs_greedy_path"] = float(
                        (results[m]["sec_per_slice"] * 2.0 ** f["n_sliced"]) /
                        (r["sec_per_slice"] * 2.0 ** vf["n_sliced"]))
    else:
        w = make_workload("rqc30")
        t0 = time.perf_counter()
        pr = P.prepare(w, reconf_k=args.reconf_k)
        t_plan = time.perf_counter() - t0
        ref_path = os.path.join(GOLDEN, "rqc30_amplitudes.npy")
        golden = {"amplitudes": np.load(ref_path)} if os.path.exists(ref_path) and not args.no_golden else None
        results, f = time_plan(torch, P, pr, "rqc30", modes, args, "rqc30", golden=golden)
        wl = WORKLOAD_TEXT["rqc30"] + ", all slices per step, randomised greedy path" + \
            (f" + subtree reconfiguration (k={args.reconf_k})" if args.reconf_k else "")
        extras = [e for e in extras if e != "rqc30"]
        variant = None
    r0 = results[main_mode]
    n_sliced = f["n_sliced"]
    line = {
        "metric": "contraction TFLOP/s + sec/slice on 1 GPU; split-FP16 vs complex64 at stated error",
        "value": round(r0["tflops"], 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r0["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"c64": "c64", "split_f16": "f16x2", "split_bf16": "bf16x2"}[main_mode],
        "data": "synthetic",
        "config": {"workload": wl, "mode": main_mode,
                   "path": "randomised greedy" + (f" + subtree reconfiguration (k={args.reconf_k})"
                                                  if args.reconf_k else ""),
                   "slices_per_step": f["per_step"], "batch": f["batch"], "sliced_indices": n_sliced,
                   "log2_C_BS": round(f["costs"].log2_sliced, 4), "overhead": round(f["costs"].overhead, 5),
                   "macs_per_slice": f["macs_slice"], "flops_per_step": f["flops_step"],
                   "plan_seconds": round(t_plan, 3)},
        "sec_per_slice": r0["sec_per_slice"],
        "projection": {"slices": float(2.0 ** n_sliced),
                       "seconds_all_slices": {m: r["sec_per_slice"] * 2.0 ** n_sliced for m, r in results.items()},
                       "total_flops_8C_BS": 8.0 * f["costs"].sliced},
        "rel_l2_error": r0.get("rel_l2_error"),
        "modes": mode_table(results),
        "roofline": roofline_of(args.workload, main_mode, r0),
        "cpu_baseline": None,
    }
    if args.workload == "rqc53" and variant is not None:
        line["path_variant"] = variant
    if "rqc30" in extras:
        line["rqc30"] = rqc30_extra(torch, P, args)
    if "grad" in extras:
        line["gradient"] = gradient_leg(torch, P, args)
    if not args.no_cpu:
        log("timing the CPU oracle ...")
        if args.workload == "rqc53":
            line["cpu_baseline"] = cpu_rqc53(pr.sliced)
        else:
            line["cpu_baseline"] = cpu_rqc30()
        if line["cpu_baseline"] is not None:
            cb = line["cpu_baseline"]
            log(f"oracle: {cb['sec_per_slice']:.2f} s/slice, {cb['value']:.4f} TFLOP/s on {cb['cores']} cores")
        if "rqc30" in line:
            line["rqc30"]["cpu_baseline"] = cpu_rqc30()
        if "gradient" in line:
            line["gradient"]["cpu_baseline"] = cpu_gradient()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "summarize":
        summarize_main(sys.argv[2:])
    else:
        main()
