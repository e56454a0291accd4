"""Benchmark of the headline workload: ground states (energy + configuration)
of 64 seeded 16x16 open square-lattice Ising spin glasses with Gaussian
couplings J ~ N(0, 1) and fields h ~ N(0, 0.1^2), float32, in one batch.

One step = the whole hot path on one batch: the max-plus sweep (all passes),
the final reduction and the argmax-routing backward that returns sigma and
dE/dJ, dE/dh. Inputs are resident in HBM before timing starts.

Prints one JSON line (metric, value = solves/s, roofline of the dominant
kernel, CPU-oracle baseline). Only one GPU is used; --gpus above 1 exits.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "max-plus Gop/s & % VALU peak; ground-state solves/s (energy+config), 16x16 ±J"
VALU_PEAK_OPS = 256 * 64 * 2.4e9 * 2      # max-plus ops/s: one term (add + max) per lane per cycle
# HBM bytes per k_pass launch of the headline workload (one of the two
# concurrent half-batch launches of a pass), by tile size, from rocprofv3
# counter passes: FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 (the factors a plain
# 256 MiB device copy reads for the same counters);
# profiles/k_pass_square16x16_gauss_b64.txt. Emptied whenever the pass
# kernel changes, until the counters are taken again.
K_PASS_TRAFFIC_BYTES = {11: 16.53e6, 12: 16.47e6, 13: 16.39e6, 14: 16.34e6}


def cpu_baseline(insts, seconds=15.0):
    """The oracle as it stands, on a bounded sample of the same workload."""
    from oracle import spinglass as O
    n = insts[0].n
    t0 = time.perf_counter()
    done = 0
    for x in insts:
        O.eliminate(n, x.edges, x.J, x.h, order=list(range(n)))
        done += 1
        if time.perf_counter() - t0 > seconds:
            break
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} of the 64 instances, numpy max-sum elimination (raster order) "
                      f"with traceback, single thread, {dt:.1f} s"}


def bench_tgemm(args):
    """Dense tropical product C = max_k A + B, float32, square S x S x S."""
    import torch

    from paper_2008_06888_amd import binding as B
    S = args.tgemm
    g = torch.Generator(device="cuda:0").manual_seed(0)
    A = torch.randn(S, S, device="cuda:0", generator=g)
    Bm = torch.randn(S, S, device="cuda:0", generator=g)
    C = torch.empty(S, S, device="cuda:0")
    for _ in range(args.warmup):
        B.tgemm(A, Bm, out=C)
    torch.cuda.synchronize()
    B.prof_reset()
    B.prof_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        B.tgemm(A, Bm, out=C)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    B.prof_enable(False)
    ms, n = B.prof_read("tgemm")
    ops = 2.0 * S * S * S        # one add and one max per term
    achieved = ops * n / (ms * 1e-3) if ms > 0 else 0.0
    print(json.dumps({"metric": "tropical GEMM max-plus TFLOP/s", "value": ops * args.steps / dt / 1e12,
                      "unit": "TFLOP/s", "steps": args.steps, "warmup": args.warmup, "dtype": "f32",
                      "config": {"workload": f"tgemm_{S}x{S}x{S}"},
                      "roofline": {"kernel": "k_tgemm", "bound": "alu", "achieved": achieved / 1e12,
                                   "peak": VALU_PEAK_OPS / 1e12, "unit": "TFLOP/s",
                                   "frac": achieved / VALU_PEAK_OPS, "avg_launch_ms": ms / max(n, 1)}}))


def _timed(fn, steps):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def bench_chimera(args):
    """Chimera graph of 8 x 8 K_{4,4} cells (512 spins), J = +-1, h = 0: ground-state
    energy and configuration, and separately the exact degeneracy count."""
    import numpy as np
    import torch

    from paper_2008_06888_amd import binding as B
    from paper_2008_06888_amd import instances as I
    x = I.config_instances(4)[0]
    J = torch.tensor(x.J[None], device="cuda:0")
    plan = B.Plan(512, x.edges, chimera=(8, 8))
    tile_bits, _ = B.autotune(plan, J, config=True)
    steps = max(1, min(args.steps, 5))
    for _ in range(min(args.warmup, 1)):
        B.backward(plan, J)
    B.prof_reset()
    B.prof_enable(True)
    t_solve = _timed(lambda: B.backward(plan, J), steps)
    B.prof_enable(False)
    kern = {k: B.prof_read(k) for k in ("sweep_pass", "chain", "final_reduce", "row_argmax", "chimera_finish")}
    E, sig, _, _ = B.backward(plan, J)
    plan.close()
    cplan = B.Plan(512, x.edges, chimera=(8, 8))
    t0 = time.perf_counter()
    Ec, res, g = B.count(cplan, J)
    t_count = time.perf_counter() - t0
    cplan.close()
    print(json.dumps({"metric": "chimera 8x8 ground state (energy + configuration) wall time", "value": t_solve,
                      "unit": "s", "higher_is_better": False, "steps": steps, "dtype": "f32 (integer-valued)",
                      "config": {"workload": "chimera8x8_pm1", "spins": 512, "couplers": int(len(x.edges)), "tile_bits": tile_bits},
                      "energy": float(E[0].item()), "count_s": t_count, "count_energy": int(Ec[0]),
                      "degeneracy": str(g[0]), "entropy_per_spin": math.log(g[0]) / 512,
                      "kernel_ms_per_solve": {k: v[0] / steps for k, v in kern.items()}}))


def bench_square32(args):
    """32 x 32 open square lattice, J = +-1: ground-state energy and exact degeneracy."""
    import numpy as np
    import torch

    from paper_2008_06888_amd import binding as B
    from paper_2008_06888_amd import instances as I
    x = I.config_instances(2)[0]
    J = torch.tensor(x.J[None], device="cuda:0")
    plan = B.Plan(1024, x.edges, order=list(range(1024)))
    B.count(plan, J)
    B.prof_reset()
    B.prof_enable(True)
    t0 = time.perf_counter()
    Ec, res, g = B.count(plan, J)
    dt = time.perf_counter() - t0
    B.prof_enable(False)
    kern = {k: B.prof_read(k) for k in ("count_pass", "count_reduce")}
    t_e = _timed(lambda: B.contract(plan, J), max(1, min(args.steps, 5)))
    print(json.dumps({"metric": "32x32 +-J ground-state energy and degeneracy wall time", "value": dt, "unit": "s",
                      "higher_is_better": False, "dtype": "f32 (integer-valued) + 3 x u64 residues",
                      "config": {"workload": "square32_pm1_count", "spins": 1024},
                      "energy": int(Ec[0]), "degeneracy": str(g[0]), "entropy_per_spin": math.log(g[0]) / 1024,
                      "energy_only_s": t_e, "kernel_ms": {k: v[0] for k, v in kern.items()}}))


def bench_uneven(args):
    """16 random 3-regular graphs, N = 100 + 20 (i mod 7), J ~ N(0, 1), h = 0, greedy
    orders, tile sizes autotuned per plan: energy + configuration of all 16 in one
    call (grouped launches) against one call per instance."""
    import torch

    from paper_2008_06888_amd import binding as B
    from paper_2008_06888_amd import instances as I
    insts = I.config_instances(3)
    t0 = time.perf_counter()
    plans = [B.Plan(x.n, x.edges, seed=i) for i, x in enumerate(insts)]
    t_plan = time.perf_counter() - t0
    Js = [torch.tensor(x.J, device="cuda:0") for x in insts]
    t0 = time.perf_counter()
    tiles = [B.autotune(p, j[None], config=True)[0] for p, j in zip(plans, Js)]
    t_tune = time.perf_counter() - t0
    steps = max(1, min(args.steps, 3))
    for _ in range(2):
        B.contract_uneven(plans, Js)
        for p, j in zip(plans, Js):
            B.backward(p, j[None])
    t_batched = _timed(lambda: B.contract_uneven(plans, Js), steps)

    def one_by_one():
        for p, j in zip(plans, Js):
            B.backward(p, j[None])
    t_single = _timed(one_by_one, steps)
    widths = [p.info()["width"] for p in plans]
    print(json.dumps({"metric": "uneven batch ground states (energy + configuration) solves/s",
                      "value": len(insts) / t_batched, "unit": "solves/s", "higher_is_better": True,
                      "steps": steps, "dtype": "f32",
                      "config": {"workload": "reg3_uneven_b16", "n": [x.n for x in insts], "widths": widths},
                      "one_call_per_instance_solves_s": len(insts) / t_single, "planning_s": t_plan,
                      "tile_bits": tiles, "autotune_s": t_tune}))


def copy_calibration(args):
    """A plain copy of known size: its FETCH_SIZE / WRITE_SIZE readings scale the counters."""
    import torch
    n = args.copy_calibration * (1 << 20) // 4
    src = torch.ones(n, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(max(args.steps, 1)):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_each_way": 4 * n, "launches": max(args.steps, 1)}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--headline-only", action="store_true",
                    help="run only the timed headline steps (for profilers): no context runs, no CPU baseline")
    ap.add_argument("--tgemm", type=int, default=0, metavar="S",
                    help="instead: time the dense tropical product at M = N = K = S")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="instead: run a plain device copy of MIB MiB (scale for HBM byte counters)")
    ap.add_argument("--workload", default="square16_gauss_b64",
                    choices=["square16_gauss_b64", "chimera8x8_pm1", "square32_pm1_count", "reg3_uneven_b16"],
                    help="the headline workload (default) or one of the other measured cases")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    if args.tgemm:
        return bench_tgemm(args)
    if args.copy_calibration:
        return copy_calibration(args)
    if args.workload == "chimera8x8_pm1":
        return bench_chimera(args)
    if args.workload == "square32_pm1_count":
        return bench_square32(args)
    if args.workload == "reg3_uneven_b16":
        return bench_uneven(args)

    import numpy as np
    import torch

    from paper_2008_06888_amd import binding as B
    from paper_2008_06888_amd import instances as I

    insts = I.config_instances(1)
    L, batch = 16, len(insts)
    n = L * L
    plan = B.Plan(n, insts[0].edges, order=list(range(n)), has_field=True)
    info = plan.info()
    dev = torch.device("cuda:0")
    J = torch.tensor(np.stack([x.J for x in insts]), device=dev)
    h = torch.tensor(np.stack([x.h for x in insts]), device=dev)

    # tile size chosen by the autotuner on this batch (outside the timed region)
    tile_bits, _ = B.autotune(plan, J, h, config=True)
    info = plan.info()
    # warm-up: the second call is captured as a HIP graph, later calls replay it
    for _ in range(max(args.warmup, 2)):
        B.backward(plan, J, h)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        B.backward(plan, J, h)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # kernel durations: the same steps again with every launch bracketed by HIP
    # events on its stream (timed calls run eagerly: same kernels and grids)
    B.prof_reset()
    B.prof_enable(True)
    for _ in range(args.steps):
        B.backward(plan, J, h)
    torch.cuda.synchronize()
    B.prof_enable(False)
    ms_pass, n_pass = B.prof_read("sweep_pass")
    ms_bwd, n_bwd = B.prof_read("sweep_backward")
    ms_red, n_red = B.prof_read("final_reduce")

    dt = t1 - t0
    ms_per_step = dt * 1e3 / args.steps
    solves = batch * args.steps / dt
    # algorithmic max-plus work of one step (forward sweep + final reduction)
    ops_step = 2.0 * info["terms"] * batch
    ops_pass = 2.0 * (info["terms"] - info["reduce_terms"]) * batch * args.steps
    achieved = ops_pass / (ms_pass * 1e-3) if ms_pass > 0 else 0.0
    out = {
        "metric": METRIC,
        "value": solves,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "square16x16_gauss_h_b64", "L": L, "batch": batch, "couplings": "N(0,1) fp32",
                   "fields": "N(0,0.1^2) fp32", "outputs": "E*, sigma, dE/dJ, dE/dh", "parallelism": "single GPU"},
        "maxplus_gops": ops_step * args.steps / dt / 1e9,
        "valu_frac": ops_step * args.steps / dt / VALU_PEAK_OPS,
        "roofline": {"kernel": "k_pass", "bound": "alu", "achieved": achieved / 1e12,
                     "peak": VALU_PEAK_OPS / 1e12, "unit": "TFLOP/s", "frac": achieved / VALU_PEAK_OPS,
                     "traffic": K_PASS_TRAFFIC_BYTES.get(tile_bits),
                     "avg_launch_ms": ms_pass / max(n_pass, 1), "launches": n_pass,
                     # the batch runs in parts on concurrent streams: each launch does its part's
                     # work, so the whole-step rate (valu_frac) exceeds the per-launch one
                     "concurrent_parts": round(n_pass / max(args.steps, 1) / max(info["n_passes"], 1))},
        "kernel_ms_per_step": {"sweep_pass": ms_pass / args.steps, "sweep_backward": ms_bwd / args.steps,
                               "final_reduce": ms_red / args.steps},
        "plan": {"width": info["width"], "passes": info["n_passes"], "terms_per_instance": info["terms"],
                 "tile_bits": tile_bits},
    }
    if args.headline_only:
        print(json.dumps(out))
        return
    # context, outside the timed region: the same shape with J = +-1 (the metric's
    # name), and the batch solved as 64 one-instance calls
    extra_steps = max(1, min(args.steps, 10))
    pm1 = I.config_instances(0, batch=batch, L=L)
    Jp = torch.tensor(np.stack([x.J for x in pm1]), device=dev)
    pplan = B.Plan(n, pm1[0].edges, order=list(range(n)))
    B.backward(pplan, Jp)
    B.backward(pplan, Jp)
    t_pm1 = _timed(lambda: B.backward(pplan, Jp), extra_steps)
    rows = [(J[b:b + 1].contiguous(), h[b:b + 1].contiguous()) for b in range(batch)]

    def one_by_one():
        for jb, hb in rows:
            B.backward(plan, jb, hb)
    B.graphs_enable(False)   # the plain path: eager launches, one instance per call
    one_by_one()
    t_single = _timed(one_by_one, extra_steps)
    B.graphs_enable(True)
    out["context"] = {"pm1_int32_h0_solves_s": batch / t_pm1, "one_instance_per_call_solves_s": batch / t_single}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(insts)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
