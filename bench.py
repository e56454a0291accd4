"""Benchmark of the headline workload: ground states (energy + configuration)
of 64 seeded 16x16 open square-lattice Ising spin glasses with couplings
J = +-1 (int32) and h = 0, in one batch (the workload the solves/s metric
names). The same shape with Gaussian couplings and fields is timed as a
second figure.

One step = the whole hot path on one batch: the input check, the max-plus
sweep (all passes, the final maximum fused into the last one) and the
argmax-routing backward that returns sigma and dE/dJ. Inputs are resident in
HBM before timing starts.

Work is counted as max-plus ops = 2 x contraction terms + elementwise ops
(a gate is a contraction with K = 2: two terms per output entry; diagonal and
field absorbs, cuts and the final maximum are one op per entry), from the
plan's own counts at the live width of every step (for a half-state plan the
entries its passes visit).

Without fields the half-state plan (z2: the energy is even under flipping all
spins, so half of every state is stored) and the full-state plan are both
autotuned and the faster is timed; the JSON line says which. The steps are
timed one after another on one stream, and going round two, three or four
plans of the chosen configuration on as many streams (batches in flight, so
that one batch's walk and passes overlap the next batches' passes); the
fastest schedule is the measured figure and the line gives all four.

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
# HBM bytes per launch of the pass kernel, by workload and tile size, from
# rocprofv3 FETCH_SIZE / WRITE_SIZE counter runs scaled by a plain device copy
# (the summary and its commands are in this file).
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_pass_traffic.json")


def pass_traffic(workload, tile_bits, parts):
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
        return t[workload][f"tile{tile_bits}_parts{parts}"]["bytes_per_launch"]
    except (OSError, KeyError, ValueError):
        return None


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def _oracle_solve(args):
    """One instance by the oracle (its process runs single-threaded numpy)."""
    from oracle import spinglass as O
    n, edges, J, h = args
    O.eliminate(n, edges, J, h, order=list(range(n)))
    return 1


def cpu_baseline(insts, seconds=10.0, workers=16):
    """The oracle as it stands, on bounded samples of the same workload: one
    thread, then `workers` processes (the machine's CPU share) over the batch."""
    import multiprocessing as mp
    n = insts[0].n
    work = [(n, x.edges, x.J, x.h) for x in insts]
    t0 = time.perf_counter()
    done = 0
    while time.perf_counter() - t0 < seconds:
        _oracle_solve(work[done % len(work)])
        done += 1
    t1 = time.perf_counter() - t0
    single = done / t1
    workers = max(1, min(workers, os.cpu_count() or 1))
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        pool.map(_oracle_solve, work[:workers])        # start-up outside the timing
        t0 = time.perf_counter()
        rounds = 0
        while True:
            pool.map(_oracle_solve, work)
            rounds += 1
            if time.perf_counter() - t0 > seconds / 2:
                break
        t2 = time.perf_counter() - t0
    model, ncpu = host_cpu()
    return {"value": rounds * len(work) / t2, "unit": "solves/s", "cores": workers, "kind": "oracle",
            "sample": f"{rounds} x the {len(work)} instances over {workers} processes in {t2:.1f} s; "
                      f"single thread: {done} instances in {t1:.1f} s",
            "single_thread": {"value": single, "unit": "solves/s", "cores": 1},
            "host": {"cpu_model": model, "nproc": ncpu},
            "method": "numpy max-sum bucket elimination (raster order) with traceback, int64 / float64"}


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
    # the same solve with int16 couplings (int16 state, as the paper's Int16 chimera sweep)
    J16 = J.to(torch.int16)
    tile16, _ = B.autotune(plan, J16, config=True)
    E16, sig16, _, _ = B.backward(plan, J16)
    assert float(E16[0].item()) == float(E[0].item())
    t_solve16 = _timed(lambda: B.backward(plan, J16), steps)
    plan.close()
    # h = 0: the same solve and count on the half state (2^31 stored entries)
    hplan = B.Plan(512, x.edges, chimera=(8, 8), z2=True)
    htile, _ = B.autotune(hplan, J, config=True)
    Eh, _, _, _ = B.backward(hplan, J)
    assert float(Eh[0].item()) == float(E[0].item())
    t_half = _timed(lambda: B.backward(hplan, J), steps)
    htile16, _ = B.autotune(hplan, J16, config=True)
    B.backward(hplan, J16)
    t_half16 = _timed(lambda: B.backward(hplan, J16), steps)
    B.count(hplan, J)
    t0 = time.perf_counter()
    Ech, _, gh = B.count(hplan, J)
    t_count_half = time.perf_counter() - t0
    hplan.close()
    cplan = B.Plan(512, x.edges, chimera=(8, 8))
    B.count(cplan, J)   # first call: device buffers (about 150 GB with four residue planes)
    t0 = time.perf_counter()
    Ec, res, g = B.count(cplan, J)
    t_count = time.perf_counter() - t0
    cplan.close()
    assert int(Ech[0]) == int(Ec[0]) and gh[0] == g[0]
    print(json.dumps({"metric": "chimera 8x8 ground state (energy + configuration) wall time",
                      "value": min(t_solve, t_half), "full_state_s": t_solve,
                      "unit": "s", "higher_is_better": False, "steps": steps, "dtype": "f32 (integer-valued)",
                      "config": {"workload": "chimera8x8_pm1", "spins": 512, "couplers": int(len(x.edges)), "tile_bits": tile_bits,
                                 "half_state": t_half < t_solve},
                      "energy": float(E[0].item()), "int16_couplings_s": t_solve16, "int16_tile_bits": tile16,
                      "half_state_s": t_half, "half_state_tile_bits": htile,
                      "half_state_int16_s": t_half16, "half_state_int16_tile_bits": htile16,
                      "count_s": t_count, "count_half_state_s": t_count_half, "count_energy": int(Ec[0]),
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
    # the count on the half state (h = 0: every (x, n) state is even under
    # flipping all spins, half of it is stored and swept) is the timed value;
    # the full-state count is the second figure
    hplan = B.Plan(1024, x.edges, order=list(range(1024)), z2=True)
    B.count(hplan, J)
    B.prof_reset()
    B.prof_enable(True)
    t0 = time.perf_counter()
    Ec, res, g = B.count(hplan, J)
    dt = time.perf_counter() - t0
    B.prof_enable(False)
    kern = {k: B.prof_read(k) for k in ("count_pass", "count_reduce")}
    B.count(plan, J)
    t0 = time.perf_counter()
    Ef, _, gf = B.count(plan, J)
    dt_full = time.perf_counter() - t0
    assert int(Ef[0]) == int(Ec[0]) and gf[0] == g[0]
    t_e = _timed(lambda: B.contract(plan, J), max(1, min(args.steps, 5)))
    # the same energy with int16 couplings: int16 state, packed 16-bit passes
    J16 = J.to(torch.int16)
    E16 = B.contract(plan, J16)
    assert int(E16.cpu().numpy()[0]) == int(Ec[0])
    t_e16 = _timed(lambda: B.contract(plan, J16), max(1, min(args.steps, 5)))
    # the energy on the half-state plan
    Eh, Eh16 = B.contract(hplan, J), B.contract(hplan, J16)
    assert float(Eh.cpu().numpy()[0]) == int(Ec[0]) and int(Eh16.cpu().numpy()[0]) == int(Ec[0])
    t_h = _timed(lambda: B.contract(hplan, J), max(1, min(args.steps, 5)))
    t_h16 = _timed(lambda: B.contract(hplan, J16), max(1, min(args.steps, 5)))
    # a ground state and dE/dJ on the half-state plan with int16 couplings:
    # every pass input would need about 0.5 TB, so the backward keeps the
    # snapshots that fit (4 GiB each) and recomputes the rest; the other
    # plans' device states are released first so that the snapshots get the
    # memory
    plan.close()
    hplan.close()
    torch.cuda.empty_cache()
    gplan = B.Plan(1024, x.edges, order=list(range(1024)), z2=True)
    Eg = B.backward(gplan, J16)[0]   # the first call allocates the snapshots
    assert int(Eg.cpu().numpy()[0]) == int(Ec[0])
    B.prof_reset()
    B.prof_enable(True)
    t_gs = _timed(lambda: B.backward(gplan, J16), 2)
    B.prof_enable(False)
    kern_gs = {k: B.prof_read(k)[0] / 2 for k in ("sweep_pass", "final_reduce", "sweep_backward")}
    gplan.close()
    print(json.dumps({"metric": "32x32 +-J ground-state energy and degeneracy wall time", "value": dt, "unit": "s",
                      "higher_is_better": False, "dtype": "f32 (integer-valued) + 3 x u64 residues",
                      "config": {"workload": "square32_pm1_count", "spins": 1024, "half_state": True},
                      "energy": int(Ec[0]), "degeneracy": str(g[0]), "entropy_per_spin": math.log(g[0]) / 1024,
                      "full_state_count_s": dt_full,
                      "energy_only_s": t_e, "energy_only_int16_s": t_e16,
                      "energy_only_half_state_s": t_h, "energy_only_half_state_int16_s": t_h16,
                      "ground_state_half_state_int16_recompute_s": t_gs,
                      "ground_state_kernel_ms": kern_gs,
                      "kernel_ms": {k: v[0] for k, v in kern.items()}}))


def bench_uneven(args):
    """16 random 3-regular graphs, N = 100 + 20 (i mod 7), J ~ N(0, 1), h = 0, greedy
    orders (2048 randomised greedy trials per graph: the widest graphs come out
    two or three spins narrower than with the default 32, i.e. four to eight
    times less work), tile sizes autotuned per plan: energy + configuration of
    all 16 in one call (grouped launches) against one call per instance."""
    import torch

    from paper_2008_06888_amd import binding as B
    from paper_2008_06888_amd import instances as I
    insts = I.config_instances(3)
    t0 = time.perf_counter()
    plans = [B.Plan(x.n, x.edges, seed=i, trials=2048) for i, x in enumerate(insts)]
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
    t_full = _timed(lambda: B.contract_uneven(plans, Js), steps)
    # h = 0: the same instances on half-state plans (same orders), the faster is the value
    hplans = [B.Plan(x.n, x.edges, order=p.order().tolist(), z2=True) for x, p in zip(insts, plans)]
    htiles = [B.autotune(p, j[None], config=True)[0] for p, j in zip(hplans, Js)]
    Ef = B.contract_uneven(plans, Js)[0].cpu().numpy()
    Eh = B.contract_uneven(hplans, Js)[0].cpu().numpy()
    assert abs(Ef - Eh).max() <= 1e-5 * max(x.n for x in insts)
    t_half = _timed(lambda: B.contract_uneven(hplans, Js), steps)
    half = t_half < t_full
    t_batched = min(t_full, t_half)
    best = hplans if half else plans

    def one_by_one():
        for p, j in zip(best, Js):
            B.backward(p, j[None])
    t_single = _timed(one_by_one, steps)
    widths = [p.info()["width"] for p in plans]
    print(json.dumps({"metric": "uneven batch ground states (energy + configuration) solves/s",
                      "value": len(insts) / t_batched, "unit": "solves/s", "higher_is_better": True,
                      "steps": steps, "dtype": "f32",
                      "config": {"workload": "reg3_uneven_b16", "n": [x.n for x in insts], "widths": widths,
                                 "half_state": half},
                      "one_call_per_instance_solves_s": len(insts) / t_single, "planning_s": t_plan,
                      "full_state_solves_s": len(insts) / t_full, "half_state_solves_s": len(insts) / t_half,
                      "tile_bits": htiles if half else tiles, "autotune_s": t_tune}))


def bench_potts(args):
    """3-state Potts glasses (App. C) on the open 18 x 18 lattice, J = +-1: ground-state
    energy of a batch of instances (timed steps), then energy and exact degeneracy of
    one instance (the paper's energy-and-entropy run)."""
    import numpy as np
    import torch

    from paper_2008_06888_amd import binding as B
    from paper_2008_06888_amd import instances as I
    L, batch = 18, 4
    insts = I.potts_lattice(L, batch=batch)
    n = L * L
    plan = B.Plan(n, insts[0].edges, order=list(range(n)), q=3)
    info = plan.info()
    J = torch.tensor(np.stack([x.J for x in insts]), device="cuda:0")
    steps = max(1, min(args.steps, 10))
    for _ in range(max(1, min(args.warmup, 2))):
        B.potts_contract(plan, J)
    t = _timed(lambda: B.potts_contract(plan, J), steps)
    B.prof_reset()
    B.prof_enable(True)
    for _ in range(steps):
        B.potts_contract(plan, J)
    torch.cuda.synchronize()
    B.prof_enable(False)
    ms, launches = B.prof_read("potts_pass")
    E = B.potts_contract(plan, J).cpu().numpy()
    # HBM roofline of the pass kernel: every pass reads and writes the whole state once
    state_bytes = batch * 3 ** info["width"] * 4
    per_launch = 2 * state_bytes
    avg_ms = ms / max(launches, 1)
    achieved = per_launch / (avg_ms * 1e-3) if ms > 0 else 0.0
    ops = 2 * info["terms"] + info["elementwise"]
    J1 = J[:1].contiguous()
    B.potts_count(plan, J1)
    t0 = time.perf_counter()
    E2, _, g, exact = B.potts_count(plan, J1, flags=True)
    t_count = time.perf_counter() - t0
    print(json.dumps({"metric": "3-state Potts 18x18 ground-state energy solves/s", "value": batch / t,
                      "unit": "solves/s", "higher_is_better": True, "steps": steps, "dtype": "f32 (doubled energies, integer-valued)",
                      "config": {"workload": "potts18x18_pm1", "spins": n, "batch": batch, "width_digits": info["width"],
                                 "passes": info["n_passes"], "count_passes": info["n_count_passes"]},
                      "s_per_batch": t, "energies": [float(e) for e in E],
                      "maxplus_gops": ops * batch / t / 1e9,
                      "roofline": {"kernel": "k_potts_pass", "bound": "hbm", "achieved": achieved / 1e9,
                                   "peak": 8000.0, "unit": "GB/s", "frac": achieved / 8e12, "traffic": None,
                                   "avg_launch_ms": avg_ms, "launches": launches, "bytes_per_launch": per_launch},
                      "count": {"s": t_count, "energy": int(E2[0]) / 2, "degeneracy": str(g[0]), "exact": bool(exact[0]),
                                "entropy_per_spin": math.log(g[0]) / n}}))


def bench_cubic(args):
    """6 x 6 x 6 open cubic lattice (216 spins), J = +-1, h = 0: ground-state energy and
    configuration (tt_backward), and the exact degeneracy."""
    import numpy as np
    import torch

    from paper_2008_06888_amd import binding as B
    from paper_2008_06888_amd import instances as I
    x = I.cubic_instances(6)[0]
    J = torch.tensor(x.J[None], device="cuda:0")
    t0 = time.perf_counter()
    plan = B.Plan(216, x.edges, seed=0)
    t_plan = time.perf_counter() - t0
    info = plan.info()
    steps = max(1, min(args.steps, 5))
    B.backward(plan, J)
    t_solve = _timed(lambda: B.backward(plan, J), steps)
    t_energy = _timed(lambda: B.contract(plan, J), steps)
    E, sig, _, _ = B.backward(plan, J)
    hplan = B.Plan(216, x.edges, seed=0, z2=True)
    Eh, sh, _, _ = B.backward(hplan, J)
    assert float(Eh[0].item()) == float(E[0].item())
    t_half = _timed(lambda: B.backward(hplan, J), steps)
    B.count(hplan, J)
    t0 = time.perf_counter()
    Ech, _, gh, exh = B.count_with_flags(hplan, J)
    t_count_half = time.perf_counter() - t0
    hplan.close()
    B.count(plan, J)
    t0 = time.perf_counter()
    Ec, _, g, exact = B.count_with_flags(plan, J)
    t_count = time.perf_counter() - t0
    assert int(Ech[0]) == int(Ec[0]) and gh[0] == g[0]
    print(json.dumps({"metric": "6x6x6 +-J ground state (energy + configuration) wall time",
                      "value": min(t_solve, t_half),
                      "unit": "s", "higher_is_better": False, "steps": steps, "dtype": "f32 (integer-valued)",
                      "config": {"workload": "cubic6_pm1", "spins": 216, "couplers": int(len(x.edges)),
                                 "width": info["width"], "passes": info["n_passes"], "planning_s": t_plan,
                                 "half_state": t_half < t_solve},
                      "full_state_s": t_solve,
                      "energy": float(E[0].item()), "energy_only_s": t_energy, "half_state_s": t_half,
                      "count_s": t_count, "count_half_state_s": t_count_half,
                      "count_energy": int(Ec[0]), "degeneracy": str(g[0]), "exact": bool(exact[0]),
                      "entropy_per_spin": math.log(g[0]) / 216}))


def bench_pass_profile(args):
    """The headline batch's energy passes alone (tt_contract, one part, tile 2^bits),
    `steps` calls: a clean per-launch shape for kernel traces and counter runs."""
    import numpy as np
    import torch

    from paper_2008_06888_amd import binding as B
    from paper_2008_06888_amd import instances as I
    L, batch = 16, args.pass_batch
    pm1 = I.config_instances(0, batch=batch, L=L)
    J = torch.tensor(np.stack([x.J for x in pm1]), device="cuda:0")
    if args.i16:
        J = J.to(torch.int16)
    plan = B.Plan(L * L, pm1[0].edges, order=list(range(L * L)), tile_bits=args.pass_profile, parts=1,
                  z2=args.half)
    for _ in range(max(args.warmup, 1)):
        B.contract(plan, J)
    torch.cuda.synchronize()
    B.prof_reset()
    B.prof_enable(True)
    for _ in range(args.steps):
        B.contract(plan, J)
    torch.cuda.synchronize()
    B.prof_enable(False)
    ms, launches = B.prof_read("sweep_pass")
    print(json.dumps({"workload": f"square16x16_pm1_b{batch} energy passes", "tile_bits": args.pass_profile,
                      "couplings": str(J.dtype).replace("torch.", ""), "half_state": args.half,
                      "passes": plan.info()["n_passes"], "launches": launches,
                      "avg_launch_ms": ms / max(launches, 1)}))


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
    ap.add_argument("--pass-profile", type=int, default=0, metavar="BITS",
                    help="instead: only the headline batch's energy passes at tile 2^BITS, one part (profiling)")
    ap.add_argument("--pass-batch", type=int, default=64, help="with --pass-profile: lattices per call")
    ap.add_argument("--i16", action="store_true", help="with --pass-profile: int16 couplings (TT_I16)")
    ap.add_argument("--half", action="store_true", help="with --pass-profile: half-state plan (z2)")
    ap.add_argument("--workload", default="square16_pm1_b64",
                    choices=["square16_pm1_b64", "chimera8x8_pm1", "square32_pm1_count", "reg3_uneven_b16",
                             "potts18_pm1", "cubic6_pm1"],
                    help="the headline workload (default) or one of the other measured cases")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    if args.tgemm:
        return bench_tgemm(args)
    if args.copy_calibration:
        return copy_calibration(args)
    if args.pass_profile:
        return bench_pass_profile(args)
    if args.workload == "chimera8x8_pm1":
        return bench_chimera(args)
    if args.workload == "square32_pm1_count":
        return bench_square32(args)
    if args.workload == "reg3_uneven_b16":
        return bench_uneven(args)
    if args.workload == "potts18_pm1":
        return bench_potts(args)
    if args.workload == "cubic6_pm1":
        return bench_cubic(args)

    import numpy as np
    import torch

    from paper_2008_06888_amd import binding as B
    from paper_2008_06888_amd import instances as I

    L, batch = 16, 64
    n = L * L
    dev = torch.device("cuda:0")
    pm1 = I.config_instances(0, batch=batch, L=L)          # J = +-1 int32, h = 0
    J = torch.tensor(np.stack([x.J for x in pm1]), device=dev)
    line = run_lattice(args, B, pm1[0].edges, n, J, None, "square16x16_pm1_b64")
    out = {
        "metric": METRIC,
        "value": line["solves_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": line["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "square16x16_pm1_b64", "L": L, "batch": batch, "couplings": "+-1 int32 (exact "
                   "integers in the float32 state)", "fields": "none (h = 0)", "outputs": "E*, sigma, dE/dJ",
                   "half_state": line["plan"]["half_state"], "batches_in_flight": line["batches_in_flight"],
                   "parallelism": "single GPU"},
        "schedules": line["schedules"],
        "maxplus_gops": line["maxplus_gops"],
        "valu_frac": line["valu_frac"],
        "roofline": line["roofline"],
        "roofline_one_part": line["roofline_one_part"],
        **({"full_state": line["full_state"]} if "full_state" in line else {}),
        "kernel_ms_per_step": line["kernel_ms_per_step"],
        "plan": line["plan"],
    }
    if args.headline_only:
        print(json.dumps(out))
        return
    # second figure: the same shape with Gaussian couplings and fields (float32)
    gauss = I.config_instances(1)
    Jg = torch.tensor(np.stack([x.J for x in gauss]), device=dev)
    hg = torch.tensor(np.stack([x.h for x in gauss]), device=dev)
    gl = run_lattice(args, B, gauss[0].edges, n, Jg, hg, "square16x16_gauss_h_b64")
    out["gauss_h_b64"] = {k: gl[k] for k in ("solves_s", "ms_per_step", "batches_in_flight", "schedules",
                                             "maxplus_gops", "valu_frac", "roofline", "kernel_ms_per_step", "plan")}
    out["gauss_h_b64"]["outputs"] = "E*, sigma, dE/dJ, dE/dh"
    # the plain path: the same 64 +-J instances, one eager call each
    plan1 = B.Plan(n, pm1[0].edges, order=list(range(n)), tile_bits=line["plan"]["tile_bits"],
                   z2=line["plan"]["half_state"])
    rows = [J[b:b + 1].contiguous() for b in range(batch)]
    extra_steps = max(1, min(args.steps, 10))

    def one_by_one():
        for jb in rows:
            B.backward(plan1, jb)
    B.graphs_enable(False)
    one_by_one()
    t_single = _timed(one_by_one, extra_steps)
    B.graphs_enable(True)
    out["context"] = {"one_instance_per_call_solves_s": batch / t_single}
    # the same batch with int16 couplings (TT_I16: int16 state, packed 16-bit passes)
    li = run_lattice(args, B, pm1[0].edges, n, J.to(torch.int16), None, "square16x16_pm1_b64_i16")
    out["context"]["int16_couplings"] = {k: li[k] for k in ("solves_s", "ms_per_step", "batches_in_flight",
                                                            "schedules", "kernel_ms_per_step", "plan")}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(pm1)
    print(json.dumps(out))


def run_lattice(args, B, edges, n, J, h, workload):
    """Times tt_backward (E*, sigma and the gradients) on one batch: the autotuned
    plan, `steps` timed calls, then the same calls with per-launch kernel timing,
    and once more with the batch in one part (no concurrent halves)."""
    import torch
    batch = J.shape[0]
    has_h = h is not None
    plan = B.Plan(n, edges, order=list(range(n)), has_field=has_h)
    tile_bits, _ = B.autotune(plan, J, h, config=True)
    fbits = tile_bits
    half = False
    trial = {}
    full_plan = plan
    if not has_h:
        # without fields a half-state plan (z2) is the other candidate: both
        # autotuned, the faster over a few timed calls is the one measured
        hplan = B.Plan(n, edges, order=list(range(n)), z2=True)
        hbits, _ = B.autotune(hplan, J, None, config=True)
        for _ in range(2):
            B.backward(plan, J)
            B.backward(hplan, J)
        trial = {"full_state_ms": _timed(lambda: B.backward(plan, J), 20) * 1e3,
                 "half_state_ms": _timed(lambda: B.backward(hplan, J), 20) * 1e3}
        if trial["half_state_ms"] < trial["full_state_ms"]:
            plan, tile_bits, half = hplan, hbits, True
    info = plan.info()
    for _ in range(max(args.warmup, 2)):
        B.backward(plan, J, h)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        B.backward(plan, J, h)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    # batches in flight: k plans of the chosen configuration, each on a
    # stream of its own, consecutive steps going round them, so that one
    # batch's walk (one workgroup per instance) and passes overlap the next
    # batches' passes; every step still solves a whole batch. The streams are
    # k consecutive ones of torch's pool, not the current stream: the pool's
    # streams take the device's hardware queues in turn, so consecutive ones
    # (up to the number of queues, four) run on different queues, while
    # the current stream may share its queue with one of them
    def in_flight(k):
        torch.cuda.synchronize()
        streams = [torch.cuda.Stream() for _ in range(k)]
        ring = [(plan if j == 0 else B.Plan(n, edges, order=list(range(n)), has_field=has_h, tile_bits=tile_bits,
                                           parts=info["parts"], z2=half), streams[j]) for j in range(k)]

        def step(i):
            p, st = ring[i % k]
            with torch.cuda.stream(st):
                B.backward(p, J, h)
        for i in range(max(args.warmup, 2) * k):
            step(i)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for i in range(args.steps):
            step(i)
        torch.cuda.synchronize()
        t = time.perf_counter() - t
        for p, _ in ring[1:]:
            p.close()
        return t
    dt_k = {1: dt, 2: in_flight(2), 3: in_flight(3), 4: in_flight(4)}

    def kernel_times(p, steps):
        B.prof_reset()
        B.prof_enable(True)
        for _ in range(steps):
            B.backward(p, J, h)
        torch.cuda.synchronize()
        B.prof_enable(False)
        return {k: B.prof_read(k) for k in ("sweep_pass", "sweep_backward", "final_reduce", "check_inputs")}

    kt = kernel_times(plan, args.steps)
    one = B.Plan(n, edges, order=list(range(n)), has_field=has_h, tile_bits=tile_bits, parts=1, z2=half)
    B.backward(one, J, h)
    kt1 = kernel_times(one, args.steps)
    large = (batch << info["width"]) >= (1 << 20)

    def work(inf):
        # max-plus ops per step (the final maximum runs inside the last pass)
        return (2.0 * inf["terms"] + inf["elementwise"]) * batch

    def roof(k, nparts, ops_step, is_half, tb):
        ms, launches = k["sweep_pass"]
        per_launch = ops_step * args.steps / max(launches, 1)
        avg_ms = ms / max(launches, 1)
        ach = per_launch / (avg_ms * 1e-3) if ms > 0 else 0.0
        return {"kernel": "k_pass", "bound": "alu", "achieved": ach / 1e12, "peak": VALU_PEAK_OPS / 1e12,
                "unit": "TFLOP/s", "frac": ach / VALU_PEAK_OPS,
                "traffic": pass_traffic(workload + ("_half" if is_half else ""), tb, nparts),
                "avg_launch_ms": avg_ms, "launches": launches, "ops_per_launch": per_launch,
                "concurrent_parts": nparts}

    ops_inst = work(info) / batch
    ops_step = work(info)
    parts = info["parts"] if (large and batch >= 2) else 1   # the autotuner may have chosen one part
    r = roof(kt, parts, ops_step, half, tile_bits)
    if parts > 1:
        r["note"] = ("each launch is half a pass and runs beside the other half's launch; the whole-step "
                     "rate is valu_frac, the unsplit per-launch rate roofline_one_part")
    if half:
        r["note_half_state"] = ("a half-state pass computes half of the entries: its ops per launch are half "
                                "those of the full-state pass (full_state holds that plan's figures)")
    extra = {}
    if half:
        # the full-state plan of the same batch, as measured in the selection
        fi = full_plan.info()
        fparts = fi["parts"] if (large and batch >= 2) else 1
        extra["full_state"] = {"ms_per_step": trial["full_state_ms"],
                               "solves_s": batch / (trial["full_state_ms"] * 1e-3),
                               "roofline": roof(kernel_times(full_plan, args.steps), fparts, work(fi), False,
                                                fbits),
                               "plan": {"tile_bits": fbits, "parts": fparts, "passes": fi["n_passes"]}}
    # the measured figure is that of the fastest schedule
    schedules = {f"{k}_in_flight": {"solves_s": batch * args.steps / t, "ms_per_step": t * 1e3 / args.steps}
                 for k, t in dt_k.items()}
    n_flight = min(dt_k, key=dt_k.get)
    dt = dt_k[n_flight]
    return {
        "solves_s": batch * args.steps / dt,
        "ms_per_step": dt * 1e3 / args.steps,
        "batches_in_flight": n_flight,
        "schedules": schedules,
        "maxplus_gops": ops_step * args.steps / dt / 1e9,
        "valu_frac": ops_step * args.steps / dt / VALU_PEAK_OPS,
        "roofline": r,
        "roofline_one_part": roof(kt1, 1, ops_step, half, tile_bits),
        **extra,
        "kernel_ms_per_step": {k: v[0] / args.steps for k, v in kt.items()},
        "plan": {"width": info["width"], "passes": info["n_passes"], "tile_bits": tile_bits,
                 "half_state": half, "parts": parts, "terms_per_instance": info["terms"],
                 "elementwise_per_instance": info["elementwise"], "maxplus_ops_per_instance": ops_inst,
                 **({"selection": trial} if trial else {})},
    }


if __name__ == "__main__":
    main()
