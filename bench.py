#!/usr/bin/env python3
"""Benchmark of the simulation hot path on one MI355X.

Default workload: a 30-qubit complex64 circuit of 200 Haar-random dense
blocks (k ~ U{2..6} on seeded qubit subsets, seed 2).  One step = |x0> initialisation
(which also resets the qubit layout), one run of the whole fused plan over the
2^30-amplitude state (tile passes with vector-ALU and matrix-core blocks),
then the FP64 <Z_i> reduction.  The plan is
built once before the timed region (its host time is reported as plan_s).

Prints ONE JSON line.  `value` is the step's algorithmic HBM throughput
(sum over passes of 2 * 2^n * 8 bytes, plus the 2^n * 8 bytes the reduction
reads, divided by the step time).  The roofline object describes the kernel
that takes most of the step, timed live with HIP events on the simulator's
stream; the CPU baseline is the FP64 oracle on a bounded sample of the same
circuit.
"""
from __future__ import annotations

import argparse
import gc
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_F32_PEAK_TFLOPS = 157.3
MFMA_F64_PEAK_TFLOPS = 78.6
# vector ALU: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz, the
# rate of unpacked FP32 and of FP64 FMAs (the library builds without packed
# FP32 instructions)
VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
MATRIX_KERNELS = ("tile_lds_kernel", "state_lds_kernel")
PASS_NAMES = {0: "tile_pass_kernel", 1: "tile_lds_kernel", 2: "state_lds_kernel", 3: "sweep_kernel",
              4: "swap_bits_kernel"}


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("kernels.hip", "planner.cpp"):
        with open(os.path.join(ROOT, "paper_2410_09326_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def make_workload(name: str):
    from workloads import circuits as W
    if name == "haar30":
        c = W.haar_blocks(2, n=30, nblocks=200)
        return c, 0, "30-qubit circuit of 200 Haar-random dense blocks (k~U{2..6}, seed 2), complex64"
    if name == "qft28":
        c = W.qft_then_layers(1, n=28, layers=40)
        return c, 0, "28-qubit QFT of a seeded basis state + 40 random U3/CZ layers, complex64, virtual swaps"
    if name == "haar20":
        c = W.haar_blocks(2, n=20, nblocks=200)
        return c, 0, "20-qubit circuit of 200 Haar-random dense blocks (k~U{2..6}, seed 2), complex64"
    raise SystemExit(f"unknown workload {name}")


def traffic_for(kernel: str, workload: str, launches_bytes: float):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("source_hash") != kernel_source_hash():
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(circ, seconds: float):
    """The FP64 oracle (plain OpenMP loops, one pass per block) on the first
    blocks of the same circuit until `seconds` of work have been done."""
    import numpy as np
    from oracle import oracle as orc
    n = circ.n
    psi = np.zeros(2 ** n, dtype=np.complex128)
    psi[circ.x0] = 1.0
    done = 0
    t0 = time.perf_counter()
    for g in circ.gates:
        u = orc.gate_matrix(g.kind, g.params, dense=g.matrix)
        orc.apply_matrix_inplace(n, psi, u, g.qubits)
        done += 1
        if time.perf_counter() - t0 > seconds:
            break
    el = time.perf_counter() - t0
    bytes_c64 = done * 2.0 * (2 ** n) * 8
    return {"value": bytes_c64 / el / 1e9, "unit": "GB/s", "cores": orc.num_threads(), "kind": "oracle",
            "sample": f"first {done} of {len(circ.gates)} blocks at n={n} in FP64 ({el:.1f} s; bytes counted "
                      f"as the complex64 path's 2*2^n*8 per block)", "seconds": el, "blocks": done}


MODELS = os.path.join(ROOT, "paper_2410_09326_amd", "models")


def learned_vs_plain(n_circ: int):
    """Plans seeded 32-qubit complex64 depth-60 circuits (U3/CZ/SWAP/RZZ
    layers) twice -- priced by the plain cost table fitted to the shipped
    profiling corpus, and by the trained perceptron -- and times both plans on
    the GPU (best of two runs each).  Both runs are checked to agree."""
    import numpy as np
    import torch
    import paper_2410_09326_amd as q
    from workloads import circuits as W
    model = q.CostModel.load(os.path.join(MODELS, "cost_mlp.bin"))
    prof = q.Profile.load(os.path.join(MODELS, "corpus_profile.bin"))
    with open(os.path.join(MODELS, "cost_model_summary.json")) as fh:
        summ = json.load(fh)
    n = 32
    sim = q.Simulator(n, q.C64)
    t_plain = t_learned = t_fused = 0.0
    detail = []
    for i in range(n_circ):
        c = W.eval_circuit(9000 + i, n=n, depth=60)
        plans = {"plain": q.Plan(n, c.gates, precision=q.C64, mode=q.PLAN_PROFILED, profile=prof),
                 "learned": q.Plan(n, c.gates, precision=q.C64, mode=q.PLAN_LEARNED, model=model),
                 "fused": q.Plan(n, c.gates, precision=q.C64)}
        times, zs = {}, {}
        for name, plan in plans.items():
            best = None
            for _ in range(2):
                sim.init_basis(0)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                sim.run(plan)
                sim.synchronize()
                el = time.perf_counter() - t0
                best = el if best is None else min(best, el)
            zs[name] = sim.expect_z()
            times[name] = best
        agree = float(max(np.max(np.abs(zs["plain"] - zs["learned"])), np.max(np.abs(zs["plain"] - zs["fused"]))))
        t_plain += times["plain"]
        t_learned += times["learned"]
        t_fused += times["fused"]
        detail.append({"seed": 9000 + i, "plain_ms": round(times["plain"] * 1e3, 2),
                       "learned_ms": round(times["learned"] * 1e3, 2), "fused_ms": round(times["fused"] * 1e3, 2),
                       "plain_passes": plans["plain"].stats()["n_passes"],
                       "learned_passes": plans["learned"].stats()["n_passes"],
                       "plain_predicted_ms": round(plans["plain"].stats()["predicted_s"] * 1e3, 2),
                       "learned_predicted_ms": round(plans["learned"].stats()["predicted_s"] * 1e3, 2),
                       "max_abs_expz_diff": agree})
    sim.close()
    return {"workload": "32-qubit complex64 random U3/CZ/SWAP/RZZ layers, depth 60 (seeds 9000+)",
            "speedup": round(t_plain / t_learned, 4), "plain_ms": round(t_plain * 1e3, 2),
            "learned_ms": round(t_learned * 1e3, 2), "fused_heuristic_ms": round(t_fused * 1e3, 2),
            "heldout_mape_learned": round(summ["mape_learned"], 4), "heldout_mape_plain": round(summ["mape_plain"], 4),
            "corpus_passes": summ["passes"], "circuits": detail}


def batch_sweep(reps: int):
    """The parameter-sweep batch: 512 circuits of 10..22 qubits (RY/RZ layers
    plus a CZ ladder, depth 8..32, seed 5) in complex64, all in one graph
    launch producing <Z_i> for every qubit of every circuit.  The autotuner
    picks the whole-state-in-LDS cut-off, the tile width and the block fusion
    width first.  A sample
    of eight circuits is re-run one at a time in complex128 on the
    single-circuit path to state the batch's max-abs error."""
    import tempfile
    import numpy as np
    import paper_2410_09326_amd as q
    from workloads import circuits as W
    circs = W.param_sweep_batch(5)
    spec = [(c.n, q.GateArray(c.gates)) for c in circs]
    cache = os.path.join(tempfile.gettempdir(), "qops_batch_tune.txt")
    t0 = time.perf_counter()
    sm, tb, kf, _ = q.Batch.autotune(spec, precision=q.C64, cache=cache)
    tune_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    b = q.Batch(spec, precision=q.C64, small_max_n=sm, tile_bits=tb, max_fuse_k=kf)
    create_s = time.perf_counter() - t0
    info = b.info()
    b.launch()
    res = b.results()
    sec = b.time(reps)
    b.close()
    err = 0.0
    pick = np.linspace(0, len(circs) - 1, 8).astype(int)
    for i in pick:
        c = circs[i]
        sim = q.Simulator(c.n, q.C128)
        sim.init_basis(0)
        sim.run(q.Plan(c.n, spec[i][1], precision=q.C128))
        err = max(err, float(np.max(np.abs(sim.expect_z() - res[i]))))
        sim.close()
    return {"workload": "512 parameterised circuits, n~U{10..22}, RY/RZ layers + CZ ladder, depth U{8..32} "
                        "(seed 5), complex64, one graph launch, <Z_i> of every qubit",
            "circuits_per_s": round(len(circs) / sec, 1), "launch_ms": round(sec * 1e3, 3),
            "gates": int(sum(len(c.gates) for c in circs)),
            "autotuned": {"small_max_n": sm, "tile_bits": tb, "max_fuse_k": kf, "tune_s": round(tune_s, 2)},
            "create_s": round(create_s, 2), "small_circuits": info["small_circuits"],
            "tile_circuits": info["tile_circuits"], "graph_kernel_nodes": info["graph_nodes"],
            "max_abs_vs_c128_sample": err}


def qaoa_sweep(n: int = 28, layers: int = 3, evals: int = 16):
    """Repeated QAOA Max-Cut runs on a seeded 3-regular weighted graph: the
    plan is built once and re-bound to each new angle set; one evaluation =
    re-bind + |0..0> + the circuit + the edge correlators <Z_a Z_b>, from
    which <C> = sum_e w_e (1 - <Z_a Z_b>) / 2 follows."""
    import numpy as np
    import torch
    import paper_2410_09326_amd as q
    from workloads import circuits as W
    edges, w = W.regular_graph(11, n, 3)
    rng = np.random.default_rng(5)
    sets = [(rng.uniform(0, np.pi, layers), rng.uniform(0, np.pi / 2, layers)) for _ in range(evals + 1)]
    c0 = W.qaoa_maxcut(n, edges, w, *sets[0])
    t0 = time.perf_counter()
    plan = q.Plan(n, c0.gates, precision=q.C64)
    plan_s = time.perf_counter() - t0
    sim = q.Simulator(n, q.C64)
    sim.init_basis(0)
    sim.run(plan)
    sim.expect_zz(edges)
    costs, t_upd = [], 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for gm, bt in sets[1:]:
        c = W.qaoa_maxcut(n, edges, w, gm, bt)
        ga = q.GateArray(c.gates)
        u0 = time.perf_counter()
        plan.update(ga)
        t_upd += time.perf_counter() - u0
        sim.init_basis(0)
        sim.run(plan)
        zz = sim.expect_zz(edges)
        costs.append(float(np.sum(w * (1.0 - zz)) / 2.0))
    el = time.perf_counter() - t0
    sim.close()
    return {"workload": f"QAOA Max-Cut, {n} qubits, p={layers}, seeded 3-regular weighted graph "
                        f"({len(edges)} edges), complex64, {evals} angle sets on one re-bound plan",
            "evals_per_s": round(evals / el, 2), "ms_per_eval": round(el / evals * 1e3, 3),
            "rebind_ms_per_eval": round(t_upd / evals * 1e3, 3), "plan_ms": round(plan_s * 1e3, 3),
            "passes": plan.stats()["n_passes"], "best_cost": round(max(costs), 6),
            "total_weight": round(float(np.sum(w)), 6)}


def main() -> None:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="haar30")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-learned-eval", action="store_true")
    ap.add_argument("--eval-circuits", type=int, default=10)
    ap.add_argument("--no-batch-eval", action="store_true")
    ap.add_argument("--no-qaoa-eval", action="store_true")
    ap.add_argument("--batch-reps", type=int, default=5)
    ap.add_argument("--dump-passes", default="", help="write the last step's pass records (JSON) here")
    ap.add_argument("--trace", default="", help="write the last step's profile as a Chrome trace here")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 2^30 x 8-byte device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this simulator has no multi-GPU path (state sharding is a design "
              "note only); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2410_09326_amd as q

    circ, prec, desc = make_workload(args.workload)
    n = circ.n
    amp = 8 if prec == q.C64 else 16
    t0 = time.perf_counter()
    plan = q.Plan(n, circ.gates, precision=prec)
    plan_s = time.perf_counter() - t0
    st = plan.stats()
    passes = plan.passes()

    sim = q.Simulator(n, prec)
    for _ in range(args.warmup):       # the same work as a timed step
        sim.init_basis(circ.x0)
        sim.profile(plan).records()
        sim.expect_z()
    torch.cuda.synchronize()

    recs_all = []
    gc.collect()
    gc.disable()                       # no collector pauses inside the timed steps
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sim.init_basis(circ.x0)
        prof = sim.profile(plan)          # the plan, with HIP events around every pass
        recs_all.append(prof.records())
        last_prof = prof
        z = sim.expect_z()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    gc.enable()
    ms = el / args.steps * 1e3
    norm = sim.norm()

    if args.copy_calibration:
        a = torch.empty(2 ** 30, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    if args.trace:
        last_prof.trace(args.trace)
    if args.dump_passes:
        with open(args.dump_passes, "w") as fh:
            json.dump({"passes": passes, "records": recs_all[-1]}, fh)

    # per-kernel totals over the timed steps
    per = {}
    for recs in recs_all:
        for r in recs:
            k = PASS_NAMES[r["type"]]
            d = per.setdefault(k, {"seconds": 0.0, "launches": 0, "bytes": 0.0, "flops": 0.0})
            d["seconds"] += r["seconds"]
            d["launches"] += 1
            d["bytes"] += r["bytes_alg"]
            d["flops"] += r["flops"]
    dom = max(per, key=lambda k: per[k]["seconds"])
    d = per[dom]
    avg_s = d["seconds"] / d["launches"]
    bytes_launch = d["bytes"] / d["launches"]
    flops_launch = d["flops"] / d["launches"]
    gbs = bytes_launch / avg_s / 1e9
    tfl = flops_launch / avg_s / 1e12
    if dom in MATRIX_KERNELS:
        cbound, fpeak = "mfma", (MFMA_F32_PEAK_TFLOPS if prec == q.C64 else MFMA_F64_PEAK_TFLOPS)
    else:
        cbound, fpeak = "alu", round(VALU_PEAK_TFLOPS, 1)
    if tfl / fpeak > gbs / HBM_PEAK_GBS:
        roof = {"bound": cbound, "achieved": round(tfl, 2), "peak": fpeak, "unit": "TFLOP/s",
                "frac": round(tfl / fpeak, 4)}
    else:
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4)}
    tr = traffic_for(dom, args.workload, bytes_launch)
    roof["traffic"] = tr
    roof["kernel"] = dom
    roof["launches_per_step"] = d["launches"] // args.steps
    roof["avg_launch_ms"] = round(avg_s * 1e3, 4)
    roof["alg_bytes_per_launch"] = bytes_launch
    roof["alg_flops_per_launch"] = flops_launch

    step_bytes = sum(p["bytes_alg"] for p in passes) + 2 * (2 ** n) * amp   # + init write, reduction read
    value = step_bytes / (ms * 1e-3) / 1e9
    pass_time = sum(r["seconds"] for r in recs_all[-1])
    out = {
        "metric": "circuit wall time + HBM GB/s at 30q c64; learned vs plain plan speedup",
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == q.C64 else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": desc, "n_qubits": n, "gates": len(circ.gates),
                   "passes": st["n_passes"], "plan": "fused"},
        "circuit_ms": round(pass_time * 1e3, 3),
        "plan_s": round(plan_s, 4),
        "norm_error": abs(norm - 1.0),
        "kernels": {k: {"ms_per_step": round(v["seconds"] / args.steps * 1e3, 3),
                        "launches_per_step": v["launches"] // args.steps} for k, v in per.items()},
        "roofline": roof,
    }
    if not args.no_learned_eval:
        sim.close()
        torch.cuda.empty_cache()
        out["learned_vs_plain"] = learned_vs_plain(args.eval_circuits)
    if not args.no_batch_eval:
        out["batch_sweep"] = batch_sweep(args.batch_reps)
    if not args.no_qaoa_eval:
        out["qaoa_sweep"] = qaoa_sweep()
    if not args.no_cpu_baseline:
        cb = cpu_baseline(circ, args.cpu_seconds)
        out["cpu_baseline"] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in cb.items()
                               if k in ("value", "unit", "cores", "kind", "sample")}
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)
    sim.close()


if __name__ == "__main__":
    main()
