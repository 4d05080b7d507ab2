#!/usr/bin/env python3
"""Benchmark of the simulation hot path on one MI355X.

Default workload: a 30-qubit complex64 circuit of 200 Haar-random dense
blocks (k ~ U{2..6} on seeded qubit subsets, seed 2).  One step = |x0> initialisation
(which also resets the qubit layout), one run of the whole fused plan over the
2^30-amplitude state (tile passes with vector-ALU and matrix-core blocks),
then the FP64 <Z_i> reduction.  The plan is
built once before the timed region (its host time is reported as plan_s).

Prints ONE JSON line.  `value` is the step's algorithmic HBM throughput
(sum over passes of 2 * 2^n * 8 bytes, plus the 2^n * 8 bytes the
initialisation writes and the reduction reads, divided by the step time) of
plain (unprofiled) steps.  The same number of profiling-run steps follows:
HIP events around every pass on the simulator's stream give each kernel's
average launch time for the roofline object, and the two step times give
the profiling overhead.  The headline result is compared with a complex128
run of the same circuit (fidelity, max-abs error).  The CPU baseline is the
FP64 oracle on a bounded sample of the same circuit; `oracle_timing` times
the oracle per workload at one thread and at all host threads.
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


def profile_for(kernel: str, workload: str):
    """The committed rocprofv3 summary of `kernel` on `workload` (HBM bytes per
    launch from FETCH_SIZE/WRITE_SIZE, SQ counter figures), if it was taken on
    the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("source_hash") != kernel_source_hash():
        return None
    return d


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
            "speedup": round(t_plain / t_learned, 4),
            "speedup_learned_vs_fused_default": round(t_fused / t_learned, 4),
            "speedup_plain_vs_fused_default": round(t_fused / t_plain, 4),
            "training": "plain table and perceptron fitted to the same profiled training passes",
            "plain_ms": round(t_plain * 1e3, 2),
            "learned_ms": round(t_learned * 1e3, 2), "fused_heuristic_ms": round(t_fused * 1e3, 2),
            "heldout_mape_learned": round(summ["mape_learned"], 4), "heldout_mape_plain": round(summ["mape_plain"], 4),
            "heldout_mape_plain_full_table": round(summ.get("mape_plain_full_table", float("nan")), 4),
            "corpus_passes": summ["passes"], "circuits": detail}


def batch_sweep(reps: int, shape=None):
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
    if shape is None:
        sm, tb, kf, _ = q.Batch.autotune(spec, precision=q.C64, cache=cache)
    else:
        sm, tb, kf = shape
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


def _compare_states(torch, a, b, chunk: int = 1 << 26):
    """Max-abs error, max |b|, fidelity |<b|a>|^2 and relative norm of two
    device states in logical order (a: complex64 or complex128, b: the
    complex128 reference), chunk by chunk on the GPU in FP64."""
    err, amax, ov, nb = 0.0, 0.0, 0.0 + 0.0j, 0.0
    for o in range(0, b.numel(), chunk):
        x = a[o:o + chunk].to(torch.complex128)
        y = b[o:o + chunk]
        err = max(err, float((x - y).abs().max()))
        amax = max(amax, float(y.abs().max()))
        ov += complex(torch.vdot(y, x).item())
        nb += float((y.abs() ** 2).sum())
    return err, amax, abs(ov) ** 2 / nb


def headline_accuracy(q, torch, sim, plan, circ, prec):
    """The headline result against the same circuit in complex128 on the GPU
    (both end in the same layout; the 30-qubit FP64 oracle is checked on a
    prefix of this circuit by the full-size tests).  Also times the complex128
    run."""
    import numpy as np
    n = circ.n
    sim.init_basis(circ.x0)
    sim.run(plan)
    l2p = sim.layout()
    ref = q.Simulator(n, q.C128)
    plan128 = q.Plan(n, circ.gates, precision=q.C128)
    ref.init_basis(circ.x0)
    ref.run(plan128)
    ref.synchronize()
    t0 = time.perf_counter()
    ref.init_basis(circ.x0)
    ref.run(plan128)
    ref.synchronize()
    t128 = time.perf_counter() - t0
    assert np.array_equal(ref.layout(), l2p)
    a = sim.buffer.view(torch.complex64 if prec == q.C64 else torch.complex128)
    b = ref.buffer.view(torch.complex128)
    err, amax, fid = _compare_states(torch, a, b)   # same physical layout on both sides
    ref.close()
    torch.cuda.empty_cache()
    return {"reference": "complex128 run of the same circuit on the GPU", "max_abs": err,
            "max_abs_over_max_amp": err / amax, "one_minus_fidelity": max(0.0, 1.0 - fid),
            "c128_ms": round(t128 * 1e3, 2), "c128_passes": plan128.stats()["n_passes"]}


def swap_modes(reps: int = 3):
    """The 28-qubit QFT of a seeded basis state + 40 random U3/CZ layers with
    its SWAP network handled physically (bit-exchange passes) and virtually
    (layout relabelling), in complex64 and complex128: best-of-`reps` circuit
    wall times, T_phys / T_virt, and the complex64 results against the
    complex128 ones (fidelity, max-abs).  Context (other hardware, a CPU
    storage-based simulator): the paper reports 1.10x at 28 qubits."""
    import numpy as np
    import torch
    import paper_2410_09326_amd as q
    from workloads import circuits as W
    c = W.qft_then_layers(1, n=28, layers=40)
    n = c.n
    res = {"workload": "28-qubit QFT of a seeded basis state (28 H, 378 CP, 14 SWAP) + 40 U3/CZ layers (seed 1)"}
    states, layouts = {}, {}
    for prec, tag in ((q.C64, "c64"), (q.C128, "c128")):
        for mode, mname in ((q.SWAP_PHYSICAL, "physical"), (q.SWAP_VIRTUAL, "virtual")):
            plan = q.Plan(n, c.gates, precision=prec, swap_mode=mode)
            sim = q.Simulator(n, prec)
            best = None
            for _ in range(reps + 1):
                sim.init_basis(c.x0)
                sim.synchronize()
                t0 = time.perf_counter()
                sim.run(plan)
                sim.synchronize()
                el = time.perf_counter() - t0
                best = el if best is None else min(best, el)
            st = plan.stats()
            res[f"{tag}_{mname}_ms"] = round(best * 1e3, 3)
            res[f"{tag}_{mname}_passes"] = st["n_passes"]
            if mname == "virtual":
                res[f"{tag}_virtual_swaps"] = st["n_virtual_swaps"]
            if mname == "physical":
                res[f"{tag}_permute_passes"] = st["n_permute_passes"]
            # c64 and c128 plans of one mode end in the same layout, so the
            # two are compared in physical order
            layouts[(tag, mname)] = sim.layout()
            buf = sim.buffer.view(torch.complex64 if prec == q.C64 else torch.complex128)
            states[(tag, mname)] = buf.clone()
            sim.close()
            del buf
            torch.cuda.empty_cache()
        res[f"{tag}_phys_over_virt"] = round(res[f"{tag}_physical_ms"] / res[f"{tag}_virtual_ms"], 4)
    for mname in ("physical", "virtual"):
        assert np.array_equal(layouts[("c64", mname)], layouts[("c128", mname)])
        err, amax, fid = _compare_states(torch, states[("c64", mname)], states[("c128", mname)])
        res[f"c64_{mname}_vs_c128"] = {"max_abs": err, "max_abs_over_max_amp": err / amax,
                                       "one_minus_fidelity": max(0.0, 1.0 - fid)}
    res["virtual_final_layout_is_reversal"] = bool(np.array_equal(layouts[("c64", "virtual")], np.arange(n)[::-1]))
    states.clear()
    torch.cuda.empty_cache()
    res["paper_context"] = "1.10x at 28 qubits (QFT, CPU + SSD storage-based simulator; Table V)"
    return res


def _host_info():
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    mem = None
    try:
        with open("/proc/meminfo") as fh:
            for line in fh:
                if line.startswith("MemTotal"):
                    mem = round(int(line.split()[1]) / 2 ** 20, 1)
    except OSError:
        pass
    return {"cpu_model": model, "nproc": avail, "os_cpu_count": os.cpu_count(), "mem_gib": mem}


def _oracle_rate(orc, circ, n_eval: int, max_gates: int, budget_s: float):
    """Runs the oracle on the first gates of `circ` whose qubits all lie
    below n_eval (all of them when n_eval = circ.n), on an n_eval-qubit
    state, until `budget_s` elapse or `max_gates` are done; returns (gates
    done, seconds, amplitude-gate updates per second)."""
    import numpy as np
    psi = np.zeros(2 ** n_eval, dtype=np.complex128)
    psi[0] = 1.0
    done, t0 = 0, time.perf_counter()
    for g in circ.gates[:max_gates]:
        qs = tuple(g.qubits)
        if max(qs) >= n_eval or g.controls:
            continue
        u = orc.gate_matrix(g.kind, g.params, dense=g.matrix)
        orc.apply_matrix_inplace(n_eval, psi, u, qs)
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    el = time.perf_counter() - t0
    return done, el, done * (2 ** n_eval) / el


def oracle_timing(out, cb=None):
    """The FP64 oracle per workload, at one thread and at all host threads,
    next to the GPU's time for the same workload:
    * 12-qubit layered U3/CNOT circuit with SWAPs (complex128): in full;
    * 28-qubit QFT + layers and the 30-qubit Haar-block benchmark: per-gate
      rates on samples (all threads: the first gates at full size; one
      thread: the same gate sequence on 22 qubits, where the state is 64 MiB),
      extrapolated to the whole circuit at full size by amplitude count.  The
      all-thread sample of the benchmark circuit is the CPU-baseline run
      `cb` when given."""
    import numpy as np
    import torch
    import paper_2410_09326_amd as q
    from oracle import oracle as orc
    from workloads import circuits as W
    host = _host_info()
    all_threads = orc.num_threads()
    res = {"host": host, "threads_all": all_threads}
    # 12-qubit layered circuit, in full, both thread counts, vs the GPU c128 plan
    c1 = W.layered_u3_cx(0, n=12, depth=20)
    rows = {}
    for t in (1, all_threads):
        orc.set_num_threads(t)
        best = None
        for _ in range(5):
            t0 = time.perf_counter()
            orc.run_circuit(c1)
            el = time.perf_counter() - t0
            best = el if best is None else min(best, el)
        rows[t] = best
    sim = q.Simulator(12, q.C128)
    plan = q.Plan(12, c1.gates, precision=q.C128)
    gbest = None
    for _ in range(10):
        sim.init_basis(0)
        sim.synchronize()
        t0 = time.perf_counter()
        sim.run(plan)
        sim.synchronize()
        el = time.perf_counter() - t0
        gbest = el if gbest is None else min(gbest, el)
    sim.close()
    res["layered12_c128"] = {"gates": len(c1.gates), "oracle_1t_ms": round(rows[1] * 1e3, 3),
                             "oracle_all_ms": round(rows[all_threads] * 1e3, 3),
                             "gpu_ms": round(gbest * 1e3, 3), "speedup_vs_all": round(rows[all_threads] / gbest, 1),
                             "note": "oracle and GPU: whole circuit, best of repeats (GPU: wall time incl. launch)"}
    # 28-qubit QFT + layers and the 30-qubit benchmark: sampled
    sw = out.get("swap_modes") or {}
    for name, circ, gpu_ms in (("qft28", W.qft_then_layers(1, n=28, layers=40), sw.get("c128_virtual_ms")),
                               ("haar30", W.haar_blocks(2, n=30, nblocks=200),
                                (out.get("accuracy") or {}).get("c128_ms"))):
        n = circ.n
        orc.set_num_threads(all_threads)
        if name == "haar30" and cb is not None:
            done_a, el_a = cb["blocks"], cb["seconds"]
        else:
            done_a, el_a, _ = _oracle_rate(orc, circ, n, len(circ.gates), 6.0)
        orc.set_num_threads(1)
        done_1, el_1, _ = _oracle_rate(orc, circ, 22, len(circ.gates), 4.0)
        # per-amplitude-gate cost varies with k for dense blocks: scale by the
        # sample's own mix (sum of 2^k) against the whole circuit's
        def work(gs, nq):
            return sum((2 ** len(g.qubits)) * (2 ** nq) for g in gs)
        whole = work(circ.gates, n)
        samp_a = work(circ.gates[:done_a], n)
        est_all = el_a * whole / samp_a
        g22 = [g for g in circ.gates if max(g.qubits) < 22][:done_1]
        samp_1 = work(g22, 22)
        est_1 = el_1 * whole / samp_1
        res[name] = {"sample_all_threads": f"first {done_a} gates at n={n}, {el_a:.1f} s",
                     "sample_one_thread": f"first {done_1} gates with all qubits < 22 at n=22, {el_1:.1f} s",
                     "oracle_all_est_s": round(est_all, 1), "oracle_1t_est_s": round(est_1, 1),
                     "gpu_c128_ms": gpu_ms,
                     "speedup_c128_vs_all": round(est_all / (gpu_ms * 1e-3), 1) if gpu_ms else None,
                     "estimate": "sample time x (whole circuit's sum of 2^k * 2^n) / (sample's)"}
    orc.set_num_threads(all_threads)
    return res


def host_tier(n: int, g: int = 2, amax: int = 1):
    """The out-of-core tier: an n-qubit complex64 QFT of a seeded basis state
    whose top g index bits live in pinned host memory (segments of 2^(n-g)
    amplitudes), streamed through two device group slots, with the
    profile-guided placement on and off.  Sampled amplitudes are checked
    against the QFT's closed form (magnitude 2^(-n/2), phase 2 pi x y / 2^n
    from the exact integer product).  For n that fits the device, the same
    circuit is also timed with the state in HBM."""
    import numpy as np
    import torch
    import paper_2410_09326_amd as q
    from workloads import circuits as W
    x0 = int(W.rng_for(1).integers(2 ** n))
    c = W.qft(n, x0)
    res = {"workload": f"{n}-qubit QFT of a seeded basis state, complex64, top {g} bits in pinned host memory "
                       f"({2 ** g} segments of {2 ** (n - g) * 8 / 2 ** 30:.2f} GiB), {amax} active segment bit(s) per "
                       f"device group", "state_gib": 2 ** n * 8 / 2 ** 30}
    t0 = time.perf_counter()
    t = q.TieredSimulator(n, q.C64, global_bits=g, max_active=amax)
    res["create_s"] = round(time.perf_counter() - t0, 2)
    ys = np.concatenate([np.arange(64, dtype=np.uint64),
                         np.random.default_rng(11).integers(0, 2 ** n, 1 << 14).astype(np.uint64)])
    ph = ((np.uint64(x0) * ys) % np.uint64(2 ** n)).astype(np.float64) * (2 * np.pi / 2 ** n)
    ref = np.exp(1j * ph) * 2.0 ** (-n / 2)
    for remap in (1, 0):
        t.init_basis(x0)
        st = t.run(c.gates, remap=remap)
        l2p = t.layout()
        phys = np.zeros(ys.size, dtype=np.uint64)
        for qb in range(n):
            phys |= ((ys >> np.uint64(qb)) & np.uint64(1)) << np.uint64(int(l2p[qb]))
        seg = (phys >> np.uint64(n - g)).astype(np.int64)
        off = (phys & np.uint64(2 ** (n - g) - 1)).astype(np.int64)
        got = np.zeros(ys.size, dtype=np.complex128)
        for sgi in range(2 ** g):
            m = seg == sgi
            got[m] = t.segment_view(sgi)[off[m]]
        err = float(np.max(np.abs(got - ref)))
        tag = "placed" if remap else "identity"
        res[tag] = {"seconds": round(st["seconds"], 3), "stages": st["stages"], "groups": st["groups"],
                    "exchanges": st["exchanges"], "gpu_passes": st["gpu_passes"],
                    "h2d_gb": round(st["h2d_bytes"] / 1e9, 2), "d2h_gb": round(st["d2h_bytes"] / 1e9, 2),
                    "pcie_gbs_each_way": round(st["h2d_bytes"] / st["seconds"] / 1e9, 1),
                    "plan_s": round(st["plan_seconds"], 4), "sampled_max_abs": err,
                    "sampled_max_abs_over_amp": err * 2 ** (n / 2)}
    t0 = time.perf_counter()
    z = t.expect_z()
    res["expect_z_s"] = round(time.perf_counter() - t0, 3)
    res["max_abs_expect_z"] = float(np.max(np.abs(z)))   # a QFT of a basis state has <Z_q> = 0
    t.close()
    free, _ = torch.cuda.mem_get_info()
    if 2 ** n * 8 * 1.1 < free:
        sim = q.Simulator(n, q.C64)
        plan = q.Plan(n, c.gates, precision=q.C64)
        sim.init_basis(x0)
        sim.run(plan)
        sim.synchronize()
        t0 = time.perf_counter()
        sim.init_basis(x0)
        sim.run(plan)
        sim.synchronize()
        res["in_hbm_seconds"] = round(time.perf_counter() - t0, 4)
        sim.close()
        torch.cuda.empty_cache()
    return res


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
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-swap-eval", action="store_true")
    ap.add_argument("--no-oracle-timing", action="store_true")
    ap.add_argument("--no-tier-eval", action="store_true")
    ap.add_argument("--tier-qubits", type=int, default=30,
                    help="qubits of the host-memory tier leg (34 needs 128 GiB of pinned host memory)")
    ap.add_argument("--tier-only", action="store_true", help="only the host-memory tier leg")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the headline steps (no accuracy check, extra legs or CPU baseline): profiler runs")
    ap.add_argument("--batch-shape", default="",
                    help="small_max_n,tile_bits,max_fuse_k for the batch leg instead of autotuning")
    ap.add_argument("--batch-only", action="store_true",
                    help="skip the headline steps and every leg but the batch sweep (profiler runs)")
    ap.add_argument("--dump-passes", default="", help="write the last step's pass records (JSON) here")
    ap.add_argument("--trace", default="", help="write the last step's profile as a Chrome trace here")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 2^30 x 8-byte device copy (counter calibration)")
    args = ap.parse_args()
    if args.headline_only or args.batch_only:
        args.no_accuracy = args.no_swap_eval = args.no_learned_eval = args.no_qaoa_eval = True
        args.no_cpu_baseline = args.no_oracle_timing = args.no_tier_eval = True
        args.no_batch_eval = not args.batch_only
    batch_shape = tuple(int(v) for v in args.batch_shape.split(",")) if args.batch_shape else None
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this simulator has no multi-GPU path (state sharding is a design "
              "note only); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2410_09326_amd as q

    if args.batch_only:
        print(json.dumps({"batch_sweep": batch_sweep(args.batch_reps, batch_shape)}), flush=True)
        return
    if args.tier_only:
        print(json.dumps({"host_tier": host_tier(args.tier_qubits)}), flush=True)
        return

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
        sim.run(plan)
        sim.expect_z()
    torch.cuda.synchronize()

    # timed region: plain steps (no per-pass events)
    gc.collect()
    gc.disable()                       # no collector pauses inside the timed steps
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sim.init_basis(circ.x0)
        sim.run(plan)
        z = sim.expect_z()             # blocking: ends the step
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    gc.enable()
    ms = el / args.steps * 1e3

    # profiled region: the same steps as profiling runs (HIP events around
    # every pass on the simulator's stream)
    sim.init_basis(circ.x0)
    sim.profile(plan).records()
    sim.expect_z()
    torch.cuda.synchronize()
    recs_all = []
    gc.collect()
    gc.disable()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sim.init_basis(circ.x0)
        prof = sim.profile(plan)
        recs_all.append(prof.records())
        last_prof = prof
        sim.expect_z()
    torch.cuda.synchronize()
    el_prof = time.perf_counter() - t0
    gc.enable()
    ms_prof = el_prof / args.steps * 1e3
    norm = sim.norm()
    accuracy = None
    if not args.no_accuracy:
        accuracy = headline_accuracy(q, torch, sim, plan, circ, prec)

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
    pr = profile_for(dom, args.workload)
    roof["traffic"] = pr.get("bytes_per_launch") if pr else None
    if pr and pr.get("counters"):
        c = pr["counters"]
        # matrix-core work the kernel really issues (the three-product form
        # runs 6·2^k flops per amplitude for k >= 4) and its busy fraction,
        # from the committed SQ counter run of the same source
        roof["counters"] = {"source": f"profiles/{dom}_{args.workload}.md",
                            "mfma_busy_frac": round(c["mfma_busy_frac"], 4),
                            "mfma_executed_tflops": round(c["mfma_exec_tflops"], 2),
                            "mfma_executed_frac": round(c["mfma_exec_frac_of_peak"], 4),
                            "valu_insts_per_launch": c["valu_insts_per_launch"],
                            "lds_bank_conflict_frac": round(c["lds_bank_conflict_frac"], 4)}
        if "valu_fp_busy_frac" in c:
            # share of the SIMDs' cycles the vector FP pipe is busy (4 cycles
            # per wave64 FMA/MUL/ADD): the bound of the vector-ALU kernels
            roof["counters"]["valu_fp_insts_per_launch"] = c["valu_fp_insts_per_launch"]
            roof["counters"]["valu_fp_busy_frac"] = round(c["valu_fp_busy_frac"], 4)
    roof["hbm_frac"] = round(gbs / HBM_PEAK_GBS, 4)
    roof["kernel"] = dom
    roof["timed_over"] = f"{args.steps} profiling-run steps after the timed plain steps (HIP events per pass)"
    roof["launches_per_step"] = d["launches"] // args.steps
    roof["avg_launch_ms"] = round(avg_s * 1e3, 4)
    roof["alg_bytes_per_launch"] = bytes_launch
    roof["alg_flops_per_launch"] = flops_launch
    # the same rate on the input circuit's own blocks (8·2^k·2^n per dense
    # gate): the plan merges blocks, which raises the flops it executes
    dense_in = [g for g in circ.gates if g.kind == "dense" and not g.controls]
    if dom in MATRIX_KERNELS and len(dense_in) == len(circ.gates):
        circ_flops = sum(8.0 * 2 ** len(g.qubits) * 2 ** n for g in dense_in)
        cf_launch = circ_flops / roof["launches_per_step"]
        roof["circuit_flops_per_launch"] = cf_launch
        roof["circuit_tflops"] = round(cf_launch / avg_s / 1e12, 2)
        roof["circuit_frac"] = round(cf_launch / avg_s / 1e12 / fpeak, 4)

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
        "profiled_ms_per_step": round(ms_prof, 3),
        "profiling_overhead": round(ms_prof / ms - 1.0, 4),
        "plan_s": round(plan_s, 4),
        "norm_error": abs(norm - 1.0),
        "accuracy": accuracy,
        "kernels": {k: {"ms_per_step": round(v["seconds"] / args.steps * 1e3, 3),
                        "launches_per_step": v["launches"] // args.steps} for k, v in per.items()},
        "roofline": roof,
    }
    sim.close()
    torch.cuda.empty_cache()
    t_leg = time.perf_counter()

    def leg_done(name):
        # one line per finished leg on stderr (the JSON line stays alone on stdout)
        nonlocal t_leg
        now = time.perf_counter()
        print(f"[bench] {name} done in {now - t_leg:.1f} s", file=sys.stderr, flush=True)
        t_leg = now

    leg_done("headline")
    if not args.no_swap_eval:
        out["swap_modes"] = swap_modes()
        torch.cuda.empty_cache()
        leg_done("swap_modes")
    if not args.no_tier_eval:
        out["host_tier"] = host_tier(args.tier_qubits)
        leg_done("host_tier")
    if not args.no_learned_eval:
        out["learned_vs_plain"] = learned_vs_plain(args.eval_circuits)
        leg_done("learned_vs_plain")
    if not args.no_batch_eval:
        out["batch_sweep"] = batch_sweep(args.batch_reps, batch_shape)
        leg_done("batch_sweep")
    if not args.no_qaoa_eval:
        out["qaoa_sweep"] = qaoa_sweep()
        leg_done("qaoa_sweep")
    cb = None
    if not args.no_cpu_baseline:
        cb = cpu_baseline(circ, args.cpu_seconds)
        out["cpu_baseline"] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in cb.items()
                               if k in ("value", "unit", "cores", "kind", "sample")}
        leg_done("cpu_baseline")
    else:
        out["cpu_baseline"] = None
    if not args.no_oracle_timing:
        out["oracle_timing"] = oracle_timing(out, cb if args.workload == "haar30" else None)
        leg_done("oracle_timing")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
