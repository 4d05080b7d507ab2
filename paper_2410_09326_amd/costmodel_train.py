"""Builds the cost-model corpus with profiling runs and trains the learned
cost model on the GPU.

Corpus: seeded random circuits of 20..30 qubits (U3 / CZ / SWAP / RZZ
layers, depth 20..100), each planned under a randomly drawn candidate (tile
width 4..7, qubit remap on/off, block fusion width 1..4) and executed once as
a profiling run; every
fused pass is one sample (64 features -> log seconds, scaled to 30 qubits).  Circuits are split
90/10 into training and held-out sets.  The plain cost table is the
library's per-shape table of median times (kernel kind, tile width,
register/wave split, widest block, operation count) fitted to the same
training passes; the learned one is the perceptron trained here.  Both are
scored on the held-out passes.

    python -m paper_2410_09326_amd.costmodel_train --circuits 600 --out paper_2410_09326_amd/models
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def collect(n_circuits: int, seed0: int = 1000, time_budget: float = 240.0, max_n: int = 30):
    import torch
    import paper_2410_09326_amd as q
    from workloads import circuits as W

    rng = np.random.default_rng(seed0)
    sims = {}
    feats, logt, cid, ns = [], [], [], []
    train_prof = None
    hold_prof = None
    t0 = time.time()
    done = 0
    for i in range(n_circuits):
        if time.time() - t0 > time_budget:
            break
        seed = seed0 + i
        c = W.corpus_circuit(seed)
        if c.n > max_n:
            continue
        up = int(rng.integers(4, 8))
        remap = int(rng.integers(0, 2))
        kf = int(rng.integers(1, 5))
        plan = q.Plan(c.n, c.gates, precision=q.C64, tile_upper=up, remap=remap, max_fuse_k=kf)
        if c.n not in sims:
            for k in list(sims):
                sims.pop(k).close()
            torch.cuda.empty_cache()
            sims[c.n] = q.Simulator(c.n, q.C64)
        sim = sims[c.n]
        sim.init_basis(0)
        prof = sim.profile(plan)
        recs = prof.records()
        f = prof.features()
        t = np.array([max(r["seconds"], 1e-7) for r in recs])
        held = (i % 10) == 9
        if held:
            hold_prof = prof if hold_prof is None else (hold_prof.merge(prof) or hold_prof)
        else:
            # every training circuit feeds the plain table as well
            train_prof = prof if train_prof is None else (train_prof.merge(prof) or train_prof)
        feats.append(f)
        logt.append(np.log(t))
        cid.append(np.full(len(t), i))
        ns.append(np.full(len(t), c.n))
        done += 1
        if done % 50 == 0:
            print(f"  profiled {done} circuits, {sum(len(x) for x in logt)} passes, {time.time() - t0:.0f}s",
                  flush=True)
    for s in sims.values():
        s.close()
    return (np.concatenate(feats), np.concatenate(logt), np.concatenate(cid), np.concatenate(ns),
            train_prof, hold_prof, done)


def mape(pred, true):
    return float(np.mean(np.abs(pred - true) / true))


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--circuits", type=int, default=600)
    ap.add_argument("--time-budget", type=float, default=240.0)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--out", default=os.path.join(HERE, "models"))
    args = ap.parse_args()
    import paper_2410_09326_amd as q
    from workloads import circuits as W

    os.makedirs(args.out, exist_ok=True)
    X, y, cid, ns, train_prof, hold_prof, done = collect(args.circuits, time_budget=args.time_budget)
    held = (cid % 10) == 9
    # the network learns ln(t) scaled to 30 qubits (plan pricing scales back)
    yn = y - (ns - 30) * np.log(2.0)
    Xtr, ytr = X[~held], yn[~held]
    mu = Xtr.mean(axis=0)
    sd = Xtr.std(axis=0)
    sd[sd < 1e-6] = 1.0
    model = q.CostModel(W.mlp_init(7).astype(np.float32))
    model.set_normalization(mu, sd)
    t0 = time.time()
    loss = model.train(Xtr, ytr, epochs=args.epochs, batch=256, lr=1e-3, seed=3)
    train_s = time.time() - t0
    model.save(os.path.join(args.out, "cost_mlp.bin"))
    shipped = train_prof.compact()
    shipped.save(os.path.join(args.out, "corpus_profile.bin"))
    true = np.exp(y[held])
    pred_mlp = hold_prof.predict_passes(mode=q.PLAN_LEARNED, model=model)
    pred_plain = hold_prof.predict_passes(mode=q.PLAN_PROFILED, profile=shipped)
    pred_plain_full = hold_prof.predict_passes(mode=q.PLAN_PROFILED, profile=train_prof)
    summary = {
        "circuits": int(done), "passes": int(len(y)), "train_passes": int((~held).sum()),
        "heldout_passes": int(held.sum()), "final_train_loss": loss, "train_seconds": train_s,
        "mape_learned": mape(pred_mlp, true), "mape_plain": mape(pred_plain, true),
        "mape_plain_full_table": mape(pred_plain_full, true),
        "plain_table_passes": int(len(train_prof.records())), "shipped_profile_passes": int(len(shipped.records())),
        "median_ape_learned": float(np.median(np.abs(pred_mlp - true) / true)),
        "median_ape_plain": float(np.median(np.abs(pred_plain - true) / true)),
    }
    with open(os.path.join(args.out, "cost_model_summary.json"), "w") as fh:
        json.dump(summary, fh, indent=1)
    print(json.dumps(summary), flush=True)


if __name__ == "__main__":
    main()
