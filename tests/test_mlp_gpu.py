"""The learned cost model's GPU kernels against the FP64 CPU reference:
gradients of the MSE loss (rel. err <= 1e-4, FP32 vs FP64), predictions,
and a training run that reduces the loss.  Save/load round trip on the CPU."""
import os
import tempfile

import numpy as np
import pytest

from oracle import mlp_oracle as mo
from workloads import circuits as W


def test_model_file_roundtrip_cpu():
    import paper_2410_09326_amd as q
    p0 = W.mlp_init(3).astype(np.float32)
    m = q.CostModel(p0)
    mu = np.linspace(-1, 1, 64).astype(np.float32)
    sd = np.linspace(0.5, 2, 64).astype(np.float32)
    m.set_normalization(mu, sd)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "m.bin")
        m.save(path)
        m2 = q.CostModel.load(path)
        p, mu2, sd2 = m2.params()
    assert np.array_equal(p, p0) and np.array_equal(mu2, mu) and np.array_equal(sd2, sd)
    assert q.CostModel.num_params() == p0.size
    # the flat layout round-trips through the FP64 oracle's dict form
    assert np.array_equal(mo.flatten(mo.unflatten(p0.astype(np.float64))), p0.astype(np.float64))


@pytest.fixture(scope="module")
def q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_09326_amd as qq
    return qq


def data(seed, rows):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(rows, 64)).astype(np.float32)
    t = (0.3 * X[:, 0] - 0.7 * X[:, 5] + 0.2 * X[:, 9] * X[:, 3]).astype(np.float32)
    return X, t


@pytest.mark.gpu
@pytest.mark.parametrize("rows", [1, 7, 64, 300])
def test_gradients_match_fp64_reference(q, rows):
    p0 = W.mlp_init(11)
    X, t = data(rows, rows)
    m = q.CostModel(p0.astype(np.float32))
    loss, g = m.grad(X, t)
    ref_p = mo.unflatten(p0.astype(np.float32).astype(np.float64))
    ref_loss, ref_g = mo.backward(ref_p, X.astype(np.float64), t.astype(np.float64))
    ref_flat = mo.flatten(ref_g)
    assert abs(loss - ref_loss) <= 1e-4 * max(1.0, abs(ref_loss))
    scale = np.max(np.abs(ref_flat))
    assert np.max(np.abs(g - ref_flat)) <= 1e-4 * scale


@pytest.mark.gpu
def test_training_reduces_loss_and_predicts(q):
    X, t = data(0, 2048)
    m = q.CostModel(W.mlp_init(5).astype(np.float32))
    l0, _ = m.grad(X, t)
    final = m.train(X, t, epochs=30, batch=128, lr=2e-3, seed=1)
    l1, _ = m.grad(X, t)
    assert l1 < 0.2 * l0 and final < 0.5 * l0
    p, _, _ = m.params()
    pred = m.predict(X[:100])
    ref, _ = mo.forward(mo.unflatten(p.astype(np.float64)), X[:100].astype(np.float64))
    assert np.max(np.abs(pred - ref)) <= 1e-4 * max(1.0, np.max(np.abs(ref)))
    # a second run from the same seed is bitwise identical
    m2 = q.CostModel(W.mlp_init(5).astype(np.float32))
    m2.train(X, t, epochs=30, batch=128, lr=2e-3, seed=1)
    assert np.array_equal(m2.params()[0], p)


@pytest.mark.gpu
def test_gpu_adam_steps_match_fp64_reference(q):
    """Full-batch training (batch = rows, so the epoch shuffle only reorders
    the rows of one sum) for S steps against S FP64 backward + Adam steps of
    the reference, parameter by parameter.  Adam moves every parameter by
    about lr per step whatever the gradient's size, so the natural scale of
    the comparison is the step, S * lr: where FP32 resolves the gradient (at
    least 1e-3 of the largest of its tensor at every step) the parameters
    agree to 1e-4 of S * lr, which is a few FP32 units of the parameters
    themselves; the others (a gradient near zero whose sign FP32 may not
    resolve) to 1e-2 of S * lr.  A wrong bias correction, beta or moment
    update moves parameters by O(lr) and fails both bounds."""
    rows, steps, lr = 64, 4, 1e-3
    X, t = data(123, rows)
    p0 = W.mlp_init(21).astype(np.float32)
    m = q.CostModel(p0)
    m.train(X, t, epochs=steps, batch=rows, lr=lr, seed=3)
    got = m.params()[0].astype(np.float64)

    ref = mo.unflatten(p0.astype(np.float64))
    mom = {k: np.zeros_like(v) for k, v in ref.items()}
    vel = {k: np.zeros_like(v) for k, v in ref.items()}
    gmin = {k: np.full(v.shape, np.inf) for k, v in ref.items()}
    Xd, td = X.astype(np.float64), t.astype(np.float64)
    for s in range(1, steps + 1):
        _, g = mo.backward(ref, Xd, td)
        for k in g:
            gmin[k] = np.minimum(gmin[k], np.abs(g[k]) / max(float(np.max(np.abs(g[k]))), 1e-300))
        mo.adam_step(ref, g, mom, vel, s, lr)
    want = mo.flatten(ref)
    resolved = mo.flatten(gmin) > 1e-3
    assert resolved.mean() > 0.8
    err = np.abs(got - want) / (steps * lr)
    print(f"adam: max err / (S lr) {err[resolved].max():.2e} resolved, {err.max():.2e} all")
    assert np.all(err[resolved] <= 1e-4)
    assert np.all(err <= 1e-2)
    # the run moved the parameters by Adam's step size, not by lr * gradient
    moved = np.abs(want - p0.astype(np.float64))[resolved]
    assert np.median(moved) > 0.5 * lr


@pytest.mark.gpu
def test_learned_model_gains_over_plain_table(q):
    """The shipped network (trained on the GPU from profiling runs) against
    the plain cost table fitted to the shipped profile, on passes of fresh
    circuits it never saw: its per-pass time predictions are closer, and the
    plans it picks compute the same result."""
    here = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    models = os.path.join(here, "paper_2410_09326_amd", "models")
    model = q.CostModel.load(os.path.join(models, "cost_mlp.bin"))
    prof = q.Profile.load(os.path.join(models, "corpus_profile.bin"))
    rng = np.random.default_rng(77)
    true, p_learned, p_plain = [], [], []
    for seed in range(30000, 30006):
        c = W.corpus_circuit(seed, n_override=int(rng.integers(20, 25)))
        plan = q.Plan(c.n, c.gates, precision=q.C64, tile_upper=int(rng.integers(4, 8)),
                      remap=int(rng.integers(0, 2)), max_fuse_k=int(rng.integers(1, 5)))
        sim = q.Simulator(c.n, q.C64)
        sim.init_basis(0)
        sim.run(plan)                      # warm
        sim.init_basis(0)
        pr = sim.profile(plan)
        sim.close()
        true.append(np.array([r["seconds"] for r in pr.records()]))
        p_learned.append(pr.predict_passes(mode=q.PLAN_LEARNED, model=model))
        p_plain.append(pr.predict_passes(mode=q.PLAN_PROFILED, profile=prof))
    t = np.concatenate(true)
    mape_l = float(np.mean(np.abs(np.concatenate(p_learned) - t) / t))
    mape_p = float(np.mean(np.abs(np.concatenate(p_plain) - t) / t))
    print(f"held-out passes {t.size}: MAPE learned {mape_l:.3f}, plain table {mape_p:.3f}")
    assert mape_l < mape_p and mape_l < 0.25
    # both pricings pick plans that compute the same <Z>
    c = W.eval_circuit(9100, n=22, depth=20)
    zs = []
    for mode, kw in ((q.PLAN_LEARNED, {"model": model}), (q.PLAN_PROFILED, {"profile": prof})):
        sim = q.Simulator(c.n, q.C64)
        sim.init_basis(0)
        sim.run(q.Plan(c.n, c.gates, precision=q.C64, mode=mode, **kw))
        zs.append(sim.expect_z())
        sim.close()
    assert np.max(np.abs(zs[0] - zs[1])) <= 1e-5
