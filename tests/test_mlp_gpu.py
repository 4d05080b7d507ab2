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
    # the flat layout round-trips through the reference's dict form
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
