"""Batched executor: per-circuit <Z_q> of a batch of uneven parameterised
circuits in one graph launch, against the FP64 oracle; graph replays give
bitwise-identical results; new parameters are re-bound without re-planning;
the autotuner returns a valid shape."""
import numpy as np
import pytest

from oracle import oracle as orc
from workloads import circuits as W


def small_batch(seed=5, count=18, nmin=6, nmax=16, dmin=2, dmax=5):
    return W.param_sweep_batch(seed=seed, count=count, nmin=nmin, nmax=nmax, dmin=dmin, dmax=dmax)


def test_batch_rejects_bad_input_cpu():
    import paper_2410_09326_amd as q
    with pytest.raises(q.QopsError) as e:
        q.Batch([(30, [("h", (0,))])])
    assert e.value.code == -4
    with pytest.raises(q.QopsError) as e:
        q.Batch([(8, [("h", (9,))])])
    assert e.value.code == -2


@pytest.fixture(scope="module")
def q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_09326_amd as qq
    return qq


@pytest.mark.gpu
@pytest.mark.parametrize("prec,tol", [(0, 2e-5), (1, 1e-11)])
def test_batch_matches_oracle(q, prec, tol):
    circs = small_batch()
    b = q.Batch([(c.n, c.gates) for c in circs], precision=prec, small_max_n=11, tile_bits=11)
    info = b.info()
    assert info["small_circuits"] > 0 and info["tile_circuits"] > 0
    b.launch()
    res = b.results()
    for c, z in zip(circs, res):
        ref = orc.expect_z(orc.run_circuit(c))
        assert np.max(np.abs(z - ref)) <= tol, (c.name, np.max(np.abs(z - ref)))
    b.launch()
    b.launch()
    res2 = b.results()
    for a, r in zip(res, res2):
        assert np.array_equal(a, r)
    b.close()


@pytest.mark.gpu
@pytest.mark.parametrize("kf", [2, 3])
def test_batch_fused_blocks(q, kf):
    circs = small_batch(seed=8, count=10)
    b = q.Batch([(c.n, c.gates) for c in circs], precision=1, small_max_n=11, tile_bits=12, max_fuse_k=kf)
    assert b.info()["max_fuse_k"] == kf
    b.launch()
    for c, z in zip(circs, b.results()):
        assert np.max(np.abs(z - orc.expect_z(orc.run_circuit(c)))) <= 1e-11
    b.close()


@pytest.mark.gpu
def test_batch_wide_blocks_on_the_full_tile(q):
    """complex64 circuits of Haar blocks of 2..6 qubits on 2^13-amplitude
    tiles: the 5- and 6-qubit blocks run the 32x32x2 matrix-core form, and
    the block a single-circuit pass would keep in registers reads its
    fragments from global memory."""
    circs = [W.Circuit(c.n, c.gates, name=c.name) for c in
             (W.haar_blocks(40 + i, n=14 + i % 3, nblocks=14) for i in range(4))]
    assert max(len(g.qubits) for c in circs for g in c.gates) == 6
    b = q.Batch([(c.n, c.gates) for c in circs], precision=0, small_max_n=12, tile_bits=13, max_fuse_k=6)
    assert b.info()["tile_circuits"] == 4
    b.launch()
    for c, z in zip(circs, b.results()):
        err = np.max(np.abs(z - orc.expect_z(orc.run_circuit(c))))
        assert err <= 2e-5, (c.name, err)
    b.close()


@pytest.mark.gpu
def test_batch_parameter_update(q):
    circs = small_batch(seed=6, count=10)
    b = q.Batch([(c.n, c.gates) for c in circs], precision=1, small_max_n=10, tile_bits=10)
    rng = np.random.default_rng(1)
    new = [W.Circuit(c.n, [W.Gate(g.kind, g.qubits, g.controls, tuple(rng.uniform(0, 6.28, len(g.params))))
                           for g in c.gates]) for c in circs]
    b.update([c.gates for c in new])
    b.launch()
    for c, z in zip(new, b.results()):
        assert np.max(np.abs(z - orc.expect_z(orc.run_circuit(c)))) <= 1e-11
    b.close()


@pytest.mark.gpu
def test_batch_autotune(q, tmp_path):
    circs = small_batch(seed=7, count=8, nmin=10, nmax=14)
    cache = str(tmp_path / "tune.txt")
    sm, tb, kf, sec = q.Batch.autotune([(c.n, c.gates) for c in circs], precision=0, cache=cache)
    assert 10 <= sm <= 13 and 11 <= tb <= 13 and 1 <= kf <= 3 and sec > 0
    sm2, tb2, kf2, sec2 = q.Batch.autotune([(c.n, c.gates) for c in circs], precision=0, cache=cache)
    assert (sm2, tb2, kf2) == (sm, tb, kf)


@pytest.mark.gpu
def test_batch_edge_cases(q):
    """Empty circuits (small and tile-pass), a 1-qubit circuit, and a batch of
    one circuit."""
    cases = [(1, [("x", (0,))]), (9, []), (14, []), (14, [("h", (13,)), ("cx", (13, 0))]), (3, [("h", (1,))])]
    b = q.Batch(cases, precision=1, small_max_n=10, tile_bits=10)
    b.launch()
    res = b.results()
    assert np.allclose(res[0], [-1.0])
    assert np.allclose(res[1], np.ones(9)) and np.allclose(res[2], np.ones(14))
    exp3 = np.ones(14); exp3[13] = 0.0; exp3[0] = 0.0
    assert np.max(np.abs(res[3] - exp3)) < 1e-12
    assert np.allclose(res[4], [1.0, 0.0, 1.0])
    b.close()
    b1 = q.Batch([(12, [("ry", (5,), (0.3,))])], precision=0, small_max_n=10, tile_bits=11)
    b1.launch()
    z = b1.results()[0]
    assert abs(z[5] - np.cos(0.3)) < 1e-6 and np.allclose(np.delete(z, 5), 1.0)
    b1.close()


@pytest.mark.gpu
def test_batch_with_swaps_reports_logical_order(q):
    """SWAPs are virtual: <Z_q> still comes back per logical qubit."""
    c1 = W.layered_u3_cx(3, n=16, depth=6)          # contains SWAPs
    c2 = W.layered_u3_cx(4, n=10, depth=6)
    assert any(g.kind == "swap" for g in c1.gates)
    b = q.Batch([(c1.n, c1.gates), (c2.n, c2.gates)], precision=1, small_max_n=11, tile_bits=12)
    b.launch()
    for c, z in zip((c1, c2), b.results()):
        assert np.max(np.abs(z - orc.expect_z(orc.run_circuit(c)))) <= 1e-11
    b.close()
