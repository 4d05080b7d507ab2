"""Two-qubit correlators <Z_a Z_b> on the GPU against the oracle, and
repeated QAOA Max-Cut runs (paper Sec. IV-E) with one plan re-bound to new
angles: <C> from the correlators agrees with the oracle for every parameter
set."""
import numpy as np
import pytest

from oracle import oracle as orc
from workloads import circuits as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_09326_amd as qq
    qq.lib()
    return qq


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n,npairs", [(4, 1), (9, 7), (14, 8), (17, 9), (21, 20)])
def test_expect_zz_random_states(q, prec, n, npairs):
    rng = np.random.default_rng(n * 100 + npairs)
    psi = rng.normal(size=2 ** n) + 1j * rng.normal(size=2 ** n)
    psi /= np.linalg.norm(psi)
    pairs = rng.integers(0, n, size=(npairs, 2))
    sim = q.Simulator(n, prec)
    sim.init_amplitudes(psi)
    got = sim.expect_zz(pairs)
    # the oracle reduces the same (rounded) amplitudes the device holds
    held = psi.astype(np.complex64 if prec == 0 else np.complex128)
    ref = orc.expect_zz(held, pairs)
    assert np.max(np.abs(got - ref)) <= 1e-12
    # a second call is bitwise identical (fixed summation order)
    assert np.array_equal(sim.expect_zz(pairs), got)
    sim.close()


def test_expect_zz_logical_after_virtual_swaps(q):
    c = W.layered_u3_cx(5, n=15, depth=8, swap_frac=0.5)
    pairs = [(a, b) for a in range(0, 15, 2) for b in range(1, 15, 3)]
    sim = q.Simulator(c.n, q.C128)
    sim.init_basis(0)
    sim.apply(c.gates)
    assert not np.array_equal(sim.layout(), np.arange(c.n))
    got = sim.expect_zz(pairs)
    sim.close()
    assert np.max(np.abs(got - orc.expect_zz(orc.run_circuit(c), pairs))) <= 1e-11


def test_expect_zz_rejects_bad_qubits(q):
    sim = q.Simulator(6, q.C64)
    sim.init_basis(0)
    with pytest.raises(q.QopsError) as e:
        sim.expect_zz([(0, 6)])
    assert e.value.code == -2
    assert sim.expect_zz(np.zeros((0, 2))).size == 0
    sim.close()


@pytest.mark.parametrize("prec,tol", [(0, 2e-5), (1, 1e-10)])
def test_qaoa_parameter_sweep_with_plan_reuse(q, prec, tol):
    n = 16
    edges, w = W.regular_graph(11, n, 3)
    rng = np.random.default_rng(4)
    params = [(rng.uniform(0, np.pi, 2), rng.uniform(0, np.pi / 2, 2)) for _ in range(4)]
    c0 = W.qaoa_maxcut(n, edges, w, *params[0])
    plan = q.Plan(n, c0.gates, precision=prec)
    sim = q.Simulator(n, prec)
    for gm, bt in params:
        c = W.qaoa_maxcut(n, edges, w, gm, bt)
        plan.update(c.gates)
        sim.init_basis(0)
        sim.run(plan)
        cost = orc.maxcut_expectation(sim.expect_zz(edges), w)
        ref = orc.maxcut_expectation(orc.expect_zz(orc.run_circuit(c), edges), w)
        assert abs(cost - ref) <= tol * max(1.0, abs(ref)), (gm, bt, cost, ref)
    sim.close()
