"""Full-size checks, in the launch configuration the benchmark times, through
properties that hold at any size (the FP64 oracle cannot hold these states):

* 30-qubit circuit of 200 Haar blocks (k ~ U{2..6}), complex64 with the
  default fused plan: norm, fidelity and max-abs error against the same
  circuit in complex128 on the GPU, and the circuit followed by its inverse
  returning |0..0>;
* 28-qubit QFT of a seeded basis state, both swap modes, both precisions:
  every sampled amplitude equals 2^(-n/2) exp(2 pi i x y / 2^n), the phase
  taken from the exact integer product;
* the 512-circuit parameter sweep as one batch: <Z> of sampled circuits
  against the oracle (n <= 16) and against the complex128 single-circuit path;
* 28-qubit QFT + 40 U3/CZ layers, both swap modes: complex64 against
  complex128 and the inverse circuit returning the seeded basis state;
* a 32-qubit depth-60 evaluation circuit under the learned and the plain
  cost-model plans: <Z_i> against the complex128 run;
* the first blocks of the 30-qubit Haar-block benchmark circuit in the
  default plan and launch against the FP64 oracle itself, element by
  element (16 GiB of host memory for the oracle's state);
* the largest states the library accepts (34 qubits complex64, 33 qubits
  complex128: 128 GiB, indices past 2^32): a circuit whose <Z_q> has a closed
  form (pinned against the oracle at small n), and the norm.
"""
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


def _as_complex(q, sim):
    import torch
    return sim.buffer.view(torch.complex64 if sim.precision == q.C64 else torch.complex128)


def test_haar30_c64_against_c128_and_inverse(q):
    import torch
    c = W.haar_blocks(2, n=30, nblocks=200)
    inv = W.inverse(c)
    s64 = q.Simulator(30, q.C64)
    s64.init_basis(c.x0)
    s64.run(q.Plan(30, c.gates, precision=q.C64))
    s128 = q.Simulator(30, q.C128)
    s128.init_basis(c.x0)
    s128.run(q.Plan(30, c.gates, precision=q.C128))
    assert abs(s64.norm() - 1.0) < 1e-5 and abs(s128.norm() - 1.0) < 1e-12
    l64, l128 = s64.layout(), s128.layout()
    assert np.array_equal(l64, l128)
    a, b = _as_complex(q, s64), _as_complex(q, s128)
    err, amax, ov = 0.0, 0.0, 0.0 + 0.0j
    step = 1 << 26
    for o in range(0, 1 << 30, step):
        x = a[o:o + step].to(torch.complex128)
        y = b[o:o + step]
        err = max(err, float((x - y).abs().max()))
        amax = max(amax, float(y.abs().max()))
        ov += complex(torch.vdot(y, x).item())
    fid = abs(ov) ** 2
    print(f"haar30 c64 vs c128: max-abs {err:.3e}, max|psi| {amax:.3e}, 1-F {1 - fid:.3e}")
    assert err <= 2e-5 and err / amax <= 1e-4 and 1 - fid <= 1e-6
    # circuit then inverse returns |x0>
    for sim, prec, tol in ((s64, q.C64, 1e-4), (s128, q.C128, 1e-11)):
        sim.run(q.Plan(30, inv.gates, precision=prec, l2p=sim.layout()))
        z = _as_complex(q, sim)
        l2p = sim.layout()
        phys0 = sum(1 << int(l2p[k]) for k in range(30) if (c.x0 >> k) & 1)
        assert abs(complex(z[phys0].item()) - 1.0) <= tol
        rest = z.abs()
        rest[phys0] = 0
        assert float(rest.max()) <= tol
    s64.close()
    s128.close()


def test_haar30_prefix_against_oracle(q):
    """The benchmark's own launch path (30 qubits, complex64, default plan:
    LDS tile passes over 2^17 tiles on the persistent grid, matrix-core
    blocks, fragments held in registers across tiles) against the FP64
    oracle on the circuit's first four blocks (k = 6, 6, 3, 3)."""
    c = W.haar_blocks(2, n=30, nblocks=200)
    pre = W.Circuit(30, c.gates[:4], x0=c.x0, name="haar30_prefix4")
    assert [len(g.qubits) for g in pre.gates] == [6, 6, 3, 3]
    sim = q.Simulator(30, q.C64)
    sim.init_basis(pre.x0)
    plan = q.Plan(30, pre.gates, precision=q.C64)
    assert any(p["type"] == 1 for p in plan.passes())
    sim.run(plan)
    assert np.array_equal(sim.layout(), np.arange(30))
    got = sim.state()
    sim.close()
    ref = orc.run_circuit(pre)
    err, amax, ov = 0.0, 0.0, 0.0 + 0.0j
    step = 1 << 26
    for o in range(0, 1 << 30, step):
        x = got[o:o + step].astype(np.complex128)
        y = ref[o:o + step]
        err = max(err, float(np.max(np.abs(x - y))))
        amax = max(amax, float(np.max(np.abs(y))))
        ov += np.vdot(y, x)
    fid = abs(ov) ** 2
    print(f"haar30 prefix vs oracle: max-abs {err:.3e}, max|psi| {amax:.3e}, 1-F {1 - fid:.3e}")
    assert err <= 2e-5 and err / amax <= 1e-4 and 1 - fid <= 1e-6


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("swap_mode", [0, 1])
def test_qft28_closed_form(q, prec, swap_mode):
    n = 28
    x0 = int(W.rng_for(1).integers(2 ** n))
    c = W.qft(n, x0)
    sim = q.Simulator(n, prec)
    sim.init_basis(x0)
    sim.run(q.Plan(n, c.gates, precision=prec, swap_mode=swap_mode))
    if swap_mode == q.SWAP_VIRTUAL:
        assert np.array_equal(sim.layout(), orc.expected_layout(n, c.gates))
    else:
        assert np.array_equal(sim.layout(), np.arange(n))
    psi = sim.state()
    sim.close()
    ys = np.concatenate([np.arange(64, dtype=np.uint64),
                         np.random.default_rng(11).integers(0, 2 ** n, 1 << 16).astype(np.uint64)])
    ph = ((np.uint64(x0) * ys) % np.uint64(2 ** n)).astype(np.float64) * (2 * np.pi / 2 ** n)
    ref = np.exp(1j * ph) * 2.0 ** (-n / 2)
    err = float(np.max(np.abs(psi[ys.astype(np.int64)].astype(np.complex128) - ref)))
    assert err <= (2e-5 if prec == 0 else 1e-12), err
    mag = np.abs(psi[:1 << 20].astype(np.complex128))
    assert np.max(np.abs(mag - 2.0 ** (-n / 2))) <= (1e-6 if prec == 0 else 1e-14)


def test_param_sweep_batch_full(q):
    circs = W.param_sweep_batch(5)
    spec = [(c.n, q.GateArray(c.gates)) for c in circs]
    b = q.Batch(spec, precision=q.C64)
    b.launch()
    res = b.results()
    b.close()
    for z in res:
        assert np.all(np.abs(z) <= 1 + 1e-5)
    small = [i for i, c in enumerate(circs) if c.n <= 16][:6]
    for i in small:
        ref = orc.expect_z(orc.run_circuit(circs[i]))
        assert np.max(np.abs(res[i] - ref)) <= 2e-5, (i, circs[i].n)
    big = [i for i, c in enumerate(circs) if c.n >= 20][:4]
    for i in big:
        sim = q.Simulator(circs[i].n, q.C128)
        sim.init_basis(0)
        sim.run(q.Plan(circs[i].n, spec[i][1], precision=q.C128))
        assert np.max(np.abs(res[i] - sim.expect_z())) <= 2e-5, (i, circs[i].n)
        sim.close()


@pytest.mark.parametrize("swap_mode", [0, 1])
def test_qft28_layers_c64_c128_and_inverse(q, swap_mode):
    """The 28-qubit QFT + 40 U3/CZ layers workload at full size, both swap
    modes: complex64 against complex128 on the GPU, and the complex128 state
    followed by the inverse circuit returning the seeded basis state."""
    import torch
    c = W.qft_then_layers(1, n=28, layers=40)
    sims = {}
    for prec in (q.C64, q.C128):
        sim = q.Simulator(28, prec)
        sim.init_basis(c.x0)
        sim.run(q.Plan(28, c.gates, precision=prec, swap_mode=swap_mode))
        sims[prec] = sim
    assert np.array_equal(sims[q.C64].layout(), sims[q.C128].layout())
    assert abs(sims[q.C64].norm() - 1) < 1e-5 and abs(sims[q.C128].norm() - 1) < 1e-12
    a = _as_complex(q, sims[q.C64]).to(torch.complex128)
    b = _as_complex(q, sims[q.C128])
    err = float((a - b).abs().max())
    # fidelity of the normalised states: the complex64 norm drift is bounded
    # on its own above
    fid = abs(complex(torch.vdot(b, a).item())) ** 2 / (
        float(torch.vdot(a, a).real) * float(torch.vdot(b, b).real))
    del a
    assert err <= 2e-5 and 1 - fid <= 1e-6, (err, fid)
    s = sims[q.C128]
    s.run(q.Plan(28, W.inverse(c).gates, precision=q.C128, swap_mode=swap_mode, l2p=s.layout()))
    z = _as_complex(q, s)
    l2p = s.layout()
    phys0 = sum(1 << int(l2p[k]) for k in range(28) if (c.x0 >> k) & 1)
    assert abs(complex(z[phys0].item()) - 1.0) <= 1e-10
    for sim in sims.values():
        sim.close()


def test_eval32_priced_plans_agree_with_c128(q):
    """A 32-qubit depth-60 evaluation circuit: the plans the learned and the
    plain cost models pick (complex64) give the <Z_i> of the complex128 run."""
    import os
    here = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    models = os.path.join(here, "paper_2410_09326_amd", "models")
    model = q.CostModel.load(os.path.join(models, "cost_mlp.bin"))
    prof = q.Profile.load(os.path.join(models, "corpus_profile.bin"))
    c = W.eval_circuit(9000, n=32, depth=60)
    ref = q.Simulator(32, q.C128)
    ref.init_basis(0)
    ref.run(q.Plan(32, c.gates, precision=q.C128))
    zref = ref.expect_z()
    ref.close()
    sim = q.Simulator(32, q.C64)
    for mode, kw in ((q.PLAN_LEARNED, {"model": model}), (q.PLAN_PROFILED, {"profile": prof})):
        sim.init_basis(0)
        sim.run(q.Plan(32, c.gates, precision=q.C64, mode=mode, **kw))
        assert np.max(np.abs(sim.expect_z() - zref)) <= 1e-5
    sim.close()


@pytest.mark.parametrize("n,prec", [(34, 0), (33, 1)])
def test_largest_states_closed_form(q, n, prec):
    """RY layers, Kronecker-product RY blocks of 2..6 qubits (register and
    LDS tile passes, matrix cores), diagonals and virtual SWAPs on the
    largest state of each precision: <Z_q> = cos of the summed RY angles."""
    import torch
    from product_state import product_state_circuit
    c, z = product_state_circuit(n, 40 + n)
    sim = q.Simulator(n, prec)
    try:
        sim.init_basis(0)
        sim.run(q.Plan(n, c.gates, precision=prec))
        got = sim.expect_z()
        nrm = sim.norm()
    finally:
        sim.close()
        del sim
        torch.cuda.empty_cache()
    tol = 2e-5 if prec == q.C64 else 1e-10
    assert abs(nrm - 1.0) <= tol
    assert np.max(np.abs(got - z)) <= tol
