"""GPU parity: the HIP path against the FP64 oracle on the same seeded
inputs.  Tolerances: max-abs amplitude error <= 1e-12 for complex128 and
<= 2e-5 for complex64 (logical order, after the layout readout); FP64
reductions within 1e-12 of the oracle's on the same amplitudes; layouts and
index maps bit-exact."""
import numpy as np
import pytest

from oracle import oracle as orc
from workloads import circuits as W

pytestmark = pytest.mark.gpu

TOL = {0: 2e-5, 1: 1e-12}


@pytest.fixture(scope="module")
def q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_09326_amd as qq
    qq.lib()
    return qq


def run_gpu(q, c, prec, **opts):
    sim = q.Simulator(c.n, prec)
    sim.init_basis(c.x0)
    sim.apply(c.gates, **opts)
    out = sim.state()
    l2p = sim.layout()
    sim.close()
    return out, l2p


def check_state(got, ref, prec, what=""):
    err = float(np.max(np.abs(got.astype(np.complex128) - ref)))
    assert err <= TOL[prec], f"{what}: max-abs {err:.3e} > {TOL[prec]:.0e}"
    return err


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n", [4, 6, 7, 8, 9, 10, 12])
def test_small_state_in_lds(q, n, prec):
    c = W.random_mixed(100 + n, n, 120, max_dense_k=min(6, n))
    got, _ = run_gpu(q, c, prec)
    check_state(got, orc.run_circuit(c), prec, f"n={n}")


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n", [13, 14, 17, 20])
@pytest.mark.parametrize("seed", [0, 1])
def test_tile_passes_mixed(q, n, prec, seed):
    c = W.random_mixed(1000 * seed + n, n, 160, max_dense_k=6)
    got, l2p = run_gpu(q, c, prec)
    check_state(got, orc.run_circuit(c), prec, f"n={n} seed={seed}")
    assert np.array_equal(l2p, orc.expected_layout(n, c.gates))


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n", [13, 16, 21])
def test_gatewise_sweeps(q, n, prec):
    c = W.random_mixed(7 + n, n, 60, max_dense_k=6)
    got, _ = run_gpu(q, c, prec, mode=q.PLAN_GATEWISE)
    check_state(got, orc.run_circuit(c), prec, f"gatewise n={n}")


@pytest.mark.parametrize("prec", [0, 1])
def test_ghz_and_qft_closed_forms(q, prec):
    n = 20
    got, _ = run_gpu(q, W.ghz(n), prec)
    ref = np.zeros(2 ** n, complex)
    ref[0] = ref[-1] = 2 ** -0.5
    check_state(got, ref, prec, "ghz")
    x0 = 654321
    got, l2p = run_gpu(q, W.qft(n, x0), prec)
    y = np.arange(2 ** n, dtype=np.int64)
    ref = np.exp(2j * np.pi * ((x0 * y) % 2 ** n) / 2 ** n) / 2 ** (n / 2)
    check_state(got, ref, prec, "qft")
    assert np.array_equal(l2p, np.arange(n)[::-1])   # final swap network = reversal


def test_layered_circuit_c128(q):
    """12-qubit layered U3 + CNOT circuit with SWAPs in 10 % of the layers,
    complex128, whole circuit in one work-group."""
    for seed in range(3):
        c = W.layered_u3_cx(seed, n=12, depth=20)
        got, l2p = run_gpu(q, c, 1)
        check_state(got, orc.run_circuit(c), 1, f"layered seed {seed}")
        assert np.array_equal(l2p, orc.expected_layout(12, c.gates))


@pytest.mark.parametrize("prec", [0, 1])
def test_physical_and_virtual_swap(q, prec):
    """QFT + random layers: virtual and physical SWAP handling give the same
    logical state; unfused they are bitwise identical."""
    c = W.qft_then_layers(1, n=18, layers=4)
    ref = orc.run_circuit(c)
    virt, l2p_v = run_gpu(q, c, prec, swap_mode=q.SWAP_VIRTUAL)
    phys, l2p_p = run_gpu(q, c, prec, swap_mode=q.SWAP_PHYSICAL)
    check_state(virt, ref, prec, "virtual")
    check_state(phys, ref, prec, "physical")
    assert np.array_equal(l2p_p, np.arange(18))
    assert np.array_equal(l2p_v, orc.expected_layout(18, c.gates))
    gv, _ = run_gpu(q, c, prec, swap_mode=q.SWAP_VIRTUAL, mode=q.PLAN_GATEWISE)
    gp, _ = run_gpu(q, c, prec, swap_mode=q.SWAP_PHYSICAL, mode=q.PLAN_GATEWISE)
    assert np.array_equal(gv.view(np.uint8), gp.view(np.uint8))


@pytest.mark.parametrize("prec", [0, 1])
def test_haar_blocks_mfma(q, prec):
    c = W.haar_blocks(2, n=18, nblocks=40)
    ref = orc.run_circuit(c)
    got, _ = run_gpu(q, c, prec)
    check_state(got, ref, prec, "haar mfma")
    got2, _ = run_gpu(q, c, prec, use_mfma=0)
    check_state(got2, ref, prec, "haar valu")
    if prec == 0:
        f = orc.fidelity(ref, got)
        assert 1 - f < 1e-8


@pytest.mark.parametrize("prec", [0, 1])
def test_measurements(q, prec):
    n = 17
    c = W.random_mixed(42, n, 120, max_dense_k=3)
    sim = q.Simulator(n, prec)
    sim.init_basis(c.x0)
    sim.apply(c.gates)
    psi = sim.state().astype(np.complex128)
    assert abs(sim.norm() - orc.norm(psi)) <= 1e-12
    assert np.max(np.abs(sim.expect_z() - orc.expect_z(psi))) <= 1e-12
    for qs in ([3], [16, 0, 5], list(range(12)), [4, 15, 7, 9, 1, 13, 2, 11, 6, 10, 0, 14, 3], list(range(n))[::-1]):
        got = sim.probabilities(qs)
        assert np.max(np.abs(got - orc.probabilities(psi, qs))) <= 1e-12, qs
    # deterministic: the same call gives the same bits
    a, b = sim.expect_z(), sim.expect_z()
    assert np.array_equal(a, b)
    sim.close()


def test_layout_calls(q):
    n = 15
    c = W.random_mixed(5, n, 80, max_dense_k=3)
    sim = q.Simulator(n, 1)
    sim.init_basis(c.x0)
    sim.apply(c.gates)
    ref = sim.state()
    sim.swap(2, 9)                       # virtual: data untouched, map changes
    sw = orc.run(n, [W.Gate("swap", (2, 9))], psi=ref)
    assert np.array_equal(sim.state(), sw)
    sim.swap(2, 9, q.SWAP_PHYSICAL)      # physical exchange of the same bits
    perm = np.random.default_rng(1).permutation(n).astype(np.int32)
    before = sim.state()
    sim.set_layout(perm)
    assert np.array_equal(sim.layout(), perm)
    assert np.array_equal(sim.state(), before)
    phys = sim.state(q.ORDER_PHYSICAL)
    assert np.array_equal(orc.logical_from_physical(phys, perm), before)
    sim.close()


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("kmax", [3, 4, 5, 6])
def test_fused_blocks(q, prec, kmax):
    """Gates fused into dense k-qubit blocks (matrix cores for k >= 3) agree
    with the gate-by-gate oracle."""
    for c in (W.qft_then_layers(1, n=16, layers=4), W.random_mix_layers(9, 17, 6)):
        got, l2p = run_gpu(q, c, prec, max_fuse_k=kmax)
        check_state(got, orc.run_circuit(c), prec, f"{c.name} kmax={kmax}")


@pytest.mark.parametrize("prec", [0, 1])
def test_rotation_folding(q, prec):
    """Clifford+T circuits with rotation folding on, off and by the T-gate
    rule agree with the oracle (exact folding: no global-phase freedom)."""
    for c in (W.clifford_t(1, 15, 600), W.clifford_t(3, 19, 900, t_frac=0.5)):
        ref = orc.run_circuit(c)
        for fold in (1, -1, 0):
            got, _ = run_gpu(q, c, prec, fold_rotations=fold)
            check_state(got, ref, prec, f"{c.name} fold={fold}")


@pytest.mark.parametrize("prec", [0, 1])
def test_wide_blocks_sharing_a_pass(q, prec):
    """A 6-qubit block and 5-qubit blocks in one LDS pass (the widest keeps
    its fragments in registers, the others are staged in LDS), on a state of
    2^20 amplitudes."""
    rng = W.rng_for(31)
    mk = lambda qs: W.Gate("dense", tuple(qs), (), (), W.haar_unitary(rng, 2 ** len(qs)))
    gates = [mk((0, 1, 2, 8, 9, 10)), mk((3, 4, 11, 12, 13)), mk((1, 5, 8, 11, 14)), mk((2, 9, 12, 4, 0)),
             mk((6, 7, 15, 16, 17, 18)), mk((19, 6, 15, 3, 0))]
    c = W.Circuit(20, gates)
    got, _ = run_gpu(q, c, prec)
    check_state(got, orc.run_circuit(c), prec, "wide blocks")


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("tile_upper", [4, 5, 6, 7])
def test_lds_tiles_of_every_width(q, prec, tile_upper):
    """LDS tile passes of 10..13 bits (6 + tile_upper, at most 13 for
    complex64 and 12 for complex128): the largest tile runs the branch-free
    load/store variant, the smaller ones the element-tested one; blocks of
    2..6 qubits on 16 qubits against the oracle."""
    c = W.haar_blocks(7, n=16, nblocks=30)
    ref = orc.run_circuit(c)
    got, _ = run_gpu(q, c, prec, tile_upper=tile_upper)
    check_state(got, ref, prec, f"lds tile upper={tile_upper}")
