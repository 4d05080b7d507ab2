"""GPU parity on degenerate inputs: empty circuits, one- and two-qubit
states, circuits of SWAPs only, of diagonals only, identity blocks and gates
on the highest qubit alone.  Each result is compared with the FP64 oracle
(max-abs <= 2e-5 complex64, <= 1e-12 complex128) or, where the answer is a
basis state, exactly."""
import numpy as np
import pytest

from oracle import oracle as orc
from workloads import circuits as W

pytestmark = pytest.mark.gpu

TOL = {0: 2e-5, 1: 1e-12}
G, C = W.Gate, W.Circuit


@pytest.fixture(scope="module")
def q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_09326_amd as qq
    qq.lib()
    return qq


def run(q, c, prec, **opts):
    sim = q.Simulator(c.n, prec)
    sim.init_basis(c.x0)
    sim.apply(c.gates, **opts)
    out = sim.state()
    l2p = sim.layout()
    sim.close()
    return out, l2p


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n", [1, 5, 14, 21])
def test_empty_circuit_leaves_the_basis_state(q, n, prec):
    x0 = (0x5A5A5 * n + 3) % (1 << n)
    got, l2p = run(q, C(n, [], x0=x0), prec)
    want = np.zeros(1 << n, dtype=np.complex128)
    want[x0] = 1.0
    assert np.array_equal(got.astype(np.complex128), want)
    assert np.array_equal(l2p, np.arange(n))


@pytest.mark.parametrize("prec", [0, 1])
def test_one_and_two_qubit_states(q, prec):
    rng = np.random.default_rng(11)
    cases = [
        C(1, [G("h", (0,))]),
        C(1, [G("x", (0,)), G("rz", (0,), params=(0.3,)), G("sx", (0,))], x0=1),
        C(1, [G("u3", (0,), params=tuple(rng.uniform(0, 6.28, 3)))]),
        C(2, [G("h", (0,)), G("cx", (0, 1)), G("rzz", (0, 1), params=(0.7,))]),
        C(2, [G("dense", (1, 0), matrix=W.haar_unitary(rng, 4))], x0=2),
    ]
    for c in cases:
        got, _ = run(q, c, prec)
        err = float(np.max(np.abs(got.astype(np.complex128) - orc.run_circuit(c))))
        assert err <= TOL[prec], (c.n, [g.kind for g in c.gates], err)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n", [3, 16])
def test_swaps_only_move_no_amplitude(q, n, prec):
    """Virtual SWAPs: the device data keep the input basis state where it
    was, the layout records the permutation, and the logical readout equals
    the oracle's state."""
    rng = np.random.default_rng(n)
    gates = [G("swap", tuple(int(v) for v in rng.choice(n, 2, replace=False))) for _ in range(3 * n)]
    c = C(n, gates, x0=(1 << n) - 2)
    sim = q.Simulator(n, prec)
    sim.init_basis(c.x0)
    sim.apply(c.gates)
    phys = sim.state(order=q.ORDER_PHYSICAL)
    logical = sim.state()
    l2p = sim.layout()
    sim.close()
    assert np.array_equal(l2p, orc.expected_layout(n, gates))
    assert int(np.flatnonzero(phys)[0]) == c.x0 and np.count_nonzero(phys) == 1
    assert np.array_equal(logical.astype(np.complex128), orc.run_circuit(c))


@pytest.mark.parametrize("prec", [0, 1])
def test_diagonals_only(q, prec):
    """A 22-qubit circuit of phases only (Z, S, T, RZ, CZ, CP, RZZ) after a
    layer of H: every amplitude keeps its modulus."""
    n = 22
    rng = np.random.default_rng(5)
    gates = [G("h", (j,)) for j in range(n)]
    kinds = ["z", "s", "t", "rz", "cz", "cp", "rzz"]
    for _ in range(120):
        k = kinds[int(rng.integers(len(kinds)))]
        if k in ("cz", "cp", "rzz"):
            a, b = (int(v) for v in rng.choice(n, 2, replace=False))
            params = (float(rng.uniform(0, 6.28)),) if k != "cz" else ()
            gates.append(G(k, (a, b), params=params))
        else:
            params = (float(rng.uniform(0, 6.28)),) if k == "rz" else ()
            gates.append(G(k, (int(rng.integers(n)),), params=params))
    c = C(n, gates)
    got, _ = run(q, c, prec)
    ref = orc.run_circuit(c)
    assert float(np.max(np.abs(got.astype(np.complex128) - ref))) <= TOL[prec]
    assert float(np.max(np.abs(np.abs(got) - 2.0 ** (-n / 2)))) <= TOL[prec]


@pytest.mark.parametrize("prec", [0, 1])
def test_identity_blocks_change_nothing(q, prec):
    """Dense identity blocks of 2..6 qubits (matrix cores and the vector ALU)
    on a random state leave it unchanged."""
    n = 18
    rng = np.random.default_rng(9)
    psi = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    psi /= np.linalg.norm(psi)
    gates = []
    for k in (2, 3, 4, 5, 6, 6, 5, 3):
        qs = tuple(int(v) for v in rng.choice(n, k, replace=False))
        gates.append(G("dense", qs, matrix=np.eye(1 << k, dtype=np.complex128)))
    sim = q.Simulator(n, prec)
    sim.init_amplitudes(psi)
    sim.apply(gates)
    got = sim.state()
    sim.close()
    assert float(np.max(np.abs(got.astype(np.complex128) - psi))) <= TOL[prec]


@pytest.mark.parametrize("prec", [0, 1])
def test_gates_on_the_highest_qubit_only(q, prec):
    """Every gate acts on qubit n-1 (controls below it): the high-stride
    pairs of the sweep and the tile passes' upper bits."""
    n = 22
    rng = np.random.default_rng(4)
    gates = [G("h", (j,)) for j in range(0, n, 3)]
    for i in range(40):
        k = ["u3", "rx", "h", "x"][i % 4]
        params = tuple(float(v) for v in rng.uniform(0, 6.28, 3 if k == "u3" else 1)) if k in ("u3", "rx") else ()
        ctl = (int(rng.integers(n - 1)),) if i % 3 == 0 else ()
        gates.append(G(k, (n - 1,), controls=ctl, params=params))
    c = C(n, gates, x0=12345)
    for mode in (q.PLAN_FUSED, q.PLAN_GATEWISE):
        got, _ = run(q, c, prec, mode=mode)
        err = float(np.max(np.abs(got.astype(np.complex128) - orc.run_circuit(c))))
        assert err <= TOL[prec], (mode, err)
