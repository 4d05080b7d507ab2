"""Pins the FP64 oracle to facts that do not come from the oracle itself:
algebraic identities between gate matrices, an independent tensor-contraction
simulator for small n, closed forms (GHZ, QFT of a basis state, RY + CZ
expectations), circuit-then-inverse, norm preservation and the virtual-swap
layout rule.  CPU only."""
import numpy as np
import pytest
import scipy.linalg

from oracle import oracle as orc
from oracle import mlp_oracle as mlp
from workloads import circuits as W

TOL = 1e-13


def M(kind, *params, dense=None):
    return orc.gate_matrix(kind, params, dense=dense)


I2 = np.eye(2)


def close(a, b, tol=TOL):
    return np.max(np.abs(np.asarray(a) - np.asarray(b))) <= tol


# ---------------------------------------------------------------- matrices --

@pytest.mark.parametrize("kind", ["h", "x", "y", "z", "s", "sdg", "t", "tdg", "sx"])
def test_fixed_gates_unitary(kind):
    u = M(kind)
    assert close(u.conj().T @ u, np.eye(2))


def test_pauli_and_clifford_identities():
    X, Y, Z, H, S, T = M("x"), M("y"), M("z"), M("h"), M("s"), M("t")
    assert close(X @ X, I2) and close(Y @ Y, I2) and close(Z @ Z, I2)
    assert close(X @ Y, 1j * Z)            # Pauli algebra fixes the sign of Y
    assert close(H @ X @ H, Z) and close(H @ Z @ H, X)
    assert close(S @ S, Z) and close(T @ T, S)
    assert close(M("sdg"), S.conj().T) and close(M("tdg"), T.conj().T)
    assert close(M("sx") @ M("sx"), X)
    assert close(Z, np.diag([1, -1]))      # |0> is the +1 eigenvector of Z
    assert close(H @ np.array([1, 0]), np.array([1, 1]) / np.sqrt(2))


@pytest.mark.parametrize("theta", [0.0, 0.3, 1.7, np.pi, 4.1, 2 * np.pi - 0.2])
def test_rotations_are_pauli_exponentials(theta):
    X, Y, Z = M("x"), M("y"), M("z")
    assert close(M("rx", theta), scipy.linalg.expm(-0.5j * theta * X))
    assert close(M("ry", theta), scipy.linalg.expm(-0.5j * theta * Y))
    assert close(M("rz", theta), scipy.linalg.expm(-0.5j * theta * Z))
    assert close(M("p", theta), np.exp(0.5j * theta) * M("rz", theta))


@pytest.mark.parametrize("seed", range(6))
def test_u3_is_zyz(seed):
    rng = np.random.default_rng(seed)
    t, p, l = rng.uniform(0, 2 * np.pi, 3)
    zyz = np.exp(0.5j * (p + l)) * M("rz", p) @ M("ry", t) @ M("rz", l)
    assert close(M("u3", t, p, l), zyz)
    assert close(M("u3", t, -np.pi / 2, np.pi / 2), M("rx", t))
    assert close(M("u3", t, 0, 0), M("ry", t))


def test_two_qubit_gates():
    X, Z = M("x"), M("z")
    P0, P1 = np.diag([1, 0]), np.diag([0, 1])
    # index bit 0 <-> first listed qubit, so kron(op_on_q1, op_on_q0)
    assert close(M("cx"), np.kron(I2, P0) + np.kron(X, P1))
    assert close(M("cz"), np.kron(I2, P0) + np.kron(Z, P1))
    for lam in (0.4, np.pi, 5.0):
        assert close(M("cp", lam), np.kron(I2, P0) + np.kron(M("p", lam), P1))
        assert close(M("rzz", lam), scipy.linalg.expm(-0.5j * lam * np.kron(Z, Z)))
    assert close(M("cp", np.pi), M("cz"))
    A, B = M("u3", 0.3, 1.1, 2.3), M("h")
    sw = M("swap")
    assert close(sw @ np.kron(A, B) @ sw, np.kron(B, A))


def test_dense_passthrough_and_haar_unitarity():
    rng = W.rng_for(11)
    for k in range(1, 7):
        u = W.haar_unitary(rng, 2 ** k)
        assert np.max(np.abs(u.conj().T @ u - np.eye(2 ** k))) <= 1e-13
        assert close(M("dense", dense=u), u)


# ---------------------------------------------- independent small simulator --

def tensor_apply(psi, n, u, qubits, controls=()):
    """Independent reference: contract the gate with the state viewed as an
    n-axis tensor (axis n-1-q holds qubit q), restricted to the slice where
    every control qubit is 1."""
    k = len(qubits)
    t = psi.reshape([2] * n).copy()
    ax = [n - 1 - q for q in qubits]
    sl = [slice(None)] * n
    for c in controls:
        sl[n - 1 - c] = 1
    sl = tuple(sl)
    sub = t[sl]
    # axes of `sub`: remove the control axes, keep order
    remaining = [a for a in range(n) if not any(a == n - 1 - c for c in controls)]
    sax = [remaining.index(a) for a in ax]
    # u index bit j <-> qubit j; as a tensor: u[(r_{k-1}..r_0), (s_{k-1}..s_0)]
    ut = u.reshape([2] * (2 * k))
    # ut axes: out bits (k-1..0), in bits (k-1..0); qubit j's in-axis is 2k-1-j
    in_axes = [2 * k - 1 - j for j in range(k)]
    moved = np.tensordot(ut, sub, axes=(in_axes, sax))
    # moved axes: out bits (k-1..0) then the untouched sub axes in order
    out_pos = [k - 1 - j for j in range(k)]        # position of qubit j's out-axis
    rest = [a for a in range(sub.ndim) if a not in sax]
    order = [None] * sub.ndim
    for j in range(k):
        order[sax[j]] = out_pos[j]
    for i, a in enumerate(rest):
        order[a] = k + i
    t[sl] = np.transpose(moved, order)
    return t.reshape(-1)


def kron_embed_1q(n, u, q):
    """Full 2^n x 2^n matrix of a one-qubit gate by Kronecker products."""
    full = np.array([[1.0 + 0j]])
    for j in range(n - 1, -1, -1):
        full = np.kron(full, u if j == q else I2)
    return full


def test_tensor_reference_matches_kronecker():
    rng = np.random.default_rng(1)
    n = 5
    psi = rng.normal(size=2 ** n) + 1j * rng.normal(size=2 ** n)
    u = M("u3", 0.7, 1.9, 2.6)
    for q in range(n):
        assert close(tensor_apply(psi, n, u, [q]), kron_embed_1q(n, u, q) @ psi, 1e-12)


@pytest.mark.parametrize("n", [3, 5, 8])
@pytest.mark.parametrize("seed", range(4))
def test_oracle_matches_tensor_reference(n, seed):
    c = W.random_mixed(seed * 31 + n, n, 60, max_dense_k=min(3, n))
    rng = np.random.default_rng(seed)
    psi0 = rng.normal(size=2 ** n) + 1j * rng.normal(size=2 ** n)
    psi0 /= np.linalg.norm(psi0)
    ref = psi0.copy()
    for g in c.gates:
        u = M(g.kind, *g.params, dense=g.matrix)
        ref = tensor_apply(ref, n, u, list(g.qubits), list(g.controls))
    got = orc.run(n, c.gates, psi=psi0)
    assert np.max(np.abs(got - ref)) <= 1e-13


def test_full_unitary_product_n4():
    """Brute force: the ordered product of full embeddings, applied to e_0 and
    to random states, equals the oracle's gate-by-gate result."""
    n = 4
    c = W.random_mixed(77, n, 30, max_dense_k=3)
    U = np.eye(2 ** n, dtype=np.complex128)
    for g in c.gates:
        u = M(g.kind, *g.params, dense=g.matrix)
        cols = [tensor_apply(np.eye(2 ** n)[:, j].astype(complex), n, u, list(g.qubits), list(g.controls))
                for j in range(2 ** n)]
        U = np.stack(cols, axis=1) @ U
    rng = np.random.default_rng(3)
    for trial in range(4):
        psi = np.zeros(2 ** n, complex)
        if trial == 0:
            psi[0] = 1
        else:
            psi = rng.normal(size=2 ** n) + 1j * rng.normal(size=2 ** n)
        assert np.max(np.abs(orc.run(n, c.gates, psi=psi) - U @ psi)) <= 1e-13


# ------------------------------------------------------------- closed forms --

@pytest.mark.parametrize("n", [2, 3, 7, 12, 16])
def test_ghz(n):
    psi = orc.run_circuit(W.ghz(n))
    ref = np.zeros(2 ** n, complex)
    ref[0] = ref[-1] = 1 / np.sqrt(2)
    assert np.max(np.abs(psi - ref)) <= 1e-15
    p = orc.probabilities(psi, list(range(n)))
    assert abs(p[0] - 0.5) < 1e-15 and abs(p[-1] - 0.5) < 1e-15
    assert np.max(np.abs(orc.expect_z(psi))) < 1e-15


@pytest.mark.parametrize("n,x0", [(3, 5), (5, 19), (8, 201), (12, 3001), (14, 12345)])
def test_qft_of_basis_state(n, x0):
    psi = orc.run_circuit(W.qft(n, x0))
    y = np.arange(2 ** n, dtype=np.int64)
    phase = 2 * np.pi * ((x0 * y) % (2 ** n)) / 2 ** n     # integer product, no FP loss
    ref = np.exp(1j * phase) / np.sqrt(2 ** n)
    assert np.max(np.abs(psi - ref)) <= 1e-12
    assert np.max(np.abs(np.abs(psi) - 2 ** (-n / 2))) <= 1e-13


@pytest.mark.parametrize("n", [4, 9, 13])
def test_ry_cz_ladder_expectations(n):
    th = np.random.default_rng(n).uniform(0, 2 * np.pi, n)
    psi = orc.run_circuit(W.ry_cz_ladder(n, th))
    assert np.max(np.abs(orc.expect_z(psi) - np.cos(th))) <= 1e-13


@pytest.mark.parametrize("n,seed", [(8, 1), (11, 2), (13, 3)])
def test_product_state_circuit_expectations(n, seed):
    """The closed form the largest-size GPU test relies on: RY layers,
    Kronecker-product RY blocks, diagonals and SWAPs give <Z_q> = cos of the
    summed RY angles of the qubit state that q holds."""
    from product_state import product_state_circuit
    c, z = product_state_circuit(n, seed)
    psi = orc.run_circuit(c)
    assert abs(np.vdot(psi, psi).real - 1.0) <= 1e-13
    assert np.max(np.abs(orc.expect_z(psi) - z)) <= 1e-13


@pytest.mark.parametrize("seed", range(5))
def test_circuit_then_inverse(seed):
    n = 7
    c = W.random_mixed(seed, n, 80, max_dense_k=4)
    both = c.gates + W.inverse(c).gates
    psi = orc.run(n, both, x0=c.x0)
    ref = orc.basis_state(n, c.x0)
    assert np.max(np.abs(psi - ref)) <= 1e-12


def test_norm_preserved_and_measurements_independent():
    n = 10
    c = W.random_mixed(5, n, 120, max_dense_k=3)
    psi = orc.run_circuit(c)
    assert abs(orc.norm(psi) - 1.0) <= 1e-12
    p = np.abs(psi) ** 2
    assert abs(orc.norm(psi) - p.sum()) <= 1e-14
    qs = [7, 2, 4]
    t = p.reshape([2] * n)
    keep = [n - 1 - q for q in qs]
    marg = t.sum(axis=tuple(a for a in range(n) if a not in keep))
    # marg axes are in increasing axis order = decreasing qubit order among qs
    got = orc.probabilities(psi, qs).reshape([2] * len(qs))  # axes: bit2 (q=4), bit1 (q=2), bit0 (q=7)
    srt = sorted(qs, reverse=True)                           # qubits in marg's axis order
    perm = [srt.index(q) for q in reversed(qs)]
    assert np.max(np.abs(np.transpose(marg, perm) - got)) <= 1e-14
    z = orc.expect_z(psi)
    for q in range(n):
        bits = (np.arange(2 ** n) >> q) & 1
        assert abs(z[q] - np.sum(p * (1 - 2 * bits))) <= 1e-13


def test_virtual_swap_layout_rule():
    """Dropping every SWAP and reading the result through the expected
    logical-to-physical map gives the state of the circuit with SWAPs."""
    n = 9
    c = W.layered_u3_cx(3, n=n, depth=12, swap_frac=0.5)
    assert any(g.kind == "swap" for g in c.gates)
    with_swaps = orc.run_circuit(c)
    # without swaps: relabel the remaining gates through the running map
    l2p = np.arange(n)
    relabelled = []
    for g in c.gates:
        if g.kind == "swap":
            a, b = g.qubits
            l2p[a], l2p[b] = l2p[b], l2p[a]
        else:
            relabelled.append(W.Gate(g.kind, tuple(int(l2p[q]) for q in g.qubits),
                                     tuple(int(l2p[q]) for q in g.controls), g.params, g.matrix))
    phys = orc.run(n, relabelled)
    expected = orc.expected_layout(n, c.gates)
    assert np.array_equal(expected, l2p)
    assert np.max(np.abs(orc.logical_from_physical(phys, expected) - with_swaps)) <= 1e-13


def test_oracle_rejects_bad_gates():
    with pytest.raises(ValueError):
        orc.run(3, [W.Gate("cx", (1, 1))])
    with pytest.raises(ValueError):
        orc.run(3, [W.Gate("h", (3,))])
    with pytest.raises(ValueError):
        orc.run(3, [W.Gate("x", (0,), controls=(0,))])


# ------------------------------------------------------------------ MLP -----

def test_mlp_gradients_match_finite_differences():
    p = mlp.init_params(7)
    rng = np.random.default_rng(0)
    X = rng.normal(size=(9, 64))
    t = rng.normal(size=9)
    _, g = mlp.backward(p, X, t)
    h = 1e-6
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        flat = p[name].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = mlp.loss(p, X, t)
            flat[idx] = old - h
            lm = mlp.loss(p, X, t)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = g[name].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (name, idx, fd, an)


def _sparse_params():
    """Small fixed weights with most entries zero, so that the forward pass
    can be followed by hand (only the first few units are live)."""
    p = {k: np.zeros_like(v) for k, v in mlp.init_params(0).items()}
    p["W1"][0, :2] = [1.0, 1.0]
    p["W1"][1, :2] = [1.0, -1.0]
    p["W1"][2, :2] = [0.5, 0.0]
    p["b1"][:3] = [0.0, 0.5, -2.0]
    p["W2"][0, :3] = [1.0, 1.0, 1.0]
    p["W2"][1, :3] = [0.0, -1.0, 0.0]
    p["b2"][:2] = [0.0, 1.0]
    p["W3"][0, :2] = [2.0, -3.0]
    p["b3"][0] = 0.25
    return p


def test_mlp_forward_hand_computed():
    """Two rows through the 64-128-128-1 perceptron, worked by hand:
    row a = (2, -1, 0, ...):  z1 = (2-1, 2+1+0.5, 1-2) = (1, 3.5, -1) -> h1 = (1, 3.5, 0)
                              z2 = (1+3.5+0, -3.5+1) = (4.5, -2.5)     -> h2 = (4.5, 0)
                              y  = 2*4.5 - 3*0 + 0.25 = 9.25
    row b = (-1, 3, 0, ...):  z1 = (-1+3, -1-3+0.5, -0.5-2) = (2, -3.5, -2.5) -> h1 = (2, 0, 0)
                              z2 = (2, 0+1) = (2, 1)                    -> h2 = (2, 1)
                              y  = 2*2 - 3*1 + 0.25 = 1.25
    Both ReLUs clip a negative pre-activation that would otherwise reach the
    output (z1[2] of row a through W2[0, 2]; z2[1] of row a through W3), and
    every bias enters.  With targets (9, 2) the mean squared error is
    ((0.25)^2 + (-0.75)^2) / 2 = 0.3125."""
    p = _sparse_params()
    X = np.zeros((2, 64))
    X[0, :2] = [2.0, -1.0]
    X[1, :2] = [-1.0, 3.0]
    y, cache = mlp.forward(p, X)
    assert np.array_equal(y, [9.25, 1.25])
    assert np.array_equal(cache["h1"][:, :3], [[1.0, 3.5, 0.0], [2.0, 0.0, 0.0]])
    assert np.array_equal(cache["h2"][:, :2], [[4.5, 0.0], [2.0, 1.0]])
    assert not cache["h1"][:, 3:].any() and not cache["h2"][:, 2:].any()
    assert mlp.loss(p, X, [9.0, 2.0]) == 0.3125


def test_mlp_backward_hand_computed():
    """Gradient of the hand-worked case above.  dL/dy = 2 (y - t) / B =
    (0.25, -0.75); dL/db3 = -0.5; dL/dW3 = 0.25*h2_a + (-0.75)*h2_b =
    (1.125 - 1.5, -0.75) = (-0.375, -0.75)."""
    p = _sparse_params()
    X = np.zeros((2, 64))
    X[0, :2] = [2.0, -1.0]
    X[1, :2] = [-1.0, 3.0]
    _, g = mlp.backward(p, X, [9.0, 2.0])
    assert g["b3"][0] == -0.5
    assert np.array_equal(g["W3"][0, :2], [-0.375, -0.75]) and not g["W3"][0, 2:].any()
    # unit 0 of layer 2 is live for both rows: dL/db2[0] = W3[0] * sum dy = 2 * (-0.5)
    # unit 1 only for row b: dL/db2[1] = W3[1] * dy_b = -3 * -0.75
    assert np.array_equal(g["b2"][:2], [-1.0, 2.25])


def test_adam_first_step_closed_form():
    """Kingma & Ba: from zero moments, the bias-corrected first step is
    lr * g / (|g| + eps) element-wise (bias correction undoes the (1 - beta)
    factors exactly).  A large eps makes its placement visible: eps added
    inside the square root, or a missing bias correction, give other values."""
    g = {"w": np.array([0.5, -2.0, 1e-3, 0.0])}
    for eps in (1e-8, 0.1):
        p = {"w": np.array([1.0, 1.0, 1.0, 1.0])}
        m = {"w": np.zeros(4)}
        v = {"w": np.zeros(4)}
        mlp.adam_step(p, g, m, v, 1, 0.1, eps=eps)
        want = 1.0 - 0.1 * g["w"] / (np.abs(g["w"]) + eps)
        assert np.max(np.abs(p["w"] - want)) <= 1e-15
    # eps = 0.1, g = 0.5: 1 - 0.1 * 0.5 / 0.6 exactly
    assert abs(p["w"][0] - (1.0 - 0.05 / 0.6)) <= 1e-15


def test_adam_second_step_hand_computed():
    """Two steps with gradients 0.5 then -0.25, lr 0.1, betas (0.9, 0.999):
    m2 = 0.9*0.05 - 0.025 = 0.02, corrected 0.02 / 0.19 = 2/19;
    v2 = 0.999*0.00025 + 0.001*0.0625 = 0.00031225, corrected
    0.00031225 / 0.001999 = 312.25 / 1999."""
    eps = 1e-8
    p = {"w": np.array([0.0])}
    m = {"w": np.zeros(1)}
    v = {"w": np.zeros(1)}
    mlp.adam_step(p, {"w": np.array([0.5])}, m, v, 1, 0.1, eps=eps)
    mlp.adam_step(p, {"w": np.array([-0.25])}, m, v, 2, 0.1, eps=eps)
    assert abs(m["w"][0] - 0.02) <= 1e-17 and abs(v["w"][0] - 0.00031225) <= 1e-18
    step1 = 0.1 * 0.5 / (0.5 + eps)
    step2 = 0.1 * (2.0 / 19.0) / (np.sqrt(312.25 / 1999.0) + eps)
    assert abs(p["w"][0] - (-step1 - step2)) <= 1e-15


def test_adam_reduces_loss():
    p = mlp.init_params(1)
    rng = np.random.default_rng(1)
    X = rng.normal(size=(64, 64))
    t = X[:, 0] * 0.5 - X[:, 1]
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(v) for k, v in p.items()}
    l0 = mlp.loss(p, X, t)
    for s in range(1, 201):
        _, g = mlp.backward(p, X, t)
        mlp.adam_step(p, g, m, v, s, 1e-3)
    assert mlp.loss(p, X, t) < 0.1 * l0


# ---------------------------------------------------------------------------
# Two-qubit correlators and the Max-Cut cost (repeated QAOA runs, Sec. IV-E)
# ---------------------------------------------------------------------------

def test_expect_zz_closed_forms():
    n = 6
    # GHZ: every pair perfectly correlated
    pairs = [(a, b) for a in range(n) for b in range(a + 1, n)]
    zz = orc.expect_zz(orc.run_circuit(W.ghz(n)), pairs)
    assert np.allclose(zz, 1.0, atol=1e-14)
    # product state RY(t_q)|0>: <Z_a Z_b> = cos t_a cos t_b; <Z_a Z_a> = 1
    th = np.linspace(0.3, 2.9, n)
    c = W.Circuit(n, [W.Gate("ry", (q,), params=(float(th[q]),)) for q in range(n)])
    zz = orc.expect_zz(orc.run_circuit(c), pairs + [(2, 2)])
    ref = [np.cos(th[a]) * np.cos(th[b]) for a, b in pairs] + [1.0]
    assert np.max(np.abs(zz - ref)) < 1e-14


def test_maxcut_of_basis_states_is_the_cut_weight():
    edges, w = W.regular_graph(3, 8, 3)
    for x in (0, 0b10110010, 0b11111111, 0b01010101):
        zz = orc.expect_zz(orc.basis_state(8, x), edges)
        cut = sum(wi for (a, b), wi in zip(edges, w) if ((x >> a) ^ (x >> b)) & 1)
        assert abs(orc.maxcut_expectation(zz, w) - cut) < 1e-13


def test_qaoa_single_edge_closed_form():
    # one edge, p = 1: <C> = 1/2 + sin(4 beta) sin(gamma) / 2
    for gm, bt in ((0.3, 0.7), (1.1, 0.2), (2.0, 1.3)):
        c = W.qaoa_maxcut(2, [(0, 1)], [1.0], [gm], [bt])
        zz = orc.expect_zz(orc.run_circuit(c), [(0, 1)])
        assert abs(orc.maxcut_expectation(zz, [1.0]) - (0.5 + 0.5 * np.sin(4 * bt) * np.sin(gm))) < 1e-13


def test_qaoa_matches_dense_matrix_exponentials():
    """n = 6, p = 2 on a weighted graph against numpy matrix exponentials of
    the cost and mixer Hamiltonians built from Kronecker products."""
    from scipy.linalg import expm
    n = 6
    edges, w = W.regular_graph(1, n, 3)
    gms, bts = [0.4, 0.9], [0.6, 0.25]
    X = np.array([[0, 1], [1, 0]], dtype=complex)
    Z = np.diag([1.0, -1.0]).astype(complex)

    def on(op, q):   # qubit q = bit q: the Kronecker factor order is reversed
        mats = [np.eye(2, dtype=complex)] * n
        mats = list(mats)
        mats[n - 1 - q] = op
        out = mats[0]
        for m in mats[1:]:
            out = np.kron(out, m)
        return out
    C = sum(wi * (np.eye(2 ** n) - on(Z, a) @ on(Z, b)) / 2 for (a, b), wi in zip(edges, w))
    B = sum(on(X, q) for q in range(n))
    psi = np.ones(2 ** n, dtype=complex) / np.sqrt(2 ** n)
    for gm, bt in zip(gms, bts):
        psi = expm(-1j * bt * B) @ (expm(-1j * gm * C) @ psi)
    ref = float(np.real(np.conj(psi) @ C @ psi))
    got_psi = orc.run_circuit(W.qaoa_maxcut(n, edges, w, gms, bts))
    # equal up to a global phase; the expectation is phase free
    assert abs(abs(np.vdot(psi, got_psi)) - 1) < 1e-12
    assert abs(orc.maxcut_expectation(orc.expect_zz(got_psi, edges), w) - ref) < 1e-12
