"""A seeded circuit whose <Z_q> has a closed form at any size: RY rotations
on every qubit, then dense blocks that are Kronecker products of RY
rotations (so the state stays a product of real rotations; RY angles add),
then diagonal gates (CZ, RZ, CP), which leave every <Z_q> unchanged, then
SWAPs, which permute the qubits' states.  <Z_q> = cos(total RY angle of the
qubit whose state q holds at the end)."""
import numpy as np

from workloads import circuits as W


def _ry(a):
    c, s = np.cos(a / 2), np.sin(a / 2)
    return np.array([[c, -s], [s, c]], dtype=np.complex128)


def product_state_circuit(n: int, seed: int, block_widths=(6, 5, 4, 3, 6, 2)):
    """Returns (circuit, <Z_q> for q = 0..n-1)."""
    rng = np.random.default_rng(seed)
    theta = rng.uniform(0, np.pi, n)
    gates = [W.Gate("ry", (j,), params=(float(theta[j]),)) for j in range(n)]
    total = theta.copy()
    for k in block_widths:
        qs = tuple(int(v) for v in rng.choice(n, k, replace=False))
        phi = rng.uniform(0, np.pi, k)
        m = np.ones((1, 1), dtype=np.complex128)
        for j in range(k):
            m = np.kron(_ry(phi[j]), m)     # matrix bit j acts on qs[j]
        gates.append(W.Gate("dense", qs, matrix=m))
        for j, q in enumerate(qs):
            total[q] += phi[j]
    for j in range(0, n - 1, 2):
        gates.append(W.Gate("cz", (j, j + 1)))
    for j in range(n):
        gates.append(W.Gate("rz", (j,), params=(float(rng.uniform(0, 2 * np.pi)),)))
    for _ in range(3):
        a, b = (int(v) for v in rng.choice(n, 2, replace=False))
        gates.append(W.Gate("cp", (a, b), params=(float(rng.uniform(0, 2 * np.pi)),)))
    holder = list(range(n))
    for _ in range(4):
        a, b = (int(v) for v in rng.choice(n, 2, replace=False))
        gates.append(W.Gate("swap", (a, b)))
        holder[a], holder[b] = holder[b], holder[a]
    z = np.array([np.cos(total[holder[q]]) for q in range(n)])
    return W.Circuit(n, gates, name=f"product{n}_s{seed}"), z
