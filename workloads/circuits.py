"""Seeded synthetic circuit generators.

This module only draws circuits: gate kinds, qubit indices, FP64 angles and,
for dense blocks, Haar-random unitaries.  It holds none of the simulation
arithmetic (no gate matrices, no state updates); the simulator and the FP64
checker each turn a gate description into numbers on their own.

Conventions (fixed for every consumer):
  * qubit q is bit q of the basis index (qubit 0 = least significant bit);
  * a gate on ordered qubits (q_0..q_{k-1}) has a matrix whose row/column
    index bit j belongs to q_j;
  * two-qubit kinds list their qubits as (q0, q1); for "cx" q0 is the control
    and q1 the target; "cz", "cp", "rzz" and "swap" are symmetric;
  * extra controls (all on |1>) go in ``controls``.

The workloads follow the paper's evaluation (Sec. IV): random layered circuits
stand in for its benchmark programs, a QFT followed by random layers for the
QFT scaling study (Table V), Haar-random fused blocks for the merged gates, and
a batch of parameterised RY/RZ + CZ circuits for the repeated-run QAOA study
(Sec. IV-E).  None of the paper's benchmark files are reproduced.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

TWO_PI = 2.0 * np.pi

ONE_QUBIT_FIXED = ("h", "x", "y", "z", "s", "sdg", "t", "tdg", "sx")
ONE_QUBIT_PARAM = {"rx": 1, "ry": 1, "rz": 1, "p": 1, "u3": 3}
TWO_QUBIT = {"cx": 0, "cz": 0, "cp": 1, "swap": 0, "rzz": 1}
ALL_KINDS = ONE_QUBIT_FIXED + tuple(ONE_QUBIT_PARAM) + tuple(TWO_QUBIT) + ("dense",)


@dataclass
class Gate:
    kind: str
    qubits: Tuple[int, ...]
    controls: Tuple[int, ...] = ()
    params: Tuple[float, ...] = ()
    matrix: Optional[np.ndarray] = field(default=None, repr=False)

    def all_qubits(self) -> Tuple[int, ...]:
        return tuple(self.qubits) + tuple(self.controls)


@dataclass
class Circuit:
    n: int
    gates: List[Gate]
    x0: int = 0                      # initial basis state |x0>
    name: str = ""

    def __len__(self) -> int:
        return len(self.gates)


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def haar_unitary(rng: np.random.Generator, dim: int) -> np.ndarray:
    """Haar-random unitary by Mezzadri's recipe: QR of a complex Gaussian
    matrix, with the phases of R's diagonal moved into Q."""
    z = (rng.standard_normal((dim, dim)) + 1j * rng.standard_normal((dim, dim))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r)
    return q * (d / np.abs(d))[None, :]


def _disjoint_pairs(rng: np.random.Generator, n: int) -> List[Tuple[int, int]]:
    p = rng.permutation(n)
    return [(int(p[2 * i]), int(p[2 * i + 1])) for i in range(n // 2)]


# ---------------------------------------------------------------------------
# Small named circuits (closed forms exist for these)
# ---------------------------------------------------------------------------

def ghz(n: int) -> Circuit:
    g = [Gate("h", (0,))] + [Gate("cx", (q - 1, q)) for q in range(1, n)]
    return Circuit(n, g, name=f"ghz{n}")


def qft_gates(n: int, with_swaps: bool = True) -> List[Gate]:
    """QFT with H and controlled phases pi/2^(j-m), then the reversal SWAPs."""
    g: List[Gate] = []
    for j in range(n - 1, -1, -1):
        g.append(Gate("h", (j,)))
        for m in range(j - 1, -1, -1):
            g.append(Gate("cp", (m, j), params=(np.pi / float(2 ** (j - m)),)))
    if with_swaps:
        for i in range(n // 2):
            g.append(Gate("swap", (i, n - 1 - i)))
    return g


def qft(n: int, x0: int = 0) -> Circuit:
    return Circuit(n, qft_gates(n), x0=x0, name=f"qft{n}")


def ry_cz_ladder(n: int, thetas: Sequence[float]) -> Circuit:
    g = [Gate("ry", (q,), params=(float(thetas[q]),)) for q in range(n)]
    g += [Gate("cz", (q, q + 1)) for q in range(n - 1)]
    return Circuit(n, g, name=f"rycz{n}")


def random_mixed(seed: int, n: int, ngates: int, kinds: Sequence[str] = ALL_KINDS,
                 max_dense_k: int = 3, max_ctrl: int = 2, ctrl_prob: float = 0.15) -> Circuit:
    """A random circuit over the whole gate set, with extra controls on some
    gates; used to cover every kind, qubit position and control pattern."""
    rng = rng_for(seed)
    gates: List[Gate] = []
    kinds = list(kinds)
    for _ in range(ngates):
        kind = kinds[int(rng.integers(len(kinds)))]
        if kind in ONE_QUBIT_FIXED or kind in ONE_QUBIT_PARAM:
            k = 1
        elif kind in TWO_QUBIT:
            k = 2
        else:
            k = int(rng.integers(1, min(max_dense_k, n) + 1))
        if k > n:
            continue
        qs = [int(v) for v in rng.choice(n, size=k, replace=False)]
        nparam = ONE_QUBIT_PARAM.get(kind, TWO_QUBIT.get(kind, 0))
        params = tuple(float(v) for v in rng.uniform(0.0, TWO_PI, size=nparam))
        mat = haar_unitary(rng, 2 ** k) if kind == "dense" else None
        ctrls: Tuple[int, ...] = ()
        if kind != "swap" and rng.random() < ctrl_prob:
            free = [q for q in range(n) if q not in qs]
            nc = int(rng.integers(1, max_ctrl + 1))
            nc = min(nc, len(free))
            if nc > 0:
                ctrls = tuple(int(v) for v in rng.choice(free, size=nc, replace=False))
        gates.append(Gate(kind, tuple(qs), ctrls, params, mat))
    x0 = int(rng.integers(2 ** n))
    return Circuit(n, gates, x0=x0, name=f"mixed{n}_s{seed}")


def inverse(c: Circuit) -> Circuit:
    """The circuit C^-1 (gates reversed, each replaced by its inverse).  Every
    inverse is stated as another gate description (an angle negation or a
    conjugate-transposed input block), so the simulators still build all
    matrices themselves."""
    inv: List[Gate] = []
    for g in reversed(c.gates):
        k, p = g.kind, g.params
        if k in ("h", "x", "y", "z", "cx", "cz", "swap"):
            inv.append(Gate(k, g.qubits, g.controls))
        elif k == "s":
            inv.append(Gate("sdg", g.qubits, g.controls))
        elif k == "sdg":
            inv.append(Gate("s", g.qubits, g.controls))
        elif k == "t":
            inv.append(Gate("tdg", g.qubits, g.controls))
        elif k == "tdg":
            inv.append(Gate("t", g.qubits, g.controls))
        elif k == "sx":
            # SX^-1 = SX^3
            inv += [Gate("sx", g.qubits, g.controls)] * 3
        elif k in ("rx", "ry", "rz", "p", "cp", "rzz"):
            inv.append(Gate(k, g.qubits, g.controls, (-p[0],)))
        elif k == "u3":
            inv.append(Gate("u3", g.qubits, g.controls, (-p[0], -p[2], -p[1])))
        elif k == "dense":
            inv.append(Gate("dense", g.qubits, g.controls, (), np.conj(g.matrix.T).copy()))
        else:
            raise ValueError(k)
    return Circuit(c.n, inv, name=c.name + "_inv")


# ---------------------------------------------------------------------------
# The five workload families
# ---------------------------------------------------------------------------

def layered_u3_cx(seed: int, n: int = 12, depth: int = 20, swap_frac: float = 0.1) -> Circuit:
    """Random layered circuit: U3 on every qubit (angles U[0, 2pi)), CNOTs on a
    random disjoint pairing (first of each pair controls), and a SWAP on a
    random pair appended to round(swap_frac*depth) randomly chosen layers."""
    rng = rng_for(seed)
    nswap = int(round(swap_frac * depth))
    swap_layers = set(int(v) for v in rng.choice(depth, size=nswap, replace=False))
    gates: List[Gate] = []
    for layer in range(depth):
        ang = rng.uniform(0.0, TWO_PI, size=(n, 3))
        for q in range(n):
            gates.append(Gate("u3", (q,), params=tuple(float(a) for a in ang[q])))
        for a, b in _disjoint_pairs(rng, n):
            gates.append(Gate("cx", (a, b)))
        if layer in swap_layers:
            a, b = (int(v) for v in rng.choice(n, size=2, replace=False))
            gates.append(Gate("swap", (a, b)))
    return Circuit(n, gates, name=f"layered{n}_d{depth}_s{seed}")


def qft_then_layers(seed: int = 1, n: int = 28, layers: int = 40) -> Circuit:
    """QFT of a seeded random basis state, then `layers` random layers of U3 on
    every qubit and CZ on a random disjoint pairing."""
    rng = rng_for(seed)
    x0 = int(rng.integers(2 ** n))
    gates = qft_gates(n)
    for _ in range(layers):
        ang = rng.uniform(0.0, TWO_PI, size=(n, 3))
        for q in range(n):
            gates.append(Gate("u3", (q,), params=tuple(float(a) for a in ang[q])))
        for a, b in _disjoint_pairs(rng, n):
            gates.append(Gate("cz", (a, b)))
    return Circuit(n, gates, x0=x0, name=f"qft{n}+{layers}layers_s{seed}")


def haar_blocks(seed: int = 2, n: int = 30, nblocks: int = 200, kmin: int = 2, kmax: int = 6) -> Circuit:
    """`nblocks` Haar-random dense blocks, k ~ U{kmin..kmax}, each on k distinct
    qubits drawn without replacement (the draw order is the matrix bit order)."""
    rng = rng_for(seed)
    gates: List[Gate] = []
    for _ in range(nblocks):
        k = int(rng.integers(kmin, kmax + 1))
        qs = tuple(int(v) for v in rng.choice(n, size=k, replace=False))
        gates.append(Gate("dense", qs, (), (), haar_unitary(rng, 2 ** k)))
    return Circuit(n, gates, name=f"haar{n}_b{nblocks}_s{seed}")


def random_mix_layers(seed: int, n: int, depth: int) -> Circuit:
    """Cost-model corpus circuit: per layer a random disjoint pairing; each
    pair gets one of {U3 x U3, CZ, SWAP, RZZ} (uniform); an odd qubit out gets
    a U3."""
    rng = rng_for(seed)
    gates: List[Gate] = []
    for _ in range(depth):
        pairs = _disjoint_pairs(rng, n)
        used = set()
        for a, b in pairs:
            used.update((a, b))
            c = int(rng.integers(4))
            if c == 0:
                for q in (a, b):
                    gates.append(Gate("u3", (q,), params=tuple(float(v) for v in rng.uniform(0, TWO_PI, 3))))
            elif c == 1:
                gates.append(Gate("cz", (a, b)))
            elif c == 2:
                gates.append(Gate("swap", (a, b)))
            else:
                gates.append(Gate("rzz", (a, b), params=(float(rng.uniform(0, TWO_PI)),)))
        for q in range(n):
            if q not in used:
                gates.append(Gate("u3", (q,), params=tuple(float(v) for v in rng.uniform(0, TWO_PI, 3))))
    return Circuit(n, gates, name=f"mix{n}_d{depth}_s{seed}")


def corpus_spec(seed: int) -> Tuple[int, int]:
    """(n, depth) of corpus circuit `seed`: n ~ U{20..30}, depth ~ U{20..100}."""
    rng = rng_for(seed)
    return int(rng.integers(20, 31)), int(rng.integers(20, 101))


def corpus_circuit(seed: int, n_override: Optional[int] = None) -> Circuit:
    n, depth = corpus_spec(seed)
    if n_override is not None:
        n = n_override
    return random_mix_layers(seed + 7919, n, depth)


def eval_circuit(seed: int, n: int = 32, depth: int = 60) -> Circuit:
    return random_mix_layers(seed, n, depth)


def param_sweep_batch(seed: int = 5, count: int = 512, nmin: int = 10, nmax: int = 22,
                      dmin: int = 8, dmax: int = 32) -> List[Circuit]:
    """Parameterised circuits: per layer RY and RZ (angles U[0, 2pi)) on every
    qubit, then a CZ ladder (q, q+1); n ~ U{nmin..nmax}, depth ~ U{dmin..dmax}."""
    rng = rng_for(seed)
    out: List[Circuit] = []
    for i in range(count):
        n = int(rng.integers(nmin, nmax + 1))
        d = int(rng.integers(dmin, dmax + 1))
        gates: List[Gate] = []
        for _ in range(d):
            ry = rng.uniform(0, TWO_PI, n)
            rz = rng.uniform(0, TWO_PI, n)
            for q in range(n):
                gates.append(Gate("ry", (q,), params=(float(ry[q]),)))
                gates.append(Gate("rz", (q,), params=(float(rz[q]),)))
            for q in range(n - 1):
                gates.append(Gate("cz", (q, q + 1)))
        out.append(Circuit(n, gates, name=f"sweep{i}_n{n}_d{d}"))
    return out


def clifford_t(seed: int, n: int, ngates: int, t_frac: float = 0.3) -> Circuit:
    """Seeded Clifford+T circuit (the gate mix of reversible arithmetic
    benchmarks): with probability t_frac a T or T-dagger, otherwise H, S, X, Z,
    CX or CZ, on uniformly drawn qubits."""
    rng = rng_for(seed)
    g: List[Gate] = []
    for _ in range(ngates):
        if rng.random() < t_frac:
            g.append(Gate("t" if rng.random() < 0.5 else "tdg", (int(rng.integers(n)),)))
            continue
        kind = ("h", "s", "x", "z", "cx", "cx", "cz")[int(rng.integers(7))]
        if kind in ("cx", "cz"):
            a, b = rng.choice(n, 2, replace=False)
            g.append(Gate(kind, (int(a), int(b))))
        else:
            g.append(Gate(kind, (int(rng.integers(n)),)))
    return Circuit(n, g, name=f"clifft{n}_{ngates}_s{seed}")


def regular_graph(seed: int, n: int, degree: int = 3) -> Tuple[List[Tuple[int, int]], np.ndarray]:
    """A seeded random degree-regular simple graph on n vertices (pairing
    model: shuffle the n*degree half-edges, pair them in order, redraw until
    there is no self-loop or double edge) and edge weights U[0.5, 1.5)."""
    rng = rng_for(seed)
    assert (n * degree) % 2 == 0 and degree < n
    while True:
        stubs = np.repeat(np.arange(n), degree)
        rng.shuffle(stubs)
        pairs = stubs.reshape(-1, 2)
        edges = {(int(min(a, b)), int(max(a, b))) for a, b in pairs}
        if len(edges) == len(pairs) and all(a != b for a, b in edges):
            break
    e = sorted(edges)
    return e, rng.uniform(0.5, 1.5, len(e))


def qaoa_maxcut(n: int, edges, weights, gammas: Sequence[float], betas: Sequence[float]) -> Circuit:
    """QAOA for weighted Max-Cut, C = sum_e w_e (1 - Z_a Z_b) / 2: H on every
    qubit, then per layer l the cost unitary exp(-i gamma_l C) (up to a global
    phase: RZZ(-gamma_l w_e) on every edge, RZZ(t) = exp(-i t/2 Z Z)) and the
    mixer exp(-i beta_l sum X) (RX(2 beta_l) on every qubit)."""
    g: List[Gate] = [Gate("h", (q,)) for q in range(n)]
    for gm, bt in zip(gammas, betas):
        for (a, b), w in zip(edges, weights):
            g.append(Gate("rzz", (int(a), int(b)), params=(float(-gm * w),)))
        for q in range(n):
            g.append(Gate("rx", (q,), params=(float(2.0 * bt),)))
    return Circuit(n, g, name=f"qaoa{n}_p{len(gammas)}")


def mlp_init(seed: int, sizes: Sequence[int] = (64, 128, 128, 1)) -> np.ndarray:
    """Seeded He-uniform initial weights of the cost-model perceptron, flat
    float64 in the order W1, b1, W2, b2, W3, b3 (W_i is out x in, row-major;
    biases start at zero)."""
    rng = rng_for(seed)
    parts = []
    for i in range(len(sizes) - 1):
        fan_in, fan_out = sizes[i], sizes[i + 1]
        lim = np.sqrt(6.0 / fan_in)
        parts.append(rng.uniform(-lim, lim, size=fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts)


def swap_positions(c: Circuit) -> List[int]:
    return [i for i, g in enumerate(c.gates) if g.kind == "swap"]
