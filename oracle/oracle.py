"""Python side of the FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the package smoke check
and by the benchmark's CPU-baseline leg, never by the simulator.  It shares no
code with the GPU path; both sides read the same seeded gate descriptions
from ``workloads`` and build every number themselves.

Definitions followed (paper Sec. II-B): the state holds 2^n complex
amplitudes, updated gate by gate in list order; results are the final
probability distribution (or marginals of it) and Z expectation values.
Virtual swap (Sec. III-D): a SWAP handled virtually moves no amplitude and
only exchanges two entries of the logical-to-physical qubit map; the oracle
always applies SWAP physically and separately states the map a virtual
treatment must end with.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qops_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# The oracle's own kind numbering (matches the enum in qops_oracle.c).
KIND = {name: i for i, name in enumerate(
    ["h", "x", "y", "z", "s", "sdg", "t", "tdg", "sx", "rx", "ry", "rz", "p", "u3",
     "cx", "cz", "cp", "swap", "rzz", "dense"])}

_lib = None


def build(force: bool = False) -> str:
    """Compiles the oracle with gcc (FP64, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.orc_gate_matrix.argtypes = [ctypes.c_int, dp, ctypes.c_int, dp, dp]
        L.orc_apply_matrix.argtypes = [ctypes.c_int, dp, ctypes.c_int, ip, ctypes.c_int, ip, dp]
        L.orc_run.argtypes = [ctypes.c_int, dp, ctypes.c_int, ip, ip, ip, ip, ip, dp, dp,
                              ctypes.POINTER(ctypes.c_int64)]
        L.orc_basis.argtypes = [ctypes.c_int, dp, ctypes.c_uint64]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        L.orc_norm.argtypes = [ctypes.c_int, dp]
        L.orc_norm.restype = ctypes.c_double
        L.orc_probabilities.argtypes = [ctypes.c_int, dp, ctypes.c_int, ip, dp]
        L.orc_expect_z.argtypes = [ctypes.c_int, dp, dp]
        L.orc_expect_zz.argtypes = [ctypes.c_int, dp, ip, ctypes.c_int, dp]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def gate_matrix(kind: str, params: Sequence[float] = (), k: int = 1,
                dense: Optional[np.ndarray] = None) -> np.ndarray:
    """The oracle's matrix for one gate (complex128, 2^k x 2^k)."""
    prm = np.zeros(3, dtype=np.float64)
    prm[:len(params)] = params
    if kind == "dense":
        k = int(round(np.log2(dense.shape[0])))
        d = np.ascontiguousarray(dense.astype(np.complex128)).view(np.float64).ravel()
    else:
        k = 1 if KIND[kind] <= KIND["u3"] else 2
        d = np.zeros(2, dtype=np.float64)
    out = np.zeros(2 * 4 ** k, dtype=np.float64)
    rc = lib().orc_gate_matrix(KIND[kind], _dp(prm), k, _dp(d), _dp(out))
    if rc != 0:
        raise ValueError(f"oracle: bad gate {kind}")
    return out.view(np.complex128).reshape(2 ** k, 2 ** k)


class Marshalled:
    """A gate list laid out as the oracle's flat arrays."""

    def __init__(self, gates) -> None:
        m = len(gates)
        self.m = m
        self.kind = np.zeros(m, dtype=np.int32)
        self.nq = np.zeros(m, dtype=np.int32)
        self.qubits = np.zeros((m, 8), dtype=np.int32)
        self.nctrl = np.zeros(m, dtype=np.int32)
        self.ctrls = np.zeros((m, 8), dtype=np.int32)
        self.params = np.zeros((m, 3), dtype=np.float64)
        self.mat_off = np.zeros(m, dtype=np.int64)
        chunks: List[np.ndarray] = []
        off = 0
        for i, g in enumerate(gates):
            self.kind[i] = KIND[g.kind]
            self.nq[i] = len(g.qubits)
            self.qubits[i, :len(g.qubits)] = g.qubits
            self.nctrl[i] = len(g.controls)
            self.ctrls[i, :len(g.controls)] = g.controls
            self.params[i, :len(g.params)] = g.params
            if g.kind == "dense":
                d = np.ascontiguousarray(g.matrix.astype(np.complex128)).view(np.float64).ravel()
                self.mat_off[i] = off
                chunks.append(d)
                off += d.size
        self.mats = np.concatenate(chunks) if chunks else np.zeros(2, dtype=np.float64)


def basis_state(n: int, x0: int = 0) -> np.ndarray:
    psi = np.zeros(2 ** n, dtype=np.complex128)
    psi[x0] = 1.0
    return psi


def run(n: int, gates, psi: Optional[np.ndarray] = None, x0: int = 0) -> np.ndarray:
    """Applies `gates` in order to psi (default |x0>) and returns the state
    (complex128, logical index order)."""
    if psi is None:
        psi = basis_state(n, x0)
    psi = np.ascontiguousarray(psi, dtype=np.complex128).copy()
    mg = Marshalled(gates)
    flat = psi.view(np.float64)
    rc = lib().orc_run(n, _dp(flat), mg.m, _ip(mg.kind), _ip(mg.nq), _ip(mg.qubits), _ip(mg.nctrl),
                       _ip(mg.ctrls), _dp(mg.params), _dp(mg.mats),
                       mg.mat_off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if rc != 0:
        raise ValueError(f"oracle: gate {-rc - 1} rejected")
    return psi


def run_circuit(c) -> np.ndarray:
    return run(c.n, c.gates, x0=c.x0)


def apply_matrix(n: int, psi: np.ndarray, u: np.ndarray, qubits: Sequence[int],
                 controls: Sequence[int] = ()) -> np.ndarray:
    psi = np.ascontiguousarray(psi, dtype=np.complex128).copy()
    q = np.asarray(qubits, dtype=np.int32)
    c = np.asarray(list(controls) + [0], dtype=np.int32)
    uu = np.ascontiguousarray(u.astype(np.complex128)).view(np.float64).ravel()
    rc = lib().orc_apply_matrix(n, _dp(psi.view(np.float64)), len(q), _ip(q), len(controls), _ip(c), _dp(uu))
    if rc != 0:
        raise ValueError(f"oracle: apply rejected ({rc})")
    return psi


def apply_matrix_inplace(n: int, psi: np.ndarray, u: np.ndarray, qubits: Sequence[int]) -> None:
    """Like apply_matrix, without the copy (for large states)."""
    assert psi.dtype == np.complex128 and psi.flags.c_contiguous
    q = np.asarray(qubits, dtype=np.int32)
    c = np.zeros(1, dtype=np.int32)
    uu = np.ascontiguousarray(u.astype(np.complex128)).view(np.float64).ravel()
    rc = lib().orc_apply_matrix(n, _dp(psi.view(np.float64)), len(q), _ip(q), 0, _ip(c), _dp(uu))
    if rc != 0:
        raise ValueError(f"oracle: apply rejected ({rc})")


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(t: int) -> None:
    """Threads of the oracle's OpenMP loops from now on (timing only)."""
    lib().orc_set_num_threads(int(t))


def norm(psi: np.ndarray) -> float:
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    n = int(round(np.log2(psi.size)))
    return float(lib().orc_norm(n, _dp(psi.view(np.float64))))


def probabilities(psi: np.ndarray, qubits: Sequence[int]) -> np.ndarray:
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    n = int(round(np.log2(psi.size)))
    q = np.asarray(list(qubits) + [0], dtype=np.int32)
    out = np.zeros(2 ** len(qubits), dtype=np.float64)
    lib().orc_probabilities(n, _dp(psi.view(np.float64)), len(qubits), _ip(q), _dp(out))
    return out


def expect_z(psi: np.ndarray) -> np.ndarray:
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    n = int(round(np.log2(psi.size)))
    out = np.zeros(n, dtype=np.float64)
    lib().orc_expect_z(n, _dp(psi.view(np.float64)), _dp(out))
    return out


def expect_zz(psi: np.ndarray, pairs) -> np.ndarray:
    """<Z_a Z_b> for every (a, b) in pairs (Sec. IV-E: the correlators of a
    diagonal cost Hamiltonian)."""
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    n = int(round(np.log2(psi.size)))
    pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
    out = np.zeros(len(pr), dtype=np.float64)
    lib().orc_expect_zz(n, _dp(psi.view(np.float64)), pr.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), len(pr),
                        _dp(out))
    return out


def maxcut_expectation(zz: np.ndarray, weights) -> float:
    """<C> of the Max-Cut cost C = sum_e w_e (1 - Z_a Z_b) / 2 from its
    correlators."""
    w = np.asarray(weights, dtype=np.float64)
    return float(np.sum(w * (1.0 - np.asarray(zz, dtype=np.float64))) / 2.0)


def expected_layout(n: int, gates, virtual_swaps: bool = True) -> np.ndarray:
    """The logical-to-physical map after the circuit when every SWAP is taken
    virtually: start from the identity and exchange the two entries of each
    SWAP (Sec. III-D, virtual swap).  With virtual_swaps False it stays the
    identity."""
    l2p = np.arange(n, dtype=np.int32)
    if virtual_swaps:
        for g in gates:
            if g.kind == "swap" and not g.controls:
                a, b = g.qubits
                l2p[a], l2p[b] = l2p[b], l2p[a]
    return l2p


def logical_from_physical(phys: np.ndarray, l2p: Sequence[int]) -> np.ndarray:
    """psi_logical[x] = psi_physical[sum_q b_q(x) 2^{l2p[q]}] (exact index map)."""
    n = len(l2p)
    x = np.arange(2 ** n, dtype=np.int64)
    idx = np.zeros_like(x)
    for q in range(n):
        idx |= ((x >> q) & 1) << int(l2p[q])
    return phys[idx]


def fidelity(a: np.ndarray, b: np.ndarray) -> float:
    """|<a|b>|^2 in FP64."""
    return float(abs(np.vdot(a.astype(np.complex128), b.astype(np.complex128))) ** 2)


def max_abs(a: np.ndarray, b: np.ndarray) -> float:
    return float(np.max(np.abs(a.astype(np.complex128) - b.astype(np.complex128))))
