"""GPU parity on the paths a full-size state takes, at sizes the FP64 oracle
still finishes in seconds:

* work-groups that walk many tiles: every state-pass kernel under a launch
  limit of 1, 3 and 7 work-groups (the persistent LDS tile loop with its
  prefetch of the next tile and the stores that drain under it, the
  register tile loop, grid-stride sweeps and bit exchanges), against the
  oracle, element by element;
* the default launch at 23 and 24 qubits, where the LDS tile kernel's
  persistent grid gives each work-group 4 (complex64, 24 qubits) to 16
  (complex128, 24 qubits) tiles, and the gate-wise sweeps stride past their
  grid;
* gates with 3 and 4 controls;
* a profiling run: its state is the normal result and its gate counters
  equal a tally of the gate list.

Tolerances as everywhere: max-abs <= 2e-5 (complex64), <= 1e-12
(complex128); layouts bit-exact."""
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


_REF = {}


def oracle_state(c):
    key = (c.name, c.n, len(c.gates))
    if key not in _REF:
        _REF[key] = orc.run_circuit(c)
    return _REF[key]


def run_gpu(q, c, prec, limit=0, **opts):
    print(f"[case] {c.name} n={c.n} prec={prec} limit={limit} opts={opts}", flush=True)
    sim = q.Simulator(c.n, prec)
    sim.set_launch_limit(limit)
    sim.init_basis(c.x0)
    sim.apply(c.gates, **opts)
    out = sim.state()
    l2p = sim.layout()
    sim.close()
    return out, l2p


def check(got, ref, prec, what):
    err = float(np.max(np.abs(got.astype(np.complex128) - ref)))
    assert err <= TOL[prec], f"{what}: max-abs {err:.3e} > {TOL[prec]:.0e}"
    return err


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("limit", [1, 3, 7])
def test_lds_tiles_many_per_workgroup(q, prec, limit):
    """LDS tile passes of every width (the full tile with branch-free loads
    and stores, the smaller element-tested ones) with each work-group
    walking 2^16 / 2^L / limit tiles."""
    c = W.haar_blocks(7, n=16, nblocks=30)
    ref = oracle_state(c)
    for tile_upper in (4, 6, 7):
        got, _ = run_gpu(q, c, prec, limit, tile_upper=tile_upper)
        check(got, ref, prec, f"lds tiles upper={tile_upper} limit={limit}")


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("limit", [1, 3])
def test_hoisted_blocks_across_tiles(q, prec, limit):
    """A 6-qubit block whose fragments stay in registers across all tiles
    of a work-group, with 5-qubit blocks staged in LDS, on 2^20 amplitudes."""
    rng = W.rng_for(31)
    mk = lambda qs: W.Gate("dense", tuple(qs), (), (), W.haar_unitary(rng, 2 ** len(qs)))
    gates = [mk((0, 1, 2, 8, 9, 10)), mk((3, 4, 11, 12, 13)), mk((1, 5, 8, 11, 14)), mk((2, 9, 12, 4, 0)),
             mk((6, 7, 15, 16, 17, 18)), mk((19, 6, 15, 3, 0))]
    c = W.Circuit(20, gates, name="wide20")
    got, _ = run_gpu(q, c, prec, limit)
    check(got, oracle_state(c), prec, f"hoisted limit={limit}")


@pytest.mark.parametrize("limit", [0, 3])
def test_five_qubit_blocks_with_controls_full_tile(q, limit):
    """complex64 on 2^13-amplitude tiles, where 5-qubit blocks run the 32x32x2
    form: two 5-qubit blocks per pass (one keeps its fragments in registers,
    the other reads them from LDS), with controls on tile positions and on
    bits outside the tile, and a 6-qubit block beside a 5-qubit one."""
    rng = W.rng_for(53)
    mk = lambda qs, cs=(): W.Gate("dense", tuple(qs), tuple(cs), (), W.haar_unitary(rng, 2 ** len(qs)))
    gates = [mk((0, 3, 7, 9, 12)), mk((1, 2, 8, 10, 11), (4,)), mk((5, 6, 13, 14, 15), (0, 12)),
             mk((2, 4, 9, 11, 13), (16,)), mk((0, 1, 5, 8, 12, 15)), mk((3, 6, 10, 14, 16), (2, 7)),
             mk((1, 7, 11, 12, 16))]
    c = W.Circuit(17, gates, x0=12345, name="wide5ctl17")
    got, l2p = run_gpu(q, c, 0, limit)
    check(got, oracle_state(c), 0, f"5-qubit blocks with controls limit={limit}")
    assert np.array_equal(l2p, orc.expected_layout(c.n, c.gates))


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("limit", [1, 5])
def test_register_tiles_and_sweeps_many_per_workgroup(q, prec, limit):
    """Register tile passes (fused plans), gate-wise sweeps and physical bit
    exchanges with a small grid, so every loop strides."""
    c = W.random_mixed(41, 17, 160, max_dense_k=6, max_ctrl=4, ctrl_prob=0.3)
    ref = oracle_state(c)
    got, l2p = run_gpu(q, c, prec, limit)
    check(got, ref, prec, f"fused limit={limit}")
    assert np.array_equal(l2p, orc.expected_layout(c.n, c.gates))
    got, _ = run_gpu(q, c, prec, limit, mode=q.PLAN_GATEWISE)
    check(got, ref, prec, f"gatewise limit={limit}")
    got, l2p = run_gpu(q, c, prec, limit, swap_mode=q.SWAP_PHYSICAL)
    check(got, ref, prec, f"physical swaps limit={limit}")
    assert np.array_equal(l2p, np.arange(c.n))


@pytest.mark.parametrize("prec,n", [(0, 24), (1, 23), (1, 24)])
def test_haar_blocks_default_launch_several_tiles_each(q, prec, n):
    """The benchmark's circuit family (Haar blocks, k ~ U{2..6}) with the
    default plan and launch at 23-24 qubits: 2^(n-L) LDS tiles over the
    persistent grid (512 work-groups for complex64, 256 for complex128), so
    each work-group processes 4 to 16 tiles."""
    c = W.haar_blocks(2, n=n, nblocks=60)
    got, l2p = run_gpu(q, c, prec)
    err = check(got, oracle_state(c), prec, f"haar n={n}")
    print(f"haar n={n} prec={prec}: max-abs {err:.3e}")
    assert np.array_equal(l2p, orc.expected_layout(n, c.gates))


@pytest.mark.parametrize("prec", [0, 1])
def test_gatewise_sweeps_past_the_grid(q, prec):
    """One-qubit sweeps at 24 qubits have 2^23 pairs, twice the sweep grid
    (16384 work-groups of 256 threads): the grid-stride loop runs."""
    c = W.random_mixed(77, 24, 40, max_dense_k=4, max_ctrl=3)
    got, _ = run_gpu(q, c, prec, mode=q.PLAN_GATEWISE)
    check(got, oracle_state(c), prec, "gatewise n=24")


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n", [9, 14, 19])
def test_three_and_four_controls(q, prec, n):
    c = W.random_mixed(500 + n, n, 150, max_dense_k=4, max_ctrl=4, ctrl_prob=0.6)
    assert max(len(g.controls) for g in c.gates) >= 3
    ref = oracle_state(c)
    for opts in ({}, {"mode": q.PLAN_GATEWISE}, {"max_fuse_k": 4}):
        got, _ = run_gpu(q, c, prec, **opts)
        check(got, ref, prec, f"controls n={n} {opts}")


def _tally(c, swap_virtual=True):
    """Per-kind, per-qubit gate counts of a gate list: every target and
    control of a gate counts once for its kind; physical counts use the
    layout at the time of the gate (unconditioned SWAPs relabel it)."""
    from paper_2410_09326_amd import _binding as B
    nk = len(B.KINDS)
    lc = np.zeros((nk, c.n), dtype=np.int64)
    pc = np.zeros((nk, c.n), dtype=np.int64)
    l2p = list(range(c.n))
    for g in c.gates:
        kid = B.KIND_ID[g.kind]
        for qb in tuple(g.qubits) + tuple(g.controls):
            lc[kid, qb] += 1
            pc[kid, l2p[qb]] += 1
        if g.kind == "swap" and not g.controls and swap_virtual:
            a, b = g.qubits
            l2p[a], l2p[b] = l2p[b], l2p[a]
    return lc, pc


@pytest.mark.parametrize("prec", [0, 1])
def test_profiling_run_is_a_valid_simulation(q, prec):
    """A profiling run leaves the normal result (the oracle's state and
    layout), its per-kind, per-qubit counters equal the tally of the gate
    list, and its pass records cover the plan's passes in order."""
    c = W.random_mixed(61, 18, 220, max_dense_k=5, max_ctrl=3)
    ref = oracle_state(c)
    plan = q.Plan(c.n, c.gates, precision=prec)
    sim = q.Simulator(c.n, prec)
    sim.init_basis(c.x0)
    prof = sim.profile(plan)
    check(sim.state(), ref, prec, "profiled run")
    assert np.array_equal(sim.layout(), orc.expected_layout(c.n, c.gates))
    sim.close()
    lc, pc = prof.counts()
    want_l, want_p = _tally(c)
    assert np.array_equal(lc, want_l) and np.array_equal(pc, want_p)
    recs = prof.records()
    assert [r["pass"] for r in recs] == list(range(plan.stats()["n_passes"]))
    assert all(r["seconds"] >= 0 for r in recs) and sum(r["seconds"] for r in recs) > 0
    begins = [r["t_begin"] for r in recs]
    assert begins == sorted(begins)
    total, n = prof.total()
    assert n == c.n and abs(total - sum(r["seconds"] for r in recs)) <= 1e-12 * max(1.0, total)
