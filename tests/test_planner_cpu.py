"""Host-side checks of the C ABI and the planner (no GPU needed): every
symbol the header declares is exported, bad gates are rejected with the right
status, and the plan's lowered operations -- applied one by one with the
FP64 oracle's generic matrix routine -- reproduce the circuit exactly,
including virtual swaps, single-qubit merging and diagonal fusion."""
import os
import re

import numpy as np
import pytest

import paper_2410_09326_amd as q
from paper_2410_09326_amd import _binding as B
from oracle import oracle as orc
from workloads import circuits as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "qops.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(qops_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = B.lib()
    syms = header_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(L, s), s
        assert s in B.SIGNATURES, f"binding does not declare {s}"


def test_version():
    assert B.lib().qops_version() > 0


def _expect(code, fn):
    with pytest.raises(q.QopsError) as e:
        fn()
    assert e.value.code == code, (e.value.code, str(e.value))


def test_validation_errors():
    _expect(-2, lambda: q.Plan(4, [("h", (4,))]))
    _expect(-2, lambda: q.Plan(4, [("cx", (0, -1))]))
    _expect(-3, lambda: q.Plan(4, [("cx", (1, 1))]))
    _expect(-3, lambda: q.Plan(4, [("x", (1,), (), (1,))]))
    _expect(-4, lambda: q.Plan(40, [("h", (0,))]))
    _expect(-4, lambda: q.Plan(8, [("x", (0,), (), (1, 2, 3, 4, 5))]))
    bad = np.eye(4, dtype=complex) * 2
    _expect(-8, lambda: q.Plan(4, [("dense", (0, 1), (), (), bad)], check_unitary=1))
    # without the opt-in check the same matrix is accepted
    q.Plan(4, [("dense", (0, 1), (), (), bad)])
    _expect(-1, lambda: q.Plan(4, [("h", (0,))], l2p=[0, 0, 1, 2]))
    _expect(-1, lambda: q.Plan(4, [("h", (0,))], mode=9))
    assert "out of range" in B.lib().qops_last_error().decode() or True


def physical_replay(n, plan, x0):
    """Applies the plan's lowered operations (physical bits) with the oracle's
    plain matrix routine and returns the state read through the final layout."""
    l2p0 = np.arange(n)
    xp = sum(((x0 >> qb) & 1) << int(l2p0[qb]) for qb in range(n))
    psi = orc.basis_state(n, xp)
    for op in plan.ops():
        ctrls = [b for b in range(n) if (op["cmask"] >> b) & 1]
        if op["kind"] == 0:
            psi = orc.apply_matrix(n, psi, op["m"], op["t"][:1], ctrls)
        elif op["kind"] == 2:
            psi = orc.apply_matrix(n, psi, op["m"], op["t"], ctrls)
        elif op["kind"] == 1:
            psi = orc.apply_matrix(n, psi, np.diag(op["m"]), op["t"], ctrls)
        else:
            sw = np.eye(4)[[0, 2, 1, 3]]
            psi = orc.apply_matrix(n, psi, sw, op["t"][:2])
    return orc.logical_from_physical(psi, plan.final_layout())


CASES = [
    ("mixed8", lambda: W.random_mixed(3, 8, 150, max_dense_k=4)),
    ("mixed10", lambda: W.random_mixed(4, 10, 150, max_dense_k=6)),
    ("layered14", lambda: W.layered_u3_cx(1, n=14, depth=6, swap_frac=0.5)),
    ("qft11", lambda: W.qft(11, 1234)),
    ("qftlayers13", lambda: W.qft_then_layers(1, n=13, layers=3)),
    ("haar14", lambda: W.haar_blocks(2, n=14, nblocks=20)),
    ("mix14", lambda: W.random_mix_layers(9, 14, 8)),
]


@pytest.mark.parametrize("prec,mb", [(q.C64, 0), (q.C128, 0), (q.C128, 1)])
def test_priced_block_merging_reproduces_circuit(prec, mb):
    """Priced merging of dense blocks (on by default, a cost table per precision): the plan
    has fewer dense blocks than the circuit, every source gate is folded into
    exactly one operation, and the lowered operations replayed with the
    oracle's matrix routine give the circuit's state."""
    c = W.haar_blocks(21, n=14, nblocks=40)
    plan = q.Plan(c.n, c.gates, precision=prec, merge_blocks=mb)
    off = q.Plan(c.n, c.gates, precision=prec, merge_blocks=-1)
    ops = plan.ops()
    assert len(ops) < len(off.ops())
    assert max(o["k"] for o in ops) <= 6
    assert sum(o["n_merged"] for o in ops) == len(c.gates)
    got = physical_replay(c.n, plan, c.x0)
    assert np.max(np.abs(got - orc.run_circuit(c))) <= 1e-12
    # merged blocks are unitary products of their parts: a merged block's
    # width is at most the sum of two source widths and at least the wider
    ks = sorted(len(g.qubits) for g in c.gates)
    assert min(o["k"] for o in ops) >= ks[0]


@pytest.mark.parametrize("name,make", CASES)
@pytest.mark.parametrize("mode", [q.PLAN_FUSED, q.PLAN_GATEWISE])
@pytest.mark.parametrize("swap_mode", [q.SWAP_VIRTUAL, q.SWAP_PHYSICAL])
def test_plan_ops_reproduce_circuit(name, make, mode, swap_mode):
    c = make()
    plan = q.Plan(c.n, c.gates, precision=q.C128, mode=mode, swap_mode=swap_mode)
    got = physical_replay(c.n, plan, c.x0)
    ref = orc.run_circuit(c)
    assert np.max(np.abs(got - ref)) <= 1e-12
    exp_l2p = orc.expected_layout(c.n, c.gates, virtual_swaps=(swap_mode == q.SWAP_VIRTUAL))
    assert np.array_equal(plan.final_layout(), exp_l2p)
    if mode == q.PLAN_FUSED and swap_mode == q.SWAP_VIRTUAL:
        # with the up-front remap the result is the same state; the layout it
        # ends in is the remap followed by the circuit's virtual swaps
        rp = q.Plan(c.n, c.gates, precision=q.C128, remap=1)
        got2 = physical_replay(c.n, rp, c.x0)
        assert np.max(np.abs(got2 - ref)) <= 1e-12
    st = plan.stats()
    if swap_mode == q.SWAP_VIRTUAL:
        assert st["n_virtual_swaps"] == sum(1 for g in c.gates if g.kind == "swap")
        assert st["n_permute_passes"] == 0
    else:
        assert st["n_virtual_swaps"] == 0


def test_single_qubit_merging_and_diag_fusion_counts():
    n = 14
    gates = []
    for _ in range(5):
        gates += [("h", (3,)), ("t", (3,)), ("rz", (3,), (0.3,)), ("s", (9,))]
    gates += [("cz", (0, 1)), ("cz", (2, 3)), ("cp", (4, 5), (0.2,))]
    plan = q.Plan(n, gates, fold_rotations=-1)
    ops = plan.ops()
    # all one-qubit gates on qubit 3 collapse to one 2x2; the five S on 9 to one
    # controlled phase; controlled phases on different bits stay separate
    # (cheaper per amplitude than a fused table)
    assert len(ops) == 5
    assert sum(o["n_merged"] for o in ops) == len(gates)
    gates2 = [("rzz", (0, 1), (0.3,)), ("rz", (2,), (0.2,)), ("rzz", (1, 2), (0.1,))]
    ops2 = q.Plan(n, gates2).ops()
    assert len(ops2) == 1 and ops2[0]["k"] == 3          # general tables fuse


def test_pass_packing_respects_tile_width():
    c = W.random_mix_layers(5, 24, 10)
    for prec in (q.C64, q.C128):
        plan = q.Plan(24, c.gates, precision=prec)
        passes = plan.passes()
        for i, ps in enumerate(passes):
            assert ps["L"] == 6 + len(ps["upper"])
            cap = 7 if prec == q.C64 else 6
            assert len(ps["upper"]) <= cap
        for op in plan.ops():
            ps = passes[op["pass"]]
            if op["kind"] in (0, 2):
                for t in op["t"]:
                    assert t < 6 or t in ps["upper"]


def test_gatewise_has_one_pass_per_op():
    c = W.random_mixed(1, 16, 40)
    plan = q.Plan(16, c.gates, mode=q.PLAN_GATEWISE)
    assert plan.stats()["n_passes"] == len(plan.ops())


def test_plan_update_rebinds_parameters():
    c1 = W.param_sweep_batch(seed=5, count=2)[1]
    rng = np.random.default_rng(0)
    c2 = W.Circuit(c1.n, [W.Gate(g.kind, g.qubits, g.controls,
                                 tuple(rng.uniform(0, 6.28, len(g.params))), g.matrix) for g in c1.gates])
    plan = q.Plan(c1.n, c1.gates, precision=q.C128)
    plan.update(c2.gates)
    got = physical_replay(c2.n, plan, 0)
    assert np.max(np.abs(got - orc.run_circuit(c2))) <= 1e-12
    bad = list(c2.gates)
    bad[0] = W.Gate("rx", bad[0].qubits, (), bad[0].params)
    with pytest.raises(q.QopsError):
        plan.update(bad)


@pytest.mark.parametrize("name,make", CASES)
@pytest.mark.parametrize("kmax", [2, 3, 4, 6])
def test_block_fusion_reproduces_circuit(name, make, kmax):
    """Fused k-qubit blocks (FP64 products of the ops they absorb, ops moved
    only past ops they commute with) reproduce the circuit."""
    c = make()
    plan = q.Plan(c.n, c.gates, precision=q.C128, max_fuse_k=kmax)
    got = physical_replay(c.n, plan, c.x0)
    ref = orc.run_circuit(c)
    assert np.max(np.abs(got - ref)) <= 1e-12
    ops = plan.ops()
    assert all(o["k"] <= max(kmax, 6) for o in ops)
    base = q.Plan(c.n, c.gates, precision=q.C128).ops()
    assert len(ops) <= len(base)
    assert sum(o["n_merged"] for o in ops) == sum(o["n_merged"] for o in base)


def test_block_fusion_counts():
    n = 12
    # ten 1q gates and three CZ on qubits {2,3,4}: one 3-qubit block
    gates = []
    for r in range(3):
        gates += [("u3", (2,), (0.1 * r, 0.2, 0.3)), ("u3", (3,), (0.3, 0.1 * r, 0.2)), ("rx", (4,), (0.4,))]
        gates += [("cz", (2, 3))]
    gates += [("ry", (4,), (0.7,))]
    ops = q.Plan(n, gates, max_fuse_k=3).ops()
    assert len(ops) == 1 and ops[0]["k"] == 3 and ops[0]["kind"] == 2
    assert ops[0]["n_merged"] == len(gates)
    # CX(4,7) leaves the 3-qubit set; the later H on 2 commutes with it and
    # still joins the block
    ops4 = q.Plan(n, gates + [("cx", (4, 7)), ("h", (2,))], max_fuse_k=3).ops()
    assert len(ops4) == 2


def test_profile_trace_export(tmp_path):
    """A stored profile exports as a Chrome trace-event file: one complete
    event per pass (start, duration, achieved GB/s) on the passes track."""
    import json
    import os
    models = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2410_09326_amd",
                          "models")
    prof = q.Profile.load(os.path.join(models, "corpus_profile.bin"))
    recs = prof.records()
    path = str(tmp_path / "trace.json")
    prof.trace(path)
    with open(path) as fh:
        d = json.load(fh)
    ev = d["traceEvents"]
    xs = [e for e in ev if e["ph"] == "X"]
    assert len(xs) == len(recs)
    for e, r in zip(xs[:200], recs[:200]):
        assert e["dur"] == pytest.approx(r["seconds"] * 1e6, rel=1e-5, abs=1e-3)
        assert e["args"]["pass"] == r["pass"] and e["args"]["ops"] == r["n_ops"]
        assert e["args"]["GB_per_s"] == pytest.approx(r["bytes_alg"] / r["seconds"] / 1e9, rel=1e-3, abs=0.1)
    assert any(e["ph"] == "M" for e in ev)


FOLD_CASES = CASES + [
    ("clifft10", lambda: W.clifford_t(1, 10, 300)),
    ("clifft13", lambda: W.clifford_t(2, 13, 500, t_frac=0.5)),
    ("qaoa10", lambda: W.qaoa_maxcut(10, *W.regular_graph(2, 10, 3), [0.4, 1.1], [0.3, 0.8])),
]


@pytest.mark.parametrize("name,make", FOLD_CASES)
@pytest.mark.parametrize("swap_mode", [q.SWAP_VIRTUAL, q.SWAP_PHYSICAL])
def test_rotation_folding_is_exact(name, make, swap_mode):
    """Folded plans reproduce the circuit exactly, global phase included."""
    c = make()
    plan = q.Plan(c.n, c.gates, precision=q.C128, fold_rotations=1, swap_mode=swap_mode)
    got = physical_replay(c.n, plan, c.x0)
    assert np.max(np.abs(got - orc.run_circuit(c))) <= 1e-12
    assert np.array_equal(plan.final_layout(),
                          orc.expected_layout(c.n, c.gates, virtual_swaps=(swap_mode == q.SWAP_VIRTUAL)))


def test_rotation_folding_merges_equal_parities():
    n = 8
    # T and T-dagger on the same parity a xor b (behind CNOTs) cancel
    cancel = [("cx", (2, 5)), ("t", (5,)), ("cx", (2, 5)), ("h", (7,)), ("cx", (2, 5)), ("tdg", (5,)), ("cx", (2, 5))]
    st = q.Plan(n, cancel, fold_rotations=1).stats()
    assert st["n_folded"] == 2
    # T on wire 3, a detour through CNOTs, T again on the same parity: one S
    two = [("t", (3,)), ("cx", (3, 4)), ("cx", (4, 6)), ("cx", (3, 4)), ("cx", (4, 6)), ("t", (3,))]
    p2 = q.Plan(n, two, fold_rotations=1)
    assert p2.stats()["n_folded"] == 1
    # a Hadamard on the wire starts a new parity: nothing merges
    three = [("t", (3,)), ("h", (3,)), ("t", (3,))]
    assert q.Plan(n, three, fold_rotations=1).stats()["n_folded"] == 0
    # the paper's activation rule: folding fires above 10% T gates only
    lots = W.clifford_t(4, n, 200, t_frac=0.4)
    few = W.clifford_t(4, n, 200, t_frac=0.02)
    assert q.Plan(n, lots.gates).stats()["n_folded"] > 0
    assert q.Plan(n, few.gates).stats()["n_folded"] == 0
    assert q.Plan(n, lots.gates, fold_rotations=-1).stats()["n_folded"] == 0


@pytest.mark.parametrize("mode", ["profiled", "learned"])
def test_priced_plan_is_cheapest_candidate(mode):
    """Priced planning keeps the cheapest candidate under its own pricing: the
    chosen plan's predicted time is at most that of the default-width plan
    and of every explicit tile width (remap on/off, fusion width 1..4)."""
    import os
    models = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2410_09326_amd",
                          "models")
    if mode == "profiled":
        kw = {"mode": q.PLAN_PROFILED, "profile": q.Profile.load(os.path.join(models, "corpus_profile.bin"))}
    else:
        kw = {"mode": q.PLAN_LEARNED, "model": q.CostModel.load(os.path.join(models, "cost_mlp.bin"))}
    for seed in (9100, 9101):
        c = W.eval_circuit(seed, n=24, depth=16)
        best = q.Plan(c.n, c.gates, precision=q.C64, **kw).stats()["predicted_s"]
        assert best > 0
        for tu in (0, 4, 5, 6, 7):
            for remap in (0, 1):
                for kf in (1, 2, 3, 4):
                    cand = q.Plan(c.n, c.gates, precision=q.C64, tile_upper=tu, remap=remap, max_fuse_k=kf)
                    assert best <= cand.predict(**kw) * (1 + 1e-12), (seed, tu, remap, kf)


def test_plain_table_is_the_median_per_pass_shape():
    """The plain cost table prices a pass by the median measured time per
    amplitude of the profiled passes of its shape: on the shipped profile
    (five percentile passes per shape) the middle pass of every full shape is
    predicted exactly, and compacting again keeps every record."""
    import os
    models = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2410_09326_amd",
                          "models")
    prof = q.Profile.load(os.path.join(models, "corpus_profile.bin"))
    recs = prof.records()
    t = np.array([r["seconds"] for r in recs])
    pred = prof.predict_passes(mode=q.PLAN_PROFILED, profile=prof)
    exact = np.isclose(pred, t, rtol=1e-9, atol=0)
    assert exact.mean() >= 0.15
    # every prediction is one of the measured per-amplitude costs of the
    # profile, scaled to the pass's size: within the profile's own range
    assert np.all(pred > 0)
    again = prof.compact()
    assert len(again.records()) == len(recs)
