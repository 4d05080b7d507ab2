"""Host-memory state tier (the storage simulator's file segment, paper
Sec. II-B, with the virtual-swap placement of Sec. III-D).

CPU: the host-only staging (qops_tier_plan) -- stage counts for circuits
whose answer is known (diagonal-only gates on segment bits need no active
bit; max_active = g needs one stage; a hotspot on the top logical qubits
needs a stage per use unless the placement moves it), and errors.
GPU: tiered runs against the FP64 oracle element by element, with 2..3
segment bits forced on 20-22 qubit states, both precisions, placement on
and off, and <Z> streamed from the segments."""
import numpy as np
import pytest

from oracle import oracle as orc
from workloads import circuits as W

TOL = {0: 2e-5, 1: 1e-12}


def _lib():
    import paper_2410_09326_amd as q
    return q


def hotspot(n, reps=12, seed=3):
    """Non-diagonal gates that keep returning to the two top logical qubits,
    with diagonal and local gates in between."""
    rng = W.rng_for(seed)
    gates = []
    for r in range(reps):
        for q in (n - 1, n - 2):
            gates.append(W.Gate("u3", (q,), params=tuple(float(v) for v in rng.uniform(0, 2 * np.pi, 3))))
        gates.append(W.Gate("cx", (n - 1, int(rng.integers(0, n - 2)))))
        gates.append(W.Gate("rz", (n - 2,), params=(float(rng.uniform(0, 2 * np.pi)),)))
        gates.append(W.Gate("h", (int(rng.integers(0, n - 2)),)))
        gates.append(W.Gate("cz", (n - 1, int(rng.integers(0, n - 2)))))
    return W.Circuit(n, gates, x0=int(rng.integers(2 ** n)), name=f"hotspot{n}")


def test_tier_staging_known_counts():
    q = _lib()
    n = 20
    diag_only = [W.Gate("rz", (19,), params=(0.3,)), W.Gate("cz", (18, 2)), W.Gate("h", (3,)),
                 W.Gate("cp", (19, 18), params=(0.7,))]
    st, _ = q.tier_plan(n, diag_only, 2, 1, remap=0)
    assert st["stages"] == 1 and st["groups"] == 4 and st["exchanges"] == 0
    c = W.random_mixed(5, n, 200, max_dense_k=2, max_ctrl=2)
    st, _ = q.tier_plan(n, c.gates, 3, 3, remap=0)
    assert st["stages"] == 1 and st["groups"] == 1
    h = hotspot(n)
    st0, l0 = q.tier_plan(n, h.gates, 2, 1, remap=0)
    st1, l1 = q.tier_plan(n, h.gates, 2, 1, remap=1)
    # without placement every return to the other top qubit is a new stage;
    # with it the hot qubits never occupy a segment bit
    assert st0["stages"] >= 2 * 12 - 1
    assert st1["stages"] == 1 and st1["exchanges"] == 0
    assert sorted(l1) == list(range(n)) and max(l1[[n - 1, n - 2]]) < n - 2
    # a layout given explicitly is kept as the start; exchanges then move the
    # hot qubits out of the segment bits once
    st2, l2 = q.tier_plan(n, h.gates, 2, 1, remap=1, l2p=list(range(n)))
    assert st2["stages"] <= 2 and st2["exchanges"] >= 1
    assert max(l2[[n - 1, n - 2]]) < n - 2


def test_tier_staging_errors():
    q = _lib()
    rng = W.rng_for(1)
    g = [W.Gate("dense", (18, 19), (), (), W.haar_unitary(rng, 4))]
    with pytest.raises(q.QopsError) as e:
        q.tier_plan(20, g, 2, 1, remap=0)
    assert e.value.status == "UNSUPPORTED"
    with pytest.raises(q.QopsError):
        q.tier_plan(20, g, 0, 1)
    with pytest.raises(q.QopsError):
        q.tier_plan(20, g, 2, 3)
    # with two active bits allowed it stages fine
    st, _ = q.tier_plan(20, g, 2, 2, remap=0)
    assert st["stages"] == 1


@pytest.fixture(scope="module")
def qg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    q = _lib()
    q.lib()
    return q


def _tier_run(q, c, prec, g, amax, remap, **opts):
    print(f"[case] tier {c.name} n={c.n} prec={prec} g={g} amax={amax} remap={remap} {opts}", flush=True)
    t = q.TieredSimulator(c.n, prec, global_bits=g, max_active=amax)
    t.init_basis(c.x0)
    st = t.run(c.gates, remap=remap, **opts)
    psi = t.state()
    z = t.expect_z()
    t.close()
    return psi, z, st


@pytest.mark.gpu
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("remap", [0, 1])
@pytest.mark.parametrize("shape", [(3, 1), (4, 2)])
def test_tier_mixed_against_oracle(qg, prec, remap, shape):
    """Every gate kind with up to 3 controls: controls and diagonal phases on
    inactive segment bits are resolved per device group."""
    c = W.random_mixed(71, 21, 240, max_dense_k=2, max_ctrl=3, ctrl_prob=0.3)
    ref = orc.run_circuit(c)
    psi, z, st = _tier_run(qg, c, prec, shape[0], shape[1], remap)
    err = float(np.max(np.abs(psi.astype(np.complex128) - ref)))
    print(f"tier mixed: {st} max-abs {err:.2e}")
    assert err <= TOL[prec]
    assert np.max(np.abs(z - orc.expect_z(ref))) <= (1e-5 if prec == 0 else 1e-12)
    assert st["h2d_bytes"] == st["d2h_bytes"] > 0


@pytest.mark.gpu
@pytest.mark.parametrize("prec", [0, 1])
def test_tier_qft_layers_two_segment_bits(qg, prec):
    """QFT + U3/CZ layers on 22 qubits with a forced 2-bit host tier and one
    active segment bit per device group: every layer activates both segment
    bits, so the run goes through many stages and exchanges."""
    c = W.qft_then_layers(1, n=22, layers=3)
    ref = orc.run_circuit(c)
    for remap in (0, 1):
        psi, z, st = _tier_run(qg, c, prec, 2, 1, remap)
        err = float(np.max(np.abs(psi.astype(np.complex128) - ref)))
        print(f"tier qft22 remap={remap}: {st} max-abs {err:.2e}")
        assert st["stages"] >= 2
        assert err <= TOL[prec]


@pytest.mark.gpu
@pytest.mark.parametrize("prec", [0, 1])
def test_tier_hotspot_placement(qg, prec):
    """The hotspot circuit: placement keeps the hot qubits local (one
    stage); without it the run takes a stage per return to a top qubit.
    Both give the oracle's state."""
    c = hotspot(20)
    ref = orc.run_circuit(c)
    res = {}
    for remap in (0, 1):
        psi, z, st = _tier_run(qg, c, prec, 2, 1, remap)
        err = float(np.max(np.abs(psi.astype(np.complex128) - ref)))
        print(f"tier hotspot remap={remap}: {st} max-abs {err:.2e}")
        assert err <= TOL[prec]
        res[remap] = st
    assert res[1]["stages"] == 1 and res[0]["stages"] > 10


@pytest.mark.gpu
def test_tier_three_segment_bits_dense_blocks(qg):
    c = W.haar_blocks(9, n=20, nblocks=24, kmin=2, kmax=4)
    ref = orc.run_circuit(c)
    for g, amax in ((3, 2), (3, 3)):
        psi, z, st = _tier_run(qg, c, 0, g, amax, 1, max_fuse_k=3)
        err = float(np.max(np.abs(psi.astype(np.complex128) - ref)))
        print(f"tier haar g={g} amax={amax}: {st} max-abs {err:.2e}")
        assert err <= TOL[0]
