"""qops_expect_z_noalloc (the readout that allocates nothing, its partial
sums in a fixed device array) against qops_expect_z on the same states:
within 1e-12 (FP64 reductions of the same amplitudes), twice in a row with
the second state smaller, in both precisions, for a virtual-swap layout,
and for a state large enough that the fixed array's bounded chunking differs
from the handle's."""
import numpy as np
import pytest

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


def _both(q, c, prec):
    import torch
    sim = q.Simulator(c.n, prec)
    sim.init_basis(c.x0)
    sim.apply(c.gates)
    ref = sim.expect_z()
    out = torch.full((c.n,), float("nan"), dtype=torch.float64, device="cuda:0")
    sim.expect_z_noalloc(out)
    sim.synchronize()
    got = out.cpu().numpy()
    l2p = sim.layout()
    sim.close()
    return got, ref, l2p


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_matches_expect_z_twice(q, prec):
    # a QFT ends in a swap network: the layout is a reversal, so the
    # logical-order mapping of the fixed-array path is exercised
    first = W.qft_then_layers(4, n=20, layers=3)
    second = W.random_mixed(9, 14, 90, max_dense_k=4)
    for i, c in enumerate((first, second)):
        got, ref, l2p = _both(q, c, prec)
        print(f"n={c.n} prec={prec} max |diff| {np.max(np.abs(got - ref)):.2e}")
        assert np.all(np.isfinite(got))
        assert np.max(np.abs(got - ref)) <= 1e-12
        if i == 0:
            assert not np.array_equal(l2p, np.arange(c.n))


def test_noalloc_bounded_chunks_at_29_qubits(q):
    """At 29 qubits the fixed array holds 2^11 records of 2^18-amplitude
    chunks (the handle's path uses 2^13 chunks of 2^16)."""
    import torch
    n = 29
    sim = q.Simulator(n, q.C64)
    sim.init_basis(0)
    c = W.haar_blocks(3, n=n, nblocks=6)
    sim.apply(c.gates)
    sim.swap(0, 27)
    ref = sim.expect_z()
    out = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    sim.expect_z_noalloc(out)
    sim.synchronize()
    got = out.cpu().numpy()
    print(f"n={n} max |diff| {np.max(np.abs(got - ref)):.2e}")
    assert np.max(np.abs(got - ref)) <= 1e-12
    # a second, smaller call reuses the array
    small = W.random_mixed(5, 12, 40, max_dense_k=3)
    g2, r2, _ = _both(q, small, q.C64)
    assert np.max(np.abs(g2 - r2)) <= 1e-12
    sim.close()


def test_noalloc_rejects_bad_arguments(q):
    sim = q.Simulator(10, q.C64)
    with pytest.raises(q.QopsError):
        q._binding.check(q.lib().qops_expect_z_noalloc(sim.handle, None))
    sim.close()
