"""The allocation-free logits entry point (static device scratch) against
dqmc_net_logits (caller workspace): the same kernels on the same inputs, so
the logits must be identical; two calls in a row, the second on a smaller
input, so that the shared scratch keeps the larger first call's contents."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _sim():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_14668_amd import Simulation
    return Simulation([workloads.desc(3, 3.7, 1.0, n_stab=5)])


def test_noalloc_logits_equal_workspace_logits():
    sim = _sim()
    sim.net_set_weights(workloads.net_weights(21, gain=1.5))
    cases = [(6, 40, 3), (3, 6, 2)]        # (L, M, n): the second call is smaller
    for L, M, n in cases:
        xs = np.stack([workloads.random_fields(600 + 10 * L + b, M, 2 * L * L) for b in range(n)])
        ref = sim.net_logits(xs, L)
        out = sim.net_logits_noalloc(xs, L)
        assert out.shape == ref.shape
        assert np.array_equal(out, ref), (L, M, n, np.abs(out - ref).max())


def test_noalloc_logits_reject_too_large_inputs():
    from paper_2609_14668_amd import DqmcError
    sim = _sim()
    L, M, n = 18, 180, 2               # about 27 MB of scratch, above the 16 MiB array
    xs = np.ones((n, M, 2 * L * L), dtype=np.int8)
    with pytest.raises(DqmcError) as e:
        sim.net_logits_noalloc(xs, L)
    assert e.value.status == -6
