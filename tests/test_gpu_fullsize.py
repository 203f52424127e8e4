"""The L=18 twisted batch at its full size (64 complex128 L=18 chains on a 4x4
twist grid, four per twist, plus 16 L=12 chains: N = 648 and 288, M = 180 and
120) in the launch configuration that the benchmark times: the library's
default instance groups for this batch (three, on three streams),
stabilisation blocks replayed as HIP graphs, the flush rank and kernel and the
FFT tiles picked by the autotuners.

Sampled outputs are checked against the oracle where it can compute them one
by one at this size (the scratch G of an L=18 and an L=12 instance from
seeded fields, one wrap of a seeded G on both), and a sweep is checked
through properties that hold at any size: the exact proposal count, the drift
between the wrapped-and-updated G and the scratch recomputation at every
stabilisation point, and the sign and range of the estimators.

Tolerances.  Scratch G: both sides run a QR-stabilised product of M/n_s = 18
blocks in FP64, each block backward stable to a small multiple of N eps, and
the scale-separated inversion keeps the result's error at that level relative
to max|G| = O(1): 1e-9 absolute leaves a factor 100 over N eps * 18 blocks.
Wrap: one FFT pass per side, 1e-13 relative to the largest entry as at the
small sizes.  Drift: the wrapped G carries the rounding of ten wraps and
about 0.7 N accepted rank-one terms per slice (each O(1e-16) relative),
amplified through the slice propagators (cond(B_l) of a few per slice); on
this batch intact sweeps measure max |G_wrap - G_scratch| between 1e-7 and
3e-6 depending on the configurations, so the check uses the library's own
drift tolerance (1e-4, which also sets numeric_err); one wrong rank-one term
or one wrong wrap gives O(1e-2) or more.
"""
import numpy as np
import pytest

import workloads
from oracle.dqmc import Model

pytestmark = pytest.mark.gpu

L18, L12 = 5, 70          # a twisted L=18 chain and a twisted L=12 chain of the batch


def _model(d):
    return Model(d["L"], d["U"], d["beta"], d["dtau"], t=d["t"], theta1=d["theta1"], theta2=d["theta2"],
                 n_stab=d["n_stab"])


@pytest.fixture(scope="module")
def batch():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_14668_amd import Simulation
    descs = workloads.twist_L18()
    assert len(descs) == 80 and descs[L18]["L"] == 18 and descs[L12]["L"] == 12
    sim = Simulation(descs)
    sim.set_graphs(True)
    best, _ = sim.autotune([24, 64], 2 * descs[0]["n_stab"])
    tiles, _ = sim.autotune_fft(5)
    print("autotuned fft tiles %s" % tiles, flush=True)
    print("autotuned flush rank %d, kernel %s" % (best[0], ("direct", "tiled", "queue")[best[1]]), flush=True)
    yield sim, descs
    sim.close()


def test_fullsize_scratch_green_matches_oracle(batch):
    sim, descs = batch
    for inst, seed in ((L18, 301), (L12, 302)):
        d = descs[inst]
        N, M, cx = sim.shapes[inst]
        assert cx
        f = workloads.random_fields(seed, M, N)
        sim.set_fields(inst, f)
        ref = _model(d).green_scratch(f, 0, 0)
        err = np.abs(sim.green(inst) - ref).max()
        print("instance %d (L=%d): max |G - G_oracle| = %.2e" % (inst, d["L"], err), flush=True)
        assert err < 1e-9


def test_fullsize_sweep_properties(batch):
    sim, descs = batch
    n = len(descs)
    sim.reset_obs()
    st0 = [sim.stats(i) for i in range(n)]
    sim.sweep(1, measure=True)
    st1 = [sim.stats(i) for i in range(n)]
    drift = max(s["drift_max"] for s in st1)
    acc = sum(b["accepted"] - a["accepted"] for a, b in zip(st0, st1)) / \
        sum(b["proposals"] - a["proposals"] for a, b in zip(st0, st1))
    print("drift_max %.2e, acceptance %.3f" % (drift, acc), flush=True)
    Mmax = max(s[1] for s in sim.shapes)
    for i in range(n):
        N, M, _ = sim.shapes[i]
        # one call runs 2 Mmax slice steps; every step visits one slice of
        # every instance (the L=12 chains run one and a half sweeps)
        assert st1[i]["proposals"] - st0[i]["proposals"] == 2 * Mmax * N
        if M == Mmax:
            assert st1[i]["sweeps"] - st0[i]["sweeps"] == 1
        assert st1[i]["numeric_err"] == 0
        assert st1[i]["drift_max"] < 1e-4
        ob = sim.measure(i)
        assert ob["n_meas"] > 0
        assert 0.0 < ob["D"] < 0.3
        assert ob["ekin"] < 0.0
    assert 0.05 < acc < 0.99


def test_fullsize_wrap_matches_dense_propagation(batch):
    sim, descs = batch
    rng = np.random.default_rng(303)
    cases = []
    # fields first: setting an instance's fields recomputes G of every instance
    for inst in (L18, L12):
        N, M, _ = sim.shapes[inst]
        f = workloads.random_fields(310 + inst, M, N)
        sim.set_fields(inst, f)
        cases.append((inst, f))
    for i, (inst, f) in enumerate(cases):
        N = sim.shapes[inst][0]
        G = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
        sim.set_green(inst, G)
        cases[i] = (inst, f, G)
    sl = 7
    sim.wrap(0, sl)
    for inst, f, G in cases:
        m = _model(descs[inst])
        ref = m.B(0, f[sl - 1]) @ G @ m.Binv(0, f[sl - 1])
        out = sim.green(inst)
        assert np.abs(out - ref).max() / np.abs(ref).max() < 1e-13
