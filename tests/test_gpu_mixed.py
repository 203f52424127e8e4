"""Mixed precision (DQMC_MIXED): wraps in complex64, flushes with FP32 MFMA,
ratios and the QR stabilisation in FP64.  The paper fixes no accuracy for
this mode, so the bounds are derived from the arithmetic:

  flush    |G - X Y - out| <= (k + 2) u (|X| |Y|) + 4 u_64 |G| elementwise
           (FP32 inner products of length k with rounded operands,
           u = 2^-24; the FP64 subtraction adds a few u_64);
  wrap     ||out - ref||_F <= 64 log2(N) u ||ref||_F per wrap (two 2-D
           transforms per side, each a product of log2 N_c butterflies);
  replay   fields follow the fed bits exactly, and every G rebuilt by the
           FP64 stabilisation matches the FP64 oracle to 1e-10 again.
           Between rebuilds G carries the FP32 error that the wraps amplify
           (each wrap multiplies it by up to cond(B_l)); its size at the
           rebuild is the reported drift delta = max |G_wrap - G_scratch|.
           A ratio depends on G through r = 1 + D (1 - G_ii), |D| <= e^{2 lam} - 1,
           and R = e^{2 lam x} |r|^2, so |dR| <= e^{2 lam} (2 |r| + |dr|) |dr| with
           |dr| <= (e^{2 lam} - 1) |dG_ii|; the test takes |dG_ii| <= 2 delta
           (the error inside a segment stays below twice its end value).
"""
import numpy as np
import pytest

import workloads
from oracle.dqmc import BitSource, Chain, Model

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
U64 = 2.0 ** -53


def _sim(descs):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_14668_amd import Simulation
    return Simulation(descs)


def _model(d):
    return Model(d["L"], d["U"], d["beta"], d["dtau"], t=d["t"], theta1=d["theta1"], theta2=d["theta2"],
                 n_stab=d["n_stab"])


def _rand(shape, cx, seed):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(shape)
    if cx:
        a = a + 1j * rng.standard_normal(shape)
    return a


@pytest.mark.parametrize("L,th", [(3, (0, 0)), (6, (0, 0)), (4, (0.7, 2.1)), (5, (0.3, 0.0)), (12, (1.0, 0.5))])
def test_mixed_wrap_error_bound(L, th):
    d = workloads.desc(L, 3.7, 1.0, theta=th, n_stab=5, precision=1)
    sim = _sim([d])
    m = _model(d)
    N, M, cx = sim.shapes[0]
    f = sim.fields(0)
    for direction, sl in ((0, 1), (1, 3)):
        G = _rand((N, N), cx, L + sl)
        sim.set_green(0, G)
        sim.wrap(direction, sl)
        out = sim.green(0)
        B, Bi = m.B(0, f[sl - 1]), m.Binv(0, f[sl - 1])
        ref = B @ G @ Bi if direction == 0 else Bi @ G @ B
        err = np.linalg.norm(out - ref) / np.linalg.norm(ref)
        assert err < 64 * np.log2(N) * U32, err
        # single precision really is in use: the error exceeds FP64 rounding
        assert err > 1e3 * U64


@pytest.mark.parametrize("L,th,k", [(3, (0, 0), 8), (12, (0, 0), 64), (4, (0.5, 1.0), 16), (9, (0.2, 0.9), 64)])
def test_mixed_flush_error_bound(L, th, k):
    d = workloads.desc(L, 3.7, 1.0, theta=th, n_stab=5, k=k, precision=1)
    sim = _sim([d])
    N, _, cx = sim.shapes[0]
    k = min(k, N)
    G = _rand((N, N), cx, 1)
    X = _rand((N, k), cx, 2)
    Y = _rand((k, N), cx, 3)
    sim.set_green(0, G)
    sim.flush_test(0, X, Y)
    ref = G - X @ Y
    bound = (k + 2) * U32 * (np.abs(X) @ np.abs(Y)) * (2 if cx else 1) + 4 * U64 * np.abs(G)
    assert np.all(np.abs(sim.green(0) - ref) <= bound)


@pytest.mark.parametrize("L,th,beta,k", [(3, (0, 0), 3.0, 8), (4, (0.7, 2.2), 2.0, 16)])
def test_mixed_replay_against_fp64_oracle(L, th, beta, k):
    import torch
    d = workloads.desc(L, 3.8, beta, theta=th, k=k, n_stab=10, precision=1)
    sim = _sim([d])
    m = _model(d)
    N, M, cx = sim.shapes[0]
    f0 = workloads.random_fields(13, M, N)
    sim.set_fields(0, f0)
    bits = workloads.accept_bits(14, 2 * M * N, 0.4)
    tb = torch.from_numpy(bits).reshape(1, -1).cuda()
    ratios = torch.zeros((1, bits.size), dtype=torch.float64, device="cuda")
    sim.replay(tb, ratios, n_sweeps=1, measure=False)
    ch = Chain(m, f0)
    ch.sweep(BitSource(bits), measure=False)
    assert np.array_equal(sim.fields(0), ch.fields)
    # the sweep ends on a stabilisation point: G comes from the FP64 QR chain
    assert np.abs(sim.green(0) - ch.G[0]).max() < 1e-10
    st = sim.stats(0)
    assert st["accepted"] == ch.accepted
    delta = st["drift_max"]
    # the wrap/flush drift is visible and of single-precision size
    assert 1e-12 < delta < 1e-2
    r = ratios.cpu().numpy().ravel()
    ref = np.array(ch.ratios)
    lam = np.arccosh(np.exp(d["dtau"] * d["U"] / 2))
    e2 = np.exp(2 * lam)
    dr = (e2 - 1) * 2 * delta
    rmax = np.sqrt(e2 * ref.max())
    assert np.abs(r - ref).max() <= e2 * (2 * rmax + dr) * dr
    print("mixed replay L=%d: drift %.3g, max |dR| %.3g" % (L, delta, np.abs(r - ref).max()))


def test_mixed_time_displaced_pass():
    """A time-displaced pass in a mixed-precision handle: its wraps run in
    complex64, its recomputations in FP64.  After one slice each function
    carries one complex64 side pass (G(tau,tau): two) and obeys the wrap
    bound above; right after a recomputation (l = n_stab, M/2) all three
    match the FP64 oracle to 1e-10 of their largest entry."""
    from oracle import tau
    d = workloads.desc(4, 3.8, 2.0, theta=(0.7, 2.1), n_stab=5, precision=1, seed=3)
    sim = _sim([d])
    m = _model(d)
    N, M, _ = sim.shapes[0]
    f = sim.fields(0)
    ref = tau.tau_greens(m, f, 0, M // 2)
    sim.measure_tau(1)
    for which, sides in ((0, 2), (1, 1), (2, 1)):
        got, r = sim.green_tau(0, which), ref[1][which]
        bound = sides * 64 * np.log2(N) * U32 * np.linalg.norm(r)
        assert np.linalg.norm(got - r) <= bound, (which, np.linalg.norm(got - r), bound)
    for lstop in (5, M // 2):
        sim.measure_tau(lstop)
        for which in range(3):
            r = ref[lstop][which]
            err = np.abs(sim.green_tau(0, which) - r).max()
            assert err < 1e-10 * max(1.0, np.abs(r).max()), (lstop, which, err)
