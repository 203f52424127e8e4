"""The time-displaced pass (Sec. II C, eqs. DouOccDerive, fidelitysusp) on
the GPU against the oracle on the same configuration: G(tau,tau), G(tau,0),
G(0,tau) at chosen slices (before and after the recomputations), the series
<A(tau_l) A(0)> and <A> of one pass, both HS channels, PBC and twisted, an
uneven batch, a pass after sweeps (the stack of the last downward pass), and
sampled checks at the full L = 18 shape.  A pass must leave the chain
untouched: a sweep after it is bit-identical to one without it.

Tolerances: the functions 1e-10 relative to their largest entry (at least 1;
the charge channel's functions have entries far above 1), since wraps and
recomputations agree with the oracle's block inverse to rounding amplified by
the conditioning of n_stab slices, as for the equal-time G; the series 1e-10
relative.
"""
import numpy as np
import pytest

import workloads
from oracle import tau
from oracle.dqmc import Model

pytestmark = pytest.mark.gpu


def _sim(descs):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_14668_amd import Simulation
    return Simulation(descs)


def _model(d):
    return Model(d["L"], d["U"], d["beta"], d["dtau"], t=d["t"], theta1=d["theta1"], theta2=d["theta2"],
                 n_stab=d["n_stab"], channel="charge" if d.get("channel", 0) else "spin")


CASES = [  # L, twist, beta, n_stab, channel
    (3, (0.0, 0.0), 2.0, 5, 0),
    (4, (0.7, 2.1), 2.0, 5, 0),
    (4, (0.5, -1.2), 2.0, 5, 1),
    (6, (0.0, 0.0), 2.0, 10, 0),
]


@pytest.mark.parametrize("L,th,beta,ns,ch", CASES)
def test_tau_greens_match_oracle(L, th, beta, ns, ch):
    d = workloads.desc(L, 3.8, beta, theta=th, n_stab=ns, channel=ch, seed=7)
    sim = _sim([d])
    m = _model(d)
    f = sim.fields(0)
    M = m.M
    ref = tau.tau_greens(m, f, 0, M // 2)
    for lstop in sorted(x for x in {1, ns - 1, ns, ns + 1, M // 2} if x <= M // 2):
        print("case", L, th, ch, "slice", lstop, flush=True)
        sim.measure_tau(lstop)
        for which in range(3):
            got = sim.green_tau(0, which)
            scale = max(1.0, np.abs(ref[lstop][which]).max())
            err = np.abs(got - ref[lstop][which]).max()
            assert err < 1e-10 * scale, (lstop, which, err, scale)
    st = sim.stats(0)
    assert st["drift_last"] < 1e-9


@pytest.mark.parametrize("L,th,beta,ns,ch", CASES)
def test_tau_series_matches_oracle(L, th, beta, ns, ch):
    d = workloads.desc(L, 3.8, beta, theta=th, n_stab=ns, channel=ch, seed=3)
    sim = _sim([d])
    m = _model(d)
    f = sim.fields(0)
    sim.measure_tau()
    aa, at, n = sim.get_tau(0)
    assert n == 1
    AA, At = tau.tau_correlator(m, f, m.M // 2)
    np.testing.assert_allclose(aa, AA.real, rtol=1e-10, atol=0)
    np.testing.assert_allclose(at, At.real, rtol=1e-10, atol=0)
    lc = m.M // 2
    rows = sim.tau_rows(0)
    assert rows.shape == (1, 2 * lc + 2)
    np.testing.assert_array_equal(rows[0, :lc + 1], aa)
    np.testing.assert_array_equal(rows[0, lc + 1:], at)
    # a second pass on the same configuration doubles nothing but the count
    sim.measure_tau()
    aa2, at2, n2 = sim.get_tau(0)
    assert n2 == 2
    np.testing.assert_allclose(aa2, aa, rtol=1e-13, atol=0)
    np.testing.assert_allclose(at2, at, rtol=1e-13, atol=0)


def test_uneven_batch_tau():
    """Instances of different M end their passes at their own M/2; a shorter
    l_max cuts every instance."""
    ds = [workloads.desc(4, 3.8, 2.0, theta=(0.7, 2.1), n_stab=5, seed=5),
          workloads.desc(3, 3.7, 3.0, n_stab=5, seed=6)]
    sim = _sim(ds)
    sim.measure_tau()
    for i, d in enumerate(ds):
        m = _model(d)
        AA, At = tau.tau_correlator(m, sim.fields(i), m.M // 2)
        aa, at, n = sim.get_tau(i)
        assert n == 1
        np.testing.assert_allclose(aa, AA.real, rtol=1e-10, atol=0)
        np.testing.assert_allclose(at, At.real, rtol=1e-10, atol=0)
    sim.reset_obs()
    sim.measure_tau(7)
    for i, d in enumerate(ds):
        m = _model(d)
        AA, _ = tau.tau_correlator(m, sim.fields(i), 7)
        aa, _, n = sim.get_tau(i)
        assert n == 1
        np.testing.assert_allclose(aa[:8], AA.real, rtol=1e-10, atol=0)
        assert np.all(aa[8:] == 0.0)


@pytest.mark.parametrize("ch", [0, 1])
def test_tau_after_sweeps(ch):
    """After whole sweeps the partner chains come from the last downward pass."""
    d = workloads.desc(4, 3.8, 2.0, theta=(0.3, 1.1), n_stab=5, channel=ch, seed=9)
    sim = _sim([d])
    sim.sweep(2, measure=False)
    m = _model(d)
    f = sim.fields(0)
    sim.measure_tau()
    AA, At = tau.tau_correlator(m, f, m.M // 2)
    aa, at, n = sim.get_tau(0)
    np.testing.assert_allclose(aa, AA.real, rtol=1e-10, atol=0)
    np.testing.assert_allclose(at, At.real, rtol=1e-10, atol=0)
    ref = tau.tau_greens(m, f, 0, m.M // 2)[m.M // 2]
    for which in range(3):
        scale = max(1.0, np.abs(ref[which]).max())
        assert np.abs(sim.green_tau(0, which) - ref[which]).max() < 1e-10 * scale


def test_tau_pass_leaves_the_chain():
    """Same seed, same replayed decisions: a pass between sweeps changes
    neither the fields nor G of the following sweep."""
    import torch
    d = workloads.desc(4, 3.8, 2.0, theta=(0.7, 2.1), n_stab=5, seed=4)
    out = []
    for with_pass in (False, True):
        sim = _sim([d])
        N, M, _ = sim.shapes[0]
        bits = workloads.accept_bits(17, 2 * 2 * M * N, 0.4)
        b = torch.from_numpy(bits).reshape(1, -1).cuda()
        sim.replay(b[:, :2 * M * N].contiguous(), None, n_sweeps=1)
        if with_pass:
            sim.measure_tau()
        sim.replay(b[:, 2 * M * N:].contiguous(), None, n_sweeps=1)
        out.append((sim.fields(0), sim.green(0)))
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])


def test_tau_pass_leaves_parked_chains():
    """An instance that is not at the start of a sweep is parked during a
    pass; its working chain (mid upward pass) must come through unchanged.
    M = 20 and M = 25: after one handle sweep (50 steps) the first instance
    stands at phase 10 with two chain steps done, the second at phase 0."""
    import torch
    ds = [workloads.desc(4, 3.8, 2.0, theta=(0.7, 2.1), n_stab=5, seed=4),
          workloads.desc(3, 3.7, 2.5, n_stab=5, seed=8)]
    out = []
    for with_pass in (False, True):
        sim = _sim(ds)
        per = 2 * 25 * 32
        bits = workloads.accept_bits(23, 2 * per * 2, 0.4).reshape(2, -1)
        b = torch.from_numpy(bits).cuda()
        sim.replay(b[:, :per].contiguous(), None, n_sweeps=1)
        if with_pass:
            sim.measure_tau()
            assert sim.get_tau(0)[2] == 0 and sim.get_tau(1)[2] == 1
        sim.replay(b[:, per:2 * per].contiguous(), None, n_sweeps=1)
        out.append([(sim.fields(i), sim.green(i)) for i in range(2)])
    for i in range(2):
        np.testing.assert_array_equal(out[0][i][0], out[1][i][0])
        np.testing.assert_array_equal(out[0][i][1], out[1][i][1])


def test_autotune_returns_to_a_sweep_boundary():
    """The flush autotuner runs slice steps that are not whole sweeps; it ends
    with the steps that put the instances of the largest M back at the start
    of a sweep, where a pass can measure them."""
    ds = [workloads.desc(4, 3.8, 2.0, theta=(0.7, 2.1), n_stab=5, seed=4, k=8),
          workloads.desc(3, 3.7, 1.0, n_stab=5, seed=8, k=8)]
    sim = _sim(ds)
    sim.autotune([8, 16], 10)
    sim.sweep(1, measure=False)
    sim.measure_tau()
    assert sim.get_tau(0)[2] == 1
    m = _model(ds[0])
    AA, _ = tau.tau_correlator(m, sim.fields(0), m.M // 2)
    np.testing.assert_allclose(sim.get_tau(0)[0], AA.real, rtol=1e-10, atol=0)


@pytest.mark.parametrize("ch,th", [(0, (0.0, 0.0)), (0, (0.7, -0.4)), (1, (0.7, -0.4))])
def test_tau_chains_match_exact_l2(ch, th):
    """End to end against exact diagonalisation: 128 independent GPU chains
    on the L = 2 honeycomb torus at M = 2 (the Trotterised ensemble that the
    Fock-space ED evaluates exactly), one pass after every sweep.  The chain
    means of <A(tau_l) A(0)> (l = 0, 1) and <A> agree with the ED values, and
    dD/dU from the trapezoid of C with the central difference of the exact D,
    within 4 standard errors over chains (jackknife for dD/dU)."""
    from oracle import exact
    from paper_2609_14668_amd import tau_integrals
    U, dt, M = 3.8, 0.25, 2
    n, sweeps = 128, 150
    ds = [workloads.desc(2, U, M * dt, dtau=dt, theta=th, k=8, n_stab=2, seed=300 + i, channel=ch)
          for i in range(n)]
    sim = _sim(ds)
    sim.sweep(20, measure=False)
    for _ in range(sweeps):
        sim.sweep(1, measure=False)
        sim.measure_tau()
    # per chain: <A(tau_l) A(0)> (l = 0, 1), <A> at slice 0 and at slice 1
    X = np.array([np.concatenate([sim.get_tau(i)[0], sim.get_tau(i)[1]]) for i in range(n)])
    assert all(sim.get_tau(i)[2] == sweeps for i in range(n))
    kw = dict(U=U, dtau=dt, M=M, theta1=th[0], theta2=th[1], channel="charge" if ch else "spin")
    ed = exact.exact_tau_trotter2(exact.tiny_model(**kw))
    ref = np.concatenate([ed["AA"], [ed["A"], ed["A"]]])
    mean = X.mean(axis=0)
    err = X.std(axis=0, ddof=1) / np.sqrt(n)
    assert np.all(np.abs(mean - ref) < 4 * err), (mean, ref, err)
    Ns = 8

    def dd(rows):
        m = rows.mean(axis=0)
        return tau_integrals(m[:2] - m[2] ** 2, dt, Ns, -1)[0]

    jk = np.array([dd(np.delete(X, i, axis=0)) for i in range(n)])
    d_err = np.sqrt((n - 1) * np.mean((jk - jk.mean()) ** 2))
    h = 1e-4
    fd = (exact.exact_trotter(exact.tiny_model(**dict(kw, U=U + h)))["D"]
          - exact.exact_trotter(exact.tiny_model(**dict(kw, U=U - h)))["D"]) / (2 * h)
    print("dD/dU", dd(X), "+-", d_err, "exact", fd, flush=True)
    assert d_err < 0.02 * abs(fd)              # the comparison resolves dD/dU
    assert abs(dd(X) - fd) < 4 * d_err, (dd(X), fd, d_err)


def test_tau_large_l_stockham_path():
    """L = 30 twisted (N = 1800, the LDS Stockham FFT path), beta = 1, n_stab = 5:
    the pass to l = 5 (one recomputation) against the oracle's UDV G and
    explicit propagation, and its series at l = 5 from those matrices."""
    d = workloads.desc(30, 3.73, 1.0, theta=(0.4, 1.7), n_stab=5, k=64, seed=5)
    sim = _sim([d])
    m = _model(d)
    f = sim.fields(0)
    lm = 5
    sim.measure_tau(lm)
    G0 = m.green_scratch(f, 0, 0)
    Gt = m.green_scratch(f, lm, 0)
    P = np.eye(m.N, dtype=complex)
    Pi = np.eye(m.N, dtype=complex)
    for l in range(1, lm + 1):
        P = m.B(0, f[l - 1]) @ P
        Pi = Pi @ m.Binv(0, f[l - 1])
    Gt0 = P @ G0
    G0t = -(np.eye(m.N) - G0) @ Pi
    for which, ref in enumerate((Gt, Gt0, G0t)):
        err = np.abs(sim.green_tau(0, which) - ref).max()
        assert err < 1e-9, (which, err)
    aa, at, n = sim.get_tau(0)
    assert n == 1
    t = (0.5 - np.diag(Gt))[:, None] * (0.5 - np.diag(G0))[None, :] - G0t.T * Gt0
    ref = np.sum(np.abs(t) ** 2)
    assert abs(aa[lm] - ref) < 1e-9 * ref, (aa[lm], ref)


def test_tau_rows_ring():
    """The per-pass rows keep the last 1024 passes (oldest overwritten) while
    the sums and the count cover all of them; passes do not touch the
    equal-time estimators."""
    d = workloads.desc(3, 3.8, 0.6, n_stab=3, seed=12)
    sim = _sim([d])
    sim.sweep(1, measure=True)
    n_meas0 = sim.measure(0)["n_meas"]
    assert n_meas0 > 0
    sim.measure_tau()
    one_aa, one_at, n = sim.get_tau(0)
    assert n == 1
    for _ in range(1029):
        sim.measure_tau()
    aa, at, n = sim.get_tau(0)
    assert n == 1030
    np.testing.assert_allclose(aa, one_aa, rtol=1e-13, atol=0)
    np.testing.assert_allclose(at, one_at, rtol=1e-13, atol=0)
    rows = sim.tau_rows(0, max_rows=2000)
    lc = sim.shapes[0][1] // 2
    assert rows.shape == (1024, 2 * lc + 2)
    np.testing.assert_array_equal(rows, np.broadcast_to(np.concatenate([one_aa, one_at]), rows.shape))
    assert sim.tau_rows(0, max_rows=5).shape == (5, 2 * lc + 2)
    assert sim.measure(0)["n_meas"] == n_meas0


def test_tau_full_size_sampled():
    """Twisted L = 18, beta = 18 (N = 648, M = 180), the benched shape: the
    pass up to l = 10 (one recomputation) against the oracle's pinned UDV G
    at slices 0 and 10 and explicit propagation over the 10 slices, and the
    series at l = 0 and l = 10 from those matrices."""
    d = workloads.desc(18, 3.73, 18.0, theta=(0.9, 2.3), n_stab=10, k=32, seed=2)
    sim = _sim([d])
    m = _model(d)
    f = sim.fields(0)
    lm = 10
    sim.measure_tau(lm)
    G0 = m.green_scratch(f, 0, 0)
    Gt = m.green_scratch(f, lm, 0)
    P = np.eye(m.N, dtype=complex)
    Pi = np.eye(m.N, dtype=complex)
    for l in range(1, lm + 1):
        P = m.B(0, f[l - 1]) @ P
        Pi = Pi @ m.Binv(0, f[l - 1])
    Gt0 = P @ G0
    G0t = -(np.eye(m.N) - G0) @ Pi
    for which, ref in enumerate((Gt, Gt0, G0t)):
        err = np.abs(sim.green_tau(0, which) - ref).max()
        assert err < 1e-8, (which, err)
    assert sim.stats(0)["drift_last"] < 1e-8
    aa, at, n = sim.get_tau(0)
    assert n == 1
    for l, (gtt, gt0, g0t) in ((0, (G0, G0, G0 - np.eye(m.N))), (lm, (Gt, Gt0, G0t))):
        t = (0.5 - np.diag(gtt))[:, None] * (0.5 - np.diag(G0))[None, :] - g0t.T * gt0
        ref = np.sum(np.abs(t) ** 2)
        assert abs(aa[l] - ref) < 1e-8 * ref, (l, aa[l], ref)
        a_ref = -np.sum(np.abs(0.5 - np.diag(gtt)) ** 2)
        assert abs(at[l] - a_ref) < 1e-9 * abs(a_ref), (l, at[l], a_ref)
