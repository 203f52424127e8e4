"""Pins of the oracle's time-displaced Green's functions, the interaction-energy
correlator C(tau) and the integrals of eqs. DouOccDerive and fidelitysusp
(Sec. II C) against exact diagonalisation, closed forms and the oracle's own
(separately pinned) equal-time Green's function."""
import numpy as np
import pytest

from oracle import dqmc, exact, tau


@pytest.mark.parametrize("channel", ["spin", "charge"])
@pytest.mark.parametrize("cluster", ["dimer", "ring4_flux"])
def test_brute_force_correlator_matches_fock_ed(cluster, channel):
    """<A(tau_l) A(0)> for every slice l = 0..M: the weighted average of the
    per-configuration Wick estimator over all HS configurations equals
    Tr[T^{M-l} A T^l A]/Z of the Trotterised Hamiltonian in full Fock space."""
    if cluster == "dimer":
        K, M = exact.dimer_hopping(), 6
    else:
        K, M = exact.ring4_hopping(phi=0.3), 4
    U, dt = 3.0, 0.2
    m = dqmc.Model.from_hopping(K, U, M * dt, dt, channel=channel)
    bf = exact.brute_force_tau(m, M)
    ed = exact.exact_tau_fock(K, U, dt, M)
    assert ed["max_imag"] < 1e-14
    assert bf["AA_imag"] < 1e-12
    np.testing.assert_allclose(bf["AA"], ed["AA"], rtol=0, atol=1e-12)
    assert abs(bf["A"] - ed["A"]) < 1e-12
    # C(tau) = C(beta - tau), half filling
    np.testing.assert_allclose(ed["AA"], ed["AA"][::-1], rtol=0, atol=1e-13)
    assert abs(ed["Ntot"] - K.shape[0]) < 1e-12


@pytest.mark.parametrize("channel", ["spin", "charge"])
@pytest.mark.parametrize("twist", [(0.0, 0.0), (0.7, -0.4)])
def test_honeycomb_l2_correlator_matches_ed(twist, channel):
    """The honeycomb torus L = 2 (N = 8), M = 2: l = 0 and l = 1 = beta/2."""
    m = exact.tiny_model(U=3.8, dtau=0.25, M=2, theta1=twist[0], theta2=twist[1], channel=channel)
    bf = exact.brute_force_tau(m, 1)
    ed = exact.exact_tau_trotter2(m)
    np.testing.assert_allclose(bf["AA"], ed["AA"], rtol=1e-12, atol=0)
    assert abs(bf["A"] - ed["A"]) < 1e-12


@pytest.mark.parametrize("cluster", ["dimer", "ring4_flux"])
def test_trotter_derivative_identity(cluster):
    """dD/dU of the Trotterised ensemble (central difference of the exact D)
    equals -(2/N_s) times the trapezoid integral of C over [0, beta/2]
    (eq. DouOccDerive on the slice grid), both from the exact C and from the
    brute-force average of the oracle's estimator."""
    if cluster == "dimer":
        K, M = exact.dimer_hopping(), 6
    else:
        K, M = exact.ring4_hopping(phi=0.3), 4
    U, dt, h = 3.0, 0.2, 1e-4
    N = K.shape[0]
    fd = (exact.exact_tau_fock(K, U + h, dt, M)["D"] - exact.exact_tau_fock(K, U - h, dt, M)["D"]) / (2 * h)
    ed = exact.exact_tau_fock(K, U, dt, M)
    d_ed, _ = tau.tau_integrals(tau.connected(ed["AA"], ed["A"])[:M // 2 + 1], dt, N)
    assert abs(d_ed - fd) < 1e-8
    m = dqmc.Model.from_hopping(K, U, M * dt, dt, channel="spin")
    bf = exact.brute_force_tau(m, M // 2)
    d_bf, _ = tau.tau_integrals(tau.connected(bf["AA"], bf["A"]), dt, N)
    assert abs(d_bf - fd) < 1e-8


def test_u0_closed_form():
    """U = 0 (lambda = 0): G(tau,0) = e^{-tau K}(1 + e^{-beta K})^{-1},
    G(0,tau) = -(1 - G) e^{tau K}, G(tau,tau) = G for any fields (twisted L = 3)."""
    m = dqmc.Model(3, 0.0, 2.0, 0.1, theta1=0.9, theta2=0.35, n_stab=10)
    rng = np.random.default_rng(5)
    X = rng.choice([-1, 1], size=(m.M, m.N))
    w, V = np.linalg.eigh(m.K)
    G = (V / (1 + np.exp(-m.beta * w))) @ V.conj().T
    for s in (0, 1):
        gs = tau.tau_greens(m, X, s, m.M // 2)
        for l, (gtt, gt0, g0t) in enumerate(gs):
            t = l * m.dtau
            et = (V * np.exp(-t * w)) @ V.conj().T
            emt = (V * np.exp(t * w)) @ V.conj().T
            np.testing.assert_allclose(gtt, G, rtol=0, atol=1e-12)
            np.testing.assert_allclose(gt0, et @ G, rtol=0, atol=1e-12)
            if l > 0:
                np.testing.assert_allclose(g0t, -(np.eye(m.N) - G) @ emt, rtol=0, atol=1e-12)


@pytest.mark.parametrize("channel", ["spin", "charge"])
def test_block_inverse_matches_propagation(channel):
    """At U > 0 with random fields (twisted L = 3, beta = 0.8): the blocks of
    the block-cyclic inverse against the oracle's UDV G(l) (pinned by mpmath
    and ED elsewhere) and explicit propagation,
    G(tau_l, 0) = B_l..B_1 G(0), G(0, tau_l) = -(1 - G(0)) (B_l..B_1)^{-1}."""
    m = dqmc.Model(3, 3.73, 0.8, 0.1, theta1=0.6, theta2=-0.25, n_stab=4, channel=channel)
    rng = np.random.default_rng(11)
    X = rng.choice([-1, 1], size=(m.M, m.N))
    for s in (0, 1):
        g0 = m.green_scratch(X, 0, s)
        gs = tau.tau_greens(m, X, s, m.M - 1)
        P = np.eye(m.N, dtype=complex)
        for l, (gtt, gt0, g0t) in enumerate(gs):
            if l > 0:
                P = m.B(s, X[l - 1]) @ P
            np.testing.assert_allclose(gtt, m.green_scratch(X, l, s), rtol=0, atol=1e-11)
            np.testing.assert_allclose(gt0, P @ g0, rtol=0, atol=1e-11)
            ref = -(np.eye(m.N) - g0) @ np.linalg.inv(P) if l > 0 else g0 - np.eye(m.N)
            np.testing.assert_allclose(g0t, ref, rtol=0, atol=1e-10)


def test_equal_time_correlator_matches_observables():
    """l = 0 of the correlator is the equal-time <A^2>_X; its diagonal part
    reproduces D through <A>_X = sum_i m_up m_dn = N_s (D - 1/4) per
    configuration (spin channel, G_dn from the explicit spin-down B's)."""
    m = dqmc.Model(3, 3.73, 1.0, 0.1, theta1=0.3, theta2=0.2, n_stab=5)
    rng = np.random.default_rng(2)
    X = rng.choice([-1, 1], size=(m.M, m.N))
    AA, At = tau.tau_correlator(m, X, 0)
    A1 = At[0]
    Gu, Gd = m.green_scratch(X, 0, 0), m.green_scratch(X, 0, 1)
    D = np.mean((1 - np.diag(Gu)) * (1 - np.diag(Gd)))
    # sum_i (n_up - 1/2)(n_dn - 1/2) = sum n_up n_dn - (N_up + N_dn)/2 + N/4
    nt = np.sum(2 - np.diag(Gu) - np.diag(Gd))
    assert abs(A1 - (m.N * D - nt / 2 + m.N / 4)) < 1e-12


def test_improved_estimator_matches_plain_average():
    """The improved connected estimator equals <AA> - <A>^2 of the same
    rows exactly when <A>_X(tau) is the same in every slice of a row
    (constructed rows)."""
    rng = np.random.default_rng(0)
    n, lt = 400, 6
    a0 = -3.0 + 0.7 * rng.standard_normal(n)
    at = np.repeat(a0[:, None], lt, axis=1)
    ferm = 0.4 * np.exp(-np.arange(lt))[None, :] + 0.05 * rng.standard_normal((n, lt))
    aa = ferm + at * at[:, :1]
    imp = tau.connected_improved(aa, at)
    plain = tau.connected(aa.mean(axis=0), a0.mean())
    np.testing.assert_allclose(imp, plain, rtol=0, atol=1e-12)


def test_integrals_closed_forms():
    """Trapezoid: exact for linear C, and for tau C quadratic off by exactly
    the rule's error term;
    the polynomial fit of degree p reproduces the analytic integrals of a
    degree-p polynomial C(tau)."""
    dt, n, Ns = 0.1, 21, 18
    t = dt * np.arange(n)
    tb = t[-1]
    c = 2.0 - 0.5 * t
    d, chi = tau.tau_integrals(c, dt, Ns)
    assert abs(d - (-2.0 / Ns) * (2.0 * tb - 0.25 * tb ** 2)) < 1e-13
    # tau C = 2 tau - tau^2 / 2: the trapezoid error of a quadratic is (b - a) h^2 f'' / 12
    assert abs(chi - (tb ** 2 - tb ** 3 / 6 + tb * dt ** 2 * (-1.0) / 12)) < 1e-13
    coef = [1.3, -2.0, 0.7, -0.05]
    c = sum(a * t ** k for k, a in enumerate(coef))
    d, chi = tau.tau_integrals(c, dt, Ns, degree=3)
    i0 = sum(a * tb ** (k + 1) / (k + 1) for k, a in enumerate(coef))
    i1 = sum(a * tb ** (k + 2) / (k + 2) for k, a in enumerate(coef))
    assert abs(d - (-2.0 / Ns) * i0) < 1e-12
    assert abs(chi - i1) < 1e-12
