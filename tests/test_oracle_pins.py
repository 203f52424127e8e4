"""Pins of the CPU oracle against what the paper and the mathematics fix:
closed forms, brute force, exact diagonalisation, known-answer vectors and
extended-precision inversion.  None of these re-types an oracle formula."""
import numpy as np
import pytest

from oracle import exact, philox, stats
from oracle.dqmc import BitSource, Chain, Model, RandomSource, g_down_from_up, hs_alpha, hs_lambda
from oracle.lattice import Lattice


# ---- Philox: published known-answer vectors ------------------------------------------
@pytest.mark.parametrize("ctr,key,out", [
    ((0, 0, 0, 0), (0, 0), (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
    ((0xffffffff,) * 4, (0xffffffff,) * 2, (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
    ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
     (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
])
def test_philox_kat(ctr, key, out):
    assert philox.philox4x32_10(ctr, key) == out


def test_philox_uniform_range_and_mean():
    u = np.array([philox.uniform_site(12345, 0, 0, 1, i) for i in range(4000)])
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 5 * np.sqrt(1 / 12 / len(u))


# ---- lattice and hopping matrix ---------------------------------------------------------
@pytest.mark.parametrize("L,th", [(2, (0, 0)), (3, (0, 0)), (4, (0.0, 0.0)), (3, (0.9, 2.3)),
                                  (5, (np.pi / 2, np.pi)), (6, (0.3 * np.pi, 0.7 * np.pi))])
def test_spectrum_is_pm_abs_f_on_shifted_grid(L, th):
    lat = Lattice(L, 1.0, *th)
    K = lat.hopping_matrix()
    w = np.linalg.eigvalsh(K)
    ref = np.sort(lat.dispersion())
    assert np.allclose(np.sort(w), ref, atol=1e-13)


def test_gauge_two_is_unitarily_equivalent_and_twist_sign_is_conjugation():
    lat = Lattice(4, 1.0, 0.8, 2.0)
    K1 = lat.hopping_matrix("I")
    K2 = lat.hopping_matrix("II")
    assert np.allclose(np.linalg.eigvalsh(K1), np.linalg.eigvalsh(K2), atol=1e-13)
    # the two gauges differ by one uniform phase on the B sublattice
    ratio = K2[:lat.Nc, lat.Nc:][K1[:lat.Nc, lat.Nc:] != 0] / K1[:lat.Nc, lat.Nc:][K1[:lat.Nc, lat.Nc:] != 0]
    assert np.allclose(ratio, ratio[0], atol=1e-14)
    assert np.allclose(Lattice(4, 1.0, -0.8, -2.0).hopping_matrix(), np.conj(K1), atol=1e-15)


def test_small_torus_bond_count_and_hermiticity():
    lat = Lattice(2)
    K = lat.hopping_matrix()
    assert np.allclose(K, K.T)
    # 3 N_c bonds; on L=2 none coincide, so every nonzero entry is -t
    assert np.count_nonzero(K) == 2 * 3 * lat.Nc
    assert np.allclose(K[K != 0], -1.0)


def test_gauges_give_identical_physics():
    fields = np.random.default_rng(3).choice([-1, 1], size=(20, 32))
    a = Model(4, 3.7, 2.0, 0.1, theta1=1.1, theta2=0.4, gauge="I")
    b = Model(4, 3.7, 2.0, 0.1, theta1=1.1, theta2=0.4, gauge="II")
    from oracle.dqmc import observables
    ga = [a.green_scratch(fields, 5, s) for s in (0, 1)]
    gb = [b.green_scratch(fields, 5, s) for s in (0, 1)]
    oa = observables(a.lat, a.K, *ga, a.U)
    ob = observables(b.lat, b.K, *gb, b.U)
    for k in ("D", "ekin", "m2", "Rm2"):
        assert abs(oa[k] - ob[k]) < 1e-11


# ---- propagator: k-space closed form through the Fourier matrix ---------------------------
@pytest.mark.parametrize("L,th", [(3, (0, 0)), (4, (0.5, 1.7)), (6, (0.0, 0.0))])
def test_propagator_matches_kspace_closed_form(L, th):
    m = Model(L, 3.8, 1.0, 0.1, theta1=th[0], theta2=th[1])
    Ek = exact.kspace_block_matrix(m.lat, lambda h, f: exact.exp_h_closed(h, f, -m.dtau))
    assert np.abs(Ek - m.Ep).max() < 1e-13
    Ekm = exact.kspace_block_matrix(m.lat, lambda h, f: exact.exp_h_closed(h, f, +m.dtau))
    assert np.abs(Ekm - m.Em).max() < 1e-13


def test_hs_coupling_identity():
    # 1/2 sum_x exp(lambda x (n_up - n_dn)) equals exp(-dtau U (n_up n_dn - (n_up+n_dn)/2))
    U, dtau = 3.73, 0.1
    lam = hs_lambda(U, dtau)
    for nu in (0, 1):
        for nd in (0, 1):
            lhs = 0.5 * sum(np.exp(lam * x * (nu - nd)) for x in (1, -1))
            rhs = np.exp(-dtau * U * (nu * nd - (nu + nd) / 2))
            assert abs(lhs - rhs) < 1e-15


def test_hs_charge_coupling_identity():
    # eq. DensityHS: (e^{dtau U/2}/2) sum_x exp(gamma_c x (n_up + n_dn - 1)) with
    # gamma_c = i alpha, cos(alpha) = exp(-dtau U/2) (eq. coupling)
    U, dtau = 3.73, 0.1
    gc = 1j * hs_alpha(U, dtau)
    for nu in (0, 1):
        for nd in (0, 1):
            lhs = 0.5 * np.exp(dtau * U / 2) * sum(np.exp(gc * x * (nu + nd - 1)) for x in (1, -1))
            rhs = np.exp(-dtau * U * (nu * nd - (nu + nd) / 2))
            assert abs(lhs - rhs) < 1e-15


# ---- U = 0 closed form ------------------------------------------------------------------
@pytest.mark.parametrize("L,beta,th", [(3, 3.0, (0, 0)), (4, 4.0, (0.6, 1.3)), (6, 6.0, (0, 0))])
def test_u0_green_energy_double_occupancy(L, beta, th):
    m = Model(L, 0.0, beta, 0.1, theta1=th[0], theta2=th[1])
    fields = np.random.default_rng(L).choice([-1, 1], size=(m.M, m.N))
    ch = Chain(m, fields)
    G0 = exact.green_u0(m.lat, beta)
    assert np.abs(ch.G[0] - G0).max() < 1e-12
    assert np.abs(ch.G[1] - G0).max() < 1e-12
    ch.sweep(RandomSource(1))
    o = ch.samples[-1]
    assert abs(o["ekin"] - exact.energy_u0(m.lat, beta)) < 1e-12
    assert abs(o["D"] - 0.25) < 1e-12
    assert abs(o["n"] - 1.0) < 1e-12
    # momentum distribution (eq. nkMatrix): band occupations are Fermi functions
    from oracle.dqmc import nk_bands
    npl, nmi = nk_bands(o["nk"])
    ref_p, ref_m = exact.bands_u0(m.lat, beta)
    assert np.abs(npl - ref_p).max() < 1e-12 and np.abs(nmi - ref_m).max() < 1e-12
    # charge compressibility (eq. ChiCharge): sum of level variances
    assert abs(o["chi_e"] - exact.chi_e_u0(m.lat, beta)) < 1e-11


# ---- brute force over all HS configurations vs Fock-space ED ----------------------------
@pytest.mark.parametrize("channel", ["spin", "charge"])
@pytest.mark.parametrize("th", [(0.0, 0.0), (0.7, 1.9)])
def test_bruteforce_equals_exact_diagonalisation(th, channel):
    """Both HS channels (eqs. SzHS and DensityHS) decouple the same
    Trotterised interaction, so the sum of either channel's weights over
    every configuration reproduces the Fock-space trace, and every weight is
    real and positive (for HS-n by the partial particle-hole symmetry of
    Sec. II B, with the phase of P(X) included)."""
    m = exact.tiny_model(U=3.8, dtau=0.25, M=2, theta1=th[0], theta2=th[1], channel=channel)
    bf = exact.brute_force(m)
    ed = exact.exact_trotter(m)
    assert bf["wmin"] > 0 and bf["w_max_rel_imag"] < 1e-12
    for k in ("Z", "D", "H0", "SzzG", "Szzdk", "N2", "Ntot"):
        assert abs(bf[k] - ed[k]) <= 1e-12 * max(1.0, abs(ed[k])), k
    # momentum distribution: Fourier sums of the Fock-space one-body density matrix
    Nc = m.Nc
    Uc = exact.fourier_matrix(m.lat)[:Nc, :Nc]
    nk_ed = np.zeros((Nc, 2, 2), dtype=complex)
    for spin in (0, 1):
        for a in (0, 1):
            for b in (0, 1):
                blk = ed["rho"][spin][a * Nc:(a + 1) * Nc, b * Nc:(b + 1) * Nc]
                nk_ed[:, a, b] += 0.5 * np.einsum("kr,rs,ks->k", Uc.conj(), blk, Uc)
    assert np.abs(bf["nk"] - nk_ed).max() < 1e-12


@pytest.mark.parametrize("th", [(0.0, 0.0), (0.7, 1.9)])
def test_charge_channel_configurations_are_particle_hole_symmetric(th):
    """HS-n couples both spins identically (G_dn = G_up in the original
    basis), and at half filling every configuration has Re G_ii = 1/2 and a
    real positive weight P(X) det^2; a planted sign error in the prior phase
    breaks the positivity."""
    m = exact.tiny_model(U=3.8, dtau=0.25, M=2, theta1=th[0], theta2=th[1], channel="charge")
    X = np.random.default_rng(5).choice([-1, 1], size=(64, m.M, m.N))
    c = exact.config_estimators(m, X)
    assert np.abs(c["Gup"] - c["Gdn"]).max() == 0.0
    assert np.abs(np.einsum("bii->bi", c["Gup"]).real - 0.5).max() < 1e-13
    assert np.max(np.abs(c["W"].imag) / np.abs(c["W"])) < 1e-12 and c["W"].real.min() > 0
    # planted mistake: the prior phase with the wrong sign
    bad = c["W"] * np.exp(2j * m.alpha * X.reshape(len(X), -1).sum(axis=1))
    assert np.max(np.abs(bad.imag) / np.abs(bad)) > 1e-3


def test_single_slice_exact_diagonalisation():
    m = exact.tiny_model(U=2.5, dtau=0.3, M=1)
    bf = exact.brute_force(m)
    ed = exact.exact_trotter(m)
    for k in ("Z", "D", "H0"):
        assert abs(bf[k] - ed[k]) <= 1e-12 * max(1.0, abs(ed[k]))


# ---- determinant ratio and Sherman-Morrison against brute-force determinants ---------------
@pytest.mark.parametrize("th", [(0.0, 0.0), (1.3, 0.2)])
def test_ratio_and_update_against_determinants(th):
    m = Model(2, 3.8, 1.0, 0.25, theta1=th[0], theta2=th[1], n_stab=2)
    rng = np.random.default_rng(7)
    fields = rng.choice([-1, 1], size=(m.M, m.N)).astype(np.int8)
    ch = Chain(m, fields)
    w0 = np.prod(m.weight_dets(ch.fields))
    # walk the upward pass with bits: accept every second proposal
    bits = np.tile([1, 0], m.M * m.N * 2)
    src = BitSource(bits)
    for l in range(1, m.M + 1):
        ch.wrap_up(l)
        for i in range(m.N):
            before = ch.fields.copy()
            w_before = np.prod(m.weight_dets(before))
            trial = before.copy()
            trial[l - 1, i] = -trial[l - 1, i]
            w_after = np.prod(m.weight_dets(trial))
            ch_ratio_index = len(ch.ratios)
            # run exactly one proposal
            lam = m.lam
            x = float(before[l - 1, i])
            dl = (np.exp(-2 * lam * x) - 1, np.exp(2 * lam * x) - 1)
            r = [1 + dl[s] * (1 - ch.G[s][i, i]) for s in (0, 1)]
            R = (r[0] * r[1]).real
            assert abs(R - (w_after / w_before).real) < 1e-10 * max(1, abs(R))
            if src(0, 0, l, i, R):
                for s in (0, 1):
                    G = ch.G[s]
                    xv = G[:, i] * (dl[s] / r[s])
                    yv = -G[i, :].copy()
                    yv[i] += 1
                    ch.G[s] = G - np.outer(xv, yv)
                ch.fields[l - 1, i] *= -1
                for s in (0, 1):
                    Gs = m.green_direct(ch.fields, l, s)
                    assert np.abs(Gs - ch.G[s]).max() < 1e-10
            del ch_ratio_index
    assert w0 > 0


@pytest.mark.parametrize("th", [(0.0, 0.0), (1.3, 0.2)])
def test_charge_ratio_and_update_against_determinants(th):
    """HS-n chain: every ratio R = exp(2 i alpha x) r_up r_dn equals the
    brute-force weight ratio P(X') det'^2 / P(X) det^2, and the
    Sherman-Morrison G equals the direct recomputation after each flip."""
    m = Model(2, 3.8, 1.0, 0.25, theta1=th[0], theta2=th[1], n_stab=2, channel="charge")
    rng = np.random.default_rng(9)
    ch = Chain(m, rng.choice([-1, 1], size=(m.M, m.N)).astype(np.int8))

    def weight(f):
        return np.exp(m.log_prior(f)) * np.prod(m.weight_dets(f))

    src = BitSource(np.tile([1, 0], m.M * m.N))
    for l in range(1, m.M + 1):
        ch.wrap_up(l)
        for i in range(m.N):
            trial = ch.fields.copy()
            trial[l - 1, i] = -trial[l - 1, i]
            ratio = weight(trial) / weight(ch.fields)
            R, dl, r = ch.site_ratio(l, i)
            assert abs(ratio.imag) < 1e-10 * abs(ratio) and abs(R - ratio.real) < 1e-10 * max(1.0, abs(R))
            if src(0, 0, l, i, R):
                for s in (0, 1):
                    G = ch.G[s]
                    xv = G[:, i] * (dl[s] / r[s])
                    yv = -G[i, :].copy()
                    yv[i] += 1
                    ch.G[s] = G - np.outer(xv, yv)
                ch.fields[l - 1, i] *= -1
                for s in (0, 1):
                    assert np.abs(m.green_direct(ch.fields, l, s) - ch.G[s]).max() < 1e-10


def test_weight_ratio_factorises_through_spin_up_only():
    # W'/W = exp(2 lambda x) |r_up|^2 (particle-hole relation of Sec. II B)
    m = Model(3, 3.7, 1.0, 0.1, theta1=0.4, theta2=2.2)
    fields = np.random.default_rng(11).choice([-1, 1], size=(m.M, m.N))
    G = [m.green_scratch(fields, 4, s) for s in (0, 1)]
    lam = m.lam
    for i in range(m.N):
        x = fields[3, i]
        ru = 1 + (np.exp(-2 * lam * x) - 1) * (1 - G[0][i, i])
        rd = 1 + (np.exp(2 * lam * x) - 1) * (1 - G[1][i, i])
        assert abs(ru * rd - np.exp(2 * lam * x) * abs(ru) ** 2) < 1e-12 * abs(ru * rd)


def test_particle_hole_partner_from_independent_spin_down():
    m = Model(3, 3.8, 3.0, 0.1, theta1=0.9, theta2=2.1)
    fields = np.random.default_rng(1).choice([-1, 1], size=(m.M, m.N))
    for l in (0, 7, 30):
        Gu = m.green_scratch(fields, l, 0)
        Gd = m.green_scratch(fields, l, 1)
        assert np.abs(Gd - g_down_from_up(Gu, m.Nc)).max() < 1e-12


def test_symmetric_split_has_the_same_weight():
    m = Model(2, 3.8, 1.0, 0.25)
    fields = np.random.default_rng(5).choice([-1, 1], size=(m.M, m.N))
    for spin in (0, 1):
        P1 = np.eye(m.N)
        P2 = np.eye(m.N)
        for l in range(m.M):
            v = m.vdiag(spin, fields[l])
            P1 = (v[:, None] * m.Ep) @ P1
            P2 = (m.Ehp @ (v[:, None] * m.Ehp)) @ P2
        assert abs(np.linalg.det(np.eye(m.N) + P1) / np.linalg.det(np.eye(m.N) + P2) - 1) < 1e-12


# ---- stabilised G against 50-digit arithmetic ------------------------------------------------
def test_stabilised_green_against_extended_precision():
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 50
    m = Model(3, 3.8, 3.0, 0.1, n_stab=10)
    fields = np.random.default_rng(2).choice([-1, 1], size=(m.M, m.N))
    l = 10
    G = m.green_scratch(fields, l, 0)
    # exp(-dtau K) to 50 digits from the k-space closed form via mpmath
    Kmp = mp.matrix(m.K.real.tolist())
    Ep = mp.expm(-mp.mpf("0.1") * Kmp)
    lam = mp.acosh(mp.exp(mp.mpf("0.1") * mp.mpf("3.8") / 2))
    P = mp.eye(m.N)
    for j in range(m.M):
        s = ((l + j) % m.M) + 1
        V = mp.diag([mp.exp(lam * int(x)) for x in fields[s - 1]])
        P = V * Ep * P
    Gmp = (mp.eye(m.N) + P) ** -1
    Gref = np.array([[float(Gmp[i, j]) for j in range(m.N)] for i in range(m.N)])
    assert np.abs(G - Gref).max() < 1e-12


# ---- the chain: wrap invariant, replay determinism, MC vs ED ---------------------------------
def test_wrap_invariant_over_full_sweep():
    m = Model(3, 3.8, 3.0, 0.1, n_stab=10)
    fields = np.random.default_rng(4).choice([-1, 1], size=(m.M, m.N))
    ch = Chain(m, fields)
    ch.sweep(RandomSource(9))
    assert len(ch.drift) == 2 * 2 * m.M // m.n_stab
    assert max(ch.drift) < 1e-10
    assert 0.05 < ch.accepted / ch.proposals < 0.95


def test_replay_all_reject_keeps_fields_and_all_accept_flips_all():
    m = Model(2, 3.8, 1.0, 0.25, n_stab=2)
    f0 = np.random.default_rng(0).choice([-1, 1], size=(m.M, m.N))
    ch = Chain(m, f0)
    ch.sweep(BitSource(np.zeros(2 * m.M * m.N)))
    assert np.array_equal(ch.fields, f0)
    ch2 = Chain(m, f0)
    ch2.sweep(BitSource(np.ones(2 * m.M * m.N)))
    assert np.array_equal(ch2.fields, f0)   # every field flipped twice


@pytest.mark.slow
@pytest.mark.parametrize("channel", ["spin", "charge"])
def test_markov_chain_reproduces_exact_diagonalisation(channel):
    m = exact.tiny_model(U=3.8, dtau=0.25, M=2, channel=channel)
    ed = exact.exact_trotter(m)
    rng = np.random.default_rng(17)
    ch = Chain(m, rng.choice([-1, 1], size=(m.M, m.N)))
    src = RandomSource(23)
    for _ in range(200):
        ch.sweep(src, measure=False)
    ch.samples = []
    per_sweep = []
    for _ in range(3000):
        n0 = len(ch.samples)
        ch.sweep(src)
        per_sweep.append({k: np.mean([s[k] for s in ch.samples[n0:]])
                          for k in ("D", "ekin", "Szz_G", "Szz_dk", "chi_e")})
    chi_ref = (m.beta / m.N) * (ed["N2"] - ed["Ntot"] ** 2)
    for key, ref in (("D", ed["D"]), ("ekin", ed["H0"] / m.N), ("Szz_G", ed["SzzG"]),
                     ("Szz_dk", ed["Szzdk"]), ("chi_e", chi_ref)):
        x = np.array([p[key] for p in per_sweep])
        mu, err = stats.mean_err(x)
        assert abs(mu - ref) < 4 * err, (key, mu, ref, err)
    # R_m2 = 1 - <S_zz(b1/L)> / <S_zz(Gamma)> (eq. CrfRatio): a ratio of means,
    # its error from a jackknife over 50 blocks of sweeps
    a = np.array([p["Szz_dk"] for p in per_sweep])
    b = np.array([p["Szz_G"] for p in per_sweep])
    nb = 50
    a_b = a[: len(a) // nb * nb].reshape(nb, -1).mean(axis=1)
    b_b = b[: len(b) // nb * nb].reshape(nb, -1).mean(axis=1)
    r = 1.0 - a_b.mean() / b_b.mean()
    jk = np.array([1.0 - (a_b.sum() - a_b[j]) / (b_b.sum() - b_b[j]) for j in range(nb)])
    err = np.sqrt((nb - 1) / nb * np.sum((jk - jk.mean()) ** 2))
    ref = 1.0 - ed["Szzdk"] / ed["SzzG"]
    assert abs(r - ref) < 4 * err, ("Rm2", r, ref, err)


# ---- statistics helpers ---------------------------------------------------------------------
def test_tau_int_of_ar1_process():
    phi = 0.8
    rng = np.random.default_rng(0)
    n = 400000
    e = rng.standard_normal(n)
    x = np.empty(n)
    x[0] = e[0]
    for i in range(1, n):
        x[i] = phi * x[i - 1] + e[i]
    tau = stats.tau_int(x)
    exact_tau = (1 + phi) / (2 * (1 - phi))
    assert abs(tau - exact_tau) / exact_tau < 0.05
    err = stats.binning_error(x)
    sig = np.sqrt(1 / (1 - phi ** 2))
    assert abs(err - sig * np.sqrt(2 * exact_tau / n)) / (sig * np.sqrt(2 * exact_tau / n)) < 0.25
