"""Pin of the oracle's equal-time estimators (``oracle.dqmc.observables``)
configuration by configuration.

The reference is ``exact.config_estimators``: for a batch of HS
configurations it propagates both spins densely, inverts 1 + B..B and takes
D, <H_0>, S_zz(Gamma) and S_zz(b1/L) by contracting the whole same-sublattice
spin-correlation block with plane waves (eqs. SzSzCrF, SpinStrucF).  Its
W-weighted averages over all 2^16 configurations of the L=2, M=2 lattice equal
the Fock-space exact diagonalisation of the Trotterised partition function
(``test_oracle_pins.test_bruteforce_equals_exact_diagonalisation``), so it is
pinned by ED; here it pins ``observables()``, which builds S_zz(k) from the
real-space correlation C_zz(d1, d2) of eq. SzSzCrF, for every configuration.

S_zz(k) per configuration is real and even in k (the Wick estimate of
<s_i s_j> is symmetric in i, j), so the sign of the plane-wave phase is not
observable; what can go wrong is the axis the phase runs along (d1 vs d2), the
momentum, the exchange term and the normalisation.  Each such mistake,
planted in a copy of the oracle's function, must fail this pin.
"""
import inspect
import textwrap

import numpy as np
import pytest

import oracle.dqmc as odq
from oracle import exact
from oracle.dqmc import Model, g_down_from_up, observables


def _cases(channel="spin"):
    out = []
    for L, M, th, n_cfg, seed in ((2, 2, (0.0, 0.0), 96, 1), (2, 2, (0.7, 1.9), 96, 2),
                                  (3, 2, (0.0, 0.0), 24, 3), (3, 2, (1.1, 0.4), 24, 4),
                                  (4, 2, (0.3 * np.pi, 0.7 * np.pi), 8, 5)):
        m = Model(L, 3.8, M * 0.25, 0.25, theta1=th[0], theta2=th[1], n_stab=M, channel=channel)
        X = np.random.default_rng(seed).choice([-1.0, 1.0], size=(n_cfg, M, m.N))
        out.append((m, X))
    return out


CASES = _cases()
CHARGE_CASES = _cases("charge")


def _violations(obs_fn, tol=1e-12, cases=None):
    """Largest deviation of obs_fn from the per-configuration reference.  In
    the charge channel the per-configuration estimators are complex (only
    their averages are real): observables() returns their real parts."""
    worst = 0.0
    for m, X in (CASES if cases is None else cases):
        ref = exact.config_estimators(m, X)
        for b in range(len(X)):
            Gu, Gd = ref["Gup"][b], ref["Gdn"][b]
            if not m.complex:
                Gu, Gd = Gu.real, Gd.real
            o = obs_fn(m.lat, m.K, Gu, Gd, m.U, beta=m.beta)
            worst = max(worst, float(np.abs(o["nk"] - ref["nk"][b]).max()))
            chi = (m.beta / m.N) * (ref["N2"][b].real - m.N ** 2)
            worst = max(worst, abs(o["chi_e"] - chi) / max(1.0, abs(chi)))
            want = {"D": ref["D"][b].real, "ekin": ref["H0"][b].real / m.N,
                    "e": ref["H0"][b].real / m.N + m.U * ref["D"][b].real,
                    "Szz_G": ref["SzzG"][b].real, "Szz_dk": ref["Szzdk"][b].real,
                    "m2": ref["SzzG"][b].real / (2 * m.Nc),
                    "Rm2": (1.0 - ref["Szzdk"][b] / ref["SzzG"][b]).real}
            for k, v in want.items():
                worst = max(worst, abs(o[k] - v) / max(1.0, abs(v)))
    return worst


def test_reference_is_real_and_uses_both_spins_consistently():
    for m, X in CASES:
        ref = exact.config_estimators(m, X)
        assert np.abs(ref["SzzG"].imag).max() < 1e-12 and np.abs(ref["Szzdk"].imag).max() < 1e-12
        # the independently propagated spin down is the particle-hole partner of spin up
        for b in range(min(4, len(X))):
            assert np.abs(ref["Gdn"][b] - g_down_from_up(ref["Gup"][b], m.Nc)).max() < 1e-11


def test_observables_match_per_configuration_reference():
    assert _violations(observables) < 1e-12


def test_observables_match_per_configuration_reference_charge_channel():
    # HS-n: G_dn = G_up for every configuration (same B for both spins)
    for m, X in CHARGE_CASES:
        ref = exact.config_estimators(m, X[:4])
        assert np.abs(ref["Gdn"] - ref["Gup"]).max() == 0.0
    assert _violations(observables, cases=CHARGE_CASES) < 1e-12


def _mutant(old, new):
    src = textwrap.dedent(inspect.getsource(observables))
    assert old in src, old
    ns = dict(vars(odq))
    exec(compile(src.replace(old, new), "<planted>", "exec"), ns)
    return ns["observables"]


@pytest.mark.parametrize("old,new", [
    ("ph[None, :]", "ph[:, None]"),                                  # phase along d2 instead of d1
    ("2j * np.pi * np.arange(L) / L", "4j * np.pi * np.arange(L) / L"),  # momentum 2 b1/L
    ("(I - Gu.T) * Gu", "0.0 * Gu"),                                 # exchange term of spin up dropped
    ("Czz /= 2 * Nc", "Czz /= Nc"),                                  # normalisation
    ("-(np.trace(K @ Gu)", "+(np.trace(K @ Gu)"),                    # sign of the hopping energy
    ("np.trace(G) - np.trace(G @ G)", "np.trace(G)"),                # pair term of chi_e dropped
])
def test_planted_mistakes_fail_the_pin(old, new):
    assert _violations(_mutant(old, new)) > 1e-6


def _mutant_nk(old, new):
    from oracle import dqmc
    src = textwrap.dedent(inspect.getsource(dqmc.momentum_distribution))
    assert old in src, old
    ns = dict(vars(odq))
    exec(compile(src.replace(old, new), "<planted>", "exec"), ns)
    planted = ns["momentum_distribution"]

    def obs(lat, K, Gu, Gd, U, beta=None):
        o = observables(lat, K, Gu, Gd, U, beta=beta)
        o["nk"] = planted(lat, Gu, Gd)
        return o
    return obs


@pytest.mark.parametrize("old,new", [
    ("G[b * Nc:(b + 1) * Nc, a * Nc:(a + 1) * Nc]", "G[a * Nc:(a + 1) * Nc, b * Nc:(b + 1) * Nc]"),  # block G_ab
    ("t = np.fft.fft2(t, axes=(0, 1))", "t = np.fft.ifft2(t, axes=(0, 1)) * Nc"),  # n(-k) for n(k)
    ("(1.0 if a == b else 0.0) - diag / Nc", "- diag / Nc"),                       # delta term dropped
])
def test_planted_momentum_distribution_mistakes_fail_the_pin(old, new):
    assert _violations(_mutant_nk(old, new)) > 1e-6
