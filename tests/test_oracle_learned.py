"""Pins of the learned-move oracle (oracle/pnet.py) against what the
mathematics fixes: finite differences of the loss, the index convention of a
single-tap convolution written out with explicit loops, translation
equivariance, normalisation and sampling law of the Plackett-Luce proposal,
the block determinant ratio against brute-force weights det(1 + B..B), the
block update against a recomputation of G, and detailed balance of the
Metropolis-Hastings move computed from brute-force weights."""
import itertools

import numpy as np
import pytest

import workloads
from oracle import pnet
from oracle.dqmc import Chain
from oracle.exact import tiny_model


def _params(seed=3, gain=1.0):
    return pnet.unpack(workloads.net_weights(seed, gain=gain))


def test_parameter_count():
    assert pnet.N_PARAMS == 27 * 32 * 2 + 32 + 27 * 32 * 32 + 32 + 27 * 2 * 32 + 2
    assert workloads.net_weights(1).size == pnet.N_PARAMS


def test_loss_gradient_matches_central_differences():
    L, T, B = 2, 3, 2
    p = _params(5, gain=1.5)
    xs = np.stack([workloads.random_fields(10 + b, T, 2 * L * L) for b in range(B)])
    tg = workloads.net_targets(7, (B, T, 2 * L * L))
    _, g = pnet.loss_and_grad(p, xs, tg, L)
    flat = pnet.pack(p)
    rng = np.random.default_rng(0)
    idx = list(rng.choice(flat.size, 40, replace=False)) + list(range(flat.size - 2, flat.size))
    h = 1e-5
    for i in idx:
        fp, fm = flat.copy(), flat.copy()
        fp[i] += h
        fm[i] -= h
        fd = (pnet.loss(pnet.unpack(fp), xs, tg, L) - pnet.loss(pnet.unpack(fm), xs, tg, L)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_single_tap_convolution_index_convention():
    # W1 = one-hot at tap (dt, d2, d1) = (+1, 0, -1), out 0 <- in 1 (B sublattice)
    L, T = 3, 4
    p = {name: np.zeros(shp) for name, shp in pnet.SHAPES}
    tap = (1 + 1) * 9 + (0 + 1) * 3 + (-1 + 1)
    p["W1"][tap, 0, 1] = 0.7
    x = workloads.random_fields(2, T, 2 * L * L)
    _, (a0, h1, _) = pnet.forward(p, x, L, cache=True)
    Nc = L * L
    for t in range(T):
        for n2 in range(L):
            for n1 in range(L):
                src = x[(t + 1) % T, Nc + ((n1 - 1) % L) + L * n2]
                assert h1[t, n2, n1, 0] == pytest.approx(np.tanh(0.7 * src), abs=1e-15)
                assert h1[t, n2, n1, 1] == 0.0


def test_logits_are_translation_equivariant():
    L, T = 3, 5
    p = _params(8)
    x = workloads.random_fields(4, T, 2 * L * L)
    z = pnet.forward(p, x, L)
    a = pnet.fields_to_input(x, L)
    a2 = np.roll(a, shift=(2, 1, -1), axis=(0, 1, 2))
    Nc = L * L
    x2 = np.concatenate([a2[..., 0].reshape(T, Nc), a2[..., 1].reshape(T, Nc)], axis=1)
    z2 = pnet.forward(p, x2, L)
    assert np.abs(z2 - np.roll(z, shift=(2, 1, -1), axis=(0, 1, 2))).max() < 1e-12


def test_plackett_luce_is_normalised():
    z = np.array([0.3, -1.2, 2.0, 0.0, 0.7])
    for m in (1, 2, 3):
        tot = sum(np.exp(pnet.log_q(z, S)) for S in itertools.permutations(range(5), m))
        assert tot == pytest.approx(1.0, abs=1e-13)


def test_gumbel_top_m_samples_plackett_luce():
    z = np.array([1.0, -0.5, 0.2, 2.0])
    rng = np.random.default_rng(1)
    n = 60000
    counts = {}
    for _ in range(n):
        S = tuple(pnet.gumbel_top_m(z, rng.random(4), 2))
        counts[S] = counts.get(S, 0) + 1
    for S in itertools.permutations(range(4), 2):
        q = np.exp(pnet.log_q(z, S))
        f = counts.get(S, 0) / n
        assert abs(f - q) < 5 * np.sqrt(q * (1 - q) / n) + 1e-4, (S, f, q)


def test_philox_gumbel_uniforms_are_open_and_distinct():
    u = pnet.gumbel_uniforms(9, 0, 1, 3, 2, 64)
    assert np.all(u > 0) and np.all(u < 1) and len(set(u)) == 64
    assert 0 <= pnet.accept_uniform(9, 0, 1, 3, 2) < 1


@pytest.mark.parametrize("theta", [(0.0, 0.0), (0.9, 2.3)])
def test_block_ratio_matches_brute_force_weights(theta):
    m = tiny_model(U=3.8, dtau=0.25, M=2, theta1=theta[0], theta2=theta[1])
    x = workloads.random_fields(5, m.M, m.N)
    l = 2
    S = [6, 1, 3]
    d0 = m.weight_dets(x)
    xp = x.copy()
    xp[l - 1, S] = -xp[l - 1, S]
    d1 = m.weight_dets(xp)
    W0 = (d0[0] * d0[1]).real
    W1 = (d1[0] * d1[1]).real
    ch = Chain(m, x)
    for k in range(1, l + 1):
        ch.wrap_up(k)
    R = 1.0 + 0j
    for s in (0, 1):
        det, _ = pnet.block_ratio(ch.G[s], S, x[l - 1, S], m.lam, s)
        R *= det
    assert abs(R.imag) < 1e-10 * abs(R)
    assert R.real == pytest.approx(W1 / W0, rel=1e-10)


def test_block_update_matches_recomputation():
    m = tiny_model(U=3.8, dtau=0.25, M=2, theta1=0.4, theta2=1.1)
    x = workloads.random_fields(6, m.M, m.N)
    l = 1
    S = [2, 7, 4, 0]
    ch = Chain(m, x)
    ch.wrap_up(l)
    xp = x.copy()
    xp[l - 1, S] = -xp[l - 1, S]
    for s in (0, 1):
        _, dl = pnet.block_ratio(ch.G[s], S, x[l - 1, S], m.lam, s)
        Gn = pnet.block_update(ch.G[s], S, dl)
        assert np.abs(Gn - m.green_scratch(xp, l, s)).max() < 1e-10


def test_learned_move_satisfies_detailed_balance():
    """W(X) q(S|X) a(X->X') = W(X') q(S|X') a(X'->X), with W from the
    brute-force determinants and a = min(1, R q(S|X')/q(S|X))."""
    m = tiny_model(U=4.0, dtau=0.25, M=2)
    p = _params(11, gain=2.0)
    L = m.lat.L
    x = workloads.random_fields(12, m.M, m.N)
    l = 2
    S = [5, 0]
    xp = x.copy()
    xp[l - 1, S] = -xp[l - 1, S]

    def weight(f):
        d = m.weight_dets(f)
        return (d[0] * d[1]).real

    def ratio(f):
        G = [m.green_scratch(f, l, s) for s in (0, 1)]
        R = 1.0 + 0j
        for s in (0, 1):
            det, _ = pnet.block_ratio(G[s], S, f[l - 1, S], m.lam, s)
            R *= det
        return R.real

    lq = pnet.log_q(pnet.proposal_logits(p, x, L, l), S)
    lqp = pnet.log_q(pnet.proposal_logits(p, xp, L, l), S)
    a_fwd = min(1.0, ratio(x) * np.exp(lqp - lq))
    a_bwd = min(1.0, ratio(xp) * np.exp(lq - lqp))
    lhs = weight(x) * np.exp(lq) * a_fwd
    rhs = weight(xp) * np.exp(lqp) * a_bwd
    assert lhs == pytest.approx(rhs, rel=1e-10)
    assert abs(lq - lqp) > 1e-3   # the proposal really is asymmetric here


def test_window_loss_gradient_matches_central_differences():
    L, B = 2, 2
    p = _params(6, gain=1.5)
    wins = np.stack([workloads.random_fields(40 + b, 7, 2 * L * L) for b in range(B)])
    tg = workloads.net_targets(9, (B, 2 * L * L))
    _, g = pnet.window_loss_and_grad(p, wins, tg, L)
    flat = pnet.pack(p)
    rng = np.random.default_rng(2)
    idx = list(rng.choice(flat.size, 30, replace=False)) + [flat.size - 1]
    h = 1e-5

    def f(v):
        return pnet.loss(pnet.unpack(v), wins, tg[:, None, :], L, slices=[3])
    for i in idx:
        fp, fm = flat.copy(), flat.copy()
        fp[i] += h
        fm[i] -= h
        fd = (f(fp) - f(fm)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_centre_logits_of_a_window_equal_the_full_configuration():
    # the centre slice of a 7-slice window sees exactly its receptive field
    L, M = 3, 11
    p = _params(4)
    x = workloads.random_fields(3, M, 2 * L * L)
    l = 2
    rows = [(l - 1 + a - 3) % M for a in range(7)]
    zw = pnet.logits(p, x[rows], L)[3]
    assert np.abs(zw - pnet.slice_logits(p, x, L, l)).max() < 1e-12


def test_collected_targets_are_post_decision_acceptances():
    from oracle.dqmc import BitSource
    m = tiny_model(U=3.8, dtau=0.25, M=4)
    x = workloads.random_fields(8, m.M, m.N)
    bits = workloads.accept_bits(9, 2 * m.M * m.N, 0.5)
    ch = Chain(m, x, collect_every=2)
    ch.sweep(BitSource(bits), measure=False)
    assert [c[0] for c in ch.collected] == [4, 2]
    R = np.array(ch.ratios[m.M * m.N:])            # downward pass, slices M..1
    b = bits[m.M * m.N:]
    Rt = np.where(b == 1, 1.0 / R, R)        # ratio of flipping back after the decision
    a = Rt / (1.0 + Rt)
    for k, l in enumerate(range(m.M, 0, -1)):
        assert np.allclose(ch.targets[l - 1], a[k * m.N:(k + 1) * m.N], rtol=1e-15, atol=0)
    l, win, tg = ch.collected[0]
    assert np.array_equal(tg, ch.targets[l - 1])
    assert win.shape == (7, m.N)


def test_log_sigmoid_is_stable_and_exact():
    y = np.array([-800.0, -30.0, -1.0, 0.0, 2.5, 40.0, 800.0])
    ref = np.array([-800.0, -30.0 - np.log1p(np.exp(-30.0)), -np.log1p(np.e), -np.log(2.0),
                    -np.log1p(np.exp(-2.5)), -np.log1p(np.exp(-40.0)), 0.0])
    assert np.allclose(pnet.log_sigmoid(y), ref, rtol=1e-15, atol=1e-300)
