"""More GPU-vs-oracle parity on the configurations the benchmark runs:
twisted estimators, per-instance symmetric measurement, an uneven batch
replayed instance by instance, a twisted N = 648 sweep, the tracked phase of
det(1 + B..B), the recomputation drift check and multi-chunk network
gradients.

Tolerances as in test_gpu_parity: replayed sweeps max |dG| <= 1e-10, ratios
1e-10 relative, estimators 1e-10 absolute (they are O(1) sums of G entries
with the same rounding).  Phase of det_up: the GPU anchors it at every
recomputation from the Householder factors of the UDV chains (unit-modulus
products of O(N) reflector and pivot phases, each with relative error of a
few eps) and tracks it between recomputations by the phases of the accepted
ratios; 1e-9 leaves room for N eps growth over the chain.
"""
import numpy as np
import pytest

import workloads
from oracle import pnet
from oracle.dqmc import BitSource, Chain, Model, PhiloxSource

pytestmark = pytest.mark.gpu

EST_KEYS = ("n", "D", "ekin", "e", "Szz_G", "Szz_dk", "m2", "chi_e")


def _sim(descs):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_14668_amd import Simulation
    return Simulation(descs)


def _model(d):
    return Model(d["L"], d["U"], d["beta"], d["dtau"], t=d["t"], theta1=d["theta1"], theta2=d["theta2"],
                 n_stab=d["n_stab"])


def _check_estimators(o, samples, tol=1e-10, sim=None, inst=0, lat=None):
    assert o["n_meas"] == len(samples)
    for key in EST_KEYS:
        ref = np.mean([s[key] for s in samples])
        assert abs(o[key] - ref) < tol, (key, o[key], ref)
    rm2 = 1.0 - np.mean([s["Szz_dk"] for s in samples]) / np.mean([s["Szz_G"] for s in samples])
    assert abs(o["Rm2"] - rm2) < tol
    if sim is not None:
        # momentum distribution (eq. nkMatrix): mean of the spin-averaged 2 x 2 n(k)
        from oracle.dqmc import gab_dirac, nk_bands
        nk_ref = np.mean([s["nk"] for s in samples], axis=0)
        nk = sim.nk(inst, raw=True)
        assert np.abs(nk - nk_ref).max() < tol
        assert abs(o["GAB_dirac"] - gab_dirac(lat, nk_ref)) < tol
        herm = 0.5 * (nk_ref + np.conj(np.transpose(nk_ref, (0, 2, 1))))
        npl, nmi = nk_bands(herm)
        d = sim.nk(inst)
        assert np.abs(d["n_plus"] - npl).max() < tol and np.abs(d["n_minus"] - nmi).max() < tol
        assert np.abs(d["eps"] - np.abs(lat.f_of_k(lat.kpoints()))).max() < 1e-12


def _det_phase(model, fields):
    du, _ = model.weight_dets(fields)
    return du / abs(du)


@pytest.mark.parametrize("sym", [0, 1])
def test_replay_twisted_estimators_match_oracle(sym):
    """Twisted L=4 chain (complex G, Peierls-phased Tr(K G)), two replayed
    sweeps with measurements on G or on the half-step G~."""
    import torch
    d = workloads.desc(4, 3.8, 2.0, theta=(0.7, 2.2), k=16, n_stab=10, sym_measure=sym)
    sim = _sim([d])
    m = _model(d)
    N, M, cx = sim.shapes[0]
    assert cx
    f0 = workloads.random_fields(501 + sym, M, N)
    sim.set_fields(0, f0)
    bits = workloads.accept_bits(502 + sym, 2 * 2 * M * N, 0.4)
    sim.replay(torch.from_numpy(bits).reshape(1, -1).cuda(), None, n_sweeps=2, measure=True)
    ch = Chain(m, f0, sym_measure=bool(sym))
    src = BitSource(bits)
    for _ in range(2):
        ch.sweep(src, measure=True)
    assert np.array_equal(sim.fields(0), ch.fields)
    assert np.abs(sim.green(0) - ch.G[0]).max() < 1e-10
    _check_estimators(sim.measure(0), ch.samples, sim=sim, inst=0, lat=m.lat)


def test_instances_choose_their_own_measurement():
    """One handle, two twisted instances, only the second measures on the
    symmetric-split G~: each matches the oracle with its own choice."""
    import torch
    base = dict(L=4, U=3.8, beta=2.0, theta=(0.4, 1.3), k=16, n_stab=10)
    descs = [workloads.desc(sym_measure=0, seed=1, **base), workloads.desc(sym_measure=1, seed=2, **base)]
    sim = _sim(descs)
    N, M, _ = sim.shapes[0]
    fs = [workloads.random_fields(511 + i, M, N) for i in range(2)]
    for i in range(2):
        sim.set_fields(i, fs[i])
    bits = np.stack([workloads.accept_bits(513 + i, 2 * M * N, 0.4) for i in range(2)])
    sim.replay(torch.from_numpy(bits).cuda(), None, n_sweeps=1, measure=True)
    for i in range(2):
        ch = Chain(_model(descs[i]), fs[i], sym_measure=bool(i))
        ch.sweep(BitSource(bits[i]), measure=True)
        assert np.abs(sim.green(i) - ch.G[0]).max() < 1e-10
        _check_estimators(sim.measure(i), ch.samples, sim=sim, inst=i, lat=ch.m.lat)


def test_uneven_batch_replay_matches_oracle():
    """A twisted L=4 chain (beta=2, M=20) and an L=3 chain (beta=3, M=30) in
    one handle with the default instance groups and graphs.  One call runs
    2 * 30 slice steps: the L=3 chain one sweep, the L=4 chain one sweep and
    the upward pass of the next (all instances advance one slice per step).
    Each instance is replayed against its own oracle chain."""
    import torch
    descs = [workloads.desc(4, 3.8, 2.0, theta=(0.7, 2.2), k=16, n_stab=10, seed=5),
             workloads.desc(3, 3.8, 3.0, k=8, n_stab=10, seed=6)]
    sim = _sim(descs)
    sim.set_graphs(True)
    shapes = sim.shapes
    Mmax = max(s[1] for s in shapes)
    fs = [workloads.random_fields(521 + i, shapes[i][1], shapes[i][0]) for i in range(2)]
    for i in range(2):
        sim.set_fields(i, fs[i])
    per = 2 * Mmax * max(s[0] for s in shapes)
    bits = np.stack([workloads.accept_bits(523 + i, per, 0.4) for i in range(2)])
    ratios = torch.zeros((2, per), dtype=torch.float64, device="cuda")
    sim.replay(torch.from_numpy(bits).cuda(), ratios, n_sweeps=1, measure=True)
    ratios = ratios.cpu().numpy()
    for i, d in enumerate(descs):
        N, M, _ = shapes[i]
        m = _model(d)
        ch = Chain(m, fs[i])
        src = BitSource(bits[i])
        steps = 0
        while steps + 2 * M <= 2 * Mmax:
            ch.sweep(src, measure=True)
            steps += 2 * M
        if steps < 2 * Mmax:            # the upward pass of the next sweep
            assert 2 * Mmax - steps == M
            for l in range(1, M + 1):
                ch.wrap_up(l)
                ch.update_slice(l, 0, src)
                if l % m.n_stab == 0:
                    ch.stabilise(l, True)
        assert np.array_equal(sim.fields(i), ch.fields), i
        assert np.abs(sim.green(i) - ch.G[0]).max() < 1e-10, i
        nr = len(ch.ratios)
        assert np.abs(ratios[i, :nr] - np.array(ch.ratios)).max() / np.abs(ch.ratios).max() < 1e-10
        st = sim.stats(i)
        assert st["accepted"] == ch.accepted and st["proposals"] == ch.proposals
        _check_estimators(sim.measure(i), ch.samples, sim=sim, inst=i, lat=m.lat)


def test_replay_twisted_L18_matches_oracle():
    """N = 648 (11 windows per slice, fill carried across windows, the
    register-line FFT at L = 18), twisted, beta = 1 (M = 10): one replayed
    sweep against the oracle."""
    import torch
    d = workloads.desc(18, 3.73, 1.0, theta=(np.pi / 2, np.pi), k=32, n_stab=10, seed=7)
    sim = _sim([d])
    m = _model(d)
    N, M, _ = sim.shapes[0]
    f0 = workloads.random_fields(531, M, N)
    sim.set_fields(0, f0)
    bits = workloads.accept_bits(532, 2 * M * N, 0.4)
    ratios = torch.zeros((1, bits.size), dtype=torch.float64, device="cuda")
    sim.replay(torch.from_numpy(bits).reshape(1, -1).cuda(), ratios, n_sweeps=1, measure=False)
    ch = Chain(m, f0)
    ch.sweep(BitSource(bits), measure=False)
    assert np.array_equal(sim.fields(0), ch.fields)
    err = np.abs(sim.green(0) - ch.G[0]).max()
    print("L=18 replay: max |dG| = %.2e" % err, flush=True)
    assert err < 1e-10
    r = ratios.cpu().numpy().ravel()
    assert np.abs(r - np.array(ch.ratios)).max() / np.abs(ch.ratios).max() < 1e-10
    st = sim.stats(0)
    assert st["accepted"] == ch.accepted and st["proposals"] == ch.proposals


@pytest.mark.parametrize("th", [(0.0, 0.0), (0.7, 2.2)])
def test_tracked_phase_equals_determinant_phase(th):
    """The phase of det(1 + B_M..B_1) of spin up after two Philox sweeps
    equals that of the oracle's unstabilised determinant of the same fields,
    and the tracked phase agreed with the anchored one at every
    recomputation.  Periodic instances are real: the phase is a sign."""
    d = workloads.desc(4, 3.8, 2.0, theta=th, k=16, n_stab=10, seed=9)
    sim = _sim([d])
    m = _model(d)
    p0 = _det_phase(m, sim.fields(0))
    st = sim.stats(0)
    assert abs(complex(st["phase_re"], st["phase_im"]) - p0) < 1e-9
    sim.sweep(2, measure=True)
    st = sim.stats(0)
    p1 = _det_phase(m, sim.fields(0))
    assert abs(complex(st["phase_re"], st["phase_im"]) - p1) < 1e-9
    assert st["phase_drift"] < 1e-9
    o = sim.measure(0)
    assert o["n_meas"] > 0 and abs(complex(o["phase_cos"], o["phase_sin"])) <= 1.0 + 1e-12
    if th == (0.0, 0.0):
        assert abs(st["phase_im"]) < 1e-12 and abs(abs(st["phase_re"]) - 1) < 1e-12


def test_tracked_phase_with_learned_block_moves():
    """Block moves change det_up by the block determinant prod_k r_k; with a
    non-trivial network the tracked phase still agrees with the anchored
    one at every recomputation and with the oracle's determinant."""
    d = workloads.desc(4, 3.8, 2.0, theta=(0.9, 0.3), k=16, n_stab=10, seed=10)
    sim = _sim([d])
    sim.net_set_weights(workloads.net_weights(12, gain=2.0, bias=0.5))
    sim.set_proposals(2, 4)
    sim.sweep(2, measure=False)
    st = sim.stats(0)
    assert st["learn_accepted"] > 0
    assert st["phase_drift"] < 1e-9
    p = _det_phase(_model(d), sim.fields(0))
    assert abs(complex(st["phase_re"], st["phase_im"]) - p) < 1e-9


def test_drift_above_tolerance_is_a_numeric_error():
    """A G perturbed by 1e-2 between recomputations is caught at the next
    one: drift_last ~ 1e-2 > the default tolerance 1e-4 sets numeric_err
    (bit 2) and dqmc_measure / dqmc_get_stats return DQMC_ENUMERIC; an
    intact sweep after dqmc_reset_obs passes, and drift_last is the last
    recomputation's value, not a running maximum."""
    from paper_2609_14668_amd import DqmcError
    d = workloads.desc(4, 3.8, 2.0, theta=(0.4, 1.1), k=16, n_stab=10, seed=11)
    sim = _sim([d])
    sim.sweep(1, measure=True)
    st = sim.stats(0, check=True)
    assert st["numeric_err"] == 0 and st["drift_last"] < 1e-8
    G = sim.green(0)
    sim.set_green(0, G + 1e-2 * np.random.default_rng(1).standard_normal(G.shape))
    sim.sweep(1, measure=True)
    st = sim.stats(0)
    assert st["numeric_err"] & 2
    assert st["drift_max"] > 1e-3
    with pytest.raises(DqmcError) as e:
        sim.measure(0)
    assert e.value.status == -4
    with pytest.raises(DqmcError):
        sim.stats(0, check=True)
    sim.reset_obs()
    sim.sweep(1, measure=True)
    st = sim.stats(0, check=True)
    assert st["numeric_err"] == 0 and st["drift_last"] < 1e-8 and st["drift_max"] < 1e-8


@pytest.mark.parametrize("L,window,M,B", [(18, True, 7, 2), (6, False, 40, 2)])
def test_network_gradient_over_several_chunks(L, window, M, B):
    """Weight gradients are reduced over chunks of 1024 output voxels per
    item: 7-slice windows at L = 18 (1620 voxels in the first layer) and
    whole L = 6, M = 40 configurations (1440 voxels in every layer) take
    more than one chunk."""
    sim = _sim([workloads.desc(3, 3.7, 1.0, n_stab=5)])
    w = workloads.net_weights(15, gain=1.5)
    sim.net_set_weights(w)
    N = 2 * L * L
    xs = np.stack([workloads.random_fields(540 + b, M, N) for b in range(B)])
    if window:
        tg = workloads.net_targets(541, (B, N))
        loss, g = sim.net_grad(xs, tg, L, window=True)
        ref_loss, ref_g = pnet.window_loss_and_grad(pnet.unpack(w), xs, tg, L)
    else:
        tg = workloads.net_targets(542, xs.shape)
        loss, g = sim.net_grad(xs, tg, L)
        ref_loss, ref_g = pnet.loss_and_grad(pnet.unpack(w), xs, tg, L)
    assert abs(loss - ref_loss) <= 1e-2 * abs(ref_loss)
    gp, rp = pnet.unpack(g), pnet.unpack(ref_g)
    for name, _ in pnet.SHAPES:
        rel = np.linalg.norm(gp[name] - rp[name]) / np.linalg.norm(rp[name])
        assert rel < 6e-2, (name, rel)


@pytest.mark.parametrize("L", [12, 18])
def test_every_fft_tile_gives_the_dense_wrap(L):
    """Each register-line tile (wide, narrow, eight vectors per workgroup)
    on both sides equals dense propagation; the tile autotuner keeps one of
    them per (L, side)."""
    d = workloads.desc(L, 3.7, 1.0, theta=(0.4, 1.9), n_stab=5)
    sim = _sim([d])
    m = _model(d)
    N, M, cx = sim.shapes[0]
    f = sim.fields(0)
    rng = np.random.default_rng(L)
    for tile in (0, 1, 2):
        for side in (0, 1):
            sim.set_fft_tile(L, side, tile)
        for direction, sl in ((0, 2), (1, 4)):
            G = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
            sim.set_green(0, G)
            sim.wrap(direction, sl)
            B, Bi = m.B(0, f[sl - 1]), m.Binv(0, f[sl - 1])
            ref = B @ G @ Bi if direction == 0 else Bi @ G @ B
            assert np.abs(sim.green(0) - ref).max() / np.abs(ref).max() < 1e-13, (tile, direction)
    choice, times = sim.autotune_fft(5)
    assert set(choice) == {(L, 0), (L, 1)} and all(t in (0, 1, 2) for t in choice.values())
    assert all(v > 0 for v in times.values())


def test_fft_tiles_do_not_change_the_chain():
    """A sweep with the narrow tile on the columns and eight-vector tiles on
    the rows reproduces the default tiles' chain (fields exactly, G to FP64
    rounding)."""
    d = workloads.desc(12, 3.7, 2.0, theta=(0.4, 1.9), k=32, n_stab=10, seed=77)
    a, b = _sim([d]), _sim([d])
    b.set_fft_tile(12, 0, 1)
    b.set_fft_tile(12, 1, 2)
    a.sweep(1, measure=True)
    b.sweep(1, measure=True)
    assert np.array_equal(a.fields(0), b.fields(0))
    assert np.abs(a.green(0) - b.green(0)).max() < 1e-12
    assert abs(a.measure(0)["D"] - b.measure(0)["D"]) < 1e-12
