"""GPU (HIP path, through the C ABI) against the CPU oracle on the same
seeded inputs.  FP64 tolerances: single kernels 1e-13 (relative to the
largest entry), whole sweeps in replay mode 1e-10 (max |dG|)."""
import numpy as np
import pytest

import workloads
from oracle.dqmc import BitSource, Chain, Model, PhiloxSource, observables

pytestmark = pytest.mark.gpu


def _sim(descs):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_14668_amd import Simulation
    return Simulation(descs)


def _model(d):
    return Model(d["L"], d["U"], d["beta"], d["dtau"], t=d["t"], theta1=d["theta1"], theta2=d["theta2"],
                 n_stab=d["n_stab"])


def _rand_g(N, cx, seed):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((N, N))
    if cx:
        G = G + 1j * rng.standard_normal((N, N))
    return G


@pytest.mark.parametrize("L,th", [(3, (0, 0)), (4, (0, 0)), (6, (0.0, 0.0)), (12, (0, 0)), (4, (0.7, 2.1)),
                                  (6, (np.pi / 2, np.pi)), (5, (0.3, 0.0)), (14, (0.0, 0.0)),
                                  (30, (0.3 * np.pi, 0.7 * np.pi)), (42, (0.0, 0.0))])
def test_wrap_matches_dense_propagation(L, th):
    d = workloads.desc(L, 3.7, 1.0, theta=th, n_stab=5)
    sim = _sim([d])
    m = _model(d)
    N, M, cx = sim.shapes[0]
    f = sim.fields(0)
    for direction, sl in ((0, 1), (1, 3), (0, M)):
        G = _rand_g(N, cx, L + sl)
        sim.set_green(0, G)
        sim.wrap(direction, sl)
        out = sim.green(0)
        B, Bi = m.B(0, f[sl - 1]), m.Binv(0, f[sl - 1])
        ref = B @ G @ Bi if direction == 0 else Bi @ G @ B
        assert np.abs(out - ref).max() / np.abs(ref).max() < 1e-13


@pytest.mark.parametrize("kernel", [0, 1, 2])
@pytest.mark.parametrize("L,th,k", [(3, (0, 0), 8), (12, (0, 0), 32), (12, (0, 0), 96), (4, (0.5, 1.0), 16),
                                    (9, (0.2, 0.9), 64), (42, (0, 0), 64), (18, (0.4, 2.0), 45)])
def test_flush_matches_numpy(L, th, k, kernel):
    d = workloads.desc(L, 3.7, 1.0, theta=th, n_stab=5, k=min(k, 192))
    sim = _sim([d])
    sim.set_flush_kernel(kernel)
    N, _, cx = sim.shapes[0]
    G = _rand_g(N, cx, 1)
    X = _rand_g(N, cx, 2)[:, :k] if k <= N else np.vstack([_rand_g(N, cx, 2)] * 1)[:, :k]
    Y = _rand_g(N, cx, 3)[:k, :]
    kk = X.shape[1]
    Y = Y[:kk]
    sim.set_green(0, G)
    sim.flush_test(0, X, Y)
    ref = G - X @ Y
    assert np.abs(sim.green(0) - ref).max() / np.abs(ref).max() < 1e-13


@pytest.mark.parametrize("L,th,beta", [(3, (0, 0), 3.0), (4, (0.6, 1.3), 2.0), (6, (0, 0), 2.0), (12, (0.4, 1.9), 1.0),
                                         (42, (0, 0), 1.0)])
def test_initial_green_matches_oracle(L, th, beta):
    d = workloads.desc(L, 3.8, beta, theta=th, n_stab=5 if L > 20 else 10)
    sim = _sim([d])
    f = sim.fields(0)
    m = _model(d)
    ref = m.green_scratch(f, 0, 0)
    assert np.abs(sim.green(0) - ref).max() < 1e-10
    refd = m.green_scratch(f, 0, 1)
    assert np.abs(sim.green(0, spin=1) - refd).max() < 1e-10


def _replay_case(d, seed, p=0.4, sweeps=1, measure=False, y_solver=1, expand=0, scheme=0):
    import torch
    sim = _sim([d])
    sim.set_y_solver(y_solver)
    sim.set_expand_kernel(expand)
    sim.set_update_scheme(scheme)
    m = _model(d)
    N, M, cx = sim.shapes[0]
    f0 = workloads.random_fields(seed, M, N)
    sim.set_fields(0, f0)
    bits = workloads.accept_bits(seed + 1, sweeps * 2 * M * N, p)
    tb = torch.from_numpy(bits).reshape(1, -1).cuda()
    ratios = torch.zeros((1, bits.size), dtype=torch.float64, device="cuda")
    sim.replay(tb, ratios, n_sweeps=sweeps, measure=measure)
    ch = Chain(m, f0, sym_measure=bool(d["sym_measure"]))
    src = BitSource(bits)
    for _ in range(sweeps):
        ch.sweep(src, measure=measure)
    return sim, ch, ratios.cpu().numpy().ravel()


@pytest.mark.parametrize("y_solver", [1, 0])
@pytest.mark.parametrize("L,th,beta,k", [(3, (0, 0), 3.0, 8), (4, (0.7, 2.2), 2.0, 16), (6, (0, 0), 2.0, 24)])
def test_replay_sweep_matches_oracle(L, th, beta, k, y_solver):
    """Both ways of applying Y^{-1} in the recomputations (pivoted LU, the
    default, and Householder QR) reproduce the oracle's chain."""
    d = workloads.desc(L, 3.8, beta, theta=th, k=k, n_stab=10)
    sim, ch, ratios = _replay_case(d, 11, y_solver=y_solver)
    assert np.array_equal(sim.fields(0), ch.fields)
    assert np.abs(sim.green(0) - ch.G[0]).max() < 1e-10
    assert np.abs(sim.green(0, spin=1) - ch.G[1]).max() < 1e-10
    assert np.abs(ratios - np.array(ch.ratios)).max() / np.abs(ch.ratios).max() < 1e-10
    st = sim.stats(0)
    assert st["accepted"] == ch.accepted and st["proposals"] == ch.proposals
    assert st["drift_max"] < 1e-8


def test_replay_measurements_match_oracle():
    d = workloads.desc(3, 3.8, 3.0, k=8, n_stab=10, sym_measure=1)
    sim, ch, _ = _replay_case(d, 21, measure=True, sweeps=2)
    o = sim.measure(0)
    assert o["n_meas"] == len(ch.samples)
    for key, okey in (("D", "D"), ("ekin", "ekin"), ("e", "e"), ("Szz_G", "Szz_G"), ("Szz_dk", "Szz_dk"),
                      ("m2", "m2"), ("n", "n"), ("chi_e", "chi_e")):
        ref = np.mean([s[okey] for s in ch.samples])
        assert abs(o[key] - ref) < 1e-10, key


def test_philox_chain_matches_oracle():
    d = workloads.desc(3, 3.8, 3.0, k=8, n_stab=10, seed=77)
    sim = _sim([d])
    m = _model(d)
    f0 = sim.fields(0)
    sim.sweep(1, measure=False)
    ch = Chain(m, f0)
    ch.sweep(PhiloxSource(77), measure=False)
    assert np.array_equal(sim.fields(0), ch.fields)
    assert np.abs(sim.green(0) - ch.G[0]).max() < 1e-10


@pytest.mark.parametrize("expand", [1, 0])
@pytest.mark.parametrize("L,th,k", [(4, (0.7, 2.2), 16), (12, (0.0, 0.0), 128), (12, (0.4, 1.9), 96)])
def test_replay_expand_kernels_match_oracle(L, th, k, expand):
    """Both ways of forming the window's delayed vectors (matrix form and
    recursion, eq. DelayRgenk) reproduce the oracle's chain; at k = 96 and
    128 on L = 12 (five windows per slice) windows start with pending terms
    from earlier windows of the slice."""
    d = workloads.desc(L, 3.7, 1.0, theta=th, k=k, n_stab=10)
    sim, ch, ratios = _replay_case(d, 61, p=0.3, expand=expand)
    assert np.array_equal(sim.fields(0), ch.fields)
    assert np.abs(sim.green(0) - ch.G[0]).max() < 1e-10
    assert np.abs(ratios - np.array(ch.ratios)).max() / np.abs(ch.ratios).max() < 1e-10
    st = sim.stats(0)
    assert st["accepted"] == ch.accepted
    if k >= 96:   # windows of ~19 accepted flips accumulate: most windows start with pending terms
        assert st["accepted"] / st["flushes"] > 40


@pytest.mark.parametrize("L,th,beta,k", [(3, (0, 0), 3.0, 8), (4, (0.7, 2.2), 2.0, 16), (6, (0, 0), 2.0, 24),
                                        (12, (0.4, 1.9), 1.0, 32)])
def test_replay_submatrix_update_matches_oracle(L, th, beta, k):
    """The submatrix update (each window's accepted flips as one block
    Sherman-Morrison update) reproduces the oracle's sequential chain:
    fields, G, every ratio and the counters; with measurements."""
    d = workloads.desc(L, 3.8, beta, theta=th, k=k, n_stab=10)
    sim, ch, ratios = _replay_case(d, 71, scheme=1, sweeps=2, measure=True)
    assert np.array_equal(sim.fields(0), ch.fields)
    assert np.abs(sim.green(0) - ch.G[0]).max() < 1e-10
    assert np.abs(ratios - np.array(ch.ratios)).max() / np.abs(ch.ratios).max() < 1e-10
    st = sim.stats(0)
    assert st["accepted"] == ch.accepted and st["proposals"] == ch.proposals
    assert st["drift_max"] < 1e-8
    o = sim.measure(0)
    for key in ("D", "ekin", "e", "Szz_G", "Szz_dk", "m2", "chi_e"):
        ref = np.mean([x[key] for x in ch.samples])
        assert abs(o[key] - ref) < 1e-10, key


def test_submatrix_update_keeps_the_chain():
    """Philox chains (no replay): the delayed and the submatrix update take the
    same decisions on a twisted uneven batch."""
    import torch
    descs = [workloads.desc(4, 3.7, 2.0, theta=(0.3, 1.1), k=16, seed=5),
             workloads.desc(6, 3.7, 2.0, k=24, seed=6)]
    out = []
    for scheme in (0, 1):
        sim = _sim(descs)
        sim.set_update_scheme(scheme)
        sim.sweep(2, measure=False)
        torch.cuda.synchronize()
        out.append(([sim.fields(i) for i in range(2)], [sim.green(i) for i in range(2)]))
    for i in range(2):
        assert np.array_equal(out[0][0][i], out[1][0][i])
        assert np.abs(out[0][1][i] - out[1][1][i]).max() < 1e-10


def test_replay_larger_lattice():
    d = workloads.desc(12, 3.7, 1.0, k=32, n_stab=10)
    sim, ch, _ = _replay_case(d, 31, p=0.3)
    assert np.array_equal(sim.fields(0), ch.fields)
    assert np.abs(sim.green(0) - ch.G[0]).max() < 1e-10


def test_flush_rank_does_not_change_the_chain():
    """The flush rank only regroups the rank-1 terms: the same Philox chain
    with ranks 8 and 100 (set at run time) has identical fields and G to
    FP64 rounding, and the autotuner keeps one of its candidates."""
    d = workloads.desc(4, 3.8, 2.0, theta=(0.4, 1.1), k=8, n_stab=10, seed=91)
    a, b = _sim([d]), _sim([d])
    b.set_delay(100)
    a.sweep(1, measure=False)
    b.sweep(1, measure=False)
    assert np.array_equal(a.fields(0), b.fields(0))
    assert np.abs(a.green(0) - b.green(0)).max() < 1e-10
    best, per = a.autotune([8, 32, 64], 20)
    assert best[0] in (8, 32, 64) and best[1] in (0, 1, 2) and all(v > 0 for v in per.values())
    assert len(per) == 9
    # the tiled and the work-queue flush kernels give the same chain
    for kernel in (1, 2):
        c = _sim([d])
        c.set_flush_kernel(kernel)
        c.sweep(1, measure=False)
        assert np.array_equal(c.fields(0), b.fields(0))
        assert np.abs(c.green(0) - b.green(0)).max() < 1e-10


@pytest.mark.parametrize("groups", [1, 2, 3])
def test_graph_replay_matches_eager(groups):
    """Sweeps replayed from the captured block equal eager sweeps (fields,
    G, estimators), over several replays with eager work in between, with
    with one, two and three instance groups."""
    descs = [workloads.desc(4, 3.8, 2.0, theta=(0.4 * i, 1.1), k=16, n_stab=10, seed=120 + i) for i in range(3)]
    a, b = _sim(descs), _sim(descs)
    a.set_graphs(False)
    for sim in (a, b):
        sim.set_streams(groups)
    for _ in range(3):
        a.sweep(1, measure=True)
        b.sweep(1, measure=True)
        for i in range(3):
            assert a.stats(i)["accepted"] == b.stats(i)["accepted"]
    for i in range(3):
        assert np.array_equal(a.fields(i), b.fields(i))
        assert np.abs(a.green(i) - b.green(i)).max() < 1e-12
        oa, ob = a.measure(i), b.measure(i)
        assert oa["n_meas"] == ob["n_meas"] and abs(oa["D"] - ob["D"]) < 1e-12


def test_instance_groups_do_not_change_the_chain():
    """The chains are independent, so splitting them over one or four
    streams gives the same fields, G and estimators."""
    descs = [workloads.desc(3 + i % 3, 3.8, 2.0, theta=(0.3 * i, 0.9), k=16, n_stab=10, seed=140 + i)
             for i in range(5)]
    a, b = _sim(descs), _sim(descs)
    a.set_streams(1)
    b.set_streams(4)
    for _ in range(2):
        a.sweep(1, measure=True)
        b.sweep(1, measure=True)
    for i in range(5):
        assert np.array_equal(a.fields(i), b.fields(i))
        assert np.abs(a.green(i) - b.green(i)).max() < 1e-12
        assert a.measure(i)["D"] == pytest.approx(b.measure(i)["D"], abs=1e-12)


@pytest.mark.parametrize("kernel", [0, 1, 2])
def test_flush_every_instance_of_an_uneven_batch(kernel):
    """Nine instances (the instance dimension of the grid is padded to 16 and
    the instances are spread unevenly over the XCD slots; the work-queue
    kernel puts instances 0 and 8 in one queue and has eight queues with a
    single active instance at most): a flush on each instance in turn
    matches G - X Y and leaves the others unchanged, also on a second round
    (the queues reset themselves after every launch)."""
    descs = [workloads.desc(3 + (i % 3) * 3, 3.7, 1.0, theta=(0.3 * i, 0.7), n_stab=5, seed=160 + i)
             for i in range(9)]
    sim = _sim(descs)
    sim.set_flush_kernel(kernel)
    cx = sim.shapes[0][2]
    k = 8
    G = [_rand_g(sim.shapes[i][0], cx, 200 + i) for i in range(9)]
    for i in range(9):
        sim.set_green(i, G[i])
    for rnd in range(2):
        for i in range(9):
            N = sim.shapes[i][0]
            X = _rand_g(N, cx, 300 + i + 10 * rnd)[:, :k]
            Y = _rand_g(N, cx, 400 + i + 10 * rnd)[:k, :]
            sim.flush_test(i, X, Y)
            G[i] = G[i] - X @ Y
            for j in range(9):
                assert np.abs(sim.green(j) - G[j]).max() / np.abs(G[j]).max() < 1e-13, (rnd, i, j)
