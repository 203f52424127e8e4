"""Seeded synthetic inputs and the workload shapes, shared by the tests, the
benchmark and the CPU oracle's timing leg.  This module holds no part of the
method's arithmetic: only sizes, seeds and random draws.

Workload shapes follow the paper's simulations (beta t = L, U near U_c,
L up to 42, Sec. III-IV) at dtau = 0.1 and a stabilisation interval of 10:

  plain_L3     L=3  (N=18),   U=3.8,  beta=3,  k=8,  PBC, FP64 real
  plain_L12    L=12 (N=288),  U=3.7,  beta=12, k=32, PBC, FP64 real, 4 chains
  twist_L18    L=18 (N=648),  U=3.73, beta=18, complex128, twists on a 4x4 grid
               of (Theta1, Theta2) in [0, 2pi)^2, 4 chains per twist, plus 16
               L=12 instances (beta=12) in the same batch
  mixed_L30    L=30 (N=1800), U=3.73, beta=30, twist (0.3 pi, 0.7 pi), k=64
  plain_L42    L=42 (N=3528), U=3.73, beta=42, PBC, FP64 real (plain_L42x4: four chains)
"""
import math

import numpy as np

TWO_PI = 2.0 * math.pi


def random_fields(seed, M, N):
    """HS fields x_{l,i} = +-1 with probability 1/2 each, shape (M, N), int8."""
    rng = np.random.default_rng(int(seed))
    return (2 * rng.integers(0, 2, size=(M, N), dtype=np.int8) - 1).astype(np.int8)


def accept_bits(seed, n, p=0.4):
    """Replay stream: one uint8 per proposal, 1 with probability p."""
    rng = np.random.default_rng(int(seed))
    return (rng.random(n) < p).astype(np.uint8)


def twist_grid(n=4):
    """(Theta1, Theta2) = (2 pi a / n, 2 pi b / n), a, b = 0..n-1."""
    return [(TWO_PI * a / n, TWO_PI * b / n) for b in range(n) for a in range(n)]


def desc(L, U, beta, dtau=0.1, theta=(0.0, 0.0), k=None, n_stab=10, seed=1,
         precision=0, sym_measure=0, t=1.0, channel=0):
    N = 2 * L * L
    if k is None:
        k = max(8, int(round(math.sqrt(N))))
    return {"L": L, "t": t, "U": U, "beta": beta, "dtau": dtau,
            "theta1": float(theta[0]), "theta2": float(theta[1]),
            "n_delay": int(k), "n_stab": int(n_stab), "precision": int(precision),
            "sym_measure": int(sym_measure), "seed": int(seed), "channel": int(channel)}


def plain_L3(seed=1):
    return [desc(3, 3.8, 3.0, k=8, seed=seed)]


def plain_L3_chains(n_chains):
    """n independent chains of the plain L=3 shape, seeds 1..n."""
    return [desc(3, 3.8, 3.0, k=8, seed=s) for s in range(1, n_chains + 1)]


def plain_L12(n_chains=4):
    return [desc(12, 3.7, 12.0, k=32, seed=s) for s in range(1, n_chains + 1)]


def twist_L18(chains_per_twist=4, n_grid=4, n_small=16, k=None):
    out = []
    seed = 1
    for th in twist_grid(n_grid):
        for _ in range(chains_per_twist):
            out.append(desc(18, 3.73, 18.0, theta=th, k=k, seed=seed))
            seed += 1
    grid = twist_grid(n_grid)
    for j in range(n_small):
        out.append(desc(12, 3.73, 12.0, theta=grid[j % len(grid)], k=k, seed=101 + j))
    return out


def mixed_L30(precision=1, n_stab=10):
    return [desc(30, 3.73, 30.0, theta=(0.3 * math.pi, 0.7 * math.pi), k=64, precision=precision, n_stab=n_stab)]


def plain_L42(n_chains=1):
    return [desc(42, 3.73, 42.0, k=64, seed=1 + i) for i in range(n_chains)]


# The paper's Table III/IV points used for a physics pin (PBC, HS in the spin
# channel, beta t = L, dtau = 0.05, symmetric Trotter measurement).
def table_point(L, U=3.75, seed=1):
    return desc(L, U, float(L), dtau=0.05, sym_measure=1, seed=seed)


# ---- proposal network inputs (random weights of the layout [tap][out][in]) ----------
NET_SHAPES = [(27, 32, 2), (32,), (27, 32, 32), (32,), (27, 2, 32), (2,)]


def net_weights(seed, gain=1.0, bias=0.1):
    """Flat parameter vector W1, b1, W2, b2, W3, b3 with N(0, gain^2 / fan_in)
    weights and N(0, bias^2) biases."""
    rng = np.random.default_rng(int(seed))
    out = []
    for shp in NET_SHAPES:
        if len(shp) == 3:
            fan = shp[0] * shp[2]
            out.append(rng.standard_normal(shp).ravel() * gain / math.sqrt(fan))
        else:
            out.append(rng.standard_normal(shp) * bias)
    return np.concatenate(out)


def net_targets(seed, shape):
    """Targets in [0, 1] for loss/gradient checks."""
    rng = np.random.default_rng(int(seed))
    return rng.random(shape)
