"""Proposal network and learned multi-site move, plain FP64 NumPy.  Test
infrastructure only: the product path never imports this module.

The paper proposes single-site flips only.  The learned move is an
extension whose exactness rests on two things the paper does define:
  * the weight ratio of changing several fields of one slice at once, which
    is the determinant form of eqs. DRatio and rRatioLocal applied to a block
    of sites: with Delta^s = diag(exp(-2 s lambda x_i) - 1) on the set S,
        R_S = prod_s det(1_m + Delta^s_S (1 - G^s)_{SS}),
    and the matching block Sherman-Morrison update of G (the m-site form of
    eq. GupdateLocal),
        G' = G - G[:, S] Delta_S (1_m + (1 - G)_{SS} Delta_S)^{-1} (1 - G)[S, :];
  * the Metropolis-Hastings rule (eq. DetailBalance generalised to an
    asymmetric proposal): accept with min(1, R_S q(S | X') / q(S | X)).

Network (not in the paper).  Input: the fields of every slice on the cell
grid, channels (x_A, x_B) per cell.  Three periodic 3x3x3 convolutions over
(slice, n2, n1), widths 2 -> 32 -> 32 -> 2, tanh after the first two, bias
everywhere.  Output channel 0 is the logit of the A site of the cell,
channel 1 of the B site.  Tap index (dt+1)*9 + (d2+1)*3 + (d1+1): output
(t, n2, n1) reads input (t+dt, n2+d2, n1+d1), all periodic.  Weights are
stored [tap][out channel][in channel]; the flat parameter vector is
W1 (27x32x2), b1 (32), W2 (27x32x32), b2 (32), W3 (27x2x32), b3 (2).

Training loss: mean binary cross-entropy between sigmoid(y_i) of the
network output y_i and a target a_i in [0, 1] (the Barker acceptance
Rt/(1+Rt) of a single flip, recorded by the sampler), over all sites and
slices of the batch.

Proposal: an ordered set S = (s_1..s_m) of distinct sites of slice l drawn
from the Plackett-Luce distribution of the weights w_i = sigmoid(y_i), i.e.
of the logits z_i = log sigmoid(y_i),
    q(S | X) = prod_j exp(z_{s_j}) / sum_{i not in s_1..s_{j-1}} exp(z_i),
sampled as the m largest z_i + g_i (Gumbel-top-m, Gumbel noise
g = -log(-log u)).  A network that predicts y = log Rt turns this into the
locally balanced (Barker) informed proposal.  Uniforms: Philox4x32-10 with key (seed lo, seed hi) and
counter (site, slice, sweep, 4 + 4 move + pass) for the Gumbel noise of a
site, (0xffffffff, slice, sweep, 4 + 4 move + pass) for the acceptance.  The
acceptance uniform is the usual 53-bit k 2^-53, k = w0 2^21 + (w1 >> 11); the
Gumbel uniform is the open-interval value (floor(k / 2) + 1/2) 2^-52, exact in
double precision and never 0 or 1.
"""
import numpy as np

from .philox import MASK, philox4x32_10, u53

CH = 32
TAPS = [(dt, d2, d1) for dt in (-1, 0, 1) for d2 in (-1, 0, 1) for d1 in (-1, 0, 1)]
SHAPES = [("W1", (27, CH, 2)), ("b1", (CH,)), ("W2", (27, CH, CH)), ("b2", (CH,)),
          ("W3", (27, 2, CH)), ("b3", (2,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(flat):
    flat = np.asarray(flat, dtype=np.float64).ravel()
    if flat.size != N_PARAMS:
        raise ValueError("expected %d parameters" % N_PARAMS)
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = flat[o:o + n].reshape(shp).copy()
        o += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def fields_to_input(x, L):
    """x: (T, N) fields +-1 -> (T, L, L, 2) with [t, n2, n1, sub] = x[t, sub*Nc + n1 + L n2]."""
    x = np.asarray(x, dtype=np.float64)
    T = x.shape[0]
    Nc = L * L
    a = np.empty((T, L, L, 2))
    a[..., 0] = x[:, :Nc].reshape(T, L, L)
    a[..., 1] = x[:, Nc:].reshape(T, L, L)
    return a


def output_to_sites(z):
    """(T, L, L, 2) -> (T, N) in site order (A cells, then B cells)."""
    T, L = z.shape[0], z.shape[1]
    return np.concatenate([z[..., 0].reshape(T, L * L), z[..., 1].reshape(T, L * L)], axis=1)


def _shift(a, dt, d2, d1):
    # result[t, n2, n1] = a[t+dt, n2+d2, n1+d1] (periodic)
    return np.roll(a, shift=(-dt, -d2, -d1), axis=(0, 1, 2))


def conv(a, W, b):
    """out[t, n2, n1, co] = b[co] + sum_tap sum_ci W[tap, co, ci] a[t+dt, n2+d2, n1+d1, ci]."""
    out = np.zeros(a.shape[:3] + (W.shape[1],)) + b
    for tap, (dt, d2, d1) in enumerate(TAPS):
        out += _shift(a, dt, d2, d1) @ W[tap].T
    return out


def conv_backward(a, W, dout):
    """Gradients of conv w.r.t. its input a and weights W, given dout."""
    dW = np.zeros_like(W)
    da = np.zeros_like(a)
    Ci, Co = W.shape[2], W.shape[1]
    g = dout.reshape(-1, Co)
    for tap, (dt, d2, d1) in enumerate(TAPS):
        sa = _shift(a, dt, d2, d1)
        dW[tap] = g.T @ sa.reshape(-1, Ci)
        # d out / d a[p] where p = q + d: shift dout back
        da += _shift(dout @ W[tap], -dt, -d2, -d1)
    db = g.sum(axis=0)
    return da, dW, db


def forward(p, x, L, cache=False):
    a0 = fields_to_input(x, L)
    h1 = np.tanh(conv(a0, p["W1"], p["b1"]))
    h2 = np.tanh(conv(h1, p["W2"], p["b2"]))
    z = conv(h2, p["W3"], p["b3"])
    if cache:
        return z, (a0, h1, h2)
    return z


def logits(p, x, L):
    """Logits of every site of every slice, (T, N)."""
    return output_to_sites(forward(p, x, L))


def slice_logits(p, x, L, l):
    """Network outputs y of the N sites of slice l (1-based) of the configuration x (M, N)."""
    return logits(p, x, L)[l - 1]


def log_sigmoid(y):
    y = np.asarray(y, dtype=np.float64)
    return np.where(y >= 0, -np.log1p(np.exp(-np.abs(y))), y - np.log1p(np.exp(-np.abs(y))))


def proposal_logits(p, x, L, l):
    """Plackett-Luce logits z = log sigmoid(y) of the sites of slice l."""
    return log_sigmoid(slice_logits(p, x, L, l))


def bce(z, a):
    """Binary cross-entropy of sigmoid(z) against a, elementwise, stable form."""
    return np.maximum(z, 0.0) - a * z + np.log1p(np.exp(-np.abs(z)))


def loss_and_grad(p, xs, targets, L, slices=None):
    """Mean BCE over a batch of configurations xs (B, T, N) with targets
    (B, T, N); returns (loss, flat gradient).  With slices (a list of slice
    indices) the targets are (B, len(slices), N) and only those slices'
    logits enter the loss."""
    xs = np.asarray(xs)
    targets = np.asarray(targets, dtype=np.float64)
    B = xs.shape[0]
    count = targets.size
    tot = 0.0
    grads = {name: np.zeros(shp) for name, shp in SHAPES}
    for b in range(B):
        z, (a0, h1, h2) = forward(p, xs[b], L, cache=True)
        zs = output_to_sites(z)
        tb = targets[b]
        if slices is not None:
            full = np.full(zs.shape, np.nan)
            full[list(slices)] = tb
            tb = full
        live = ~np.isnan(tb)
        tot += bce(zs[live], tb[live]).sum()
        dzs = np.where(live, 1.0 / (1.0 + np.exp(-zs)) - np.nan_to_num(tb), 0.0) / count
        T = zs.shape[0]
        Nc = L * L
        dz = np.empty_like(z)
        dz[..., 0] = dzs[:, :Nc].reshape(T, L, L)
        dz[..., 1] = dzs[:, Nc:].reshape(T, L, L)
        dh2, dW3, db3 = conv_backward(h2, p["W3"], dz)
        dp2 = dh2 * (1.0 - h2 ** 2)
        dh1, dW2, db2 = conv_backward(h1, p["W2"], dp2)
        dp1 = dh1 * (1.0 - h1 ** 2)
        _, dW1, db1 = conv_backward(a0, p["W1"], dp1)
        for name, g in (("W1", dW1), ("b1", db1), ("W2", dW2), ("b2", db2), ("W3", dW3), ("b3", db3)):
            grads[name] += g
    return tot / count, pack(grads)


def loss(p, xs, targets, L, slices=None):
    xs = np.asarray(xs)
    targets = np.asarray(targets, dtype=np.float64)
    tot = 0.0
    for b in range(xs.shape[0]):
        z = logits(p, xs[b], L)
        if slices is not None:
            z = z[list(slices)]
        tot += bce(z, targets[b]).sum()
    return tot / targets.size


WINDOW = 7      # slices l-3 .. l+3 around the proposal slice; its logits depend on no other slice


def window_loss_and_grad(p, wins, targets, L):
    """Loss and gradient for 7-slice windows (B, 7, N) with targets of the
    centre slice (B, N)."""
    t = np.asarray(targets, dtype=np.float64)[:, None, :]
    return loss_and_grad(p, wins, t, L, slices=[3])


# ---- Plackett-Luce proposal ---------------------------------------------------------
def log_q(z, S):
    """log q(S | X) of the ordered tuple S under logits z (all N sites)."""
    z = np.asarray(z, dtype=np.float64)
    zmax = z.max()
    w = np.exp(z - zmax)
    tot = w.sum()
    out = 0.0
    for s in S:
        out += (z[s] - zmax) - np.log(tot)
        tot -= w[s]
    return out


def move_counter(move, pas):
    return 4 + 4 * int(move) + int(pas)


def gumbel_uniforms(seed, sweep, pas, l, move, N):
    seed = int(seed)
    key = (seed & MASK, (seed >> 32) & MASK)
    c3 = move_counter(move, pas)
    out = np.empty(N)
    for i in range(N):
        w = philox4x32_10((i, l, sweep, c3), key)
        k = (w[0] << 21) + (w[1] >> 11)
        out[i] = ((k >> 1) + 0.5) * (1.0 / 4503599627370496.0)
    return out


def accept_uniform(seed, sweep, pas, l, move):
    seed = int(seed)
    w = philox4x32_10((MASK, l, sweep, move_counter(move, pas)), (seed & MASK, (seed >> 32) & MASK))
    return u53(w[0], w[1])


def gumbel_top_m(z, u, m):
    """The m largest z_i - log(-log u_i), largest first (ties: lower index first)."""
    key = np.asarray(z, dtype=np.float64) - np.log(-np.log(u))
    order = sorted(range(len(key)), key=lambda i: (-key[i], i))
    return order[:m]


# ---- the block ratio and update -----------------------------------------------------
def block_ratio(G, S, x, lam, spin):
    """det(1_m + Delta_S (1 - G)_{SS}) for spin s (s_up = +1, s_dn = -1)."""
    S = list(S)
    sgn = 1.0 if spin == 0 else -1.0
    dl = np.exp(-2.0 * sgn * lam * np.asarray(x, dtype=np.float64)) - 1.0
    m = len(S)
    A = np.eye(m) + dl[:, None] * (np.eye(m) - G[np.ix_(S, S)])
    return np.linalg.det(A), dl


def block_update(G, S, dl):
    S = list(S)
    m = len(S)
    Gs = G[np.ix_(S, S)]
    inner = np.linalg.inv(np.eye(m) + (np.eye(m) - Gs) * dl[None, :])
    left = G[:, S] * dl[None, :]
    right = -G[S, :].copy()
    right[np.arange(m), S] += 1.0
    return G - left @ inner @ right


class LearnedMoves:
    """Learned m-site moves applied after the single-site updates of every
    slice visit: per_slice moves, each drawing S with Gumbel-top-m on the
    slice's logits and accepting with min(1, R_S q(S|X') / q(S|X))."""

    def __init__(self, params, per_slice, m, seed):
        self.p = params if isinstance(params, dict) else unpack(params)
        self.per_slice = int(per_slice)
        self.m = int(m)
        self.seed = int(seed)
        self.proposals = 0
        self.accepted = 0

    def apply(self, chain, l, pas):
        mdl = chain.m
        L, N = mdl.lat.L, mdl.N
        for j in range(self.per_slice):
            z = proposal_logits(self.p, chain.fields, L, l)
            u = gumbel_uniforms(self.seed, chain.sweep_index, pas, l, j, N)
            S = gumbel_top_m(z, u, self.m)
            lq = log_q(z, S)
            x = chain.fields[l - 1, S].astype(np.float64)
            dets, dls = [], []
            for s in (0, 1):
                dt_, dl = block_ratio(chain.G[s], S, x, mdl.lam, s)
                dets.append(dt_)
                dls.append(dl)
            R = (dets[0] * dets[1]).real
            xp = chain.fields.copy()
            xp[l - 1, S] = -xp[l - 1, S]
            lq2 = log_q(proposal_logits(self.p, xp, L, l), S)
            ua = accept_uniform(self.seed, chain.sweep_index, pas, l, j)
            self.proposals += 1
            if ua < R * np.exp(lq2 - lq):
                for s in (0, 1):
                    chain.G[s] = block_update(chain.G[s], S, dls[s])
                chain.fields = xp
                self.accepted += 1
