"""Plain dense FP64 DQMC for the honeycomb Hubbard model, HS in the spin-s^z
channel or in the charge channel, written from the paper's formalism.  Test
infrastructure only.

What is computed, and where it is defined:
  * spin channel (HS-s^z, eq. SzHS): lambda = gamma_s = arccosh(exp(dtau U/2))
    (eq. coupling), B^sigma_l = exp(s_sigma lambda diag(x_l)) exp(-dtau K),
    s_up = +1, s_dn = -1, p(x_l) = 2^{-N_s}      (eqs. BIOpSz, ConfgWeight)
  * charge channel (HS-n, eq. DensityHS): gamma_c = i alpha with
    alpha = arccos(exp(-dtau U/2)) (eq. coupling), the same
    B_l = exp(i alpha diag(x_l)) exp(-dtau K) for both spins (eq. BIOpnT),
    p(x_l) = (exp(dtau U N_s/2) / 2^{N_s}) exp(-i alpha sum_i x_{l,i})
  * G^sigma(l) = (1 + B_l..B_1 B_M..B_{l+1})^{-1}                (eq. GrFMat)
    recomputed with a UDV chain over chunks of n_stab slices using pivoted
    Householder QR (the periodic QR stabilisation of Sec. II B), with the
    usual split of D into factors >= 1 and <= 1 before the inversion.
  * wraps G -> B_l G B_l^{-1} (upward) and G -> B_l^{-1} G B_l (downward),
    with dense exp(-+dtau K) from an eigendecomposition of K   (Sec. III A)
  * single-site Metropolis: Delta^sigma = v_sigma(-x)/v_sigma(x) - 1 with
    v_sigma the diagonal of exp(H_I^sigma), r_sigma = 1 + Delta^sigma
    (1 - G^sigma_ii), accept if u < R = [p(x')/p(x)] r_up r_dn, the prior
    ratio being 1 (spin) or exp(2 i alpha x) (charge; R is real and positive
    up to rounding)                            (eqs. DetailBalance, rRatioLocal)
  * Sherman-Morrison G' = G - x y^T with x = G[:, i] Delta / r and
    y^T = (1 - G)[i, :]                                    (eq. GupdateLocal)
  * both spins are propagated independently: no particle-hole shortcut.
  * a sweep is the upward pass l = 1..M (wrap, then update slice l) followed
    by the downward pass l = M..1 (update slice l, then wrap); sites are
    visited in the order 0..N_s-1 (A sublattice first).   (Sec. III A-B)

Readings of points the paper leaves open (each is listed in the design doc):
  * stabilisation (G replaced by its recomputation) after slice l when
    l % n_stab == 0 in the upward pass and when the downward wrap reaches
    l-1 with (l-1) % n_stab == 0;
  * measurements are taken on the recomputed G at those points, optionally on
    the symmetric-split G~ = exp(-dtau K/2) G exp(+dtau K/2);
  * the acceptance test is u < R with u in [0, 1).
"""
import numpy as np
import scipy.linalg as sla

from .lattice import Lattice


def hs_lambda(U, dtau):
    """gamma_s = arccosh(exp(dtau U / 2))   (eq. coupling)."""
    return float(np.arccosh(np.exp(dtau * U / 2.0)))


def hs_alpha(U, dtau):
    """alpha = arccos(exp(-dtau U / 2)), gamma_c = i alpha   (eq. coupling)."""
    return float(np.arccos(np.exp(-dtau * U / 2.0)))


CHANNELS = ("spin", "charge")


def hermitian_expm(K, c):
    """exp(c K) for Hermitian K via its eigendecomposition."""
    w, V = np.linalg.eigh(K)
    return (V * np.exp(c * w)) @ V.conj().T


class Model:
    """Dense single-particle matrices of one (L, U, beta, dtau, twist) point."""

    def __init__(self, L, U, beta, dtau, t=1.0, theta1=0.0, theta2=0.0,
                 n_stab=10, gauge="I", channel="spin"):
        M = beta / dtau
        if abs(M - round(M)) > 1e-9:
            raise ValueError("beta/dtau must be an integer")
        self.lat = Lattice(L, t, theta1, theta2)
        self.L, self.N, self.Nc = self.lat.L, self.lat.N, self.lat.Nc
        self.U, self.beta, self.dtau = float(U), float(beta), float(dtau)
        self.M = int(round(M))
        self.n_stab = int(n_stab)
        if channel not in CHANNELS:
            raise ValueError("channel must be 'spin' or 'charge'")
        self.channel = channel
        self.lam = hs_lambda(U, dtau)
        self.alpha = hs_alpha(U, dtau)
        self.K = self.lat.hopping_matrix(gauge)
        self.complex = np.iscomplexobj(self.K) or channel == "charge"
        dt = complex if self.complex else float
        self.Ep = hermitian_expm(self.K, -self.dtau).astype(dt)       # exp(-dtau K)
        self.Em = hermitian_expm(self.K, +self.dtau).astype(dt)       # exp(+dtau K)
        self.Ehp = hermitian_expm(self.K, -self.dtau / 2).astype(dt)  # exp(-dtau K/2)
        self.Ehm = hermitian_expm(self.K, +self.dtau / 2).astype(dt)  # exp(+dtau K/2)
        self.dtype = dt

    @classmethod
    def from_hopping(cls, K, U, beta, dtau, n_stab=1, channel="spin"):
        """A model on an arbitrary small bipartite cluster given by its
        hopping matrix K (sites ordered sublattice A first); only the
        propagators, weights and Green's functions are defined (no lattice)."""
        M = beta / dtau
        if abs(M - round(M)) > 1e-9:
            raise ValueError("beta/dtau must be an integer")
        if channel not in CHANNELS:
            raise ValueError("channel must be 'spin' or 'charge'")
        m = cls.__new__(cls)
        m.lat = None
        m.K = np.array(K)
        m.N = m.K.shape[0]
        m.L, m.Nc = None, m.N // 2
        m.U, m.beta, m.dtau = float(U), float(beta), float(dtau)
        m.M = int(round(M))
        m.n_stab = int(n_stab)
        m.channel = channel
        m.lam = hs_lambda(U, dtau)
        m.alpha = hs_alpha(U, dtau)
        m.complex = np.iscomplexobj(m.K) or channel == "charge"
        dt = complex if m.complex else float
        m.Ep = hermitian_expm(m.K, -m.dtau).astype(dt)
        m.Em = hermitian_expm(m.K, +m.dtau).astype(dt)
        m.Ehp = hermitian_expm(m.K, -m.dtau / 2).astype(dt)
        m.Ehm = hermitian_expm(m.K, +m.dtau / 2).astype(dt)
        m.dtype = dt
        return m

    # ---- propagators ----------------------------------------------------------
    def vdiag(self, spin, x):
        """Diagonal of exp(H_I^sigma(x)): exp(s_sigma lambda x) (spin channel)
        or exp(i alpha x) for both spins (charge channel)."""
        x = np.asarray(x, dtype=float)
        if self.channel == "charge":
            return np.exp(1j * self.alpha * x)
        s = 1.0 if spin == 0 else -1.0
        return np.exp(s * self.lam * x)

    def prior_ratio(self, x):
        """p(x')/p(x) of flipping one field x -> -x: 1 (spin channel) or
        exp(-gamma_c (x' - x)) = exp(2 i alpha x) (charge channel)."""
        if self.channel == "charge":
            return np.exp(2j * self.alpha * float(x))
        return 1.0

    def log_prior(self, fields):
        """log P(X) of a whole configuration (eqs. BIOpSz, BIOpnT)."""
        X = np.asarray(fields, dtype=float)
        nf = X.size
        if self.channel == "charge":
            return nf * (self.dtau * self.U / 2.0 - np.log(2.0)) - 1j * self.alpha * X.sum()
        return -nf * np.log(2.0)

    def B(self, spin, x):
        return self.vdiag(spin, x)[:, None] * self.Ep

    def Binv(self, spin, x):
        return self.Em * (1.0 / self.vdiag(spin, x))[None, :]

    # ---- stabilised Green's function ------------------------------------------
    def green_scratch(self, fields, l, spin):
        """G(l) = (1 + B_l..B_1 B_M..B_{l+1})^{-1} by a UDV chain (eq. GrFMat).

        The cyclic product is built right to left (B_{l+1} first), n_stab
        slices per chunk, each chunk followed by a pivoted QR.
        """
        M, N = self.M, self.N
        order = [((l + j) % M) + 1 for j in range(M)]  # 1-based slice indices
        U = np.eye(N, dtype=self.dtype)
        D = np.ones(N)
        T = np.eye(N, dtype=self.dtype)
        for c0 in range(0, M, self.n_stab):
            A = U * D[None, :]
            for s in order[c0:c0 + self.n_stab]:
                A = self.B(spin, fields[s - 1]) @ A
            Q, R, P = sla.qr(A, pivoting=True)
            d = np.abs(np.diag(R))
            Rs = R / d[:, None]
            RP = np.empty_like(Rs)
            RP[:, P] = Rs                       # Rs P^T
            T = RP @ T
            U, D = Q, d
        return self._inv_one_plus_udt(U, D, T)

    @staticmethod
    def _inv_one_plus_udt(U, D, T):
        """(1 + U D T)^{-1} with D split into Db = max(D,1), Ds = min(D,1):
        1 + UDT = U Db (Db^{-1} U^H T^{-1} + Ds) T."""
        Db = np.maximum(D, 1.0)
        Ds = np.minimum(D, 1.0)
        Tinv = np.linalg.inv(T)
        UH = U.conj().T
        Mid = (UH @ Tinv) / Db[:, None] + np.diag(Ds)
        return Tinv @ np.linalg.solve(Mid, UH / Db[:, None])

    def green_direct(self, fields, l, spin):
        """Unstabilised (1 + B_l..B_1 B_M..B_{l+1})^{-1}; only for short chains."""
        P = np.eye(self.N, dtype=self.dtype)
        for j in range(self.M):
            s = ((l + j) % self.M) + 1
            P = self.B(spin, fields[s - 1]) @ P
        return np.linalg.inv(np.eye(self.N) + P)

    def weight_dets(self, fields):
        """(det(1 + B^up_M..B^up_1), det(1 + B^dn_M..B^dn_1)) without stabilisation."""
        out = []
        for spin in (0, 1):
            P = np.eye(self.N, dtype=complex)
            for l in range(1, self.M + 1):
                P = self.B(spin, fields[l - 1]) @ P
            out.append(np.linalg.det(np.eye(self.N) + P))
        return tuple(out)


# ---- accept sources ------------------------------------------------------------
class BitSource:
    """Replay: the decision for proposal number n is bits[n] (1 = accept)."""

    def __init__(self, bits):
        self.bits = np.asarray(bits, dtype=np.uint8).ravel()
        self.n = 0

    def __call__(self, sweep, pas, l, i, R):
        b = bool(self.bits[self.n])
        self.n += 1
        return b


class PhiloxSource:
    """u from Philox4x32-10 with counter (site, slice, sweep, pass) and the
    64-bit seed as key; accept iff u < R."""

    def __init__(self, seed):
        from .philox import uniform_site
        self.seed = int(seed)
        self._u = uniform_site

    def __call__(self, sweep, pas, l, i, R):
        return self._u(self.seed, sweep, pas, l, i) < R


class RandomSource:
    """Independent-run source backed by NumPy's generator."""

    def __init__(self, seed):
        self.rng = np.random.default_rng(seed)

    def __call__(self, sweep, pas, l, i, R):
        return self.rng.random() < R


# ---- the Markov chain ------------------------------------------------------------
class Chain:
    """One DQMC Markov chain; both spins propagated densely and independently."""

    def __init__(self, model, fields, sym_measure=False, learned=None, collect_every=0):
        self.m = model
        self.learned = learned     # oracle.pnet.LearnedMoves applied after each slice's site updates
        # training data of the proposal network: for every site, the Barker
        # acceptance Rt/(1+Rt) of flipping it again right after its decision in
        # the downward pass (Rt = 1/R after an accepted flip, R after a
        # rejected one), and
        # (every collect_every-th slice l of that pass, l % collect_every == 0)
        # the 7-slice field window l-3 .. l+3 (mod M) with slice l's targets,
        # taken after the slice's single-site updates
        self.targets = np.zeros((model.M, model.N))
        self.collect_every = int(collect_every)
        self.collected = []
        self.fields = np.array(fields, dtype=np.int8).reshape(model.M, model.N).copy()
        if not np.all(np.abs(self.fields) == 1):
            raise ValueError("fields must be +-1")
        self.sym = bool(sym_measure)
        self.sweep_index = 0
        self.G = [model.green_scratch(self.fields, 0, s) for s in (0, 1)]
        self.ratios = []
        self.drift = []
        self.samples = []          # observables at each checkpoint
        self.accepted = 0
        self.proposals = 0

    # wraps (Sec. III A)
    def wrap_up(self, l):
        x = self.fields[l - 1]
        for s in (0, 1):
            v = self.m.vdiag(s, x)
            self.G[s] = v[:, None] * (self.m.Ep @ self.G[s] @ self.m.Em) / v[None, :]

    def wrap_down(self, l):
        x = self.fields[l - 1]
        for s in (0, 1):
            v = self.m.vdiag(s, x)
            self.G[s] = self.m.Em @ ((self.G[s] / v[:, None]) * v[None, :]) @ self.m.Ep

    def site_ratio(self, l, i):
        """Metropolis ratio of flipping x_{l,i} on the current G (eqs.
        DetailBalance, DRatio, rRatioLocal): (R, Delta^sigma, r_sigma)."""
        x = float(self.fields[l - 1, i])
        dl = tuple(complex(self.m.vdiag(s, -x) / self.m.vdiag(s, x)) - 1.0 for s in (0, 1))
        if not self.m.complex:
            dl = tuple(d.real for d in dl)
        r = [1.0 + dl[s] * (1.0 - self.G[s][i, i]) for s in (0, 1)]
        R = (self.m.prior_ratio(x) * r[0] * r[1]).real
        return R, dl, r

    def update_slice(self, l, pas, decide):
        """Sequential single-site Metropolis on slice l (eqs. rRatioLocal, GupdateLocal)."""
        N = self.m.N
        for i in range(N):
            R, dl, r = self.site_ratio(l, i)
            self.ratios.append(R)
            self.proposals += 1
            acc = decide(self.sweep_index, pas, l, i, R)
            if acc:
                for s in (0, 1):
                    G = self.G[s]
                    xv = G[:, i] * (dl[s] / r[s])
                    yv = -G[i, :].copy()
                    yv[i] += 1.0
                    self.G[s] = G - np.outer(xv, yv)
                self.fields[l - 1, i] = -self.fields[l - 1, i]
                self.accepted += 1
            if pas == 1:
                self.targets[l - 1, i] = 1.0 / (1.0 + R) if acc else R / (1.0 + R)
        if pas == 1 and self.collect_every and l % self.collect_every == 0:
            rows = [(l - 1 + a - 3) % self.m.M for a in range(7)]
            self.collected.append((l, self.fields[rows].copy(), self.targets[l - 1].copy()))
        if self.learned is not None:
            self.learned.apply(self, l, pas)

    def stabilise(self, l, measure=True):
        for s in (0, 1):
            Gs = self.m.green_scratch(self.fields, l, s)
            self.drift.append(float(np.max(np.abs(Gs - self.G[s]))))
            self.G[s] = Gs
        if measure:
            self.samples.append(self.measure())

    def sweep(self, decide, measure=True):
        m = self.m
        for l in range(1, m.M + 1):
            self.wrap_up(l)
            self.update_slice(l, 0, decide)
            if l % m.n_stab == 0:
                self.stabilise(l, measure)
        for l in range(m.M, 0, -1):
            self.update_slice(l, 1, decide)
            self.wrap_down(l)
            if (l - 1) % m.n_stab == 0:
                self.stabilise(l - 1, measure)
        self.sweep_index += 1

    def measured_greens(self):
        if not self.sym:
            return self.G
        return [self.m.Ehp @ G @ self.m.Ehm for G in self.G]

    def measure(self):
        Gu, Gd = self.measured_greens()
        return observables(self.m.lat, self.m.K, Gu, Gd, self.m.U, beta=self.m.beta)


def momentum_distribution(lat, Gu, Gd):
    """Spin-averaged 2 x 2 momentum distribution of eq. nkMatrix on the
    instance's momentum grid (plain index k = l1 + L l2; with a twist the
    physical momentum is shifted by the vector potential, eq. kpoints):
        n_ab(k) = (1/N_c) sum_{r,r'} e^{i k.(r - r')} <c^+_{a r} c_{b r'}>,
    <c^+_i c_j> = delta_ij - G_ji, i.e. n_ab(k) = delta_ab - [F G_ba F^dagger]_kk / N_c
    with F the 2-D DFT over the cell grid (numpy fft2 over (n2, n1) on the
    left, inverse on the right).  Returns an array (N_c, 2, 2), [k, a, b]."""
    L, Nc = lat.L, lat.Nc
    out = np.zeros((Nc, 2, 2), dtype=complex)
    for G in (Gu, Gd):
        for a in (0, 1):
            for b in (0, 1):
                blk = np.asarray(G[b * Nc:(b + 1) * Nc, a * Nc:(a + 1) * Nc], dtype=complex)
                t = blk.reshape(L, L, L, L)                  # [n2', n1', n2, n1]
                t = np.fft.fft2(t, axes=(0, 1))              # sum_r' e^{-i k r'}
                t = np.fft.ifft2(t, axes=(2, 3)) * Nc        # sum_r  e^{+i k r}
                diag = np.array([t[l2, l1, l2, l1] for l2 in range(L) for l1 in range(L)])
                out[:, a, b] += (1.0 if a == b else 0.0) - diag / Nc
    return out / 2.0


def nk_bands(nk):
    """Eigenvalues (n_+, n_-) of each Hermitian 2 x 2 n(k) (n_+ >= n_-): n_+
    belongs to the lower band eps_{k,-} and n_- to eps_{k,+} (Sec. II C)."""
    tr = (nk[:, 0, 0] + nk[:, 1, 1]).real
    df = (nk[:, 0, 0] - nk[:, 1, 1]).real
    r = np.sqrt(0.25 * df * df + np.abs(nk[:, 0, 1]) ** 2)
    return 0.5 * tr + r, 0.5 * tr - r


def dirac_points(L):
    """Plain-grid indices (l1, l2) of the two inequivalent Dirac points, where
    f(k) = 0 (K = (2 b1 + b2)/3 and K' = (b1 + 2 b2)/3); on the grid when
    L % 3 == 0, else the nearest grid points."""
    return [(int(round(2 * L / 3)) % L, int(round(L / 3)) % L), (int(round(L / 3)) % L, int(round(2 * L / 3)) % L)]


def gab_dirac(lat, nk):
    """|G_AB(K + dk)| of Sec. IV A: the modulus of the spin-averaged n_AB at
    K + b1/L, averaged over the two inequivalent Dirac points."""
    L = lat.L
    vals = [abs(nk[((l1 + 1) % L) + L * l2, 0, 1]) for (l1, l2) in dirac_points(L)]
    return float(np.mean(vals))


def observables(lat, K, Gu, Gd, U, beta=None):
    """Equal-time estimators for one configuration from G^up, G^dn (Wick).

    <n_is> = 1 - G_ii; <c_i^+ c_j> = delta_ij - G_ji;
    <n_is n_js> = (1-G_ii)(1-G_jj) + (delta_ij - G_ji) G_ij (same spin),
    opposite spins factorise.  D (Sec. II C), E = <H_0> + N_s U D (Sec. IV C),
    C_zz(r) (eq. SzSzCrF), S_zz(k) (eq. SpinStrucF), m^2 and R_m2 (eq. CrfRatio),
    the momentum distribution n(k) (eq. nkMatrix) and, given beta, the
    charge-compressibility estimator of eq. ChiCharge,
    chi = (beta/N_s) Re[(sum_i n_i)^2 + sum_s (Tr G^s - Tr G^s G^s)] - beta N_s,
    whose mean over configurations is (beta/N_s)(<N^2> - <N>^2) at half
    filling, where the real part of sum_i n_i is N_s in every configuration.
    """
    N, Nc, L = lat.N, lat.Nc, lat.L
    nu = 1.0 - np.diag(Gu)
    nd = 1.0 - np.diag(Gd)
    D = np.mean(nu * nd)
    Ekin = -(np.trace(K @ Gu) + np.trace(K @ Gd)) + 2 * np.trace(K)
    ekin = Ekin / N
    I = np.eye(N)
    sz = nu - nd
    SS = 0.25 * (np.outer(sz, sz) + (I - Gu.T) * Gu + (I - Gd.T) * Gd)
    Czz = np.zeros((L, L), dtype=complex)          # index [d2, d1]
    for sub in (0, 1):
        for I0 in range(Nc):
            n1, n2 = I0 % L, I0 // L
            i = sub * Nc + I0
            for d2 in range(L):
                for d1 in range(L):
                    j = sub * Nc + ((n1 + d1) % L) + L * ((n2 + d2) % L)
                    Czz[d2, d1] += SS[i, j]
    Czz /= 2 * Nc
    SzzG = Czz.sum()
    ph = np.exp(2j * np.pi * np.arange(L) / L)     # k = b1/L: e^{i k.r} = e^{2 pi i d1/L}
    Szzdk = (Czz * ph[None, :]).sum()
    m2 = SzzG / (2 * Nc)
    extra = {"nk": momentum_distribution(lat, Gu, Gd)}
    if beta is not None:
        ntot = np.sum(nu + nd)
        c1 = ntot * ntot + sum(np.trace(G) - np.trace(G @ G) for G in (Gu, Gd))
        extra["chi_e"] = float((beta / N) * c1.real - beta * N)
    return {**extra,
        "n": float(np.mean(nu + nd).real),
        "D": float(D.real),
        "ekin": float(ekin.real),
        "e": float((ekin + U * D).real),
        "Szz_G": float(SzzG.real),
        "Szz_dk": float(Szzdk.real),
        "m2": float(m2.real),
        "Rm2": float((1.0 - Szzdk / SzzG).real),
        "Czz": Czz.real.copy(),
    }


def g_down_from_up(Gu, Nc):
    """Particle-hole relation in the original basis: G_dn = P (1 - G_up^H) P with
    P = diag(+1 on A, -1 on B) (the spin-down partner of Sec. II B)."""
    N = Gu.shape[0]
    p = np.ones(N)
    p[Nc:] = -1.0
    return p[:, None] * (np.eye(N) - Gu.conj().T) * p[None, :]
