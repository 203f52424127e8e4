"""Exact references for tiny systems.  Test infrastructure only.

* U = 0: G = (1 + exp(-beta K))^{-1} block by block in momentum space,
  (1 + exp(-beta h))^{-1} = 1/2 + tanh(beta |f| / 2) h / (2 |f|), with h(k) of
  eq. h0kMat at the shifted grid of eq. kpoints and the Fourier matrix
  U_{k,r} = exp(-i k.r)/L of eq. NewBlMat; energy per site
  e = -(1/N_c) sum_k |f(k)| tanh(beta |f(k)| / 2); D = 1/4.
* Brute force: Z = sum_X W(X), W = P(X) det(1 + B^up_M..B^up_1)
  det(1 + B^dn_M..B^dn_1) over every HS configuration (eq. ConfgWeight), in
  either HS channel (P(X) = 2^{-N M} for HS-s^z; for HS-n the prefactor and
  the phase exp(-gamma_c sum x) of eq. BIOpnT), with estimators taken on
  G(l = M).  Both channels represent the same Trotterised partition function,
  so both must reproduce the exact diagonalisation below.
* Exact diagonalisation of the Trotterised partition function
  Tr[(exp(-dtau H_U) exp(-dtau H_0))^M] in the 4^N-dimensional Fock space
  for M in {1, 2}, H_U = U sum_i (n_up n_dn - (n_up + n_dn)/2)
  (eq. HubbModel).  Observables are inserted at the left end of the product.
"""
import itertools

import numpy as np

from .dqmc import Model
from .lattice import Lattice


# ---- U = 0 --------------------------------------------------------------------------
def fourier_matrix(lat):
    """Per-sublattice unitary DFT on the plain grid, U_{k,r} = exp(-i k.r)/L."""
    L, Nc = lat.L, lat.Nc
    Uc = np.zeros((Nc, Nc), dtype=complex)
    for kI in range(Nc):
        l1, l2 = kI % L, kI // L
        for rI in range(Nc):
            n1, n2 = rI % L, rI // L
            Uc[kI, rI] = np.exp(-2j * np.pi * (l1 * n1 + l2 * n2) / L) / L
    Z = np.zeros_like(Uc)
    return np.block([[Uc, Z], [Z, Uc]])


def kspace_block_matrix(lat, fn):
    """Assemble U^dagger Lambda U where Lambda is block diagonal with the 2x2
    block fn(h(k+A)) at plain momentum index k (A enters through f(k+A))."""
    Nc = lat.Nc
    f = lat.f_of_k(lat.kpoints())
    Lam = np.zeros((lat.N, lat.N), dtype=complex)
    for kI in range(Nc):
        h = np.array([[0.0, f[kI]], [np.conj(f[kI]), 0.0]])
        blk = fn(h, f[kI])
        Lam[kI, kI] = blk[0, 0]
        Lam[kI, Nc + kI] = blk[0, 1]
        Lam[Nc + kI, kI] = blk[1, 0]
        Lam[Nc + kI, Nc + kI] = blk[1, 1]
    Uf = fourier_matrix(lat)
    return Uf.conj().T @ Lam @ Uf


def exp_h_closed(h, f, c):
    """exp(c h) for h = [[0,f],[f*,0]]: cosh(c|f|) 1 + sinh(c|f|)/|f| h."""
    a = abs(f)
    s = c if a < 1e-12 else np.sinh(c * a) / a
    return np.cosh(c * a) * np.eye(2) + s * h


def green_u0(lat, beta):
    def g(h, f):
        a = abs(f)
        if a < 1e-14:
            return 0.5 * np.eye(2)
        return 0.5 * np.eye(2) + np.tanh(beta * a / 2) * h / (2 * a)
    return kspace_block_matrix(lat, g)


def energy_u0(lat, beta):
    f = np.abs(lat.f_of_k(lat.kpoints()))
    return -np.sum(f * np.tanh(beta * f / 2)) / lat.Nc


def bands_u0(lat, beta):
    """Free-fermion band occupations on the instance's grid: the lower band
    eps_- = -|f| holds n_+ = 1/(1 + e^{-beta |f|}), the upper band n_- =
    1/(1 + e^{+beta |f|})."""
    f = np.abs(lat.f_of_k(lat.kpoints()))
    return 1.0 / (1.0 + np.exp(-beta * f)), 1.0 / (1.0 + np.exp(beta * f))


def chi_e_u0(lat, beta):
    """(beta/N_s)(<N^2> - <N>^2) of free fermions: every single-particle level
    of either spin contributes its occupation variance n(1 - n)."""
    npl, nmi = bands_u0(lat, beta)
    return (beta / lat.N) * 2.0 * np.sum(npl * (1 - npl) + nmi * (1 - nmi))


# ---- brute force over HS configurations ---------------------------------------------
def config_estimators(model, X):
    """Per-configuration weights and Wick estimators for a batch of HS
    configurations X (B x M x N, entries +-1): both spins propagated densely,
    G^sigma = (1 + B^sigma_M..B^sigma_1)^{-1} (G at l = M), and for each
    configuration W = 2^{-N M} det(1 + B^up..) det(1 + B^dn..)
    (eq. ConfgWeight) together with D, <H_0> = Tr(K G^up) + Tr(K G^dn) summed
    with the sign of a hopping term (c_i^+ c_j -> -G_ji), and
    S_zz(k) = (1/2N_c) sum_sub sum_ij e^{-i k r_i} e^{+i k r_j} <s_i s_j> at
    k = 0 and k = b1/L (eqs. SzSzCrF, SpinStrucF) from the contraction of
    the whole same-sublattice block with plane waves."""
    M, N, Nc, L = model.M, model.N, model.Nc, model.L
    X = np.asarray(X, dtype=float).reshape(-1, M, N)
    K = model.K
    pos = np.array([[I % L, I // L] for I in range(Nc)])
    ph = np.exp(2j * np.pi * pos[:, 0] / L)
    B = len(X)
    dets, Gs = [], []
    for spin in (0, 1):
        P = np.broadcast_to(np.eye(N, dtype=complex), (B, N, N)).copy()
        for l in range(M):
            v = model.vdiag(spin, X[:, l, :])
            P = v[:, :, None] * (model.Ep[None] @ P)
        A = np.eye(N)[None] + P
        dets.append(np.linalg.det(A))
        Gs.append(np.linalg.inv(A))
    W = dets[0] * dets[1] * np.exp(np.array([model.log_prior(x) for x in X]))
    nu = 1 - np.einsum("bii->bi", Gs[0])
    nd = 1 - np.einsum("bii->bi", Gs[1])
    D = np.mean(nu * nd, axis=1)
    H0 = -(np.einsum("ij,bji->b", K, Gs[0]) + np.einsum("ij,bji->b", K, Gs[1]))
    sz = nu - nd
    SS = 0.25 * (sz[:, :, None] * sz[:, None, :]
                 + (np.eye(N)[None] - np.transpose(Gs[0], (0, 2, 1))) * Gs[0]
                 + (np.eye(N)[None] - np.transpose(Gs[1], (0, 2, 1))) * Gs[1])
    SzzG = np.zeros(B, dtype=complex)
    Szzdk = np.zeros(B, dtype=complex)
    for sub in (0, 1):
        blk = SS[:, sub * Nc:(sub + 1) * Nc, sub * Nc:(sub + 1) * Nc]
        SzzG += blk.sum(axis=(1, 2))
        Szzdk += np.einsum("bij,i,j->b", blk, ph.conj(), ph)
    SzzG /= 2 * Nc
    Szzdk /= 2 * Nc
    # one-body density matrices rho_ij = <c_i^+ c_j> = delta_ij - G_ji, the
    # momentum distribution n_ab(k) = (1/N_c) sum_{r,r'} e^{i k (r - r')}
    # rho_{a r, b r'} (spin average) by explicit Fourier sums with the
    # unitary U_{k,r} = e^{-i k.r}/L, and the Wick value of N_tot^2 summed
    # pair by pair
    Uc = fourier_matrix(model.lat)[:Nc, :Nc]
    rhos = [np.eye(N)[None] - np.transpose(G, (0, 2, 1)) for G in Gs]
    nk = np.zeros((B, Nc, 2, 2), dtype=complex)
    for rho in rhos:
        for a in (0, 1):
            for b2 in (0, 1):
                blk = rho[:, a * Nc:(a + 1) * Nc, b2 * Nc:(b2 + 1) * Nc]
                m = np.einsum("kr,brs,ks->bk", Uc.conj(), blk, Uc)
                nk[:, :, a, b2] += 0.5 * m
    N2 = np.zeros(B, dtype=complex)
    occ = [np.einsum("bii->bi", rho) for rho in rhos]
    for s1 in (0, 1):
        for s2 in (0, 1):
            if s1 == s2:
                rho = rhos[s1]
                N2 += np.einsum("bi,bj->b", occ[s1], occ[s1]) + np.einsum(
                    "bij,bij->b", rho, np.eye(N)[None] - np.transpose(rho, (0, 2, 1)))
            else:
                N2 += occ[s1].sum(axis=1) * occ[s2].sum(axis=1)
    return {"W": W, "D": D, "H0": H0, "SzzG": SzzG, "Szzdk": Szzdk, "Gup": Gs[0], "Gdn": Gs[1],
            "nk": nk, "Ntot": sum(o.sum(axis=1) for o in occ), "N2": N2}


def brute_force(model, batch=4096):
    """Exact Z and weighted averages of D, <H_0>, S_zz(Gamma), S_zz(b1/L) by
    summing W(X) over all 2^(N M) configurations (eq. ConfgWeight)."""
    M, N = model.M, model.N
    nf = M * N
    if nf > 20:
        raise ValueError("too many fields for brute force")
    tot = {"Z": 0.0, "D": 0.0, "H0": 0.0, "SzzG": 0.0, "Szzdk": 0.0, "N2": 0.0, "Ntot": 0.0}
    nk_sum = 0.0
    wmin = np.inf
    max_imag = 0.0
    allcfg = np.array(list(itertools.product((1, -1), repeat=nf)), dtype=float)
    for s0 in range(0, len(allcfg), batch):
        c = config_estimators(model, allcfg[s0:s0 + batch])
        W = c["W"]
        max_imag = max(max_imag, float(np.max(np.abs(W.imag) / np.abs(W))))
        W = W.real
        wmin = min(wmin, float(W.min()))
        tot["Z"] += W.sum()
        for k in ("D", "H0", "SzzG", "Szzdk", "N2", "Ntot"):
            tot[k] += (W * c[k]).sum().real
        nk_sum = nk_sum + np.einsum("b,bkxy->kxy", W, c["nk"])
    Z = tot["Z"]
    return {"Z": Z, "D": tot["D"] / Z, "H0": tot["H0"] / Z, "SzzG": tot["SzzG"] / Z,
            "Szzdk": tot["Szzdk"] / Z, "N2": tot["N2"] / Z, "Ntot": tot["Ntot"] / Z, "nk": nk_sum / Z,
            "wmin": wmin, "w_max_rel_imag": max_imag}


# ---- Fock-space exact diagonalisation ------------------------------------------------
def fock_hopping(K):
    """Many-body matrix of sum_ij K_ij c_i^+ c_j on one spin species
    (Jordan-Wigner ordering of modes 0..N-1; state bit i = occupation of i)."""
    N = K.shape[0]
    dim = 1 << N
    H = np.zeros((dim, dim), dtype=complex)
    for a in range(dim):
        for j in range(N):
            if not (a >> j) & 1:
                continue
            sj = (-1) ** bin(a & ((1 << j) - 1)).count("1")
            a1 = a ^ (1 << j)
            for i in range(N):
                if K[i, j] == 0:
                    continue
                if (a1 >> i) & 1:
                    continue
                si = (-1) ** bin(a1 & ((1 << i) - 1)).count("1")
                H[a1 | (1 << i), a] += K[i, j] * sj * si
    return H


def exact_trotter(model):
    """Z = Tr[T^M], T = exp(-dtau H_U) exp(-dtau H_0) and <O> = Tr[O T^M]/Z for
    O in {D, H_0, S_zz(Gamma), S_zz(b1/L)}; M in {1, 2}."""
    M, N, Nc, L = model.M, model.N, model.Nc, model.L
    if M not in (1, 2):
        raise ValueError("exact_trotter supports M = 1 or 2")
    dim = 1 << N
    H = fock_hopping(model.K)
    w, V = np.linalg.eigh(H)
    E = (V * np.exp(-model.dtau * w)) @ V.conj().T
    occ = np.array([[(a >> i) & 1 for i in range(N)] for a in range(dim)], dtype=float)
    nn = occ @ occ.T                                   # sum_i n_i(a) n_i(b)
    ntot = occ.sum(axis=1)
    HU = model.U * (nn - (ntot[:, None] + ntot[None, :]) / 2.0)
    Dm = np.exp(-model.dtau * HU)                      # [a_up, b_dn]
    Docc = nn / N
    pos = np.array([[I % L, I // L] for I in range(Nc)])
    ph = np.exp(2j * np.pi * pos[:, 0] / L)
    SG = np.zeros((dim, dim))
    Sdk = np.zeros((dim, dim))
    for sub in (0, 1):
        oa = occ[:, sub * Nc:(sub + 1) * Nc]
        s = 0.5 * (oa[:, None, :] - oa[None, :, :])    # s^z_i for state (a, b)
        SG += np.sum(s, axis=2) ** 2
        Sdk += np.abs(np.sum(s * ph[None, None, :], axis=2)) ** 2
    SG /= 2 * Nc
    Sdk /= 2 * Nc
    EH = E @ H
    if M == 1:
        dE = np.diag(E)
        dEH = np.diag(EH)

        def tr(O, left_up=False, left_dn=False):
            eu = dEH if left_up else dE
            ed = dEH if left_dn else dE
            return np.einsum("ab,a,b->", O * Dm, eu, ed)
    else:
        P = E * E.T
        Pt = E * EH.T

        def tr(O, left_up=False, left_dn=False):
            pu = Pt if left_up else P
            pd = Pt if left_dn else P
            return np.sum(pu * ((O * Dm) @ pd @ Dm.T))
    one = np.ones((dim, dim))
    Z = tr(one)
    Ntot = ntot[:, None] + ntot[None, :]

    def tr_onebody(Oop, spin):
        """Tr[O T^M] / Z for a one-body Fock operator O acting on one species."""
        EO = E @ Oop
        if M == 1:
            eo, e = np.diag(EO), np.diag(E)
            return np.einsum("ab,a,b->", Dm, eo if spin == 0 else e, e if spin == 0 else eo) / Z
        Po = E * EO.T
        return np.sum((Po if spin == 0 else P) * (Dm @ (P if spin == 0 else Po) @ Dm.T)) / Z

    # one-body density matrix <c^+_i c_j> of each spin from the Fock operators c^+_i c_j
    rho = np.zeros((2, N, N), dtype=complex)
    for i in range(N):
        for j in range(N):
            Kij = np.zeros((N, N))
            Kij[i, j] = 1.0
            Op = fock_hopping(Kij)
            for spin in (0, 1):
                rho[spin, i, j] = tr_onebody(Op, spin)
    return {"Z": Z.real, "D": (tr(Docc) / Z).real,
            "H0": ((tr(one, left_up=True) + tr(one, left_dn=True)) / Z).real,
            "SzzG": (tr(SG) / Z).real, "Szzdk": (tr(Sdk) / Z).real,
            "N2": (tr(Ntot * Ntot) / Z).real, "Ntot": (tr(Ntot) / Z).real, "rho": rho}


# ---- time-displaced references (Sec. II C, eqs. DouOccDerive, fidelitysusp) -----------
def fock_annihilators(n_modes):
    """Jordan-Wigner annihilation operators of n_modes fermion modes (bit k of
    a basis index = occupation of mode k)."""
    dim = 1 << n_modes
    ops = []
    for k in range(n_modes):
        c = np.zeros((dim, dim))
        for a in range(dim):
            if (a >> k) & 1:
                c[a ^ (1 << k), a] = (-1) ** bin(a & ((1 << k) - 1)).count("1")
        ops.append(c)
    return ops


def exact_tau_fock(K, U, dtau, M):
    """Full Fock-space evaluation (both spins, 4^N states; N <= 4) of the
    Trotterised ensemble Tr[T^M], T = exp(-dtau H_U) exp(-dtau H_0),
    H_0 = sum_sigma sum_ij K_ij c^+_i c_j, H_U = U sum_i (n_up n_dn - (n_up + n_dn)/2):
    <A(tau_l) A(0)> = Tr[T^{M-l} A T^l A] / Z for l = 0..M, <A>, the double
    occupancy D and <N>; A = sum_i (n_up,i - 1/2)(n_dn,i - 1/2)."""
    K = np.asarray(K)
    N = K.shape[0]
    if N > 4:
        raise ValueError("at most 4 sites")
    c = fock_annihilators(2 * N)            # modes 0..N-1 spin up, N..2N-1 spin down
    cd = [x.T for x in c]
    n = [cd[k] @ c[k] for k in range(2 * N)]
    H0 = sum(K[i, j] * (cd[i] @ c[j] + cd[N + i] @ c[N + j]) for i in range(N) for j in range(N))
    nud = [n[i] @ n[N + i] for i in range(N)]
    HU = U * sum(nud[i] - 0.5 * (n[i] + n[N + i]) for i in range(N))
    A = sum((n[i] - 0.5 * np.eye(len(H0))) @ (n[N + i] - 0.5 * np.eye(len(H0))) for i in range(N))
    w, V = np.linalg.eigh(H0)
    E0 = (V * np.exp(-dtau * w)) @ V.conj().T
    T = np.diag(np.exp(-dtau * np.diag(HU))) @ E0
    Tp = [np.eye(len(T))]
    for _ in range(M):
        Tp.append(Tp[-1] @ T)
    Z = np.trace(Tp[M])
    AA = np.array([np.trace(Tp[M - l] @ A @ Tp[l] @ A) / Z for l in range(M + 1)])
    return {"Z": Z.real, "AA": AA.real, "A": (np.trace(A @ Tp[M]) / Z).real,
            "D": (np.trace(sum(nud) @ Tp[M]) / Z).real / N,
            "Ntot": (np.trace(sum(n) @ Tp[M]) / Z).real, "max_imag": float(np.max(np.abs(AA.imag)))}


def exact_tau_trotter2(model):
    """<A(tau_l) A(0)> for l = 0, 1 and <A> of an M = 2 model on the honeycomb
    torus (N up to 8), with the Fock space as (spin-up state, spin-down state)
    pairs: T = D_U o (E x E), so Tr[T X T Y] = sum P[a,c] (D_U X)[a,b] P[b,d]
    (D_U Y)[c,d] with P = E o E^T for diagonal X, Y."""
    if model.M != 2:
        raise ValueError("M = 2 only")
    N = model.N
    dim = 1 << N
    H = fock_hopping(model.K)
    w, V = np.linalg.eigh(H)
    E = (V * np.exp(-model.dtau * w)) @ V.conj().T
    occ = np.array([[(a >> i) & 1 for i in range(N)] for a in range(dim)], dtype=float)
    nn = occ @ occ.T
    ntot = occ.sum(axis=1)
    Dm = np.exp(-model.dtau * model.U * (nn - (ntot[:, None] + ntot[None, :]) / 2.0))
    mm = occ - 0.5
    A = mm @ mm.T                                     # sum_i m_up,i(a) m_dn,i(b)
    P = E * E.T

    def tr2(X, Y):
        return np.sum(P * ((Dm * X) @ P @ (Dm * Y).T))

    one = np.ones((dim, dim))
    Z = tr2(one, one)
    return {"Z": Z.real, "AA": np.array([(tr2(A * A, one) / Z).real, (tr2(A, A) / Z).real]),
            "A": (tr2(A, one) / Z).real}


def brute_force_tau(model, lmax, batch=2048):
    """Exact weighted averages over every HS configuration of the oracle's
    per-configuration <A(tau_l) A(0)>_X (l = 0..lmax) and <A>_X, with
    W = P(X) det O_up det O_dn (eq. ConfgWeight)."""
    from .tau import tau_correlator
    M, N = model.M, model.N
    nf = M * N
    if nf > 24:
        raise ValueError("too many fields for brute force")
    Z = 0.0
    aa = np.zeros(lmax + 1, dtype=complex)
    a1 = 0.0 + 0.0j
    wmin = np.inf
    allcfg = np.array(list(itertools.product((1, -1), repeat=nf)), dtype=float).reshape(-1, M, N)
    for s0 in range(0, len(allcfg), batch):
        X = allcfg[s0:s0 + batch]
        W = np.exp(np.array([model.log_prior(x) for x in X]))
        for spin in (0, 1):
            P = np.broadcast_to(np.eye(N, dtype=complex), (len(X), N, N)).copy()
            for l in range(M):
                P = model.vdiag(spin, X[:, l, :])[:, :, None] * (model.Ep[None] @ P)
            W = W * np.linalg.det(np.eye(N)[None] + P)
        AA, At = tau_correlator(model, X, lmax)
        wmin = min(wmin, float(np.min(W.real)))
        Z += W.sum().real
        aa += W @ AA
        a1 += W @ At[:, 0]
    return {"Z": Z, "AA": (aa / Z).real, "A": (a1 / Z).real, "AA_imag": float(np.max(np.abs((aa / Z).imag))),
            "wmin": wmin}


def dimer_hopping(t=1.0):
    """Two sites (A, B) joined by one bond."""
    return np.array([[0.0, -t], [-t, 0.0]])


def ring4_hopping(t=1.0, phi=0.0):
    """Four sites on a ring (A = 0, 1; B = 2, 3; bonds 0-2, 2-1, 1-3, 3-0),
    each bond with the Peierls phase phi (a flux 4 phi through the ring)."""
    K = np.zeros((4, 4), dtype=complex)
    for a, b in ((0, 2), (2, 1), (1, 3), (3, 0)):
        K[a, b] += -t * np.exp(1j * phi)
        K[b, a] += -t * np.exp(-1j * phi)
    return K if phi != 0.0 else K.real.copy()


def tiny_model(U=3.8, dtau=0.25, M=2, theta1=0.0, theta2=0.0, L=2, channel="spin"):
    return Model(L, U, M * dtau, dtau, theta1=theta1, theta2=theta2, n_stab=max(1, M), channel=channel)
