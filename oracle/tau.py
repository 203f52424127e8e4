"""Time-displaced Green's functions and the interaction-energy correlator of
the dynamical estimators (Sec. II C, eqs. DouOccDerive and fidelitysusp).
Test infrastructure only.

Definitions used here (tau_l = l dtau, tau_M = beta, one HS configuration and
one spin species, B_l as in ``dqmc.Model.B``):

* G(tau_l, tau_m) = <T c(tau_l) c^dagger(tau_m)> is block (l, m) of the
  inverse of the MN x MN block-cyclic matrix
      O = 1 - sum_{l=2..M} E_{l,l-1} (x) B_l + E_{1,M} (x) B_1,
  the determinant formulation of the finite-temperature fermion path
  integral (det O = det(1 + B_M .. B_1)).  Solving O X = 1 block by block
  gives X_ll = (1 + B_l..B_1 B_M..B_{l+1})^{-1} = G(l) (eq. GrFMat),
  X_lm = B_l..B_{m+1} G(m) for l > m and X_lm = -(1 - G(l)) (B_m..B_{l+1})^{-1}
  for l < m.
* With 0 identified with beta (antiperiodicity),
      G(tau_l, 0) = -X_{l,M},   G(0, tau_l) = -X_{M,l}       (0 < l < M),
  G(tau_0, 0) = G(0, 0) = X_{MM}, G(0, tau_0) = G(0, 0) - 1 (equal time with
  the creation operator to the left), G(beta, 0) = 1 - G(0, 0),
  G(0, beta) = -G(0, 0).
* H_I = sum_i [n_up,i n_dn,i - (n_up,i + n_dn,i)/2] = A - N_s/4 with
  A = sum_i m_up,i m_dn,i, m = n - 1/2.  For a fixed configuration the two
  spins are independent and Wick's theorem gives
      <A(tau) A(0)>_X = sum_ij prod_sigma [ m_sigma,i(tau) m_sigma,j(0)
                                 - G_sigma(0,tau)_ji G_sigma(tau,0)_ij ],
  m_sigma,i(tau) = 1/2 - G_sigma(tau,tau)_ii; the equal-time <A>_X(tau) is
  sum_i m_up,i(tau) m_dn,i(tau).  Both spins are propagated explicitly here.
* C(tau) = <A(tau) A(0)> - <A>^2 (the constant in H_I drops out).
  dD/dU = -(2/N_s) int_0^{beta/2} C dtau (eq. DouOccDerive) and
  chi_F = int_0^{beta/2} tau C dtau (eq. fidelitysusp).  For the Trotterised
  partition function Tr[(e^{-dtau H_U} e^{-dtau H_0})^M] differentiating each
  factor e^{-dtau U A} gives exactly dD/dU = -(dtau/N_s) sum_{l=1..M} C(tau_l),
  which with C(tau_l) = C(tau_{M-l}) is the trapezoid rule on [0, beta/2]
  (M even); the paper instead fits a polynomial to C(tau) and integrates it
  analytically, which ``tau_integrals`` offers as well.
"""
import numpy as np


def tau_greens(model, fields, spin, lmax):
    """[(G(t,t), G(t,0), G(0,t)) for t = tau_0 .. tau_lmax] of one spin from
    the block-cyclic inverse.  fields: (M, N) or a batch (B, M, N) of +-1;
    the matrices then carry the batch as their leading axis."""
    M, N = model.M, model.N
    if not 0 <= lmax <= M:
        raise ValueError("lmax must be in [0, M]")
    X = np.asarray(fields, dtype=float)
    single = X.ndim == 2
    X = X.reshape(-1, M, N)
    nb = X.shape[0]
    O = np.zeros((nb, M * N, M * N), dtype=complex)
    idx = np.arange(M * N)
    O[:, idx, idx] = 1.0
    for l in range(1, M + 1):
        B = model.vdiag(spin, X[:, l - 1, :])[:, :, None] * model.Ep[None]
        r0 = (l - 1) * N
        if l == 1:
            O[:, 0:N, (M - 1) * N:M * N] += B
        else:
            O[:, r0:r0 + N, r0 - N:r0] -= B
    Xi = np.linalg.inv(O)

    def blk(l, m):
        return Xi[:, (l - 1) * N:l * N, (m - 1) * N:m * N]

    eye = np.eye(N)[None]
    g00 = blk(M, M)
    out = []
    for l in range(lmax + 1):
        if l == 0:
            t = (g00, g00, g00 - eye)
        elif l == M:
            t = (g00, eye - g00, -g00)
        else:
            t = (blk(l, l), -blk(l, M), -blk(M, l))
        out.append(tuple(a[0] for a in t) if single else t)
    return out


def tau_correlator(model, fields, lmax):
    """Per configuration: (<A(tau_l) A(0)>_X, <A>_X at slice tau_l) for
    l = 0..lmax, both complex in general (their weighted averages are real);
    batched like ``tau_greens``.  The equal-time <A>_X(tau) = sum_i
    m_up,i(tau) m_dn,i(tau) depends on the slice for a fixed configuration;
    its average does not."""
    gs = [tau_greens(model, fields, s, lmax) for s in (0, 1)]
    m0 = [0.5 - np.diagonal(g[0][0], axis1=-2, axis2=-1) for g in gs]
    AA, At = [], []
    for l in range(lmax + 1):
        P, mts = [], []
        for s in (0, 1):
            gtt, gt0, g0t = gs[s][l]
            mt = 0.5 - np.diagonal(gtt, axis1=-2, axis2=-1)
            mts.append(mt)
            P.append(mt[..., :, None] * m0[s][..., None, :] - np.swapaxes(g0t, -1, -2) * gt0)
        AA.append(np.sum(P[0] * P[1], axis=(-2, -1)))
        At.append(np.sum(mts[0] * mts[1], axis=-1))
    return np.stack(AA, axis=-1), np.stack(At, axis=-1)


def connected(aa, a1):
    """C(tau_l) = <A(tau_l) A(0)> - <A>^2 from the averaged series."""
    return np.asarray(aa) - np.asarray(a1) ** 2


def connected_improved(aa_rows, at_rows):
    """C(tau_l) from per-configuration rows (aa_rows[n, l] = <A(tau_l) A(0)>_X,
    at_rows[n, l] = <A>_X(tau_l)) as the mean of the fermionic part
    <A(tau) A(0)>_X - <A>_X(tau) <A>_X(0) plus the covariance over
    configurations of <A>_X(tau) and <A>_X(0) about the mean of <A>_X over all
    rows and slices (the same in every slice by time-translation invariance).
    Equal to ``connected`` of the averages up to O(1/n) terms, without the
    cancellation of two large numbers."""
    aa = np.asarray(aa_rows, dtype=float)
    at = np.asarray(at_rows, dtype=float)
    mean_a = at.mean()
    ferm = np.mean(aa - at * at[:, :1], axis=0)
    cov = np.mean((at - mean_a) * (at[:, :1] - mean_a), axis=0)
    return ferm + cov


def tau_integrals(c, dtau, n_sites, degree=None):
    """(dD/dU, chi_F) from C(tau_l), l = 0..n-1 on tau_l = l dtau, the last
    point being beta/2: trapezoid rule (degree None) or the integral of the
    least-squares polynomial of the given degree in tau."""
    c = np.asarray(c, dtype=float)
    tau = dtau * np.arange(len(c))
    if degree is None:
        w = np.full(len(c), dtau)
        w[0] = w[-1] = dtau / 2
        i0 = float(np.sum(w * c))
        i1 = float(np.sum(w * tau * c))
    else:
        a = np.polynomial.polynomial.polyfit(tau, c, degree)       # C(tau) = sum_k a_k tau^k
        b = tau[-1]
        i0 = float(sum(a[k] * b ** (k + 1) / (k + 1) for k in range(degree + 1)))
        i1 = float(sum(a[k] * b ** (k + 2) / (k + 2) for k in range(degree + 1)))
    return -2.0 * i0 / n_sites, i1
