"""Honeycomb torus and its hopping matrix, written from the model definition.

Test infrastructure only (see ``oracle/__init__.py``).

Conventions (Sec. II A, eq. HubbModel and eq. h0kMat; Sec. III C):
  * primitive vectors a1 = (sqrt3, 0), a2 = (sqrt3/2, 3/2); reciprocal
    b1 = (2pi/sqrt3, -2pi/3), b2 = (0, 4pi/3); a_i . b_j = 2 pi delta_ij.
  * L x L unit cells, cell index I = n1 + L*n2 (0-based); N_c = L^2,
    N_s = 2 N_c.  A sites are 0..N_c-1, B sites are N_c..N_s-1 (the paper
    labels A first, then B, in the multi-sublattice FFT subsection).
  * Each A site at cell r bonds to the B site of cells r + delta_eta with
    delta_1 = (0,0), delta_2 = (1,-1) (i.e. a1 - a2), delta_3 = (0,-1)
    (i.e. -a2), as in the Gauge-I list of hopping vectors.
  * Twist: Theta_alpha = 2 pi theta_alpha (radians, along a_alpha).  The
    uniform vector potential satisfies A . a_alpha = Theta_alpha / L
    (eq. VecATBC).  Peierls phase of the hop A(r) -> B(r+delta) is
    Phi = A . d, with d the cell displacement (Gauge-I, eq. GaugeIPhase) or
    the true bond vector (Gauge-II, eq. GaugeIIPhase).

Reading adopted for the phase sign: the matrix element K[A(r), B(r+delta)] is
-t * exp(+i Phi).  With this sign the k-space block is f(k + A), i.e. the
shifted grid k = ((l1+theta1)/L) b1 + ((l2+theta2)/L) b2 of eq. kpoints.
The opposite sign printed with the Peierls substitution gives f(k - A); the
two differ by theta -> -theta, which is complex conjugation of K.
"""
import numpy as np

SQ3 = np.sqrt(3.0)
A1 = np.array([SQ3, 0.0])
A2 = np.array([SQ3 / 2.0, 1.5])
B1 = np.array([2 * np.pi / SQ3, -2 * np.pi / 3.0])
B2 = np.array([0.0, 4 * np.pi / 3.0])
TAU_AB = np.array([0.0, 1.0])

# Gauge-I cell displacements (n1, n2) of the three A->B hops.
DELTAS = ((0, 0), (1, -1), (0, -1))


class Lattice:
    """L x L honeycomb torus with hopping t and twist (Theta1, Theta2)."""

    def __init__(self, L, t=1.0, theta1=0.0, theta2=0.0):
        if L < 2:
            raise ValueError("L >= 2 required")
        self.L = int(L)
        self.t = float(t)
        self.theta1 = float(theta1)
        self.theta2 = float(theta2)
        self.Nc = self.L * self.L
        self.N = 2 * self.Nc

    @property
    def twisted(self):
        return (self.theta1 % (2 * np.pi)) != 0.0 or (self.theta2 % (2 * np.pi)) != 0.0

    def cell(self, n1, n2):
        L = self.L
        return (n1 % L) + L * (n2 % L)

    def site_A(self, n1, n2):
        return self.cell(n1, n2)

    def site_B(self, n1, n2):
        return self.Nc + self.cell(n1, n2)

    def cell_coords(self, I):
        return I % self.L, I // self.L

    def positions(self):
        """Real-space coordinates of all N_s sites (A at r_I, B at r_I + tau_AB)."""
        pos = np.zeros((self.N, 2))
        for I in range(self.Nc):
            n1, n2 = self.cell_coords(I)
            r = n1 * A1 + n2 * A2
            pos[I] = r
            pos[self.Nc + I] = r + TAU_AB
        return pos

    def vector_potential(self):
        """A with A . a_alpha = Theta_alpha / L  (eq. VecATBC with L1 = L2 = L)."""
        th1 = self.theta1 / (2 * np.pi)
        th2 = self.theta2 / (2 * np.pi)
        return (th1 / self.L) * B1 + (th2 / self.L) * B2

    def bonds(self):
        """List of (A site, B site, Gauge-I displacement d, Gauge-II displacement d')."""
        out = []
        for I in range(self.Nc):
            n1, n2 = self.cell_coords(I)
            for (d1, d2) in DELTAS:
                dI = d1 * A1 + d2 * A2
                out.append((self.site_A(n1, n2), self.site_B(n1 + d1, n2 + d2), dI, dI + TAU_AB))
        return out

    def hopping_matrix(self, gauge="I"):
        """Dense N_s x N_s hopping matrix K of H_0 = sum_ij K_ij c_i^+ c_j.

        Entries accumulate, so a bond that appears twice on a small torus is
        counted twice, as the sum over nearest-neighbour pairs requires.
        """
        A = self.vector_potential()
        twisted = self.twisted
        K = np.zeros((self.N, self.N), dtype=complex)
        for a, b, dI, dII in self.bonds():
            d = dI if gauge == "I" else dII
            phase = np.exp(1j * np.dot(A, d))
            K[a, b] += -self.t * phase
            K[b, a] += -self.t * np.conj(phase)
        if not twisted and gauge == "I":
            return K.real.copy()
        return K

    # ---- momentum space (eq. h0kMat, eq. kpoints) --------------------------
    def kpoints(self):
        """Shifted grid k = ((l1+theta1)/L) b1 + ((l2+theta2)/L) b2, ordered l1 + L*l2."""
        th1 = self.theta1 / (2 * np.pi)
        th2 = self.theta2 / (2 * np.pi)
        ks = np.zeros((self.Nc, 2))
        for l2 in range(self.L):
            for l1 in range(self.L):
                ks[l1 + self.L * l2] = ((l1 + th1) / self.L) * B1 + ((l2 + th2) / self.L) * B2
        return ks

    def f_of_k(self, k):
        """f(k) = -t [1 + exp(i k.(a1-a2)) + exp(-i k.a2)]   (eq. h0kMat)."""
        k = np.atleast_2d(k)
        return -self.t * (1.0 + np.exp(1j * (k @ (A1 - A2))) + np.exp(-1j * (k @ A2)))

    def dispersion(self):
        """All single-particle energies +-|f(k)| on the shifted grid."""
        f = np.abs(self.f_of_k(self.kpoints()))
        return np.concatenate([-f, f])
