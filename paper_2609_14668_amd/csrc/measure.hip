// Equal-time estimators from the spin-up Green's function alone (Sec. II B-C).
//
// In the spin channel the spin-down partner follows from the particle-hole
// relation in the original basis, G_dn = P (1 - G_up^dagger) P with P = +1 on
// A and -1 on B, so <n_dn,i> = b_i = conj(G_ii); in the charge channel both
// spins see the same B's, G_dn = G_up and b_i = 1 - G_ii.  For i != j
//   4 <s_i s_j> = (a_i - b_i)(a_j - b_j) - 2 Re(G_ij G_ji),
//   a_i = 1 - G_ii;  4 <s_i^2> = a_i + b_i - 2 a_i b_i
// (real parts: the charge channel's per-configuration estimators are complex
// and only their averages are real).
// D = mean a_i b_i; <H_0> = -2 Re Tr(K G); e = <H_0>/N_s + U D
// (Sec. IV C); S_zz(k) of eq. SpinStrucF from the intra-sublattice
// correlations of eq. SzSzCrF at k = 0 and k = b1/L; m^2 = S_zz(0)/(2 N_c).
// The weight is real and non-negative (spin channel: det_dn is the complex
// conjugate of det_up up to a positive factor; charge channel: P(X) det_up^2
// with the phase of P(X), by the partial particle-hole symmetry of Sec. II B);
// the phase of det_up itself (tracked per accepted flip, anchored at every
// recomputation) is recorded with each measurement.
#include "common.hpp"
#include "kernels.hpp"

namespace {

constexpr int MT = 256;

__device__ __forceinline__ double bsum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

// Pair sums over i != j within each sublattice,
//   pG = sum Re(G_ij G_ji),  pK = sum Re(G_ij G_ji) cos(2 pi (n1_j - n1_i) / L),
// one workgroup per (sublattice, strip of PB rows i), and over the
// cross-sublattice pairs (i on A, j on B) pX = sum Re(G_ij G_ji) for the
// charge compressibility, one workgroup per strip of A rows; each strip is
// walked in PB x PB tiles, G[i, j] and G[j, i] both read down columns
// (coalesced) into LDS.  The partials go to VEC_NORM (two per same-sublattice
// strip, then one per cross strip) and are summed in strip order by k_measure.
constexpr int PB = 32;
template <typename S>
__global__ void __launch_bounds__(MT) k_measure_pairs(const InstDev* __restrict__ insts, int mat) {
  const InstDev& d = insts[blockIdx.y];
  InstState* st = d.st;
  if (st->init_mode || st->idle) return;
  const int N = d.N, Nc = d.Nc, L = d.L;
  const int nb = (Nc + PB - 1) / PB;
  if ((int)blockIdx.x >= 3 * nb) return;
  const bool cross = (int)blockIdx.x >= 2 * nb;
  const int sub = cross ? 0 : (blockIdx.x & 1);
  const int I0 = (cross ? (int)blockIdx.x - 2 * nb : (int)(blockIdx.x >> 1)) * PB;
  const int base = sub * Nc, jbase = cross ? Nc : base;
  const S* G = matp<S>(d, mat);
  __shared__ S Aij[PB][PB + 1], Aji[PB][PB + 1];
  __shared__ double cosL[64];
  __shared__ double red[4];
  const double twopiL = 2.0 * M_PI / L;
  for (int m = threadIdx.x; m < L; m += MT) cosL[m] = cos(twopiL * m);
  const int r = threadIdx.x % PB, c0 = threadIdx.x / PB;   // 8 column groups
  double pG = 0, pK = 0;
  for (int J0 = 0; J0 < Nc; J0 += PB) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PB / 8; ++u) {
      const int cc = c0 + 8 * u;
      const int i = min(I0 + r, Nc - 1), j = min(J0 + cc, Nc - 1);
      const int jr = min(J0 + r, Nc - 1), ic = min(I0 + cc, Nc - 1);
      Aij[r][cc] = gld(G + (base + i) + (size_t)(jbase + j) * N);     // G[I0 + r, J0 + cc]
      Aji[r][cc] = gld(G + (jbase + jr) + (size_t)(base + ic) * N);   // G[J0 + r, I0 + cc]
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PB / 8; ++u) {
      const int a = r, b = c0 + 8 * u;
      const int ii = I0 + a, jj = J0 + b;
      if (ii < Nc && jj < Nc && (cross || ii != jj)) {
        const double re = real_part(Aij[a][b] * Aji[b][a]);
        pG += re;
        pK += re * cosL[((jj % L) - (ii % L) + L) % L];
      }
    }
  }
  pG = bsum(pG, red);
  pK = bsum(pK, red);
  if (threadIdx.x == 0) {
    if (cross) {
      d.vec[VEC_NORM][4 * nb + (blockIdx.x - 2 * nb)] = pG;
    } else {
      d.vec[VEC_NORM][2 * blockIdx.x] = pG;
      d.vec[VEC_NORM][2 * blockIdx.x + 1] = pK;
    }
  }
}

template <typename S>
__global__ void __launch_bounds__(MT) k_measure(const InstDev* __restrict__ insts, int mat) {
  const InstDev& d = insts[blockIdx.y];
  InstState* st = d.st;
  if (st->init_mode || st->idle) return;
  const int N = d.N, Nc = d.Nc, L = d.L;
  const S* G = matp<S>(d, mat);
  const bool charge = d.channel != 0;   // G_dn = G_up (else the particle-hole partner)
  __shared__ double red[4];
  const double twopiL = 2.0 * M_PI / L;
  double sn = 0, sD = 0, sdc = 0;
  double zsum[2] = {0, 0}, zc[2] = {0, 0}, zs[2] = {0, 0};
  double trr = 0, tri = 0, dsq = 0;   // Re, Im Tr G; sum_i Re(G_ii^2)
  for (int i = threadIdx.x; i < N; i += MT) {
    S g = G[i + (size_t)i * N];
    trr += real_part(g);
    tri += imag_part(g);
    dsq += real_part(g * g);
    S a = ST<S>::one() - g;                       // <n_up,i>
    S b = charge ? ST<S>::one() - g : conjg(g);   // <n_dn,i>
    double ab = real_part(a * b);
    double z = real_part(a - b);
    sn += real_part(a + b);
    sD += ab;
    sdc += real_part(a + b) - 2.0 * ab - z * z;
    int sub = i >= Nc;
    int n1 = (i - sub * Nc) % L;
    zsum[sub] += z;
    zc[sub] += z * cos(twopiL * n1);
    zs[sub] += z * sin(twopiL * n1);
  }
  // pair terms within each sublattice (i != j): partial sums of k_measure_pairs
  double pG = 0, pK = 0, pX = 0;
  const int nbs = (Nc + PB - 1) / PB, nstrip = 2 * nbs;
  for (int x = threadIdx.x; x < nstrip; x += MT) {
    pG += d.vec[VEC_NORM][2 * x];
    pK += d.vec[VEC_NORM][2 * x + 1];
  }
  for (int x = threadIdx.x; x < nbs; x += MT) pX += d.vec[VEC_NORM][4 * nbs + x];
  // Tr(K G): K[A(r), B(r+delta)] = -t e^{+i Phi_delta}, Gauge-I phases
  const double ph[3] = {0.0, (d.theta1 - d.theta2) / L, -d.theta2 / L};
  const int dn1[3] = {0, 1, 0}, dn2[3] = {0, -1, -1};
  double tk = 0;
  for (int r = threadIdx.x; r < Nc; r += MT) {
    int n1 = r % L, n2 = r / L;
    for (int e = 0; e < 3; ++e) {
      int m1 = (n1 + dn1[e] + L) % L, m2 = (n2 + dn2[e] + L) % L;
      int ia = r, ib = Nc + m1 + L * m2;
      S gba = G[ib + (size_t)ia * N];
      S gab = G[ia + (size_t)ib * N];
      double c = cos(ph[e]), s = sin(ph[e]);
      // -t [e^{i phi} G_ba + e^{-i phi} G_ab], real part
      tk += -d.t * ((c * real_part(gba) - s * imag_part(gba)) + (c * real_part(gab) + s * imag_part(gab)));
    }
  }
  sn = bsum(sn, red);
  sD = bsum(sD, red);
  sdc = bsum(sdc, red);
  double z0 = bsum(zsum[0], red), z1 = bsum(zsum[1], red);
  double c0 = bsum(zc[0], red), c1 = bsum(zc[1], red);
  double s0 = bsum(zs[0], red), s1 = bsum(zs[1], red);
  pG = bsum(pG, red);
  pK = bsum(pK, red);
  pX = bsum(pX, red);
  tk = bsum(tk, red);
  trr = bsum(trr, red);
  tri = bsum(tri, red);
  dsq = bsum(dsq, red);
  if (threadIdx.x == 0) {
    double n = sn / N;
    double D = sD / N;
    double ekin = -2.0 * tk / N;
    double e = ekin + d.U * D;
    double SG = (0.25 * (z0 * z0 + z1 * z1) - 0.5 * pG + 0.25 * sdc) / (2.0 * Nc);
    double Sdk = (0.25 * (c0 * c0 + s0 * s0 + c1 * c1 + s1 * s1) - 0.5 * pK + 0.25 * sdc) / (2.0 * Nc);
    double v[OBS_COUNT] = {0};
    v[OBS_N] = n; v[OBS_D] = D; v[OBS_EKIN] = ekin; v[OBS_E] = e;
    v[OBS_SZZ_G] = SG; v[OBS_SZZ_DK] = Sdk; v[OBS_M2] = SG / (2.0 * Nc);
    v[OBS_RM2_NUM] = Sdk; v[OBS_PHASE_RE] = st->ph_re; v[OBS_PHASE_IM] = st->ph_im;
    // charge compressibility (eq. ChiCharge): (beta/N)(Re[(sum_i n_i)^2 +
    // sum_s (Tr G^s - Tr G^s G^s)] - N^2) with sum_i n_i = N - 2 i Im Tr G and
    // the spin-down traces the conjugates of the spin-up ones
    const double retr2 = dsq + pG + 2.0 * pX;   // Re Tr(G G) over all pairs
    const double beta = d.M * d.dtau;
    v[OBS_CHI] = (beta / N) * (-4.0 * tri * tri + 2.0 * (trr - retr2));
    for (int k = 0; k < OBS_COUNT; ++k) {
      d.obs[k] += v[k];
      d.obs[OBS_COUNT + k] += v[k];
    }
    d.obs[2 * OBS_COUNT] += 1.0;
    st->n_meas += 1;
  }
}

// Momentum distribution (eq. nkMatrix) from Ghat = F G F^dagger (the forward
// 2-D DFT of both sides, in mat): spin up n_ab(k) = delta_ab - Ghat[b k, a k] / Nc,
// spin down (G_dn = P (1 - G_up^dagger) P) n_ab(k) = s_a s_b conj(Ghat[a k, b k]) / Nc,
// s_A = 1, s_B = -1 (charge channel: equal to spin up); the spin average is
// added to the instance's sums.
template <typename S>
__global__ void __launch_bounds__(MT) k_measure_k(const InstDev* __restrict__ insts, int mat) {
  const InstDev& d = insts[blockIdx.y];
  const InstState* st = d.st;
  if (st->init_mode || st->idle) return;
  const int N = d.N, Nc = d.Nc;
  const int k = blockIdx.x * MT + threadIdx.x;
  if (k >= Nc) return;
  const S* G = matp<S>(d, mat);
  const double inv = 1.0 / Nc;
  double* o = d.nk_sum + (size_t)8 * k;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      const S gba = G[(b * Nc + k) + (size_t)(a * Nc + k) * N];   // Ghat[b k, a k]
      const S gab = G[(a * Nc + k) + (size_t)(b * Nc + k) * N];   // Ghat[a k, b k]
      const double sab = (a == b) ? 1.0 : -1.0;
      const double up_re = (a == b ? 1.0 : 0.0) - real_part(gba) * inv, up_im = -imag_part(gba) * inv;
      double dn_re = sab * real_part(gab) * inv, dn_im = -sab * imag_part(gab) * inv;
      if (d.channel) { dn_re = up_re; dn_im = up_im; }   // charge channel: G_dn = G_up
      o[4 * a + 2 * b] += 0.5 * (up_re + dn_re);
      o[4 * a + 2 * b + 1] += 0.5 * (up_im + dn_im);
    }
}

// ---- time-displaced pass (Sec. II C, eqs. DouOccDerive, fidelitysusp) ----------------
// With A = sum_i m_up,i m_dn,i (m = n - 1/2; H_I = A - N_s/4) and, per spin,
//   t_ij = a_i b_j - G(0,tau)_ji G(tau,0)_ij,  a_i = 1/2 - G(tau,tau)_ii,
//   b_j = 1/2 - G(0,0)_jj,
// Wick's theorem gives <A(tau) A(0)>_X = sum_ij t_ij^up t_ij^dn.  In the spin
// channel the spin-down functions are the particle-hole partners
// G_dn(tau,0) = -P G_up(0,tau)^dagger P, G_dn(0,tau) = -P G_up(tau,0)^dagger P,
// G_dn(tau,tau) = P (1 - G_up(tau,tau)^dagger) P, so t^dn = conj(t^up) and the
// sum is sum_ij |t_ij|^2; in the charge channel G_dn = G_up and it is
// sum_ij t_ij^2 (real part: only the weighted average is real).  The
// equal-time <A>_X = sum_i m_up,i m_dn,i is -sum_i |1/2 - G_ii|^2 (spin) or
// Re sum_i (1/2 - G_ii)^2 (charge).

// Instance state around a pass.  mode 0: instances at the start of a sweep
// (phase 0) take part up to slice min(M/2, lmax_req) (lmax_req < 0: M/2); the
// others are parked idle.  mode 1, slice l: a taking part instance whose last
// slice is below l is parked, the others get the upward phase of slice l (so
// that the chain steps, stack slots and wraps resolve to slice l).  mode 2:
// phases back to 0, idle flags restored.
__global__ void k_tau_state(const InstDev* __restrict__ insts, int mode, int l, int lmax_req) {
  const InstDev& d = insts[blockIdx.y];
  InstState* st = d.st;
  if (threadIdx.x != 0) return;
  if (mode == 0) {
    const int ok = !st->idle && !st->init_mode && st->phase == 0;
    st->tau_saved_idle = st->idle;
    st->tau_active = ok;
    st->tau_lmax = ok ? (lmax_req < 0 ? d.M / 2 : min(d.M / 2, lmax_req)) : -1;
    if (!ok) st->idle = 1;
  } else if (mode == 1) {
    if (!st->tau_active) return;
    if (l > st->tau_lmax) st->idle = 1;
    else st->phase = l - 1;
  } else {
    if (st->tau_active) st->phase = 0;
    st->idle = st->tau_saved_idle;
    st->tau_active = 0;
  }
}

// Partial sums of sum_ij term(t_ij) over one strip of PB rows i per
// workgroup: G(tau,0)[i, j] and G(0,tau)[j, i] tiles both read down columns
// into LDS; the partial goes to VEC_NORM[strip].
template <typename S>
__global__ void __launch_bounds__(MT) k_measure_tau_pairs(const InstDev* __restrict__ insts) {
  const InstDev& d = insts[blockIdx.y];
  const InstState* st = d.st;
  if (st->idle || !st->tau_active) return;
  const int N = d.N;
  const int nb = (N + PB - 1) / PB;
  if ((int)blockIdx.x >= nb) return;
  const int I0 = blockIdx.x * PB;
  const S* gt0 = matp<S>(d, MAT_GT0);
  const S* g0t = matp<S>(d, MAT_G0T);
  const S* gtt = matp<S>(d, MAT_GTT);
  const S* g = matp<S>(d, MAT_G);
  const bool charge = d.channel != 0;
  __shared__ S At[PB][PB + 1], Bt[PB][PB + 1];
  __shared__ S ai[PB], bj[PB];
  __shared__ double red[4];
  const S half = ST<S>::from_re(0.5);
  if (threadIdx.x < PB) {
    const int i = min(I0 + (int)threadIdx.x, N - 1);
    ai[threadIdx.x] = half - gtt[i + (size_t)i * N];
  }
  const int r = threadIdx.x % PB, c0 = threadIdx.x / PB;   // 8 column groups
  double acc = 0.0;
  for (int J0 = 0; J0 < N; J0 += PB) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PB / 8; ++u) {
      const int cc = c0 + 8 * u;
      const int i = min(I0 + r, N - 1), j = min(J0 + cc, N - 1);
      const int jr = min(J0 + r, N - 1), ic = min(I0 + cc, N - 1);
      At[r][cc] = gld(gt0 + i + (size_t)j * N);    // G(tau,0)[I0 + r, J0 + cc]
      Bt[r][cc] = gld(g0t + jr + (size_t)ic * N);  // G(0,tau)[J0 + r, I0 + cc]
    }
    if (threadIdx.x < PB) {
      const int j = min(J0 + (int)threadIdx.x, N - 1);
      bj[threadIdx.x] = half - g[j + (size_t)j * N];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PB / 8; ++u) {
      const int a = r, b = c0 + 8 * u;
      if (I0 + a < N && J0 + b < N) {
        const S t = ai[a] * bj[b] - Bt[b][a] * At[a][b];
        acc += charge ? real_part(t * t) : absq(t);
      }
    }
  }
  acc = bsum(acc, red);
  if (threadIdx.x == 0) d.vec[VEC_NORM][blockIdx.x] = acc;
}

// Strip partials summed in strip order into slice l's sums and this pass's
// row, with <A>_X(tau_l) from the diagonal of G(tau_l, tau_l); the pass count
// advances at the instance's last slice.  Layout (lc = M/2): sums and rows
// hold <A(tau_l) A(0)>_X at [l] and <A>_X(tau_l) at [lc + 1 + l]; the sums end
// with the pass count at [2 lc + 2].
template <typename S>
__global__ void __launch_bounds__(MT) k_measure_tau_fin(const InstDev* __restrict__ insts, int l) {
  const InstDev& d = insts[blockIdx.y];
  InstState* st = d.st;
  if (st->idle || !st->tau_active) return;
  const int N = d.N;
  const int nb = (N + PB - 1) / PB;
  __shared__ double red[4];
  double v = 0.0;
  for (int x = threadIdx.x; x < nb; x += MT) v += d.vec[VEC_NORM][x];
  v = bsum(v, red);
  double at = 0.0;
  {
    const S* g = matp<S>(d, MAT_GTT);
    const S half = ST<S>::from_re(0.5);
    for (int i = threadIdx.x; i < N; i += MT) {
      const S m = half - g[i + (size_t)i * N];
      at += d.channel != 0 ? real_part(m * m) : -absq(m);
    }
    at = bsum(at, red);
  }
  const int lc = d.M / 2, stride = 2 * lc + 2;
  const int64_t pass = (int64_t)d.tau_sum[2 * lc + 2];
  double* row = d.tau_rows + (size_t)(pass % d.tau_cap) * stride;
  if (l == 0)
    for (int x = threadIdx.x; x < stride; x += MT) row[x] = 0.0;
  __syncthreads();
  if (threadIdx.x == 0) {
    d.tau_sum[l] += v;
    d.tau_sum[lc + 1 + l] += at;
    row[l] = v;
    row[lc + 1 + l] = at;
    if (l == st->tau_lmax) d.tau_sum[2 * lc + 2] += 1.0;
  }
}

}  // namespace

hipError_t launch_tau_state(const InstDev* insts, int n_inst, int mode, int l, int lmax_req, hipStream_t s) {
  hipLaunchKernelGGL(k_tau_state, dim3(1, n_inst), dim3(64), 0, s, insts, mode, l, lmax_req);
  return hipGetLastError();
}

hipError_t launch_measure_tau(const InstDev* insts, int n_inst, int Nmax, bool cplx_, int l, hipStream_t s) {
  dim3 grid((Nmax + PB - 1) / PB, n_inst);
  if (cplx_) {
    hipLaunchKernelGGL(k_measure_tau_pairs<cplx>, grid, dim3(MT), 0, s, insts);
    hipLaunchKernelGGL(k_measure_tau_fin<cplx>, dim3(1, n_inst), dim3(MT), 0, s, insts, l);
  } else {
    hipLaunchKernelGGL(k_measure_tau_pairs<double>, grid, dim3(MT), 0, s, insts);
    hipLaunchKernelGGL(k_measure_tau_fin<double>, dim3(1, n_inst), dim3(MT), 0, s, insts, l);
  }
  return hipGetLastError();
}

hipError_t launch_measure_k(const InstDev* insts, int n_inst, int Nmax, bool cplx_, int mat, hipStream_t s) {
  const int ncm = Nmax / 2;
  dim3 grid((ncm + MT - 1) / MT, n_inst);
  if (cplx_) hipLaunchKernelGGL(k_measure_k<cplx>, grid, dim3(MT), 0, s, insts, mat);
  else hipLaunchKernelGGL(k_measure_k<double>, grid, dim3(MT), 0, s, insts, mat);
  return hipGetLastError();
}

hipError_t launch_measure(const InstDev* insts, int n_inst, int Nmax, bool cplx_, int mat, hipStream_t s) {
  const int ncm = Nmax / 2;
  dim3 grid(3 * ((ncm + PB - 1) / PB), n_inst);
  if (cplx_) hipLaunchKernelGGL(k_measure_pairs<cplx>, grid, dim3(MT), 0, s, insts, mat);
  else hipLaunchKernelGGL(k_measure_pairs<double>, grid, dim3(MT), 0, s, insts, mat);
  if (cplx_) hipLaunchKernelGGL(k_measure<cplx>, dim3(1, n_inst), dim3(MT), 0, s, insts, mat);
  else hipLaunchKernelGGL(k_measure<double>, dim3(1, n_inst), dim3(MT), 0, s, insts, mat);
  return hipGetLastError();
}
