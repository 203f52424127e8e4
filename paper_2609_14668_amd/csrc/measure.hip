// Equal-time estimators from the spin-up Green's function alone (Sec. II B-C).
//
// The spin-down partner follows from the particle-hole relation in the
// original basis, G_dn = P (1 - G_up^dagger) P with P = +1 on A and -1 on B,
// so <n_dn,i> = conj(G_ii) and for i != j
//   4 <s_i s_j> = (a_i - b_i)(a_j - b_j) - 2 Re(G_ij G_ji),
//   a_i = 1 - G_ii, b_i = conj(G_ii);  4 <s_i^2> = a_i + b_i - 2 a_i b_i.
// D = mean a_i b_i; <H_0> = -2 Re Tr(K G); e = <H_0>/N_s + U D
// (Sec. IV C); S_zz(k) of eq. SpinStrucF from the intra-sublattice
// correlations of eq. SzSzCrF at k = 0 and k = b1/L; m^2 = S_zz(0)/(2 N_c).
// The weight det_up det_dn is real and non-negative, since det_dn is the
// complex conjugate of det_up up to a positive factor (Sec. II B); the phase
// of det_up itself (tracked per accepted flip, anchored at every
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
// one workgroup per (sublattice, strip of PB rows i); the strip is walked in
// PB x PB tiles, G[i, j] and G[j, i] both read down columns (coalesced) into
// LDS.  The partials go to VEC_NORM (two per strip) and are summed in strip
// order by k_measure.
constexpr int PB = 32;
template <typename S>
__global__ void __launch_bounds__(MT) k_measure_pairs(const InstDev* __restrict__ insts, int mat) {
  const InstDev& d = insts[blockIdx.y];
  InstState* st = d.st;
  if (st->init_mode || st->idle) return;
  const int N = d.N, Nc = d.Nc, L = d.L;
  const int nb = (Nc + PB - 1) / PB;
  if ((int)blockIdx.x >= 2 * nb) return;
  const int sub = blockIdx.x & 1, I0 = (blockIdx.x >> 1) * PB, base = sub * Nc;
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
      Aij[r][cc] = gld(G + (base + i) + (size_t)(base + j) * N);     // G[I0 + r, J0 + cc]
      Aji[r][cc] = gld(G + (base + jr) + (size_t)(base + ic) * N);   // G[J0 + r, I0 + cc]
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PB / 8; ++u) {
      const int a = r, b = c0 + 8 * u;
      const int ii = I0 + a, jj = J0 + b;
      if (ii < Nc && jj < Nc && ii != jj) {
        const double re = real_part(Aij[a][b] * Aji[b][a]);
        pG += re;
        pK += re * cosL[((jj % L) - (ii % L) + L) % L];
      }
    }
  }
  pG = bsum(pG, red);
  pK = bsum(pK, red);
  if (threadIdx.x == 0) {
    d.vec[VEC_NORM][2 * blockIdx.x] = pG;
    d.vec[VEC_NORM][2 * blockIdx.x + 1] = pK;
  }
}

template <typename S>
__global__ void __launch_bounds__(MT) k_measure(const InstDev* __restrict__ insts, int mat) {
  const InstDev& d = insts[blockIdx.y];
  InstState* st = d.st;
  if (st->init_mode || st->idle) return;
  const int N = d.N, Nc = d.Nc, L = d.L;
  const S* G = matp<S>(d, mat);
  __shared__ double red[4];
  const double twopiL = 2.0 * M_PI / L;
  double sn = 0, sD = 0, sdc = 0;
  double zsum[2] = {0, 0}, zc[2] = {0, 0}, zs[2] = {0, 0};
  for (int i = threadIdx.x; i < N; i += MT) {
    S g = G[i + (size_t)i * N];
    S a = ST<S>::one() - g;
    S b = conjg(g);
    double ab = real_part(a * b);
    double z = 1.0 - 2.0 * real_part(g);
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
  double pG = 0, pK = 0;
  const int nstrip = 2 * ((Nc + PB - 1) / PB);
  for (int x = threadIdx.x; x < nstrip; x += MT) {
    pG += d.vec[VEC_NORM][2 * x];
    pK += d.vec[VEC_NORM][2 * x + 1];
  }
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
  tk = bsum(tk, red);
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
    for (int k = 0; k < OBS_COUNT; ++k) {
      d.obs[k] += v[k];
      d.obs[OBS_COUNT + k] += v[k];
    }
    d.obs[2 * OBS_COUNT] += 1.0;
    st->n_meas += 1;
  }
}

}  // namespace

hipError_t launch_measure(const InstDev* insts, int n_inst, int Nmax, bool cplx_, int mat, hipStream_t s) {
  const int ncm = Nmax / 2;
  dim3 grid(2 * ((ncm + PB - 1) / PB), n_inst);
  if (cplx_) hipLaunchKernelGGL(k_measure_pairs<cplx>, grid, dim3(MT), 0, s, insts, mat);
  else hipLaunchKernelGGL(k_measure_pairs<double>, grid, dim3(MT), 0, s, insts, mat);
  if (cplx_) hipLaunchKernelGGL(k_measure<cplx>, dim3(1, n_inst), dim3(MT), 0, s, insts, mat);
  else hipLaunchKernelGGL(k_measure<double>, dim3(1, n_inst), dim3(MT), 0, s, insts, mat);
  return hipGetLastError();
}
