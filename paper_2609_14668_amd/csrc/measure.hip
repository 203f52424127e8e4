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
  // pair terms within each sublattice, i != j
  double pG = 0, pK = 0;
  for (size_t x = threadIdx.x; x < (size_t)2 * Nc * Nc; x += MT) {
    int sub = (int)(x / ((size_t)Nc * Nc));
    size_t y = x - (size_t)sub * Nc * Nc;
    int ii = (int)(y % Nc), jj = (int)(y / Nc);
    if (ii == jj) continue;
    int i = sub * Nc + ii, j = sub * Nc + jj;
    double re = real_part(G[i + (size_t)j * N] * G[j + (size_t)i * N]);
    pG += re;
    pK += re * cos(twopiL * ((jj % L) - (ii % L)));
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
    v[OBS_RM2_NUM] = Sdk; v[OBS_PHASE_RE] = 1.0; v[OBS_PHASE_IM] = 0.0;
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
  (void)Nmax;
  if (cplx_) hipLaunchKernelGGL(k_measure<cplx>, dim3(1, n_inst), dim3(MT), 0, s, insts, mat);
  else hipLaunchKernelGGL(k_measure<double>, dim3(1, n_inst), dim3(MT), 0, s, insts, mat);
  return hipGetLastError();
}
