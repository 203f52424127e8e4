// FFT propagation of the kinetic factor (Sec. III A, eqs. NewBlMat,
// ExpLambda, FourierMat, ColumnDem).
//
// exp(-+dtau K) = F^dagger T F per sublattice pair, with F the unnormalised
// 2-D DFT over the L x L cell grid (forward sign e^{-i k.r}, plain momenta
// k = (l1 b1 + l2 b2)/L) and T(k) the 2x2 table exp(-+dtau h(k+A))/N_c.  A
// twist only enters through the table, because the momentum grid of eq.
// kpoints is the plain grid shifted by the vector potential A.
//
// One workgroup transforms nv vectors (columns, or rows) of one instance held
// in LDS: optional diagonal, forward 2-D FFT on both sublattices (mixed-radix
// Stockham, one radix per stage, in place with register staging), 2x2 block
// multiply per momentum, inverse 2-D FFT, optional diagonal, store.  Real
// matrices pack two real vectors as one complex vector (the operator is real).
// Rows are transformed with the transpose: E^T = conj(E) for Hermitian K, so a
// row is conjugated on load and on store.
#include "common.hpp"
#include "kernels.hpp"

namespace {

constexpr int FFT_THREADS = 256;
constexpr int FFT_REGS = 16;  // complex values staged per thread per stage

struct Resolved {
  int active, slice, pre, post, tab;
};

__device__ __forceinline__ Resolved resolve(const InstDev& d, const FftArgs& a) {
  Resolved r{0, 0, 0, 0, TAB_P};
  const InstState& st = *d.st;
  if (st.idle) return r;
  int M = d.M;
  int up = sched_is_up(st.phase, M);
  int l = sched_slice(st.phase, M);
  switch (a.op) {
    case FOP_WRAP_PRE:  // G <- e^{V} E+ G E- e^{-V} before updating slice l (upward)
      if (!up || st.init_mode) return r;
      r.active = 1; r.slice = l;
      if (a.side == 0) { r.pre = 0; r.tab = TAB_P; r.post = +1; }
      else { r.pre = 0; r.tab = TAB_M; r.post = -1; }
      return r;
    case FOP_WRAP_POST:  // G <- E- e^{-V} G e^{V} E+ after updating slice l (downward)
      if (up || st.init_mode) return r;
      r.active = 1; r.slice = l;
      if (a.side == 0) { r.pre = -1; r.tab = TAB_M; r.post = 0; }
      else { r.pre = +1; r.tab = TAB_P; r.post = 0; }
      return r;
    case FOP_STAB_B: {  // columns of the working U: B (upward) or B^dagger (downward)
      if (a.side != 0) return r;
      int c = sched_ckpt(st.phase, M, d.n_stab);
      r.active = 1;
      if (up) {  // R_c = B_{c ns} .. B_{(c-1) ns + 1} R_{c-1}: lowest slice first
        r.slice = (c - 1) * d.n_stab + 1 + a.j;
        r.pre = 0; r.tab = TAB_P; r.post = +1;
      } else {   // L_c^dag = B^dag_{c ns+1} .. B^dag_{(c+1) ns} L_{c+1}^dag: highest first
        r.slice = c * d.n_stab + d.n_stab - a.j;
        r.pre = +1; r.tab = TAB_P; r.post = 0;
      }
      return r;
    }
    case FOP_HALF:  // G~ = e^{-dtau K/2} G e^{+dtau K/2}
      r.active = 1; r.slice = 0;
      r.tab = (a.side == 0) ? TAB_HP : TAB_HM;
      return r;
    case FOP_EXPLICIT:
      r.active = 1; r.slice = a.ex_slice; r.pre = a.ex_pre; r.post = a.ex_post; r.tab = a.ex_tab;
      return r;
  }
  return r;
}

__device__ __forceinline__ cplx root_pow(const cplx* roots, int L, int m, int sign) {
  cplx w = roots[m % L];
  return sign < 0 ? w : conjg(w);
}

// One Stockham stage of radix R on all lines of the nv vectors in LDS.
template <int R>
__device__ void fft_stage(cplx* buf, const cplx* roots, int L, int Nc, int N, int nv,
                          int axis, int Ns, int sign) {
  constexpr int MAXB = (FFT_REGS + R - 1) / R;
  const int per_line = L / R;
  const int nlines = nv * 2 * L;
  const int nb = nlines * per_line;
  const int estride = axis == 0 ? 1 : L;
  const int ostride = axis == 0 ? L : 1;
  cplx v[MAXB][R];
  int dst[MAXB];
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    int b = threadIdx.x + q * FFT_THREADS;
    dst[q] = -1;
    if (b < nb) {
      int line = b / per_line, j = b - line * per_line;
      int vv = line / (2 * L);
      int rem = line - vv * 2 * L;
      int s = rem / L, o = rem - s * L;
      int base = vv * N + s * Nc + o * ostride;
      int jm = j % Ns;
      int tw = (L / (Ns * R)) * jm;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        cplx x = buf[base + (j + r * per_line) * estride];
        v[q][r] = r ? x * root_pow(roots, L, tw * r, sign) : x;
      }
      // R-point DFT
      cplx out[R];
#pragma unroll
      for (int s2 = 0; s2 < R; ++s2) {
        cplx acc = v[q][0];
#pragma unroll
        for (int r = 1; r < R; ++r) acc = acc + v[q][r] * root_pow(roots, L, (L / R) * ((r * s2) % R), sign);
        out[s2] = acc;
      }
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = out[r];
      dst[q] = base + ((j / Ns) * Ns * R + jm) * estride;
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    if (dst[q] >= 0) {
      int ostep = (axis == 0 ? 1 : L);
      // outputs of one butterfly are Ns apart along the line
#pragma unroll
      for (int r = 0; r < R; ++r) buf[dst[q] + r * Ns * ostep] = v[q][r];
    }
  }
  __syncthreads();
}

__device__ void fft_2d(cplx* buf, const cplx* roots, const int* fac, int L, int Nc, int N,
                       int nv, int sign) {
  for (int axis = 0; axis < 2; ++axis) {
    int Ns = 1;
    for (int f = 0; fac[f]; ++f) {
      int R = fac[f];
      switch (R) {
        case 2: fft_stage<2>(buf, roots, L, Nc, N, nv, axis, Ns, sign); break;
        case 3: fft_stage<3>(buf, roots, L, Nc, N, nv, axis, Ns, sign); break;
        case 4: fft_stage<4>(buf, roots, L, Nc, N, nv, axis, Ns, sign); break;
        case 5: fft_stage<5>(buf, roots, L, Nc, N, nv, axis, Ns, sign); break;
        case 7: fft_stage<7>(buf, roots, L, Nc, N, nv, axis, Ns, sign); break;
        case 11: fft_stage<11>(buf, roots, L, Nc, N, nv, axis, Ns, sign); break;
        case 13: fft_stage<13>(buf, roots, L, Nc, N, nv, axis, Ns, sign); break;
        default: break;  // rejected on the host
      }
      Ns *= R;
    }
  }
}

template <typename S>
__global__ void __launch_bounds__(FFT_THREADS)
k_fft_apply(const InstDev* __restrict__ insts, FftArgs a, int nv) {
  extern __shared__ char smem_raw[];
  const InstDev& d = insts[blockIdx.y];
  Resolved rs = resolve(d, a);
  if (!rs.active) return;
  const int N = d.N, Nc = d.Nc, L = d.L;
  const int nvec = ST<S>::is_complex ? N : N / 2;
  const int v0 = blockIdx.x * nv;
  if (v0 >= nvec) return;
  const int nvl = min(nv, nvec - v0);
  cplx* buf = reinterpret_cast<cplx*>(smem_raw);
  __shared__ cplx roots[64];
  __shared__ int fac[16];
  __shared__ double dpre[1], dpost[1];
  (void)dpre; (void)dpost;
  if (threadIdx.x < L) roots[threadIdx.x] = d.roots[threadIdx.x];
  if (threadIdx.x < 16) fac[threadIdx.x] = d.factors[threadIdx.x];
  S* Mx = matp<S>(d, a.mat);
  const int8_t* xs = rs.slice > 0 ? d.fields + (size_t)(rs.slice - 1) * N : nullptr;
  const double lam = d.lam;
  const bool rows = a.side != 0;
  // load (+ pre diagonal)
  const int tot = nvl * N;
  for (int e = threadIdx.x; e < tot; e += FFT_THREADS) {
    int vv, r;
    if (!rows) { vv = e / N; r = e - vv * N; }
    else { vv = e % nvl; r = e / nvl; }
    int q = v0 + vv;
    cplx val;
    if constexpr (ST<S>::is_complex) {
      cplx g = rows ? Mx[(size_t)r * N + q] : Mx[(size_t)q * N + r];
      val = rows ? conjg(g) : g;
    } else {
      if (!rows) val = cmake(Mx[(size_t)(2 * q) * N + r], Mx[(size_t)(2 * q + 1) * N + r]);
      else val = cmake(Mx[(size_t)r * N + 2 * q], Mx[(size_t)r * N + 2 * q + 1]);
    }
    if (rs.pre) val = val * exp(rs.pre * lam * (double)xs[r]);
    buf[vv * N + r] = val;
  }
  __syncthreads();
  fft_2d(buf, roots, fac, L, Nc, N, nvl, -1);
  // 2x2 block per momentum
  const cplx* T = d.tab + (size_t)rs.tab * Nc * 4;
  for (int e = threadIdx.x; e < nvl * Nc; e += FFT_THREADS) {
    int vv = e / Nc, k = e - vv * Nc;
    cplx qa = buf[vv * N + k], qb = buf[vv * N + Nc + k];
    cplx t00 = T[4 * k], t01 = T[4 * k + 1], t10 = T[4 * k + 2], t11 = T[4 * k + 3];
    buf[vv * N + k] = t00 * qa + t01 * qb;
    buf[vv * N + Nc + k] = t10 * qa + t11 * qb;
  }
  __syncthreads();
  fft_2d(buf, roots, fac, L, Nc, N, nvl, +1);
  // store (+ post diagonal)
  for (int e = threadIdx.x; e < tot; e += FFT_THREADS) {
    int vv, r;
    if (!rows) { vv = e / N; r = e - vv * N; }
    else { vv = e % nvl; r = e / nvl; }
    int q = v0 + vv;
    cplx val = buf[vv * N + r];
    if (rs.post) val = val * exp(rs.post * lam * (double)xs[r]);
    if constexpr (ST<S>::is_complex) {
      if (rows) Mx[(size_t)r * N + q] = conjg(val);
      else Mx[(size_t)q * N + r] = val;
    } else {
      if (!rows) { Mx[(size_t)(2 * q) * N + r] = val.x; Mx[(size_t)(2 * q + 1) * N + r] = val.y; }
      else { Mx[(size_t)r * N + 2 * q] = val.x; Mx[(size_t)r * N + 2 * q + 1] = val.y; }
    }
  }
}

}  // namespace

int fft_vectors_per_block(int N, size_t lds_budget) {
  int nv = (int)(lds_budget / ((size_t)N * sizeof(cplx)));
  int cap = (FFT_THREADS * FFT_REGS) / N;
  if (nv > cap) nv = cap;
  if (nv > 16) nv = 16;
  return nv < 1 ? 1 : nv;
}

hipError_t launch_fft(const InstDev* insts, int n_inst, int Nmax, bool cplx_, const FftArgs& a,
                      size_t lds_budget, hipStream_t s) {
  int nv = fft_vectors_per_block(Nmax, lds_budget);
  int nvec = cplx_ ? Nmax : Nmax / 2;
  dim3 grid((nvec + nv - 1) / nv, n_inst);
  size_t lds = (size_t)nv * Nmax * sizeof(cplx);
  if (cplx_) hipLaunchKernelGGL(k_fft_apply<cplx>, grid, dim3(FFT_THREADS), lds, s, insts, a, nv);
  else hipLaunchKernelGGL(k_fft_apply<double>, grid, dim3(FFT_THREADS), lds, s, insts, a, nv);
  return hipGetLastError();
}
