// Periodic recomputation of G from UDV factors (Sec. II B: the stable
// evaluation of eq. GrFMat with periodic QR stabilisation of L and R).
//
// Chain step (every n_stab slices):  A = B_chunk U D  ->  columns sorted by
// norm (pre-pivoting)  ->  blocked Householder QR A P = Q R  ->  U' = Q,
// D' = |diag R|, T' = D'^{-1} R P^T T.  The upward pass advances R = U D T,
// the downward pass advances L^dagger = U D T.
// Recompute:  G = U_L D_Lb^{-1} Y^{-1} D_Rb^{-1} U_R^dagger with
//   Y = D_Rb^{-1} U_R^dagger U_L D_Lb^{-1} + D_Rs T_R T_L^dagger D_Ls,
// D = D_b D_s split into factors max(D,1), min(D,1).  Y^{-1} is applied by a
// second Householder QR and an upper-triangular solve.
//
// Dense products run on the MFMA GEMM; this file holds the panel
// factorisation, the triangular block solve, the pre-pivot sort and the
// element-wise steps.
#include "common.hpp"
#include "kernels.hpp"

namespace {

constexpr int EW_THREADS = 256;

__device__ __forceinline__ void atomic_max_pos(double* addr, double v) {
  // non-negative doubles order like their bit patterns
  atomicMax(reinterpret_cast<unsigned long long*>(addr), (unsigned long long)__double_as_longlong(v));
}

template <typename S>
__device__ __forceinline__ double absval(S v) { return sqrt(absq(v)); }

template <typename S>
__global__ void __launch_bounds__(EW_THREADS)
k_elem(const InstDev* __restrict__ insts, ElemArgs e) {
  const InstDev& d = insts[blockIdx.y];
  InstState* st = d.st;
  const int N = d.N;
  const size_t NN = (size_t)N * N;
  const size_t stride = (size_t)gridDim.x * EW_THREADS;
  const size_t e0 = (size_t)blockIdx.x * EW_THREADS + threadIdx.x;
  if (st->idle && e.op != EO_STACK_IDENTITY && e.op != EO_IDENTITY && e.op != EO_SET_ONES) return;
  switch (e.op) {
    case EO_COPY: {
      const S* a = matp<S>(d, e.a);
      S* c = matp<S>(d, e.c);
      for (size_t x = e0; x < NN; x += stride) c[x] = a[x];
      break;
    }
    case EO_IDENTITY: {
      S* c = matp<S>(d, e.c);
      for (size_t x = e0; x < NN; x += stride) c[x] = (x % N == x / N) ? ST<S>::one() : ST<S>::zero();
      break;
    }
    case EO_SCALE_COLS: {
      S* c = matp<S>(d, e.c);
      const double* v = vec_ptr(d, e.v);
      for (size_t x = e0; x < NN; x += stride) c[x] = c[x] * v[x / N];
      break;
    }
    case EO_SCALE_ROWS_INV: {
      S* c = matp<S>(d, e.c);
      const double* v = vec_ptr(d, e.v);
      for (size_t x = e0; x < NN; x += stride) c[x] = c[x] * (1.0 / v[x % N]);
      break;
    }
    case EO_SCALE_ROWS_DLB: {
      S* c = matp<S>(d, e.c);
      const double* v = vec_ptr(d, VEC_LD);
      for (size_t x = e0; x < NN; x += stride) c[x] = c[x] * (1.0 / fmax(v[x % N], 1.0));
      break;
    }
    case EO_GATHER_COLS: {
      const S* a = matp<S>(d, e.a);
      S* c = matp<S>(d, e.c);
      for (size_t x = e0; x < NN; x += stride) {
        size_t i = x % N, j = x / N;
        c[x] = a[i + (size_t)d.perm[j] * N];
      }
      break;
    }
    case EO_GATHER_ROWS: {
      const S* a = matp<S>(d, e.a);
      S* c = matp<S>(d, e.c);
      for (size_t x = e0; x < NN; x += stride) {
        size_t i = x % N, j = x / N;
        c[x] = a[(size_t)d.perm[i] + j * N];
      }
      break;
    }
    case EO_BUILD_Y: {
      const S* a = matp<S>(d, e.a);
      const S* b = matp<S>(d, e.b);
      S* c = matp<S>(d, e.c);
      const double* dr = vec_ptr(d, VEC_RD);
      const double* dl = vec_ptr(d, VEC_LD);
      for (size_t x = e0; x < NN; x += stride) {
        size_t i = x % N, j = x / N;
        double rb = fmax(dr[i], 1.0), rs = fmin(dr[i], 1.0);
        double lb = fmax(dl[j], 1.0), ls = fmin(dl[j], 1.0);
        c[x] = a[x] * (1.0 / (rb * lb)) + b[x] * (rs * ls);
      }
      break;
    }
    case EO_BUILD_RHS: {
      const S* u = matp<S>(d, MAT_RU);
      S* c = matp<S>(d, e.c);
      const double* dr = vec_ptr(d, VEC_RD);
      for (size_t x = e0; x < NN; x += stride) {
        size_t i = x % N, j = x / N;
        c[x] = conjg(u[j + i * N]) * (1.0 / fmax(dr[i], 1.0));
      }
      break;
    }
    case EO_STACK_STORE: {
      int c = sched_ckpt(st->phase, d.M, d.n_stab);
      if (c < 1 || c > d.n_ckpt - 1) break;
      const S* u = matp<S>(d, MAT_UW);
      const S* t = matp<S>(d, MAT_TW);
      S* su = matp<S>(d, MAT_SU);
      S* stt = matp<S>(d, MAT_ST);
      for (size_t x = e0; x < NN; x += stride) { su[x] = u[x]; stt[x] = t[x]; }
      const double* dw = d.vec[VEC_DW];
      double* sd = vec_ptr(d, VEC_SD);
      for (size_t x = e0; x < (size_t)N; x += stride) sd[x] = dw[x];
      break;
    }
    case EO_STACK_IDENTITY: {
      size_t tot = NN * (size_t)(d.n_ckpt + 1);
      S* su = reinterpret_cast<S*>(d.stackU);
      S* stt = reinterpret_cast<S*>(d.stackT);
      for (size_t x = e0; x < tot; x += stride) {
        size_t y = x % NN;
        S v = (y % N == y / N) ? ST<S>::one() : ST<S>::zero();
        su[x] = v;
        stt[x] = v;
      }
      for (size_t x = e0; x < (size_t)N * (d.n_ckpt + 1); x += stride) d.stackD[x] = 1.0;
      break;
    }
    case EO_RESET_CHAIN: {
      int c = sched_ckpt(st->phase, d.M, d.n_stab);
      int first = sched_is_up(st->phase, d.M) ? (c == 1) : (c == d.n_ckpt - 1);
      if (!first) break;
      S* u = matp<S>(d, MAT_UW);
      S* t = matp<S>(d, MAT_TW);
      for (size_t x = e0; x < NN; x += stride) {
        S v = (x % N == x / N) ? ST<S>::one() : ST<S>::zero();
        u[x] = v;
        t[x] = v;
      }
      double* dw = d.vec[VEC_DW];
      for (size_t x = e0; x < (size_t)N; x += stride) dw[x] = 1.0;
      break;
    }
    case EO_SET_ONES: {
      double* v = vec_ptr(d, e.v);
      for (size_t x = e0; x < (size_t)N; x += stride) v[x] = 1.0;
      break;
    }
    case EO_DRIFT_REPLACE: {
      S* g = matp<S>(d, MAT_G);
      const S* gs = matp<S>(d, MAT_GS);
      double m = 0.0;
      for (size_t x = e0; x < NN; x += stride) {
        S diff = g[x] - gs[x];
        double a = absval(diff);
        if (!(a == a)) a = INFINITY;
        m = fmax(m, a);
        g[x] = gs[x];
      }
      if (!st->init_mode) {
        for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
        if ((threadIdx.x & 63) == 0) {
          atomic_max_pos(&st->drift_last, m);
          atomic_max_pos(&st->drift_max, m);
        }
      }
      break;
    }
  }
}

// ---- pre-pivoting: column norms, then a stable descending sort --------------------------
template <typename S>
__global__ void __launch_bounds__(256) k_colnorm_sort(const InstDev* __restrict__ insts, int mat) {
  const InstDev& d = insts[blockIdx.y];
  if (d.st->idle) return;
  const int N = d.N;
  const S* A = matp<S>(d, mat);
  __shared__ double key[4096];
  __shared__ int idx[4096];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) d.st->drift_last = 0.0;
  for (int j = wave; j < N; j += 4) {
    double s = 0.0;
    for (int i = lane; i < N; i += 64) s += absq(A[i + (size_t)j * N]);
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) { key[j] = s; idx[j] = j; }
  }
  int P = 1;
  while (P < N) P <<= 1;
  for (int j = N + threadIdx.x; j < P; j += 256) { key[j] = -1.0; idx[j] = j; }
  __syncthreads();
  // bitonic sort: descending key, ascending index among equal keys
  for (int k = 2; k <= P; k <<= 1) {
    for (int jj = k >> 1; jj > 0; jj >>= 1) {
      for (int i = threadIdx.x; i < P; i += 256) {
        int ixj = i ^ jj;
        if (ixj > i) {
          bool before = key[i] > key[ixj] || (key[i] == key[ixj] && idx[i] < idx[ixj]);
          bool dirdesc = (i & k) == 0;
          if (dirdesc ? !before : before) {
            double tk = key[i]; key[i] = key[ixj]; key[ixj] = tk;
            int ti = idx[i]; idx[i] = idx[ixj]; idx[ixj] = ti;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int j = threadIdx.x; j < N; j += 256) d.perm[j] = idx[j];
}

// ---- Householder panel factorisation (one workgroup per instance) ---------------------------
// Columns [j0, j0 + nbe) of MAT_QA: H_j = I - tau_j v_j v_j^H with v_j[j] = 1,
// H_j^H applied from the left; beta = -sign(Re alpha) ||(alpha, x)||.
// Writes explicit V (MAT_V) and the compact-WY factor T (MAT_TB), so that
// H_j0 ... H_{j0+nbe-1} = I - V T V^H.
constexpr int QR_T = 256;
constexpr int NBMAX = 32;

template <typename S>
__device__ __forceinline__ S block_sum(S v, S* red, int tid) {
  // reduce over 256 threads; red has 4 entries
  for (int off = 32; off > 0; off >>= 1) {
    if constexpr (ST<S>::is_complex) { v.x += __shfl_xor(v.x, off); v.y += __shfl_xor(v.y, off); }
    else v += __shfl_xor(v, off);
  }
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

template <typename S>
__global__ void __launch_bounds__(QR_T) k_qr_panel(const InstDev* __restrict__ insts, int p, int nb) {
  const InstDev& d = insts[blockIdx.y];
  if (d.st->idle) return;
  const int N = d.N;
  const int j0 = p * nb;
  if (j0 >= N) return;
  const int nbe = min(nb, N - j0);
  S* A = matp<S>(d, MAT_QA);
  S* V = matp<S>(d, MAT_V);
  S* TB = matp<S>(d, MAT_TB);
  double* tauv = d.vec[VEC_TAU];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ S red[4];
  __shared__ S part[4][NBMAX];
  __shared__ S wsum[NBMAX];
  __shared__ S tau_s[NBMAX];
  __shared__ S Tm[NBMAX][NBMAX + 1];
  __shared__ S sh_scal;

  for (int jj = 0; jj < nbe; ++jj) {
    const int j = j0 + jj;
    // norm of the sub-diagonal part
    double xs = 0.0;
    for (int i = j + 1 + tid; i < N; i += QR_T) xs += absq(A[i + (size_t)j * N]);
    double xn2 = block_sum<double>(xs, reinterpret_cast<double*>(red), tid);
    if (tid == 0) {
      S alpha = A[j + (size_t)j * N];
      S tau, scal;
      if (xn2 == 0.0 && imag_part(alpha) == 0.0) {
        tau = ST<S>::zero();
        scal = ST<S>::one();
      } else {
        double ar = real_part(alpha);
        double nrm = sqrt(absq(alpha) + xn2);
        double beta = ar >= 0.0 ? -nrm : nrm;
        S bS = ST<S>::from_re(beta);
        tau = cdiv(bS - alpha, bS);
        scal = cdiv(ST<S>::one(), alpha - bS);
        A[j + (size_t)j * N] = bS;
      }
      tau_s[jj] = tau;
      sh_scal = scal;
    }
    __syncthreads();
    const S scal = sh_scal;
    const S ctau = conjg(tau_s[jj]);
    for (int i = j + 1 + tid; i < N; i += QR_T) A[i + (size_t)j * N] = A[i + (size_t)j * N] * scal;
    __syncthreads();
    // w_c = v^H A[j:, c] for the remaining panel columns
    const int nc = nbe - jj - 1;
    if (nc > 0) {
      S acc[NBMAX];
#pragma unroll
      for (int c = 0; c < NBMAX; ++c) acc[c] = ST<S>::zero();
      for (int i = j + tid; i < N; i += QR_T) {
        S vi = (i == j) ? ST<S>::one() : A[i + (size_t)j * N];
        S cv = conjg(vi);
#pragma unroll
        for (int c = 0; c < NBMAX; ++c)
          if (c < nc) acc[c] = acc[c] + cv * A[i + (size_t)(j + 1 + c) * N];
      }
#pragma unroll
      for (int c = 0; c < NBMAX; ++c) {
        if (c < nc) {
          S v = acc[c];
          for (int off = 32; off > 0; off >>= 1) {
            if constexpr (ST<S>::is_complex) { v.x += __shfl_xor(v.x, off); v.y += __shfl_xor(v.y, off); }
            else v += __shfl_xor(v, off);
          }
          if (lane == 0) part[wave][c] = v;
        }
      }
      __syncthreads();
      if (tid < nc) wsum[tid] = part[0][tid] + part[1][tid] + part[2][tid] + part[3][tid];
      __syncthreads();
      for (int i = j + tid; i < N; i += QR_T) {
        S vi = (i == j) ? ST<S>::one() : A[i + (size_t)j * N];
        S f = ctau * vi;
        for (int c = 0; c < nc; ++c) {
          size_t o = i + (size_t)(j + 1 + c) * N;
          A[o] = A[o] - f * wsum[c];
        }
      }
      __syncthreads();
    }
  }
  // explicit V and tau
  for (int jj = 0; jj < nbe; ++jj) {
    const int j = j0 + jj;
    for (int i = j0 + tid; i < N; i += QR_T) {
      S v = i < j ? ST<S>::zero() : (i == j ? ST<S>::one() : A[i + (size_t)j * N]);
      V[i + (size_t)j * N] = v;
    }
  }
  if (tid < nbe) tauv[2 * (j0 + tid)] = real_part(tau_s[tid]), tauv[2 * (j0 + tid) + 1] = imag_part(tau_s[tid]);
  __syncthreads();
  // T (forward, columnwise): T[jj][jj] = tau_jj, T[0:jj, jj] = -tau_jj T[0:jj, 0:jj] V[:, 0:jj]^H v_jj
  for (int r = tid; r < NBMAX * (NBMAX + 1); r += QR_T) (&Tm[0][0])[r] = ST<S>::zero();
  __syncthreads();
  for (int jj = 0; jj < nbe; ++jj) {
    const int j = j0 + jj;
    if (jj > 0) {
      S acc[NBMAX];
#pragma unroll
      for (int m = 0; m < NBMAX; ++m) acc[m] = ST<S>::zero();
      for (int i = j + tid; i < N; i += QR_T) {
        S vj = V[i + (size_t)j * N];
#pragma unroll
        for (int m = 0; m < NBMAX; ++m)
          if (m < jj) acc[m] = acc[m] + conjg(V[i + (size_t)(j0 + m) * N]) * vj;
      }
#pragma unroll
      for (int m = 0; m < NBMAX; ++m) {
        if (m < jj) {
          S v = acc[m];
          for (int off = 32; off > 0; off >>= 1) {
            if constexpr (ST<S>::is_complex) { v.x += __shfl_xor(v.x, off); v.y += __shfl_xor(v.y, off); }
            else v += __shfl_xor(v, off);
          }
          if (lane == 0) part[wave][m] = v;
        }
      }
      __syncthreads();
      if (tid < jj) wsum[tid] = part[0][tid] + part[1][tid] + part[2][tid] + part[3][tid];
      __syncthreads();
      if (tid < jj) {
        S s = ST<S>::zero();
        for (int m = tid; m < jj; ++m) s = s + Tm[tid][m] * wsum[m];
        Tm[tid][jj] = -(tau_s[jj] * s);
      }
    }
    if (tid == 0) Tm[jj][jj] = tau_s[jj];
    __syncthreads();
  }
  for (int x = tid; x < nbe * nbe; x += QR_T) {
    int r = x % nbe, c = x / nbe;
    TB[(j0 + r) + (size_t)c * N] = Tm[r][c];
  }
}

template <typename S>
__global__ void k_diag_abs(const InstDev* __restrict__ insts) {
  const InstDev& d = insts[blockIdx.y];
  if (d.st->idle) return;
  const S* A = matp<S>(d, MAT_QA);
  double* D = d.vec[VEC_DW];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < d.N; i += gridDim.x * blockDim.x)
    D[i] = sqrt(absq(A[i + (size_t)i * d.N]));
}

// Upper-triangular solve on one 32-row block of MAT_W3, R from MAT_QA:
// rows [i0, i1), i1 = N - 32 blk; each thread owns one column.
constexpr int TB_ROWS = 32;
template <typename S>
__global__ void __launch_bounds__(256) k_trsm_diag(const InstDev* __restrict__ insts, int blk) {
  const InstDev& d = insts[blockIdx.y];
  if (d.st->idle) return;
  const int N = d.N;
  const int i1 = N - TB_ROWS * blk;
  if (i1 <= 0) return;
  const int i0 = max(0, i1 - TB_ROWS);
  const int nr = i1 - i0;
  const S* R = matp<S>(d, MAT_QA);
  S* B = matp<S>(d, MAT_W3);
  __shared__ S Rb[TB_ROWS][TB_ROWS + 1];
  for (int x = threadIdx.x; x < nr * nr; x += blockDim.x) {
    int r = x % nr, c = x / nr;
    Rb[r][c] = R[(i0 + r) + (size_t)(i0 + c) * N];
  }
  __syncthreads();
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  S z[TB_ROWS];
#pragma unroll
  for (int r = 0; r < TB_ROWS; ++r) z[r] = r < nr ? B[(i0 + r) + (size_t)j * N] : ST<S>::zero();
#pragma unroll
  for (int r = TB_ROWS - 1; r >= 0; --r) {
    if (r < nr) {
      S s = z[r];
#pragma unroll
      for (int c = r + 1; c < TB_ROWS; ++c)
        if (c < nr) s = s - Rb[r][c] * z[c];
      z[r] = cdiv(s, Rb[r][r]);
    }
  }
#pragma unroll
  for (int r = 0; r < TB_ROWS; ++r)
    if (r < nr) B[(i0 + r) + (size_t)j * N] = z[r];
}

}  // namespace

hipError_t launch_elem(const InstDev* insts, int n_inst, int Nmax, bool cplx_, ElemArgs e, hipStream_t s) {
  size_t NN = (size_t)Nmax * Nmax;
  int gx = (int)((NN + EW_THREADS * 4 - 1) / (EW_THREADS * 4));
  if (gx > 2048) gx = 2048;
  if (gx < 1) gx = 1;
  dim3 grid(gx, n_inst);
  if (cplx_) hipLaunchKernelGGL(k_elem<cplx>, grid, dim3(EW_THREADS), 0, s, insts, e);
  else hipLaunchKernelGGL(k_elem<double>, grid, dim3(EW_THREADS), 0, s, insts, e);
  return hipGetLastError();
}

hipError_t launch_colnorm_sort(const InstDev* insts, int n_inst, int Nmax, bool cplx_, int mat, hipStream_t s) {
  (void)Nmax;
  if (cplx_) hipLaunchKernelGGL(k_colnorm_sort<cplx>, dim3(1, n_inst), dim3(256), 0, s, insts, mat);
  else hipLaunchKernelGGL(k_colnorm_sort<double>, dim3(1, n_inst), dim3(256), 0, s, insts, mat);
  return hipGetLastError();
}

hipError_t launch_qr_panel(const InstDev* insts, int n_inst, bool cplx_, int p, int nb, hipStream_t s) {
  if (nb > NBMAX) return hipErrorInvalidValue;
  if (cplx_) hipLaunchKernelGGL(k_qr_panel<cplx>, dim3(1, n_inst), dim3(QR_T), 0, s, insts, p, nb);
  else hipLaunchKernelGGL(k_qr_panel<double>, dim3(1, n_inst), dim3(QR_T), 0, s, insts, p, nb);
  return hipGetLastError();
}

hipError_t launch_diag_abs(const InstDev* insts, int n_inst, int Nmax, bool cplx_, hipStream_t s) {
  dim3 grid((Nmax + 255) / 256, n_inst);
  if (cplx_) hipLaunchKernelGGL(k_diag_abs<cplx>, grid, dim3(256), 0, s, insts);
  else hipLaunchKernelGGL(k_diag_abs<double>, grid, dim3(256), 0, s, insts);
  return hipGetLastError();
}

hipError_t launch_trsm_diag(const InstDev* insts, int n_inst, int Nmax, bool cplx_, int blk, hipStream_t s) {
  dim3 grid((Nmax + 255) / 256, n_inst);
  if (cplx_) hipLaunchKernelGGL(k_trsm_diag<cplx>, grid, dim3(256), 0, s, insts, blk);
  else hipLaunchKernelGGL(k_trsm_diag<double>, grid, dim3(256), 0, s, insts, blk);
  return hipGetLastError();
}
