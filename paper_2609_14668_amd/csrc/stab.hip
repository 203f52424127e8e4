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
#include <algorithm>

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

typedef double d4 __attribute__((ext_vector_type(4)));
template <typename S>
__device__ __forceinline__ void split_s(S v, double& re, double& im);
template <>
__device__ __forceinline__ void split_s<double>(double v, double& re, double& im) { re = v; im = 0.0; }
template <>
__device__ __forceinline__ void split_s<cplx>(cplx v, double& re, double& im) { re = v.x; im = v.y; }

template <typename S>
__global__ void __launch_bounds__(EW_THREADS)
k_elem(const InstDev* __restrict__ insts, ElemArgs e) {
  const InstDev& d = insts[blockIdx.y];
  InstState* st = d.st;
  const int N = d.N;
  const size_t NN = (size_t)N * N;
  const size_t stride = (size_t)gridDim.x * EW_THREADS;
  const size_t e0 = (size_t)blockIdx.x * EW_THREADS + threadIdx.x;
  // idle instances skip everything, except the identity fills of the initial
  // stack build (an instance parked by a time-displaced pass may be in the
  // middle of a sweep: its working chain must survive)
  if (st->idle && !(st->init_mode && (e.op == EO_STACK_IDENTITY || e.op == EO_IDENTITY || e.op == EO_SET_ONES)))
    return;
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
      for (size_t x = e0; x < (size_t)N; x += stride) d.perm[N + x] = (int)x;   // row order of the LU
      for (size_t x = e0; x < NN; x += stride) {
        size_t i = x % N, j = x / N;
        double rb = fmax(dr[i], 1.0), rs = fmin(dr[i], 1.0);
        double lb = fmax(dl[j], 1.0), ls = fmin(dl[j], 1.0);
        c[x] = a[x] * (1.0 / (rb * lb)) + b[x] * (rs * ls);
      }
      break;
    }
    case EO_BUILD_RHS: {   // v = 1: rows in the LU's order, row i from row perm[N + i]
      const S* u = matp<S>(d, MAT_RU);
      S* c = matp<S>(d, e.c);
      const double* dr = vec_ptr(d, VEC_RD);
      const int* rp = d.perm + N;
      for (size_t x = e0; x < NN; x += stride) {
        size_t i = x % N, j = x / N;
        if (e.v) i = (size_t)rp[i];
        c[x] = conjg(u[j + i * N]) * (1.0 / fmax(dr[i], 1.0));
      }
      break;
    }
    case EO_STACK_STORE: {
      int c = sched_ckpt(st->phase, d.M, d.n_stab);
      if (c < 1 || c > d.n_ckpt - 1) break;
      if (e0 == 0) {
        d.stackPh[2 * c] = st->phw_re;
        d.stackPh[2 * c + 1] = st->phw_im;
      }
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
      for (size_t x = e0; x < (size_t)(d.n_ckpt + 1); x += stride) {
        d.stackPh[2 * x] = 1.0;
        d.stackPh[2 * x + 1] = 0.0;
      }
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
    case EO_TAU_INIT: {
      if (!st->tau_active) break;
      const S* g = matp<S>(d, MAT_G);
      S* gtt = matp<S>(d, MAT_GTT);
      S* gt0 = matp<S>(d, MAT_GT0);
      S* g0t = matp<S>(d, MAT_G0T);
      for (size_t x = e0; x < NN; x += stride) {
        const S v = g[x];
        gtt[x] = v;
        gt0[x] = v;
        g0t[x] = (x % N == x / N) ? v - ST<S>::one() : v;
      }
      break;
    }
    case EO_SCALE_ROWS_DL: {
      S* c = matp<S>(d, e.c);
      const double* v = vec_ptr(d, VEC_LD);
      for (size_t x = e0; x < NN; x += stride) c[x] = c[x] * v[x % N];
      break;
    }
    case EO_BUILD_RHS_T: {
      const S* t = matp<S>(d, MAT_RT);
      S* c = matp<S>(d, e.c);
      const double* dr = vec_ptr(d, VEC_RD);
      const int* rp = d.perm + N;
      for (size_t x = e0; x < NN; x += stride) {
        const size_t i = (size_t)rp[x % N], j = x / N;
        c[x] = t[i + j * N] * fmin(dr[i], 1.0);
      }
      break;
    }
    case EO_TAU_REPLACE: {
      S* gtt = matp<S>(d, MAT_GTT);
      S* gt0 = matp<S>(d, MAT_GT0);
      S* g0t = matp<S>(d, MAT_G0T);
      const S* gs = matp<S>(d, MAT_GS);
      const S* w2 = matp<S>(d, MAT_W2);
      const S* w1 = matp<S>(d, MAT_W1);
      double m = 0.0;
      for (size_t x = e0; x < NN; x += stride) {
        double a = fmax(absval(gtt[x] - gs[x]), fmax(absval(gt0[x] - w2[x]), absval(g0t[x] - w1[x])));
        if (!(a == a)) a = INFINITY;
        m = fmax(m, a);
        gtt[x] = gs[x];
        gt0[x] = w2[x];
        g0t[x] = w1[x];
      }
      for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
      if ((threadIdx.x & 63) == 0) atomic_max_pos(&st->drift_acc, m);
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
        if ((threadIdx.x & 63) == 0) atomic_max_pos(&st->drift_acc, m);
      }
      break;
    }
  }
}

// ---- pre-pivoting: column norms, then a stable descending sort --------------------------
template <typename S>
__global__ void __launch_bounds__(256) k_colnorm(const InstDev* __restrict__ insts, int mat) {
  const InstDev& d = insts[blockIdx.y];
  if (d.st->idle) return;
  const int N = d.N;
  const S* A = matp<S>(d, mat);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (blockIdx.x == 0 && threadIdx.x == 0) d.st->drift_last = 0.0;
  // one wave per column, 16 columns per workgroup
  for (int u = 0; u < 4; ++u) {
    const int j = blockIdx.x * 16 + wave * 4 + u;
    if (j >= N) break;
    double s = 0.0;
    for (int i = lane; i < N; i += 64) s += absq(gld(A + i + (size_t)j * N));
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) d.vec[VEC_NORM][j] = s;
  }
}

// Pivot order of the pre-pivoted QR: columns by descending norm (ties by
// ascending index), one workgroup per instance, bitonic sort in LDS.
__global__ void __launch_bounds__(256) k_sort_cols(const InstDev* __restrict__ insts) {
  const InstDev& d = insts[blockIdx.y];
  if (d.st->idle) return;
  const int N = d.N;
  __shared__ double key[4096];
  __shared__ int idx[4096];
  int P = 1;
  while (P < N) P <<= 1;
  for (int j = threadIdx.x; j < P; j += 256) {
    key[j] = j < N ? d.vec[VEC_NORM][j] : -1.0;
    idx[j] = j;
  }
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

// Register-resident panel: thread t owns rows j0 + t + PT*q (q < RPT) of the
// NBR panel columns for the whole factorisation, so the column loop touches no
// global memory.  Per column one block-wide sum of 16 values (||x||^2 and
// x^H A[j+1:, c] for the later columns) with a single barrier: a butterfly
// transpose-sum across the 64 lanes of each wave, per-wave partials in LDS
// (double-buffered, so the next column may write while this one is read),
// and every thread adds the partials and forms the reflector itself.
// PT = 256 threads for up to 1024 rows, else 512 (two waves per SIMD).
constexpr int NBR = 16;

template <typename S, int PT>
struct PanelShared {
  S part[2][PT / 64][NBR];   // per-wave sums of the 16 values
  S totw[PT / 64][NBR];      // block totals, one copy per wave (read by that wave only)
  S rowj[2][NBR];            // the pivot row j of the panel
  S tau_s[NBR];
  S Tm[NBR][NBR + 1];
};

template <typename S>
__device__ __forceinline__ S shfl_x(S v, int m) {
  if constexpr (ST<S>::is_complex) return cmake(__shfl_xor(v.x, m), __shfl_xor(v.y, m));
  else return __shfl_xor(v, m);
}

// Wave-wide sums of acc[0..16): after the call lane l holds the sum of value
// (l >> 2) & 15 (17 exchanges instead of 16 x 6).
template <typename S>
__device__ __forceinline__ S wave_transpose_sum(const S (&acc)[NBR]) {
  const int lane = threadIdx.x & 63;
  S b8[8], b4[4], b2[2];
  {
    const bool hi = lane & 32;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const S send = hi ? acc[v] : acc[v + 8], keep = hi ? acc[v + 8] : acc[v];
      b8[v] = keep + shfl_x(send, 32);
    }
  }
  {
    const bool hi = lane & 16;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const S send = hi ? b8[v] : b8[v + 4], keep = hi ? b8[v + 4] : b8[v];
      b4[v] = keep + shfl_x(send, 16);
    }
  }
  {
    const bool hi = lane & 8;
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const S send = hi ? b4[v] : b4[v + 2], keep = hi ? b4[v + 2] : b4[v];
      b2[v] = keep + shfl_x(send, 8);
    }
  }
  const bool hi = lane & 4;
  S b1 = (hi ? b2[1] : b2[0]) + shfl_x(hi ? b2[0] : b2[1], 4);
  b1 = b1 + shfl_x(b1, 2);
  b1 = b1 + shfl_x(b1, 1);
  return b1;
}

// Publish the wave sums of acc into sh.part[buf] and wait for every wave.
template <typename S, int PT>
__device__ __forceinline__ void panel_publish(PanelShared<S, PT>& sh, const S (&acc)[NBR], int buf) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const S v = wave_transpose_sum<S>(acc);
  if ((lane & 3) == 0) sh.part[buf][wave][(lane >> 2) & 15] = v;
  __syncthreads();
}

// Block totals of the 16 published values into this wave's copy of totw:
// lanes 0..15 add the per-wave sums of one value each.  Only this wave reads
// its copy afterwards, and the LDS operations of one wave complete in order,
// so no further barrier is needed.
template <typename S, int PT>
__device__ __forceinline__ void panel_totals(PanelShared<S, PT>& sh, int buf) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane < NBR) {
    S t = sh.part[buf][0][lane];
#pragma unroll
    for (int w = 1; w < PT / 64; ++w) t = t + sh.part[buf][w][lane];
    sh.totw[wave][lane] = t;
  }
  __builtin_amdgcn_wave_barrier();
}

// Component-wise select (a struct-valued ?: can demote a register array to
// scratch memory).
__device__ __forceinline__ double psel(bool p, double a, double b) { return p ? a : b; }
__device__ __forceinline__ cplx psel(bool p, cplx a, cplx b) { return cmake(p ? a.x : b.x, p ? a.y : b.y); }

// Column JJ of the panel (compile-time, so the register array is indexed
// with constants and only the later columns are touched).  One barrier per
// column; every thread forms the reflector from the same shared values.
template <typename S, int RPT, int PT, int JJ>
struct PanelColumn {
  static __device__ __forceinline__ void run(S (&a)[RPT][NBR], PanelShared<S, PT>& sh, int j0, int N, int nbe) {
    if constexpr (JJ < NBR) {
      if (JJ < nbe) {
        constexpr int buf = JJ & 1;
        const int tid = threadIdx.x;
        const int j = j0 + JJ;
        // acc[0] = ||x||^2 below the diagonal, acc[c - JJ] = x^H A[j+1:, c]
        S acc[NBR];
#pragma unroll
        for (int c = 0; c < NBR; ++c) acc[c] = ST<S>::zero();
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          const int i = j0 + tid + PT * q;
          if (i > j && i < N) {
            const S x = a[q][JJ];
            const S cx = conjg(x);
            acc[0] = acc[0] + ST<S>::from_re(absq(x));
#pragma unroll
            for (int c = JJ + 1; c < NBR; ++c) acc[c - JJ] = acc[c - JJ] + cx * a[q][c];
          }
        }
        if (tid == JJ) {
#pragma unroll
          for (int c = JJ; c < NBR; ++c) sh.rowj[buf][c] = a[0][c];
        }
        panel_publish<S, PT>(sh, acc, buf);
        panel_totals<S, PT>(sh, buf);
        const S* tot = sh.totw[tid >> 6];
        const S alpha = sh.rowj[buf][JJ];
        const double xn2 = real_part(tot[0]);
        S tau, scal, bnew = alpha;
        if (xn2 == 0.0 && imag_part(alpha) == 0.0) {
          tau = ST<S>::zero();
          scal = ST<S>::one();
        } else {
          const double nrm = sqrt(absq(alpha) + xn2);
          const double beta = real_part(alpha) >= 0.0 ? -nrm : nrm;
          const S bS = ST<S>::from_re(beta);
          tau = cdiv(bS - alpha, bS);
          scal = cdiv(ST<S>::one(), alpha - bS);
          bnew = bS;
        }
        if (tid == 0) sh.tau_s[JJ] = tau;
        const S cscal = conjg(scal), ctau = conjg(tau);
        S w[NBR];
#pragma unroll
        for (int c = JJ + 1; c < NBR; ++c) w[c] = sh.rowj[buf][c] + cscal * tot[c - JJ];
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          const int i = j0 + tid + PT * q;
          if (i == j) {
            a[q][JJ] = bnew;
#pragma unroll
            for (int c = JJ + 1; c < NBR; ++c) a[q][c] = a[q][c] - ctau * w[c];
          } else if (i > j && i < N) {
            const S vi = a[q][JJ] * scal;
            a[q][JJ] = vi;
            const S f = ctau * vi;
#pragma unroll
            for (int c = JJ + 1; c < NBR; ++c) a[q][c] = a[q][c] - f * w[c];
          }
        }
      }
      PanelColumn<S, RPT, PT, JJ + 1>::run(a, sh, j0, N, nbe);
    }
  }
};

// Column JJ of the compact-WY factor T from the register-held V:
// T[0:JJ, JJ] = -tau_JJ T[0:JJ, 0:JJ] (V[:, 0:JJ]^H v_JJ).
template <typename S, int RPT, int PT, int JJ>
struct PanelT {
  static __device__ __forceinline__ void run(S (&a)[RPT][NBR], PanelShared<S, PT>& sh, int j0, int N, int nbe) {
    if constexpr (JJ < NBR) {
      if (JJ < nbe) {
        constexpr int buf = JJ & 1;
        const int tid = threadIdx.x;
        const int j = j0 + JJ;
        S acc[NBR];
#pragma unroll
        for (int m = 0; m < NBR; ++m) acc[m] = ST<S>::zero();
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          const int i = j0 + tid + PT * q;
          if (i >= j && i < N) {
            const S vj = i == j ? ST<S>::one() : a[q][JJ];
#pragma unroll
            for (int m = 0; m < JJ; ++m) acc[m] = acc[m] + conjg(a[q][m]) * vj;   // i > j0 + m
          }
        }
        panel_publish<S, PT>(sh, acc, buf);
        panel_totals<S, PT>(sh, buf);
        const S* tot = sh.totw[tid >> 6];
        if (tid < JJ) {
          S s2 = ST<S>::zero();
          for (int m = tid; m < JJ; ++m) s2 = s2 + (m == tid ? sh.tau_s[m] : sh.Tm[tid][m]) * tot[m];
          sh.Tm[tid][JJ] = -(sh.tau_s[JJ] * s2);
        }
      }
      PanelT<S, RPT, PT, JJ + 1>::run(a, sh, j0, N, nbe);
    }
  }
};

template <typename S, int RPT, int PT>
__global__ void __launch_bounds__(PT) k_qr_panel_reg(const InstDev* __restrict__ insts, int p) {
  const InstDev& d = insts[blockIdx.y];
  if (d.st->idle) return;
  const int N = d.N;
  const int j0 = p * NBR;
  if (j0 >= N) return;
  const int nbe = min(NBR, N - j0);
  S* A = matp<S>(d, MAT_QA);
  S* V = matp<S>(d, MAT_V);
  S* TB = matp<S>(d, MAT_TB);
  double* tauv = d.vec[VEC_TAU];
  const int tid = threadIdx.x;
  __shared__ PanelShared<S, PT> sh;

  // clamped loads issued back to back, masked afterwards
  S a[RPT][NBR];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int i = j0 + tid + PT * q;
#pragma unroll
    for (int c = 0; c < NBR; ++c) a[q][c] = gld(A + min(i, N - 1) + (size_t)(j0 + min(c, nbe - 1)) * N);
  }
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int i = j0 + tid + PT * q;
#pragma unroll
    for (int c = 0; c < NBR; ++c) a[q][c] = psel(i < N && c < nbe, a[q][c], ST<S>::zero());
  }
  for (int r = tid; r < NBR * (NBR + 1); r += PT) (&sh.Tm[0][0])[r] = ST<S>::zero();
  PanelColumn<S, RPT, PT, 0>::run(a, sh, j0, N, nbe);
  // write back R (upper part) and the Householder vectors, plus explicit V
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int i = j0 + tid + PT * q;
    if (i < N) {
#pragma unroll
      for (int c = 0; c < NBR; ++c) {
        if (c < nbe) {
          const int j = j0 + c;
          A[i + (size_t)j * N] = a[q][c];
          V[i + (size_t)j * N] = i < j ? ST<S>::zero() : (i == j ? ST<S>::one() : a[q][c]);
        }
      }
    }
  }
  __syncthreads();   // tau_s of the last column; part/totw free for the T pass
  if (tid < nbe) tauv[2 * (j0 + tid)] = real_part(sh.tau_s[tid]), tauv[2 * (j0 + tid) + 1] = imag_part(sh.tau_s[tid]);
  PanelT<S, RPT, PT, 1>::run(a, sh, j0, N, nbe);
  __syncthreads();   // the last column of Tm
  for (int x = tid; x < nbe * nbe; x += PT) {
    int r = x % nbe, c = x / nbe;
    TB[(j0 + r) + (size_t)c * N] = r == c ? sh.tau_s[r] : sh.Tm[r][c];
  }
}

// C <- (I - V op(T) V^H) C on rows [j0, N) and a range of columns of a
// target matrix, with the 16-column V and T of panel p (eq. of the compact-WY
// representation H_1..H_k = I - V T V^H):
//   W = V^H C (MFMA, rows staged through LDS), W' = op(T) W, C -= V W'.
// op(T) = T^H applies Q^H (QR trailing update, Q^H RHS), T applies Q (forming Q).
// cols: 0 -> [j0 + 16, N), 1 -> [j0, N), 2 -> [0, N).
constexpr int AR_CT = 64;
template <typename S>
__global__ void __launch_bounds__(256) k_apply_refl(const InstDev* __restrict__ insts, int p, int target,
                                                    int cols, int use_th) {
  constexpr bool CX = ST<S>::is_complex;
  const InstDev& d = insts[blockIdx.y];
  if (d.st->idle) return;
  const int N = d.N;
  const int j0 = p * NBR;
  if (j0 >= N) return;
  const int nbe = min(NBR, N - j0);
  const int cbeg = (cols == 0 || cols == 3) ? j0 + NBR : (cols == 1 ? j0 : 0);
  const int cend = cols == 3 ? min(N, j0 + 2 * NBR) : N;   // 3: the partner panel of a pair only
  const int c0 = cbeg + blockIdx.x * AR_CT;
  if (c0 >= cend) return;
  const S* V = matp<S>(d, MAT_V);
  const S* TB = matp<S>(d, MAT_TB);
  S* C = matp<S>(d, target);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  constexpr int RB = 32;   // rows of V and C staged per step
  __shared__ double Vr[RB][NBR + 1], Vi[CX ? RB : 1][NBR + 1];
  __shared__ double Cr[RB][AR_CT + 1], Ci[CX ? RB : 1][AR_CT + 1];
  __shared__ S Ws[NBR][AR_CT + 1];
  __shared__ S Tt[NBR][NBR + 1];
  // ---- W = V^H C: wave w owns columns 16w..16w+15 of the tile.  Each
  // thread stages 2 elements of V and 8 of C per row block; all loads read
  // clamped addresses and are issued before the first is used.
  constexpr int NV = RB * NBR / 256, NC = RB * AR_CT / 256;
  d4 wr = d4{0, 0, 0, 0}, wi = d4{0, 0, 0, 0};
#pragma unroll 1
  for (int i0 = j0; i0 < N; i0 += RB) {
    S vv[NV], cv[NC];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int x = tid + 256 * q, r = x % RB, m = x / RB;
      vv[q] = gld(V + min(i0 + r, N - 1) + (size_t)(j0 + min(m, nbe - 1)) * N);
    }
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      const int x = tid + 256 * q, r = x % RB, cc = x / RB;
      cv[q] = gld(C + min(i0 + r, N - 1) + (size_t)min(c0 + cc, cend - 1) * N);
    }
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int x = tid + 256 * q, r = x % RB, m = x / RB;
      const bool in = i0 + r < N && m < nbe;
      double re, im;
      split_s<S>(vv[q], re, im);
      Vr[r][m] = in ? re : 0.0;
      if constexpr (CX) Vi[r][m] = in ? im : 0.0;
    }
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      const int x = tid + 256 * q, r = x % RB, cc = x / RB;
      const bool in = i0 + r < N && c0 + cc < cend;
      double re, im;
      split_s<S>(cv[q], re, im);
      Cr[r][cc] = in ? re : 0.0;
      if constexpr (CX) Ci[r][cc] = in ? im : 0.0;
    }
    __syncthreads();
#pragma unroll 2
    for (int ks = 0; ks < RB / 4; ++ks) {
      const int k = ks * 4 + lk;
      // A = V^H: A[m][k] = conj(V[k][m]); B = C: B[k][c]
      double ar = Vr[k][lr], br = Cr[k][wave * 16 + lr];
      wr = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, wr, 0, 0, 0);
      if constexpr (CX) {
        double ai = -Vi[k][lr], bi = Ci[k][wave * 16 + lr];
        wr = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai, bi, wr, 0, 0, 0);
        wi = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, bi, wi, 0, 0, 0);
        wi = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, br, wi, 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // D layout: lane holds W[m = lk + 4 r][c = 16 wave + lr]
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    if constexpr (CX) Ws[lk + 4 * r][wave * 16 + lr] = cmake(wr[r], wi[r]);
    else Ws[lk + 4 * r][wave * 16 + lr] = wr[r];
  }
  // op(T) into LDS: T itself, or T^H[r][c] = conj(T[c][r])
  for (int x = tid; x < NBR * NBR; x += 256) {
    const int r = x % NBR, c = x / NBR;
    const int tr = use_th ? c : r, tc = use_th ? r : c;
    S t = (tr < nbe && tc < nbe) ? TB[(j0 + tr) + (size_t)tc * N] : ST<S>::zero();
    Tt[r][c] = use_th ? conjg(t) : t;
  }
  __syncthreads();
  // ---- W' = op(T) W (16 x 64), written over Ws after a barrier; thread:
  // row m = tid % 16, columns tid / 16 + 16 u
  S wp[4];
  {
    const int m = tid % NBR, cb = tid / NBR;
#pragma unroll
    for (int u = 0; u < 4; ++u) wp[u] = ST<S>::zero();
#pragma unroll 2
    for (int k = 0; k < NBR; ++k) {
      const S t = Tt[m][k];
#pragma unroll
      for (int u = 0; u < 4; ++u) wp[u] = wp[u] + t * Ws[k][cb + 16 * u];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) Ws[m][cb + 16 * u] = wp[u];
  }
  __syncthreads();
  // ---- C -= V W': wave w updates columns 16w..16w+15, 16 rows at a time.
  // Operands fed as (W', V) so a lane owns one row and four columns of the
  // block and the stores coalesce along the column.
  const int cw = c0 + wave * 16;
  double br[4], bi[4];
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) split_s<S>(Ws[ks * 4 + lk][wave * 16 + lr], br[ks], bi[ks]);
#pragma unroll 1
  for (int i0 = j0; i0 < N; i0 += 16) {
    const int i = i0 + lr, ic = min(i, N - 1);
    S cl[4], vl[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) cl[r] = gld(C + ic + (size_t)min(cw + lk + 4 * r, cend - 1) * N);
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) vl[ks] = gld(V + ic + (size_t)(j0 + min(ks * 4 + lk, nbe - 1)) * N);
    d4 cr, ci;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double re, im;
      split_s<S>(cl[r], re, im);
      cr[r] = -re;
      ci[r] = -im;
    }
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int m = ks * 4 + lk;
      double vr, vi;
      split_s<S>(vl[ks], vr, vi);
      if (!(i < N && m < nbe)) { vr = 0.0; vi = 0.0; }
      // acc^T += W'^T V^T : A-operand W'[m][c] as (c, m), B-operand V[i][m] as (m, i)
      cr = __builtin_amdgcn_mfma_f64_16x16x4f64(br[ks], vr, cr, 0, 0, 0);
      if constexpr (CX) {
        cr = __builtin_amdgcn_mfma_f64_16x16x4f64(-bi[ks], vi, cr, 0, 0, 0);
        ci = __builtin_amdgcn_mfma_f64_16x16x4f64(bi[ks], vr, ci, 0, 0, 0);
        ci = __builtin_amdgcn_mfma_f64_16x16x4f64(br[ks], vi, ci, 0, 0, 0);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int c = cw + lk + 4 * r;
      if (i < N && c < cend) {
        if constexpr (CX) gst(C + i + (size_t)c * N, cmake(-cr[r], -ci[r]));
        else gst(C + i + (size_t)c * N, -cr[r]);
      }
    }
  }
}

// Compact-WY factor of a pair of panels (2q, 2q+1), 32 reflectors:
//   T = [[T1, T12], [0, T2]],  T12 = -T1 (V1^H V2) T2,
// written over the two 16 x 16 blocks in MAT_TB (rows j0 .. j0+31, columns
// 0 .. 31).  V2 is read as zero above its own panel's first row.
constexpr int PR = 2 * NBR;
template <typename S>
__global__ void __launch_bounds__(256) k_pair_t(const InstDev* __restrict__ insts, int q) {
  const InstDev& d = insts[blockIdx.y];
  if (d.st->idle) return;
  const int N = d.N;
  const int j0 = q * PR, j1 = j0 + NBR;
  if (j0 >= N) return;
  const int nb1 = min(NBR, N - j0), nb2 = max(0, min(NBR, N - j1));
  const S* V = matp<S>(d, MAT_V);
  S* TB = matp<S>(d, MAT_TB);
  const int tid = threadIdx.x;
  constexpr bool CX = ST<S>::is_complex;
  __shared__ S part[4][NBR][NBR + 1];
  __shared__ S Mm[NBR][NBR + 1], T1[NBR][NBR + 1], T2[NBR][NBR + 1], Pm[NBR][NBR + 1];
  const int a = tid / NBR, b = tid % NBR;   // one entry of the 16 x 16 products per thread
  // M12 = V1^H V2 on the matrix cores: wave w takes rows j1 + 4 (w + 4 s) .. + 3;
  // lane (lr, lk) feeds A[a = lr][k = lk] = conj(V1[i][a]) and B[k = lk][b = lr] = V2[i][b]
  {
    const int lane = tid & 63, wave = tid >> 6, lr = lane & 15, lk = lane >> 4;
    d4 mr = d4{0, 0, 0, 0}, mi = d4{0, 0, 0, 0};
    if (nb2 > 0) {
      const S* v1 = V + (size_t)(j0 + min(lr, nb1 - 1)) * N;
      const S* v2 = V + (size_t)(j1 + min(lr, nb2 - 1)) * N;
      const bool ca = lr < nb1, cb = lr < nb2;
#pragma unroll 4
      for (int i0 = j1 + 4 * wave; i0 < N; i0 += 16) {
        const int i = i0 + lk, ic = min(i, N - 1);
        const S x1 = gld(v1 + ic), x2 = gld(v2 + ic);
        double ar, ai, br, bi;
        split_s<S>(x1, ar, ai);
        split_s<S>(x2, br, bi);
        if (!(i < N && ca)) { ar = 0.0; ai = 0.0; }
        if (!(i < N && cb)) { br = 0.0; bi = 0.0; }
        mr = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, mr, 0, 0, 0);
        if constexpr (CX) {
          mr = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, bi, mr, 0, 0, 0);
          mi = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, bi, mi, 0, 0, 0);
          mi = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai, br, mi, 0, 0, 0);
        }
      }
    }
    // lane holds M[a = lk + 4 r][b = lr]
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if constexpr (CX) part[wave][lk + 4 * r][lr] = cmake(mr[r], mi[r]);
      else part[wave][lk + 4 * r][lr] = mr[r];
    }
  }
  __syncthreads();
  Mm[a][b] = part[0][a][b] + part[1][a][b] + part[2][a][b] + part[3][a][b];
  T1[a][b] = (a < nb1 && b < nb1) ? TB[(j0 + a) + (size_t)b * N] : ST<S>::zero();
  T2[a][b] = (a < nb2 && b < nb2) ? TB[(j1 + a) + (size_t)b * N] : ST<S>::zero();
  __syncthreads();
  S p = ST<S>::zero();   // P = M12 T2
  for (int k = 0; k < NBR; ++k) p = p + Mm[a][k] * T2[k][b];
  Pm[a][b] = p;
  __syncthreads();
  S t12 = ST<S>::zero();   // T12 = -T1 P
  for (int k = 0; k < NBR; ++k) t12 = t12 - T1[a][k] * Pm[k][b];
  // only entries inside the N x N matrix (N may be below 32)
  if (j0 + a < N && NBR + b < N) TB[(j0 + a) + (size_t)(NBR + b) * N] = (a < nb1 && b < nb2) ? t12 : ST<S>::zero();
  if (j1 + a < N) {
    if (NBR + b < N) TB[(j1 + a) + (size_t)(NBR + b) * N] = T2[a][b];
    if (b < N) TB[(j1 + a) + (size_t)b * N] = ST<S>::zero();
  }
}

// C <- (I - V op(T) V^H) C with the 32 reflectors of pair q (columns
// j0 .. j0+31 of MAT_V, T from k_pair_t), rows [j0, N):
//   W = V^H C (32 x 64 tile per workgroup), W' = op(T) W, C -= V W'.
// cols: 0 -> [j0 + 32, N), 1 -> [j0, N), 2 -> [0, N).  The second panel's
// vectors are read as zero above their own first row.
template <typename S>
__global__ void __launch_bounds__(256) k_apply_refl2(const InstDev* __restrict__ insts, int n_inst, int q,
                                                     int target, int cols, int use_th) {
  constexpr bool CX = ST<S>::is_complex;
  int inst, bx;
  xcd_slot(n_inst, inst, bx);   // all column tiles of an instance on one XCD: V is read into one L2
  if (inst < 0) return;
  const InstDev& d = insts[inst];
  if (d.st->idle) return;
  const int N = d.N;
  const int j0 = q * PR;
  if (j0 >= N) return;
  const int nbe = min(PR, N - j0);
  const int cbeg = cols == 0 ? j0 + PR : (cols == 1 ? j0 : 0);
  const int c0 = cbeg + bx * AR_CT;
  if (c0 >= N) return;
  const S* V = matp<S>(d, MAT_V);
  const S* TB = matp<S>(d, MAT_TB);
  S* C = matp<S>(d, target);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  constexpr int RB = 32;
  __shared__ double Vr[RB][PR + 1], Vi[CX ? RB : 1][PR + 1];
  // C staging planes during W = V^H C; then W / W' (PR x AR_CT) in the same bytes
  constexpr int CPL = RB * (AR_CT + 1);
  constexpr int CBYTES = (CX ? 2 : 1) * CPL * 8 > PR * (AR_CT + 1) * (int)sizeof(S)
                             ? (CX ? 2 : 1) * CPL * 8 : PR * (AR_CT + 1) * (int)sizeof(S);
  __shared__ __attribute__((aligned(16))) char cbuf[CBYTES];
  double* Cr = reinterpret_cast<double*>(cbuf);
  double* Ci = Cr + CPL;
  S* Ws = reinterpret_cast<S*>(cbuf);
  __shared__ S Tt[PR][PR + 1];
  constexpr int NV = RB * PR / 256, NC = RB * AR_CT / 256;
  // complex products with three real ones: P1 = ar br (wr), P2 = ai bi (wi),
  // P3 = (ar + ai)(br + bi) (wq); re = P1 - P2, im = P3 - P1 - P2
  d4 wr[2], wi[2], wq[CX ? 2 : 1];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    wr[t] = d4{0, 0, 0, 0};
    wi[t] = d4{0, 0, 0, 0};
    if constexpr (CX) wq[t] = d4{0, 0, 0, 0};
  }
  // the loads of row chunk i0 + RB are issued before chunk i0 is multiplied
  S vv[NV], cv[NC];
  auto load_chunk = [&](int i0) {
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      const int x = tid + 256 * u, r = x % RB, m = x / RB;
      vv[u] = gld(V + min(i0 + r, N - 1) + (size_t)(j0 + min(m, nbe - 1)) * N);
    }
#pragma unroll
    for (int u = 0; u < NC; ++u) {
      const int x = tid + 256 * u, r = x % RB, cc = x / RB;
      cv[u] = gld(C + min(i0 + r, N - 1) + (size_t)min(c0 + cc, N - 1) * N);
    }
  };
  load_chunk(j0);
#pragma unroll 1
  for (int i0 = j0; i0 < N; i0 += RB) {
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      const int x = tid + 256 * u, r = x % RB, m = x / RB;
      const int i = i0 + r;
      const bool in = i < N && m < nbe && i >= j0 + (m / NBR) * NBR;
      double re, im;
      split_s<S>(vv[u], re, im);
      Vr[r][m] = in ? re : 0.0;
      if constexpr (CX) Vi[r][m] = in ? im : 0.0;
    }
#pragma unroll
    for (int u = 0; u < NC; ++u) {
      const int x = tid + 256 * u, r = x % RB, cc = x / RB;
      const bool in = i0 + r < N && c0 + cc < N;
      double re, im;
      split_s<S>(cv[u], re, im);
      Cr[r * (AR_CT + 1) + cc] = in ? re : 0.0;
      if constexpr (CX) Ci[r * (AR_CT + 1) + cc] = in ? im : 0.0;
    }
    __syncthreads();
    if (i0 + RB < N) load_chunk(i0 + RB);
#pragma unroll 2
    for (int ks = 0; ks < RB / 4; ++ks) {
      const int k = ks * 4 + lk;
      const double br = Cr[k * (AR_CT + 1) + wave * 16 + lr];
      const double bi = CX ? Ci[k * (AR_CT + 1) + wave * 16 + lr] : 0.0;
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        // A = V^H: A[m][k] = conj(V[k][m]) = (ar, ai); B = C: B[k][c] = (br, bi)
        const double ar = Vr[k][t * 16 + lr];
        wr[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, wr[t], 0, 0, 0);
        if constexpr (CX) {
          const double ai = -Vi[k][t * 16 + lr];
          wi[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, bi, wi[t], 0, 0, 0);
          wq[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar + ai, br + bi, wq[t], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  // W[m = 16 t + lk + 4 r][c = 16 wave + lr] (the C planes are free now)
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = t * 16 + lk + 4 * r, c = wave * 16 + lr;
      if constexpr (CX) Ws[m * (AR_CT + 1) + c] = cmake(wr[t][r] - wi[t][r], wq[t][r] - wr[t][r] - wi[t][r]);
      else Ws[m * (AR_CT + 1) + c] = wr[t][r];
    }
  for (int x = tid; x < PR * PR; x += 256) {
    const int r = x % PR, c = x / PR;
    const int tr = use_th ? c : r, tc = use_th ? r : c;
    S t = (tr < nbe && tc < nbe) ? TB[(j0 + tr) + (size_t)tc * N] : ST<S>::zero();
    Tt[r][c] = use_th ? conjg(t) : t;
  }
  __syncthreads();
  // W' = op(T) W: 32 x 64; thread: row m = tid % 32, columns tid / 32 + 8 u
  S wp[8];
  {
    const int m = tid % PR, cb = tid / PR;
#pragma unroll
    for (int u = 0; u < 8; ++u) wp[u] = ST<S>::zero();
#pragma unroll 2
    for (int k = 0; k < PR; ++k) {
      const S t = Tt[m][k];
#pragma unroll
      for (int u = 0; u < 8; ++u) wp[u] = wp[u] + t * Ws[k * (AR_CT + 1) + cb + 8 * u];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 8; ++u) Ws[m * (AR_CT + 1) + cb + 8 * u] = wp[u];
  }
  __syncthreads();
  // C -= V W': wave w updates columns 16w .. 16w+15, 16 rows at a time, K = 32;
  // the next 16 rows' C and V are loaded while these are multiplied
  const int cw = c0 + wave * 16;
  S cl[4], vl[8];
  auto load_rows = [&](int i0) {
    const int ic = min(i0 + lr, N - 1);
#pragma unroll
    for (int r = 0; r < 4; ++r) cl[r] = gld(C + ic + (size_t)min(cw + lk + 4 * r, N - 1) * N);
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) vl[ks] = gld(V + ic + (size_t)(j0 + min(ks * 4 + lk, nbe - 1)) * N);
  };
  load_rows(j0);
#pragma unroll 1
  for (int i0 = j0; i0 < N; i0 += 16) {
    const int i = i0 + lr;
    // (W' V)(c, i) with three real products: Q1 = br vr (q1), Q2 = bi vi (q2),
    // Q3 = (br + bi)(vr + vi) (q3), started at -C so that
    // C - W'V = -((q1 - q2) + i (q3 - q1 - q2)) with q1 = -Cre, q3 = -Cre - Cim
    d4 q1, q2, q3;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double re, im;
      split_s<S>(cl[r], re, im);
      q1[r] = -re;
      q2[r] = 0.0;
      q3[r] = -re - im;
    }
    double vr[8], vi[8];
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      const int m = ks * 4 + lk;
      split_s<S>(vl[ks], vr[ks], vi[ks]);
      if (!(i < N && m < nbe && i >= j0 + (m / NBR) * NBR)) { vr[ks] = 0.0; vi[ks] = 0.0; }
    }
    if (i0 + 16 < N) load_rows(i0 + 16);
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      const int m = ks * 4 + lk;
      double br, bi;
      split_s<S>(Ws[m * (AR_CT + 1) + wave * 16 + lr], br, bi);
      q1 = __builtin_amdgcn_mfma_f64_16x16x4f64(br, vr[ks], q1, 0, 0, 0);
      if constexpr (CX) {
        q2 = __builtin_amdgcn_mfma_f64_16x16x4f64(bi, vi[ks], q2, 0, 0, 0);
        q3 = __builtin_amdgcn_mfma_f64_16x16x4f64(br + bi, vr[ks] + vi[ks], q3, 0, 0, 0);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int c = cw + lk + 4 * r;
      if (i < N && c < N) {
        if constexpr (CX) gst(C + i + (size_t)c * N, cmake(-(q1[r] - q2[r]), -(q3[r] - q1[r] - q2[r])));
        else gst(C + i + (size_t)c * N, -q1[r]);
      }
    }
  }
}

// ---- Row-split block-reflector update --------------------------------------------------------
// For batches too small to fill the GPU with column tiles alone (one large
// instance), the rows [j0, N) of the update C <- (I - V op(T) V^H) C are cut
// into nsplit chunks (multiples of 32 rows).  Phase 1: each (column tile,
// chunk) workgroup writes its partial W = V^H C (NR x 64) to the instance's
// split buffer.  Phase 2: each (column tile, chunk) workgroup sums the
// partials in chunk order (deterministic), forms W' = op(T) W, and updates
// its chunk's rows of C.  NR = 16 (one panel) or 32 (a pair of panels; the
// second panel's vectors are read as zero above its own first row).
struct ReflRange {
  int j0, nbe, cbeg, cend;
};
template <int NR>
__device__ __forceinline__ ReflRange refl_range(int N, int blk, int cols) {
  ReflRange g;
  g.j0 = blk * NR;
  g.nbe = min(NR, N - g.j0);
  g.cbeg = cols == 2 ? 0 : (cols == 1 ? g.j0 : g.j0 + NR);
  g.cend = cols == 3 ? min(N, g.j0 + 2 * NBR) : N;
  return g;
}
__device__ __forceinline__ int refl_chunk(int N, int j0, int nsplit) {
  return ((((N - j0) + nsplit - 1) / nsplit) + 31) & ~31;
}

template <typename S, int NR>
__global__ void __launch_bounds__(256) k_refl_w(const InstDev* __restrict__ insts, int blk, int target, int cols,
                                                int nsplit) {
  constexpr bool CX = ST<S>::is_complex;
  constexpr int NT = NR / 16;
  const InstDev& d = insts[blockIdx.y];
  if (d.st->idle) return;
  const int N = d.N;
  const ReflRange g = refl_range<NR>(N, blk, cols);
  if (g.j0 >= N) return;
  const int c0 = g.cbeg + blockIdx.x * AR_CT;
  if (c0 >= g.cend) return;
  const int chunk = refl_chunk(N, g.j0, nsplit);
  const int r0 = g.j0 + blockIdx.z * chunk, r1 = min(N, r0 + chunk);
  const S* V = matp<S>(d, MAT_V);
  const S* C = matp<S>(d, target);
  S* Wp = reinterpret_cast<S*>(d.rsplit) + (size_t)blockIdx.z * NR * N;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  constexpr int RB = 32;
  __shared__ double Vr[RB][NR + 1], Vi[CX ? RB : 1][NR + 1];
  __shared__ double Cr[RB][AR_CT + 1], Ci[CX ? RB : 1][AR_CT + 1];
  constexpr int NV = RB * NR / 256, NC = RB * AR_CT / 256;
  d4 wr[NT], wi[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) { wr[t] = d4{0, 0, 0, 0}; wi[t] = d4{0, 0, 0, 0}; }
#pragma unroll 1
  for (int i0 = r0; i0 < r1; i0 += RB) {
    S vv[NV], cv[NC];
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      const int x = tid + 256 * u, r = x % RB, m = x / RB;
      vv[u] = gld(V + min(i0 + r, N - 1) + (size_t)(g.j0 + min(m, g.nbe - 1)) * N);
    }
#pragma unroll
    for (int u = 0; u < NC; ++u) {
      const int x = tid + 256 * u, r = x % RB, cc = x / RB;
      cv[u] = gld(C + min(i0 + r, N - 1) + (size_t)min(c0 + cc, g.cend - 1) * N);
    }
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      const int x = tid + 256 * u, r = x % RB, m = x / RB;
      const int i = i0 + r;
      const bool in = i < r1 && m < g.nbe && i >= g.j0 + (m / NBR) * NBR;
      double re, im;
      split_s<S>(vv[u], re, im);
      Vr[r][m] = in ? re : 0.0;
      if constexpr (CX) Vi[r][m] = in ? im : 0.0;
    }
#pragma unroll
    for (int u = 0; u < NC; ++u) {
      const int x = tid + 256 * u, r = x % RB, cc = x / RB;
      const bool in = i0 + r < r1 && c0 + cc < g.cend;
      double re, im;
      split_s<S>(cv[u], re, im);
      Cr[r][cc] = in ? re : 0.0;
      if constexpr (CX) Ci[r][cc] = in ? im : 0.0;
    }
    __syncthreads();
#pragma unroll 2
    for (int ks = 0; ks < RB / 4; ++ks) {
      const int k = ks * 4 + lk;
      const double br = Cr[k][wave * 16 + lr];
      const double bi = CX ? Ci[k][wave * 16 + lr] : 0.0;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        // A = V^H: A[m][k] = conj(V[k][m]); B = C: B[k][c]
        const double ar = Vr[k][t * 16 + lr];
        wr[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, wr[t], 0, 0, 0);
        if constexpr (CX) {
          const double ai = Vi[k][t * 16 + lr];
          wr[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, bi, wr[t], 0, 0, 0);
          wi[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, bi, wi[t], 0, 0, 0);
          wi[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai, br, wi[t], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  // lane holds W[m = 16 t + lk + 4 r][c = 16 wave + lr]; an empty chunk stores zeros
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = t * 16 + lk + 4 * r, c = c0 + wave * 16 + lr;
      if (c < g.cend) {
        if constexpr (CX) gst(Wp + (size_t)m * N + c, cmake(wr[t][r], wi[t][r]));
        else gst(Wp + (size_t)m * N + c, wr[t][r]);
      }
    }
}

template <typename S, int NR>
__global__ void __launch_bounds__(256) k_refl_c(const InstDev* __restrict__ insts, int blk, int target, int cols,
                                                int use_th, int nsplit) {
  constexpr bool CX = ST<S>::is_complex;
  const InstDev& d = insts[blockIdx.y];
  if (d.st->idle) return;
  const int N = d.N;
  const ReflRange g = refl_range<NR>(N, blk, cols);
  if (g.j0 >= N) return;
  const int c0 = g.cbeg + blockIdx.x * AR_CT;
  if (c0 >= g.cend) return;
  const int chunk = refl_chunk(N, g.j0, nsplit);
  const int r0 = g.j0 + blockIdx.z * chunk, r1 = min(N, r0 + chunk);
  const S* V = matp<S>(d, MAT_V);
  const S* TB = matp<S>(d, MAT_TB);
  const S* Wp = reinterpret_cast<const S*>(d.rsplit);
  S* C = matp<S>(d, target);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  __shared__ S Ws[NR][AR_CT + 1];
  __shared__ S Tt[NR][NR + 1];
  // W = sum of the chunk partials, in chunk order
  for (int x = tid; x < NR * AR_CT; x += 256) {
    const int m = x / AR_CT, cc = x % AR_CT;
    const int c = min(c0 + cc, g.cend - 1);
    S acc = ST<S>::zero();
    for (int z = 0; z < nsplit; ++z) acc = acc + gld(Wp + (size_t)(z * NR + m) * N + c);
    Ws[m][cc] = acc;
  }
  for (int x = tid; x < NR * NR; x += 256) {
    const int r = x % NR, c = x / NR;
    const int tr = use_th ? c : r, tc = use_th ? r : c;
    S t = (tr < g.nbe && tc < g.nbe) ? TB[(g.j0 + tr) + (size_t)tc * N] : ST<S>::zero();
    Tt[r][c] = use_th ? conjg(t) : t;
  }
  __syncthreads();
  // W' = op(T) W: thread row m = tid % NR, columns tid / NR + (256 / NR) u
  {
    constexpr int NU = AR_CT * NR / 256, CS = 256 / NR;
    const int m = tid % NR, cb = tid / NR;
    S wp[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) wp[u] = ST<S>::zero();
#pragma unroll 2
    for (int k = 0; k < NR; ++k) {
      const S t = Tt[m][k];
#pragma unroll
      for (int u = 0; u < NU; ++u) wp[u] = wp[u] + t * Ws[k][cb + CS * u];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NU; ++u) Ws[m][cb + CS * u] = wp[u];
  }
  __syncthreads();
  // C -= V W' on rows [r0, r1): wave w updates columns 16w .. 16w+15, 16 rows at a time
  constexpr int NK = NR / 4;
  const int cw = c0 + wave * 16;
#pragma unroll 1
  for (int i0 = r0; i0 < r1; i0 += 16) {
    const int i = i0 + lr, ic = min(i, N - 1);
    S cl[4], vl[NK];
#pragma unroll
    for (int r = 0; r < 4; ++r) cl[r] = gld(C + ic + (size_t)min(cw + lk + 4 * r, g.cend - 1) * N);
#pragma unroll
    for (int ks = 0; ks < NK; ++ks) vl[ks] = gld(V + ic + (size_t)(g.j0 + min(ks * 4 + lk, g.nbe - 1)) * N);
    d4 cr, ci;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double re, im;
      split_s<S>(cl[r], re, im);
      cr[r] = -re;
      ci[r] = -im;
    }
#pragma unroll
    for (int ks = 0; ks < NK; ++ks) {
      const int m = ks * 4 + lk;
      double vr, vi;
      split_s<S>(vl[ks], vr, vi);
      if (!(i < r1 && m < g.nbe && i >= g.j0 + (m / NBR) * NBR)) { vr = 0.0; vi = 0.0; }
      double br, bi;
      split_s<S>(Ws[m][wave * 16 + lr], br, bi);
      // acc^T += W'^T V^T: A-operand W'[m][c] as (c, m), B-operand V[i][m] as (m, i)
      cr = __builtin_amdgcn_mfma_f64_16x16x4f64(br, vr, cr, 0, 0, 0);
      if constexpr (CX) {
        cr = __builtin_amdgcn_mfma_f64_16x16x4f64(-bi, vi, cr, 0, 0, 0);
        ci = __builtin_amdgcn_mfma_f64_16x16x4f64(bi, vr, ci, 0, 0, 0);
        ci = __builtin_amdgcn_mfma_f64_16x16x4f64(br, vi, ci, 0, 0, 0);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int c = cw + lk + 4 * r;
      if (i < r1 && c < g.cend) {
        if constexpr (CX) gst(C + i + (size_t)c * N, cmake(-cr[r], -ci[r]));
        else gst(C + i + (size_t)c * N, -cr[r]);
      }
    }
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

// ---- LU with partial pivoting of Y (MAT_QA), for G = ... Y^{-1} ... ----------------------
template <typename S, int PT>
struct LuShared {
  double redv[PT / 64];
  int redi[PT / 64];
  S prow[NBR], orow[NBR];
};

// Column C of the leaf panel (compile-time, so the register array is indexed
// with constants): the pivot (largest |a|^2 on or below the diagonal row
// r = c0 + C, ties to the smaller row) by a block-wide arg-max, the swap of
// rows r and p through LDS, the multipliers and the update of the later
// panel columns.  Two barriers per column.
template <typename S, int RPT, int PT, int C>
struct LuColumn {
  static __device__ __forceinline__ void run(S (&a)[RPT][NBR], LuShared<S, PT>& sh, int* piv, int c0, int N,
                                             int nbe) {
    if constexpr (C < NBR) {
      if (C < nbe) {
        const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
        const int r = c0 + C;
        double best = -1.0;
        int bi = N;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          const int i = c0 + tid + PT * q;
          const double v = absq(a[q][C]);
          if (i >= r && i < N && v > best) { best = v; bi = i; }
        }
        for (int off = 32; off > 0; off >>= 1) {
          const double ob = __shfl_xor(best, off);
          const int oi = __shfl_xor(bi, off);
          if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
        }
        if (lane == 0) { sh.redv[wave] = best; sh.redi[wave] = bi; }
        __syncthreads();
        best = sh.redv[0];
        bi = sh.redi[0];
#pragma unroll
        for (int w = 1; w < PT / 64; ++w)
          if (sh.redv[w] > best || (sh.redv[w] == best && sh.redi[w] < bi)) { best = sh.redv[w]; bi = sh.redi[w]; }
        const int p = bi < N ? bi : r;
        // row r sits in thread C (q = 0); row p in thread (p - c0) % PT
        const int ow_p = (p - c0) % PT, q_p = (p - c0) / PT;
        // (selects rather than branches on q: merged branches would index the
        // register array with a variable and demote it to scratch memory)
        if (tid == ow_p) {
          S sel[NBR];
#pragma unroll
          for (int cc = 0; cc < NBR; ++cc) sel[cc] = a[0][cc];
#pragma unroll
          for (int q = 1; q < RPT; ++q)
#pragma unroll
            for (int cc = 0; cc < NBR; ++cc) sel[cc] = psel(q == q_p, a[q][cc], sel[cc]);
#pragma unroll
          for (int cc = 0; cc < NBR; ++cc) sh.prow[cc] = sel[cc];
        }
        if (tid == C) {
#pragma unroll
          for (int cc = 0; cc < NBR; ++cc) sh.orow[cc] = a[0][cc];
          piv[r] = p;
        }
        __syncthreads();
        if (tid == C) {
#pragma unroll
          for (int cc = 0; cc < NBR; ++cc) a[0][cc] = sh.prow[cc];
        }
        if (tid == ow_p && p != r) {
#pragma unroll
          for (int q = 0; q < RPT; ++q)
#pragma unroll
            for (int cc = 0; cc < NBR; ++cc) a[q][cc] = psel(q == q_p, sh.orow[cc], a[q][cc]);
        }
        const S inv = cdiv(ST<S>::one(), sh.prow[C]);
        S pr[NBR];
#pragma unroll
        for (int cc = C + 1; cc < NBR; ++cc) pr[cc] = sh.prow[cc];
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          const int i = c0 + tid + PT * q;
          if (i > r && i < N) {
            const S l = a[q][C] * inv;
            a[q][C] = l;
#pragma unroll
            for (int cc = C + 1; cc < NBR; ++cc) a[q][cc] = a[q][cc] - l * pr[cc];
          }
        }
      }
      LuColumn<S, RPT, PT, C + 1>::run(a, sh, piv, c0, N, nbe);
    }
  }
};

// Leaf panel of the recursive LU: columns [c0, c0 + nbw) (nbw <= 16), rows
// [c0, N) held in registers (thread t owns rows c0 + t + PT q).  The
// interchanges go to perm[c0 ..] (row r swapped with perm[r]); applying them
// to the other columns is k_lu_swap's job.
template <typename S, int RPT, int PT>
__global__ void __launch_bounds__(PT) k_lu_panel(const InstDev* __restrict__ insts, int c0, int nbw) {
  const InstDev& d = insts[blockIdx.y];
  if (d.st->idle) return;
  const int N = d.N;
  if (c0 >= N) return;
  const int nbe = min(nbw, N - c0);
  S* A = matp<S>(d, MAT_QA);
  const int tid = threadIdx.x;
  __shared__ LuShared<S, PT> sh;
  S a[RPT][NBR];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int i = c0 + tid + PT * q;
#pragma unroll
    for (int c = 0; c < NBR; ++c) a[q][c] = gld(A + min(i, N - 1) + (size_t)(c0 + min(c, nbe - 1)) * N);
  }
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int i = c0 + tid + PT * q;
#pragma unroll
    for (int c = 0; c < NBR; ++c) a[q][c] = psel(i < N && c < nbe, a[q][c], ST<S>::zero());
  }
  LuColumn<S, RPT, PT, 0>::run(a, sh, d.perm, c0, N, nbe);
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int i = c0 + tid + PT * q;
    if (i < N) {
#pragma unroll
      for (int c = 0; c < NBR; ++c)
        if (c < nbe) A[i + (size_t)(c0 + c) * N] = a[q][c];
    }
  }
}

// The interchanges of the leaf panel [c0, c0 + nbw), in order, on every
// column of MAT_QA outside the panel.  Every wave first composes them into
// one map of at most 2 nbw rows (lane e holds row pos_e, whose new content
// is the old row src_e): the panel rows start in lanes 0 .. nbe - 1, a pivot
// row outside the panel takes the next free lane.  Each half-wave then moves
// the rows of one column: a coalesced gather of the sources, then the stores.
template <typename S>
__global__ void __launch_bounds__(256) k_lu_swap(const InstDev* __restrict__ insts, int c0, int nbw) {
  const InstDev& d = insts[blockIdx.y];
  if (d.st->idle) return;
  const int N = d.N;
  if (c0 >= N) return;
  const int nbe = min(nbw, N - c0);
  const int lane = threadIdx.x & 63, e = lane & 31;
  const int* piv = d.perm;
  int pos = e < nbe ? c0 + e : -1;
  int src = pos;
  int cnt = nbe;
  for (int c = 0; c < nbe; ++c) {
    const int b = piv[c0 + c];
    if (b == c0 + c) continue;
    unsigned long long m = __ballot(pos == b) & 0xffffffffull;
    int lb;
    if (m == 0) {
      lb = cnt++;
      if (e == lb) { pos = b; src = b; }
    } else {
      lb = __ffsll(m) - 1;
    }
    const int sa = __shfl(src, c), sb = __shfl(src, lb);
    if (e == c) src = sb;
    if (e == lb) src = sa;
  }
  const bool mv = e < cnt && src != pos;
  if (!__any(mv)) return;
  S* A = matp<S>(d, MAT_QA);
  const int half = lane >> 5;
  const int wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
  if (blockIdx.x == 0 && threadIdx.x < 32 && mv) {   // the composed row order of Y
    int* rp = d.perm + N;
    const int v = rp[src];
    rp[pos] = v;
  }
  // columns handled by this block: [j0, j0 + 64)
  const int j0 = blockIdx.x * 64;
  for (int jj = 2 * wave + half; jj < 64; jj += 2 * nwave) {
    const int j = j0 + jj;
    if (j >= N || (j >= c0 && j < c0 + nbe)) continue;
    S* col = A + (size_t)j * N;
    S v = ST<S>::zero();
    if (mv) v = col[src];
    if (mv) col[pos] = v;
  }
}

// Unit lower-triangular solve on rows [r0, r0 + nb) (nb <= 32) of columns
// [col0, col1) of a target, L from the strict lower part of MAT_QA: one thread
// per column, the L block in LDS.
static_assert(TL_NB == 32, "k_trsm_lower holds 32 rows");
constexpr int TL_ROWS = TL_NB;
template <typename S>
__global__ void __launch_bounds__(256) k_trsm_lower(const InstDev* __restrict__ insts, int r0, int nb, int col0,
                                                    int col1, int target) {
  const InstDev& d = insts[blockIdx.y];
  if (d.st->idle) return;
  const int N = d.N;
  if (r0 >= N) return;
  const int nr = min(nb, N - r0);
  const S* Lm = matp<S>(d, MAT_QA);
  S* B = matp<S>(d, target);
  __shared__ S Lb[TL_ROWS][TL_ROWS + 1];
  for (int x = threadIdx.x; x < nr * nr; x += blockDim.x) {
    const int r = x % nr, c = x / nr;
    Lb[r][c] = Lm[(r0 + r) + (size_t)(r0 + c) * N];
  }
  __syncthreads();
  const int j = col0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= min(col1, N)) return;
  S z[TL_ROWS];
#pragma unroll
  for (int r = 0; r < TL_ROWS; ++r) z[r] = r < nr ? B[(r0 + r) + (size_t)j * N] : ST<S>::zero();
#pragma unroll
  for (int r = 1; r < TL_ROWS; ++r) {
    if (r < nr) {
      S s2 = z[r];
#pragma unroll
      for (int c = 0; c < r; ++c) s2 = s2 - Lb[r][c] * z[c];
      z[r] = s2;
    }
  }
#pragma unroll
  for (int r = 0; r < TL_ROWS; ++r)
    if (r < nr) B[(r0 + r) + (size_t)j * N] = z[r];
}

// After the drift of a recomputation has been accumulated (EO_DRIFT_REPLACE):
// drift_last = this recomputation's max |G_wrap - G_scratch|, drift_max the
// running maximum, NUMERR_DRIFT when it exceeds the instance's tolerance.
__global__ void k_stab_finish(const InstDev* __restrict__ insts) {
  const InstDev& d = insts[blockIdx.y];
  InstState* st = d.st;
  if (threadIdx.x != 0 || st->idle) return;
  const double dl = st->drift_acc;
  st->drift_acc = 0.0;
  if (st->init_mode) return;
  st->drift_last = dl;
  st->drift_max = fmax(st->drift_max, dl);
  if (!(dl <= d.drift_tol)) atomicOr(&st->numeric_err, NUMERR_DRIFT);
}

// Phase of a determinant from a Householder QR in MAT_QA / VEC_TAU.  A
// reflector H = 1 - tau v v^H with tau = (beta - alpha)/beta (beta real) has
// det H = 1 - tau |v|^2 = -tau / conj(tau) (1 when tau = 0), and
// det Q = prod_j det H_j.
//   mode 0 (after the chain step's QR A P = Q R): the working chain's new U is
//          Q, so phw = phase det Q.
//   mode 2 (after the LU P Y = L U of the recomputation): as mode 1 with
//          ph(det Y) = (-1)^(number of interchanges) prod_i ph(U_ii).
//   mode 1 (after the QR Y = Q_Y R_Y of the recomputation): with
//          1 + R L = U_R D_Rb Y D_Lb U_L^dagger (D positive), the phase of
//          det(1 + B_M .. B_1) = det(1 + R L) (cyclic invariance) is
//          ph(det U_R) ph(det Q_Y) prod_i ph(R_Y,ii) conj(ph(det U_L)).  It
//          replaces the tracked phase; the difference is recorded.
template <typename S>
__global__ void __launch_bounds__(256) k_detphase(const InstDev* __restrict__ insts, int mode) {
  const InstDev& d = insts[blockIdx.y];
  InstState* st = d.st;
  if (st->idle) return;
  const int N = d.N;
  const double* tauv = d.vec[VEC_TAU];
  const S* A = matp<S>(d, MAT_QA);
  double pr = 1.0, pi = 0.0;
  for (int j = threadIdx.x; j < N; j += blockDim.x) {
    double fr = 1.0, fi = 0.0;
    if (mode == 2) {
      if (d.perm[j] != j) fr = -1.0;
    } else {
      const double tr = tauv[2 * j], ti = tauv[2 * j + 1];
      const double t2 = tr * tr + ti * ti;
      if (t2 > 0.0) {   // -tau^2 / |tau|^2
        fr = -(tr * tr - ti * ti) / t2;
        fi = -(2.0 * tr * ti) / t2;
      }
    }
    if (mode >= 1) {
      const S rjj = A[j + (size_t)j * N];
      const double ra = sqrt(absq(rjj));
      if (ra > 0.0) {
        const double qr = real_part(rjj) / ra, qi = imag_part(rjj) / ra;
        const double a = fr, b = fi;
        fr = a * qr - b * qi;
        fi = a * qi + b * qr;
      }
    }
    const double a = pr, b = pi;
    pr = a * fr - b * fi;
    pi = a * fi + b * fr;
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double qr = __shfl_xor(pr, off), qi = __shfl_xor(pi, off);
    const double a = pr, b = pi;
    pr = a * qr - b * qi;
    pi = a * qi + b * qr;
  }
  __shared__ double part[2][4];
  if ((threadIdx.x & 63) == 0) { part[0][threadIdx.x >> 6] = pr; part[1][threadIdx.x >> 6] = pi; }
  __syncthreads();
  if (threadIdx.x != 0) return;
  pr = 1.0; pi = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
    const double a = pr, b = pi;
    pr = a * part[0][w] - b * part[1][w];
    pi = a * part[1][w] + b * part[0][w];
  }
  double nrm = sqrt(pr * pr + pi * pi);
  if (!(nrm > 0.0)) { pr = 1.0; pi = 0.0; nrm = 1.0; }
  pr /= nrm; pi /= nrm;
  if (mode == 0) {
    st->phw_re = pr;
    st->phw_im = pi;
    return;
  }
  // U_R, U_L: the working chain and the stack slot, by pass (as MAT_RU / MAT_LU)
  const int up = sched_is_up(st->phase, d.M);
  const int c = sched_ckpt(st->phase, d.M, d.n_stab);
  const double wr = st->phw_re, wi = st->phw_im, sr = d.stackPh[2 * c], si = d.stackPh[2 * c + 1];
  const double rr = up ? wr : sr, ri = up ? wi : si;   // ph det U_R
  const double lr = up ? sr : wr, li = up ? si : wi;   // ph det U_L
  double ar = rr * pr - ri * pi, ai = rr * pi + ri * pr;        // ph(U_R) ph(Y)
  const double br = ar * lr + ai * li, bi = ai * lr - ar * li;  // times conj ph(U_L)
  nrm = sqrt(br * br + bi * bi);
  ar = br / nrm;
  ai = bi / nrm;
  if (!st->init_mode) {
    const double dr = st->ph_re - ar, di = st->ph_im - ai;
    st->ph_drift = fmax(st->ph_drift, sqrt(dr * dr + di * di));
  }
  st->ph_re = ar;
  st->ph_im = ai;
}

}  // namespace

hipError_t launch_lu_panel(const InstDev* insts, int n_inst, int Nmax, bool cplx_, int c0, int nbw, hipStream_t s) {
#define DQMC_LUP(R, T)                                                                                          \
  if (cplx_) hipLaunchKernelGGL((k_lu_panel<cplx, R, T>), dim3(1, n_inst), dim3(T), 0, s, insts, c0, nbw);      \
  else hipLaunchKernelGGL((k_lu_panel<double, R, T>), dim3(1, n_inst), dim3(T), 0, s, insts, c0, nbw);
  const int rows = Nmax - c0;
  if (rows <= 0) return hipSuccess;
  if (rows <= 1024) {
    const int rpt = (rows + 255) / 256;
    if (rpt <= 1) { DQMC_LUP(1, 256) }
    else if (rpt <= 2) { DQMC_LUP(2, 256) }
    else if (rpt <= 3) { DQMC_LUP(3, 256) }
    else { DQMC_LUP(4, 256) }
  } else if (rows <= 2048) {
    if (rows <= 1536) { DQMC_LUP(3, 512) }
    else { DQMC_LUP(4, 512) }
  } else if (rows <= 4096) {
    if (rows <= 3072) { DQMC_LUP(3, 1024) }
    else { DQMC_LUP(4, 1024) }
  } else {
    return hipErrorInvalidValue;
  }
#undef DQMC_LUP
  return hipGetLastError();
}

hipError_t launch_lu_swap(const InstDev* insts, int n_inst, int Nmax, bool cplx_, int c0, int nbw, hipStream_t s) {
  dim3 grid((Nmax + 63) / 64, n_inst);
  if (cplx_) hipLaunchKernelGGL(k_lu_swap<cplx>, grid, dim3(256), 0, s, insts, c0, nbw);
  else hipLaunchKernelGGL(k_lu_swap<double>, grid, dim3(256), 0, s, insts, c0, nbw);
  return hipGetLastError();
}

hipError_t launch_trsm_lower(const InstDev* insts, int n_inst, bool cplx_, int r0, int nb, int col0, int col1,
                             int target, hipStream_t s) {
  if (nb > TL_ROWS || col1 <= col0) return col1 <= col0 ? hipSuccess : hipErrorInvalidValue;
  dim3 grid((col1 - col0 + 255) / 256, n_inst);
  if (cplx_) hipLaunchKernelGGL(k_trsm_lower<cplx>, grid, dim3(256), 0, s, insts, r0, nb, col0, col1, target);
  else hipLaunchKernelGGL(k_trsm_lower<double>, grid, dim3(256), 0, s, insts, r0, nb, col0, col1, target);
  return hipGetLastError();
}

hipError_t launch_stab_finish(const InstDev* insts, int n_inst, hipStream_t s) {
  hipLaunchKernelGGL(k_stab_finish, dim3(1, n_inst), dim3(64), 0, s, insts);
  return hipGetLastError();
}

hipError_t launch_detphase(const InstDev* insts, int n_inst, bool cplx_, int mode, hipStream_t s) {
  if (cplx_) hipLaunchKernelGGL(k_detphase<cplx>, dim3(1, n_inst), dim3(256), 0, s, insts, mode);
  else hipLaunchKernelGGL(k_detphase<double>, dim3(1, n_inst), dim3(256), 0, s, insts, mode);
  return hipGetLastError();
}

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
  dim3 grid((Nmax + 15) / 16, n_inst);
  if (cplx_) hipLaunchKernelGGL(k_colnorm<cplx>, grid, dim3(256), 0, s, insts, mat);
  else hipLaunchKernelGGL(k_colnorm<double>, grid, dim3(256), 0, s, insts, mat);
  hipLaunchKernelGGL(k_sort_cols, dim3(1, n_inst), dim3(256), 0, s, insts);
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

hipError_t launch_qr_panel_reg(const InstDev* insts, int n_inst, int Nmax, bool cplx_, int p, hipStream_t s) {
#define DQMC_QRP(R, T)                                                                                        \
  if (cplx_) hipLaunchKernelGGL((k_qr_panel_reg<cplx, R, T>), dim3(1, n_inst), dim3(T), 0, s, insts, p);      \
  else hipLaunchKernelGGL((k_qr_panel_reg<double, R, T>), dim3(1, n_inst), dim3(T), 0, s, insts, p);
  // only rows [16 p, N) take part: the register count follows the panel's rows
  const int rows = Nmax - p * NBR;
  if (rows <= 0) return hipSuccess;
  if (rows <= 1024) {
    const int rpt = (rows + 255) / 256;
    if (rpt <= 1) { DQMC_QRP(1, 256) }
    else if (rpt <= 2) { DQMC_QRP(2, 256) }
    else if (rpt <= 3) { DQMC_QRP(3, 256) }
    else { DQMC_QRP(4, 256) }
  } else {
    const int rpt = (rows + 511) / 512;
    if (rpt <= 3) { DQMC_QRP(3, 512) }
    else if (rpt <= 4) { DQMC_QRP(4, 512) }
    else if (rpt > 8) return hipErrorInvalidValue;
    else if (cplx_) hipLaunchKernelGGL((k_qr_panel_reg<cplx, 8, 512>), dim3(1, n_inst), dim3(512), 0, s, insts, p);
    // real panels: the smallest register array that holds the rows
    else if (rpt == 5) hipLaunchKernelGGL((k_qr_panel_reg<double, 5, 512>), dim3(1, n_inst), dim3(512), 0, s, insts, p);
    else if (rpt == 6) hipLaunchKernelGGL((k_qr_panel_reg<double, 6, 512>), dim3(1, n_inst), dim3(512), 0, s, insts, p);
    else if (rpt == 7) hipLaunchKernelGGL((k_qr_panel_reg<double, 7, 512>), dim3(1, n_inst), dim3(512), 0, s, insts, p);
    else hipLaunchKernelGGL((k_qr_panel_reg<double, 8, 512>), dim3(1, n_inst), dim3(512), 0, s, insts, p);
  }
#undef DQMC_QRP
  return hipGetLastError();
}

hipError_t launch_pair_t(const InstDev* insts, int n_inst, bool cplx_, int q, hipStream_t s) {
  if (cplx_) hipLaunchKernelGGL(k_pair_t<cplx>, dim3(1, n_inst), dim3(256), 0, s, insts, q);
  else hipLaunchKernelGGL(k_pair_t<double>, dim3(1, n_inst), dim3(256), 0, s, insts, q);
  return hipGetLastError();
}

// Row chunks for a block-reflector update: 1 (fused kernel) when the column
// tiles of all instances fill the GPU; else enough chunks of at least 128 rows
// for about two workgroups per compute unit.
static int refl_split(int n_inst, int ncol, int rows, int nr) {
  const int tiles = ((ncol + AR_CT - 1) / AR_CT) * n_inst;
  if (tiles >= 256) return 1;
  int ns = (512 + tiles - 1) / tiles;
  ns = std::min(ns, rows / 128);
  ns = std::min(ns, RSPLIT_ROWS / nr);
  return std::max(ns, 1);
}

template <int NR>
static hipError_t launch_refl_split(const InstDev* insts, int n_inst, bool cplx_, int blk, int target, int cols,
                                    int use_th, int ncol, int ns, hipStream_t s) {
  dim3 grid((ncol + AR_CT - 1) / AR_CT, n_inst, ns);
  if (cplx_) {
    hipLaunchKernelGGL((k_refl_w<cplx, NR>), grid, dim3(256), 0, s, insts, blk, target, cols, ns);
    hipLaunchKernelGGL((k_refl_c<cplx, NR>), grid, dim3(256), 0, s, insts, blk, target, cols, use_th, ns);
  } else {
    hipLaunchKernelGGL((k_refl_w<double, NR>), grid, dim3(256), 0, s, insts, blk, target, cols, ns);
    hipLaunchKernelGGL((k_refl_c<double, NR>), grid, dim3(256), 0, s, insts, blk, target, cols, use_th, ns);
  }
  return hipGetLastError();
}

hipError_t launch_apply_refl2(const InstDev* insts, int n_inst, int Nmax, bool cplx_, int q, int target, int cols,
                              int use_th, hipStream_t s) {
  int j0 = q * PR;
  int cbeg = cols == 0 ? j0 + PR : (cols == 1 ? j0 : 0);
  int ncol = Nmax - cbeg;
  if (ncol <= 0 || j0 >= Nmax) return hipSuccess;
  const int ns = refl_split(n_inst, ncol, Nmax - j0, PR);
  if (ns > 1) return launch_refl_split<PR>(insts, n_inst, cplx_, q, target, cols, use_th, ncol, ns, s);
  dim3 grid((ncol + AR_CT - 1) / AR_CT, xcd_grid_y(n_inst));
  if (cplx_) hipLaunchKernelGGL(k_apply_refl2<cplx>, grid, dim3(256), 0, s, insts, n_inst, q, target, cols, use_th);
  else hipLaunchKernelGGL(k_apply_refl2<double>, grid, dim3(256), 0, s, insts, n_inst, q, target, cols, use_th);
  return hipGetLastError();
}

hipError_t launch_apply_refl(const InstDev* insts, int n_inst, int Nmax, bool cplx_, int p, int target, int cols,
                             int use_th, hipStream_t s) {
  int j0 = p * NBR;
  int cbeg = (cols == 0 || cols == 3) ? j0 + NBR : (cols == 1 ? j0 : 0);
  int ncol = (cols == 3 ? std::min(Nmax, j0 + 2 * NBR) : Nmax) - cbeg;
  if (ncol <= 0 || j0 >= Nmax) return hipSuccess;
  const int ns = refl_split(n_inst, ncol, Nmax - j0, NBR);
  if (ns > 1) return launch_refl_split<NBR>(insts, n_inst, cplx_, p, target, cols, use_th, ncol, ns, s);
  dim3 grid((ncol + AR_CT - 1) / AR_CT, n_inst);
  if (cplx_) hipLaunchKernelGGL(k_apply_refl<cplx>, grid, dim3(256), 0, s, insts, p, target, cols, use_th);
  else hipLaunchKernelGGL(k_apply_refl<double>, grid, dim3(256), 0, s, insts, p, target, cols, use_th);
  return hipGetLastError();
}
