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
// Stockham, one radix per stage, ping-pong between two LDS buffers), 2x2 block
// multiply per momentum, inverse 2-D FFT, optional diagonal, store.  Real
// matrices pack two real vectors as one complex vector (the operator is real).
// Rows are transformed with the transpose: E^T = conj(E) for Hermitian K, so a
// row is conjugated on load and on store.
#include "common.hpp"
#include "kernels.hpp"

namespace {

constexpr int FFT_THREADS = 256;

struct Resolved {
  int active, slice, pre, post, tab;
  int cj;   // 1: the HS diagonal enters conjugated (B^dagger of the downward chain)
};

template <typename C> using real_of_t = decltype(C::x);

__device__ __forceinline__ Resolved resolve(const InstDev& d, const FftArgs& a) {
  Resolved r{0, 0, 0, 0, TAB_P, 0};
  // the state fields read here, loaded together before the first test
  const InstState* st = d.st;
  const int idle = gldi(&st->idle), phase = gldi(&st->phase), init_mode = gldi(&st->init_mode);
  if (idle) return r;
  int M = d.M;
  int up = sched_is_up(phase, M);
  int l = sched_slice(phase, M);
  switch (a.op) {
    case FOP_WRAP_PRE:  // G <- e^{V} E+ G E- e^{-V} before updating slice l (upward)
      if (!up || init_mode) return r;
      r.active = 1; r.slice = l;
      if (a.side == 0) { r.pre = 0; r.tab = TAB_P; r.post = +1; }
      else { r.pre = 0; r.tab = TAB_M; r.post = -1; }
      return r;
    case FOP_WRAP_POST:  // G <- E- e^{-V} G e^{V} E+ after updating slice l (downward)
      if (up || init_mode) return r;
      r.active = 1; r.slice = l;
      if (a.side == 0) { r.pre = -1; r.tab = TAB_M; r.post = 0; }
      else { r.pre = +1; r.tab = TAB_P; r.post = 0; }
      return r;
    case FOP_STAB_B: {  // columns of the working U: B (upward) or B^dagger (downward)
      if (a.side != 0) return r;
      int c = sched_ckpt(phase, M, d.n_stab);
      r.active = 1;
      if (up) {  // R_c = B_{c ns} .. B_{(c-1) ns + 1} R_{c-1}: lowest slice first
        r.slice = (c - 1) * d.n_stab + 1 + a.j;
        r.pre = 0; r.tab = TAB_P; r.post = +1;
      } else {   // L_c^dag = B^dag_{c ns+1} .. B^dag_{(c+1) ns} L_{c+1}^dag: highest first,
                 // B^dag = E+ conj(e^{V}) (E+ is Hermitian)
        r.slice = c * d.n_stab + d.n_stab - a.j;
        r.pre = +1; r.tab = TAB_P; r.post = 0; r.cj = 1;
      }
      return r;
    }
    case FOP_HALF:  // G~ = e^{-dtau K/2} G e^{+dtau K/2} (instances that measure on it)
      if (!d.sym_measure) return r;
      r.active = 1; r.slice = 0;
      r.tab = (a.side == 0) ? TAB_HP : TAB_HM;
      return r;
    case FOP_EXPLICIT:
      r.active = 1; r.slice = a.ex_slice; r.pre = a.ex_pre; r.post = a.ex_post; r.tab = a.ex_tab;
      return r;
    case FOP_STAB_CHAIN:   // resolved step by step inside the kernel
      if (a.side != 0) return r;
      r.active = 1;
      return r;
    case FOP_FOURIER:
      if (init_mode) return r;
      r.active = 1;
      return r;
  }
  return r;
}

// Step j of a chain pass: the FOP_STAB_B resolution of that step.
__device__ __forceinline__ Resolved chain_step(const InstDev& d, const FftArgs& a, int j) {
  FftArgs aj = a;
  aj.op = FOP_STAB_B;
  aj.j = j;
  return resolve(d, aj);
}


// Complex compute type C is cplx (complex128) or cplxf (complex64); RT is its
// real type.  Tables and roots are held in double and rounded once on load.
template <typename C> using real_of = decltype(C::x);
template <typename C> __device__ __forceinline__ C mkc(double a, double b) {
  return C{(real_of<C>)a, (real_of<C>)b};
}
template <typename C> __device__ __forceinline__ C to_c(cplx a) { return mkc<C>(a.x, a.y); }

// The factors of the HS diagonal exp(H_I(x)) as multipliers in the
// transform's domain: e^{+-lambda} for the spin channel, e^{+-i alpha} for
// the charge channel (eqs. BIOpSz, BIOpnT).  Real G (two real vectors packed
// per complex transform) only occurs in the spin channel and keeps real
// factors; the row side of complex G is transformed conjugated, so a complex
// factor is applied conjugated there.
// mul(v, plus, cj): v e^{+-H_I} (conjugated when cj, for B^dagger).
template <typename C, bool CX>
struct HsDiag {
  real_of_t<C> p, m;
  __device__ HsDiag(const InstDev& d, bool) : p((real_of_t<C>)exp(d.lam)), m((real_of_t<C>)exp(-d.lam)) {}
  __device__ C mul(C v, bool plus, int = 0) const { return v * (plus ? p : m); }
};
template <typename C>
struct HsDiag<C, true> {
  C p, m;
  bool charge;
  __device__ HsDiag(const InstDev& d, bool rows) : charge(d.channel != 0) {
    if (charge) {
      const double c = cos(d.lam), s = rows ? -sin(d.lam) : sin(d.lam);
      p = mkc<C>(c, s);
      m = mkc<C>(c, -s);
    } else {
      p = mkc<C>(exp(d.lam), 0.0);
      m = mkc<C>(exp(-d.lam), 0.0);
    }
  }
  // conj(e^{+i alpha}) = e^{-i alpha}; the spin factors are real
  __device__ C mul(C v, bool plus, int cj = 0) const { return v * ((plus != (charge && cj)) ? p : m); }
};

// v <- e^{sign H_I(x_r)} v on element r of every vector held in LDS.
template <typename C, typename HD>
__device__ __forceinline__ void lds_diag(C* buf, int tot, int N, int sign, int cj, const int8_t* xs,
                                         const HD& hd, int nthreads) {
  for (int e = threadIdx.x; e < tot; e += nthreads) {
    const int r = e % N;
    buf[e] = hd.mul(buf[e], (sign * xs[r]) > 0, cj);
  }
}

template <typename C>
__device__ __forceinline__ C root_pow(const C* roots, int L, int m, int sign) {
  C w = roots[m % L];
  return sign < 0 ? w : conjg(w);
}

// Radix-R DFT of v in place: y_s = sum_r v_r w^{rs}, w = exp(sign 2 pi i / R).
template <int R, typename C>
__device__ __forceinline__ void small_dft(C* v, int sign) {
  typedef real_of<C> RT;
  if constexpr (R == 2) {
    C a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
  } else if constexpr (R == 4) {
    C x0 = v[0], x1 = v[1], x2 = v[2], x3 = v[3];
    C s02 = x0 + x2, d02 = x0 - x2, s13 = x1 + x3, d13 = x1 - x3;
    // w = sign * i: w * z = (-sign * z.y, sign * z.x)
    const RT sg = (RT)sign;
    C wd13 = C{-sg * d13.y, sg * d13.x};
    v[0] = s02 + s13;
    v[1] = d02 + wd13;
    v[2] = s02 - s13;
    v[3] = d02 - wd13;
  } else if constexpr (R == 3) {
    const RT c = (RT)-0.5, sn = (RT)(0.86602540378443864676 * sign);  // w = (c, sn)
    C x0 = v[0], x1 = v[1], x2 = v[2];
    C t = x1 + x2, u = x1 - x2;
    C m = x0 + c * t;
    C ju = C{-sn * u.y, sn * u.x};  // i * sn * u
    v[0] = x0 + t;
    v[1] = m + ju;
    v[2] = m - ju;
  }
}

// One Stockham stage of radix R on all lines of the nv vectors: src -> dst.
template <int R, typename C>
__device__ void fft_stage(const C* __restrict__ src, C* __restrict__ dst, const C* roots, int L,
                          int Nc, int N, int nv, int axis, int Ns, int sign) {
  const int per_line = L / R;
  const int nb = nv * 2 * L * per_line;
  const int estride = axis == 0 ? 1 : L;
  const int ostride = axis == 0 ? L : 1;
  const int twstep = L / (Ns * R);
  for (int b = threadIdx.x; b < nb; b += FFT_THREADS) {
    int line = b / per_line, j = b - line * per_line;
    int vv = line / (2 * L);
    int rem = line - vv * 2 * L;
    int s = rem / L, o = rem - s * L;
    int base = vv * N + s * Nc + o * ostride;
    int jm = j % Ns;
    int tw = twstep * jm;
    C v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      C x = src[base + (j + r * per_line) * estride];
      v[r] = (r && tw) ? x * root_pow(roots, L, tw * r, sign) : x;
    }
    int d0 = base + ((j / Ns) * Ns * R + jm) * estride;
    if constexpr (R <= 4) {
      small_dft<R>(v, sign);
#pragma unroll
      for (int r = 0; r < R; ++r) dst[d0 + r * Ns * estride] = v[r];
    } else {
      // y_s = sum_r v_r w^{rs}, one output at a time (w^s from the root table)
#pragma unroll 1
      for (int s2 = 0; s2 < R; ++s2) {
        const C step = s2 ? root_pow(roots, L, (L / R) * s2, sign) : mkc<C>(1.0, 0.0);
        C w = step, acc = v[0];
#pragma unroll
        for (int r = 1; r < R; ++r) {
          acc = acc + v[r] * w;
          w = w * step;
        }
        dst[d0 + s2 * Ns * estride] = acc;
      }
    }
  }
  __syncthreads();
}

// Largest radix a kernel instance supports; the host picks the smallest set
// that covers the factors of every instance's L.  Ping-pongs between the two
// LDS buffers; returns the buffer that holds the result.
template <int RMAX, typename C>
__device__ C* fft_2d(C* cur, C* other, const C* roots, const int* fac, int L, int Nc, int N,
                     int nv, int sign) {
  for (int axis = 0; axis < 2; ++axis) {
    int Ns = 1;
    for (int f = 0; fac[f]; ++f) {
      int R = fac[f];
      switch (R) {
        case 2: fft_stage<2>(cur, other, roots, L, Nc, N, nv, axis, Ns, sign); break;
        case 3: fft_stage<3>(cur, other, roots, L, Nc, N, nv, axis, Ns, sign); break;
        case 4: fft_stage<4>(cur, other, roots, L, Nc, N, nv, axis, Ns, sign); break;
        case 5: if constexpr (RMAX >= 5) fft_stage<5>(cur, other, roots, L, Nc, N, nv, axis, Ns, sign); break;
        case 7: if constexpr (RMAX >= 7) fft_stage<7>(cur, other, roots, L, Nc, N, nv, axis, Ns, sign); break;
        case 11: if constexpr (RMAX >= 11) fft_stage<11>(cur, other, roots, L, Nc, N, nv, axis, Ns, sign); break;
        case 13: if constexpr (RMAX >= 13) fft_stage<13>(cur, other, roots, L, Nc, N, nv, axis, Ns, sign); break;
        default: break;  // rejected on the host
      }
      C* t = cur; cur = other; other = t;
      Ns *= R;
    }
  }
  return cur;
}

// ---- compile-time plans for the common lattice sizes ------------------------------------
// Same radix order as the host: 4s, then 2, 3, 5, 7, 11, 13.
constexpr int fac_count(int L) {
  int c = 0, n = L;
  while (n % 4 == 0) { n /= 4; ++c; }
  while (n % 2 == 0) { n /= 2; ++c; }
  for (int p : {3, 5, 7, 11, 13})
    while (n % p == 0) { n /= p; ++c; }
  return c;
}
constexpr int fac_at(int L, int i) {
  int c = 0, n = L;
  while (n % 4 == 0) { if (c == i) return 4; n /= 4; ++c; }
  while (n % 2 == 0) { if (c == i) return 2; n /= 2; ++c; }
  for (int p : {3, 5, 7, 11, 13})
    while (n % p == 0) { if (c == i) return p; n /= p; ++c; }
  return 0;
}

template <int L, int AXIS, int I, int NS, typename C>
__device__ __forceinline__ void fixed_stages(C*& cur, C*& other, const C* roots, int nv, int sign) {
  if constexpr (I < fac_count(L)) {
    constexpr int R = fac_at(L, I);
    fft_stage<R>(cur, other, roots, L, L * L, 2 * L * L, nv, AXIS, NS, sign);
    C* t = cur; cur = other; other = t;
    fixed_stages<L, AXIS, I + 1, NS * R>(cur, other, roots, nv, sign);
  }
}

template <int L, typename C>
__device__ __forceinline__ C* fft_2d_fixed(C* cur, C* other, const C* roots, int nv, int sign) {
  fixed_stages<L, 0, 0, 1>(cur, other, roots, nv, sign);
  fixed_stages<L, 1, 0, 1>(cur, other, roots, nv, sign);
  return cur;
}

template <typename S, int RMAX, int LC, typename C>
__global__ void __launch_bounds__(FFT_THREADS)
k_fft_apply(const InstDev* __restrict__ insts, FftArgs a, int nv, int generic_only) {
  typedef real_of<C> RT;
  extern __shared__ char smem_raw[];
  const InstDev& d = insts[blockIdx.y];
  if (LC > 0 ? d.L != LC : (generic_only && d.fft_fixed)) return;
  Resolved rs = resolve(d, a);
  if (!rs.active) return;
  const int L = LC > 0 ? LC : d.L;
  const int Nc = L * L, N = 2 * Nc;
  const int nvec = ST<S>::is_complex ? N : N / 2;
  // XCD-aware tile order (gridDim.x a multiple of 8), as in k_fft_reg
  const int tile = (blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
  const int v0 = tile * nv;
  if (v0 >= nvec) return;
  const int nvl = min(nv, nvec - v0);
  C* buf = reinterpret_cast<C*>(smem_raw);
  C* buf2 = buf + (size_t)nv * N;
  __shared__ C roots[64];
  __shared__ int fac[16];
  if (threadIdx.x < L) roots[threadIdx.x] = to_c<C>(d.roots[threadIdx.x]);
  if (threadIdx.x < 16) fac[threadIdx.x] = d.factors[threadIdx.x];
  S* Mx = matp<S>(d, a.mat);
  const int8_t* xs = rs.slice > 0 ? d.fields + (size_t)(rs.slice - 1) * N : nullptr;
  const bool rows = a.side != 0;
  const HsDiag<C, ST<S>::is_complex> hd(d, rows);
  const bool chain = a.op == FOP_STAB_CHAIN;
  // load (+ pre diagonal), LU elements per thread at a time: every load of a
  // group reads a clamped address and is issued before the first is used
  const int tot = nvl * N;
  constexpr int LU = 8;
  for (int e0 = threadIdx.x; e0 < tot; e0 += LU * FFT_THREADS) {
    S raw[LU][ST<S>::is_complex ? 1 : 2];
    int8_t xr[LU];
#pragma unroll
    for (int u = 0; u < LU; ++u) {
      const int e = min(e0 + u * FFT_THREADS, tot - 1);
      int vv, r;
      if (!rows) { vv = e / N; r = e - vv * N; }
      else { vv = e % nvl; r = e / nvl; }
      const int q = v0 + vv;
      if constexpr (ST<S>::is_complex) {
        raw[u][0] = gld(rows ? Mx + (size_t)r * N + q : Mx + (size_t)q * N + r);
      } else {
        raw[u][0] = gld(rows ? Mx + (size_t)r * N + 2 * q : Mx + (size_t)(2 * q) * N + r);
        raw[u][1] = gld(rows ? Mx + (size_t)r * N + 2 * q + 1 : Mx + (size_t)(2 * q + 1) * N + r);
      }
      xr[u] = rs.pre ? xs[r] : (int8_t)1;
    }
#pragma unroll
    for (int u = 0; u < LU; ++u) {
      const int e = e0 + u * FFT_THREADS;
      if (e < tot) {
        int vv, r;
        if (!rows) { vv = e / N; r = e - vv * N; }
        else { vv = e % nvl; r = e / nvl; }
        C val;
        if constexpr (ST<S>::is_complex) val = mkc<C>(raw[u][0].x, rows ? -raw[u][0].y : raw[u][0].y);
        else val = mkc<C>(raw[u][0], raw[u][1]);
        if (rs.pre) val = hd.mul(val, (rs.pre * xr[u]) > 0, rs.cj);
        buf[vv * N + r] = val;
      }
    }
  }
  __syncthreads();
  C* cur = buf;
  const int nrep = chain ? d.n_stab : 1;
  for (int rep = 0; rep < nrep; ++rep) {
    int tabi = rs.tab;
    if (chain) {   // step rep of the chain: pre diagonal in LDS
      const Resolved rj = chain_step(d, a, rep);
      tabi = rj.tab;
      if (rj.pre) {
        lds_diag(cur, tot, N, rj.pre, rj.cj, d.fields + (size_t)(rj.slice - 1) * N, hd, FFT_THREADS);
        __syncthreads();
      }
    }
    C* oth = cur == buf ? buf2 : buf;
    if constexpr (LC > 0) cur = fft_2d_fixed<LC>(cur, oth, roots, nvl, -1);
    else cur = fft_2d<RMAX>(cur, oth, roots, fac, L, Nc, N, nvl, -1);
    if (a.op == FOP_FOURIER) break;   // forward transform only
    oth = cur == buf ? buf2 : buf;
    // 2x2 block per momentum
    const cplx* T = d.tab + (size_t)tabi * Nc * 4;
    for (int e = threadIdx.x; e < nvl * Nc; e += FFT_THREADS) {
      int vv = e / Nc, k = e - vv * Nc;
      C qa = cur[vv * N + k], qb = cur[vv * N + Nc + k];
      C t00 = to_c<C>(T[4 * k]), t01 = to_c<C>(T[4 * k + 1]), t10 = to_c<C>(T[4 * k + 2]),
        t11 = to_c<C>(T[4 * k + 3]);
      cur[vv * N + k] = t00 * qa + t01 * qb;
      cur[vv * N + Nc + k] = t10 * qa + t11 * qb;
    }
    __syncthreads();
    if constexpr (LC > 0) cur = fft_2d_fixed<LC>(cur, oth, roots, nvl, +1);
    else cur = fft_2d<RMAX>(cur, oth, roots, fac, L, Nc, N, nvl, +1);
    if (chain) {   // post diagonal of step rep in LDS
      const Resolved rj = chain_step(d, a, rep);
      if (rj.post) {
        lds_diag(cur, tot, N, rj.post, rj.cj, d.fields + (size_t)(rj.slice - 1) * N, hd, FFT_THREADS);
        __syncthreads();
      }
    }
  }
  const double* dsc = chain ? d.vec[VEC_DW] : nullptr;   // chain: columns scaled by the working D
  // store (+ post diagonal)
  for (int e = threadIdx.x; e < tot; e += FFT_THREADS) {
    int vv, r;
    if (!rows) { vv = e / N; r = e - vv * N; }
    else { vv = e % nvl; r = e / nvl; }
    int q = v0 + vv;
    C val = cur[vv * N + r];
    if (rs.post) val = hd.mul(val, (rs.post * xs[r]) > 0, rs.cj);
    if (chain) {
      if constexpr (ST<S>::is_complex) val = val * (RT)dsc[q];
      else val = C{val.x * (RT)dsc[2 * q], val.y * (RT)dsc[2 * q + 1]};
    }
    const double vx = (double)val.x, vy = (double)val.y;
    if constexpr (ST<S>::is_complex) {
      if (rows) gst(Mx + (size_t)r * N + q, cmake(vx, -vy));
      else gst(Mx + (size_t)q * N + r, cmake(vx, vy));
    } else {
      if (!rows) { gst(Mx + (size_t)(2 * q) * N + r, vx); gst(Mx + (size_t)(2 * q + 1) * N + r, vy); }
      else { gst(Mx + (size_t)r * N + 2 * q, vx); gst(Mx + (size_t)r * N + 2 * q + 1, vy); }
    }
  }
}

// ---- register-resident line transforms (compile-time L <= 24) ---------------------------
// Each thread transforms whole lines of L points in registers with a
// compile-time mixed-radix Cooley-Tukey split, so a wrap side needs three
// passes over LDS (axis 0 forward; axis 1 forward, 2x2 block, axis 1 inverse
// with both sublattices of one momentum column in one thread; axis 0
// inverse) and three barriers, instead of one barrier per radix stage.
constexpr int rfac(int n) {
  if (n <= 4) return n;
  if (n % 4 == 0) return 4;
  for (int p : {2, 3, 5, 7, 11, 13})
    if (n % p == 0) return p;
  return n;
}

template <int L, bool INV, typename C>
__device__ __forceinline__ C twid(const C* roots, int m) {
  const C w = roots[m];
  return INV ? conjg(w) : w;
}

// X = DFT_N(x), W_N = exp(-+2 pi i / N) = W_L^(L/N) with W_L^m = roots[m]
// (conjugated for the inverse).  n = Q n1 + n2, k = k1 + P k2:
//   X[k1 + P k2] = sum_n2 W_Q^(n2 k2) W_N^(n2 k1) sum_n1 x[Q n1 + n2] W_P^(n1 k1).
template <int L, int N, bool INV, typename C>
__device__ __forceinline__ void rdft(const C (&x)[N], C (&X)[N], const C* roots) {
  constexpr int P = rfac(N);
  if constexpr (P == N) {
    if constexpr (N == 1) {
      X[0] = x[0];
    } else if constexpr (N <= 4) {
      C v[N];
#pragma unroll
      for (int i = 0; i < N; ++i) v[i] = x[i];
      small_dft<N>(v, INV ? +1 : -1);
#pragma unroll
      for (int i = 0; i < N; ++i) X[i] = v[i];
    } else {
#pragma unroll
      for (int k = 0; k < N; ++k) {
        C acc = x[0];
#pragma unroll
        for (int n = 1; n < N; ++n) acc = acc + x[n] * twid<L, INV>(roots, (L / N) * ((n * k) % N));
        X[k] = acc;
      }
    }
  } else {
    constexpr int Q = N / P;
    C y[Q][P];
#pragma unroll
    for (int n2 = 0; n2 < Q; ++n2) {
      C t[P], T[P];
#pragma unroll
      for (int n1 = 0; n1 < P; ++n1) t[n1] = x[Q * n1 + n2];
      rdft<L, P, INV>(t, T, roots);
#pragma unroll
      for (int k1 = 0; k1 < P; ++k1)
        y[n2][k1] = (n2 * k1 == 0) ? T[k1] : T[k1] * twid<L, INV>(roots, (L / N) * ((n2 * k1) % N));
    }
#pragma unroll
    for (int k1 = 0; k1 < P; ++k1) {
      C t[Q], T[Q];
#pragma unroll
      for (int n2 = 0; n2 < Q; ++n2) t[n2] = y[n2][k1];
      rdft<L, Q, INV>(t, T, roots);
#pragma unroll
      for (int k2 = 0; k2 < Q; ++k2) X[k1 + P * k2] = T[k2];
    }
  }
}

// Transform the line at p[0], p[st], ..., p[(L-1) st] in place.
template <int L, bool INV, typename C>
__device__ __forceinline__ void line_dft(C* p, int st, const C* roots) {
  C x[L], X[L];
#pragma unroll
  for (int n = 0; n < L; ++n) x[n] = p[n * st];
  rdft<L, L, INV>(x, X, roots);
#pragma unroll
  for (int n = 0; n < L; ++n) p[n * st] = X[n];
}

// Tiles of the register-line kernel: NV vectors per workgroup of NT threads.
//   0 wide:   as many vectors as 256 threads cover (2L threads per vector)
//   1 narrow: half as many, half the LDS (more workgroups per CU)
//   2 eight:  8 vectors, so that a row side reads 128-byte segments of
//             complex G (only where the LDS stays within 96 KB; else wide)
constexpr int reg_nv(int L, int tile) {
  const int wide = 256 / (2 * L);
  if (tile == 1) return (wide + 1) / 2;
  if (tile == 2 && 8 * 2 * L * L * 16 <= 96 * 1024) return 8;
  return wide;
}
constexpr int reg_nt(int L, int tile) { return (reg_nv(L, tile) * 2 * L + 63) / 64 * 64; }

template <typename S, int LC, typename C, int NV, int NT>
__global__ void __launch_bounds__(NT) k_fft_reg(const InstDev* __restrict__ insts, FftArgs a) {
  typedef real_of<C> RT;
  constexpr int L = LC, Nc = L * L, N = 2 * Nc;
  constexpr int FFT_THREADS = NT;
  __shared__ C buf[NV * N];
  __shared__ C roots[L];
  const InstDev& d = insts[blockIdx.y];
  if (d.L != LC) return;
  Resolved rs = resolve(d, a);
  if (!rs.active) return;
  constexpr int nvec = ST<S>::is_complex ? N : N / 2;
  // gridDim.x is a multiple of 8, so workgroup x of every instance runs on
  // XCD x % 8; each XCD takes a run of consecutive tiles, whose row segments
  // share cache lines in that XCD's L2
  const int tile = (blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
  const int v0 = tile * NV;
  if (v0 >= nvec) return;
  const int nvl = min(NV, nvec - v0);
  const int tid = threadIdx.x;
  if (tid < L) roots[tid] = to_c<C>(d.roots[tid]);
  S* Mx = matp<S>(d, a.mat);
  const int8_t* xs = rs.slice > 0 ? d.fields + (size_t)(rs.slice - 1) * N : nullptr;
  const bool rows = a.side != 0;
  const HsDiag<C, ST<S>::is_complex> hd(d, rows);
  const bool chain = a.op == FOP_STAB_CHAIN;
  // load (+ pre diagonal): clamped loads issued in groups, then masked; a
  // group covers the thread's whole share of the tile, so the workgroup
  // waits for memory once
  const int tot = nvl * N;
  constexpr int LU = (NV * N + NT - 1) / NT < 24 ? (NV * N + NT - 1) / NT : 24;
  for (int e0 = tid; e0 < tot; e0 += LU * FFT_THREADS) {
    S raw[LU][ST<S>::is_complex ? 1 : 2];
    int8_t xr[LU];
#pragma unroll
    for (int u = 0; u < LU; ++u) {
      const int e = min(e0 + u * FFT_THREADS, tot - 1);
      int vv, r;
      if (!rows) { vv = e / N; r = e - vv * N; }
      else { vv = e % nvl; r = e / nvl; }
      const int q = v0 + vv;
      if constexpr (ST<S>::is_complex) {
        raw[u][0] = gld(rows ? Mx + (size_t)r * N + q : Mx + (size_t)q * N + r);
      } else {
        raw[u][0] = gld(rows ? Mx + (size_t)r * N + 2 * q : Mx + (size_t)(2 * q) * N + r);
        raw[u][1] = gld(rows ? Mx + (size_t)r * N + 2 * q + 1 : Mx + (size_t)(2 * q + 1) * N + r);
      }
      xr[u] = rs.pre ? xs[r] : (int8_t)1;
    }
#pragma unroll
    for (int u = 0; u < LU; ++u) {
      const int e = e0 + u * FFT_THREADS;
      if (e < tot) {
        int vv, r;
        if (!rows) { vv = e / N; r = e - vv * N; }
        else { vv = e % nvl; r = e / nvl; }
        C val;
        if constexpr (ST<S>::is_complex) val = mkc<C>(raw[u][0].x, rows ? -raw[u][0].y : raw[u][0].y);
        else val = mkc<C>(raw[u][0], raw[u][1]);
        if (rs.pre) val = hd.mul(val, (rs.pre * xr[u]) > 0, rs.cj);
        buf[vv * N + r] = val;
      }
    }
  }
  __syncthreads();
  const bool b_act = tid < nvl * 2 * L;
  const int bv = tid / (2 * L), bs = (tid % (2 * L)) / L, bk1 = tid % L;
  C* pb_own = buf + bv * N + bs * Nc + bk1;
  const int nrep = chain ? d.n_stab : 1;
  for (int rep = 0; rep < nrep; ++rep) {
    int tabi = rs.tab;
    if (chain) {   // step rep of the chain: pre diagonal in LDS
      const Resolved rj = chain_step(d, a, rep);
      tabi = rj.tab;
      if (rj.pre) {
        lds_diag(buf, tot, N, rj.pre, rj.cj, d.fields + (size_t)(rj.slice - 1) * N, hd, FFT_THREADS);
        __syncthreads();
      }
    }
    // axis 0, forward: line (vector, sublattice, n2) per thread, L consecutive points
    if (tid < nvl * 2 * L) line_dft<L, false>(buf + (tid / (2 * L)) * N + (tid % (2 * L)) * L, 1, roots);
    __syncthreads();
    // axis 1, forward: line (vector, sublattice, k1) per thread
    if (b_act) line_dft<L, false>(pb_own, L, roots);
    __syncthreads();
    if (a.op == FOP_FOURIER) break;   // forward transform only
    // 2x2 block per momentum: the thread of sublattice s forms row s of the
    // block from both lines of its column, then transforms it back
    C y[L];
    if (b_act) {
      const C* pa = buf + bv * N + bk1;
      const C* pbb = pa + Nc;
      const cplx* T = d.tab + (size_t)tabi * Nc * 4 + 2 * bs;   // row bs: (t_s0, t_s1)
#pragma unroll
      for (int k2 = 0; k2 < L; ++k2) {
        const int k = bk1 + L * k2;
        const C t0 = to_c<C>(T[4 * k]), t1 = to_c<C>(T[4 * k + 1]);
        y[k2] = t0 * pa[k2 * L] + t1 * pbb[k2 * L];
      }
    }
    __syncthreads();   // both lines read before either is overwritten
    if (b_act) {
      C x[L];
      rdft<L, L, true>(y, x, roots);
#pragma unroll
      for (int n = 0; n < L; ++n) pb_own[n * L] = x[n];
    }
    __syncthreads();
    // axis 0, inverse
    if (tid < nvl * 2 * L) line_dft<L, true>(buf + (tid / (2 * L)) * N + (tid % (2 * L)) * L, 1, roots);
    __syncthreads();
    if (chain) {   // post diagonal of step rep in LDS
      const Resolved rj = chain_step(d, a, rep);
      if (rj.post) {
        lds_diag(buf, tot, N, rj.post, rj.cj, d.fields + (size_t)(rj.slice - 1) * N, hd, FFT_THREADS);
        __syncthreads();
      }
    }
  }
  const double* dsc = chain ? d.vec[VEC_DW] : nullptr;   // chain: columns scaled by the working D
  // store (+ post diagonal)
  for (int e = tid; e < tot; e += FFT_THREADS) {
    int vv, r;
    if (!rows) { vv = e / N; r = e - vv * N; }
    else { vv = e % nvl; r = e / nvl; }
    const int q = v0 + vv;
    C val = buf[vv * N + r];
    if (rs.post) val = hd.mul(val, (rs.post * xs[r]) > 0, rs.cj);
    if (chain) {
      if constexpr (ST<S>::is_complex) val = val * (RT)dsc[q];
      else val = C{val.x * (RT)dsc[2 * q], val.y * (RT)dsc[2 * q + 1]};
    }
    const double vx = (double)val.x, vy = (double)val.y;
    if constexpr (ST<S>::is_complex) {
      if (rows) gst(Mx + (size_t)r * N + q, cmake(vx, -vy));
      else gst(Mx + (size_t)q * N + r, cmake(vx, vy));
    } else {
      if (!rows) { gst(Mx + (size_t)(2 * q) * N + r, vx); gst(Mx + (size_t)(2 * q + 1) * N + r, vy); }
      else { gst(Mx + (size_t)r * N + 2 * q, vx); gst(Mx + (size_t)r * N + 2 * q + 1, vy); }
    }
  }
}

}  // namespace

int fft_vectors_per_block(int N, size_t lds_budget, size_t elem_bytes) {
  // two ping-pong buffers of nv vectors
  int nv = (int)(lds_budget / (2 * (size_t)N * elem_bytes));
  if (nv > 16) nv = 16;
  return nv < 1 ? 1 : nv;
}

// Lattice sizes with a compile-time plan (the paper's sizes and their
// neighbours); other L run the runtime-plan kernel.
#define DQMC_FIXED_L(X) X(2) X(3) X(4) X(6) X(8) X(9) X(12) X(15) X(16) X(18) X(21) X(24) X(27) \
  X(30) X(32) X(33) X(36) X(39) X(42)

bool fft_has_fixed(int L) {
  switch (L) {
#define DQMC_CASE(v) case v:
    DQMC_FIXED_L(DQMC_CASE)
#undef DQMC_CASE
    return true;
    default: return false;
  }
}

namespace {
template <typename S, int LC, typename C, int TILE>
void launch_reg(const InstDev* insts, int n_inst, const FftArgs& a, hipStream_t s) {
  constexpr int N = 2 * LC * LC;
  constexpr int NV = reg_nv(LC, TILE), NT = reg_nt(LC, TILE);
  constexpr int nvec = ST<S>::is_complex ? N : N / 2;
  const int tiles = ((nvec + NV - 1) / NV + 7) / 8 * 8;   // a multiple of 8 (XCD-aware tile order)
  hipLaunchKernelGGL((k_fft_reg<S, LC, C, NV, NT>), dim3(tiles, n_inst), dim3(NT), 0, s, insts, a);
}

template <typename S, int LC, typename C>
void launch_fixed(const InstDev* insts, int n_inst, const FftArgs& a, size_t lds_budget, int tile, hipStream_t s) {
  constexpr int N = 2 * LC * LC;
  if constexpr (LC <= 24) {
    // register line transforms, LDS sized at compile time; the single
    // precision wraps use the wide tile only
    (void)lds_budget;
    if constexpr (sizeof(C) == sizeof(cplx)) {
      if (tile == 1) launch_reg<S, LC, C, 1>(insts, n_inst, a, s);
      else if (tile == 2) launch_reg<S, LC, C, 2>(insts, n_inst, a, s);
      else launch_reg<S, LC, C, 0>(insts, n_inst, a, s);
    } else {
      (void)tile;
      launch_reg<S, LC, C, 0>(insts, n_inst, a, s);
    }
  } else {
    (void)tile;
    int nv = fft_vectors_per_block(N, lds_budget, sizeof(C));
    int nvec = ST<S>::is_complex ? N : N / 2;
    dim3 grid(((nvec + nv - 1) / nv + 7) / 8 * 8, n_inst);
    size_t lds = 2 * (size_t)nv * N * sizeof(C);
    constexpr int R = 13;  // unused by the fixed path
    hipLaunchKernelGGL((k_fft_apply<S, R, LC, C>), grid, dim3(FFT_THREADS), lds, s, insts, a, nv, 0);
  }
}

template <typename S, typename C>
void launch_generic(const InstDev* insts, int n_inst, int Nmax, const FftArgs& a, size_t lds_budget, int rmax,
                    hipStream_t s) {
  int nv = fft_vectors_per_block(Nmax, lds_budget, sizeof(C));
  int nvec = ST<S>::is_complex ? Nmax : Nmax / 2;
  dim3 grid(((nvec + nv - 1) / nv + 7) / 8 * 8, n_inst);
  size_t lds = 2 * (size_t)nv * Nmax * sizeof(C);
  if (rmax <= 4) hipLaunchKernelGGL((k_fft_apply<S, 4, 0, C>), grid, dim3(FFT_THREADS), lds, s, insts, a, nv, 1);
  else if (rmax <= 7) hipLaunchKernelGGL((k_fft_apply<S, 7, 0, C>), grid, dim3(FFT_THREADS), lds, s, insts, a, nv, 1);
  else hipLaunchKernelGGL((k_fft_apply<S, 13, 0, C>), grid, dim3(FFT_THREADS), lds, s, insts, a, nv, 1);
}
}  // namespace

hipError_t launch_fft(const InstDev* insts, int n_inst, int Nmax, bool cplx_, const FftArgs& a,
                      size_t lds_budget, int rmax, const int* Ls, int nL, bool any_generic, bool single,
                      const int* tiles, hipStream_t s) {
  for (int q = 0; q < nL; ++q) {
    const int tile = tiles ? tiles[2 * q + (a.side != 0)] : 0;
    switch (Ls[q]) {
#define DQMC_CASE(v)                                                                         \
  case v:                                                                                    \
    if (single) {                                                                            \
      if (cplx_) launch_fixed<cplx, v, cplxf>(insts, n_inst, a, lds_budget, tile, s);        \
      else launch_fixed<double, v, cplxf>(insts, n_inst, a, lds_budget, tile, s);            \
    } else {                                                                                 \
      if (cplx_) launch_fixed<cplx, v, cplx>(insts, n_inst, a, lds_budget, tile, s);         \
      else launch_fixed<double, v, cplx>(insts, n_inst, a, lds_budget, tile, s);             \
    }                                                                                        \
    break;
      DQMC_FIXED_L(DQMC_CASE)
#undef DQMC_CASE
      default: break;
    }
  }
  if (!any_generic) return hipGetLastError();
  if (single) {
    if (cplx_) launch_generic<cplx, cplxf>(insts, n_inst, Nmax, a, lds_budget, rmax, s);
    else launch_generic<double, cplxf>(insts, n_inst, Nmax, a, lds_budget, rmax, s);
  } else {
    if (cplx_) launch_generic<cplx, cplx>(insts, n_inst, Nmax, a, lds_budget, rmax, s);
    else launch_generic<double, cplx>(insts, n_inst, Nmax, a, lds_budget, rmax, s);
  }
  return hipGetLastError();
}
