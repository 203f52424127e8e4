// Batched FP64 GEMM on the matrix cores (v_mfma_f64_16x16x4_f64).
//
// C = alpha op(A) op(B) + beta C per instance, on named per-instance matrices.
// It serves the rank-k flush of the delayed update, G <- G - X Y
// (eq. FinalDelay), and the dense products of the QR stabilisation.
// Complex128 is done with three real MFMA products per tile (Gauss: Re Re,
// Im Im and (Re + Im)(Re + Im)) on split real/imaginary LDS planes.  It also
// forms the delayed vectors of a window in matrix form (k_expand_coef,
// k_expand_mm).
//
// Tiling: 64 x 64 output tile per workgroup of four 64-wide waves, each wave
// a 32 x 32 block of 2 x 2 MFMA tiles; K is staged through LDS 16 at a time.
#include "common.hpp"
#include "kernels.hpp"

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 16, PAD = 2;
constexpr int GEMM_KB = 16;   // chunk depth of the batched GEMM
constexpr int GEMM_THREADS = 256;

__host__ __device__ __forceinline__ int dimval(GemmDim g, int n) {
  int v = g.a * n + g.b;
  if (g.hi > 0 && v > g.hi) v = g.hi;
  return v;
}
__device__ __forceinline__ size_t offval(int a, int b, int n) {
  int v = a * n + b;
  return v > 0 ? (size_t)v : 0;
}

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <typename S>
__device__ __forceinline__ void split(S v, double& re, double& im);
template <>
__device__ __forceinline__ void split<double>(double v, double& re, double& im) { re = v; im = 0.0; }
template <>
__device__ __forceinline__ void split<cplx>(cplx v, double& re, double& im) { re = v.x; im = v.y; }

__device__ __forceinline__ double shfl_xor_s(double v, int m) { return __shfl_xor(v, m); }
__device__ __forceinline__ cplx shfl_xor_s(cplx v, int m) { return cmake(__shfl_xor(v.x, m), __shfl_xor(v.y, m)); }

// Shared memory of one 64 x 64 output tile (op(A) and op(B) chunks, real
// and imaginary planes).
template <bool CX, int KB = BK>
struct GemmSmem {
  double Ar[KB][BM + PAD], Br[KB][BN + PAD];
  double Ai[CX ? KB : 1][BM + PAD], Bi[CX ? KB : 1][BN + PAD];
};

// C = alpha op(A) op(B) + beta C on the tiles tile0, tile0 + tstep, ... of
// one instance (M x NC output, depth K): the tile body shared by the batched
// GEMM and the work-queue flush.
template <typename S, int KB = BK>
__device__ __forceinline__ void gemm_tiles(const S* __restrict__ pa, const S* __restrict__ pb, S* pc, int ld,
                                           int aop, int bop, int M, int NC, int K, bool a_upper, double alpha,
                                           double beta, int tile0, int tstep, GemmSmem<ST<S>::is_complex, KB>& sm) {
  static_assert(KB == 16 || KB == 32, "chunk depth");
  constexpr int P = KB / 4;          // staged values of op(A) and of op(B) per thread
  constexpr int KROW = 256 / KB;     // rows (columns) per pass of a k-contiguous load
  constexpr bool CX = ST<S>::is_complex;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform, in a scalar register
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int tm = (M + BM - 1) / BM, tn = (NC + BN - 1) / BN;
  const int ntiles = tm * tn;

  // global -> register staging of one BK chunk (4 values of op(A), 4 of op(B)
  // per thread).  Addresses are clamped and the raw values kept with an
  // in-range mask; masking and conjugation happen in store_chunk, so the
  // loads of the next chunk stay in flight while the current one is
  // multiplied (no branch, no select right behind the loads).
  S va[P], vb[P];
  unsigned mask_a = 0, mask_b = 0;
  auto load_chunk = [&](int m0, int n0, int k0) {
    mask_a = 0;
    mask_b = 0;
#pragma unroll
    for (int p = 0; p < P; ++p) {
      int i, kk;
      if (aop == 0) { i = tid & 63; kk = (tid >> 6) + 4 * p; }
      else { kk = tid % KB; i = tid / KB + KROW * p; }
      const int gi = m0 + i, gk = k0 + kk;
      if (gi < M && gk < K && !(a_upper && gi > gk)) mask_a |= 1u << p;
      const int gic = min(gi, M - 1), gkc = min(gk, K - 1);
      va[p] = gld(pa + (aop == 0 ? gic + (size_t)gkc * ld : gkc + (size_t)gic * ld));
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
      int j, kk;
      if (bop == 0) { kk = tid % KB; j = tid / KB + KROW * p; }
      else { j = tid & 63; kk = (tid >> 6) + 4 * p; }
      const int gj = n0 + j, gk = k0 + kk;
      if (gj < NC && gk < K) mask_b |= 1u << p;
      const int gjc = min(gj, NC - 1), gkc = min(gk, K - 1);
      vb[p] = gld(pb + (bop == 0 ? gkc + (size_t)gjc * ld : gjc + (size_t)gkc * ld));
    }
  };
  auto store_chunk = [&]() {
#pragma unroll
    for (int p = 0; p < P; ++p) {
      int i, kk;
      if (aop == 0) { i = tid & 63; kk = (tid >> 6) + 4 * p; }
      else { kk = tid % KB; i = tid / KB + KROW * p; }
      double re, im;
      split<S>(va[p], re, im);
      if (aop == 2) im = -im;
      const bool in = (mask_a >> p) & 1u;
      sm.Ar[kk][i] = in ? re : 0.0;
      if constexpr (CX) sm.Ai[kk][i] = in ? im : 0.0;
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
      int j, kk;
      if (bop == 0) { kk = tid % KB; j = tid / KB + KROW * p; }
      else { j = tid & 63; kk = (tid >> 6) + 4 * p; }
      double re, im;
      split<S>(vb[p], re, im);
      if (bop == 2) im = -im;
      const bool in = (mask_b >> p) & 1u;
      sm.Br[kk][j] = in ? re : 0.0;
      if constexpr (CX) sm.Bi[kk][j] = in ? im : 0.0;
    }
  };

  for (int tile = tile0; tile < ntiles; tile += tstep) {
    const int m0 = (tile % tm) * BM, n0 = (tile / tm) * BN;
    // accumulators hold transposed 16x16 blocks: operands are fed as (B, A) so
    // that a lane owns 4 columns of one row and stores coalesce along columns
    // Complex products use three real products (Gauss): P1 = Br Ar (acc_r),
    // P2 = Bi Ai (acc_i), P3 = (Br + Bi)(Ar + Ai) (acc_p); re = P1 - P2,
    // im = P3 - P1 - P2.
    d4 acc_r[2][2], acc_i[2][2], acc_p[CX ? 2 : 1][CX ? 2 : 1];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        acc_r[i][j] = d4{0, 0, 0, 0};
        acc_i[i][j] = d4{0, 0, 0, 0};
        if constexpr (CX) acc_p[i][j] = d4{0, 0, 0, 0};
      }

    // For C = alpha (op(A) op(B)) + beta C the accumulators start at
    // (beta/alpha) C, loaded before the K loop so that the read of C overlaps
    // the products; the result is alpha * acc.
    const double cscale = (beta != 0.0 && alpha != 0.0) ? beta / alpha : 0.0;
    // upper-triangular op(A): chunks with k < m0 contribute nothing
    const int kbeg = a_upper ? (m0 / KB) * KB : 0;
    if (cscale != 0.0) {
      // the C loads, then the first chunk's loads, then C into the
      // accumulators: both round trips overlap
      S craw[2][2][4];
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            int gi = m0 + wr + ti * 16 + (lane & 15);
            int gj = n0 + wc + tj * 16 + (lane >> 4) + 4 * r;
            craw[ti][tj][r] = gld(pc + min(gi, M - 1) + (size_t)min(gj, NC - 1) * ld);
          }
      if (kbeg < K) load_chunk(m0, n0, kbeg);
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            int gi = m0 + wr + ti * 16 + (lane & 15);
            int gj = n0 + wc + tj * 16 + (lane >> 4) + 4 * r;
            const bool in = gi < M && gj < NC;
            double re, im;
            split<S>(craw[ti][tj][r], re, im);
            acc_r[ti][tj][r] = in ? cscale * re : 0.0;
            if constexpr (CX) acc_p[ti][tj][r] = in ? cscale * (re + im) : 0.0;
          }
    } else if (kbeg < K) {
      load_chunk(m0, n0, kbeg);
    }
    // 16 x 16 blocks wholly outside the output are not multiplied (edge tiles
    // of sizes that are not multiples of 64 leave up to 3/4 of a tile empty)
    const bool vi0 = m0 + wr < M, vi1 = m0 + wr + 16 < M;
    const bool vj0 = n0 + wc < NC, vj1 = n0 + wc + 16 < NC;
    auto kstep = [&](int kr) {
      double ar[2], br[2], ai[2], bi[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        ar[t] = sm.Ar[kr][wr + t * 16 + (lane & 15)];
        br[t] = sm.Br[kr][wc + t * 16 + (lane & 15)];
        if constexpr (CX) {
          ai[t] = sm.Ai[kr][wr + t * 16 + (lane & 15)];
          bi[t] = sm.Bi[kr][wc + t * 16 + (lane & 15)];
        }
      }
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) {
          if ((ti ? vi1 : vi0) && (tj ? vj1 : vj0)) {
            acc_r[ti][tj] = mfma(br[tj], ar[ti], acc_r[ti][tj]);
            if constexpr (CX) {
              acc_i[ti][tj] = mfma(bi[tj], ai[ti], acc_i[ti][tj]);
              acc_p[ti][tj] = mfma(br[tj] + bi[tj], ar[ti] + ai[ti], acc_p[ti][tj]);
            }
          }
        }
    };
    for (int k0 = kbeg; k0 < K; k0 += KB) {
      store_chunk();
      __syncthreads();
      if (k0 + KB < K) load_chunk(m0, n0, k0 + KB);
      if (k0 + KB <= K) {   // full chunk: unrolled
#pragma unroll
        for (int ks = 0; ks < KB / 4; ++ks) kstep(ks * 4 + (lane >> 4));
      } else {
        const int ksn = (K - k0 + 3) / 4;
#pragma unroll 1
        for (int ks = 0; ks < ksn; ++ks) kstep(ks * 4 + (lane >> 4));
      }
      __syncthreads();
    }
    // ---- epilogue.  v_mfma_f64_16x16x4f64 leaves D[l/16 + 4r][l%16] in lane l
    //      (layout checked on the device); with operands swapped that is
    //      C[row = l%16][col = l/16 + 4r] of the block.
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int gi = m0 + wr + ti * 16 + (lane & 15);
          int gj = n0 + wc + tj * 16 + (lane >> 4) + 4 * r;
          if (gi < M && gj < NC) {
            S* cp = pc + gi + (size_t)gj * ld;
            if constexpr (CX) {
              const double p1 = acc_r[ti][tj][r], p2 = acc_i[ti][tj][r];
              cplx v = cmake(alpha * (p1 - p2), alpha * (acc_p[ti][tj][r] - p1 - p2));
              if (beta != 0.0 && cscale == 0.0) v = v + beta * (*cp);
              *cp = v;
            } else {
              double v = alpha * acc_r[ti][tj][r];
              if (beta != 0.0 && cscale == 0.0) v += beta * (*cp);
              *cp = v;
            }
          }
        }
  }
}

// ROLE only separates the flush instantiation (1) from the stabilisation
// products (0) in profiles; the code is the same.
template <typename S, int ROLE>
__global__ void __launch_bounds__(GEMM_THREADS, 2)
k_gemm(const InstDev* __restrict__ insts, int n_inst, GemmOperand A, GemmOperand B, GemmOperand C,
       GemmDim Md, GemmDim Nd, GemmDim Kd, double alpha, double beta, int flags) {
  int inst, bx;
  xcd_slot(n_inst, inst, bx);
  if (inst < 0) return;
  const InstDev& d = insts[inst];
  const int Nn = d.N;
  const InstState& st = *d.st;
  if (st.idle) return;
  if ((flags & GF_SKIP_INIT) && st.init_mode) return;
  if ((flags & GF_IF_FULL) && st.fill < d.kflush) return;
  if ((flags & GF_IF_ANY) && st.fill <= 0) return;
  const int M = dimval(Md, Nn);
  int NC = dimval(Nd, Nn);
  if (flags & GF_NC_MW) NC = min(NC, st.m_w);
  const int K = (flags & GF_K_FILL) ? st.fill : dimval(Kd, Nn);
  if (M <= 0 || NC <= 0) return;
  const int ld = Nn;
  const S* pa = reinterpret_cast<const S*>(mat_ptr(d, A.id)) + offval(A.ra, A.rb, Nn) + offval(A.ca, A.cb, Nn) * ld;
  const S* pb = reinterpret_cast<const S*>(mat_ptr(d, B.id)) + offval(B.ra, B.rb, Nn) + offval(B.ca, B.cb, Nn) * ld;
  S* pc = reinterpret_cast<S*>(mat_ptr(d, C.id)) + offval(C.ra, C.rb, Nn) + offval(C.ca, C.cb, Nn) * ld;
  __shared__ GemmSmem<ST<S>::is_complex, GEMM_KB> sm;
  gemm_tiles<S, GEMM_KB>(pa, pb, pc, ld, A.op, B.op, M, NC, K, (flags & GF_A_UPPER) != 0, alpha, beta, bx,
                         gridDim.x, sm);
}

// Flush without LDS: G <- G - X Y with X column-major N x K (op N) and Y
// stored as Y[m, j] at m*N + j (op T on a column-major N x K buffer).  Each
// wave owns a 32 x 32 block of G and reads its MFMA fragments straight from
// memory: lane l needs X[i0 + l%16, k + l/16] and Y[k + l/16, j0 + l%16], i.e.
// 16 consecutive elements per k, so every fragment load is coalesced and no
// barrier is needed.  The next k-step's fragments are loaded while the
// current one is multiplied.
template <typename S>
__global__ void __launch_bounds__(256)
k_flush_direct(const InstDev* __restrict__ insts, int n_inst, int flags) {
  constexpr bool CX = ST<S>::is_complex;
  int inst, bx;
  xcd_slot(n_inst, inst, bx);
  if (inst < 0) return;
  const InstDev& d = insts[inst];
  const InstState& st = *d.st;
  if (st.idle || st.init_mode) return;
  if ((flags & GF_IF_FULL) && st.fill < d.kflush) return;
  if ((flags & GF_IF_ANY) && st.fill <= 0) return;
  const int N = d.N;
  const int K = st.fill;
  const S* X = reinterpret_cast<const S*>(d.mat[MAT_X]);
  const S* Y = reinterpret_cast<const S*>(d.mat[MAT_Y]);
  S* G = reinterpret_cast<S*>(d.mat[MAT_G]);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nb32 = (N + 31) / 32;
  const int nblk = nb32 * nb32;
  const int lr = lane & 15, lk = lane >> 4;
  for (int blk = bx * 4 + wave; blk < nblk; blk += gridDim.x * 4) {
    const int i0 = (blk % nb32) * 32, j0 = (blk / nb32) * 32;
    // [ti][tj] accumulators (transposed blocks).  Complex products use three
    // real products (Gauss): P1 = Yr Xr, P2 = Yi Xi, P3 = (Yr + Yi)(Xr + Xi),
    // re = P1 - P2, im = P3 - P1 - P2.  The accumulators start from -G
    // (P1 at -Re G, P3 at -Re G - Im G) so that acc = X Y - G, G_new = -acc.
    // Every load reads a clamped, valid address and out-of-range values are
    // zeroed afterwards, so that no load sits behind a branch (and its wait).
    d4 ar_[2][2], ai_[2][2], ap_[CX ? 2 : 1][CX ? 2 : 1];
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gi = i0 + ti * 16 + lr, gj = j0 + tj * 16 + lk + 4 * r;
          const bool in = gi < N && gj < N;
          double re, im;
          split<S>(gld(G + min(gi, N - 1) + (size_t)min(gj, N - 1) * N), re, im);
          ar_[ti][tj][r] = in ? -re : 0.0;
          ai_[ti][tj][r] = 0.0;
          if constexpr (CX) ap_[ti][tj][r] = in ? -re - im : 0.0;
        }
    auto frag = [&](int k, double (&xr)[2], double (&xi)[2], double (&yr)[2], double (&yi)[2]) {
      const int kk = k + lk;
      const bool kin = kk < K;
      const size_t kc = (size_t)(kin ? kk : 0) * N;
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int gi = i0 + t * 16 + lr, gj = j0 + t * 16 + lr;
        const bool xin = kin && gi < N, yin = kin && gj < N;
        double a, b, c, e;
        split<S>(gld(X + min(gi, N - 1) + kc), a, b);
        split<S>(gld(Y + kc + min(gj, N - 1)), c, e);
        xr[t] = xin ? a : 0.0; xi[t] = xin ? b : 0.0;
        yr[t] = yin ? c : 0.0; yi[t] = yin ? e : 0.0;
      }
    };
    // fragments one k-step ahead; independent accumulators interleaved so
    // that no MFMA waits on the one just issued
    double xr[2], xi[2], yr[2], yi[2];
    frag(0, xr, xi, yr, yi);
    for (int k = 0; k < K; k += 4) {
      double nxr[2], nxi[2], nyr[2], nyi[2];
      frag(k + 4, nxr, nxi, nyr, nyi);
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) ar_[ti][tj] = mfma(yr[tj], xr[ti], ar_[ti][tj]);
      if constexpr (CX) {
        double xs[2], ys[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) { xs[t] = xr[t] + xi[t]; ys[t] = yr[t] + yi[t]; }
#pragma unroll
        for (int ti = 0; ti < 2; ++ti)
#pragma unroll
          for (int tj = 0; tj < 2; ++tj) ai_[ti][tj] = mfma(yi[tj], xi[ti], ai_[ti][tj]);
#pragma unroll
        for (int ti = 0; ti < 2; ++ti)
#pragma unroll
          for (int tj = 0; tj < 2; ++tj) ap_[ti][tj] = mfma(ys[tj], xs[ti], ap_[ti][tj]);
      }
#pragma unroll
      for (int t = 0; t < 2; ++t) { xr[t] = nxr[t]; xi[t] = nxi[t]; yr[t] = nyr[t]; yi[t] = nyi[t]; }
    }
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int gi = i0 + ti * 16 + lr, gj = j0 + tj * 16 + lk + 4 * r;
          if (gi < N && gj < N) {
            if constexpr (CX) {
              const double p1 = ar_[ti][tj][r], p2 = ai_[ti][tj][r];
              gst(G + gi + (size_t)gj * N, cmake(p2 - p1, p1 + p2 - ap_[ti][tj][r]));
            } else {
              gst(G + gi + (size_t)gj * N, -ar_[ti][tj][r]);
            }
          }
        }
  }
}

// Flush from device work queues: G <- G - X Y over all instances of the
// launch with persistent workgroups.  The output is cut into 64 x 64 tiles
// (a 32 x 32 block per wave); the instances are dealt to nq queues (8, one per
// XCD label, when the launch has at least 8 instances, else 1) and workgroup w
// serves queue w % nq, so with the round-robin dispatch of workgroups to XCDs
// the tiles of an instance are computed in one L2.  A workgroup takes the next
// tile of its queue with one atomic ticket; tickets past the queue's total end
// the loop, and the last workgroup of a queue to finish resets its counters
// (kept in the InstState of the launch's first instance), so no clearing
// launch is needed between flushes.
//
// Each tile runs the LDS-staged body of the batched GEMM (X and Y chunks of
// 16 shared by the four waves).
constexpr int FQ_T = BM;   // tile edge
template <typename S>
__device__ __forceinline__ bool fq_active(const InstDev& d, int flags) {
  const InstState& st = *d.st;
  if (st.idle || st.init_mode) return false;
  if ((flags & GF_IF_FULL) && st.fill < d.kflush) return false;
  if ((flags & GF_IF_ANY) && st.fill <= 0) return false;
  return true;
}

template <typename S>
__global__ void __launch_bounds__(GEMM_THREADS, 2)
k_flush_queue(const InstDev* __restrict__ insts, int n_inst, int flags) {
  const int nq = n_inst >= N_XCD ? N_XCD : 1;
  const int q = blockIdx.x % nq;
  const int wpq = gridDim.x / nq;
  InstState* qs = insts[0].st;
  const int tid = threadIdx.x;
  __shared__ int sh_t;
  __shared__ GemmSmem<ST<S>::is_complex> sm;
  // tiles of this queue: instances q, q + nq, ... that flush in this launch
  int total = 0;
  for (int i = q; i < n_inst; i += nq) {
    if (!fq_active<S>(insts[i], flags)) continue;
    const int nt = (insts[i].N + FQ_T - 1) / FQ_T;
    total += nt * nt;
  }
  for (;;) {
    if (tid == 0) sh_t = atomicAdd(&qs->fq_next[q], 1);
    __syncthreads();
    int t = sh_t;
    __syncthreads();
    if (t >= total) break;
    // ticket -> (instance, tile)
    int inst = q, nt = 1;
    for (int i = q; i < n_inst; i += nq) {
      if (!fq_active<S>(insts[i], flags)) continue;
      nt = (insts[i].N + FQ_T - 1) / FQ_T;
      inst = i;
      if (t < nt * nt) break;
      t -= nt * nt;
    }
    const InstDev& d = insts[inst];
    const int N = d.N;
    // G <- G - X Y: A = X (N x fill, column-major), B = Y read transposed
    gemm_tiles<S>(reinterpret_cast<const S*>(d.mat[MAT_X]), reinterpret_cast<const S*>(d.mat[MAT_Y]),
                  reinterpret_cast<S*>(d.mat[MAT_G]), N, 0, 1, N, N, d.st->fill, false, -1.0, 1.0, t, 1 << 30, sm);
  }
  // the last workgroup of the queue resets it for the next launch (every
  // workgroup of the queue has taken its final ticket before counting itself)
  if (tid == 0) {
    __threadfence();
    const int done = atomicAdd(&qs->fq_done[q], 1);
    if (done == wpq - 1) {
      atomicExch(&qs->fq_next[q], 0);
      atomicExch(&qs->fq_done[q], 0);
    }
  }
}

// Single-precision flush for mixed-precision instances: the product X Y is
// formed with FP32 MFMA 16x16x4 (X and Y rounded to float on load, FP32
// accumulation) and subtracted from the FP64 G.  Same block structure as the
// FP64 kernel; the FP32 MFMA result of lane l holds column l%16 of the
// transposed block at rows 4(l/16) + r.
typedef float f4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ f4 mfma32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename S>
__global__ void __launch_bounds__(256)
k_flush_f32(const InstDev* __restrict__ insts, int n_inst, int flags) {
  constexpr bool CX = ST<S>::is_complex;
  int inst, bx;
  xcd_slot(n_inst, inst, bx);
  if (inst < 0) return;
  const InstDev& d = insts[inst];
  const InstState& st = *d.st;
  if (st.idle || st.init_mode) return;
  if ((flags & GF_IF_FULL) && st.fill < d.kflush) return;
  if ((flags & GF_IF_ANY) && st.fill <= 0) return;
  const int N = d.N;
  const int K = st.fill;
  const S* X = reinterpret_cast<const S*>(d.mat[MAT_X]);
  const S* Y = reinterpret_cast<const S*>(d.mat[MAT_Y]);
  S* G = reinterpret_cast<S*>(d.mat[MAT_G]);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nb32 = (N + 31) / 32;
  const int nblk = nb32 * nb32;
  const int lr = lane & 15, lk = lane >> 4;
  for (int blk = bx * 4 + wave; blk < nblk; blk += gridDim.x * 4) {
    const int i0 = (blk % nb32) * 32, j0 = (blk / nb32) * 32;
    f4 ar_[2][2], ai_[2][2];
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj) { ar_[ti][tj] = f4{0, 0, 0, 0}; ai_[ti][tj] = f4{0, 0, 0, 0}; }
    auto frag = [&](int k, float (&xr)[2], float (&xi)[2], float (&yr)[2], float (&yi)[2]) {
      const int kk = k + lk;
      const bool kin = kk < K;
      const size_t kc = (size_t)(kin ? kk : 0) * N;
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int gi = i0 + t * 16 + lr, gj = j0 + t * 16 + lr;
        const bool xin = kin && gi < N, yin = kin && gj < N;
        double a, b, c, e;
        split<S>(gld(X + min(gi, N - 1) + kc), a, b);
        split<S>(gld(Y + kc + min(gj, N - 1)), c, e);
        xr[t] = xin ? (float)a : 0.f; xi[t] = xin ? (float)b : 0.f;
        yr[t] = yin ? (float)c : 0.f; yi[t] = yin ? (float)e : 0.f;
      }
    };
    float xr[2], xi[2], yr[2], yi[2], nxr[2], nxi[2], nyr[2], nyi[2];
    frag(0, xr, xi, yr, yi);
    frag(4, nxr, nxi, nyr, nyi);
    for (int k = 0; k < K; k += 4) {
      float mxr[2], mxi[2], myr[2], myi[2];
      frag(k + 8, mxr, mxi, myr, myi);
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) ar_[ti][tj] = mfma32(yr[tj], xr[ti], ar_[ti][tj]);
      if constexpr (CX) {
#pragma unroll
        for (int ti = 0; ti < 2; ++ti)
#pragma unroll
          for (int tj = 0; tj < 2; ++tj) ai_[ti][tj] = mfma32(yi[tj], xr[ti], ai_[ti][tj]);
#pragma unroll
        for (int ti = 0; ti < 2; ++ti)
#pragma unroll
          for (int tj = 0; tj < 2; ++tj) ar_[ti][tj] = mfma32(-yi[tj], xi[ti], ar_[ti][tj]);
#pragma unroll
        for (int ti = 0; ti < 2; ++ti)
#pragma unroll
          for (int tj = 0; tj < 2; ++tj) ai_[ti][tj] = mfma32(yr[tj], xi[ti], ai_[ti][tj]);
      }
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        xr[t] = nxr[t]; xi[t] = nxi[t]; yr[t] = nyr[t]; yi[t] = nyi[t];
        nxr[t] = mxr[t]; nxi[t] = mxi[t]; nyr[t] = myr[t]; nyi[t] = myi[t];
      }
    }
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int gi = i0 + ti * 16 + lr, gj = j0 + tj * 16 + 4 * lk + r;
          if (gi < N && gj < N) {
            S& g = G[gi + (size_t)gj * N];
            if constexpr (CX) g = cmake(g.x - (double)ar_[ti][tj][r], g.y - (double)ai_[ti][tj][r]);
            else g = g - (double)ar_[ti][tj][r];
          }
        }
  }
}

// ---- submatrix update of a window (Sec. III B) ---------------------------------------------
// The accepted flips S of a window change G as one multi-site flip (the final
// G depends only on which fields flipped):
//   G' = G - G[:, S] Delta_S (1 + (1 - G)_SS Delta_S)^{-1} (1 - G)[S, :],
// block Sherman-Morrison with G the window's starting G (the previous window
// flushed).  k_submatrix_coef inverts Q = 1 + (1 - G_SS) Delta_S (m x m) by
// Gauss-Jordan elimination in the order of acceptance, whose pivots are the
// sequential ratios r_k (no interchanges: the same divisions as the
// single-site updates), and stores M~ = P Delta_S Q^{-1} in W2 (row s_r of
// the window for accepted flip r, zero rows elsewhere).  X = G[:, window] M~
// is then a GEMM and Y the rows (1 - G)[S, :] (k_submatrix_rows).
template <typename S>
__global__ void __launch_bounds__(256) k_submatrix_coef(const InstDev* __restrict__ insts) {
  const InstDev& d = insts[blockIdx.y];
  const InstState& st = *d.st;
  if (st.idle || st.init_mode) return;
  const int m = st.m_w;
  if (m == 0) return;
  const int N = d.N, w0 = st.wstart, wn = st.wlen;
  constexpr int WM = DQMC_WMAX, CPT = 2 * WM / 4;   // augmented columns per thread
  const S* wc = reinterpret_cast<const S*>(d.wcoef);
  const S* G = matp<S>(d, MAT_G);
  S* Mt = matp<S>(d, MAT_W2);
  // [Q | 1] held in registers: row rr = tid / 4 in the four lanes 4 rr .. 4 rr + 3
  // (one wave), lane cg of them owns the augmented columns cg + 4 j.  The next
  // pivot row (scaled) and pivot column go through a double-buffered LDS area,
  // one barrier per elimination step.
  __shared__ S prow[2][2 * WM], pcol[2][WM];
  __shared__ S dl[WM];
  __shared__ int site[WM];
  const int tid = threadIdx.x, rr = tid >> 2, cg = tid & 3;
  if (tid < WM) {
    site[tid] = tid < m ? d.acc_site[tid] : 0;
    dl[tid] = tid < m ? wc[DQMC_WC_D + tid] : ST<S>::zero();
  }
  for (int e = tid; e < wn * m; e += 256) {   // zero the window rows of M~
    const int a = e % wn, c = e / wn;
    Mt[a + (size_t)c * N] = ST<S>::zero();
  }
  __syncthreads();
  const bool live = rr < m;
  S q[CPT];
  // all loads of G_SS first (clamped addresses), then the entries of Q
  const int srow = w0 + site[min(rr, m - 1)];
#pragma unroll
  for (int j = 0; j < CPT / 2; ++j) {
    const int c = min(cg + 4 * j, m - 1);
    q[j] = gld(G + srow + (size_t)(w0 + site[c]) * N);
  }
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    const int c = cg + 4 * j;
    S v = ST<S>::zero();
    if (j < CPT / 2 && c < m) {
      v = ((rr == c ? ST<S>::one() : ST<S>::zero()) - q[j]) * dl[c];
      if (rr == c) v = v + ST<S>::one();
    } else if (c >= m && c - m == rr) {
      v = ST<S>::one();
    }
    q[j] = live ? v : ST<S>::zero();
  }
  // publish row 0 (scaled) and column 0 for the first step
  auto publish = [&](int k, int buf) {
    // pivot Q[k][k] sits in lane cg = k % 4 of row k, slot k / 4
    S piv = ST<S>::zero();
#pragma unroll
    for (int j = 0; j < CPT; ++j)
      if (cg + 4 * j == k) piv = q[j];
    piv = piv + shfl_xor_s(piv, 1);
    piv = piv + shfl_xor_s(piv, 2);   // the other lanes of the row hold zero here
    if (rr == k) {
      const S inv = cdiv(ST<S>::one(), piv);
#pragma unroll
      for (int j = 0; j < CPT; ++j) {
        const int c = cg + 4 * j;
        if (c < 2 * m) prow[buf][c] = q[j] * inv;
      }
    }
    if (live) {
#pragma unroll
      for (int j = 0; j < CPT; ++j)
        if (cg + 4 * j == k) pcol[buf][rr] = q[j];
    }
  };
  publish(0, 0);
  __syncthreads();
  for (int k = 0; k < m; ++k) {
    const int buf = k & 1;
    if (live) {
      const S f = pcol[buf][rr];
#pragma unroll
      for (int j = 0; j < CPT; ++j) {
        const int c = cg + 4 * j;
        if (c < 2 * m) q[j] = rr == k ? prow[buf][c] : q[j] - f * prow[buf][c];
      }
    }
    if (k + 1 < m) publish(k + 1, buf ^ 1);
    __syncthreads();
  }
  // M~[s_r][c] = Delta_r (Q^{-1})[r][c]
  if (live) {
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      const int c = cg + 4 * j - m;
      if (c >= 0 && c < m) Mt[site[rr] + (size_t)c * N] = dl[rr] * q[j];
    }
  }
}

// Y[k, j] = delta_{j, w0 + s_k} - G[w0 + s_k, j] for the accepted flips k of
// the window; a 64-column tile through LDS, read down the window rows and
// written along the rows of Y.
template <typename S>
__global__ void __launch_bounds__(256) k_submatrix_rows(const InstDev* __restrict__ insts) {
  const InstDev& d = insts[blockIdx.y];
  const InstState& st = *d.st;
  if (st.idle || st.init_mode) return;
  const int m = st.m_w;
  const int N = d.N;
  const int j0 = blockIdx.x * 64;
  if (m == 0 || j0 >= N) return;
  const int w0 = st.wstart;
  const S* G = matp<S>(d, MAT_G);
  S* Y = matp<S>(d, MAT_Y);
  __shared__ S T[DQMC_WMAX][65];
  __shared__ int site[DQMC_WMAX];
  const int tid = threadIdx.x;
  if (tid < DQMC_WMAX) site[tid] = tid < m ? d.acc_site[tid] : 0;
  __syncthreads();
  const int cols = min(64, N - j0);
  for (int e = tid; e < m * cols; e += 256) {
    const int k = e % m, jj = e / m;
    const int gi = w0 + site[k];
    S v = -G[gi + (size_t)(j0 + jj) * N];
    if (gi == j0 + jj) v = v + ST<S>::one();
    T[k][jj] = v;
  }
  __syncthreads();
  for (int e = tid; e < m * cols; e += 256) {
    const int jj = e % cols, k = e / cols;
    Y[(size_t)k * N + j0 + jj] = T[k][jj];
  }
}

// ---- the delayed vectors of a window in matrix form (eq. DelayRgenk) --------------------
// For the m accepted sites s_0 < .. < s_{m-1} of a window (positions in the
// window, global w0 + s_k) the recursion
//   x_k = c_k (a_k - sum_{q<k} x_q u_qk),   u_qk = y_q[w0 + s_k] (window part),
//   y_k = b_k + sum_{q<k} v_kq y_q,          v_kq = x_q[w0 + s_k] (window part),
// with a_k = (G - X Y)[:, w0 + s_k] and b_k = (1 - G + X Y)[w0 + s_k, :] over the
// pending terms, is linear in the a's and b's:
//   x_k = sum_r a_r Tx[r][k],  Tx[r][k] = c_k (delta_rk - sum_{r<=q<k} Tx[r][q] u_qk),
//   y_k = sum_c Ty[k][c] b_c,  Ty[k][c] = delta_kc + sum_{c<=q<k} v_kq Ty[q][c].
// k_expand_coef forms Tx (rows placed at the window positions s_r, in W2) and
// Ty^T (rows at s_c, in QA), one workgroup per instance; k_expand_mm then forms
// X[:, f:f+m] = A~ Tx~ and Y[f:f+m, :] = (B~^T Ty~^T)^T per 64-row block with the
// GEMM tile body, A~ = (G - X Y)[:, w0 + 0..wn) in W1 and B~ = (1 - G + X Y)
// restricted to the window rows in W3 (row a of the window at W3[a + j N]).
// Both kernels read the window's table (c_k, window parts of x_q and y_q).
template <typename S>
__global__ void __launch_bounds__(256) k_expand_coef(const InstDev* __restrict__ insts) {
  const InstDev& d = insts[blockIdx.y];
  const InstState& st = *d.st;
  if (st.idle || st.init_mode) return;
  const int m = st.m_w;
  if (m == 0) return;
  const int N = d.N, wn = st.wlen;
  constexpr int WM = DQMC_WMAX;
  const S* wc = reinterpret_cast<const S*>(d.wcoef);
  S* Tx = matp<S>(d, MAT_W2);
  S* TyT = matp<S>(d, MAT_QA);
  __shared__ S Uk[WM][WM];   // Uk[k][q] = u_qk, later v_kq
  __shared__ S Tq[WM][WM];   // Tq[q][r] = Tx[r][q], later Ty[q][c]
  __shared__ int site[WM];
  __shared__ S cks[WM];      // c_k
  const int tid = threadIdx.x;
  if (tid < WM) {
    site[tid] = tid < m ? d.acc_site[tid] : 0;
    cks[tid] = tid < m ? wc[tid] : ST<S>::zero();
  }
  // zero the window rows of both coefficient blocks
  for (int e = tid; e < wn * m; e += 256) {
    const int a = e % wn, k = e / wn;
    Tx[a + (size_t)k * N] = ST<S>::zero();
    TyT[a + (size_t)k * N] = ST<S>::zero();
  }
  __syncthreads();
  for (int e = tid; e < m * m; e += 256) {
    const int k = e / m, q = e % m;
    Uk[k][q] = q < k ? wc[DQMC_WC_Y + q * WM + site[k]] : ST<S>::zero();
  }
  __syncthreads();
  // Tx: four lanes per row r split the sum over q.  A row only reads its own
  // earlier entries, written by a lane of the same wave: LDS operations of
  // one wave take effect in program order, so no workgroup barrier is needed
  // between the steps (the wavefront fences keep the compiler from moving
  // them).
  const int r = tid >> 2, part = tid & 3;
  for (int k = 0; k < m; ++k) {
    S sum = ST<S>::zero();
    if (r < m && k >= r)
      for (int q = r + part; q < k; q += 4) sum = sum + Tq[q][r] * Uk[k][q];
    sum = sum + shfl_xor_s(sum, 1);
    sum = sum + shfl_xor_s(sum, 2);
    if (r < m && k >= r && part == 0) Tq[k][r] = cks[k] * ((k == r ? ST<S>::one() : ST<S>::zero()) - sum);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  __syncthreads();
  for (int e = tid; e < m * m; e += 256) {
    const int k = e / m, rr = e % m;
    if (k >= rr) Tx[site[rr] + (size_t)k * N] = Tq[k][rr];
  }
  __syncthreads();
  for (int e = tid; e < m * m; e += 256) {
    const int k = e / m, q = e % m;
    Uk[k][q] = q < k ? wc[DQMC_WC_X + q * WM + site[k]] : ST<S>::zero();
  }
  __syncthreads();
  // Ty: four lanes per column c (a column only reads its own entries)
  const int c = r;
  for (int k = 0; k < m; ++k) {
    S sum = ST<S>::zero();
    if (c < m && k >= c)
      for (int q = c + part; q < k; q += 4) sum = sum + Uk[k][q] * Tq[q][c];
    sum = sum + shfl_xor_s(sum, 1);
    sum = sum + shfl_xor_s(sum, 2);
    if (c < m && k >= c && part == 0) Tq[k][c] = (k == c ? ST<S>::one() : ST<S>::zero()) + sum;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  __syncthreads();
  for (int e = tid; e < m * m; e += 256) {
    const int k = e / m, cc = e % m;
    if (k >= cc) TyT[site[cc] + (size_t)k * N] = Tq[k][cc];
  }
}

template <typename S>
__global__ void __launch_bounds__(GEMM_THREADS, 2) k_expand_mm(const InstDev* __restrict__ insts, int n_inst) {
  int inst, bx;
  xcd_slot(n_inst, inst, bx);
  if (inst < 0) return;
  const InstDev& d = insts[inst];
  const InstState& st = *d.st;
  if (st.idle || st.init_mode) return;
  const int m = st.m_w;
  const int N = d.N;
  const int j0 = bx * BM;
  if (m == 0 || j0 >= N) return;
  const int f = st.fill, w0 = st.wstart, wn = st.wlen;
  const int rows = min(BM, N - j0);
  const S* G = matp<S>(d, MAT_G);
  S* X = matp<S>(d, MAT_X);
  S* Y = matp<S>(d, MAT_Y);
  S* W1 = matp<S>(d, MAT_W1);
  S* W3 = matp<S>(d, MAT_W3);
  const S* Tx = matp<S>(d, MAT_W2);
  const S* TyT = matp<S>(d, MAT_QA);
  __shared__ GemmSmem<ST<S>::is_complex> sm;
  const int tid = threadIdx.x;
  // A~ = G[j0.., w0..] and B~ (window rows of 1 - G, as W3[a + j N]); both
  // copies read 64 consecutive elements per column
  for (int e = tid; e < rows * wn; e += GEMM_THREADS) {
    const int i = e % rows, a = e / rows;
    W1[(j0 + i) + (size_t)a * N] = G[(j0 + i) + (size_t)(w0 + a) * N];
  }
  for (int e = tid; e < wn * rows; e += GEMM_THREADS) {
    const int a = e % wn, j = e / wn;
    S v = -G[(w0 + a) + (size_t)(j0 + j) * N];
    if (w0 + a == j0 + j) v = v + ST<S>::one();
    W3[a + (size_t)(j0 + j) * N] = v;
  }
  __syncthreads();
  if (f > 0) {
    // A~ -= X[j0.., :f] Y[:f, w0..];   B~ += X[w0.., :f] Y[:f, j0..]
    gemm_tiles<S>(X + j0, Y + w0, W1 + j0, N, 0, 1, rows, wn, f, false, -1.0, 1.0, 0, 1, sm);
    __syncthreads();
    gemm_tiles<S>(X + w0, Y + j0, W3 + (size_t)j0 * N, N, 0, 1, wn, rows, f, false, 1.0, 1.0, 0, 1, sm);
    __syncthreads();
  }
  // X[j0.., f..f+m) = A~ Tx~;  Y[f..f+m, j0..] = B~^T Ty~^T (as columns of Y's column-major view)
  gemm_tiles<S>(W1 + j0, Tx, X + j0 + (size_t)f * N, N, 0, 0, rows, m, wn, false, 1.0, 0.0, 0, 1, sm);
  __syncthreads();
  gemm_tiles<S>(W3 + (size_t)j0 * N, TyT, Y + j0 + (size_t)f * N, N, 1, 0, rows, m, wn, false, 1.0, 0.0, 0, 1, sm);
}

}  // namespace

hipError_t launch_gemm(const InstDev* insts, int n_inst, int Nmax, bool cplx_, GemmOperand A,
                       GemmOperand B, GemmOperand C, GemmDim M, GemmDim Nn, GemmDim K,
                       double alpha, double beta, int flags, hipStream_t s) {
  int Mx = dimval(M, Nmax), Nx = dimval(Nn, Nmax);
  if (Mx <= 0 || Nx <= 0) return hipSuccess;
  // one output tile per workgroup (the grid's x extent is the tile count)
  int gx = ((Mx + BM - 1) / BM) * ((Nx + BN - 1) / BN);
  dim3 grid(gx, xcd_grid_y(n_inst));
  const bool fl = flags & GF_K_FILL;
  if (cplx_) {
    if (fl) hipLaunchKernelGGL((k_gemm<cplx, 1>), grid, dim3(GEMM_THREADS), 0, s, insts, n_inst, A, B, C, M, Nn, K, alpha, beta, flags);
    else hipLaunchKernelGGL((k_gemm<cplx, 0>), grid, dim3(GEMM_THREADS), 0, s, insts, n_inst, A, B, C, M, Nn, K, alpha, beta, flags);
  } else {
    if (fl) hipLaunchKernelGGL((k_gemm<double, 1>), grid, dim3(GEMM_THREADS), 0, s, insts, n_inst, A, B, C, M, Nn, K, alpha, beta, flags);
    else hipLaunchKernelGGL((k_gemm<double, 0>), grid, dim3(GEMM_THREADS), 0, s, insts, n_inst, A, B, C, M, Nn, K, alpha, beta, flags);
  }
  return hipGetLastError();
}

hipError_t launch_flush_queue(const InstDev* insts, int n_inst, bool cplx_, int flags, int n_wg, hipStream_t s) {
  const int nq = n_inst >= N_XCD ? N_XCD : 1;
  int g = n_wg / nq * nq;
  if (g < nq) g = nq;
  if (cplx_) hipLaunchKernelGGL(k_flush_queue<cplx>, dim3(g), dim3(256), 0, s, insts, n_inst, flags);
  else hipLaunchKernelGGL(k_flush_queue<double>, dim3(g), dim3(256), 0, s, insts, n_inst, flags);
  return hipGetLastError();
}

hipError_t launch_flush_direct(const InstDev* insts, int n_inst, int Nmax, bool cplx_, bool single, int flags,
                               hipStream_t s) {
  int nb32 = (Nmax + 31) / 32;
  int blocks = (nb32 * nb32 + 3) / 4;
  int cap = 8192 / (n_inst > 0 ? n_inst : 1);
  if (cap < 16) cap = 16;
  dim3 grid(blocks < cap ? blocks : cap, xcd_grid_y(n_inst));
  if (single) {
    if (cplx_) hipLaunchKernelGGL(k_flush_f32<cplx>, grid, dim3(256), 0, s, insts, n_inst, flags);
    else hipLaunchKernelGGL(k_flush_f32<double>, grid, dim3(256), 0, s, insts, n_inst, flags);
    return hipGetLastError();
  }
  if (cplx_) hipLaunchKernelGGL(k_flush_direct<cplx>, grid, dim3(256), 0, s, insts, n_inst, flags);
  else hipLaunchKernelGGL(k_flush_direct<double>, grid, dim3(256), 0, s, insts, n_inst, flags);
  return hipGetLastError();
}

hipError_t launch_expand_mm(const InstDev* insts, int n_inst, int Nmax, bool cplx_, hipStream_t s) {
  if (cplx_) hipLaunchKernelGGL(k_expand_coef<cplx>, dim3(1, n_inst), dim3(256), 0, s, insts);
  else hipLaunchKernelGGL(k_expand_coef<double>, dim3(1, n_inst), dim3(256), 0, s, insts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  dim3 grid((Nmax + BM - 1) / BM, xcd_grid_y(n_inst));
  if (cplx_) hipLaunchKernelGGL(k_expand_mm<cplx>, grid, dim3(GEMM_THREADS), 0, s, insts, n_inst);
  else hipLaunchKernelGGL(k_expand_mm<double>, grid, dim3(GEMM_THREADS), 0, s, insts, n_inst);
  return hipGetLastError();
}

hipError_t launch_submatrix_coef(const InstDev* insts, int n_inst, bool cplx_, hipStream_t s) {
  if (cplx_) hipLaunchKernelGGL(k_submatrix_coef<cplx>, dim3(1, n_inst), dim3(256), 0, s, insts);
  else hipLaunchKernelGGL(k_submatrix_coef<double>, dim3(1, n_inst), dim3(256), 0, s, insts);
  return hipGetLastError();
}

hipError_t launch_submatrix_rows(const InstDev* insts, int n_inst, int Nmax, bool cplx_, hipStream_t s) {
  dim3 grid((Nmax + 63) / 64, n_inst);
  if (cplx_) hipLaunchKernelGGL(k_submatrix_rows<cplx>, grid, dim3(256), 0, s, insts);
  else hipLaunchKernelGGL(k_submatrix_rows<double>, grid, dim3(256), 0, s, insts);
  return hipGetLastError();
}
