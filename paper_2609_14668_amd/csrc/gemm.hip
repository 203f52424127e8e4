// Batched FP64 GEMM on the matrix cores (v_mfma_f64_16x16x4_f64).
//
// C = alpha op(A) op(B) + beta C per instance, on named per-instance matrices.
// It serves the rank-k flush of the delayed update, G <- G - X Y
// (eq. FinalDelay), and the dense products of the QR stabilisation.
// Complex128 is done with four real MFMA products per tile (re*re - im*im,
// re*im + im*re) on split real/imaginary LDS planes.
//
// Tiling: 64 x 64 output tile per workgroup of four 64-wide waves, each wave
// a 32 x 32 block of 2 x 2 MFMA tiles; K is staged through LDS 16 at a time.
#include "common.hpp"
#include "kernels.hpp"

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 16, PAD = 2;
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

template <typename S>
__global__ void __launch_bounds__(GEMM_THREADS)
k_gemm(const InstDev* __restrict__ insts, GemmOperand A, GemmOperand B, GemmOperand C,
       GemmDim Md, GemmDim Nd, GemmDim Kd, double alpha, double beta, int flags) {
  constexpr bool CX = ST<S>::is_complex;
  const InstDev& d = insts[blockIdx.y];
  const int Nn = d.N;
  const InstState& st = *d.st;
  if (st.idle) return;
  if ((flags & GF_SKIP_INIT) && st.init_mode) return;
  if ((flags & GF_IF_FULL) && st.fill < d.kflush) return;
  if ((flags & GF_IF_ANY) && st.fill <= 0) return;
  const int M = dimval(Md, Nn);
  const int NC = dimval(Nd, Nn);
  const int K = (flags & GF_K_FILL) ? st.fill : dimval(Kd, Nn);
  if (M <= 0 || NC <= 0) return;
  const int ld = Nn;
  const S* pa = reinterpret_cast<const S*>(mat_ptr(d, A.id)) + offval(A.ra, A.rb, Nn) + offval(A.ca, A.cb, Nn) * ld;
  const S* pb = reinterpret_cast<const S*>(mat_ptr(d, B.id)) + offval(B.ra, B.rb, Nn) + offval(B.ca, B.cb, Nn) * ld;
  S* pc = reinterpret_cast<S*>(mat_ptr(d, C.id)) + offval(C.ra, C.rb, Nn) + offval(C.ca, C.cb, Nn) * ld;
  const bool a_upper = flags & GF_A_UPPER;

  __shared__ double Ar[BK][BM + PAD], Br[BK][BN + PAD];
  __shared__ double Ai[CX ? BK : 1][BM + PAD], Bi[CX ? BK : 1][BN + PAD];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int tm = (M + BM - 1) / BM, tn = (NC + BN - 1) / BN;
  const int ntiles = tm * tn;

  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int m0 = (tile % tm) * BM, n0 = (tile / tm) * BN;
    d4 acc_r[2][2], acc_i[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) { acc_r[i][j] = d4{0, 0, 0, 0}; acc_i[i][j] = d4{0, 0, 0, 0}; }

    for (int k0 = 0; k0 < K; k0 += BK) {
      // ---- stage op(A)[m0:m0+64, k0:k0+16] as [k][i]
      for (int p = 0; p < 4; ++p) {
        int i, kk;
        if (A.op == 0) { i = tid & 63; kk = (tid >> 6) + 4 * p; }
        else { kk = tid & 15; i = (tid >> 4) + 16 * p; }
        int gi = m0 + i, gk = k0 + kk;
        double re = 0.0, im = 0.0;
        if (gi < M && gk < K && !(a_upper && gi > gk)) {
          S v = A.op == 0 ? pa[gi + (size_t)gk * ld] : pa[gk + (size_t)gi * ld];
          split<S>(v, re, im);
          if (A.op == 2) im = -im;
        }
        Ar[kk][i] = re;
        if constexpr (CX) Ai[kk][i] = im;
      }
      // ---- stage op(B)[k0:k0+16, n0:n0+64] as [k][j]
      for (int p = 0; p < 4; ++p) {
        int j, kk;
        if (B.op == 0) { kk = tid & 15; j = (tid >> 4) + 16 * p; }
        else { j = tid & 63; kk = (tid >> 6) + 4 * p; }
        int gj = n0 + j, gk = k0 + kk;
        double re = 0.0, im = 0.0;
        if (gj < NC && gk < K) {
          S v = B.op == 0 ? pb[gk + (size_t)gj * ld] : pb[gj + (size_t)gk * ld];
          split<S>(v, re, im);
          if (B.op == 2) im = -im;
        }
        Br[kk][j] = re;
        if constexpr (CX) Bi[kk][j] = im;
      }
      __syncthreads();
#pragma unroll
      for (int ks = 0; ks < BK / 4; ++ks) {
        const int kr = ks * 4 + (lane >> 4);
        double ar[2], br[2], ai[2], bi[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          ar[t] = Ar[kr][wr + t * 16 + (lane & 15)];
          br[t] = Br[kr][wc + t * 16 + (lane & 15)];
          if constexpr (CX) {
            ai[t] = Ai[kr][wr + t * 16 + (lane & 15)];
            bi[t] = Bi[kr][wc + t * 16 + (lane & 15)];
          }
        }
#pragma unroll
        for (int ti = 0; ti < 2; ++ti)
#pragma unroll
          for (int tj = 0; tj < 2; ++tj) {
            acc_r[ti][tj] = mfma(ar[ti], br[tj], acc_r[ti][tj]);
            if constexpr (CX) {
              acc_r[ti][tj] = mfma(-ai[ti], bi[tj], acc_r[ti][tj]);
              acc_i[ti][tj] = mfma(ar[ti], bi[tj], acc_i[ti][tj]);
              acc_i[ti][tj] = mfma(ai[ti], br[tj], acc_i[ti][tj]);
            }
          }
      }
      __syncthreads();
    }
    // ---- epilogue: lane holds rows lane/16 + 4 r, column lane%16 of each 16x16 tile
    //      (v_mfma_f64_16x16x4f64 output layout, checked on the device)
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int gi = m0 + wr + ti * 16 + (lane >> 4) + 4 * r;
          int gj = n0 + wc + tj * 16 + (lane & 15);
          if (gi < M && gj < NC) {
            S* cp = pc + gi + (size_t)gj * ld;
            if constexpr (CX) {
              cplx v = cmake(alpha * acc_r[ti][tj][r], alpha * acc_i[ti][tj][r]);
              if (beta != 0.0) v = v + beta * (*cp);
              *cp = v;
            } else {
              double v = alpha * acc_r[ti][tj][r];
              if (beta != 0.0) v += beta * (*cp);
              *cp = v;
            }
          }
        }
  }
}

}  // namespace

hipError_t launch_gemm(const InstDev* insts, int n_inst, int Nmax, bool cplx_, GemmOperand A,
                       GemmOperand B, GemmOperand C, GemmDim M, GemmDim Nn, GemmDim K,
                       double alpha, double beta, int flags, hipStream_t s) {
  int Mx = dimval(M, Nmax), Nx = dimval(Nn, Nmax);
  if (Mx <= 0 || Nx <= 0) return hipSuccess;
  int tiles = ((Mx + BM - 1) / BM) * ((Nx + BN - 1) / BN);
  int cap = 4096 / (n_inst > 0 ? n_inst : 1);
  if (cap < 8) cap = 8;
  int gx = tiles < cap ? tiles : cap;
  dim3 grid(gx, n_inst);
  if (cplx_) hipLaunchKernelGGL(k_gemm<cplx>, grid, dim3(GEMM_THREADS), 0, s, insts, A, B, C, M, Nn, K, alpha, beta, flags);
  else hipLaunchKernelGGL(k_gemm<double>, grid, dim3(GEMM_THREADS), 0, s, insts, A, B, C, M, Nn, K, alpha, beta, flags);
  return hipGetLastError();
}
