// Learned multi-site moves and the proposal network behind them.
//
// The paper proposes single-site flips.  A learned move changes an ordered
// set S of m sites of the current slice at once; it stays exact because
//   * its weight ratio is the block form of eqs. DRatio and rRatioLocal,
//       R_S = e^{2 lambda sum_S x} |det(1_m + Delta_S (1 - G)_{SS})|^2,
//     evaluated here as the product of the sequential single-site ratios of
//     the m sites (the pivots of that determinant), and
//   * it is accepted with the Metropolis-Hastings rule (eq. DetailBalance for
//     an asymmetric proposal), min(1, R_S q(S|X') / q(S|X)).
// On acceptance the m rank-1 terms of the block Sherman-Morrison update (the
// m-site form of eq. GupdateLocal) are appended to the delayed-update buffers
// X, Y through the same recursion as the single-site windows (eq. DelayRgenk).
//
// q is the Plackett-Luce law of the weights w_i = sigmoid(y_i) of the network
// outputs y_i of the slice, sampled with Gumbel-top-m on log w_i.  Trained
// against the Barker acceptance Rt/(1+Rt) of a single flip, w approximates
// the locally balanced (Barker) informed proposal, whose acceptance tends to
// one as the neighbourhood grows.
// Uniforms: Philox4x32-10, key (seed lo, seed hi); counter (site, slice,
// sweep, 4 + 4 move + pass) for the Gumbel noise of a site, (0xffffffff,
// slice, sweep, 4 + 4 move + pass) for the acceptance.  Gumbel uniforms are
// (floor(k/2) + 1/2) 2^-52 for the 53-bit k of the site uniforms.
//
// The network: three periodic 3x3x3 convolutions over (slice, n2, n1) on the
// cell grid, channels (x_A, x_B) -> 32 -> 32 -> (z_A, z_B), tanh after the
// first two.  Activations are BF16, channels-last, with 16 or 32 channels
// (the 2-channel ends padded with zeros); every convolution is an implicit
// GEMM on the BF16 matrix cores (16x16x16, FP32 accumulation).  Training is
// mean binary cross-entropy of sigmoid(y) against the recorded single-flip
// Barker acceptances, with hand-written backward kernels and Adam on FP32
// master weights.
#include "common.hpp"
#include "kernels.hpp"
#include "philox.hpp"

namespace {

typedef __bf16 bf16;
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma_bf16(bf4 a, bf4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// v in [-n, 2n) -> v mod n
__device__ __forceinline__ int wrapi(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// ---- convolution as an implicit GEMM ---------------------------------------------------
// One wave computes 16 output voxels x all COP channels: D[co][voxel] =
// sum_{tap, ci} W[tap][co][ci] in[nbr(voxel, tap)][ci], with the weights as
// the A operand (row co, 4 consecutive ci per lane) and the activations as the
// B operand (column voxel, the same 4 ci), so that a lane ends up holding four
// consecutive output channels of one voxel.
template <int CIP, int COP, int ACT, bool OUTF>
__global__ void __launch_bounds__(256) k_conv(const bf16* __restrict__ in, void* __restrict__ outv,
                                               const bf16* __restrict__ W, const float* __restrict__ bias,
                                               ConvGeom g) {
  const int item = blockIdx.y;
  const int L = g.Ls ? g.Ls[item] : g.Lu;
  const int Nc = L * L;
  const int nvox = g.T_out * Nc;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int v0 = (blockIdx.x * 4 + wave) * 16;
  if (v0 >= nvox) return;
  const int lr = lane & 15, lg = lane >> 4;
  const int v = v0 + lr;
  const bool ok = v < nvox;
  const int vv = ok ? v : v0;
  const int t = vv / Nc, rem = vv - t * Nc, n2 = rem / L, n1 = rem - n2 * L;
  const bf16* inb = in + (size_t)item * g.in_stride;
  f4 acc[COP / 16];
#pragma unroll
  for (int ct = 0; ct < COP / 16; ++ct) acc[ct] = f4{0.f, 0.f, 0.f, 0.f};
  const bf4 zero4 = {(bf16)0.f, (bf16)0.f, (bf16)0.f, (bf16)0.f};
#pragma unroll 1
  for (int tap = 0; tap < 27; ++tap) {
    const int dt = tap / 9 - 1, d2 = (tap / 3) % 3 - 1, d1 = tap % 3 - 1;
    const int traw = t + g.toff + dt;
    const bool tin = !g.tzero || (traw >= 0 && traw < g.T_in);
    const int ts = tin ? wrapi(traw, g.T_in) : 0;
    const int s2 = wrapi(n2 + d2, L), s1 = wrapi(n1 + d1, L);
    const bf16* src = inb + (size_t)(s1 + L * (s2 + L * ts)) * CIP + 4 * lg;
    const bf16* wt = W + (size_t)(tap * COP + lr) * CIP + 4 * lg;
#pragma unroll
    for (int cc = 0; cc < CIP / 16; ++cc) {
      bf4 b = (ok && tin) ? *reinterpret_cast<const bf4*>(src + cc * 16) : zero4;
#pragma unroll
      for (int ct = 0; ct < COP / 16; ++ct) {
        bf4 a = *reinterpret_cast<const bf4*>(wt + (size_t)ct * 16 * CIP + cc * 16);
        acc[ct] = mfma_bf16(a, b, acc[ct]);
      }
    }
  }
  if (!ok) return;
  const size_t ob = (size_t)item * g.out_stride + (size_t)v * COP;
#pragma unroll
  for (int ct = 0; ct < COP / 16; ++ct) {
    float r4[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int co = ct * 16 + 4 * lg + r;
      float val = acc[ct][r] + (bias ? bias[co] : 0.f);
      if (ACT) val = tanhf(val);
      r4[r] = val;
    }
    const int c0 = ct * 16 + 4 * lg;
    if constexpr (OUTF) {
      *reinterpret_cast<f4*>(reinterpret_cast<float*>(outv) + ob + c0) = f4{r4[0], r4[1], r4[2], r4[3]};
    } else {
      bf4 o = {(bf16)r4[0], (bf16)r4[1], (bf16)r4[2], (bf16)r4[3]};
      *reinterpret_cast<bf4*>(reinterpret_cast<bf16*>(outv) + ob + c0) = o;
    }
  }
}

// ---- weight gradient ------------------------------------------------------------------
// dW[tap][co][ci] = sum_voxel dout[voxel][co] in[nbr(voxel, tap)][ci] over a
// chunk of vch output voxels per workgroup (A operand: dout, 4 consecutive
// voxels per lane; B operand: the shifted input).  Wave w owns taps w, w+4,
// ...; partial sums per chunk are reduced by k_wgrad_reduce (deterministic).
constexpr int WG_TPW = 7;
template <int CIP, int COP>
__global__ void __launch_bounds__(256) k_wgrad(const bf16* __restrict__ in, const bf16* __restrict__ dout,
                                                float* __restrict__ part, float* __restrict__ partb,
                                                ConvGeom g, int vch) {
  const int item = blockIdx.y;
  const int L = g.Ls ? g.Ls[item] : g.Lu;
  const int Nc = L * L;
  const int nvox = g.T_out * Nc;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int lr = lane & 15, lg = lane >> 4;
  const int vb0 = blockIdx.x * vch;
  const int vend = min(vb0 + vch, nvox);
  const size_t chunk = (size_t)item * gridDim.x + blockIdx.x;
  const bf16* inb = in + (size_t)item * g.in_stride;
  const bf16* dob = dout + (size_t)item * g.out_stride;
  f4 acc[WG_TPW][COP / 16][CIP / 16];
#pragma unroll
  for (int q = 0; q < WG_TPW; ++q)
#pragma unroll
    for (int ct = 0; ct < COP / 16; ++ct)
#pragma unroll
      for (int cc = 0; cc < CIP / 16; ++cc) acc[q][ct][cc] = f4{0.f, 0.f, 0.f, 0.f};
  float bs[COP / 16];
#pragma unroll
  for (int ct = 0; ct < COP / 16; ++ct) bs[ct] = 0.f;
  const bf16 z0 = (bf16)0.f;
  for (int vb = vb0; vb < vend; vb += 16) {
    int tj[4], n2j[4], n1j[4];
    bool okj[4];
    int vxj[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int vx = vb + 4 * lg + j;
      okj[j] = vx < vend;
      vxj[j] = okj[j] ? vx : vb;
      tj[j] = vxj[j] / Nc;
      int rem = vxj[j] - tj[j] * Nc;
      n2j[j] = rem / L;
      n1j[j] = rem - n2j[j] * L;
    }
    bf4 a[COP / 16];
#pragma unroll
    for (int ct = 0; ct < COP / 16; ++ct)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        bf16 x = okj[j] ? dob[(size_t)vxj[j] * COP + ct * 16 + lr] : z0;
        a[ct][j] = x;
        bs[ct] += (float)x;
      }
#pragma unroll
    for (int q = 0; q < WG_TPW; ++q) {
      const int tap = wave + 4 * q;
      if (tap < 27) {
        const int dt = tap / 9 - 1, d2 = (tap / 3) % 3 - 1, d1 = tap % 3 - 1;
        size_t src[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
          src[j] = (size_t)(wrapi(n1j[j] + d1, L) + L * (wrapi(n2j[j] + d2, L) + L * wrapi(tj[j] + g.toff + dt, g.T_in))) *
                       CIP + lr;
#pragma unroll
        for (int cc = 0; cc < CIP / 16; ++cc) {
          bf4 b;
#pragma unroll
          for (int j = 0; j < 4; ++j) b[j] = okj[j] ? inb[src[j] + cc * 16] : z0;
#pragma unroll
          for (int ct = 0; ct < COP / 16; ++ct) acc[q][ct][cc] = mfma_bf16(a[ct], b, acc[q][ct][cc]);
        }
      }
    }
  }
  float* pw = part + chunk * 27 * COP * CIP;
#pragma unroll
  for (int q = 0; q < WG_TPW; ++q) {
    const int tap = wave + 4 * q;
    if (tap < 27) {
#pragma unroll
      for (int ct = 0; ct < COP / 16; ++ct)
#pragma unroll
        for (int cc = 0; cc < CIP / 16; ++cc)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            pw[((size_t)tap * COP + ct * 16 + 4 * lg + r) * CIP + cc * 16 + lr] = acc[q][ct][cc][r];
    }
  }
  if (wave == 0) {
#pragma unroll
    for (int ct = 0; ct < COP / 16; ++ct) {
      float x = bs[ct];
      x += __shfl_xor(x, 16);
      x += __shfl_xor(x, 32);
      if (lg == 0) partb[chunk * COP + ct * 16 + lr] = x;
    }
  }
}

__global__ void k_wgrad_reduce(const float* __restrict__ part, const float* __restrict__ partb, int nchunks,
                               int COP, int CIP, int CO, int CI, float* __restrict__ gw, float* __restrict__ gb) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int nw = 27 * CO * CI;
  if (e < nw) {
    const int tap = e / (CO * CI), rem = e - tap * CO * CI, co = rem / CI, ci = rem - co * CI;
    const size_t off = ((size_t)tap * COP + co) * CIP + ci;
    const size_t stride = (size_t)27 * COP * CIP;
    float s = 0.f;
    for (int c = 0; c < nchunks; ++c) s += part[(size_t)c * stride + off];
    gw[e] = s;
  } else if (e < nw + CO) {
    const int co = e - nw;
    float s = 0.f;
    for (int c = 0; c < nchunks; ++c) s += partb[(size_t)c * COP + co];
    gb[co] = s;
  }
}

// ---- weights, inputs, loss ---------------------------------------------------------------
__global__ void k_net_prep(const float* __restrict__ P, NetW w) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  bf16* w1f = reinterpret_cast<bf16*>(w.w1f);
  bf16* w2f = reinterpret_cast<bf16*>(w.w2f);
  bf16* w3f = reinterpret_cast<bf16*>(w.w3f);
  bf16* w2b = reinterpret_cast<bf16*>(w.w2b);
  bf16* w3b = reinterpret_cast<bf16*>(w.w3b);
  if (e < 27 * 32 * 16) {
    // w1f [tap][co 32][ci 16]; w3f [tap][co 16][ci 32]; w3b [tap'][a 32][b 16] = W3[26 - tap'][b][a]
    int tap = e / 512, r = e % 512;
    int co = r / 16, ci = r % 16;
    w1f[e] = (bf16)(ci < 2 ? P[NET_OFF_W1 + (tap * 32 + co) * 2 + ci] : 0.f);
    int co3 = r / 32, ci3 = r % 32;
    w3f[e] = (bf16)(co3 < 2 ? P[NET_OFF_W3 + (tap * 2 + co3) * 32 + ci3] : 0.f);
    int a = r / 16, b = r % 16;
    w3b[e] = (bf16)(b < 2 ? P[NET_OFF_W3 + ((26 - tap) * 2 + b) * 32 + a] : 0.f);
  }
  if (e < 27 * 32 * 32) {
    // w2f = W2; w2b [tap'][a][b] = W2[26 - tap'][b][a]
    int tap = e / 1024, r = e % 1024, a = r / 32, b = r % 32;
    w2f[e] = (bf16)P[NET_OFF_W2 + e];
    w2b[e] = (bf16)P[NET_OFF_W2 + ((26 - tap) * 32 + b) * 32 + a];
  }
  if (e < 32) {
    w.b1[e] = P[NET_OFF_B1 + e];
    w.b2[e] = P[NET_OFF_B2 + e];
    if (e < 16) w.b3[e] = e < 2 ? P[NET_OFF_B3 + e] : 0.f;
  }
}

// fields (n_samples x M x N int8) -> channels-last input of the batch
__global__ void k_net_input(const int8_t* __restrict__ fields, int N, int Nc, int M, BatchIdx idx,
                            bf16* __restrict__ a0) {
  const int b = blockIdx.y;
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= M * Nc) return;
  const int t = v / Nc, c = v - t * Nc;
  const int8_t* x = fields + (size_t)idx.idx[b] * M * N + (size_t)t * N;
  bf16* o = a0 + ((size_t)b * M * Nc + v) * 16;
  const bf16 z0 = (bf16)0.f;
  bf4 lo = {(bf16)(float)x[c], (bf16)(float)x[Nc + c], z0, z0};
  bf4 zz = {z0, z0, z0, z0};
  reinterpret_cast<bf4*>(o)[0] = lo;
  reinterpret_cast<bf4*>(o)[1] = zz;
  reinterpret_cast<bf4*>(o)[2] = zz;
  reinterpret_cast<bf4*>(o)[3] = zz;
}

// 7-slice windows -> channels-last input of the batch (per-item L)
__global__ void k_net_input_window(const int8_t* __restrict__ wins, long long win_stride, int row_stride,
                                   BatchIdx idx, const int* __restrict__ Ls, int nc_max, bf16* __restrict__ a0) {
  const int b = blockIdx.y;
  const int L = Ls[b], Nc = L * L;
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= 7 * Nc) return;
  const int a = v / Nc, c = v - a * Nc;
  const int8_t* x = wins + (size_t)idx.idx[b] * win_stride + (size_t)a * row_stride;
  bf16* o = a0 + ((size_t)b * 7 * nc_max + v) * 16;
  const bf16 z0 = (bf16)0.f;
  bf4 lo = {(bf16)(float)x[c], (bf16)(float)x[Nc + c], z0, z0};
  bf4 zz = {z0, z0, z0, z0};
  reinterpret_cast<bf4*>(o)[0] = lo;
  reinterpret_cast<bf4*>(o)[1] = zz;
  reinterpret_cast<bf4*>(o)[2] = zz;
  reinterpret_cast<bf4*>(o)[3] = zz;
}

__device__ __forceinline__ float block_sum_f(float x, float* sh) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = x;
  __syncthreads();
  float s = 0.f;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
  return s;
}

// mean BCE and dz = (sigmoid(z) - a) / count, one thread per voxel (both sites)
__global__ void __launch_bounds__(256) k_net_loss(const float* __restrict__ z, const float* __restrict__ targets,
                                                  BatchIdx idx, int N, int Nc, int M, bf16* __restrict__ dz,
                                                  float* __restrict__ lossp) {
  __shared__ float sh[4];
  const int b = blockIdx.y;
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  float l = 0.f;
  if (v < M * Nc) {
    const int t = v / Nc, c = v - t * Nc;
    const float* zz = z + ((size_t)b * M * Nc + v) * 16;
    const float* tg = targets + (size_t)idx.idx[b] * M * N + (size_t)t * N;
    const float inv = 1.0f / ((float)idx.n * (float)M * (float)N);
    float gsub[2];
#pragma unroll
    for (int sub = 0; sub < 2; ++sub) {
      float zi = zz[sub], a = tg[sub * Nc + c];
      l += fmaxf(zi, 0.f) - a * zi + log1pf(expf(-fabsf(zi)));
      gsub[sub] = (1.0f / (1.0f + expf(-zi)) - a) * inv;
    }
    bf16* o = dz + ((size_t)b * M * Nc + v) * 16;
    const bf16 z0 = (bf16)0.f;
    bf4 lo = {(bf16)gsub[0], (bf16)gsub[1], z0, z0};
    bf4 zz4 = {z0, z0, z0, z0};
    reinterpret_cast<bf4*>(o)[0] = lo;
    reinterpret_cast<bf4*>(o)[1] = zz4;
    reinterpret_cast<bf4*>(o)[2] = zz4;
    reinterpret_cast<bf4*>(o)[3] = zz4;
  }
  float s = block_sum_f(l, sh);
  if (threadIdx.x == 0) lossp[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = s;
}

// centre-slice loss of window samples, one thread per cell (both sites)
__global__ void __launch_bounds__(256) k_net_loss_window(const float* __restrict__ z, const float* __restrict__ tgs,
                                                         long long tg_stride, BatchIdx idx, const int* __restrict__ Ls,
                                                         int nc_max, float inv, bf16* __restrict__ dz,
                                                         float* __restrict__ lossp) {
  __shared__ float sh[4];
  const int b = blockIdx.y;
  const int L = Ls[b], Nc = L * L;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  float l = 0.f;
  if (c < Nc) {
    const float* zz = z + ((size_t)b * nc_max + c) * 16;
    const float* tg = tgs + (size_t)idx.idx[b] * tg_stride;
    float gsub[2];
#pragma unroll
    for (int sub = 0; sub < 2; ++sub) {
      float zi = zz[sub], a = tg[sub * Nc + c];
      l += fmaxf(zi, 0.f) - a * zi + log1pf(expf(-fabsf(zi)));
      gsub[sub] = (1.0f / (1.0f + expf(-zi)) - a) * inv;
    }
    bf16* o = dz + ((size_t)b * nc_max + c) * 16;
    const bf16 z0 = (bf16)0.f;
    bf4 lo = {(bf16)gsub[0], (bf16)gsub[1], z0, z0};
    bf4 zz4 = {z0, z0, z0, z0};
    reinterpret_cast<bf4*>(o)[0] = lo;
    reinterpret_cast<bf4*>(o)[1] = zz4;
    reinterpret_cast<bf4*>(o)[2] = zz4;
    reinterpret_cast<bf4*>(o)[3] = zz4;
  }
  float s = block_sum_f(l, sh);
  if (threadIdx.x == 0) lossp[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = s;
}

// Training sample of the current slice (downward pass, l % every == 0).
__global__ void k_collect(const InstDev* __restrict__ insts, int off, int n_total, int8_t* __restrict__ ring_win,
                          float* __restrict__ ring_tg, int ring_cap, int n_max, int every) {
  const int inst = off + blockIdx.y;   // index in the handle
  const InstDev& d = insts[blockIdx.y];
  InstState* st = d.st;
  if (st->idle || st->init_mode) return;
  const int M = d.M, N = d.N;
  if (sched_is_up(st->phase, M)) return;
  const int l = sched_slice(st->phase, M);
  if (l % every) return;
  const int64_t slot = (st->collect_n * n_total + inst) % ring_cap;
  int8_t* w = ring_win + (size_t)slot * 7 * n_max;
  float* tg = ring_tg + (size_t)slot * n_max;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < 8 * N; e += gridDim.x * blockDim.x) {
    if (e < 7 * N) {
      const int a = e / N, i = e - a * N;
      const int row = ((l - 1 - 3 + a) % M + M) % M;
      w[(size_t)a * n_max + i] = d.fields[(size_t)row * N + i];
    } else {
      const int i = e - 7 * N;
      tg[i] = d.targets[(size_t)(l - 1) * N + i];
    }
  }
}

__global__ void k_collect_bump(const InstDev* __restrict__ insts, int n, int every) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const InstDev& d = insts[i];
  InstState* st = d.st;
  if (st->idle || st->init_mode || sched_is_up(st->phase, d.M)) return;
  if (sched_slice(st->phase, d.M) % every) return;
  st->collect_n += 1;
}

__global__ void __launch_bounds__(256) k_sum_scaled(const float* __restrict__ x, int n, float scale,
                                                    float* __restrict__ out) {
  __shared__ float sh[4];
  float s = 0.f;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += x[i];
  s = block_sum_f(s, sh);
  if (threadIdx.x == 0) out[0] = s * scale;
}

__global__ void k_net_logits_out(const float* __restrict__ z, BatchIdx idx, int N, int Nc, int M,
                                 float* __restrict__ out) {
  const int b = blockIdx.y;
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= M * Nc) return;
  const int t = v / Nc, c = v - t * Nc;
  const float* zz = z + ((size_t)b * M * Nc + v) * 16;
  float* o = out + (size_t)b * M * N + (size_t)t * N;
  o[c] = zz[0];
  o[Nc + c] = zz[1];
}

__global__ void k_tanh_back(bf16* __restrict__ dh, const bf16* __restrict__ h, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float y = (float)h[i];
  dh[i] = (bf16)((float)dh[i] * (1.0f - y * y));
}

__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  float gi = g[i];
  float mi = b1 * m[i] + (1.f - b1) * gi;
  float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---- sampler side ------------------------------------------------------------------------
// Input window of 7 slices l-3 .. l+3 (mod M) around the current slice; with
// flip, the sites of the move in flight are reversed wherever slice l appears.
__global__ void k_learn_window(const InstDev* __restrict__ insts, int flip) {
  const InstDev& d = insts[blockIdx.y];
  const InstState& st = *d.st;
  if (st.idle || st.init_mode) return;
  const int Nc = d.Nc, N = d.N, M = d.M;
  const int l = sched_slice(st.phase, M);
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 7 * Nc) return;
  const int a = e / Nc, c = e - a * Nc;
  int row = ((l - 1 - 3 + a) % M + M) % M;
  float xa = d.fields[(size_t)row * N + c], xb = d.fields[(size_t)row * N + Nc + c];
  if (flip && row == l - 1) {
    const LearnState& ls = *d.learn;
    for (int k = 0; k < ls.m; ++k) {
      if (ls.S[k] == c) xa = -xa;
      if (ls.S[k] == Nc + c) xb = -xb;
    }
  }
  bf16* o = reinterpret_cast<bf16*>(d.lwin[0]) + (size_t)e * 16;
  const bf16 z0 = (bf16)0.f;
  bf4 lo = {(bf16)xa, (bf16)xb, z0, z0};
  bf4 zz = {z0, z0, z0, z0};
  reinterpret_cast<bf4*>(o)[0] = lo;
  reinterpret_cast<bf4*>(o)[1] = zz;
  reinterpret_cast<bf4*>(o)[2] = zz;
  reinterpret_cast<bf4*>(o)[3] = zz;
}

// Proposal weight of site i: log sigmoid(y_i) of the network output y_i
// (the network predicts log Rt; sigmoid(log Rt) = Rt / (1 + Rt) is the
// Barker-balanced weight of flipping the site).
__device__ __forceinline__ double site_logit(const float* z, int i, int Nc) {
  const double y = i < Nc ? (double)z[(size_t)i * 16] : (double)z[(size_t)(i - Nc) * 16 + 1];
  return y >= 0.0 ? -log1p(exp(-y)) : y - log1p(exp(y));
}

constexpr int LP_THREADS = 256;
constexpr int LP_PER = 16;   // sites per thread: N <= 2 * 45^2 = 4050 <= 16 * 256

__device__ double block_max_d(double x, double* sh) {
  for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = x;
  __syncthreads();
  double r = sh[0];
  for (int w = 1; w < LP_THREADS / 64; ++w) r = fmax(r, sh[w]);
  __syncthreads();
  return r;
}

__device__ double block_sum_d(double x, double* sh) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = x;
  __syncthreads();
  double r = 0.0;
  for (int w = 0; w < LP_THREADS / 64; ++w) r += sh[w];
  __syncthreads();
  return r;
}

// (key, index) maximum; ties go to the lower index
__device__ void block_argmax(double& key, int& idx, double* shk, int* shi) {
  for (int o = 32; o > 0; o >>= 1) {
    double k2 = __shfl_xor(key, o);
    int i2 = __shfl_xor(idx, o);
    if (k2 > key || (k2 == key && i2 < idx)) { key = k2; idx = i2; }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) { shk[wave] = key; shi[wave] = idx; }
  __syncthreads();
  key = shk[0];
  idx = shi[0];
  for (int w = 1; w < LP_THREADS / 64; ++w)
    if (shk[w] > key || (shk[w] == key && shi[w] < idx)) { key = shk[w]; idx = shi[w]; }
  __syncthreads();
}

// log q(S | X) = sum_j (z_{s_j} - log sum_{i not in s_<j} e^{z_i}), by thread 0
__device__ double log_q_of(const float* z, const int* S, int m, int Nc, double zmax, double tot) {
  double lq = 0.0;
  for (int k = 0; k < m; ++k) {
    double zs = site_logit(z, S[k], Nc) - zmax;
    lq += zs - log(tot);
    tot -= exp(zs);
  }
  return lq;
}

__device__ __forceinline__ void put_s(double* p, double v) { p[0] = v; p[1] = 0.0; }
__device__ __forceinline__ void put_s(double* p, cplx v) { p[0] = v.x; p[1] = v.y; }
template <typename S> __device__ __forceinline__ S get_s(const double* p);
template <> __device__ __forceinline__ double get_s<double>(const double* p) { return p[0]; }
template <> __device__ __forceinline__ cplx get_s<cplx>(const double* p) { return cmake(p[0], p[1]); }

template <typename S>
__global__ void __launch_bounds__(LP_THREADS) k_learn_propose(const InstDev* __restrict__ insts, int move, int m) {
  const InstDev& d = insts[blockIdx.y];
  const InstState* st = d.st;
  if (st->idle || st->init_mode) return;
  const int N = d.N, Nc = d.Nc, M = d.M;
  const int l = sched_slice(st->phase, M);
  const int pass = sched_is_up(st->phase, M) ? 0 : 1;
  const int tid = threadIdx.x;
  const uint32_t sweep = (uint32_t)st->sweep;
  const uint32_t c3 = 4u + 4u * (uint32_t)move + (uint32_t)pass;
  const uint32_t k0 = (uint32_t)(d.seed & 0xffffffffu), k1 = (uint32_t)(d.seed >> 32);
  const float* z = d.zcur;
  __shared__ double shd[LP_THREADS / 64];
  __shared__ int shi[LP_THREADS / 64];
  __shared__ int Ssh[LEARN_MMAX];
  __shared__ int bad_sh;
  __shared__ S Cs[LEARN_MMAX][LEARN_MMAX];
  if (tid == 0) bad_sh = 0;
  double key[LP_PER];
  double zmx = -INFINITY;
#pragma unroll
  for (int q = 0; q < LP_PER; ++q) {
    const int i = tid + LP_THREADS * q;
    key[q] = -INFINITY;
    if (i < N) {
      const double zi = site_logit(z, i, Nc);
      philox_out o = philox4x32_10((uint32_t)i, (uint32_t)l, sweep, c3, k0, k1);
      const uint64_t kk = ((uint64_t)o.w[0] << 21) + (uint64_t)(o.w[1] >> 11);
      const double u = ((double)(kk >> 1) + 0.5) * (1.0 / 4503599627370496.0);
      key[q] = zi - log(-log(u));
      zmx = fmax(zmx, zi);
    }
  }
  const double zmax = block_max_d(zmx, shd);
  double se = 0.0;
#pragma unroll
  for (int q = 0; q < LP_PER; ++q) {
    const int i = tid + LP_THREADS * q;
    if (i < N) se += exp(site_logit(z, i, Nc) - zmax);
  }
  const double tot = block_sum_d(se, shd);
  for (int k = 0; k < m; ++k) {
    double best = -INFINITY;
    int bi = 0x7fffffff;
#pragma unroll
    for (int q = 0; q < LP_PER; ++q) {
      const int i = tid + LP_THREADS * q;
      if (i < N && (key[q] > best || (key[q] == best && i < bi))) { best = key[q]; bi = i; }
    }
    block_argmax(best, bi, shd, shi);
    // no finite key left (non-finite logits): keep the indices in range and
    // reject the move below
    if (bi < 0 || bi >= N) { bi = k; best = NAN; }
#pragma unroll
    for (int q = 0; q < LP_PER; ++q)
      if (tid + LP_THREADS * q == bi) key[q] = -INFINITY;
    if (tid == 0) { Ssh[k] = bi; if (!(best == best)) bad_sh = 1; }
  }
  __syncthreads();
  // the current G restricted to S: G0[S, S] - X[S, :fill] Y[:fill, S]
  const S* G = matp<S>(d, MAT_G);
  const S* X = matp<S>(d, MAT_X);
  const S* Y = matp<S>(d, MAT_Y);
  const int fill = st->fill;
  if (tid < m * m) {
    const int a = tid / m, b = tid - a * m;
    const int ia = Ssh[a], ib = Ssh[b];
    S v = G[ia + (size_t)ib * N];
    for (int f = 0; f < fill; ++f) v = v - X[ia + (size_t)f * N] * Y[(size_t)f * N + ib];
    Cs[a][b] = v;
  }
  __syncthreads();
  if (tid == 0) {
    LearnState* ls = d.learn;
    const double lam = d.lam;
    double R = 1.0;
    double pre = 1.0, pim = 0.0;   // phase of prod_k r_k
    int valid = 1;
    for (int k = 0; k < m; ++k) ls->S[k] = Ssh[k];
    for (int k = 0; k < m; ++k) {
      const double x = (double)d.fields[(size_t)(l - 1) * N + Ssh[k]];
      const double delta = exp(-2.0 * lam * x) - 1.0;
      const S dl = ST<S>::from_re(delta);
      const S r = ST<S>::one() + dl * (ST<S>::one() - Cs[k][k]);
      const double ar = absq(r);
      if (!(ar > 0.0) || !(ar < 1e300)) valid = 0;
      R *= exp(2.0 * lam * x) * ar;
      if (ar > 0.0) {
        const double sa = sqrt(ar), qr = real_part(r) / sa, qi = imag_part(r) / sa;
        const double a = pre, b = pim;
        pre = a * qr - b * qi;
        pim = a * qi + b * qr;
      }
      const S cf = valid ? cdiv(dl, r) : ST<S>::zero();
      put_s(ls->c[k], cf);
      S xv[LEARN_MMAX], yv[LEARN_MMAX];
      for (int a = 0; a < LEARN_MMAX; ++a) {
        xv[a] = (a > k && a < m) ? Cs[a][k] * cf : ST<S>::zero();
        yv[a] = (a > k && a < m) ? -Cs[k][a] : ST<S>::zero();
        put_s(ls->xw[k][a], xv[a]);
        put_s(ls->yw[k][a], yv[a]);
      }
      for (int a = k + 1; a < m; ++a)
        for (int b = k + 1; b < m; ++b) Cs[a][b] = Cs[a][b] - xv[a] * yv[b];
    }
    ls->m = m;
    ls->ph[0] = pre;
    ls->ph[1] = pim;
    ls->valid = valid && !bad_sh && (R == R) && R < 1e300;
    ls->R = R;
    ls->logq = log_q_of(z, Ssh, m, Nc, zmax, tot);
  }
}

template <typename S>
__global__ void __launch_bounds__(LP_THREADS) k_learn_decide(const InstDev* __restrict__ insts, int move) {
  const InstDev& d = insts[blockIdx.y];
  InstState* st = d.st;
  if (st->idle || st->init_mode) return;
  const int N = d.N, Nc = d.Nc, M = d.M;
  const int l = sched_slice(st->phase, M);
  const int pass = sched_is_up(st->phase, M) ? 0 : 1;
  const int tid = threadIdx.x;
  const LearnState* ls = d.learn;
  const float* zp = d.zprop;
  __shared__ double shd[LP_THREADS / 64];
  __shared__ int acc_sh;
  double zmx = -INFINITY;
  for (int i = tid; i < N; i += LP_THREADS) zmx = fmax(zmx, site_logit(zp, i, Nc));
  const double zmax = block_max_d(zmx, shd);
  double se = 0.0;
  for (int i = tid; i < N; i += LP_THREADS) se += exp(site_logit(zp, i, Nc) - zmax);
  const double tot = block_sum_d(se, shd);
  if (tid == 0) {
    const int m = ls->m;
    const double lq2 = log_q_of(zp, ls->S, m, Nc, zmax, tot);
    const double prob = ls->valid ? ls->R * exp(lq2 - ls->logq) : 0.0;
    const uint32_t c3 = 4u + 4u * (uint32_t)move + (uint32_t)pass;
    philox_out o = philox4x32_10(0xffffffffu, (uint32_t)l, (uint32_t)st->sweep, c3,
                                 (uint32_t)(d.seed & 0xffffffffu), (uint32_t)(d.seed >> 32));
    const double u = philox_u53(o.w[0], o.w[1]);
    const int acc = u < prob;
    st->learn_props += 1;
    if (acc) {
      S* wc = reinterpret_cast<S*>(d.wcoef);
      st->learn_acc += 1;
      for (int k = 0; k < m; ++k) {
        const int s = ls->S[k];
        d.acc_site[k] = k;
        d.acc_gsite[k] = s;
        int8_t* f = d.fields + (size_t)(l - 1) * N + s;
        *f = (int8_t)(-*f);
        wc[k] = get_s<S>(ls->c[k]);
        for (int a = 0; a < m; ++a) {
          wc[DQMC_WC_X + k * DQMC_WMAX + a] = get_s<S>(ls->xw[k][a]);
          wc[DQMC_WC_Y + k * DQMC_WMAX + a] = get_s<S>(ls->yw[k][a]);
        }
      }
      st->m_w = m;
      st->wstart = 0;
      const double a = st->ph_re, b = st->ph_im;
      st->ph_re = a * ls->ph[0] - b * ls->ph[1];
      st->ph_im = a * ls->ph[1] + b * ls->ph[0];
    } else {
      st->m_w = 0;
    }
    acc_sh = acc;
  }
  __syncthreads();
  if (acc_sh) {
    for (int e = tid; e < Nc; e += LP_THREADS) {
      d.zcur[(size_t)e * 16] = zp[(size_t)e * 16];
      d.zcur[(size_t)e * 16 + 1] = zp[(size_t)e * 16 + 1];
    }
  }
}

template <int CIP, int COP, int ACT, bool OUTF>
void conv_launch(const void* in, void* out, const void* W, const float* bias, ConvGeom g, int n_items, int max_nc,
                 hipStream_t s) {
  const int nvox = g.T_out * max_nc;
  dim3 grid((nvox + 63) / 64, n_items);
  hipLaunchKernelGGL((k_conv<CIP, COP, ACT, OUTF>), grid, dim3(256), 0, s, reinterpret_cast<const bf16*>(in), out,
                     reinterpret_cast<const bf16*>(W), bias, g);
}

template <int CIP, int COP>
void wgrad_launch(const void* in, const void* dout, float* part, float* partb, ConvGeom g, int n_items, int max_nc,
                  int vch, hipStream_t s) {
  dim3 grid(wgrad_chunks(g.T_out, max_nc, vch), n_items);
  hipLaunchKernelGGL((k_wgrad<CIP, COP>), grid, dim3(256), 0, s, reinterpret_cast<const bf16*>(in),
                     reinterpret_cast<const bf16*>(dout), part, partb, g, vch);
}

}  // namespace

hipError_t launch_net_prep(const float* master, NetW w, hipStream_t s) {
  hipLaunchKernelGGL(k_net_prep, dim3((27 * 32 * 32 + 255) / 256), dim3(256), 0, s, master, w);
  return hipGetLastError();
}

hipError_t launch_conv(int kind, const void* in, void* out, NetW w, ConvGeom g, int n_items, int max_nc,
                       hipStream_t s) {
  switch (kind) {
    case CONV_F1: conv_launch<16, 32, 1, false>(in, out, w.w1f, w.b1, g, n_items, max_nc, s); break;
    case CONV_F2: conv_launch<32, 32, 1, false>(in, out, w.w2f, w.b2, g, n_items, max_nc, s); break;
    case CONV_F3: conv_launch<32, 16, 0, true>(in, out, w.w3f, w.b3, g, n_items, max_nc, s); break;
    case CONV_B3: conv_launch<16, 32, 0, false>(in, out, w.w3b, nullptr, g, n_items, max_nc, s); break;
    case CONV_B2: conv_launch<32, 32, 0, false>(in, out, w.w2b, nullptr, g, n_items, max_nc, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int wgrad_chunks(int T_out, int Nc, int vch) { return (T_out * Nc + vch - 1) / vch; }

hipError_t launch_wgrad(int kind, const void* in, const void* dout, float* part, float* partb, ConvGeom g,
                        int n_items, int max_nc, int vch, hipStream_t s) {
  switch (kind) {
    case WGRAD_1: wgrad_launch<16, 32>(in, dout, part, partb, g, n_items, max_nc, vch, s); break;
    case WGRAD_2: wgrad_launch<32, 32>(in, dout, part, partb, g, n_items, max_nc, vch, s); break;
    case WGRAD_3: wgrad_launch<32, 16>(in, dout, part, partb, g, n_items, max_nc, vch, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_wgrad_reduce(int kind, const float* part, const float* partb, int nchunks, float* grad,
                               hipStream_t s) {
  int COP, CIP, CO, CI, ow, ob;
  switch (kind) {
    case WGRAD_1: COP = 32; CIP = 16; CO = 32; CI = 2; ow = NET_OFF_W1; ob = NET_OFF_B1; break;
    case WGRAD_2: COP = 32; CIP = 32; CO = 32; CI = 32; ow = NET_OFF_W2; ob = NET_OFF_B2; break;
    case WGRAD_3: COP = 16; CIP = 32; CO = 2; CI = 32; ow = NET_OFF_W3; ob = NET_OFF_B3; break;
    default: return hipErrorInvalidValue;
  }
  const int n = 27 * CO * CI + CO;
  hipLaunchKernelGGL(k_wgrad_reduce, dim3((n + 255) / 256), dim3(256), 0, s, part, partb, nchunks, COP, CIP, CO, CI,
                     grad + ow, grad + ob);
  return hipGetLastError();
}

hipError_t launch_net_input(const int8_t* fields, int N, int Nc, int M, BatchIdx idx, void* a0, hipStream_t s) {
  dim3 grid((M * Nc + 255) / 256, idx.n);
  hipLaunchKernelGGL(k_net_input, grid, dim3(256), 0, s, fields, N, Nc, M, idx, reinterpret_cast<bf16*>(a0));
  return hipGetLastError();
}

hipError_t launch_net_loss(const float* z, const float* targets, BatchIdx idx, int N, int Nc, int M, void* dz,
                           float* lossp, float* loss_out, hipStream_t s) {
  dim3 grid((M * Nc + 255) / 256, idx.n);
  hipLaunchKernelGGL(k_net_loss, grid, dim3(256), 0, s, z, targets, idx, N, Nc, M, reinterpret_cast<bf16*>(dz),
                     lossp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const float scale = 1.0f / ((float)idx.n * (float)M * (float)N);
  hipLaunchKernelGGL(k_sum_scaled, dim3(1), dim3(256), 0, s, lossp, (int)(grid.x * grid.y), scale, loss_out);
  return hipGetLastError();
}

hipError_t launch_net_logits_out(const float* z, BatchIdx idx, int N, int Nc, int M, float* out, hipStream_t s) {
  dim3 grid((M * Nc + 255) / 256, idx.n);
  hipLaunchKernelGGL(k_net_logits_out, grid, dim3(256), 0, s, z, idx, N, Nc, M, out);
  return hipGetLastError();
}

namespace {
__global__ void k_batch_L(BatchIdx idx, int* __restrict__ dLs) {
  const int b = threadIdx.x;
  if (b < idx.n) dLs[b] = idx.L[b];
}
}  // namespace

hipError_t launch_batch_L(const BatchIdx& idx, int* dLs, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_L, dim3(1), dim3(NET_MAXBATCH), 0, s, idx, dLs);
  return hipGetLastError();
}

hipError_t launch_net_input_window(const int8_t* wins, long long win_stride, int row_stride, BatchIdx idx,
                                   const int* Ls, int nc_max, void* a0, hipStream_t s) {
  dim3 grid((7 * nc_max + 255) / 256, idx.n);
  hipLaunchKernelGGL(k_net_input_window, grid, dim3(256), 0, s, wins, win_stride, row_stride, idx, Ls, nc_max,
                     reinterpret_cast<bf16*>(a0));
  return hipGetLastError();
}

hipError_t launch_net_loss_window(const float* z, const float* tgs, long long tg_stride, BatchIdx idx,
                                  const int* Ls, int nc_max, float inv_count, void* dz, float* lossp,
                                  float* loss_out, hipStream_t s) {
  dim3 grid((nc_max + 255) / 256, idx.n);
  hipLaunchKernelGGL(k_net_loss_window, grid, dim3(256), 0, s, z, tgs, tg_stride, idx, Ls, nc_max, inv_count,
                     reinterpret_cast<bf16*>(dz), lossp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_scaled, dim3(1), dim3(256), 0, s, lossp, (int)(grid.x * grid.y), inv_count, loss_out);
  return hipGetLastError();
}

hipError_t launch_collect(const InstDev* insts, int n_inst, int off, int n_total, int8_t* ring_win, float* ring_tg,
                          int ring_cap, int n_max, int every, hipStream_t s) {
  dim3 grid((8 * n_max + 255) / 256, n_inst);
  hipLaunchKernelGGL(k_collect, grid, dim3(256), 0, s, insts, off, n_total, ring_win, ring_tg, ring_cap, n_max,
                     every);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_collect_bump, dim3((n_inst + 63) / 64), dim3(64), 0, s, insts, n_inst, every);
  return hipGetLastError();
}

hipError_t launch_tanh_back(void* dh, const void* h, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_tanh_back, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, reinterpret_cast<bf16*>(dh),
                     reinterpret_cast<const bf16*>(h), n);
  return hipGetLastError();
}

hipError_t launch_adam(float* master, const float* g, float* m, float* v, int n, float lr, int step,
                       hipStream_t s) {
  const float c1 = 1.0f - powf(0.9f, (float)step), c2 = 1.0f - powf(0.999f, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, master, g, m, v, n, lr, c1, c2);
  return hipGetLastError();
}

hipError_t launch_learn_window(const InstDev* insts, int n_inst, int nc_max, int flip, hipStream_t s) {
  dim3 grid((7 * nc_max + 255) / 256, n_inst);
  hipLaunchKernelGGL(k_learn_window, grid, dim3(256), 0, s, insts, flip);
  return hipGetLastError();
}

hipError_t launch_learn_propose(const InstDev* insts, int n_inst, bool cplx_, int move, int m, hipStream_t s) {
  if (cplx_) hipLaunchKernelGGL(k_learn_propose<cplx>, dim3(1, n_inst), dim3(LP_THREADS), 0, s, insts, move, m);
  else hipLaunchKernelGGL(k_learn_propose<double>, dim3(1, n_inst), dim3(LP_THREADS), 0, s, insts, move, m);
  return hipGetLastError();
}

hipError_t launch_learn_decide(const InstDev* insts, int n_inst, bool cplx_, int move, hipStream_t s) {
  if (cplx_) hipLaunchKernelGGL(k_learn_decide<cplx>, dim3(1, n_inst), dim3(LP_THREADS), 0, s, insts, move);
  else hipLaunchKernelGGL(k_learn_decide<double>, dim3(1, n_inst), dim3(LP_THREADS), 0, s, insts, move);
  return hipGetLastError();
}
