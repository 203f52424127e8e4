// Delayed-update Metropolis sweep of one time slice (Sec. III B, eqs.
// DetailBalance, DRatio, rRatioLocal, DelayG0, DelayRatio, DelayRgenk,
// FinalDelay).
//
// The chain of accept/reject decisions is sequential: every accepted flip
// changes the diagonal of G seen by later sites.  It is split in windows of up
// to 64 consecutive sites.  The window kernel (one workgroup per instance)
// holds the current G restricted to the window,
//     C = G_[0][w, w] - X[w, :fill] Y[:fill, w],
// which is (G_[k-1])_{ww} of eq. DelayG0.  Proposals are scanned with a
// wave-wide ballot: the ratios of all not-yet-decided sites are evaluated from
// the current diagonal, and the first accepted site is taken, which is the
// same decision sequence as visiting the sites one by one, because a rejection
// changes nothing.  On acceptance the window parts of x_k = (Delta/r)
// G_[k-1][:, i_k] and y_k = (1 - G_[k-1])[i_k, :] (eq. DelayRgenk) are
// recorded and C is updated on the trailing block only (earlier sites of the
// window are never read again).
//
// The expand kernel then forms the full-length x_k, y_k for the accepted
// sites with the recursion of eq. DelayRgenk, in parallel over matrix rows
// (for x) and columns (for y), appending them to X and Y.  When the fill
// reaches the flush rank the MFMA GEMM applies G <- G - X Y (eq. FinalDelay).
#include "common.hpp"
#include "kernels.hpp"
#include "philox.hpp"

#include <type_traits>

namespace {

constexpr int WMAX = 64;
constexpr int WIN_THREADS = 256;

// Lane src's value of a real or complex scalar.
__device__ __forceinline__ double shfl_s(double v, int src) { return __shfl(v, src); }
__device__ __forceinline__ cplx shfl_s(cplx v, int src) { return cmake(__shfl(v.x, src), __shfl(v.y, src)); }

// window coefficient layout (in units of S): [0, WMAX) c_k; then xw[k][a]; then yw[k][b]
constexpr int WC_X = WMAX;
constexpr int WC_Y = WMAX + WMAX * WMAX;
static_assert(WMAX == DQMC_WMAX && WC_X == DQMC_WC_X && WC_Y == DQMC_WC_Y, "window table layout");

template <typename S>
__global__ void __launch_bounds__(WIN_THREADS)
k_window(const InstDev* __restrict__ insts, int W, int replay) {
  constexpr bool CX = ST<S>::is_complex;
  const InstDev& d = insts[blockIdx.y];
  InstState* st = d.st;
  if (st->init_mode || st->idle) return;
  const int N = d.N, M = d.M;
  const int phase = st->phase;
  const int up = sched_is_up(phase, M);
  const int l = sched_slice(phase, M);
  const int pass = up ? 0 : 1;
  const int w0 = st->cursor;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (w0 >= N) {
    if (tid == 0) { st->m_w = 0; st->wstart = N; st->wlen = 0; }
    return;
  }
  const int wn = min(W, N - w0);
  const int fill0 = st->fill;
  const S* G = matp<S>(d, MAT_G);
  const S* X = matp<S>(d, MAT_X);
  const S* Y = matp<S>(d, MAT_Y);
  S* wc = reinterpret_cast<S*>(d.wcoef);

  __shared__ S C[WMAX][WMAX + 1];
  __shared__ S Xw[16][WMAX];
  __shared__ S Yw[16][WMAX];
  __shared__ S xcol[WMAX], yrow[WMAX];
  __shared__ int xs[WMAX];
  __shared__ int sh_q, sh_mw;

  // ---- C = G[w,w] - X[w,:fill0] Y[:fill0,w]
  // every load below reads a clamped address and is masked afterwards, so
  // that the loads of a group are issued together
  S acc[16];
  const int ac = w0 + min(lane, wn - 1);
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = gld(G + ac + (size_t)(w0 + min(wave + 4 * q, wn - 1)) * N);
#pragma unroll
  for (int q = 0; q < 16; ++q)
    if (!(lane < wn && wave + 4 * q < wn)) acc[q] = ST<S>::zero();
  for (int m0 = 0; m0 < fill0; m0 += 16) {
    S xv[16 * WMAX / WIN_THREADS], yv[16 * WMAX / WIN_THREADS];
#pragma unroll
    for (int u = 0; u < 16 * WMAX / WIN_THREADS; ++u) {
      const int e = tid + u * WIN_THREADS, mm = e / WMAX, a = e % WMAX;
      const size_t mc = (size_t)min(m0 + mm, fill0 - 1) * N;
      const int aw = w0 + min(a, wn - 1);
      xv[u] = gld(X + aw + mc);
      yv[u] = gld(Y + mc + aw);
    }
#pragma unroll
    for (int u = 0; u < 16 * WMAX / WIN_THREADS; ++u) {
      const int e = tid + u * WIN_THREADS, mm = e / WMAX, a = e % WMAX;
      const bool ok = (m0 + mm < fill0) && a < wn;
      Xw[mm][a] = ok ? xv[u] : ST<S>::zero();
      Yw[mm][a] = ok ? yv[u] : ST<S>::zero();
    }
    __syncthreads();
    int mlim = min(16, fill0 - m0);
    for (int mm = 0; mm < mlim; ++mm) {
      S xv = Xw[mm][lane];
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[q] = acc[q] - xv * Yw[mm][wave + 4 * q];
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) C[lane][wave + 4 * q] = acc[q];
  if (tid < WMAX) xs[tid] = tid < wn ? (int)d.fields[(size_t)(l - 1) * N + w0 + tid] : 1;
  if (tid == 0) sh_mw = 0;
  __syncthreads();

  const double lam = d.lam;
  const int64_t rpos = st->replay_pos;
  // per-site constants of the scan, fixed for the whole window (a site's
  // field only changes when it is accepted, which ends its candidacy):
  // Delta, the prior factor of the ratio, and the uniform u (or the replayed
  // decision).  Spin channel: Delta = e^{-2 lambda x} - 1, R = e^{2 lambda x}
  // |r_up|^2; charge channel: Delta = e^{-2 i alpha x} - 1, R = e^{2 i alpha x}
  // r_up^2 (r_dn = r_up, prior ratio e^{2 i alpha x}), real up to rounding.
  const bool charge = d.channel != 0;
  S dls = ST<S>::zero(), pri = ST<S>::one();
  double usite = 0.0;
  bool rbit = false;
  if (wave == 0 && lane < wn) {
    const double x = (double)xs[lane];
    if constexpr (ST<S>::is_complex) {
      if (charge) {
        dls = cmake(cos(2.0 * lam * x) - 1.0, -sin(2.0 * lam * x));
        pri = cmake(cos(2.0 * lam * x), sin(2.0 * lam * x));
      } else {
        dls = ST<S>::from_re(exp(-2.0 * lam * x) - 1.0);
        pri = ST<S>::from_re(exp(2.0 * lam * x));
      }
    } else {
      dls = exp(-2.0 * lam * x) - 1.0;
      pri = exp(2.0 * lam * x);
    }
    if (replay) rbit = d.replay_bits[rpos + lane] != 0;
    else usite = site_uniform(d.seed, (uint64_t)st->sweep, pass, l, w0 + lane);
  }
  // The phase of det_up is carried in registers of thread 0 for the window.
  double ph_re = 0.0, ph_im = 0.0;
  if (tid == 0) { ph_re = st->ph_re; ph_im = st->ph_im; }
  int p = 0, k = 0;
  while (true) {
    // wave 0: ratios of the undecided sites, the first accepted one, and the
    // window parts of its x_k (column qs of C times c_k) and y_k (minus row
    // qs), zero on the sites up to qs
    if (wave == 0) {
      const int q = lane;
      const bool cand = q < wn && q >= p;
      bool acc_q = false;
      double R = 0.0;
      S r = ST<S>::one(), dl = ST<S>::zero();
      if (cand) {
        dl = dls;
        r = ST<S>::one() + dl * (ST<S>::one() - C[q][q]);
        R = charge ? real_part(pri * r * r) : real_part(pri) * absq(r);
        acc_q = replay ? rbit : usite < R;
        if (!(R == R) || R == 0.0 || R > 1e300) atomicOr(&st->numeric_err, NUMERR_RATIO);
      }
      const unsigned long long mask = __ballot(cand && acc_q);
      const int qs = mask ? (__ffsll((long long)mask) - 1) : wn;
      if (cand && q <= qs && d.replay_ratio) d.replay_ratio[rpos + q] = R;
      // training target of the proposal network: Barker acceptance Rt/(1+Rt)
      // of flipping the site again right after this decision (downward
      // pass), Rt = 1/R after an accepted flip and R after a rejected one
      if (cand && q <= qs && pass == 1 && d.targets)
        d.targets[(size_t)(l - 1) * N + w0 + q] =
            (float)(q == qs ? 1.0 / (1.0 + R) : (R < 1e300 ? R / (1.0 + R) : 1.0));
      if (lane == 0) sh_q = qs;
      if (qs < wn) {
        const S cfac = shfl_s(cdiv(dl, r), qs);
        const S rr = shfl_s(r, qs);
        const S dsel = shfl_s(dl, qs);
        const bool tail = q > qs && q < wn;
        const S xv = tail ? C[q][qs] * cfac : ST<S>::zero();
        const S yv = tail ? -C[qs][q] : ST<S>::zero();
        xcol[q] = xv;
        yrow[q] = yv;
        wc[WC_X + k * WMAX + q] = xv;
        wc[WC_Y + k * WMAX + q] = yv;
        if (lane == 0) {
          wc[k] = cfac;
          wc[DQMC_WC_D + k] = dsel;
          d.acc_site[k] = qs;
          d.acc_gsite[k] = w0 + qs;
          // det(1 + B..B) of spin up changes by the factor r_up (eq. rRatioLocal)
          const double ra = sqrt(absq(rr));
          if (ra > 0.0) {
            const double pr = real_part(rr) / ra, pi = imag_part(rr) / ra;
            const double a = ph_re, b = ph_im;
            ph_re = a * pr - b * pi;
            ph_im = a * pi + b * pr;
          }
        }
        if (q == qs) xs[qs] = -xs[qs];
      }
    }
    __syncthreads();
    const int qs = sh_q;
    if (qs >= wn) break;
    // trailing-block rank-1 update C -= x y^T: lane b of every wave takes
    // column b (a row of C is contiguous in LDS), the waves split the rows
    {
      const int b = qs + 1 + lane;
      if (b < wn) {
        const S yb = yrow[b];
        for (int a = qs + 1 + wave; a < wn; a += WIN_THREADS / 64) C[a][b] = C[a][b] - xcol[a] * yb;
      }
    }
    ++k;
    p = qs + 1;
    __syncthreads();
  }
  if (tid == 0) { st->ph_re = ph_re; st->ph_im = ph_im; sh_mw = k; }
  __syncthreads();
  // write back flipped fields and counters
  const int mw = sh_mw;
  if (tid < wn) d.fields[(size_t)(l - 1) * N + w0 + tid] = (int8_t)xs[tid];
  if (tid == 0) {
    st->m_w = mw;
    st->wstart = w0;
    st->wlen = wn;
    st->cursor = w0 + wn;
    st->proposals += wn;
    st->accepted += mw;
    if (replay) st->replay_pos = rpos + wn;
  }
}

// Full-length x_k, y_k for the accepted sites of the last window (or of an
// accepted learned block move), by the recursion of eq. DelayRgenk:
//   x_k[j] = c_k (G0[j, i_k] - sum_{m<k} x_m[j] y_m[i_k]),
//   y_k[j] = delta_{i_k j} - G0[i_k, j] + sum_{m<k} x_m[i_k] y_m[j],
// one thread per j (row of X and column of Y), accepted sites taken KC at a
// time so that every x_m[j], y_m[j] read from memory serves KC updates.
constexpr int KC = 8;
constexpr int EXP_WAVES = 4;   // each wave accumulates KC / EXP_WAVES of the chunk
template <typename S>
__global__ void __launch_bounds__(64 * EXP_WAVES)
k_expand(const InstDev* __restrict__ insts, int lcap) {
  constexpr int KW = KC / EXP_WAVES;
  const InstDev& d = insts[blockIdx.y];
  const InstState* st = d.st;
  // the state fields read here, loaded together before the exit tests
  const int init_mode = gldi(&st->init_mode), idle = gldi(&st->idle);
  const int mw = gldi(&st->m_w), fill0 = gldi(&st->fill);
  if (init_mode || idle || mw == 0) return;
  const int N = d.N;
  const int j0 = blockIdx.x * 64;
  if (j0 >= N) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int j = j0 + lane;
  const bool ok = j < N;
  const S* G = matp<S>(d, MAT_G);
  S* X = matp<S>(d, MAT_X);
  S* Y = matp<S>(d, MAT_Y);
  const S* wc = reinterpret_cast<const S*>(d.wcoef);

  extern __shared__ char xsmem[];
  // [m][kk]: y_m[i_k], x_m[i_k] for m < lcap (the launch's LDS capacity,
  // at least the largest fill a window can leave: kflush - 1 + WMAX)
  S* ycf = reinterpret_cast<S*>(xsmem);
  S* xcf = ycf + (size_t)lcap * KC;
  __shared__ S pax[KC][64], pay[KC][64];
  __shared__ int sites[WMAX], gsites[WMAX];   // table position, site index
  if (tid < WMAX) {
    sites[tid] = tid < mw ? gldi(d.acc_site + tid) : 0;
    gsites[tid] = tid < mw ? gldi(d.acc_gsite + tid) : 0;
  }
  __syncthreads();

  for (int k0 = 0; k0 < mw; k0 += KC) {
    const int kn = min(KC, mw - k0);
    const int nm = fill0 + k0 + kn;   // coefficients needed for m < nm
    for (int x = tid; x < nm * KC; x += 64 * EXP_WAVES) {
      int m = x / KC, kk = x % KC;
      S yv = ST<S>::zero(), xv = ST<S>::zero();
      if (kk < kn) {
        int ik = sites[k0 + kk], gi = gsites[k0 + kk];
        if (m < fill0) {
          yv = Y[(size_t)m * N + gi];
          xv = X[gi + (size_t)m * N];
        } else {
          int mp = m - fill0;
          yv = wc[WC_Y + mp * WMAX + ik];
          xv = wc[WC_X + mp * WMAX + ik];
        }
      }
      ycf[m * KC + kk] = yv;
      xcf[m * KC + kk] = xv;
    }
    __syncthreads();
    const int mpre = fill0 + k0;
    {
      // this wave's share of the chunk: kk = wave*KW .. wave*KW + KW - 1.
      // Lanes past N read row/column N-1 and their results are never stored.
      const int jc = min(j, N - 1);
      S ax[KW], ay[KW];
#pragma unroll
      for (int q = 0; q < KW; ++q) {
        const int kk = wave * KW + q;
        const int gi = gsites[k0 + min(kk, kn - 1)];
        ax[q] = gld(G + jc + (size_t)gi * N);
        ay[q] = -gld(G + gi + (size_t)jc * N);
        if (jc == gi) ay[q] = ay[q] + ST<S>::one();
        if (kk >= kn) { ax[q] = ST<S>::zero(); ay[q] = ST<S>::zero(); }
      }
      // rows m .. m+U-1 of X and columns of Y: all 2U loads issued as one
      // group (one memory round trip), then accumulated in ascending m
      auto rows = [&](auto count, int mb) {
        constexpr int U = decltype(count)::value;
        S xv[U], yv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          xv[u] = gld(X + jc + (size_t)(mb + u) * N);
          yv[u] = gld(Y + (size_t)(mb + u) * N + jc);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int q = 0; q < KW; ++q) {
            const int kk = wave * KW + q;
            ax[q] = ax[q] - xv[u] * ycf[(mb + u) * KC + kk];
            ay[q] = ay[q] + xcf[(mb + u) * KC + kk] * yv[u];
          }
      };
      int m = 0;
      for (; m + 8 <= mpre; m += 8) rows(std::integral_constant<int, 8>{}, m);
      if (m + 4 <= mpre) { rows(std::integral_constant<int, 4>{}, m); m += 4; }
      if (m + 2 <= mpre) { rows(std::integral_constant<int, 2>{}, m); m += 2; }
      if (m < mpre) rows(std::integral_constant<int, 1>{}, m);
#pragma unroll
      for (int q = 0; q < KW; ++q) {
        pax[wave * KW + q][lane] = ax[q];
        pay[wave * KW + q][lane] = ay[q];
      }
    }
    __syncthreads();
    if (ok && wave == 0) {
      // the recursion inside the chunk
      S ax[KC], ay[KC];
#pragma unroll
      for (int kk = 0; kk < KC; ++kk) { ax[kk] = pax[kk][lane]; ay[kk] = pay[kk][lane]; }
#pragma unroll
      for (int kk = 0; kk < KC; ++kk) {
        if (kk < kn) {
#pragma unroll
          for (int q = 0; q < kk; ++q) {
            ax[kk] = ax[kk] - ax[q] * ycf[(mpre + q) * KC + kk];
            ay[kk] = ay[kk] + xcf[(mpre + q) * KC + kk] * ay[q];
          }
          ax[kk] = wc[k0 + kk] * ax[kk];
          X[j + (size_t)(mpre + kk) * N] = ax[kk];
          Y[(size_t)(mpre + kk) * N + j] = ay[kk];
        }
      }
    }
    __syncthreads();
  }
}

__global__ void k_bump(const InstDev* __restrict__ insts, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  InstState* st = insts[i].st;
  if (st->init_mode || st->idle) return;
  st->fill += st->m_w;
  st->m_w = 0;
}

__global__ void k_flush_done(const InstDev* __restrict__ insts, int n, int any) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const InstDev& d = insts[i];
  InstState* st = d.st;
  if (st->init_mode || st->idle) return;
  if (any ? st->fill > 0 : st->fill >= d.kflush) {
    st->flush_rank_sum += st->fill;
    st->fill = 0;
    st->flushes += 1;
  }
}

__global__ void k_advance(const InstDev* __restrict__ insts, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const InstDev& d = insts[i];
  InstState* st = d.st;
  if (st->idle) return;
  st->cursor = 0;
  st->phase += 1;
  if (st->phase >= 2 * d.M) {
    st->phase = 0;
    if (st->init_mode) st->idle = 1;
    else {
      double cnt = d.obs[2 * OBS_COUNT];
      if (cnt > 0.0 && d.max_series > 0) {
        double* row = d.series + (size_t)(st->sweep % d.max_series) * OBS_COUNT;
        for (int k = 0; k < OBS_COUNT; ++k) row[k] = d.obs[OBS_COUNT + k] / cnt;
      }
      for (int k = 0; k < OBS_COUNT; ++k) d.obs[OBS_COUNT + k] = 0.0;
      d.obs[2 * OBS_COUNT] = 0.0;
      st->sweep += 1;
    }
  }
}

__global__ void k_init_state(const InstDev* __restrict__ insts, int n, int mode) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const InstDev& d = insts[i];
  InstState* st = d.st;
  st->cursor = 0;
  st->fill = 0;
  st->m_w = 0;
  st->idle = 0;
  st->init_mode = mode;
  st->phase = mode ? d.M : 0;
}

__global__ void k_replay_reset(const InstDev* __restrict__ insts, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) insts[i].st->replay_pos = 0;
}

__global__ void k_reset_counters(const InstDev* __restrict__ insts, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  InstState* st = insts[i].st;
  st->proposals = 0;
  st->accepted = 0;
  st->flushes = 0;
  st->n_meas = 0;
  st->drift_max = 0.0;
  st->drift_last = 0.0;
  st->flush_rank_sum = 0;
  st->series_base = st->sweep;
  st->learn_props = 0;
  st->learn_acc = 0;
  st->ph_drift = 0.0;
  st->numeric_err = 0;
}

}  // namespace

hipError_t launch_init_state(const InstDev* insts, int n_inst, int mode, hipStream_t s) {
  hipLaunchKernelGGL(k_init_state, dim3((n_inst + 63) / 64), dim3(64), 0, s, insts, n_inst, mode);
  return hipGetLastError();
}

hipError_t launch_replay_reset(const InstDev* insts, int n_inst, hipStream_t s) {
  hipLaunchKernelGGL(k_replay_reset, dim3((n_inst + 63) / 64), dim3(64), 0, s, insts, n_inst);
  return hipGetLastError();
}

hipError_t launch_reset_counters(const InstDev* insts, int n_inst, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_counters, dim3((n_inst + 63) / 64), dim3(64), 0, s, insts, n_inst);
  return hipGetLastError();
}

hipError_t launch_window(const InstDev* insts, int n_inst, bool cplx_, int W, int replay, hipStream_t s) {
  if (W > WMAX) W = WMAX;
  if (cplx_) hipLaunchKernelGGL(k_window<cplx>, dim3(1, n_inst), dim3(WIN_THREADS), 0, s, insts, W, replay);
  else hipLaunchKernelGGL(k_window<double>, dim3(1, n_inst), dim3(WIN_THREADS), 0, s, insts, W, replay);
  return hipGetLastError();
}

hipError_t launch_expand(const InstDev* insts, int n_inst, int Nmax, bool cplx_, int kcap_max, hipStream_t s) {
  dim3 grid((Nmax + 63) / 64, n_inst);
  size_t lds = (size_t)2 * kcap_max * KC * (cplx_ ? sizeof(cplx) : sizeof(double));
  if (cplx_) hipLaunchKernelGGL(k_expand<cplx>, grid, dim3(64 * EXP_WAVES), lds, s, insts, kcap_max);
  else hipLaunchKernelGGL(k_expand<double>, grid, dim3(64 * EXP_WAVES), lds, s, insts, kcap_max);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bump, dim3((n_inst + 63) / 64), dim3(64), 0, s, insts, n_inst);
  return hipGetLastError();
}

hipError_t launch_bump(const InstDev* insts, int n_inst, hipStream_t s) {
  hipLaunchKernelGGL(k_bump, dim3((n_inst + 63) / 64), dim3(64), 0, s, insts, n_inst);
  return hipGetLastError();
}

hipError_t launch_flush_done(const InstDev* insts, int n_inst, int any, hipStream_t s) {
  hipLaunchKernelGGL(k_flush_done, dim3((n_inst + 63) / 64), dim3(64), 0, s, insts, n_inst, any);
  return hipGetLastError();
}

hipError_t launch_advance(const InstDev* insts, int n_inst, hipStream_t s) {
  hipLaunchKernelGGL(k_advance, dim3((n_inst + 63) / 64), dim3(64), 0, s, insts, n_inst);
  return hipGetLastError();
}
