// Host side of the library: workspace layout, lattice tables, the sweep
// schedule and the C ABI declared in include/dqmc.h.
//
// The schedule is the paper's sweep (Sec. III): per instance an upward pass
// (wrap G to slice l, update slice l) and a downward pass (update slice l,
// wrap back), with a QR/UDV recomputation of G every n_stab slices (Sec. II B).
// All instances of a handle advance in lock step, one slice per step; every
// kernel handles all instances (blockIdx.y) and reads the per-instance
// schedule state from device memory, so the host issues the same launch
// sequence for every step and never waits on the device inside a sweep.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <cmath>
#include <complex>
#include <cstring>
#include <string>
#include <random>
#include <vector>

#include "common.hpp"
#include "dqmc.h"
#include "kernels.hpp"
#include "philox.hpp"

namespace {

constexpr int WINDOW = 64;
constexpr int QR_NB = 16;
constexpr int TRSM_ROWS = 32;
constexpr int GROUPS_MAX = 4;   // instance groups on separate streams
constexpr int MAX_SERIES = 4096;
constexpr int TAU_ROWS = 1024;     // per-pass rows kept of the time-displaced estimators
constexpr int MAX_DELAY = 192;
constexpr int FLUSH_KERNELS = 3;   // direct, LDS-tiled, work queue
// Default tolerance of max |G_wrap - G_scratch| at a recomputation.  FP64
// sweeps of the workloads here stay below 1e-6 (L = 3 .. 42, n_stab = 10).
constexpr double DRIFT_TOL_DEFAULT = 1e-4;

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

bool factor_L(int L, std::vector<int>& f) {
  f.clear();
  int n = L;
  while (n % 4 == 0) { f.push_back(4); n /= 4; }
  while (n % 2 == 0) { f.push_back(2); n /= 2; }
  for (int p : {3, 5, 7, 11, 13})
    while (n % p == 0) { f.push_back(p); n /= p; }
  return n == 1 && f.size() < 16;
}

bool is_twisted(const dqmc_instance_desc& d) {
  const double tp = 2.0 * M_PI;
  auto nz = [&](double th) { double r = std::fmod(th, tp); return std::fabs(r) > 1e-15 && std::fabs(std::fabs(r) - tp) > 1e-15; };
  return nz(d.theta1) || nz(d.theta2);
}

struct Offs {
  size_t st, obs, series, nk, fields, tab, roots, factors, perm, acc, gsite, wcoef, targets, learn, rsplit;
  size_t tau_sum, tau_rows;
  size_t vec[VEC_COUNT];
  size_t mat[MAT_COUNT];
  size_t stackU, stackT, stackD, stackPh;
  size_t end;
};

struct Plan {
  bool cplx = false;
  int Nmax = 0, Mmax = 0, n_stab = 0;
  size_t insts_off = 0, total = 0;
  std::vector<Offs> offs;
  // proposal network: FP32 master weights, Adam moments, gradient, BF16
  // copies; per-instance sampler windows, laid out with a common stride
  size_t net_master = 0, net_m = 0, net_v = 0, net_grad = 0, net_w = 0, net_Ls = 0;
  size_t lwin[3] = {0, 0, 0}, zcur = 0, zprop = 0;
  size_t lwin_stride[3] = {0, 0, 0}, z_stride = 0;
  // training samples: ring_cap slots of a 7 x Nmax int8 window and Nmax targets
  size_t ring_win = 0, ring_tg = 0;
  int ring_cap = 0;
};

constexpr int NET_RING = 2048;
constexpr int KTUNE_MAX = 128;   // largest flush rank dqmc_set_delay may choose without a new workspace   // training sample slots (rounded up to a multiple of the instances)

dqmc_status validate(const dqmc_instance_desc* d, int n, std::string& err) {
  if (!d || n < 1) { err = "need at least one instance"; return DQMC_EINVAL; }
  for (int i = 0; i < n; ++i) {
    const dqmc_instance_desc& x = d[i];
    std::vector<int> f;
    if (x.L < 2 || x.L > 45) { err = "L must be in [2, 45]"; return DQMC_EUNSUPPORTED; }
    if (!factor_L(x.L, f)) { err = "L must factor into 2, 3, 5, 7, 11, 13"; return DQMC_EUNSUPPORTED; }
    if (!(x.dtau > 0) || !(x.beta > 0) || !std::isfinite(x.t) || !(x.U >= 0)) { err = "need dtau > 0, beta > 0, U >= 0"; return DQMC_EINVAL; }
    double M = x.beta / x.dtau;
    if (std::fabs(M - std::round(M)) > 1e-9 || M < 1) { err = "beta/dtau must be a positive integer"; return DQMC_EINVAL; }
    if (x.n_stab < 1 || ((int)std::lround(M)) % x.n_stab != 0) { err = "n_stab must divide beta/dtau"; return DQMC_EINVAL; }
    if (x.n_stab != d[0].n_stab) { err = "all instances must share n_stab"; return DQMC_EINVAL; }
    if (x.n_delay < 1 || x.n_delay > MAX_DELAY) { err = "n_delay must be in [1, 192]"; return DQMC_EINVAL; }
    if (x.precision < DQMC_FP64 || x.precision > DQMC_MIXED_WRAP) { err = "unknown precision"; return DQMC_EINVAL; }
    if (x.precision != d[0].precision) { err = "all instances must share the precision"; return DQMC_EINVAL; }
    if (x.channel != DQMC_HS_SPIN && x.channel != DQMC_HS_CHARGE) { err = "unknown HS channel"; return DQMC_EINVAL; }
  }
  return DQMC_OK;
}

Plan make_plan(const dqmc_instance_desc* d, int n) {
  Plan p;
  for (int i = 0; i < n; ++i) p.cplx = p.cplx || is_twisted(d[i]) || d[i].channel == DQMC_HS_CHARGE;
  const size_t ss = p.cplx ? 16 : 8;
  size_t o = 0;
  p.insts_off = o;
  o = al(o + sizeof(InstDev) * n);
  p.n_stab = d[0].n_stab;
  for (int i = 0; i < n; ++i) {
    const int L = d[i].L, N = 2 * L * L, Nc = L * L;
    const int M = (int)std::lround(d[i].beta / d[i].dtau);
    const int C = M / d[i].n_stab;
    const int kcap = std::max(d[i].n_delay, KTUNE_MAX) + WINDOW;   // the flush rank can be retuned up to KTUNE_MAX
    p.Nmax = std::max(p.Nmax, N);
    p.Mmax = std::max(p.Mmax, M);
    Offs f;
    f.st = o; o = al(o + sizeof(InstState));
    f.obs = o; o = al(o + sizeof(double) * (2 * OBS_COUNT + 1));
    f.series = o; o = al(o + sizeof(double) * OBS_COUNT * MAX_SERIES);
    f.nk = o; o = al(o + sizeof(double) * 8 * Nc);
    f.tau_sum = o; o = al(o + sizeof(double) * (2 * (M / 2) + 3));
    f.tau_rows = o; o = al(o + sizeof(double) * (size_t)TAU_ROWS * (2 * (M / 2) + 2));
    f.fields = o; o = al(o + (size_t)M * N);
    f.tab = o; o = al(o + sizeof(cplx) * 16 * Nc);
    f.roots = o; o = al(o + sizeof(cplx) * 64);
    f.factors = o; o = al(o + sizeof(int32_t) * 16);
    f.perm = o; o = al(o + sizeof(int32_t) * 2 * N);
    f.acc = o; o = al(o + sizeof(int32_t) * WINDOW);
    f.gsite = o; o = al(o + sizeof(int32_t) * WINDOW);
    f.wcoef = o; o = al(o + ss * DQMC_WC_SIZE);
    f.targets = o; o = al(o + sizeof(float) * (size_t)M * N);
    f.learn = o; o = al(o + sizeof(LearnState));
    f.rsplit = o; o = al(o + ss * (size_t)RSPLIT_ROWS * N);
    for (int v = 0; v < VEC_COUNT; ++v) { f.vec[v] = o; o = al(o + sizeof(double) * 2 * N); }
    const size_t mb = ss * (size_t)N * N;
    for (int m = 0; m < MAT_COUNT; ++m) {
      f.mat[m] = o;
      if (m == MAT_SU || m == MAT_ST) continue;
      size_t bytes = (m == MAT_X || m == MAT_Y) ? ss * (size_t)N * std::max(N, kcap) : mb;
      o = al(o + bytes);
    }
    f.stackU = o; o = al(o + mb * (C + 1));
    f.stackT = o; o = al(o + mb * (C + 1));
    f.stackD = o; o = al(o + sizeof(double) * N * (C + 1));
    f.stackPh = o; o = al(o + sizeof(double) * 2 * (C + 1));
    f.end = o;
    p.offs.push_back(f);
  }
  const size_t ncm = (size_t)p.Nmax / 2;
  p.net_master = o; o = al(o + sizeof(float) * NET_NPARAM);
  p.net_m = o; o = al(o + sizeof(float) * NET_NPARAM);
  p.net_v = o; o = al(o + sizeof(float) * NET_NPARAM);
  p.net_grad = o; o = al(o + sizeof(float) * NET_NPARAM);
  p.net_w = o; o = al(o + NET_WBYTES + 256 * 8);
  p.net_Ls = o; o = al(o + sizeof(int32_t) * n);
  const int wt[3] = {7, 5, 3}, wc[3] = {16, 32, 32};
  for (int q = 0; q < 3; ++q) {
    p.lwin_stride[q] = (size_t)wt[q] * ncm * wc[q];       // bf16 elements per instance
    p.lwin[q] = o; o = al(o + 2 * p.lwin_stride[q] * n);
  }
  p.z_stride = ncm * 16;                                  // float elements per instance
  p.zcur = o; o = al(o + sizeof(float) * p.z_stride * n);
  p.zprop = o; o = al(o + sizeof(float) * p.z_stride * n);
  p.ring_cap = ((NET_RING + n - 1) / n) * n;
  p.ring_win = o; o = al(o + (size_t)p.ring_cap * 7 * p.Nmax);
  p.ring_tg = o; o = al(o + sizeof(float) * (size_t)p.ring_cap * p.Nmax);
  p.total = o;
  return p;
}

// exp(c h(k)) / Nc for h = [[0, f], [f*, 0]]: cosh(c|f|) 1 + sinh(c|f|)/|f| h.
void table_entry(std::complex<double> f, double c, double Nc, std::complex<double> out[4]) {
  double a = std::abs(f);
  double ca = c * a;
  double ch = std::cosh(ca);
  double sh;
  if (std::fabs(ca) < 1e-4) {
    double x2 = ca * ca;
    sh = c * (1.0 + x2 / 6.0 + x2 * x2 / 120.0);
  } else {
    sh = std::sinh(ca) / a;
  }
  out[0] = ch / Nc;
  out[1] = sh * f / Nc;
  out[2] = sh * std::conj(f) / Nc;
  out[3] = ch / Nc;
}

}  // namespace

struct dqmc_ctx {
  int n = 0;
  bool cplx = false;
  int Nmax = 0, Mmax = 0, n_stab = 0;
  std::vector<dqmc_instance_desc> desc;
  std::vector<InstDev> hd;
  Plan plan;
  InstDev* dinst = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t stream = nullptr;
  size_t lds_budget = 65536;
  int rmax = 4;  // largest FFT radix over the instances
  int kcap_max = 0;
  std::vector<int> fixedL;   // distinct L with a compile-time FFT plan
  std::vector<int> fft_tile; // register-line tile of fixedL[q] for side s at [2 q + s]
  bool any_generic = false;  // some L uses the runtime-plan FFT
  bool mixed = false;        // some step in single precision
  bool single_wrap = false;  // wraps run the FFT in complex64
  bool single_flush = false; // flushes form X Y with FP32 matrix cores
  // learned multi-site moves
  int learn_P = 0, learn_m = 0;   // moves per slice visit, sites per move
  int collect_every = 0;          // store a training sample every this many downward slices (0: off)
  int flush_variant = 0;          // 0: wave-per-block flush, 1: LDS-tiled GEMM, 2: work-queue flush (FP64 only)
  bool measure_k = true;          // momentum distribution with every measurement
  bool y_lu = true;               // Y^{-1} by pivoted LU (false: by Householder QR)
  bool expand_mm = false;         // window vectors in matrix form (false: by the recursion)
  bool submatrix = false;         // submatrix update: one block update per window
  int n_cu = 256;                 // compute units (persistent grids)
  // instance groups on their own streams (see issue_steps)
  int n_groups = 1;
  int group_off[GROUPS_MAX] = {0}, group_n[GROUPS_MAX] = {0};
  hipStream_t aux[GROUPS_MAX - 1] = {nullptr};   // streams of groups 1 ..
  hipEvent_t fork_ev = nullptr;
  hipEvent_t join_ev[GROUPS_MAX - 1] = {nullptr};
  int n_aux = 0;                                  // aux streams and join events created
  // captured stabilisation block (see run_steps)
  bool use_graphs = true;
  hipGraphExec_t gexec = nullptr;
  hipStream_t cap = nullptr;   // capture stream (the caller's may be the legacy null stream)
  std::vector<int> gkey;
  NetW netw{};
  float *net_master = nullptr, *net_m = nullptr, *net_v = nullptr, *net_grad = nullptr;
  int* net_Ls = nullptr;
  int adam_step = 0;
  std::string err;
  // live timing
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<int, size_t>> ev_marks;  // (class, index of start event)
  int64_t t_launch[DQMC_T_COUNT] = {0};
  double t_ms[DQMC_T_COUNT] = {0};
  double wrap_bytes = 0;
  std::vector<int64_t> rank_base;   // flush_rank_sum at timing reset
  int64_t sweeps_done = 0;
  int64_t steps_issued = 0;         // slice steps since the last initial build (all instances start at phase 0)
  int device = 0;                   // HIP device the handle was created on
};

namespace {

dqmc_status fail(dqmc_ctx* h, dqmc_status s, const std::string& msg) {
  if (h) h->err = msg;
  return s;
}

std::string numeric_message(int bits) {
  std::string m;
  if (bits & NUMERR_RATIO) m += "non-finite or zero acceptance ratio";
  if (bits & NUMERR_DRIFT) m += std::string(m.empty() ? "" : "; ") + "recomputation drift above the tolerance";
  return m;
}

#define HIPCHK(h, x)                                                                  \
  do {                                                                                \
    hipError_t e_ = (x);                                                              \
    if (e_ != hipSuccess)                                                             \
      return fail(h, DQMC_EHIP, std::string(#x) + ": " + hipGetErrorString(e_));      \
  } while (0)

hipStream_t pick(dqmc_ctx* h, void* s) { return s ? (hipStream_t)s : h->stream; }

// ---- live timing ---------------------------------------------------------------------------
hipEvent_t next_event(dqmc_ctx* h) {
  if (h->ev_used == h->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    h->ev_pool.push_back(e);
  }
  return h->ev_pool[h->ev_used++];
}

struct TimedScope {
  dqmc_ctx* h;
  hipStream_t s;
  int cls;
  size_t idx = 0;
  bool on = false;
  TimedScope(dqmc_ctx* h_, hipStream_t s_, int c) : h(h_), s(s_), cls(c) {
    if (!h->timing) return;
    idx = h->ev_used;
    hipEvent_t a = next_event(h), b = next_event(h);
    if (!a || !b) return;
    on = hipEventRecord(a, s) == hipSuccess;
  }
  ~TimedScope() {
    if (!on) return;
    if (hipEventRecord(h->ev_pool[idx + 1], s) == hipSuccess) {
      h->ev_marks.push_back({cls, idx});
      h->t_launch[cls] += 1;
    }
  }
};

// Resolve recorded event pairs into summed times (caller synchronised).
void drain_timing(dqmc_ctx* h) {
  for (auto& m : h->ev_marks) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, h->ev_pool[m.second], h->ev_pool[m.second + 1]) == hipSuccess)
      h->t_ms[m.first] += ms;
  }
  h->ev_marks.clear();
  h->ev_used = 0;
}

// ---- launch helpers ----------------------------------------------------------------------
struct Ctx {
  dqmc_ctx* h;
  hipStream_t s;
  const InstDev* di;   // first instance of the group this context launches for
  int n;               // instances in the group
  int off;             // index of di in the handle
  hipError_t e = hipSuccess;
  void chk(hipError_t x) { if (e == hipSuccess && x != hipSuccess) e = x; }
  // Mixed precision: the wraps of G run in complex64; the B products of the
  // stabilisation and the measurement's half step stay in FP64.
  void fft(int op, int side, int mat, int j = 0) {
    FftArgs a{op, side, mat, j, 0, 0, 0, 0};
    const bool single = h->single_wrap && (op == FOP_WRAP_PRE || op == FOP_WRAP_POST);
    chk(launch_fft(di, n, h->Nmax, h->cplx, a, h->lds_budget, h->rmax, h->fixedL.data(),
                   (int)h->fixedL.size(), h->any_generic, single, h->fft_tile.data(), s));
  }
  void fft_explicit(int side, int mat, int pre, int tab, int post, int slice) {
    FftArgs a{FOP_EXPLICIT, side, mat, 0, pre, tab, post, slice};
    chk(launch_fft(di, n, h->Nmax, h->cplx, a, h->lds_budget, h->rmax, h->fixedL.data(),
                   (int)h->fixedL.size(), h->any_generic, h->single_wrap, h->fft_tile.data(), s));
  }
  void gemm(GemmOperand A, GemmOperand B, GemmOperand C, GemmDim M, GemmDim N, GemmDim K,
            double alpha, double beta, int flags = 0) {
    chk(launch_gemm(di, n, h->Nmax, h->cplx, A, B, C, M, N, K, alpha, beta, flags, s));
  }
  void elem(int op, int a = 0, int b = 0, int c = 0, int v = 0) {
    ElemArgs x{op, a, b, c, v};
    chk(launch_elem(di, n, h->Nmax, h->cplx, x, s));
  }
};

GemmOperand opnd(int id, int op, int ra = 0, int rb = 0, int ca = 0, int cb = 0) {
  return GemmOperand{id, op, ra, rb, ca, cb};
}
GemmDim dim(int a, int b, int hi = 0) { return GemmDim{a, b, hi}; }

// Blocked Householder QR of MAT_QA in pairs of 16-column panels: the first
// panel is factored in registers and applied to its partner only, the
// partner is factored, the pair's 32-reflector compact-WY factor is formed,
// and one block-reflector update covers the trailing columns (half the passes
// over the trailing matrix of 16-column blocking).
void qr_factor(Ctx& c) {
  const int npair = (c.h->Nmax + 2 * QR_NB - 1) / (2 * QR_NB);
  for (int q = 0; q < npair; ++q) {
    c.chk(launch_qr_panel_reg(c.di, c.n, c.h->Nmax, c.h->cplx, 2 * q, c.s));
    c.chk(launch_apply_refl(c.di, c.n, c.h->Nmax, c.h->cplx, 2 * q, MAT_QA, 3, 1, c.s));
    c.chk(launch_qr_panel_reg(c.di, c.n, c.h->Nmax, c.h->cplx, 2 * q + 1, c.s));
    c.chk(launch_pair_t(c.di, c.n, c.h->cplx, q, c.s));
    c.chk(launch_apply_refl2(c.di, c.n, c.h->Nmax, c.h->cplx, q, MAT_QA, 0, 1, c.s));
  }
}

// target <- Q target (form Q when target = I), pairs applied last to first.
void apply_q(Ctx& c, int target) {
  const int npair = (c.h->Nmax + 2 * QR_NB - 1) / (2 * QR_NB);
  for (int q = npair - 1; q >= 0; --q)
    c.chk(launch_apply_refl2(c.di, c.n, c.h->Nmax, c.h->cplx, q, target, 1, 0, c.s));
}

// target <- Q^H target, pairs applied first to last, all columns.
void apply_qh(Ctx& c, int target) {
  const int npair = (c.h->Nmax + 2 * QR_NB - 1) / (2 * QR_NB);
  for (int q = 0; q < npair; ++q)
    c.chk(launch_apply_refl2(c.di, c.n, c.h->Nmax, c.h->cplx, q, target, 2, 1, c.s));
}

// MAT_W3 <- R^{-1} MAT_W3 with R the upper triangle of MAT_QA, recursively
// over 32-row blocks counted from the bottom (block b = rows
// [N - 32 (b + 1), N - 32 b), clipped at 0 for smaller instances of a batch):
// solve the lower half, subtract its contribution from the upper half with
// one GEMM, solve the upper half.  The large updates come first and fill the
// GPU even for a single instance.
void upper_solve_blocks(Ctx& c, int b0, int b1) {
  if (b1 - b0 == 1) {
    c.chk(launch_trsm_diag(c.di, c.n, c.h->Nmax, c.h->cplx, b0, c.s));
    return;
  }
  const int mid = (b0 + b1) / 2, T = TRSM_ROWS;
  upper_solve_blocks(c, b0, mid);
  // W3[top rows] -= R[top rows, lower cols] W3[lower rows];
  // top = [N - T b1, N - T mid), lower = [N - T mid, N - T b0)
  c.gemm(opnd(MAT_QA, 0, 1, -T * b1, 1, -T * mid), opnd(MAT_W3, 0, 1, -T * mid, 0, 0),
         opnd(MAT_W3, 0, 1, -T * b1, 0, 0), dim(1, -T * mid, T * (b1 - mid)), dim(1, 0),
         dim(1, -T * b0, T * (mid - b0)), -1.0, 1.0);
  upper_solve_blocks(c, mid, b1);
}

void upper_solve(Ctx& c) {
  const int nblk = (c.h->Nmax + TRSM_ROWS - 1) / TRSM_ROWS;
  upper_solve_blocks(c, 0, nblk);
}

// MAT_QA <- its LU factors with partial pivoting, P Y = L U (L unit lower,
// U upper, in place), recursively over column halves: factor the left half,
// A12 <- L11^{-1} A12, A22 <- A22 - A21 A12 (one MFMA GEMM whose depth is
// the left half's width), factor the right half.  The leaves are 16-column
// register panels; their row interchanges go to every other column at once,
// and the composed row permutation of Y collects in perm[N ..] (set to the
// identity by EO_BUILD_Y).  Column offsets count from 0 for every instance,
// so instances of a batch with smaller N drop out of the later launches.
void lower_solve(Ctx& c, int r0, int r1, int col0, int col1, int target);

void lu_factor(Ctx& c, int c0, int c1) {
  const int w = c1 - c0;
  if (w <= LU_NB) {
    c.chk(launch_lu_panel(c.di, c.n, c.h->Nmax, c.h->cplx, c0, w, c.s));
    c.chk(launch_lu_swap(c.di, c.n, c.h->Nmax, c.h->cplx, c0, w, c.s));
    return;
  }
  const int mid = c0 + ((w / 2 + LU_NB - 1) / LU_NB) * LU_NB;
  lu_factor(c, c0, mid);
  lower_solve(c, c0, mid, mid, c1, MAT_QA);
  // A22 -= A21 A12: rows [mid, N), columns [mid, min(c1, N)), depth mid - c0
  c.gemm(opnd(MAT_QA, 0, 0, mid, 0, c0), opnd(MAT_QA, 0, 0, c0, 0, mid), opnd(MAT_QA, 0, 0, mid, 0, mid),
         dim(1, -mid), dim(1, -mid, c1 - mid), dim(0, mid - c0), -1.0, 1.0);
  lu_factor(c, mid, c1);
}

// target[r0:r1, col0:col1] <- L^{-1} target[r0:r1, col0:col1] with L the unit
// lower triangle of MAT_QA's rows and columns [r0, r1): 32-row diagonal
// blocks, halves joined by one GEMM (rows and columns clipped at each
// instance's N).
void lower_solve(Ctx& c, int r0, int r1, int col0, int col1, int target) {
  if (r1 - r0 <= TL_NB) {
    c.chk(launch_trsm_lower(c.di, c.n, c.h->cplx, r0, r1 - r0, col0, col1, target, c.s));
    return;
  }
  const int rm = r0 + ((r1 - r0) / 2 + TL_NB - 1) / TL_NB * TL_NB;
  lower_solve(c, r0, rm, col0, col1, target);
  c.gemm(opnd(MAT_QA, 0, 0, rm, 0, r0), opnd(target, 0, 0, r0, 0, col0), opnd(target, 0, 0, rm, 0, col0),
         dim(1, -rm, r1 - rm), dim(1, -col0, col1 - col0), dim(0, rm - r0), -1.0, 1.0);
  lower_solve(c, rm, r1, col0, col1, target);
}

// Advance the working UDV chain by n_stab slices: A = B_chunk U D (the
// n_stab B's in one pass over U, columns scaled by D), pre-pivoted QR,
// U' = Q, D' = |diag R|, T' = D'^{-1} R P^T T; with phase = true the phase of
// det Q is recorded for the stack.
void chain_step(Ctx& c, bool phase) {
  dqmc_ctx* h = c.h;
  c.elem(EO_RESET_CHAIN);
  c.fft(FOP_STAB_CHAIN, 0, MAT_UW);
  c.chk(launch_colnorm_sort(c.di, c.n, h->Nmax, h->cplx, MAT_UW, c.s));
  c.elem(EO_GATHER_COLS, MAT_UW, 0, MAT_QA);
  c.elem(EO_GATHER_ROWS, MAT_TW, 0, MAT_W3);
  qr_factor(c);
  if (phase) c.chk(launch_detphase(c.di, c.n, h->cplx, 0, c.s));
  c.chk(launch_diag_abs(c.di, c.n, h->Nmax, h->cplx, c.s));
  c.gemm(opnd(MAT_QA, 0), opnd(MAT_W3, 0), opnd(MAT_TW, 0), dim(1, 0), dim(1, 0), dim(1, 0), 1.0, 0.0,
         GF_A_UPPER);
  c.elem(EO_SCALE_ROWS_INV, 0, 0, MAT_TW, VEC_DW);
  c.elem(EO_IDENTITY, 0, 0, MAT_UW);
  apply_q(c, MAT_UW);
}

// One checkpoint: advance the working UDV chain by n_stab slices, recompute
// G against the stack partner, record the drift, replace G, store the chain.
void stabilise(Ctx& c, bool measure) {
  dqmc_ctx* h = c.h;
  chain_step(c, true);
  // G = U_L D_Lb^-1 Y^-1 D_Rb^-1 U_R^H
  c.gemm(opnd(MAT_RU, 2), opnd(MAT_LU, 0), opnd(MAT_W1, 0), dim(1, 0), dim(1, 0), dim(1, 0), 1.0, 0.0);
  c.gemm(opnd(MAT_RT, 0), opnd(MAT_LT, 2), opnd(MAT_W2, 0), dim(1, 0), dim(1, 0), dim(1, 0), 1.0, 0.0);
  c.elem(EO_BUILD_Y, MAT_W1, MAT_W2, MAT_QA);
  if (h->y_lu) {
    // Y^{-1} RHS = U^{-1} L^{-1} (P RHS), the RHS built with P's row order
    lu_factor(c, 0, h->Nmax);
    c.chk(launch_detphase(c.di, c.n, h->cplx, 2, c.s));
    c.elem(EO_BUILD_RHS, 0, 0, MAT_W3, 1);
    lower_solve(c, 0, h->Nmax, 0, h->Nmax, MAT_W3);
  } else {
    c.elem(EO_BUILD_RHS, 0, 0, MAT_W3);
    qr_factor(c);
    c.chk(launch_detphase(c.di, c.n, h->cplx, 1, c.s));
    apply_qh(c, MAT_W3);
  }
  upper_solve(c);
  c.elem(EO_SCALE_ROWS_DLB, 0, 0, MAT_W3);
  c.gemm(opnd(MAT_LU, 0), opnd(MAT_W3, 0), opnd(MAT_GS, 0), dim(1, 0), dim(1, 0), dim(1, 0), 1.0, 0.0);
  c.elem(EO_DRIFT_REPLACE);
  c.chk(launch_stab_finish(c.di, c.n, c.s));
  c.elem(EO_STACK_STORE);
  if (measure) {
    // instances with sym_measure = 1 measure on the half-step G~, the others
    // on G (the half-step launches skip them; MAT_GS holds a copy of G)
    bool sym = false;
    for (int i = c.off; i < c.off + c.n; ++i) sym = sym || h->desc[i].sym_measure;
    if (sym || h->measure_k) {
      c.elem(EO_COPY, MAT_G, 0, MAT_GS);
      if (sym) {
        c.fft(FOP_HALF, 0, MAT_GS);
        c.fft(FOP_HALF, 1, MAT_GS);
      }
      c.chk(launch_measure(c.di, c.n, h->Nmax, h->cplx, MAT_GS, c.s));
    } else {
      c.chk(launch_measure(c.di, c.n, h->Nmax, h->cplx, MAT_G, c.s));
    }
    if (h->measure_k) {
      // momentum distribution: Ghat = F G F^dagger in place, its diagonal blocks
      c.fft(FOP_FOURIER, 0, MAT_GS);
      c.fft(FOP_FOURIER, 1, MAT_GS);
      c.chk(launch_measure_k(c.di, c.n, h->Nmax, h->cplx, MAT_GS, c.s));
    }
  }
}

// Checkpoint of the time-displaced pass at tau = c n_stab dtau (Sec. II C):
// with R = B(tau, 0) = U_R D_R T_R (the working chain) and
// L^dagger = B(beta, tau)^dagger = U_L D_L T_L (the stack slot of the last
// downward pass), the three functions share the Y of the equal-time
// recomputation:
//   G(tau,tau) = U_L D_Lb^{-1} Y^{-1} D_Rb^{-1} U_R^H
//   G(0,tau)   = -T_L^H D_Ls Y^{-1} D_Rb^{-1} U_R^H      (= -[B(tau,0) + B(beta,tau)^{-1}]^{-1})
//   G(tau,0)   = U_L D_Lb^{-1} Y^{-1} D_Rs T_R            (= [B(tau,0)^{-1} + B(beta,tau)]^{-1})
// so one LU of Y serves two right-hand sides.  The propagated functions are
// compared with these (drift) and replaced; the stack is not written.
void stabilise_tau(Ctx& c) {
  dqmc_ctx* h = c.h;
  chain_step(c, false);
  c.gemm(opnd(MAT_RU, 2), opnd(MAT_LU, 0), opnd(MAT_W1, 0), dim(1, 0), dim(1, 0), dim(1, 0), 1.0, 0.0);
  c.gemm(opnd(MAT_RT, 0), opnd(MAT_LT, 2), opnd(MAT_W2, 0), dim(1, 0), dim(1, 0), dim(1, 0), 1.0, 0.0);
  c.elem(EO_BUILD_Y, MAT_W1, MAT_W2, MAT_QA);
  lu_factor(c, 0, h->Nmax);
  // W3 = D_Lb^{-1} Y^{-1} D_Rb^{-1} U_R^H
  c.elem(EO_BUILD_RHS, 0, 0, MAT_W3, 1);
  lower_solve(c, 0, h->Nmax, 0, h->Nmax, MAT_W3);
  upper_solve(c);
  c.elem(EO_SCALE_ROWS_DLB, 0, 0, MAT_W3);
  c.gemm(opnd(MAT_LU, 0), opnd(MAT_W3, 0), opnd(MAT_GS, 0), dim(1, 0), dim(1, 0), dim(1, 0), 1.0, 0.0);
  c.elem(EO_SCALE_ROWS_DL, 0, 0, MAT_W3);   // D_Ls Y^{-1} D_Rb^{-1} U_R^H
  c.gemm(opnd(MAT_LT, 2), opnd(MAT_W3, 0), opnd(MAT_W1, 0), dim(1, 0), dim(1, 0), dim(1, 0), -1.0, 0.0);
  // W3 = D_Lb^{-1} Y^{-1} D_Rs T_R
  c.elem(EO_BUILD_RHS_T, 0, 0, MAT_W3);
  lower_solve(c, 0, h->Nmax, 0, h->Nmax, MAT_W3);
  upper_solve(c);
  c.elem(EO_SCALE_ROWS_DLB, 0, 0, MAT_W3);
  c.gemm(opnd(MAT_LU, 0), opnd(MAT_W3, 0), opnd(MAT_W2, 0), dim(1, 0), dim(1, 0), dim(1, 0), 1.0, 0.0);
  c.elem(EO_TAU_REPLACE);
  c.chk(launch_stab_finish(c.di, c.n, c.s));
}

// Time-displaced pass over the current configuration of every instance at
// the start of a sweep: G(tau,tau), G(tau,0), G(0,tau) for tau_l = l dtau,
// l = 0 .. min(M/2, lmax_req), propagated slice by slice (both sides, the
// left side, the right side of the upward wrap) and recomputed at every
// n_stab-th slice; the estimator of every slice is accumulated.  The fields,
// G, the stack and the schedule state are left as they were.
hipError_t tau_pass(dqmc_ctx* h, int lmax_req, hipStream_t s) {
  Ctx c{h, s, h->dinst, h->n, 0};
  int lmax = 0;
  for (auto& d : h->hd) lmax = std::max(lmax, lmax_req < 0 ? d.M / 2 : std::min(d.M / 2, lmax_req));
  c.chk(launch_tau_state(c.di, c.n, 0, 0, lmax_req, s));
  c.elem(EO_TAU_INIT);
  c.chk(launch_measure_tau(c.di, c.n, h->Nmax, h->cplx, 0, s));
  for (int l = 1; l <= lmax && c.e == hipSuccess; ++l) {
    c.chk(launch_tau_state(c.di, c.n, 1, l, lmax_req, s));
    c.fft(FOP_WRAP_PRE, 0, MAT_GTT);
    c.fft(FOP_WRAP_PRE, 1, MAT_GTT);
    c.fft(FOP_WRAP_PRE, 0, MAT_GT0);
    c.fft(FOP_WRAP_PRE, 1, MAT_G0T);
    if (l % h->n_stab == 0) stabilise_tau(c);
    c.chk(launch_measure_tau(c.di, c.n, h->Nmax, h->cplx, l, s));
  }
  c.chk(launch_tau_state(c.di, c.n, 2, 0, lmax_req, s));
  return c.e;
}

// One step of every instance (one slice of its sweep).
// Bytes of one wrap side-pass over every instance that is in the given pass.
double wrap_pass_bytes(dqmc_ctx* h, int64_t s, bool up) {
  double b = 0;
  const double ss = h->cplx ? 16.0 : 8.0;
  for (auto& d : h->hd) {
    int phase = (int)(s % (2 * d.M));
    if ((phase < d.M) == up) b += 2.0 * ss * (double)d.N * d.N;
  }
  return b;
}

// G <- G - X Y for the instances whose pending rank passes the flag's test:
// FP32 matrix cores for mixed precision, else the LDS-free wave-per-block
// kernel or the LDS-tiled GEMM (chosen by the autotuner).
void flush(Ctx& c, int flags) {
  dqmc_ctx* h = c.h;
  if (h->single_flush || h->flush_variant == 0) {
    c.chk(launch_flush_direct(c.di, c.n, h->Nmax, h->cplx, h->single_flush, flags, c.s));
  } else if (h->flush_variant == 2) {
    // resident workgroups per CU: two for complex (217 VGPRs), three for real
    c.chk(launch_flush_queue(c.di, c.n, h->cplx, flags, (h->cplx ? 2 : 3) * h->n_cu, c.s));
  } else {
    c.gemm(opnd(MAT_X, 0), opnd(MAT_Y, 1), opnd(MAT_G, 0), dim(1, 0), dim(1, 0), dim(0, 0), -1.0, 1.0,
           GF_K_FILL | flags);
  }
}

// Logits of the current slice of every instance from the 7-slice window in
// lwin[0]: three valid-in-time convolutions (7 -> 5 -> 3 -> 1 slices).
void window_logits(Ctx& c, float* z_base) {
  dqmc_ctx* h = c.h;
  const Plan& p = h->plan;
  char* b = h->ws;
  const int ncm = h->Nmax / 2;
  char* w0 = b + p.lwin[0] + 2 * p.lwin_stride[0] * c.off;
  char* w1 = b + p.lwin[1] + 2 * p.lwin_stride[1] * c.off;
  char* w2 = b + p.lwin[2] + 2 * p.lwin_stride[2] * c.off;
  const int* Ls = h->net_Ls + c.off;
  ConvGeom g1{0, Ls, 7, 5, 1, (long long)p.lwin_stride[0], (long long)p.lwin_stride[1]};
  c.chk(launch_conv(CONV_F1, w0, w1, h->netw, g1, c.n, ncm, c.s));
  ConvGeom g2{0, Ls, 5, 3, 1, (long long)p.lwin_stride[1], (long long)p.lwin_stride[2]};
  c.chk(launch_conv(CONV_F2, w1, w2, h->netw, g2, c.n, ncm, c.s));
  ConvGeom g3{0, Ls, 3, 1, 1, (long long)p.lwin_stride[2], (long long)p.z_stride};
  c.chk(launch_conv(CONV_F3, w2, z_base + p.z_stride * c.off, h->netw, g3, c.n, ncm, c.s));
}

// learn_P learned m-site moves on the current slice after its single-site
// updates (the delayed-update buffers are empty here): logits at the current
// fields, then per move: propose S and its block ratio, logits at the
// proposed fields, Metropolis-Hastings decision, and on acceptance the m
// rank-1 terms appended to X, Y; a final flush before the wrap.
void learned_moves(Ctx& c) {
  dqmc_ctx* h = c.h;
  const Plan& p = h->plan;
  float* zc = (float*)(h->ws + p.zcur);
  float* zp = (float*)(h->ws + p.zprop);
  const int ncm = h->Nmax / 2;
  c.chk(launch_learn_window(c.di, c.n, ncm, 0, c.s));
  window_logits(c, zc);
  for (int j = 0; j < h->learn_P; ++j) {
    c.chk(launch_learn_propose(c.di, c.n, h->cplx, j, h->learn_m, c.s));
    c.chk(launch_learn_window(c.di, c.n, ncm, 1, c.s));
    window_logits(c, zp);
    c.chk(launch_learn_decide(c.di, c.n, h->cplx, j, c.s));
    c.chk(launch_expand(c.di, c.n, h->Nmax, h->cplx, h->kcap_max, c.s));
  }
  flush(c, GF_IF_ANY);
  c.chk(launch_flush_done(c.di, c.n, 1, c.s));
}

void step(Ctx& c, int64_t s, bool measure, int replay) {
  dqmc_ctx* h = c.h;
  {
    TimedScope t(h, c.s, DQMC_T_WRAP);
    c.fft(FOP_WRAP_PRE, 0, MAT_G);
  }
  {
    TimedScope t(h, c.s, DQMC_T_WRAP);
    c.fft(FOP_WRAP_PRE, 1, MAT_G);
  }
  if (h->timing) h->wrap_bytes += 2 * wrap_pass_bytes(h, s, true);
  const int nwin = (h->Nmax + WINDOW - 1) / WINDOW;
  for (int w = 0; w < nwin; ++w) {
    {
      TimedScope t(h, c.s, DQMC_T_WINDOW);
      c.chk(launch_window(c.di, c.n, h->cplx, WINDOW, replay, c.s));
    }
    if (h->submatrix) {
      // the window's accepted flips as one block update (every window flushes)
      {
        TimedScope t(h, c.s, DQMC_T_EXPAND);
        const int w0 = w * WINDOW;
        c.chk(launch_submatrix_coef(c.di, c.n, h->cplx, c.s));
        c.gemm(opnd(MAT_G, 0, 0, 0, 0, w0), opnd(MAT_W2, 0), opnd(MAT_X, 0), dim(1, 0), dim(1, 0, WINDOW),
               dim(1, -w0, WINDOW), 1.0, 0.0, GF_NC_MW);
        c.chk(launch_submatrix_rows(c.di, c.n, h->Nmax, h->cplx, c.s));
        c.chk(launch_bump(c.di, c.n, c.s));
      }
      {
        TimedScope t(h, c.s, DQMC_T_FLUSH);
        flush(c, GF_IF_ANY);
      }
      c.chk(launch_flush_done(c.di, c.n, 1, c.s));
      continue;
    }
    {
      TimedScope t(h, c.s, DQMC_T_EXPAND);
      if (h->expand_mm) {
        c.chk(launch_expand_mm(c.di, c.n, h->Nmax, h->cplx, c.s));
        c.chk(launch_bump(c.di, c.n, c.s));
      } else {
        c.chk(launch_expand(c.di, c.n, h->Nmax, h->cplx, h->kcap_max, c.s));
      }
    }
    {
      TimedScope t(h, c.s, DQMC_T_FLUSH);
      flush(c, GF_IF_FULL);
    }
    c.chk(launch_flush_done(c.di, c.n, 0, c.s));
  }
  {
    TimedScope t(h, c.s, DQMC_T_FLUSH);
    flush(c, GF_IF_ANY);
  }
  c.chk(launch_flush_done(c.di, c.n, 1, c.s));
  if (h->collect_every > 0)
    c.chk(launch_collect(c.di, c.n, c.off, h->n, (int8_t*)(h->ws + h->plan.ring_win),
                         (float*)(h->ws + h->plan.ring_tg), h->plan.ring_cap, h->Nmax, h->collect_every, c.s));
  if (h->learn_P > 0 && !replay) {
    TimedScope t(h, c.s, DQMC_T_LEARN);
    learned_moves(c);
  }
  {
    TimedScope t(h, c.s, DQMC_T_WRAP);
    c.fft(FOP_WRAP_POST, 0, MAT_G);
  }
  {
    TimedScope t(h, c.s, DQMC_T_WRAP);
    c.fft(FOP_WRAP_POST, 1, MAT_G);
  }
  if (h->timing) h->wrap_bytes += 2 * wrap_pass_bytes(h, s, false);
  if ((s + 1) % h->n_stab == 0) {
    TimedScope t(h, c.s, DQMC_T_STAB);
    stabilise(c, measure);
  }
  c.chk(launch_advance(c.di, c.n, c.s));
}

dqmc_status upload_insts(dqmc_ctx* h, hipStream_t s) {
  HIPCHK(h, hipMemcpyAsync(h->dinst, h->hd.data(), sizeof(InstDev) * h->n, hipMemcpyHostToDevice, s));
  return DQMC_OK;
}

// Build the UDV stack and G(0) from the current fields: a downward pass
// without updates (only the chain steps), then the working chain is reset.
dqmc_status init_green(dqmc_ctx* h, hipStream_t s) {
  Ctx c{h, s, h->dinst, h->n, 0};
  c.chk(launch_init_state(h->dinst, h->n, 1, s));
  c.elem(EO_STACK_IDENTITY);
  c.elem(EO_IDENTITY, 0, 0, MAT_UW);
  c.elem(EO_IDENTITY, 0, 0, MAT_TW);
  c.elem(EO_SET_ONES, 0, 0, 0, VEC_DW);
  for (int64_t st = 0; st < h->Mmax; ++st) {
    if ((st + 1) % h->n_stab == 0) stabilise(c, false);
    c.chk(launch_advance(h->dinst, h->n, s));
  }
  c.chk(launch_init_state(h->dinst, h->n, 0, s));
  h->steps_issued = 0;
  if (c.e != hipSuccess) return fail(h, DQMC_EHIP, std::string("init: ") + hipGetErrorString(c.e));
  return DQMC_OK;
}

}  // namespace

// ================================ C ABI =================================================
extern "C" {

const char* dqmc_status_string(dqmc_status s) {
  switch (s) {
    case DQMC_OK: return "ok";
    case DQMC_EINVAL: return "invalid argument";
    case DQMC_ENOMEM: return "workspace too small";
    case DQMC_EHIP: return "HIP runtime error";
    case DQMC_ENUMERIC: return "numerical failure (non-finite or zero ratio, or drift above the tolerance)";
    case DQMC_ESTATE: return "invalid state";
    case DQMC_EUNSUPPORTED: return "unsupported size or option";
  }
  return "unknown status";
}

const char* dqmc_last_error(dqmc_handle h) { return h ? h->err.c_str() : "null handle"; }

// Split the instances into `groups` contiguous groups of about equal
// per-step work (~N^2 ~ L^4 per instance); fewer if there are fewer
// instances or streams.
void split_groups(dqmc_ctx* h, int groups) {
  const int n = h->n;
  int G = std::min(groups, std::min(n, h->fork_ev ? h->n_aux + 1 : 1));
  if (G < 1) G = 1;
  std::vector<double> w(n);
  double tot = 0;
  for (int i = 0; i < n; ++i) {
    const double L = h->desc[i].L;
    w[i] = L * L * L * L;
    tot += w[i];
  }
  int start = 0;
  double acc = 0;
  for (int g = 0; g < G; ++g) {
    int end = start + 1;
    acc += w[start];
    const double target = tot * (g + 1) / G;
    // extend while it brings the cumulative work closer to the target and
    // leaves at least one instance for every later group
    while (end < n - (G - 1 - g) && std::fabs(acc + w[end] - target) < std::fabs(acc - target)) acc += w[end++];
    if (g == G - 1) {
      while (end < n) acc += w[end++];
    }
    h->group_off[g] = start;
    h->group_n[g] = end - start;
    start = end;
  }
  h->n_groups = G;
}

dqmc_status dqmc_workspace_size(const dqmc_instance_desc* d, int32_t n, size_t* bytes) {
  std::string err;
  if (!bytes) return DQMC_EINVAL;
  dqmc_status st = validate(d, n, err);
  if (st != DQMC_OK) return st;
  *bytes = make_plan(d, n).total;
  return DQMC_OK;
}

dqmc_status dqmc_create(const dqmc_instance_desc* d, int32_t n, void* dev_ws, size_t bytes, void* stream,
                        dqmc_handle* out) {
  if (!out || !dev_ws) return DQMC_EINVAL;
  std::string err;
  dqmc_status vs = validate(d, n, err);
  if (vs != DQMC_OK) return vs;
  if (((uintptr_t)dev_ws) & 255) return DQMC_EINVAL;
  Plan p = make_plan(d, n);
  if (bytes < p.total) return DQMC_ENOMEM;
  dqmc_ctx* h = new dqmc_ctx();
  h->n = n;
  h->cplx = p.cplx;
  h->Nmax = p.Nmax;
  h->Mmax = p.Mmax;
  h->n_stab = p.n_stab;
  h->mixed = d[0].precision != DQMC_FP64;
  h->single_wrap = d[0].precision == DQMC_MIXED || d[0].precision == DQMC_MIXED_WRAP;
  h->single_flush = d[0].precision == DQMC_MIXED || d[0].precision == DQMC_MIXED_FLUSH;
  h->desc.assign(d, d + n);
  h->plan = p;
  for (int i = 0; i < n; ++i) {
    std::vector<int> fac;
    factor_L(d[i].L, fac);
    for (int r : fac) h->rmax = std::max(h->rmax, r);
    h->kcap_max = std::max(h->kcap_max, d[i].n_delay + WINDOW);
    if (fft_has_fixed(d[i].L)) {
      if (std::find(h->fixedL.begin(), h->fixedL.end(), d[i].L) == h->fixedL.end()) h->fixedL.push_back(d[i].L);
    } else {
      h->any_generic = true;
    }
  }
  h->fft_tile.assign(2 * h->fixedL.size(), 0);
  h->ws = (char*)dev_ws;
  h->ws_bytes = bytes;
  h->stream = (hipStream_t)stream;
  for (int g = 0; g < GROUPS_MAX - 1 && g < n - 1; ++g) {
    if (hipStreamCreateWithFlags(&h->aux[g], hipStreamNonBlocking) != hipSuccess) break;
    if (hipEventCreateWithFlags(&h->join_ev[g], hipEventDisableTiming) != hipSuccess) {
      (void)hipStreamDestroy(h->aux[g]);
      h->aux[g] = nullptr;
      break;
    }
    h->n_aux = g + 1;
  }
  if (h->n_aux > 0 && hipEventCreateWithFlags(&h->fork_ev, hipEventDisableTiming) != hipSuccess) h->fork_ev = nullptr;
  // Groups pay off when the batch has many instances whose latency-bound
  // kernels are small: 80 instances (64 L=18 + 16 L=12) run a sweep in 3.39 s
  // with 3 groups (2: 3.53 s, 4: 3.48 s), but four L=42 chains take 65 s
  // with 3 groups against 40.5 s in one.
  split_groups(h, n >= 24 ? 3 : (n >= 8 ? 2 : 1));
  if (hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking) != hipSuccess) {
    h->cap = nullptr;
    h->use_graphs = false;
  }
  h->dinst = (InstDev*)(h->ws + p.insts_off);
  const size_t ss = p.cplx ? 16 : 8;
  hipStream_t s = h->stream;
  std::vector<char> host;
  for (int i = 0; i < n; ++i) {
    const dqmc_instance_desc& x = d[i];
    const Offs& f = p.offs[i];
    InstDev dv;
    std::memset(&dv, 0, sizeof(dv));
    dv.L = x.L;
    dv.Nc = x.L * x.L;
    dv.N = 2 * dv.Nc;
    dv.M = (int)std::lround(x.beta / x.dtau);
    dv.n_stab = x.n_stab;
    dv.n_ckpt = dv.M / x.n_stab;
    dv.kflush = x.n_delay;
    dv.kcap = std::max(x.n_delay, KTUNE_MAX) + WINDOW;
    dv.is_complex = p.cplx;
    dv.sym_measure = x.sym_measure;
    dv.fft_fixed = fft_has_fixed(x.L) ? 1 : 0;
    dv.mixed = x.precision != DQMC_FP64 ? 1 : 0;
    dv.channel = x.channel;
    dv.lam = x.channel == DQMC_HS_CHARGE ? std::acos(std::exp(-x.dtau * x.U / 2.0))
                                         : std::acosh(std::exp(x.dtau * x.U / 2.0));
    dv.U = x.U; dv.dtau = x.dtau; dv.t = x.t;
    dv.theta1 = x.theta1; dv.theta2 = x.theta2;
    dv.seed = x.seed;
    char* b = h->ws;
    for (int m = 0; m < MAT_COUNT; ++m) dv.mat[m] = b + f.mat[m];
    for (int v = 0; v < VEC_COUNT; ++v) dv.vec[v] = (double*)(b + f.vec[v]);
    dv.stackU = b + f.stackU;
    dv.stackT = b + f.stackT;
    dv.stackD = (double*)(b + f.stackD);
    dv.stackPh = (double*)(b + f.stackPh);
    dv.drift_tol = DRIFT_TOL_DEFAULT;
    dv.mat_bytes = ss * (size_t)dv.N * dv.N;
    dv.fields = (int8_t*)(b + f.fields);
    dv.tab = (const cplx*)(b + f.tab);
    dv.roots = (const cplx*)(b + f.roots);
    dv.factors = (const int32_t*)(b + f.factors);
    dv.perm = (int32_t*)(b + f.perm);
    dv.acc_site = (int32_t*)(b + f.acc);
    dv.acc_gsite = (int32_t*)(b + f.gsite);
    dv.targets = (float*)(b + f.targets);
    dv.learn = (LearnState*)(b + f.learn);
    for (int q = 0; q < 3; ++q) dv.lwin[q] = b + p.lwin[q] + 2 * p.lwin_stride[q] * i;
    dv.zcur = (float*)(b + p.zcur) + p.z_stride * i;
    dv.zprop = (float*)(b + p.zprop) + p.z_stride * i;
    dv.wcoef = (double*)(b + f.wcoef);
    dv.rsplit = b + f.rsplit;
    dv.st = (InstState*)(b + f.st);
    dv.obs = (double*)(b + f.obs);
    dv.series = (double*)(b + f.series);
    dv.nk_sum = (double*)(b + f.nk);
    dv.max_series = MAX_SERIES;
    dv.tau_sum = (double*)(b + f.tau_sum);
    dv.tau_rows = (double*)(b + f.tau_rows);
    dv.tau_cap = TAU_ROWS;
    h->hd.push_back(dv);

    // momentum tables at k = ((l1 + Theta1/2pi)/L) b1 + ((l2 + Theta2/2pi)/L) b2 (eq. kpoints)
    const int L = x.L, Nc = dv.Nc;
    std::vector<std::complex<double>> tab((size_t)16 * Nc);
    const double cs[4] = {-x.dtau, x.dtau, -x.dtau / 2, x.dtau / 2};
    for (int l2 = 0; l2 < L; ++l2)
      for (int l1 = 0; l1 < L; ++l1) {
        double ka1 = (2.0 * M_PI * l1 + x.theta1) / L;  // k . a1
        double ka2 = (2.0 * M_PI * l2 + x.theta2) / L;  // k . a2
        std::complex<double> fk = -x.t * (1.0 + std::polar(1.0, ka1 - ka2) + std::polar(1.0, -ka2));
        int k = l1 + L * l2;
        for (int t = 0; t < 4; ++t) table_entry(fk, cs[t], Nc, &tab[(size_t)t * Nc * 4 + 4 * k]);
      }
    std::vector<std::complex<double>> roots(64);
    for (int m = 0; m < L; ++m) roots[m] = std::polar(1.0, -2.0 * M_PI * m / L);
    std::vector<int> fac;
    factor_L(L, fac);
    int32_t facs[16] = {0};
    for (size_t q = 0; q < fac.size(); ++q) facs[q] = fac[q];
    std::vector<int8_t> fields((size_t)dv.M * dv.N);
    for (int l = 1; l <= dv.M; ++l)
      for (int i = 0; i < dv.N; ++i) {
        philox_out o = philox4x32_10((uint32_t)i, (uint32_t)l, 0u, 2u, (uint32_t)(x.seed & 0xffffffffu),
                                     (uint32_t)(x.seed >> 32));
        fields[(size_t)(l - 1) * dv.N + i] = (o.w[0] & 1u) ? 1 : -1;
      }
    hipError_t e;
    if ((e = hipMemcpyAsync(b + f.tab, tab.data(), sizeof(cplx) * tab.size(), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(b + f.roots, roots.data(), sizeof(cplx) * 64, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(b + f.factors, facs, sizeof(facs), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(b + f.fields, fields.data(), fields.size(), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemsetAsync(b + f.st, 0, sizeof(InstState), s)) != hipSuccess ||
        (e = hipMemsetAsync(b + f.obs, 0, sizeof(double) * (2 * OBS_COUNT + 1), s)) != hipSuccess ||
        (e = hipMemsetAsync(b + f.series, 0, sizeof(double) * OBS_COUNT * MAX_SERIES, s)) != hipSuccess ||
        (e = hipMemsetAsync(b + f.nk, 0, sizeof(double) * 8 * Nc, s)) != hipSuccess ||
        (e = hipMemsetAsync(b + f.tau_sum, 0, sizeof(double) * (2 * (dv.M / 2) + 3), s)) != hipSuccess ||
        (e = hipMemsetAsync(b + f.targets, 0, sizeof(float) * (size_t)dv.M * dv.N, s)) != hipSuccess ||
        (e = hipMemsetAsync(b + f.learn, 0, sizeof(LearnState), s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess) {
      std::string m = std::string("create upload: ") + hipGetErrorString(e);
      delete h;
      (void)m;
      return DQMC_EHIP;
    }
  }
  int dev = 0, lds = 0;
  if (hipGetDevice(&dev) == hipSuccess) {
    h->device = dev;
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
      h->n_cu = ncu;
  }
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && lds > 0)
    h->lds_budget = std::min<size_t>(65536, (size_t)lds);
  {
    // proposal network: zero weights (uniform proposals) until set or trained
    char* b = h->ws;
    h->net_master = (float*)(b + p.net_master);
    h->net_m = (float*)(b + p.net_m);
    h->net_v = (float*)(b + p.net_v);
    h->net_grad = (float*)(b + p.net_grad);
    char* w = b + p.net_w;
    auto take = [&](size_t bytes) { char* r = w; w += (bytes + 255) / 256 * 256; return r; };
    h->netw.w1f = take(2 * 27 * 32 * 16);
    h->netw.w2f = take(2 * 27 * 32 * 32);
    h->netw.w3f = take(2 * 27 * 16 * 32);
    h->netw.w2b = take(2 * 27 * 32 * 32);
    h->netw.w3b = take(2 * 27 * 32 * 16);
    h->netw.b1 = (float*)take(4 * 32);
    h->netw.b2 = (float*)take(4 * 32);
    h->netw.b3 = (float*)take(4 * 16);
    h->net_Ls = (int*)(b + p.net_Ls);
    std::vector<int> Ls(n);
    for (int i = 0; i < n; ++i) Ls[i] = d[i].L;
    hipError_t e;
    if ((e = hipMemsetAsync(h->net_master, 0, sizeof(float) * NET_NPARAM, s)) != hipSuccess ||
        (e = hipMemsetAsync(h->net_m, 0, sizeof(float) * NET_NPARAM, s)) != hipSuccess ||
        (e = hipMemsetAsync(h->net_v, 0, sizeof(float) * NET_NPARAM, s)) != hipSuccess ||
        (e = hipMemcpyAsync(h->net_Ls, Ls.data(), sizeof(int) * n, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = launch_net_prep(h->net_master, h->netw, s)) != hipSuccess) {
      delete h;
      return DQMC_EHIP;
    }
  }
  dqmc_status st = upload_insts(h, s);
  if (st == DQMC_OK) st = init_green(h, s);
  if (st == DQMC_OK && hipStreamSynchronize(s) != hipSuccess) st = fail(h, DQMC_EHIP, "create: stream sync failed");
  if (st != DQMC_OK) { delete h; return st; }
  *out = h;
  return DQMC_OK;
}

dqmc_status dqmc_destroy(dqmc_handle h) {
  if (!h) return DQMC_EINVAL;
  (void)hipStreamSynchronize(h->stream);
  for (auto e : h->ev_pool) (void)hipEventDestroy(e);
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  if (h->cap) (void)hipStreamDestroy(h->cap);
  for (int g = 0; g < h->n_aux; ++g) {
    (void)hipStreamSynchronize(h->aux[g]);
    (void)hipStreamDestroy(h->aux[g]);
    (void)hipEventDestroy(h->join_ev[g]);
  }
  if (h->fork_ev) (void)hipEventDestroy(h->fork_ev);
  delete h;
  return DQMC_OK;
}

dqmc_status dqmc_shape(dqmc_handle h, int32_t inst, int32_t* N, int32_t* M, int32_t* is_complex) {
  if (!h || inst < 0 || inst >= h->n) return DQMC_EINVAL;
  if (N) *N = h->hd[inst].N;
  if (M) *M = h->hd[inst].M;
  if (is_complex) *is_complex = h->cplx ? 1 : 0;
  return DQMC_OK;
}

dqmc_status dqmc_set_fields(dqmc_handle h, int32_t inst, const int8_t* host_x) {
  if (!h || inst < 0 || inst >= h->n || !host_x) return DQMC_EINVAL;
  const InstDev& d = h->hd[inst];
  size_t n = (size_t)d.M * d.N;
  for (size_t i = 0; i < n; ++i)
    if (host_x[i] != 1 && host_x[i] != -1) return fail(h, DQMC_EINVAL, "fields must be +-1");
  HIPCHK(h, hipMemcpyAsync(d.fields, host_x, n, hipMemcpyHostToDevice, h->stream));
  dqmc_status st = init_green(h, h->stream);
  if (st != DQMC_OK) return st;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return DQMC_OK;
}

dqmc_status dqmc_get_fields(dqmc_handle h, int32_t inst, int8_t* host_x) {
  if (!h || inst < 0 || inst >= h->n || !host_x) return DQMC_EINVAL;
  const InstDev& d = h->hd[inst];
  HIPCHK(h, hipMemcpyAsync(host_x, d.fields, (size_t)d.M * d.N, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return DQMC_OK;
}

// steps is a multiple of n_stab, so the stabilisation points stay aligned
// across calls.
// With several instance groups, group 0 runs on the caller's stream and
// group g > 0 on the handle's stream g - 1; the groups' launches interleave on
// the host so that the latency-bound kernels of one group (window scan,
// expand, QR panels) overlap the bandwidth- and matrix-core-bound kernels of
// the others.  The handle's streams start after the caller's prior work (fork
// event) and the caller's stream waits for each of them at the end (join
// events).  With live timing on, one group is used so that every timed launch
// covers all instances.
static hipError_t issue_steps(dqmc_handle h, int64_t steps, int32_t measure, hipStream_t s, int replay,
                              int groups) {
  if (groups == 1) {
    Ctx c{h, s, h->dinst, h->n, 0};
    for (int64_t k = 0; k < steps && c.e == hipSuccess; ++k) step(c, k, measure != 0, replay);
    return c.e;
  }
  hipError_t e;
  if ((e = hipEventRecord(h->fork_ev, s)) != hipSuccess) return e;
  std::vector<Ctx> c;
  for (int g = 0; g < groups; ++g) {
    hipStream_t sg = g == 0 ? s : h->aux[g - 1];
    if (g > 0 && (e = hipStreamWaitEvent(sg, h->fork_ev, 0)) != hipSuccess) return e;
    c.push_back(Ctx{h, sg, h->dinst + h->group_off[g], h->group_n[g], h->group_off[g]});
  }
  bool ok = true;
  for (int64_t k = 0; k < steps && ok; ++k)
    for (int g = 0; g < groups && ok; ++g) {
      step(c[g], k, measure != 0, replay);
      ok = c[g].e == hipSuccess;
    }
  for (int g = 0; g < groups; ++g)
    if (c[g].e != hipSuccess) return c[g].e;
  for (int g = 1; g < groups; ++g) {
    if ((e = hipEventRecord(h->join_ev[g - 1], h->aux[g - 1])) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(s, h->join_ev[g - 1], 0)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// Everything a captured block of n_stab steps depends on besides device
// memory: the launches of a step are fixed by these.
static std::vector<int> graph_key(dqmc_handle h, int32_t measure, int replay, int groups) {
  std::vector<int> k = {measure != 0, replay, groups, h->learn_P, h->learn_m, h->collect_every, h->flush_variant,
                        h->kcap_max, h->measure_k ? 1 : 0, h->y_lu ? 1 : 0, h->expand_mm ? 1 : 0,
                        h->submatrix ? 1 : 0};
  k.insert(k.end(), h->fft_tile.begin(), h->fft_tile.end());
  return k;
}

// Sweeps are replayed as HIP graphs of one stabilisation block (n_stab slice
// steps: the launch sequence is the same for every block of every sweep, all
// state that changes lives in device memory), captured on first use.  The
// streams of the other instance groups join the capture through the fork
// event, so the graph keeps the overlap of the groups.  The eager path serves live
// timing and step counts that are not a whole number of blocks.
static dqmc_status run_steps(dqmc_handle h, int64_t steps, int32_t measure, hipStream_t s, int replay) {
  const int groups = h->timing ? 1 : h->n_groups;
  h->steps_issued += steps;
  if (!h->use_graphs || !h->cap || h->timing || steps % h->n_stab != 0) {
    hipError_t e = issue_steps(h, steps, measure, s, replay, groups);
    if (e != hipSuccess) return fail(h, DQMC_EHIP, std::string("sweep launch: ") + hipGetErrorString(e));
    return DQMC_OK;
  }
  const std::vector<int> key = graph_key(h, measure, replay, groups);
  if (!h->gexec || h->gkey != key) {
    if (h->gexec) {
      (void)hipGraphExecDestroy(h->gexec);
      h->gexec = nullptr;
    }
    hipGraph_t g = nullptr;
    // captured on the handle's own stream: the legacy null stream cannot be
    // captured, and recording does not execute, so no ordering with s is needed
    HIPCHK(h, hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
    hipError_t e = issue_steps(h, h->n_stab, measure, h->cap, replay, groups);
    hipError_t e2 = hipStreamEndCapture(h->cap, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return fail(h, DQMC_EHIP, std::string("graph capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
    }
    e = hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      h->gexec = nullptr;
      return fail(h, DQMC_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
    h->gkey = key;
  }
  for (int64_t b = 0; b < steps / h->n_stab; ++b) HIPCHK(h, hipGraphLaunch(h->gexec, s));
  return DQMC_OK;
}

dqmc_status dqmc_set_graphs(dqmc_handle h, int32_t on) {
  if (!h) return DQMC_EINVAL;
  h->use_graphs = on != 0;
  return DQMC_OK;
}

dqmc_status dqmc_set_streams(dqmc_handle h, int32_t groups) {
  if (!h || groups < 1 || groups > GROUPS_MAX) return DQMC_EINVAL;
  split_groups(h, groups);
  return DQMC_OK;
}

static dqmc_status run_sweeps(dqmc_handle h, int32_t n_sweeps, int32_t measure, hipStream_t s, int replay) {
  dqmc_status st = run_steps(h, (int64_t)n_sweeps * 2 * h->Mmax, measure, s, replay);
  if (st == DQMC_OK) h->sweeps_done += n_sweeps;
  return st;
}

dqmc_status dqmc_set_delay(dqmc_handle h, int32_t k) {
  if (!h || k < 1) return DQMC_EINVAL;
  for (auto& d : h->hd)
    if (k > d.kcap - WINDOW) return fail(h, DQMC_EINVAL, "flush rank exceeds the allocated capacity");
  HIPCHK(h, hipStreamSynchronize(h->stream));
  for (auto& d : h->hd) d.kflush = k;
  h->kcap_max = k + WINDOW;
  dqmc_status st = upload_insts(h, h->stream);
  if (st != DQMC_OK) return st;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return DQMC_OK;
}

dqmc_status dqmc_set_flush_kernel(dqmc_handle h, int32_t variant) {
  if (!h || variant < 0 || variant > 2) return DQMC_EINVAL;
  h->flush_variant = h->single_flush ? 0 : variant;
  return DQMC_OK;
}

dqmc_status dqmc_autotune(dqmc_handle h, int32_t steps, const int32_t* cand, int32_t n_cand, int32_t* best,
                          double* ms_per_step) {
  if (!h || !cand || n_cand < 1 || steps < 1 || steps % h->n_stab != 0) return DQMC_EINVAL;
  hipStream_t s = h->stream;
  hipEvent_t e0, e1;
  HIPCHK(h, hipEventCreate(&e0));
  HIPCHK(h, hipEventCreate(&e1));
  const bool timing = h->timing;
  h->timing = false;
  double best_ms = 1e300;
  int32_t bk = h->hd[0].kflush, bv = h->flush_variant;
  const int nvar = h->single_flush ? 1 : FLUSH_KERNELS;
  dqmc_status st = DQMC_OK;
  for (int q = 0; q < n_cand && st == DQMC_OK; ++q) {
    st = dqmc_set_delay(h, cand[q]);
    for (int v = 0; v < FLUSH_KERNELS && st == DQMC_OK; ++v) {
      if (v >= nvar) { if (ms_per_step) ms_per_step[FLUSH_KERNELS * q + v] = 0.0; continue; }
      h->flush_variant = v;
      st = run_steps(h, h->n_stab, 0, s, 0);   // untimed: captures this configuration's graph
      if (st != DQMC_OK) break;
      if (hipEventRecord(e0, s) != hipSuccess) { st = fail(h, DQMC_EHIP, "autotune event"); break; }
      st = run_steps(h, steps, 0, s, 0);
      if (st != DQMC_OK) break;
      float ms = 0.f;
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        st = fail(h, DQMC_EHIP, "autotune timing");
        break;
      }
      const double per = ms / steps;
      if (ms_per_step) ms_per_step[FLUSH_KERNELS * q + v] = per;
      if (per < best_ms) { best_ms = per; bk = cand[q]; bv = v; }
    }
  }
  h->timing = timing;
  h->flush_variant = bv;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != DQMC_OK) return st;
  if (best) { best[0] = bk; best[1] = bv; }
  st = dqmc_set_delay(h, bk);
  // back to a sweep boundary of the instances with the largest M, so that
  // later whole sweeps end where a sweep of those chains ends
  const int64_t per = 2 * (int64_t)h->Mmax, pad = (per - h->steps_issued % per) % per;
  if (st == DQMC_OK && pad > 0) st = run_steps(h, pad, 0, s, 0);
  if (st == DQMC_OK && hipStreamSynchronize(s) != hipSuccess) st = fail(h, DQMC_EHIP, "autotune sync");
  return st;
}

dqmc_status dqmc_set_fft_tile(dqmc_handle h, int32_t L, int32_t side, int32_t tile) {
  if (!h || (side != 0 && side != 1) || tile < 0 || tile >= FFT_TILES) return DQMC_EINVAL;
  for (size_t q = 0; q < h->fixedL.size(); ++q)
    if (h->fixedL[q] == L) {
      h->fft_tile[2 * q + side] = L <= 24 ? tile : 0;
      return DQMC_OK;
    }
  return fail(h, DQMC_EINVAL, "no instance of this L uses a register-line FFT plan");
}

dqmc_status dqmc_autotune_fft(dqmc_handle h, int32_t reps, int32_t* tiles_out, double* us_out) {
  if (!h || reps < 1) return DQMC_EINVAL;
  hipStream_t s = h->stream;
  hipEvent_t e0, e1;
  HIPCHK(h, hipEventCreate(&e0));
  HIPCHK(h, hipEventCreate(&e1));
  dqmc_status st = DQMC_OK;
  // each (L, side, tile): reps wrap transforms of the scratch matrix MAT_W1
  // with the e^{-dtau K} table and a diagonal (the arithmetic of a wrap)
  for (size_t q = 0; q < h->fixedL.size() && st == DQMC_OK; ++q) {
    for (int side = 0; side < 2 && st == DQMC_OK; ++side) {
      double best = 1e300;
      int bt = 0;
      for (int t = 0; t < FFT_TILES && st == DQMC_OK; ++t) {
        h->fft_tile[2 * q + side] = h->fixedL[q] <= 24 ? t : 0;
        Ctx c{h, s, h->dinst, h->n, 0};
        c.fft_explicit(side, MAT_W1, 0, TAB_P, side ? -1 : +1, 1);   // untimed first launch
        if (hipEventRecord(e0, s) != hipSuccess) { st = fail(h, DQMC_EHIP, "autotune_fft event"); break; }
        for (int r = 0; r < reps; ++r) c.fft_explicit(side, MAT_W1, 0, TAB_P, side ? -1 : +1, 1);
        float ms = 0.f;
        if (c.e != hipSuccess || hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
          st = fail(h, DQMC_EHIP, "autotune_fft timing");
          break;
        }
        const double us = 1e3 * ms / reps;
        if (us_out) us_out[(2 * q + side) * FFT_TILES + t] = us;
        if (us < best) { best = us; bt = t; }
      }
      h->fft_tile[2 * q + side] = h->fixedL[q] <= 24 ? bt : 0;
      if (tiles_out) tiles_out[2 * q + side] = h->fft_tile[2 * q + side];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

dqmc_status dqmc_fft_plan_count(dqmc_handle h, int32_t* n, int32_t* Ls) {
  if (!h || !n) return DQMC_EINVAL;
  *n = (int32_t)h->fixedL.size();
  if (Ls)
    for (size_t q = 0; q < h->fixedL.size(); ++q) Ls[q] = h->fixedL[q];
  return DQMC_OK;
}

dqmc_status dqmc_sweep(dqmc_handle h, int32_t n_sweeps, int32_t measure, void* stream) {
  if (!h || n_sweeps < 0) return DQMC_EINVAL;
  return run_sweeps(h, n_sweeps, measure, pick(h, stream), 0);
}

dqmc_status dqmc_replay(dqmc_handle h, const uint8_t* dev_bits, int64_t bits_per_inst, double* dev_ratios,
                        int32_t n_sweeps, int32_t measure, void* stream) {
  if (!h || !dev_bits || n_sweeps < 0) return DQMC_EINVAL;
  int64_t need = 0;
  for (auto& d : h->hd) need = std::max<int64_t>(need, (int64_t)n_sweeps * 2 * h->Mmax * d.N);
  if (bits_per_inst < need) return fail(h, DQMC_EINVAL, "replay stream too short");
  hipStream_t s = pick(h, stream);
  for (int i = 0; i < h->n; ++i) {
    h->hd[i].replay_bits = dev_bits + (size_t)i * bits_per_inst;
    h->hd[i].replay_ratio = dev_ratios ? dev_ratios + (size_t)i * bits_per_inst : nullptr;
    h->hd[i].replay_len = bits_per_inst;
  }
  dqmc_status st = upload_insts(h, s);
  if (st == DQMC_OK) {
    Ctx c{h, s, h->dinst, h->n, 0};
    c.chk(launch_replay_reset(h->dinst, h->n, s));
    st = c.e == hipSuccess ? run_sweeps(h, n_sweeps, measure, s, 1) : fail(h, DQMC_EHIP, "replay reset");
  }
  for (int i = 0; i < h->n; ++i) {
    h->hd[i].replay_bits = nullptr;
    h->hd[i].replay_ratio = nullptr;
    h->hd[i].replay_len = 0;
  }
  dqmc_status st2 = upload_insts(h, s);
  if (hipStreamSynchronize(s) != hipSuccess) return fail(h, DQMC_EHIP, "replay: stream sync failed");
  return st != DQMC_OK ? st : st2;
}

dqmc_status dqmc_get_green(dqmc_handle h, int32_t inst, int32_t spin, double* host_out) {
  if (!h || inst < 0 || inst >= h->n || !host_out || (spin != 0 && spin != 1)) return DQMC_EINVAL;
  const InstDev& d = h->hd[inst];
  const int N = d.N;
  const int w = h->cplx ? 2 : 1;
  std::vector<double> g((size_t)N * N * w);
  HIPCHK(h, hipMemcpyAsync(g.data(), d.mat[MAT_G], sizeof(double) * g.size(), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      if (spin == 0 || d.channel == DQMC_HS_CHARGE) {   // charge channel: G_dn = G_up
        for (int c = 0; c < w; ++c) host_out[((size_t)i * N + j) * w + c] = g[((size_t)j * N + i) * w + c];
      } else {
        // P (1 - G^dagger) P: element (i, j) = s_i s_j (delta_ij - conj(G_ji))
        double sgn = ((i < d.Nc) == (j < d.Nc)) ? 1.0 : -1.0;
        double re = g[((size_t)i * N + j) * w];  // G_ji (column-major: row j, column i)
        double im = w == 2 ? g[((size_t)i * N + j) * w + 1] : 0.0;
        host_out[((size_t)i * N + j) * w] = sgn * ((i == j ? 1.0 : 0.0) - re);
        if (w == 2) host_out[((size_t)i * N + j) * w + 1] = sgn * im;
      }
    }
  return DQMC_OK;
}

dqmc_status dqmc_set_green(dqmc_handle h, int32_t inst, const double* host_in) {
  if (!h || inst < 0 || inst >= h->n || !host_in) return DQMC_EINVAL;
  const InstDev& d = h->hd[inst];
  const int N = d.N;
  const int w = h->cplx ? 2 : 1;
  std::vector<double> g((size_t)N * N * w);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j)
      for (int c = 0; c < w; ++c) g[((size_t)j * N + i) * w + c] = host_in[((size_t)i * N + j) * w + c];
  HIPCHK(h, hipMemcpyAsync(d.mat[MAT_G], g.data(), sizeof(double) * g.size(), hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return DQMC_OK;
}

dqmc_status dqmc_wrap(dqmc_handle h, int32_t dir, int32_t slice, void* stream) {
  if (!h || (dir != 0 && dir != 1)) return DQMC_EINVAL;
  for (auto& d : h->hd)
    if (slice < 1 || slice > d.M) return fail(h, DQMC_EINVAL, "slice out of range");
  Ctx c{h, pick(h, stream), h->dinst, h->n, 0};
  if (dir == 0) {
    c.fft_explicit(0, MAT_G, 0, TAB_P, +1, slice);
    c.fft_explicit(1, MAT_G, 0, TAB_M, -1, slice);
  } else {
    c.fft_explicit(0, MAT_G, -1, TAB_M, 0, slice);
    c.fft_explicit(1, MAT_G, +1, TAB_P, 0, slice);
  }
  if (c.e != hipSuccess) return fail(h, DQMC_EHIP, hipGetErrorString(c.e));
  return DQMC_OK;
}

dqmc_status dqmc_flush_test(dqmc_handle h, int32_t inst, const double* host_X, const double* host_Y, int32_t k) {
  if (!h || inst < 0 || inst >= h->n || !host_X || !host_Y || k < 1) return DQMC_EINVAL;
  InstDev& d = h->hd[inst];
  if (k > std::max(d.N, d.kcap)) return fail(h, DQMC_EINVAL, "k exceeds the delayed-update capacity");
  const int w = h->cplx ? 2 : 1;
  hipStream_t s = h->stream;
  HIPCHK(h, hipMemcpyAsync(d.mat[MAT_X], host_X, sizeof(double) * w * (size_t)d.N * k, hipMemcpyHostToDevice, s));
  HIPCHK(h, hipMemcpyAsync(d.mat[MAT_Y], host_Y, sizeof(double) * w * (size_t)d.N * k, hipMemcpyHostToDevice, s));
  HIPCHK(h, hipMemcpyAsync((char*)d.st + offsetof(InstState, fill), &k, sizeof(int32_t), hipMemcpyHostToDevice, s));
  Ctx c{h, s, h->dinst, h->n, 0};
  flush(c, GF_IF_ANY);
  c.chk(launch_flush_done(h->dinst, h->n, 1, s));
  if (c.e != hipSuccess) return fail(h, DQMC_EHIP, hipGetErrorString(c.e));
  HIPCHK(h, hipStreamSynchronize(s));
  return DQMC_OK;
}

dqmc_status dqmc_measure(dqmc_handle h, int32_t inst, dqmc_obs* out) {
  if (!h || inst < 0 || inst >= h->n || !out) return DQMC_EINVAL;
  const InstDev& d = h->hd[inst];
  double obs[2 * OBS_COUNT + 1];
  InstState st;
  HIPCHK(h, hipMemcpyAsync(obs, d.obs, sizeof(obs), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipMemcpyAsync(&st, d.st, sizeof(st), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  double n = (double)st.n_meas;
  std::memset(out, 0, sizeof(*out));
  out->n_meas = st.n_meas;
  if (n > 0) {
    out->n = obs[OBS_N] / n;
    out->D = obs[OBS_D] / n;
    out->ekin = obs[OBS_EKIN] / n;
    out->e = obs[OBS_E] / n;
    out->Szz_G = obs[OBS_SZZ_G] / n;
    out->Szz_dk = obs[OBS_SZZ_DK] / n;
    out->m2 = obs[OBS_M2] / n;
    out->Rm2 = out->Szz_G != 0.0 ? 1.0 - out->Szz_dk / out->Szz_G : 0.0;
    out->phase_cos = obs[OBS_PHASE_RE] / n;
    out->phase_sin = obs[OBS_PHASE_IM] / n;
    out->chi_e = obs[OBS_CHI] / n;
    if (h->measure_k) {
      // |G_AB(K + dk)|: modulus of the mean spin-averaged n_AB at K + b1/L,
      // averaged over the two Dirac points K = (2 b1 + b2)/3, (b1 + 2 b2)/3
      const int L = d.L;
      const int K1[2][2] = {{(int)std::lround(2.0 * L / 3) % L, (int)std::lround(L / 3.0) % L},
                            {(int)std::lround(L / 3.0) % L, (int)std::lround(2.0 * L / 3) % L}};
      double gab = 0;
      for (int q = 0; q < 2; ++q) {
        const int k = (K1[q][0] + 1) % L + L * K1[q][1];
        double ab[2];
        HIPCHK(h, hipMemcpyAsync(ab, d.nk_sum + 8 * k + 2, sizeof(ab), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        gab += 0.5 * std::hypot(ab[0], ab[1]) / n;
      }
      out->GAB_dirac = gab;
    }
  }
  if (st.numeric_err) return fail(h, DQMC_ENUMERIC, numeric_message(st.numeric_err));
  return DQMC_OK;
}

dqmc_status dqmc_reset_obs(dqmc_handle h) {
  if (!h) return DQMC_EINVAL;
  for (auto& d : h->hd) {
    HIPCHK(h, hipMemsetAsync(d.obs, 0, sizeof(double) * (2 * OBS_COUNT + 1), h->stream));
    HIPCHK(h, hipMemsetAsync(d.nk_sum, 0, sizeof(double) * 8 * d.Nc, h->stream));
    HIPCHK(h, hipMemsetAsync(d.tau_sum, 0, sizeof(double) * (2 * (d.M / 2) + 3), h->stream));
  }
  Ctx c{h, h->stream, h->dinst, h->n, 0};
  c.chk(launch_reset_counters(h->dinst, h->n, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return DQMC_OK;
}

dqmc_status dqmc_get_series(dqmc_handle h, int32_t inst, double* host_out, int32_t max_sweeps, int32_t* n_out) {
  if (!h || inst < 0 || inst >= h->n || !host_out || !n_out || max_sweeps < 0) return DQMC_EINVAL;
  const InstDev& d = h->hd[inst];
  InstState st;
  HIPCHK(h, hipMemcpyAsync(&st, d.st, sizeof(st), hipMemcpyDeviceToHost, h->stream));
  std::vector<double> ser((size_t)OBS_COUNT * MAX_SERIES);
  HIPCHK(h, hipMemcpyAsync(ser.data(), d.series, sizeof(double) * ser.size(), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  int64_t have = std::min<int64_t>(st.sweep - st.series_base, MAX_SERIES);
  int64_t cnt = std::min<int64_t>(have, max_sweeps);
  for (int64_t q = 0; q < cnt; ++q) {
    int64_t sw = st.sweep - cnt + q;
    const double* row = &ser[(size_t)(sw % MAX_SERIES) * OBS_COUNT];
    double* o = host_out + q * OBS_COUNT;
    o[0] = row[OBS_N]; o[1] = row[OBS_D]; o[2] = row[OBS_EKIN]; o[3] = row[OBS_E];
    o[4] = row[OBS_SZZ_G]; o[5] = row[OBS_SZZ_DK]; o[6] = row[OBS_M2];
    o[7] = row[OBS_SZZ_G] != 0.0 ? 1.0 - row[OBS_SZZ_DK] / row[OBS_SZZ_G] : 0.0;
    o[8] = row[OBS_PHASE_RE]; o[9] = row[OBS_PHASE_IM]; o[10] = row[OBS_CHI];
  }
  *n_out = (int32_t)cnt;
  return DQMC_OK;
}

dqmc_status dqmc_measure_tau(dqmc_handle h, int32_t l_max, void* stream) {
  if (!h) return DQMC_EINVAL;
  hipError_t e = tau_pass(h, l_max, pick(h, stream));
  if (e != hipSuccess) return fail(h, DQMC_EHIP, std::string("time-displaced pass: ") + hipGetErrorString(e));
  return DQMC_OK;
}

dqmc_status dqmc_get_tau(dqmc_handle h, int32_t inst, double* host_aa, double* host_a, int64_t* n_pass) {
  if (!h || inst < 0 || inst >= h->n || !host_aa || !host_a || !n_pass) return DQMC_EINVAL;
  const InstDev& d = h->hd[inst];
  const int lc = d.M / 2;
  std::vector<double> sum(2 * lc + 3);
  InstState st;
  HIPCHK(h, hipMemcpyAsync(sum.data(), d.tau_sum, sizeof(double) * sum.size(), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipMemcpyAsync(&st, d.st, sizeof(st), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  const double n = sum[2 * lc + 2];
  *n_pass = (int64_t)n;
  for (int l = 0; l <= lc; ++l) {
    host_aa[l] = n > 0 ? sum[l] / n : 0.0;
    host_a[l] = n > 0 ? sum[lc + 1 + l] / n : 0.0;
  }
  if (st.numeric_err) return fail(h, DQMC_ENUMERIC, numeric_message(st.numeric_err));
  return DQMC_OK;
}

dqmc_status dqmc_get_tau_rows(dqmc_handle h, int32_t inst, double* host_rows, int32_t max_rows, int32_t* n_rows) {
  if (!h || inst < 0 || inst >= h->n || !host_rows || !n_rows || max_rows < 0) return DQMC_EINVAL;
  const InstDev& d = h->hd[inst];
  const int lc = d.M / 2, stride = 2 * lc + 2;
  double n = 0;
  std::vector<double> rows((size_t)TAU_ROWS * stride);
  HIPCHK(h, hipMemcpyAsync(&n, d.tau_sum + 2 * lc + 2, sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipMemcpyAsync(rows.data(), d.tau_rows, sizeof(double) * rows.size(), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  const int64_t have = std::min<int64_t>((int64_t)n, TAU_ROWS);
  const int64_t cnt = std::min<int64_t>(have, max_rows);
  for (int64_t q = 0; q < cnt; ++q) {
    const int64_t pass = (int64_t)n - cnt + q;
    std::memcpy(host_rows + q * stride, &rows[(size_t)(pass % TAU_ROWS) * stride], sizeof(double) * stride);
  }
  *n_rows = (int32_t)cnt;
  return DQMC_OK;
}

dqmc_status dqmc_get_green_tau(dqmc_handle h, int32_t inst, int32_t which, double* host_out) {
  if (!h || inst < 0 || inst >= h->n || !host_out || which < 0 || which > 2) return DQMC_EINVAL;
  const InstDev& d = h->hd[inst];
  const int N = d.N;
  const int w = h->cplx ? 2 : 1;
  const int mat = which == 0 ? MAT_GTT : (which == 1 ? MAT_GT0 : MAT_G0T);
  std::vector<double> g((size_t)N * N * w);
  HIPCHK(h, hipMemcpyAsync(g.data(), d.mat[mat], sizeof(double) * g.size(), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j)
      for (int c = 0; c < w; ++c) host_out[((size_t)i * N + j) * w + c] = g[((size_t)j * N + i) * w + c];
  return DQMC_OK;
}

dqmc_status dqmc_tau_integrals(const double* host_c, int32_t n, double dtau, int32_t n_sites, int32_t degree,
                               double* dD_dU, double* chi_F) {
  if (!host_c || n < 2 || !(dtau > 0) || n_sites < 1 || !dD_dU || !chi_F || degree > 12 ||
      (degree >= 0 && degree >= n))
    return DQMC_EINVAL;
  const double b = dtau * (n - 1);
  double i0 = 0, i1 = 0;
  if (degree < 0) {
    for (int l = 0; l < n; ++l) {
      const double w = (l == 0 || l == n - 1) ? 0.5 * dtau : dtau;
      i0 += w * host_c[l];
      i1 += w * (dtau * l) * host_c[l];
    }
  } else {
    // least squares C(tau) = sum_k a_k x^k, x = tau / b, by Householder QR of
    // the n x (degree + 1) Vandermonde matrix
    const int p = degree + 1;
    std::vector<double> A((size_t)n * p), r(host_c, host_c + n);
    for (int l = 0; l < n; ++l) {
      double x = (double)l / (n - 1), v = 1.0;
      for (int k = 0; k < p; ++k, v *= x) A[(size_t)k * n + l] = v;
    }
    for (int k = 0; k < p; ++k) {
      double* col = &A[(size_t)k * n];
      double nrm = 0;
      for (int l = k; l < n; ++l) nrm += col[l] * col[l];
      nrm = std::sqrt(nrm);
      if (nrm == 0) return DQMC_EINVAL;
      const double alpha = col[k] > 0 ? -nrm : nrm;
      col[k] -= alpha;   // v = x - alpha e_k, H = 1 - 2 v v^T / (v^T v)
      double vv = 0;
      for (int l = k; l < n; ++l) vv += col[l] * col[l];
      for (int q = k + 1; q < p; ++q) {
        double* cq = &A[(size_t)q * n];
        double dot = 0;
        for (int l = k; l < n; ++l) dot += col[l] * cq[l];
        for (int l = k; l < n; ++l) cq[l] -= 2.0 * dot / vv * col[l];
      }
      double dot = 0;
      for (int l = k; l < n; ++l) dot += col[l] * r[l];
      for (int l = k; l < n; ++l) r[l] -= 2.0 * dot / vv * col[l];
      col[k] = alpha;   // R_kk (the rest of the column below is no longer needed)
    }
    std::vector<double> a(p);
    for (int k = p - 1; k >= 0; --k) {
      double v = r[k];
      for (int q = k + 1; q < p; ++q) v -= A[(size_t)q * n + k] * a[q];
      a[k] = v / A[(size_t)k * n + k];
    }
    for (int k = 0; k < p; ++k) {
      i0 += b * a[k] / (k + 1);
      i1 += b * b * a[k] / (k + 2);
    }
  }
  *dD_dU = -2.0 * i0 / n_sites;
  *chi_F = i1;
  return DQMC_OK;
}

dqmc_status dqmc_set_update_scheme(dqmc_handle h, int32_t scheme) {
  if (!h || (scheme != 0 && scheme != 1)) return DQMC_EINVAL;
  h->submatrix = scheme == 1;
  return DQMC_OK;
}

dqmc_status dqmc_set_expand_kernel(dqmc_handle h, int32_t mm) {
  if (!h || (mm != 0 && mm != 1)) return DQMC_EINVAL;
  h->expand_mm = mm != 0;
  return DQMC_OK;
}

dqmc_status dqmc_set_y_solver(dqmc_handle h, int32_t lu) {
  if (!h || (lu != 0 && lu != 1)) return DQMC_EINVAL;
  h->y_lu = lu != 0;
  return DQMC_OK;
}

dqmc_status dqmc_set_measure_k(dqmc_handle h, int32_t on) {
  if (!h) return DQMC_EINVAL;
  h->measure_k = on != 0;
  return DQMC_OK;
}

dqmc_status dqmc_get_nk(dqmc_handle h, int32_t inst, int32_t raw, double* host_out) {
  if (!h || inst < 0 || inst >= h->n || !host_out) return DQMC_EINVAL;
  const InstDev& d = h->hd[inst];
  const int Nc = d.Nc, L = d.L;
  std::vector<double> sum((size_t)8 * Nc);
  InstState st;
  HIPCHK(h, hipMemcpyAsync(sum.data(), d.nk_sum, sizeof(double) * sum.size(), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipMemcpyAsync(&st, d.st, sizeof(st), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (st.n_meas < 1) return fail(h, DQMC_ESTATE, "no measurement taken");
  const double inv = 1.0 / (double)st.n_meas;
  const dqmc_instance_desc& x = h->desc[inst];
  for (int k = 0; k < Nc; ++k) {
    const double* m = &sum[(size_t)8 * k];
    if (raw) {
      for (int c = 0; c < 8; ++c) host_out[(size_t)8 * k + c] = m[c] * inv;
      continue;
    }
    // Hermitian part of the mean, its eigenvalues, and |f| at k + A (eq. kpoints)
    const double aa = m[0] * inv, bb = m[6] * inv;
    const double abr = 0.5 * (m[2] + m[4]) * inv, abi = 0.5 * (m[3] - m[5]) * inv;
    const double r = std::sqrt(0.25 * (aa - bb) * (aa - bb) + abr * abr + abi * abi);
    const int l1 = k % L, l2 = k / L;
    const double ka1 = (2.0 * M_PI * l1 + x.theta1) / L, ka2 = (2.0 * M_PI * l2 + x.theta2) / L;
    const std::complex<double> fk = -x.t * (1.0 + std::polar(1.0, ka1 - ka2) + std::polar(1.0, -ka2));
    double* o = host_out + (size_t)7 * k;
    o[0] = std::abs(fk);
    o[1] = aa; o[2] = bb; o[3] = abr; o[4] = abi;
    o[5] = 0.5 * (aa + bb) + r;
    o[6] = 0.5 * (aa + bb) - r;
  }
  return DQMC_OK;
}

dqmc_status dqmc_set_timing(dqmc_handle h, int32_t on) {
  if (!h) return DQMC_EINVAL;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  h->ev_marks.clear();
  h->ev_used = 0;
  for (int c = 0; c < DQMC_T_COUNT; ++c) { h->t_launch[c] = 0; h->t_ms[c] = 0; }
  h->wrap_bytes = 0;
  h->rank_base.assign(h->n, 0);
  for (int i = 0; i < h->n; ++i) {
    InstState st;
    HIPCHK(h, hipMemcpy(&st, h->hd[i].st, sizeof(st), hipMemcpyDeviceToHost));
    h->rank_base[i] = st.flush_rank_sum;
  }
  h->timing = on != 0;
  return DQMC_OK;
}

dqmc_status dqmc_get_timing(dqmc_handle h, dqmc_timing* out) {
  if (!h || !out) return DQMC_EINVAL;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  drain_timing(h);
  std::memset(out, 0, sizeof(*out));
  for (int c = 0; c < DQMC_T_COUNT; ++c) { out->launches[c] = h->t_launch[c]; out->ms[c] = h->t_ms[c]; }
  double flops = 0;
  for (int i = 0; i < h->n && i < (int)h->rank_base.size(); ++i) {
    InstState st;
    HIPCHK(h, hipMemcpy(&st, h->hd[i].st, sizeof(st), hipMemcpyDeviceToHost));
    double N = h->hd[i].N;
    flops += (h->cplx ? 8.0 : 2.0) * N * N * (double)(st.flush_rank_sum - h->rank_base[i]);
  }
  out->flush_flops = flops;
  out->wrap_bytes = h->wrap_bytes;
  return DQMC_OK;
}

dqmc_status dqmc_get_stats(dqmc_handle h, int32_t inst, dqmc_stats* out) {
  if (!h || inst < 0 || inst >= h->n || !out) return DQMC_EINVAL;
  InstState st;
  HIPCHK(h, hipMemcpyAsync(&st, h->hd[inst].st, sizeof(st), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  out->proposals = st.proposals;
  out->accepted = st.accepted;
  out->flushes = st.flushes;
  out->sweeps = st.sweep;
  out->drift_max = st.drift_max;
  out->drift_last = st.drift_last;
  out->numeric_err = st.numeric_err;
  out->learn_proposals = st.learn_props;
  out->learn_accepted = st.learn_acc;
  out->phase_re = st.ph_re;
  out->phase_im = st.ph_im;
  out->phase_drift = st.ph_drift;
  if (st.numeric_err) return fail(h, DQMC_ENUMERIC, numeric_message(st.numeric_err));
  return DQMC_OK;
}

dqmc_status dqmc_set_drift_tol(dqmc_handle h, double tol) {
  if (!h || !(tol > 0.0)) return DQMC_EINVAL;
  for (auto& d : h->hd) d.drift_tol = tol;
  dqmc_status st = upload_insts(h, h->stream);
  if (st != DQMC_OK) return st;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return DQMC_OK;
}

dqmc_status dqmc_set_proposals(dqmc_handle h, int32_t per_slice, int32_t m) {
  if (!h || per_slice < 0 || per_slice > 8) return DQMC_EINVAL;
  if (per_slice > 0 && (m < 1 || m > LEARN_MMAX)) return DQMC_EINVAL;
  for (auto& d : h->hd) {
    if (per_slice > 0 && m >= d.N) return fail(h, DQMC_EINVAL, "m must be smaller than the number of sites");
    if (per_slice > 0 && d.channel == DQMC_HS_CHARGE)
      return fail(h, DQMC_EUNSUPPORTED, "learned proposals support the spin channel only");
  }
  h->learn_P = per_slice;
  h->learn_m = per_slice > 0 ? m : 0;
  return DQMC_OK;
}

dqmc_status dqmc_net_set_weights(dqmc_handle h, const float* host_w, int64_t n) {
  if (!h || !host_w || n != NET_NPARAM) return DQMC_EINVAL;
  hipStream_t s = h->stream;
  HIPCHK(h, hipMemcpyAsync(h->net_master, host_w, sizeof(float) * NET_NPARAM, hipMemcpyHostToDevice, s));
  HIPCHK(h, hipMemsetAsync(h->net_m, 0, sizeof(float) * NET_NPARAM, s));
  HIPCHK(h, hipMemsetAsync(h->net_v, 0, sizeof(float) * NET_NPARAM, s));
  HIPCHK(h, launch_net_prep(h->net_master, h->netw, s));
  HIPCHK(h, hipStreamSynchronize(s));
  h->adam_step = 0;
  return DQMC_OK;
}

dqmc_status dqmc_net_init(dqmc_handle h, uint64_t seed) {
  if (!h) return DQMC_EINVAL;
  // W1, W2 ~ N(0, 1/fan_in) so that gradients reach every layer; W3 and the
  // biases zero, so that the proposals start uniform
  std::mt19937_64 g(seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  std::vector<float> w(NET_NPARAM, 0.f);
  for (int i = NET_OFF_W1; i < NET_OFF_B1; ++i) w[i] = (float)(nd(g) / std::sqrt(27.0 * 2.0));
  for (int i = NET_OFF_W2; i < NET_OFF_B2; ++i) w[i] = (float)(nd(g) / std::sqrt(27.0 * NET_CH));
  return dqmc_net_set_weights(h, w.data(), NET_NPARAM);
}

dqmc_status dqmc_net_get_weights(dqmc_handle h, float* host_w, int64_t n) {
  if (!h || !host_w || n != NET_NPARAM) return DQMC_EINVAL;
  HIPCHK(h, hipMemcpyAsync(host_w, h->net_master, sizeof(float) * NET_NPARAM, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return DQMC_OK;
}

dqmc_status dqmc_get_targets(dqmc_handle h, int32_t inst, float* host_out) {
  if (!h || inst < 0 || inst >= h->n || !host_out) return DQMC_EINVAL;
  const InstDev& d = h->hd[inst];
  HIPCHK(h, hipMemcpyAsync(host_out, d.targets, sizeof(float) * (size_t)d.M * d.N, hipMemcpyDeviceToHost,
                           h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return DQMC_OK;
}

}  // extern "C"

namespace {

constexpr int NET_VCH = 1024;   // output voxels per weight-gradient workgroup

// Layout of the training scratch for configurations of one size.
struct NetPlan {
  int L = 0, M = 0, N = 0, Nc = 0, batch = 0, chunks = 0, lblocks = 0;
  int64_t n_samples = 0;
  size_t fields = 0, targets = 0, a0 = 0, h1 = 0, h2 = 0, z = 0, dz = 0, d2 = 0, d1 = 0, part = 0, partb = 0,
         lossp = 0, lossv = 0, total = 0;
};
constexpr int NET_LOSS_SLOTS = 1024;

bool net_plan(int L, int M, int64_t n_samples, int batch, NetPlan& p) {
  if (L < 2 || L > 45 || M < 1 || n_samples < 1 || batch < 1 || batch > NET_MAXBATCH) return false;
  p.L = L; p.M = M; p.Nc = L * L; p.N = 2 * p.Nc; p.batch = batch; p.n_samples = n_samples;
  const size_t vox = (size_t)M * p.Nc, B = batch;
  p.chunks = wgrad_chunks(M, p.Nc, NET_VCH);
  p.lblocks = (int)((vox + 255) / 256);
  size_t o = 0;
  p.fields = o; o = al(o + (size_t)n_samples * M * p.N);
  p.targets = o; o = al(o + sizeof(float) * (size_t)n_samples * M * p.N);
  p.a0 = o; o = al(o + 2 * B * vox * 16);
  p.h1 = o; o = al(o + 2 * B * vox * 32);
  p.h2 = o; o = al(o + 2 * B * vox * 32);
  p.z = o; o = al(o + 4 * B * vox * 16);
  p.dz = o; o = al(o + 2 * B * vox * 16);
  p.d2 = o; o = al(o + 2 * B * vox * 32);
  p.d1 = o; o = al(o + 2 * B * vox * 32);
  p.part = o; o = al(o + sizeof(float) * B * p.chunks * 27 * 32 * 32);
  p.partb = o; o = al(o + sizeof(float) * B * p.chunks * 32);
  p.lossp = o; o = al(o + sizeof(float) * B * p.lblocks);
  p.lossv = o; o = al(o + sizeof(float) * NET_LOSS_SLOTS);
  p.total = o;
  return true;
}

// Forward pass of the batch idx; with targets, the loss into loss_slot and
// (backward) the gradient into h->net_grad.
hipError_t net_pass(dqmc_ctx* h, const NetPlan& p, char* ws, const BatchIdx& idx, bool loss, bool backward,
                    int loss_slot, hipStream_t s) {
  const int M = p.M, Nc = p.Nc, N = p.N, L = p.L;
  const long long v = (long long)M * Nc;
  hipError_t e;
  auto ok = [&](hipError_t x) { e = x; return x == hipSuccess; };
  ConvGeom g{L, nullptr, M, M, 0, v * 16, v * 32};
  if (!ok(launch_net_input((const int8_t*)(ws + p.fields), N, Nc, M, idx, ws + p.a0, s))) return e;
  if (!ok(launch_conv(CONV_F1, ws + p.a0, ws + p.h1, h->netw, g, idx.n, Nc, s))) return e;
  g.in_stride = v * 32; g.out_stride = v * 32;
  if (!ok(launch_conv(CONV_F2, ws + p.h1, ws + p.h2, h->netw, g, idx.n, Nc, s))) return e;
  g.in_stride = v * 32; g.out_stride = v * 16;
  if (!ok(launch_conv(CONV_F3, ws + p.h2, ws + p.z, h->netw, g, idx.n, Nc, s))) return e;
  if (!loss) return hipSuccess;
  float* lossv = (float*)(ws + p.lossv) + loss_slot;
  if (!ok(launch_net_loss((const float*)(ws + p.z), (const float*)(ws + p.targets), idx, N, Nc, M, ws + p.dz,
                          (float*)(ws + p.lossp), lossv, s)))
    return e;
  if (!backward) return hipSuccess;
  float* part = (float*)(ws + p.part);
  float* partb = (float*)(ws + p.partb);
  const int nch = p.chunks * idx.n;
  // layer 3: dW3 from (h2, dz); dh2 = conv^T(dz)
  ConvGeom gw{L, nullptr, M, M, 0, v * 32, v * 16};
  if (!ok(launch_wgrad(WGRAD_3, ws + p.h2, ws + p.dz, part, partb, gw, idx.n, Nc, NET_VCH, s))) return e;
  if (!ok(launch_wgrad_reduce(WGRAD_3, part, partb, nch, h->net_grad, s))) return e;
  ConvGeom gb{L, nullptr, M, M, 0, v * 16, v * 32};
  if (!ok(launch_conv(CONV_B3, ws + p.dz, ws + p.d2, h->netw, gb, idx.n, Nc, s))) return e;
  if (!ok(launch_tanh_back(ws + p.d2, ws + p.h2, (size_t)idx.n * v * 32, s))) return e;
  // layer 2
  gw.in_stride = v * 32; gw.out_stride = v * 32;
  if (!ok(launch_wgrad(WGRAD_2, ws + p.h1, ws + p.d2, part, partb, gw, idx.n, Nc, NET_VCH, s))) return e;
  if (!ok(launch_wgrad_reduce(WGRAD_2, part, partb, nch, h->net_grad, s))) return e;
  gb.in_stride = v * 32; gb.out_stride = v * 32;
  if (!ok(launch_conv(CONV_B2, ws + p.d2, ws + p.d1, h->netw, gb, idx.n, Nc, s))) return e;
  if (!ok(launch_tanh_back(ws + p.d1, ws + p.h1, (size_t)idx.n * v * 32, s))) return e;
  // layer 1
  gw.in_stride = v * 16; gw.out_stride = v * 32;
  if (!ok(launch_wgrad(WGRAD_1, ws + p.a0, ws + p.d1, part, partb, gw, idx.n, Nc, NET_VCH, s))) return e;
  return launch_wgrad_reduce(WGRAD_1, part, partb, nch, h->net_grad, s);
}

dqmc_status net_upload(dqmc_ctx* h, const NetPlan& p, char* ws, const int8_t* fields, const float* targets,
                       hipStream_t s) {
  const size_t n = (size_t)p.n_samples * p.M * p.N;
  for (size_t i = 0; i < n; ++i)
    if (fields[i] != 1 && fields[i] != -1) return fail(h, DQMC_EINVAL, "fields must be +-1");
  HIPCHK(h, hipMemcpyAsync(ws + p.fields, fields, n, hipMemcpyHostToDevice, s));
  if (targets) HIPCHK(h, hipMemcpyAsync(ws + p.targets, targets, sizeof(float) * n, hipMemcpyHostToDevice, s));
  return DQMC_OK;
}

uint64_t splitmix64(uint64_t& x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Scratch of the window (7-slice) training pass: batch items with up to
// ncm cells; host windows (n_host of them, rows of row sites) when given.
struct WinPlan {
  int ncm = 0, batch = 0, chunks = 0, lblocks = 0;
  size_t Ls = 0, wins = 0, tgs = 0, a0 = 0, h1 = 0, h2 = 0, z = 0, dz = 0, d2 = 0, d1 = 0, part = 0, partb = 0,
         lossp = 0, lossv = 0, total = 0;
};

WinPlan win_plan(int ncm, int batch, int n_host, int row) {
  WinPlan p;
  p.ncm = ncm; p.batch = batch;
  const size_t B = batch, c = ncm;
  p.chunks = wgrad_chunks(5, ncm, NET_VCH);
  p.lblocks = (ncm + 255) / 256;
  size_t o = 0;
  p.Ls = o; o = al(o + sizeof(int) * NET_MAXBATCH);
  p.wins = o; o = al(o + (size_t)n_host * 7 * row);
  p.tgs = o; o = al(o + sizeof(float) * (size_t)n_host * row);
  p.a0 = o; o = al(o + 2 * B * 7 * c * 16);
  p.h1 = o; o = al(o + 2 * B * 5 * c * 32);
  p.h2 = o; o = al(o + 2 * B * 3 * c * 32);
  p.z = o; o = al(o + 4 * B * c * 16);
  p.dz = o; o = al(o + 2 * B * c * 16);
  p.d2 = o; o = al(o + 2 * B * 3 * c * 32);
  p.d1 = o; o = al(o + 2 * B * 5 * c * 32);
  p.part = o; o = al(o + sizeof(float) * B * p.chunks * 27 * 32 * 32);
  p.partb = o; o = al(o + sizeof(float) * B * p.chunks * 32);
  p.lossp = o; o = al(o + sizeof(float) * B * p.lblocks);
  p.lossv = o; o = al(o + sizeof(float) * NET_LOSS_SLOTS);
  p.total = o;
  return p;
}

// Loss of the centre-slice logits of the windows in idx (and with backward
// the gradient into h->net_grad): valid-in-time convolutions 7 -> 5 -> 3 -> 1
// slices forward, transposed convolutions with zero time padding backward.
hipError_t net_window_pass(dqmc_ctx* h, const WinPlan& p, char* ws, const int8_t* wins, long long win_stride,
                           int row, const float* tgs, long long tg_stride, const BatchIdx& idx, bool backward,
                           int loss_slot, hipStream_t s) {
  const int c = p.ncm;
  const long long c16 = (long long)c * 16, c32 = (long long)c * 32;
  hipError_t e;
  auto ok = [&](hipError_t x) { e = x; return x == hipSuccess; };
  int* dLs = (int*)(ws + p.Ls);
  long long nsite = 0;
  for (int b = 0; b < idx.n; ++b) nsite += 2LL * idx.L[b] * idx.L[b];
  if (!ok(launch_batch_L(idx, dLs, s))) return e;
  if (!ok(launch_net_input_window(wins, win_stride, row, idx, dLs, c, ws + p.a0, s))) return e;
  ConvGeom g1{0, dLs, 7, 5, 1, 7 * c16, 5 * c32, 0};
  if (!ok(launch_conv(CONV_F1, ws + p.a0, ws + p.h1, h->netw, g1, idx.n, c, s))) return e;
  ConvGeom g2{0, dLs, 5, 3, 1, 5 * c32, 3 * c32, 0};
  if (!ok(launch_conv(CONV_F2, ws + p.h1, ws + p.h2, h->netw, g2, idx.n, c, s))) return e;
  ConvGeom g3{0, dLs, 3, 1, 1, 3 * c32, c16, 0};
  if (!ok(launch_conv(CONV_F3, ws + p.h2, ws + p.z, h->netw, g3, idx.n, c, s))) return e;
  float* lossv = (float*)(ws + p.lossv) + loss_slot;
  if (!ok(launch_net_loss_window((const float*)(ws + p.z), tgs, tg_stride, idx, dLs, c, (float)(1.0 / nsite),
                                 ws + p.dz, (float*)(ws + p.lossp), lossv, s)))
    return e;
  if (!backward) return hipSuccess;
  float* part = (float*)(ws + p.part);
  float* partb = (float*)(ws + p.partb);
  // layer 3: dW3 from (h2, dz); dh2 = conv^T(dz) over 3 slices
  ConvGeom w3{0, dLs, 3, 1, 1, 3 * c32, c16, 0};
  if (!ok(launch_wgrad(WGRAD_3, ws + p.h2, ws + p.dz, part, partb, w3, idx.n, c, NET_VCH, s))) return e;
  if (!ok(launch_wgrad_reduce(WGRAD_3, part, partb, idx.n * wgrad_chunks(1, c, NET_VCH), h->net_grad, s)))
    return e;
  ConvGeom b3{0, dLs, 1, 3, -1, c16, 3 * c32, 1};
  if (!ok(launch_conv(CONV_B3, ws + p.dz, ws + p.d2, h->netw, b3, idx.n, c, s))) return e;
  if (!ok(launch_tanh_back(ws + p.d2, ws + p.h2, (size_t)idx.n * 3 * c32, s))) return e;
  // layer 2
  ConvGeom w2{0, dLs, 5, 3, 1, 5 * c32, 3 * c32, 0};
  if (!ok(launch_wgrad(WGRAD_2, ws + p.h1, ws + p.d2, part, partb, w2, idx.n, c, NET_VCH, s))) return e;
  if (!ok(launch_wgrad_reduce(WGRAD_2, part, partb, idx.n * wgrad_chunks(3, c, NET_VCH), h->net_grad, s)))
    return e;
  ConvGeom b2{0, dLs, 3, 5, -1, 3 * c32, 5 * c32, 1};
  if (!ok(launch_conv(CONV_B2, ws + p.d2, ws + p.d1, h->netw, b2, idx.n, c, s))) return e;
  if (!ok(launch_tanh_back(ws + p.d1, ws + p.h1, (size_t)idx.n * 5 * c32, s))) return e;
  // layer 1
  ConvGeom w1{0, dLs, 7, 5, 1, 7 * c16, 5 * c32, 0};
  if (!ok(launch_wgrad(WGRAD_1, ws + p.a0, ws + p.d1, part, partb, w1, idx.n, c, NET_VCH, s))) return e;
  return launch_wgrad_reduce(WGRAD_1, part, partb, idx.n * wgrad_chunks(5, c, NET_VCH), h->net_grad, s);
}

// Ring slots holding a sample: instance i writes slots i, i + n, ...
int64_t ring_filled(dqmc_ctx* h, dqmc_status& st) {
  int64_t cmin = -1;
  for (int i = 0; i < h->n; ++i) {
    InstState x;
    if (hipMemcpyAsync(&x, h->hd[i].st, sizeof(x), hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess) {
      st = DQMC_EHIP;
      return 0;
    }
    cmin = cmin < 0 ? x.collect_n : std::min(cmin, x.collect_n);
  }
  st = DQMC_OK;
  return std::min<int64_t>((int64_t)h->plan.ring_cap, std::max<int64_t>(cmin, 0) * h->n);
}

}  // namespace

extern "C" {

dqmc_status dqmc_net_workspace_size(int32_t L, int32_t M, int64_t n_samples, int32_t batch, size_t* bytes) {
  NetPlan p;
  if (!bytes || !net_plan(L, M, n_samples, batch, p)) return DQMC_EINVAL;
  size_t t = p.total;
  if (M == 7) t = std::max(t, win_plan(L * L, (int)std::max<int64_t>(n_samples, batch), (int)n_samples, 2 * L * L).total);
  *bytes = t;
  return DQMC_OK;
}

dqmc_status dqmc_net_logits(dqmc_handle h, void* dev_ws, size_t bytes, const int8_t* host_fields, int32_t n,
                            int32_t L, int32_t M, float* host_out) {
  NetPlan p;
  if (!h || !dev_ws || !host_fields || !host_out || !net_plan(L, M, n, n, p)) return DQMC_EINVAL;
  if (((uintptr_t)dev_ws) & 255) return DQMC_EINVAL;
  if (bytes < p.total) return DQMC_ENOMEM;
  hipStream_t s = h->stream;
  char* ws = (char*)dev_ws;
  dqmc_status st = net_upload(h, p, ws, host_fields, nullptr, s);
  if (st != DQMC_OK) return st;
  BatchIdx idx{};
  idx.n = n;
  for (int b = 0; b < n; ++b) idx.idx[b] = b;
  HIPCHK(h, net_pass(h, p, ws, idx, false, false, 0, s));
  float* out = (float*)(ws + p.targets);   // reuse the target area for the logits
  HIPCHK(h, launch_net_logits_out((const float*)(ws + p.z), idx, p.N, p.Nc, M, out, s));
  HIPCHK(h, hipMemcpyAsync(host_out, out, sizeof(float) * (size_t)n * M * p.N, hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  return DQMC_OK;
}

dqmc_status dqmc_net_grad(dqmc_handle h, void* dev_ws, size_t bytes, const int8_t* host_fields,
                          const float* host_targets, int32_t n, int32_t L, int32_t M, int32_t window,
                          float* host_loss, float* host_grad) {
  NetPlan p;
  if (!h || !dev_ws || !host_fields || !host_targets || !net_plan(L, M, n, n, p)) return DQMC_EINVAL;
  if (window && M != 7) return fail(h, DQMC_EINVAL, "window samples have 7 slices");
  if (((uintptr_t)dev_ws) & 255) return DQMC_EINVAL;
  hipStream_t s = h->stream;
  char* ws = (char*)dev_ws;
  BatchIdx idx{};
  idx.n = n;
  for (int b = 0; b < n; ++b) idx.idx[b] = b;
  float* lossv = nullptr;
  if (!window) {
    if (bytes < p.total) return DQMC_ENOMEM;
    dqmc_status st = net_upload(h, p, ws, host_fields, host_targets, s);
    if (st != DQMC_OK) return st;
    HIPCHK(h, net_pass(h, p, ws, idx, true, true, 0, s));
    lossv = (float*)(ws + p.lossv);
  } else {
    const int N = 2 * L * L;
    WinPlan w = win_plan(L * L, n, n, N);
    if (bytes < w.total) return DQMC_ENOMEM;
    for (size_t i = 0; i < (size_t)n * 7 * N; ++i)
      if (host_fields[i] != 1 && host_fields[i] != -1) return fail(h, DQMC_EINVAL, "fields must be +-1");
    HIPCHK(h, hipMemcpyAsync(ws + w.wins, host_fields, (size_t)n * 7 * N, hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(ws + w.tgs, host_targets, sizeof(float) * (size_t)n * N, hipMemcpyHostToDevice, s));
    for (int b = 0; b < n; ++b) idx.L[b] = L;
    HIPCHK(h, net_window_pass(h, w, ws, (const int8_t*)(ws + w.wins), 7LL * N, N, (const float*)(ws + w.tgs), N,
                              idx, true, 0, s));
    lossv = (float*)(ws + w.lossv);
  }
  if (host_loss) HIPCHK(h, hipMemcpyAsync(host_loss, lossv, sizeof(float), hipMemcpyDeviceToHost, s));
  if (host_grad)
    HIPCHK(h, hipMemcpyAsync(host_grad, h->net_grad, sizeof(float) * NET_NPARAM, hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  return DQMC_OK;
}

dqmc_status dqmc_collect(dqmc_handle h, int32_t every) {
  if (!h || every < 0) return DQMC_EINVAL;
  h->collect_every = every;
  return DQMC_OK;
}

dqmc_status dqmc_sample_count(dqmc_handle h, int64_t* filled, int64_t* capacity) {
  if (!h) return DQMC_EINVAL;
  dqmc_status st;
  int64_t f = ring_filled(h, st);
  if (st != DQMC_OK) return fail(h, st, "sample_count");
  if (filled) *filled = f;
  if (capacity) *capacity = h->plan.ring_cap;
  return DQMC_OK;
}

dqmc_status dqmc_get_samples(dqmc_handle h, int64_t first, int32_t count, int8_t* host_win, float* host_tg) {
  if (!h || first < 0 || count < 0 || first + count > h->plan.ring_cap || !host_win || !host_tg)
    return DQMC_EINVAL;
  const size_t nm = (size_t)h->Nmax;
  HIPCHK(h, hipMemcpyAsync(host_win, h->ws + h->plan.ring_win + (size_t)first * 7 * nm, (size_t)count * 7 * nm,
                           hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipMemcpyAsync(host_tg, h->ws + h->plan.ring_tg + sizeof(float) * (size_t)first * nm,
                           sizeof(float) * (size_t)count * nm, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return DQMC_OK;
}

dqmc_status dqmc_net_train_workspace_size(dqmc_handle h, int32_t batch, size_t* bytes) {
  if (!h || !bytes || batch < 1 || batch > NET_MAXBATCH) return DQMC_EINVAL;
  *bytes = win_plan(h->Nmax / 2, batch, 0, 0).total;
  return DQMC_OK;
}

dqmc_status dqmc_net_train(dqmc_handle h, void* dev_ws, size_t bytes, int32_t steps, int32_t batch, float lr,
                           uint64_t seed, float* host_loss) {
  if (!h || !dev_ws || steps < 0 || !(lr > 0.f) || batch < 1 || batch > NET_MAXBATCH) return DQMC_EINVAL;
  if (((uintptr_t)dev_ws) & 255) return DQMC_EINVAL;
  WinPlan w = win_plan(h->Nmax / 2, batch, 0, 0);
  if (bytes < w.total) return DQMC_ENOMEM;
  dqmc_status st;
  const int64_t filled = ring_filled(h, st);
  if (st != DQMC_OK) return fail(h, st, "net_train");
  if (filled < 1) return fail(h, DQMC_ESTATE, "no training samples collected");
  hipStream_t s = h->stream;
  char* ws = (char*)dev_ws;
  const int8_t* wins = (const int8_t*)(h->ws + h->plan.ring_win);
  const float* tgs = (const float*)(h->ws + h->plan.ring_tg);
  uint64_t rs = seed;
  for (int k = 0; k < steps; ++k) {
    BatchIdx idx{};
    idx.n = batch;
    for (int b = 0; b < batch; ++b) {
      idx.idx[b] = (int)(splitmix64(rs) % (uint64_t)filled);
      idx.L[b] = h->hd[idx.idx[b] % h->n].L;
    }
    const int slot = k % NET_LOSS_SLOTS;
    HIPCHK(h, net_window_pass(h, w, ws, wins, 7LL * h->Nmax, h->Nmax, tgs, h->Nmax, idx, true, slot, s));
    HIPCHK(h, launch_adam(h->net_master, h->net_grad, h->net_m, h->net_v, NET_NPARAM, lr, ++h->adam_step, s));
    HIPCHK(h, launch_net_prep(h->net_master, h->netw, s));
    if (host_loss && (slot == NET_LOSS_SLOTS - 1 || k == steps - 1)) {
      const int first = k - slot;
      HIPCHK(h, hipMemcpyAsync(host_loss + first, ws + w.lossv, sizeof(float) * (slot + 1), hipMemcpyDeviceToHost, s));
      HIPCHK(h, hipStreamSynchronize(s));
    }
  }
  HIPCHK(h, hipStreamSynchronize(s));
  return DQMC_OK;
}

}  // extern "C"

// ---- Allocation-free network inference --------------------------------------------------
// dqmc_net_logits_noalloc runs the same kernels as dqmc_net_logits with the
// forward scratch (fields, activations, logits) in this file-scope device
// array instead of a caller workspace.  Each GPU holds its own copy, whose
// address is looked up once per device; every call on a device shares it.
namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(16) << 20;   // 16 MiB
static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {nullptr};

// Device address of `scratch` on the current device (looked up on the first
// call on that device).
hipError_t scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// Forward-only layout of n configurations of size (L, M) in the scratch:
// the inputs, the logits and the activations of net_pass without a loss.
bool net_plan_forward(int L, int M, int n, NetPlan& p) {
  if (L < 2 || L > 45 || M < 1 || n < 1 || n > NET_MAXBATCH) return false;
  p = NetPlan();
  p.L = L; p.M = M; p.Nc = L * L; p.N = 2 * p.Nc; p.batch = n; p.n_samples = n;
  const size_t vox = (size_t)M * p.Nc, B = n;
  size_t o = 0;
  p.fields = o; o = al(o + B * M * p.N);
  p.targets = o; o = al(o + sizeof(float) * B * M * p.N);   // logits out
  p.a0 = o; o = al(o + 2 * B * vox * 16);
  p.h1 = o; o = al(o + 2 * B * vox * 32);
  p.h2 = o; o = al(o + 2 * B * vox * 32);
  p.z = o; o = al(o + 4 * B * vox * 16);
  p.total = o;
  return true;
}

}  // namespace

extern "C" dqmc_status dqmc_net_logits_noalloc(dqmc_handle h, const int8_t* host_fields, int32_t n, int32_t L,
                                               int32_t M, float* host_out) {
  NetPlan p;
  if (!h || !host_fields || !host_out || !net_plan_forward(L, M, n, p)) return DQMC_EINVAL;
  if (p.total > NOALLOC_SCRATCH_BYTES)
    return fail(h, DQMC_EUNSUPPORTED, "net_logits_noalloc: " + std::to_string(p.total) +
                                          " bytes of scratch needed, the static scratch holds " +
                                          std::to_string(NOALLOC_SCRATCH_BYTES));
  int dev = -1;
  HIPCHK(h, hipGetDevice(&dev));
  if (dev != h->device) return fail(h, DQMC_ESTATE, "net_logits_noalloc: current device is not the handle's");
  void* base = nullptr;
  HIPCHK(h, scratch_address(dev, &base));
  hipStream_t s = h->stream;
  char* ws = (char*)base;
  dqmc_status st = net_upload(h, p, ws, host_fields, nullptr, s);
  if (st != DQMC_OK) return st;
  BatchIdx idx{};
  idx.n = n;
  for (int b = 0; b < n; ++b) idx.idx[b] = b;
  HIPCHK(h, net_pass(h, p, ws, idx, false, false, 0, s));
  float* out = (float*)(ws + p.targets);
  HIPCHK(h, launch_net_logits_out((const float*)(ws + p.z), idx, p.N, p.Nc, M, out, s));
  HIPCHK(h, hipMemcpyAsync(host_out, out, sizeof(float) * (size_t)n * M * p.N, hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  return DQMC_OK;
}
