// Shared device/host definitions for the DQMC hot path on gfx950.
//
// Scalars: the periodic (untwisted) path is real FP64; twisted instances are
// complex128 stored as interleaved (re, im) doubles.  Kernels are templated on
// the scalar type through the small traits below, so every kernel has one
// source for both cases.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define DQMC_HD __host__ __device__ __forceinline__

struct cplx {
  double x, y;
};

DQMC_HD cplx cmake(double a, double b) { cplx c; c.x = a; c.y = b; return c; }
DQMC_HD cplx operator+(cplx a, cplx b) { return cmake(a.x + b.x, a.y + b.y); }
DQMC_HD cplx operator-(cplx a, cplx b) { return cmake(a.x - b.x, a.y - b.y); }
DQMC_HD cplx operator-(cplx a) { return cmake(-a.x, -a.y); }
DQMC_HD cplx operator*(cplx a, cplx b) { return cmake(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
DQMC_HD cplx operator*(double s, cplx a) { return cmake(s * a.x, s * a.y); }
DQMC_HD cplx operator*(cplx a, double s) { return cmake(s * a.x, s * a.y); }
DQMC_HD cplx conjg(cplx a) { return cmake(a.x, -a.y); }
DQMC_HD double conjg(double a) { return a; }
DQMC_HD double absq(cplx a) { return a.x * a.x + a.y * a.y; }
DQMC_HD double absq(double a) { return a * a; }
DQMC_HD double real_part(cplx a) { return a.x; }
DQMC_HD double real_part(double a) { return a; }
DQMC_HD double imag_part(cplx a) { return a.y; }
DQMC_HD double imag_part(double) { return 0.0; }
DQMC_HD cplx cdiv(cplx a, cplx b) {
  double d = b.x * b.x + b.y * b.y;
  return cmake((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
DQMC_HD double cdiv(double a, double b) { return a / b; }

// Single-precision complex for the mixed-precision wrap (complex64 arithmetic).
struct cplxf {
  float x, y;
};
DQMC_HD cplxf cmakef(float a, float b) { cplxf c; c.x = a; c.y = b; return c; }
DQMC_HD cplxf operator+(cplxf a, cplxf b) { return cmakef(a.x + b.x, a.y + b.y); }
DQMC_HD cplxf operator-(cplxf a, cplxf b) { return cmakef(a.x - b.x, a.y - b.y); }
DQMC_HD cplxf operator-(cplxf a) { return cmakef(-a.x, -a.y); }
DQMC_HD cplxf operator*(cplxf a, cplxf b) { return cmakef(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
DQMC_HD cplxf operator*(float s, cplxf a) { return cmakef(s * a.x, s * a.y); }
DQMC_HD cplxf operator*(cplxf a, float s) { return cmakef(s * a.x, s * a.y); }
DQMC_HD cplxf conjg(cplxf a) { return cmakef(a.x, -a.y); }

// Complex type of a real precision: cx_of<double> = cplx, cx_of<float> = cplxf.
template <typename R> struct cx_of;
template <> struct cx_of<double> {
  typedef cplx type;
  static DQMC_HD cplx make(double a, double b) { return cmake(a, b); }
};
template <> struct cx_of<float> {
  typedef cplxf type;
  static DQMC_HD cplxf make(double a, double b) { return cmakef((float)a, (float)b); }
};

// Loads and stores through the global address space.  Pointers taken from
// the instance descriptors are generic; accesses through them compile to FLAT
// instructions, which also count against the LDS wait counter, so a wait for
// an LDS read would wait for every memory load still in flight.
typedef const __attribute__((address_space(1))) double* gdptr;
typedef __attribute__((address_space(1))) double* gdptr_w;
__device__ __forceinline__ double gld(const double* p) { return *(gdptr)p; }
__device__ __forceinline__ cplx gld(const cplx* p) {
  gdptr q = (gdptr)p;   // component loads: a struct load through the cast stays FLAT
  return cmake(q[0], q[1]);
}
__device__ __forceinline__ int32_t gldi(const int32_t* p) {
  return *(const __attribute__((address_space(1))) int32_t*)p;
}
__device__ __forceinline__ void gst(double* p, double v) { *(gdptr_w)p = v; }
__device__ __forceinline__ void gst(cplx* p, cplx v) {
  gdptr_w q = (gdptr_w)p;
  q[0] = v.x;
  q[1] = v.y;
}

template <typename S> struct ST;
template <> struct ST<double> {
  static constexpr bool is_complex = false;
  static DQMC_HD double zero() { return 0.0; }
  static DQMC_HD double one() { return 1.0; }
  static DQMC_HD double from_re(double a) { return a; }
};
template <> struct ST<cplx> {
  static constexpr bool is_complex = true;
  static DQMC_HD cplx zero() { return cmake(0.0, 0.0); }
  static DQMC_HD cplx one() { return cmake(1.0, 0.0); }
  static DQMC_HD cplx from_re(double a) { return cmake(a, 0.0); }
};

DQMC_HD double fma_s(double a, double b, double c) { return a * b + c; }
DQMC_HD cplx fma_s(cplx a, cplx b, cplx c) {
  return cmake(a.x * b.x - a.y * b.y + c.x, a.x * b.y + a.y * b.x + c.y);
}

// ---- named per-instance matrices -------------------------------------------------
// Every N x N matrix of an instance is column-major with leading dimension N.
enum MatId : int {
  MAT_G = 0,     // equal-time Green's function G (spin up)
  MAT_GS,        // scratch recomputation of G / measurement copy
  MAT_X,         // delayed-update columns x_m   (column m at X + m*N)
  MAT_Y,         // delayed-update rows y_m      (element y_m[j] at Y + m*N + j)
  MAT_UW,        // working UDV chain: U
  MAT_TW,        // working UDV chain: T
  MAT_QA,        // QR work matrix
  MAT_V,         // explicit Householder vectors of the current QR
  MAT_TB,        // compact-WY T blocks (panel p at rows p*nb.., cols 0..nb)
  MAT_W1,        // scratch
  MAT_W2,        // scratch
  MAT_W3,        // scratch
  MAT_SU,        // stack slot U (resolved from the checkpoint index)
  MAT_ST,        // stack slot T (resolved from the checkpoint index)
  MAT_GTT,       // time-displaced pass: G(tau, tau)
  MAT_GT0,       // time-displaced pass: G(tau, 0)
  MAT_G0T,       // time-displaced pass: G(0, tau)
  MAT_COUNT,
  // roles in G = (1 + R L)^{-1}: R = U_R D_R T_R, L^dagger = U_L D_L T_L.
  // Upward pass: R is the working chain, L the stack slot; downward: swapped.
  MAT_RU = 100, MAT_RT, MAT_LU, MAT_LT
};

enum VecId : int {
  VEC_DW = 0,    // working D
  VEC_SD,        // stack slot D
  VEC_TAU,       // Householder scalars
  VEC_NORM,      // column norms / scratch
  VEC_D2,        // scratch (new D)
  VEC_COUNT,
  VEC_RD = 100, VEC_LD
};

// Per-instance counters and schedule state, written by the kernels.
struct InstState {
  int32_t phase;        // step within the sweep, 0 .. 2M-1
  int32_t cursor;       // next site of the current slice
  int32_t fill;         // pending rank-1 terms in X, Y
  int32_t m_w;          // accepts in the last window
  int32_t init_mode;    // 1 while the initial stack is being built
  int32_t numeric_err;  // nonzero after a non-finite or zero ratio
  int64_t sweep;        // completed sweeps (RNG counter)
  int64_t replay_pos;   // next bit of the replay stream
  int64_t proposals, accepted, flushes, stabs, n_meas;
  double drift_max, drift_last;
  int32_t wstart, wlen;  // site range of the last window
  int32_t idle;          // 1: instance has finished its part of the initial stack build
  int32_t pad0;
  int64_t flush_rank_sum;  // sum of the ranks of all flushes
  int64_t series_base;   // sweep index at the last reset of the estimators
  int64_t learn_props, learn_acc;  // learned multi-site moves proposed / accepted
  int64_t collect_n;               // training samples stored by this instance
  // phase of det(1 + B_M .. B_1) of spin up: updated by r_up / |r_up| at every
  // accepted flip (by the phase of the block determinant for a multi-site
  // move) and re-anchored from the UDV factors at every recomputation
  double ph_re, ph_im;
  double phw_re, phw_im;           // phase of det U of the working UDV chain
  double ph_drift;                 // max |tracked - anchored| phase over recomputations
  double drift_acc;                // running max of the recomputation in progress
  // work queues of the queue flush kernel for launches whose first instance
  // this is: next ticket and finished workgroups per queue (reset to zero by
  // the last workgroup of each queue)
  int32_t fq_next[8], fq_done[8];
  // time-displaced pass: 1 while the instance takes part, the last slice it
  // measures (tau_lmax dtau), and its idle flag before the pass
  int32_t tau_active, tau_lmax, tau_saved_idle, pad1;
};
// numeric_err bits
constexpr int NUMERR_RATIO = 1;    // non-finite or zero acceptance ratio
constexpr int NUMERR_DRIFT = 2;    // drift max |G_wrap - G_scratch| above the tolerance

// One learned multi-site proposal in flight (at most LEARN_MMAX sites).
// Coefficient tables hold S-typed values (two doubles per complex entry).
constexpr int LEARN_MMAX = 8;
struct LearnState {
  int32_t S[LEARN_MMAX];                       // ordered sites
  int32_t m;                                   // sites in S
  int32_t valid;                               // 0: the block ratio was not usable
  double logq;                                 // log q(S | X)
  double R;                                    // block weight ratio R_S
  double ph[2];                                // phase of prod_k r_k (the block determinant of spin up)
  double c[LEARN_MMAX][2];                     // Delta_k / r_k
  double xw[LEARN_MMAX][LEARN_MMAX][2];        // x_k at S positions a > k
  double yw[LEARN_MMAX][LEARN_MMAX][2];        // y_k at S positions b > k
};

// Running sums of equal-time estimators.
enum ObsId : int {
  OBS_N = 0, OBS_D, OBS_EKIN, OBS_E, OBS_SZZ_G, OBS_SZZ_DK, OBS_M2, OBS_RM2_NUM,
  OBS_PHASE_RE, OBS_PHASE_IM, OBS_CHI, OBS_COUNT
};

// Rows of N elements in an instance's buffer for the partial products of a
// row-split block-reflector update (chunks x reflectors <= RSPLIT_ROWS).
constexpr int RSPLIT_ROWS = 256;

// Device-visible descriptor of one instance.
struct InstDev {
  int32_t L, N, Nc, M;
  int32_t n_stab, n_ckpt;   // n_ckpt = M / n_stab
  int32_t kflush;           // flush when fill >= kflush after a window
  int32_t kcap;             // capacity of X, Y (kflush + window)
  int32_t is_complex;
  int32_t sym_measure;
  int32_t fft_fixed;        // 1: a compile-time FFT plan exists for L
  int32_t mixed;            // 1: wraps and flushes in single precision
  double lam;               // HS coupling: lambda (spin channel) or alpha (charge channel)
  int channel;              // 0: HS-s^z, 1: HS-n
  double drift_tol;         // recomputation drift above this sets NUMERR_DRIFT
  double U, dtau, t;
  double theta1, theta2;
  uint64_t seed;
  char* mat[MAT_COUNT];     // base pointers (MAT_SU/MAT_ST unused: see stack)
  double* vec[VEC_COUNT];
  char* stackU;             // slot c at stackU + c*mat_bytes
  char* stackT;
  double* stackD;           // slot c at stackD + c*N
  double* stackPh;          // slot c: phase of det U at stackPh[2c], stackPh[2c+1]
  size_t mat_bytes;
  int8_t* fields;           // M x N, x_{l,i} at fields[(l-1)*N + i]
  const cplx* tab;          // 4 tables x Nc x (2x2): exp(-dtau h)/Nc, exp(+dtau h)/Nc, half steps
  const cplx* roots;        // L-th roots of unity exp(-2 pi i m / L)
  const int32_t* factors;   // radix list of L (terminated by 0)
  int32_t* perm;            // 2N: column permutation of the current QR, or the LU's
                            // interchanges; then the LU's composed row order of Y
  int32_t* acc_site;        // accepted sites: position in the window (or in S)
  int32_t* acc_gsite;       // accepted sites: site index
  float* targets;           // M x N single-flip acceptance after each decision (downward pass)
  LearnState* learn;        // learned move in flight
  void* lwin[3];            // bf16 activations of the proposal net: 7, 5, 3 slices around l
  float* zcur;              // logits of slice l at the current fields (Nc x 16)
  float* zprop;             // logits of slice l at the proposed fields
  double* wcoef;            // window: c_k, then x/y window vectors
  char* rsplit;             // row-split reflector updates: RSPLIT_ROWS x N partial products
  InstState* st;
  double* obs;              // running sums [OBS_COUNT]
  double* series;           // per-sweep means [max_series x OBS_COUNT]
  double* nk_sum;           // momentum distribution sums: Nc x 8 (AA, AB, BA, BB as re, im)
  int32_t max_series;
  // time-displaced estimators (lc = M/2): tau_sum[l] (l = 0 .. lc) sums of
  // <A(tau_l) A(0)>_X over passes, tau_sum[lc + 1 + l] sums of <A>_X(tau_l),
  // tau_sum[2 lc + 2] the number of passes; tau_rows holds the same values per
  // pass (row stride 2 lc + 2, tau_cap rows, the oldest overwritten)
  double* tau_sum;
  double* tau_rows;
  int32_t tau_cap;
  const uint8_t* replay_bits;  // nullable
  double* replay_ratio;        // nullable
  int64_t replay_len;
};

#define TAB_P 0   // exp(-dtau h(k)) / Nc
#define TAB_M 1   // exp(+dtau h(k)) / Nc
#define TAB_HP 2  // exp(-dtau h(k)/2) / Nc
#define TAB_HM 3  // exp(+dtau h(k)/2) / Nc

// Schedule helpers (identical on host and device).
// Up pass: phase p in [0, M): slice l = p + 1, wrap then update.
// Down pass: phase p in [M, 2M): slice l = 2M - p, update then wrap.
DQMC_HD int sched_is_up(int phase, int M) { return phase < M; }
DQMC_HD int sched_slice(int phase, int M) { return phase < M ? phase + 1 : 2 * M - phase; }
// Checkpoint index after the step (valid when (phase+1) % n_stab == 0):
// up pass: l / n_stab; down pass: (l - 1) / n_stab.
DQMC_HD int sched_ckpt(int phase, int M, int n_stab) {
  int l = sched_slice(phase, M);
  return phase < M ? l / n_stab : (l - 1) / n_stab;
}


// Workgroups are handed to the 8 XCDs (each with its own L2) round-robin in
// dispatch order.  Map the dispatch index so that all workgroups of an
// instance sit on one XCD: instance xcd + 8 q is served by the slots
// q * gx .. q * gx + gx - 1 of that XCD, and its operands stay in one L2
// instead of being fetched into all eight.  The grid's y extent is the
// instance count rounded up to a multiple of 8; slots past the last instance
// return.  Only the placement depends on the dispatch order, not the result.
// With fewer instances than XCDs the placement would leave XCDs idle, so the
// plain mapping (instance = blockIdx.y) is used and the grid is not padded.
constexpr int N_XCD = 8;
__host__ __device__ __forceinline__ int xcd_grid_y(int n_inst) {
  return n_inst >= N_XCD ? (n_inst + N_XCD - 1) / N_XCD * N_XCD : n_inst;
}
__device__ __forceinline__ void xcd_slot(int n_inst, int& inst, int& bx) {
  if (n_inst < N_XCD) {
    inst = blockIdx.y;
    bx = blockIdx.x;
    return;
  }
  const int gx = gridDim.x;
  const int lin = blockIdx.x + gx * blockIdx.y;
  const int xcd = lin % N_XCD, slot = lin / N_XCD;
  inst = xcd + N_XCD * (slot / gx);
  bx = slot % gx;
  if (inst >= n_inst) inst = -1;
}

// Base pointer of a named matrix; stack slots resolve to the checkpoint of the
// instance's current step.
__device__ __forceinline__ char* mat_ptr(const InstDev& d, int id) {
  if (id >= MAT_RU) {
    int up = sched_is_up(d.st->phase, d.M);
    int isR = (id == MAT_RU || id == MAT_RT), isU = (id == MAT_RU || id == MAT_LU);
    int working = up ? isR : !isR;
    id = working ? (isU ? MAT_UW : MAT_TW) : (isU ? MAT_SU : MAT_ST);
  }
  if (id == MAT_SU || id == MAT_ST) {
    int c = sched_ckpt(d.st->phase, d.M, d.n_stab);
    return (id == MAT_SU ? d.stackU : d.stackT) + (size_t)c * d.mat_bytes;
  }
  return d.mat[id];
}
__device__ __forceinline__ double* vec_ptr(const InstDev& d, int id) {
  if (id >= VEC_RD) {
    int up = sched_is_up(d.st->phase, d.M);
    int working = up ? (id == VEC_RD) : (id == VEC_LD);
    id = working ? VEC_DW : VEC_SD;
  }
  if (id == VEC_SD) {
    int c = sched_ckpt(d.st->phase, d.M, d.n_stab);
    return d.stackD + (size_t)c * d.N;
  }
  return d.vec[id];
}

template <typename S>
__device__ __forceinline__ S* matp(const InstDev& d, int id) { return reinterpret_cast<S*>(mat_ptr(d, id)); }
