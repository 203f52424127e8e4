// Kernel launch interfaces shared by the engine.  All kernels take the
// device array of instance descriptors and work on blockIdx.y = instance.
#pragma once
#include "common.hpp"

// ---- FFT propagation -----------------------------------------------------------------
enum FftOp : int { FOP_WRAP_PRE = 0, FOP_WRAP_POST, FOP_STAB_B, FOP_HALF, FOP_EXPLICIT };
struct FftArgs {
  int op;      // FftOp
  int side;    // 0: columns (left multiplication), 1: rows (right multiplication)
  int mat;     // MatId transformed in place
  int j;       // chunk position for FOP_STAB_B
  int ex_pre, ex_tab, ex_post, ex_slice;  // FOP_EXPLICIT: diagonal signs, table, slice
};
int fft_vectors_per_block(int N, size_t lds_budget, size_t elem_bytes);
// Ls: the distinct L with a compile-time plan among the instances;
// any_generic: some instance needs the runtime-plan kernel.
bool fft_has_fixed(int L);
hipError_t launch_fft(const InstDev* insts, int n_inst, int Nmax, bool cplx_, const FftArgs& a,
                      size_t lds_budget, int rmax, const int* Ls, int nL, bool any_generic, bool single,
                      hipStream_t s);

// ---- batched GEMM on named matrices (FP64 MFMA) --------------------------------------
// C = alpha * op(A) op(B) + beta * C for every instance.  Row/column offsets
// and sizes are (a * N + b) for the instance's N.
struct GemmOperand {
  int id;          // MatId
  int op;          // 0: N, 1: T, 2: C (conjugate transpose)
  int ra, rb;      // row offset = ra*N + rb
  int ca, cb;      // column offset = ca*N + cb
};
struct GemmDim { int a, b, hi; };  // value = min(a*N + b, hi); hi <= 0 means no cap
enum GemmFlags : int {
  GF_K_FILL = 1,       // K = the instance's pending fill
  GF_IF_FULL = 2,      // skip unless fill >= kflush
  GF_IF_ANY = 4,       // skip unless fill > 0
  GF_A_UPPER = 8,      // op(A) is upper triangular (entries below the diagonal read as 0)
  GF_SKIP_INIT = 16,   // skip while the initial stack is built
  GF_ONLY_INIT_END = 32,
};
hipError_t launch_gemm(const InstDev* insts, int n_inst, int Nmax, bool cplx_, GemmOperand A,
                       GemmOperand B, GemmOperand C, GemmDim M, GemmDim Nn, GemmDim K,
                       double alpha, double beta, int flags, hipStream_t s);

// Flush G <- G - X[:, :fill] Y[:fill, :] straight from memory (no LDS);
// flags: GF_IF_FULL or GF_IF_ANY.  single: the product X Y is formed with
// FP32 MFMA (operands rounded to float) and subtracted from the FP64 G.
hipError_t launch_flush_direct(const InstDev* insts, int n_inst, int Nmax, bool cplx_, bool single, int flags,
                               hipStream_t s);

// ---- delayed update -------------------------------------------------------------------
hipError_t launch_window(const InstDev* insts, int n_inst, bool cplx_, int W, int replay,
                         hipStream_t s);
hipError_t launch_expand(const InstDev* insts, int n_inst, int Nmax, bool cplx_, int kcap_max,
                         hipStream_t s);
hipError_t launch_flush_done(const InstDev* insts, int n_inst, int any, hipStream_t s);

// ---- schedule -------------------------------------------------------------------------
hipError_t launch_advance(const InstDev* insts, int n_inst, hipStream_t s);
// mode 1: enter the initial stack build (downward pass without updates);
// mode 0: start the first sweep.
hipError_t launch_init_state(const InstDev* insts, int n_inst, int mode, hipStream_t s);
hipError_t launch_replay_reset(const InstDev* insts, int n_inst, hipStream_t s);
hipError_t launch_reset_counters(const InstDev* insts, int n_inst, hipStream_t s);

// ---- stabilisation and measurement ------------------------------------------------------
enum ElemOp : int {
  EO_COPY = 0,        // mat c = mat a
  EO_IDENTITY,        // mat c = 1
  EO_SCALE_COLS,      // mat c[:, j] *= vec v[j]
  EO_SCALE_ROWS_INV,  // mat c[i, :] /= vec v[i]
  EO_GATHER_COLS,     // mat c[:, j] = mat a[:, perm[j]]
  EO_GATHER_ROWS,     // mat c[i, :] = mat a[perm[i], :]
  EO_BUILD_Y,         // c = D_Rb^-1 a D_Lb^-1 + D_Rs b D_Ls  (a = U_R^H U_L, b = T_R T_L^H)
  EO_BUILD_RHS,       // c = D_Rb^-1 U_R^H
  EO_SCALE_ROWS_DLB,  // c[i, :] /= max(D_L[i], 1)
  EO_STACK_STORE,     // stack slot <- working chain (interior checkpoints only)
  EO_STACK_IDENTITY,  // every stack slot <- identity chain
  EO_DRIFT_REPLACE,   // drift = max |G - GS|; G <- GS
  EO_RESET_CHAIN,     // working chain <- identity at the first checkpoint of a pass
  EO_SET_ONES,        // vec v <- 1
};
struct ElemArgs { int op, a, b, c, v; };
hipError_t launch_elem(const InstDev* insts, int n_inst, int Nmax, bool cplx_, ElemArgs e, hipStream_t s);
hipError_t launch_colnorm_sort(const InstDev* insts, int n_inst, int Nmax, bool cplx_, int mat, hipStream_t s);
hipError_t launch_qr_panel(const InstDev* insts, int n_inst, bool cplx_, int p, int nb, hipStream_t s);
// 16-column panel held in registers (rows per thread chosen from Nmax)
hipError_t launch_qr_panel_reg(const InstDev* insts, int n_inst, int Nmax, bool cplx_, int p, hipStream_t s);
// target <- (I - V op(T) V^H) target for panel p; cols 0: trailing [j0+16, N),
// 1: [j0, N), 2: all; use_th: op(T) = T^H (apply Q^H) else T (apply Q).
hipError_t launch_apply_refl(const InstDev* insts, int n_inst, int Nmax, bool cplx_, int p, int target, int cols,
                             int use_th, hipStream_t s);
hipError_t launch_diag_abs(const InstDev* insts, int n_inst, int Nmax, bool cplx_, hipStream_t s);
hipError_t launch_trsm_diag(const InstDev* insts, int n_inst, int Nmax, bool cplx_, int blk, hipStream_t s);
hipError_t launch_measure(const InstDev* insts, int n_inst, int Nmax, bool cplx_, int mat, hipStream_t s);
