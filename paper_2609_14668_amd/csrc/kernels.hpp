// Kernel launch interfaces shared by the engine.  All kernels take the
// device array of instance descriptors and work on blockIdx.y = instance.
#pragma once
#include "common.hpp"

// ---- FFT propagation -----------------------------------------------------------------
// FOP_STAB_CHAIN: all n_stab B's of one chain step applied to the columns of
// the working U in one pass (resolved per step as FOP_STAB_B with j = 0 ..
// n_stab - 1), the columns scaled by the working D on the way out.
// FOP_FOURIER: only the forward 2-D DFT of each sublattice (columns: M <- F M,
// rows: M <- M F^dagger), for the momentum-resolved estimators.
enum FftOp : int { FOP_WRAP_PRE = 0, FOP_WRAP_POST, FOP_STAB_B, FOP_HALF, FOP_EXPLICIT, FOP_STAB_CHAIN,
                   FOP_FOURIER };
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
// tiles (nullable): register-line tile per (L index q, side) at tiles[2 q + side]
// (0 wide, 1 narrow, 2 eight vectors per workgroup; L <= 24 in FP64)
constexpr int FFT_TILES = 3;
hipError_t launch_fft(const InstDev* insts, int n_inst, int Nmax, bool cplx_, const FftArgs& a,
                      size_t lds_budget, int rmax, const int* Ls, int nL, bool any_generic, bool single,
                      const int* tiles, hipStream_t s);

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
  GF_NC_MW = 64,       // NC = min(NC, the instance's accepts in the last window); skip if none
};
hipError_t launch_gemm(const InstDev* insts, int n_inst, int Nmax, bool cplx_, GemmOperand A,
                       GemmOperand B, GemmOperand C, GemmDim M, GemmDim Nn, GemmDim K,
                       double alpha, double beta, int flags, hipStream_t s);

// Flush G <- G - X[:, :fill] Y[:fill, :] straight from memory (no LDS);
// flags: GF_IF_FULL or GF_IF_ANY.  single: the product X Y is formed with
// FP32 MFMA (operands rounded to float) and subtracted from the FP64 G.
hipError_t launch_flush_direct(const InstDev* insts, int n_inst, int Nmax, bool cplx_, bool single, int flags,
                               hipStream_t s);

// Flush from device work queues with n_wg persistent workgroups (rounded to a
// multiple of the queue count); the queue counters live in the InstState of
// insts[0], so concurrent launches must start at different instances.
hipError_t launch_flush_queue(const InstDev* insts, int n_inst, bool cplx_, int flags, int n_wg, hipStream_t s);

// ---- delayed update -------------------------------------------------------------------
hipError_t launch_window(const InstDev* insts, int n_inst, bool cplx_, int W, int replay,
                         hipStream_t s);
hipError_t launch_expand(const InstDev* insts, int n_inst, int Nmax, bool cplx_, int kcap_max,
                         hipStream_t s);
// Submatrix update of the last window: M~ = P Delta_S (1 + (1 - G)_SS Delta_S)^{-1}
// into W2 (rows at the window positions of the accepted sites) and the rows
// (1 - G)[S, :] into Y; X = G[:, window] M~ is a GEMM with GF_NC_MW.
hipError_t launch_submatrix_coef(const InstDev* insts, int n_inst, bool cplx_, hipStream_t s);
hipError_t launch_submatrix_rows(const InstDev* insts, int n_inst, int Nmax, bool cplx_, hipStream_t s);
// The delayed vectors of the last window in matrix form (coefficients, then
// MFMA tile products; uses W1, W2, W3 and QA as scratch), and the fill bump.
hipError_t launch_expand_mm(const InstDev* insts, int n_inst, int Nmax, bool cplx_, hipStream_t s);
hipError_t launch_bump(const InstDev* insts, int n_inst, hipStream_t s);
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
  EO_BUILD_RHS,       // c = D_Rb^-1 U_R^H (v = 1: rows in the LU's row order)
  EO_SCALE_ROWS_DLB,  // c[i, :] /= max(D_L[i], 1)
  EO_STACK_STORE,     // stack slot <- working chain (interior checkpoints only)
  EO_STACK_IDENTITY,  // every stack slot <- identity chain
  EO_DRIFT_REPLACE,   // drift = max |G - GS|; G <- GS
  EO_RESET_CHAIN,     // working chain <- identity at the first checkpoint of a pass
  EO_SET_ONES,        // vec v <- 1
  // time-displaced pass
  EO_TAU_INIT,        // G(0,0), G(0,0), G(0,0) - 1 into MAT_GTT, MAT_GT0, MAT_G0T
  EO_SCALE_ROWS_DL,   // c[i, :] *= D_L[i]
  EO_BUILD_RHS_T,     // c = D_Rs T_R with rows in the LU's row order (row i from row perm[N + i])
  EO_TAU_REPLACE,     // drift = max of |GTT - GS|, |GT0 - W2|, |G0T - W1|; then replaced by them
};
struct ElemArgs { int op, a, b, c, v; };
hipError_t launch_elem(const InstDev* insts, int n_inst, int Nmax, bool cplx_, ElemArgs e, hipStream_t s);
hipError_t launch_colnorm_sort(const InstDev* insts, int n_inst, int Nmax, bool cplx_, int mat, hipStream_t s);

// 16-column panel held in registers (rows per thread chosen from Nmax)
hipError_t launch_qr_panel_reg(const InstDev* insts, int n_inst, int Nmax, bool cplx_, int p, hipStream_t s);
// target <- (I - V op(T) V^H) target for panel p; cols 0: trailing [j0+16, N),
// 1: [j0, N), 2: all; use_th: op(T) = T^H (apply Q^H) else T (apply Q).
// Pairs of panels (32 reflectors): combined compact-WY factor, and the
// block-reflector update with it (cols 0: [j0+32, N), 1: [j0, N), 2: all).
hipError_t launch_pair_t(const InstDev* insts, int n_inst, bool cplx_, int q, hipStream_t s);
hipError_t launch_apply_refl2(const InstDev* insts, int n_inst, int Nmax, bool cplx_, int q, int target, int cols,
                              int use_th, hipStream_t s);
hipError_t launch_apply_refl(const InstDev* insts, int n_inst, int Nmax, bool cplx_, int p, int target, int cols,
                             int use_th, hipStream_t s);
// drift of the recomputation just made: drift_last, drift_max, tolerance check
hipError_t launch_stab_finish(const InstDev* insts, int n_inst, hipStream_t s);
// phase of det U of the chain step (mode 0) / anchored phase of det(1 + B..B) (mode 1)
hipError_t launch_detphase(const InstDev* insts, int n_inst, bool cplx_, int mode, hipStream_t s);
// LU with partial pivoting of MAT_QA: leaf panel of columns [c0, c0 + nbw)
// (nbw <= 16, pivots to perm), its interchanges on the rest of MAT_QA and on
// MAT_W3, and the unit lower-triangular block solve (nb <= 32 rows from r0)
// on columns [col0, col1) of a target with L from MAT_QA.
constexpr int LU_NB = 16, TL_NB = 32;
hipError_t launch_lu_panel(const InstDev* insts, int n_inst, int Nmax, bool cplx_, int c0, int nbw, hipStream_t s);
hipError_t launch_lu_swap(const InstDev* insts, int n_inst, int Nmax, bool cplx_, int c0, int nbw, hipStream_t s);
hipError_t launch_trsm_lower(const InstDev* insts, int n_inst, bool cplx_, int r0, int nb, int col0, int col1,
                             int target, hipStream_t s);
hipError_t launch_diag_abs(const InstDev* insts, int n_inst, int Nmax, bool cplx_, hipStream_t s);
hipError_t launch_trsm_diag(const InstDev* insts, int n_inst, int Nmax, bool cplx_, int blk, hipStream_t s);
hipError_t launch_measure(const InstDev* insts, int n_inst, int Nmax, bool cplx_, int mat, hipStream_t s);
// momentum distribution sums from the forward-transformed G in mat
// time-displaced pass: instance state (mode 0 begin, 1 slice l, 2 end) and
// the estimator of slice l from MAT_GTT, MAT_GT0, MAT_G0T and MAT_G
hipError_t launch_tau_state(const InstDev* insts, int n_inst, int mode, int l, int lmax_req, hipStream_t s);
hipError_t launch_measure_tau(const InstDev* insts, int n_inst, int Nmax, bool cplx_, int l, hipStream_t s);
hipError_t launch_measure_k(const InstDev* insts, int n_inst, int Nmax, bool cplx_, int mat, hipStream_t s);

// ---- proposal network (BF16 operands, FP32 accumulation) ---------------------------
// Flat FP32 parameters: W1 [27][32][2], b1 [32], W2 [27][32][32], b2 [32],
// W3 [27][2][32], b3 [2]; tap (dt+1)*9 + (d2+1)*3 + (d1+1) reads (t+dt, n2+d2, n1+d1).
constexpr int NET_CH = 32;
constexpr int NET_OFF_W1 = 0;
constexpr int NET_OFF_B1 = NET_OFF_W1 + 27 * NET_CH * 2;
constexpr int NET_OFF_W2 = NET_OFF_B1 + NET_CH;
constexpr int NET_OFF_B2 = NET_OFF_W2 + 27 * NET_CH * NET_CH;
constexpr int NET_OFF_W3 = NET_OFF_B2 + NET_CH;
constexpr int NET_OFF_B3 = NET_OFF_W3 + 27 * 2 * NET_CH;
constexpr int NET_NPARAM = NET_OFF_B3 + 2;
// Device copies of the weights in the layouts the convolutions read:
// forward [27][out][in] with the 2-channel ends padded to 16, backward-data
// [27][in of the layer][out of the layer] with the taps mirrored.
struct NetW {
  void* w1f;   // bf16 [27][32][16]
  void* w2f;   // bf16 [27][32][32]
  void* w3f;   // bf16 [27][16][32]
  void* w2b;   // bf16 [27][32][32]
  void* w3b;   // bf16 [27][32][16]
  float* b1;   // [32]
  float* b2;   // [32]
  float* b3;   // [16]
};
constexpr size_t NET_WBYTES = 2 * (27 * 32 * 16 + 27 * 32 * 32 + 27 * 16 * 32 + 27 * 32 * 32 + 27 * 32 * 16) +
                              4 * (32 + 32 + 16);
// Grid geometry of a convolution over items (configurations or windows):
// output slice t reads input slices t + toff - 1 .. t + toff + 1 (mod T_in).
struct ConvGeom {
  int Lu;             // cells per side when Ls is null
  const int* Ls;      // per-item L (device), nullable
  int T_in, T_out, toff;
  long long in_stride, out_stride;   // elements between items
  int tzero;          // 1: input slices outside [0, T_in) read as zero instead of wrapping
};
enum ConvKind : int { CONV_F1 = 0, CONV_F2, CONV_F3, CONV_B3, CONV_B2 };
enum WgradKind : int { WGRAD_1 = 0, WGRAD_2, WGRAD_3 };
constexpr int NET_MAXBATCH = 64;
struct BatchIdx { int n; int idx[NET_MAXBATCH]; int L[NET_MAXBATCH]; };
// device copy of idx.L (stream-ordered, from the kernel arguments)
hipError_t launch_batch_L(const BatchIdx& idx, int* dLs, hipStream_t s);

hipError_t launch_net_prep(const float* master, NetW w, hipStream_t s);
hipError_t launch_conv(int kind, const void* in, void* out, NetW w, ConvGeom g, int n_items, int max_nc,
                       hipStream_t s);
// Partial weight/bias gradients per chunk of vch output voxels; returns the
// number of chunks per item.
int wgrad_chunks(int T_out, int Nc, int vch);
hipError_t launch_wgrad(int kind, const void* in, const void* dout, float* part, float* partb, ConvGeom g,
                        int n_items, int max_nc, int vch, hipStream_t s);
hipError_t launch_wgrad_reduce(int kind, const float* part, const float* partb, int nchunks, float* grad,
                               hipStream_t s);
hipError_t launch_net_input(const int8_t* fields, int N, int Nc, int M, BatchIdx idx, void* a0, hipStream_t s);
hipError_t launch_net_loss(const float* z, const float* targets, BatchIdx idx, int N, int Nc, int M, void* dz,
                           float* lossp, float* loss_out, hipStream_t s);
hipError_t launch_net_logits_out(const float* z, BatchIdx idx, int N, int Nc, int M, float* out, hipStream_t s);
hipError_t launch_tanh_back(void* dh, const void* h, size_t n, hipStream_t s);
// 7-slice windows (int8, rows of row_stride sites, win_stride bytes per
// sample) -> channels-last input; per-item L on the device.
hipError_t launch_net_input_window(const int8_t* wins, long long win_stride, int row_stride, BatchIdx idx,
                                   const int* Ls, int nc_max, void* a0, hipStream_t s);
// loss of the centre-slice logits (z: [item][nc_max][16]) against targets
// (tg_stride floats per sample, site order A then B); inv_count = 1 / sum N.
hipError_t launch_net_loss_window(const float* z, const float* tgs, long long tg_stride, BatchIdx idx,
                                  const int* Ls, int nc_max, float inv_count, void* dz, float* lossp,
                                  float* loss_out, hipStream_t s);
// Training samples: every `every`-th slice l of the downward pass (l % every
// == 0), after the slice's single-site updates, each instance stores its
// window of slices l-3 .. l+3 and the targets of slice l in ring slot
// (count * n_total + inst) % ring_cap; insts points at instance `off`.
hipError_t launch_collect(const InstDev* insts, int n_inst, int off, int n_total, int8_t* ring_win, float* ring_tg,
                          int ring_cap, int n_max, int every, hipStream_t s);
hipError_t launch_adam(float* master, const float* g, float* m, float* v, int n, float lr, int step,
                       hipStream_t s);
// Sampler side: 7-slice input windows around the current slice (flip: with
// the sites of the move in flight reversed), proposal and decision.
hipError_t launch_learn_window(const InstDev* insts, int n_inst, int nc_max, int flip, hipStream_t s);
hipError_t launch_learn_propose(const InstDev* insts, int n_inst, bool cplx_, int move, int m, hipStream_t s);
hipError_t launch_learn_decide(const InstDev* insts, int n_inst, bool cplx_, int move, hipStream_t s);
// Window coefficient table (in units of the matrix element type): c_k at
// [0, WMAX), x_k at [WC_X + k WMAX + a], y_k at [WC_Y + k WMAX + b], Delta_k
// of the accepted flips at [WC_D + k].
constexpr int DQMC_WMAX = 64;
constexpr int DQMC_WC_X = DQMC_WMAX;
constexpr int DQMC_WC_Y = DQMC_WMAX + DQMC_WMAX * DQMC_WMAX;
constexpr int DQMC_WC_D = DQMC_WMAX + 2 * DQMC_WMAX * DQMC_WMAX;
constexpr int DQMC_WC_SIZE = 2 * DQMC_WMAX + 2 * DQMC_WMAX * DQMC_WMAX;
