/*
 * dqmc.h -- C ABI of the MI355X DQMC sweep library (libdqmc.so).
 *
 * Finite-temperature determinant QMC for the half-filled honeycomb Hubbard
 * model, H = -t sum_<ij>s (c^+_is c_js + h.c.) + U sum_i (n_iu n_id - (n_iu + n_id)/2)
 * (Sec. II A, eq. HubbModel), with the Hubbard-Stratonovich transformation in
 * the spin-s^z channel, cosh(lambda) = exp(dtau U / 2) (eqs. SzHS, coupling),
 * or per instance in the charge channel (eq. DensityHS; dqmc_channel).
 * One call of dqmc_sweep runs the paper's Monte Carlo sweep (Sec. III): an
 * upward pass l = 1..M (wrap G, then update slice l) and a downward pass
 * l = M..1 (update slice l, then wrap), with
 *   - FFT propagation of exp(-+dtau K) with a 2x2 sublattice block per
 *     momentum (Sec. III A, eqs. NewBlMat, ExpLambda, FourierMat, ColumnDem),
 *   - delayed-update Metropolis on G (Sec. III B, eqs. DRatio, DelayRatio,
 *     DelayRgenk, FinalDelay),
 *   - periodic QR/UDV recomputation of G = (1 + R L)^{-1} (Sec. II B, eq.
 *     GrFMat) every n_stab slices, where the equal-time estimators are taken.
 * Twisted boundary conditions enter as the shifted momentum grid of eq.
 * kpoints (Sec. III C); Gauge-I phases.  Convention: the hop A(r) -> B(r+d)
 * carries exp(+i A.d); the opposite sign is Theta -> -Theta (complex
 * conjugation of G) and leaves weights and real observables unchanged.
 *
 * Conventions of the data exchanged through this interface:
 *   sites      A sublattice 0..Nc-1, B sublattice Nc..N-1, Nc = L*L,
 *              cell index n1 + L*n2 (positions n1 a1 + n2 a2);
 *   G          G_ij = <c_i c_j^+> of spin up at the current imaginary time,
 *              returned row-major N x N; real doubles for untwisted
 *              instances, interleaved (re, im) doubles for twisted ones;
 *   fields     int8 x_{l,i} = +-1, row-major M x N (slice l = 1..M is row l-1);
 *   RNG        u = Philox4x32-10(counter = (site, slice, sweep, pass),
 *              key = (seed & 0xffffffff, seed >> 32)) mapped to
 *              (w0 * 2^21 + (w1 >> 11)) * 2^-53; accept iff u < R, with
 *              R = r_up r_dn = exp(2 lambda x) |r_up|^2.
 *
 * Ownership: the caller owns the device workspace (dqmc_workspace_size bytes,
 * 256-byte aligned) and every buffer passed in; the library allocates no
 * device memory.  Host pointers are caller-allocated.  A handle is owned by
 * the library until dqmc_destroy.  Calls on one handle are not thread-safe;
 * distinct handles are independent.  Streams are hipStream_t passed as void*;
 * NULL selects the handle's stream.
 *
 * Errors: every call returns a dqmc_status; nothing is thrown.  Argument
 * errors return without side effects.  DQMC_ENUMERIC reports, from
 * dqmc_measure and dqmc_get_stats (which still fill their output), that the
 * device saw a non-finite or zero acceptance ratio or a recomputation whose
 * drift max |G_wrap - G_scratch| exceeded the tolerance (dqmc_set_drift_tol);
 * dqmc_stats.numeric_err says which (bit 1 ratio, bit 2 drift).  The handle
 * remains usable.  dqmc_last_error gives a message.
 */
#ifndef DQMC_H
#define DQMC_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dqmc_ctx* dqmc_handle;

typedef enum {
  DQMC_OK = 0,
  DQMC_EINVAL = -1,       /* invalid argument */
  DQMC_ENOMEM = -2,       /* workspace too small */
  DQMC_EHIP = -3,         /* a HIP runtime call failed */
  DQMC_ENUMERIC = -4,     /* non-finite or zero ratio */
  DQMC_ESTATE = -5,       /* call not valid in the current state */
  DQMC_EUNSUPPORTED = -6  /* size or option not supported */
} dqmc_status;

/* DQMC_FP64: every step in double precision.  DQMC_MIXED: the wraps run the
 * FFT in complex64 and the flushes form X Y with FP32 matrix cores (operands
 * rounded to float, FP32 accumulation); G stays stored in FP64, and the
 * acceptance ratios, the delayed-vector builder, the QR stabilisation and the
 * estimators stay FP64.  DQMC_MIXED_FLUSH: only the flushes in FP32;
 * DQMC_MIXED_WRAP: only the wraps in complex64.  The accumulated
 * single-precision error is reported as the drift max |G_wrap - G_scratch|
 * at each recomputation (dqmc_stats) and checked against the drift
 * tolerance (dqmc_set_drift_tol). */
typedef enum { DQMC_FP64 = 0, DQMC_MIXED = 1, DQMC_MIXED_FLUSH = 2, DQMC_MIXED_WRAP = 3 } dqmc_precision;

/* Hubbard-Stratonovich channel of an instance (Sec. II B).  DQMC_HS_SPIN
 * (eq. SzHS): B^sigma = exp(+-lambda diag(x)) exp(-dtau K), lambda =
 * arccosh(exp(dtau U/2)), uniform P(X); real arithmetic without a twist.
 * DQMC_HS_CHARGE (eq. DensityHS, eq. BIOpnT): B = exp(i alpha diag(x))
 * exp(-dtau K) for both spins, alpha = arccos(exp(-dtau U/2)) (gamma_c =
 * i alpha, eq. coupling), P(X) carrying exp(-gamma_c sum x); the flip ratio
 * is R = exp(2 i alpha x) r_up^2, real and positive by the partial
 * particle-hole symmetry, and G_dn = G_up.  The charge channel always runs
 * in complex arithmetic; learned proposals support the spin channel only. */
typedef enum { DQMC_HS_SPIN = 0, DQMC_HS_CHARGE = 1 } dqmc_channel;

/* One Markov chain.  All instances of a handle share n_stab, and every
 * beta/dtau must be a multiple of n_stab.  L in [2, 45] with prime factors in
 * {2, 3, 5, 7, 11, 13}. */
typedef struct {
  int32_t L;            /* unit cells per side */
  double t, U;          /* hopping and Hubbard U */
  double beta, dtau;    /* M = beta/dtau must be an integer within 1e-9 */
  double theta1, theta2;/* twist Theta_1, Theta_2 in radians along a1, a2; both 0 = periodic (real path) */
  int32_t n_delay;      /* flush rank k: flush once at least k accepted flips are pending, 1 <= k <= 192
                         * (retunable later with dqmc_set_delay / dqmc_autotune) */
  int32_t n_stab;       /* slices between recomputations of G (stabilisation) */
  int32_t precision;    /* dqmc_precision, the same for all instances of a handle */
  int32_t sym_measure;  /* 1: estimators on exp(-dtau K/2) G exp(+dtau K/2) */
  uint64_t seed;        /* Philox key */
  int32_t channel;      /* dqmc_channel: Hubbard-Stratonovich channel */
} dqmc_instance_desc;

/* Equal-time estimators (Sec. II C, Sec. IV C), means over all measurements
 * since creation or the last dqmc_reset_obs.  A measurement is taken on the
 * recomputed G at every stabilisation point of both passes (on
 * exp(-dtau K/2) G exp(+dtau K/2) for sym_measure = 1, the symmetric Trotter
 * split of Sec. II B), by Wick's theorem from G_up and G_dn = P (1 - G_up^dagger) P:
 *   n       <n_up + n_dn> per site (1 at half filling);
 *   D       double occupancy (1/N_s) sum_i <n_i,up n_i,dn>;
 *   ekin    <H_0> / N_s;  e = ekin + U D, the energy per site of Sec. IV C;
 *   Szz_G, Szz_dk  S_zz(k) of eq. SpinStrucF at k = 0 and k = b1/L, built from
 *           the intra-sublattice correlation C_zz(r) of eq. SzSzCrF;
 *   m2      S_zz(Gamma) / (2 N_c);
 *   Rm2     1 - Szz_dk / Szz_G from the means (eq. CrfRatio);
 *   phase_cos, phase_sin  mean of exp(i arg det(1 + B_M..B_1)) of spin up.
 *           The weight det_up det_dn is real and non-negative (det_dn is the
 *           complex conjugate of det_up up to a positive factor, Sec. II B);
 *           the phase of det_up alone is tracked per accepted flip and
 *           re-anchored from the UDV factors at every recomputation;
 *   chi_e   charge compressibility of eq. ChiCharge, (beta/N_s)(<N^2> - <N>^2)
 *           with the equal-time <N^2> from Wick's theorem (<N> = N_s at half
 *           filling in every configuration);
 *   GAB_dirac  |G_AB(K + dk)| of Sec. IV A: the modulus of the mean n_AB(k)
 *           (spin-averaged, eq. nkMatrix) at K + b1/L, averaged over the two
 *           Dirac points K = (2 b1 + b2)/3 and (b1 + 2 b2)/3 of the
 *           instance's grid (nearest grid points when L % 3 != 0; the grid
 *           is shifted by a twist, eq. kpoints); 0 when the momentum
 *           distribution is not measured (dqmc_set_measure_k). */
typedef struct {
  double n, D, ekin, e, Szz_G, Szz_dk, m2, Rm2, phase_cos, phase_sin, chi_e, GAB_dirac;
  int64_t n_meas;
} dqmc_obs;

/* Counters since creation or the last dqmc_reset_obs (sweeps: since creation).
 * drift_last: max |G_wrap - G_scratch| of the most recent recomputation of G,
 * drift_max: the largest so far.  phase_re/im: current exp(i arg det_up);
 * phase_drift: largest |tracked - anchored| phase at a recomputation. */
typedef struct {
  int64_t proposals, accepted, flushes, sweeps;
  double drift_max, drift_last;
  int32_t numeric_err;
  int64_t learn_proposals, learn_accepted;  /* learned multi-site moves */
  double phase_re, phase_im, phase_drift;
} dqmc_stats;

/* Bytes of device workspace for n instances (ws: output). */
dqmc_status dqmc_workspace_size(const dqmc_instance_desc* d, int32_t n, size_t* bytes);

/* Create a handle on the current HIP device.  dev_ws: caller-owned device
 * buffer of at least dqmc_workspace_size bytes; stream: hipStream_t for all
 * work of this handle.  Fields start i.i.d. +-1 from Philox(seed) and G(0) is
 * built from scratch (stream-ordered, asynchronous). */
dqmc_status dqmc_create(const dqmc_instance_desc* d, int32_t n, void* dev_ws, size_t bytes,
                        void* stream, dqmc_handle* out);
dqmc_status dqmc_destroy(dqmc_handle h);

/* Replace the fields of instance inst (host int8, M*N, values +-1) and
 * rebuild G and the UDV stack from scratch.  Synchronises the stream. */
dqmc_status dqmc_set_fields(dqmc_handle h, int32_t inst, const int8_t* host_x);
dqmc_status dqmc_get_fields(dqmc_handle h, int32_t inst, int8_t* host_x);

/* n_sweeps full sweeps of every instance (Sec. III: an upward pass l = 1..M,
 * wrap then single-site updates of slice l, and a downward pass l = M..1,
 * updates then wrap; G recomputed from the UDV chains after every n_stab
 * slices, eq. GrFMat); estimators are accumulated at every recomputation of
 * G when measure != 0.  Instances with fewer slices than the largest M of
 * the handle sweep proportionally more often in the same call.  Asynchronous
 * on the stream; errors of the device side surface as DQMC_ENUMERIC from
 * dqmc_measure / dqmc_get_stats. */
dqmc_status dqmc_sweep(dqmc_handle h, int32_t n_sweeps, int32_t measure, void* stream);

/* Replay mode: the Metropolis decision for proposal n of instance i is
 * dev_bits[i * bits_per_inst + n] (1 = accept) instead of u < R; proposals
 * are numbered in visiting order over the replayed sweeps, starting at 0.
 * dev_ratios (nullable, same layout, doubles) receives R of each proposal.
 * Both are device pointers owned by the caller; bits_per_inst must cover
 * n_sweeps * 2 * M * N proposals of the largest instance.  Synchronises. */
dqmc_status dqmc_replay(dqmc_handle h, const uint8_t* dev_bits, int64_t bits_per_inst,
                        double* dev_ratios, int32_t n_sweeps, int32_t measure, void* stream);

/* G of instance inst, the equal-time Green's function of eq. GrFMat,
 * G_ij = <c_i c_j^dagger> = (1 + B_l..B_1 B_M..B_{l+1})^{-1} at the current
 * slice l of the instance's sweep (l = 0 between sweeps), spin 0 (up) or 1
 * (down: P (1 - G_up^dagger) P with P = diag(+1 on A, -1 on B), the
 * particle-hole partner of Sec. II B in the original basis; G_up itself in the
 * charge channel).  host_out:
 * N x N row-major, real doubles or interleaved (re, im) for twisted
 * handles; caller-allocated.  Synchronises the handle's stream. */
dqmc_status dqmc_get_green(dqmc_handle h, int32_t inst, int32_t spin, double* host_out);
/* Overwrite G (spin up) of instance inst (row-major, same element format). */
dqmc_status dqmc_set_green(dqmc_handle h, int32_t inst, const double* host_in);

/* Apply one wrap to G of every instance with the fields of slice l (1..M):
 * dir 0: G <- B_l G B_l^{-1}; dir 1: G <- B_l^{-1} G B_l (Sec. III A).  In
 * DQMC_MIXED handles the transform runs in complex64 as in the sweep. */
dqmc_status dqmc_wrap(dqmc_handle h, int32_t dir, int32_t slice, void* stream);

/* Rank-k flush G <- G - X Y on instance inst with host X (N x k, column
 * j at X + j*N) and Y (k x N, row m at Y + m*N); elements as for G.
 * Exercises the MFMA flush kernel (eq. FinalDelay) of the handle's
 * precision and the selected flush kernel (dqmc_set_flush_kernel);
 * synchronises. */
dqmc_status dqmc_flush_test(dqmc_handle h, int32_t inst, const double* host_X,
                            const double* host_Y, int32_t k);

/* Estimator means of instance inst (see dqmc_obs); synchronises.
 * DQMC_ENUMERIC (out still filled) if the instance hit a numerical error. */
dqmc_status dqmc_measure(dqmc_handle h, int32_t inst, dqmc_obs* out);
/* Update scheme of the single-site sweep (Sec. III B).  0 (default): the
 * delayed update, rank-1 terms x_k y_k of eq. DelayRgenk accumulated across
 * windows and flushed at rank k (eq. FinalDelay).  1: the submatrix update
 * named in Sec. III B: after the window scan the accepted flips S of the
 * window are applied as one multi-site update,
 *   G' = G - G[:, S] Delta_S (1 + (1 - G)_SS Delta_S)^{-1} (1 - G)[S, :],
 * with the m x m inverse by Gauss-Jordan elimination in the order of
 * acceptance (its pivots are the sequential ratios), G[:, window] M~ on the
 * matrix cores, and a flush after every window (the flush rank is then the
 * window's accept count).  Same chain, G equal up to rounding.  DQMC_EINVAL
 * for other values. */
dqmc_status dqmc_set_update_scheme(dqmc_handle h, int32_t scheme);
/* How the full-length delayed vectors x_k, y_k of a window's accepted flips
 * are formed (eq. DelayRgenk): mm = 0 (default) by the recursion itself, one
 * row of X and column of Y per thread; mm = 1 in matrix form, X_new = A Tx
 * and Y_new = Ty B with A, B the window's columns and rows of G - X Y and
 * Tx, Ty the triangular coefficients of the recursion (the products on the
 * matrix cores, the coefficients by a serial recursion per row).  The same
 * vectors up to rounding; learned block moves always use the recursion.
 * DQMC_EINVAL for other values. */
dqmc_status dqmc_set_expand_kernel(dqmc_handle h, int32_t mm);
/* How a recomputation applies Y^{-1} in G = U_L D_Lb^{-1} Y^{-1} D_Rb^{-1}
 * U_R^H (eq. GrFMat with the split of D into its large and small parts,
 * Sec. II B): lu = 1 (default) factors Y by LU with partial pivoting, whose
 * trailing updates are MFMA GEMMs; lu = 0 by a second Householder QR.  Both
 * give G to rounding (Y is well conditioned after the split); the phase of
 * det Y comes from the pivots and diag U, or from the reflectors and diag R.
 * DQMC_EINVAL for other values. */
dqmc_status dqmc_set_y_solver(dqmc_handle h, int32_t lu);
/* Momentum distribution (eq. nkMatrix) with every measurement: G of each
 * instance (or its half-step G~) is Fourier transformed on both sides,
 * Ghat = F G F^dagger (F the unnormalised per-sublattice 2-D DFT of the
 * wraps), and n_ab(k) = (1/N_c) sum_{r,r'} e^{i k.(r - r')} <c^+_{a r} c_{b r'}>
 * = delta_ab - Ghat[b k, a k] / N_c (spin up; spin down from the particle-hole
 * partner) is accumulated as the spin average.  Default on. */
dqmc_status dqmc_set_measure_k(dqmc_handle h, int32_t on);
/* Mean momentum distribution of instance inst over the measurements since the
 * last dqmc_reset_obs, per plain grid index k = l1 + L l2 (momentum
 * ((l1 + Theta1/2pi) b1 + (l2 + Theta2/2pi) b2)/L).  raw = 1: N_c x 8 doubles,
 * the complex means of n_AA, n_AB, n_BA, n_BB as (re, im).  raw = 0: N_c x 7
 * doubles: |f(k)| (the band energies are -+|f|), n_AA, n_BB, Re n_AB, Im n_AB
 * of the Hermitian part of the mean, and its eigenvalues n_+ >= n_-: n_+
 * belongs to the band eps_{k,-} = -|f| and n_- to eps_{k,+} (Sec. II C).
 * DQMC_ESTATE if nothing was measured.  Synchronises. */
dqmc_status dqmc_get_nk(dqmc_handle h, int32_t inst, int32_t raw, double* host_out);

/* ---- time-displaced estimators (Sec. II C, eqs. DouOccDerive, fidelitysusp) ----
 * One pass over the current configuration of every instance that stands at
 * the start of a sweep (right after creation or after whole sweeps of the
 * handle; others are skipped): G(tau,tau), G(tau,0) = <c(tau) c^dagger(0)> and
 * G(0,tau) = -<c^dagger(tau) c(0)> of spin up for tau_l = l dtau,
 * l = 0 .. min(M/2, l_max) (l_max < 0: M/2), propagated slice by slice with
 * the wraps and recomputed every n_stab slices from the UDV chain and the
 * stack of the last downward pass (G(tau,0) = [B(tau,0)^{-1} + B(beta,tau)]^{-1},
 * G(0,tau) = -[B(tau,0) + B(beta,tau)^{-1}]^{-1}, with the scale split of the
 * equal-time recomputation; their drift enters dqmc_stats and the drift
 * tolerance; in DQMC_MIXED handles the wraps run in complex64 as in the
 * sweep).  At every slice the Wick estimator of
 *   <A(tau_l) A(0)>,  A = sum_i (n_up,i - 1/2)(n_dn,i - 1/2) = H_I + N_s/4
 * (H_I of the correlator C_{H_I}(tau)) is accumulated, the spin-down
 * functions being the particle-hole partners (spin channel) or equal to
 * spin up (charge channel).  Fields, G, the stack and the sweep schedule are
 * left unchanged.  Asynchronous on stream (NULL: the handle's stream);
 * DQMC_EHIP on a launch failure. */
dqmc_status dqmc_measure_tau(dqmc_handle h, int32_t l_max, void* stream);
/* Means over the passes of instance inst since creation or dqmc_reset_obs,
 * l = 0 .. M/2 (M/2 + 1 doubles each; slices a pass did not reach count as
 * 0): host_aa[l] = <A(tau_l) A(0)>, host_a[l] = the equal-time <A> measured
 * at slice l (the same in expectation for every l), and *n_pass.  The
 * connected C_{H_I}(tau_l) is host_aa[l] - host_a[0]^2; with few passes the
 * per-pass rows give the lower-variance form mean(<A(tau)A(0)>_X -
 * <A>_X(tau) <A>_X(0)) + Cov(<A>_X(tau), <A>_X(0)).  Synchronises;
 * DQMC_ENUMERIC (outputs still filled) after a numerical error. */
dqmc_status dqmc_get_tau(dqmc_handle h, int32_t inst, double* host_aa, double* host_a, int64_t* n_pass);
/* The same values per pass, oldest first: the last min(passes, 1024,
 * max_rows) passes of instance inst, M + 2 doubles each for even M (<A(tau_l)
 * A(0)>_X for l = 0 .. M/2, then <A>_X(tau_l) for l = 0 .. M/2); *n_rows
 * receives the count.  Synchronises. */
dqmc_status dqmc_get_tau_rows(dqmc_handle h, int32_t inst, double* host_rows, int32_t max_rows, int32_t* n_rows);
/* Spin-up G(tau,tau) (which 0), G(tau,0) (1) or G(0,tau) (2) of instance inst
 * at the last slice of the last pass that instance took part in, N x N
 * row-major, elements as in dqmc_get_green (the three matrices have storage of
 * their own, so later sweeps leave them alone; their contents are unspecified
 * before the instance's first pass).  Synchronises. */
dqmc_status dqmc_get_green_tau(dqmc_handle h, int32_t inst, int32_t which, double* host_out);
/* dD/dU = -(2/N_s) int_0^{beta/2} C dtau (eq. DouOccDerive) and
 * chi_F = int_0^{beta/2} tau C dtau (eq. fidelitysusp) from host_c[l] =
 * C_{H_I}(l dtau), l = 0 .. n-1 (the last point at beta/2).  degree < 0:
 * trapezoid rule on the slice grid, which for the Trotterised partition
 * function is exactly its derivative in U; degree >= 0: least-squares
 * polynomial of that degree (< n, <= 12) integrated analytically, as the
 * paper evaluates them.  Host arithmetic only; DQMC_EINVAL on bad sizes. */
dqmc_status dqmc_tau_integrals(const double* host_c, int32_t n, double dtau, int32_t n_sites, int32_t degree,
                               double* dD_dU, double* chi_F);

/* Restart the estimator means (also the time-displaced ones) and the
 * counters of dqmc_stats (proposals, accepted, flushes, drifts, learned
 * moves) and clear numeric_err. */
dqmc_status dqmc_reset_obs(dqmc_handle h);
/* Per-sweep means of the estimators in the order of dqmc_obs up to chi_e
 * (11 doubles per sweep), most recent max_sweeps at most, oldest first;
 * *n_out = sweeps written. */
dqmc_status dqmc_get_series(dqmc_handle h, int32_t inst, double* host_out, int32_t max_sweeps,
                            int32_t* n_out);
/* Counters of instance inst; synchronises.  DQMC_ENUMERIC (out still
 * filled) if numeric_err is set. */
dqmc_status dqmc_get_stats(dqmc_handle h, int32_t inst, dqmc_stats* out);
/* Tolerance of the recomputation drift max |G_wrap - G_scratch| of every
 * instance (default 1e-4): a larger drift sets numeric_err bit 2.
 * DQMC_EINVAL unless tol > 0.  Synchronises. */
dqmc_status dqmc_set_drift_tol(dqmc_handle h, double tol);

/* Live kernel timing with HIP events on the handle's stream.  While enabled,
 * every launch of the classes below is bracketed by an event pair; times are
 * summed when dqmc_get_timing synchronises.  Algorithmic work per class:
 * flush = sum over flushes of c N^2 k (c = 2 real, 8 complex; k = rank),
 * wrap = 2 N^2 s bytes per instance per side-pass (one read and one write of
 * G, s = bytes per element). */
typedef enum { DQMC_T_WRAP = 0, DQMC_T_WINDOW, DQMC_T_EXPAND, DQMC_T_FLUSH, DQMC_T_STAB, DQMC_T_MEASURE,
               DQMC_T_LEARN, DQMC_T_COUNT } dqmc_timing_class;
typedef struct {
  int64_t launches[DQMC_T_COUNT];
  double ms[DQMC_T_COUNT];
  double flush_flops;   /* algorithmic FP64 flops of all timed flushes */
  double wrap_bytes;    /* algorithmic HBM bytes of all timed wrap passes */
} dqmc_timing;
dqmc_status dqmc_set_timing(dqmc_handle h, int32_t on);   /* on: 1 enable (and reset), 0 disable */
dqmc_status dqmc_get_timing(dqmc_handle h, dqmc_timing* out);  /* synchronises */

/* ---- Learned multi-site moves (an extension; the paper proposes single sites).
 *
 * After the single-site updates of every slice visit, per_slice moves flip an
 * ordered set S of m distinct sites of that slice at once.  S is drawn from
 * the Plackett-Luce law of the weights sigmoid(y_i) of the network outputs
 * y_i of the slice, i.e. of the logits z_i = log sigmoid(y_i) (q(S|X) =
 * prod_j e^{z_{s_j}} / sum over the sites not yet chosen of e^{z_i}), with
 * Gumbel-top-m: the m largest z_i - log(-log u_i).  Trained on the Barker
 * acceptances below (y ~ log Rt) this is a locally balanced informed
 * proposal.  The move is accepted iff
 * u < R_S q(S|X') / q(S|X), where R_S = e^{2 lambda sum_S x} |det(1_m +
 * Delta_S (1 - G)_{SS})|^2 is the block form of the paper's single-site ratio
 * (eqs. DRatio, rRatioLocal) and X' has the sites of S flipped; on acceptance
 * G takes the block Sherman-Morrison update through the delayed-update
 * buffers (eqs. DelayRgenk, FinalDelay).  The chain stays exact for any
 * network.  Uniforms: Philox4x32-10 with the instance's key and counter
 * (site, slice, sweep, 4 + 4 move + pass) for the Gumbel noise, with
 * u = (floor(k/2) + 1/2) 2^-52 for the 53-bit k of the site uniforms, and
 * counter (0xffffffff, slice, sweep, 4 + 4 move + pass) for the acceptance
 * u = k 2^-53.
 *
 * The network maps the fields of all slices on the cell grid, channels
 * (x_A, x_B), through three periodic 3x3x3 convolutions over (slice, n2, n1)
 * of widths 2 -> 32 -> 32 -> 2 (tanh after the first two, biases everywhere)
 * to the outputs (y_A, y_B) of each cell.  Parameters, FP32, in this order:
 * W1 [27][32][2], b1 [32], W2 [27][32][32], b2 [32], W3 [27][2][32], b3 [2]
 * (DQMC_NET_NPARAM values); tap (dt+1)*9 + (d2+1)*3 + (d1+1) of an output
 * at (t, n2, n1) reads (t+dt, n2+d2, n1+d1), periodic; [tap][out][in].
 * The device computes with BF16 weights and activations and FP32
 * accumulation.  A new handle starts with all parameters zero (uniform
 * proposals).  The training loss is the mean binary cross-entropy between
 * sigmoid(y_i) and targets a_i in [0, 1] over all sites and slices. */
#define DQMC_NET_NPARAM 31170

/* Moves per slice visit (0 disables, at most 8) and sites per move (1..8);
 * not applied in replay mode. */
dqmc_status dqmc_set_proposals(dqmc_handle h, int32_t per_slice, int32_t m);

/* Parameters in and out (host FP32, n = DQMC_NET_NPARAM).  Setting them
 * resets the Adam moments. */
dqmc_status dqmc_net_set_weights(dqmc_handle h, const float* host_w, int64_t n);
dqmc_status dqmc_net_get_weights(dqmc_handle h, float* host_w, int64_t n);
/* Starting point for training: W1, W2 drawn N(0, 1/fan_in) from a generator
 * seeded with seed, W3 and all biases zero (the proposals stay uniform until
 * trained); resets the Adam moments. */
dqmc_status dqmc_net_init(dqmc_handle h, uint64_t seed);

/* Training data recorded by the sampler: for every site of instance inst,
 * the Barker acceptance Rt / (1 + Rt) of flipping it again right after its
 * single-site decision in the last downward pass (Rt = 1/R after an accepted
 * flip, R after a rejected one), M x N floats. */
dqmc_status dqmc_get_targets(dqmc_handle h, int32_t inst, float* host_out);

/* Training samples.  With every > 0, after the single-site updates of every
 * downward-pass slice l with l % every == 0, each instance stores its field
 * window of slices l-3 .. l+3 (mod M; 7 x N int8) and the targets of slice l
 * (N floats) in a device ring of `capacity` slots (a multiple of the number
 * of instances n): instance i writes slots (c n + i) % capacity for its c-th
 * sample.  The logits of slice l depend on no field outside that window. */
dqmc_status dqmc_collect(dqmc_handle h, int32_t every);
/* Slots filled so far (all instances), and the ring capacity.  Synchronises. */
dqmc_status dqmc_sample_count(dqmc_handle h, int64_t* filled, int64_t* capacity);
/* Copy count slots from slot first: windows count x 7 x Nmax int8 (rows of
 * Nmax entries, an instance's first N used), targets count x Nmax floats;
 * Nmax = the largest N of the handle.  Synchronises. */
dqmc_status dqmc_get_samples(dqmc_handle h, int64_t first, int32_t count, int8_t* host_win, float* host_tg);

/* Device scratch for dqmc_net_logits / dqmc_net_grad on configurations of one
 * size (L, M), n_samples of them per call, minibatches of batch <= 64; with
 * M = 7 also enough for window samples. */
dqmc_status dqmc_net_workspace_size(int32_t L, int32_t M, int64_t n_samples, int32_t batch, size_t* bytes);

/* Logits of n configurations (host int8 n x M x N) into host_out
 * (n x M x N floats), convolutions periodic in time; n <= 64.  dev_ws:
 * caller-owned device scratch of dqmc_net_workspace_size(L, M, n, n) bytes.
 * Synchronises. */
dqmc_status dqmc_net_logits(dqmc_handle h, void* dev_ws, size_t bytes, const int8_t* host_fields, int32_t n,
                            int32_t L, int32_t M, float* host_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the logits
 * of dqmc_net_logits, computed by the same kernels, with the scratch taken
 * from a static device array of the library (16 MiB on each GPU it runs on,
 * held until the process ends) instead of a caller workspace.  Needs
 * 5 n M N + 224 n M N_c bytes (fields, logits, activations; each part
 * rounded up to 256 bytes; DQMC_EUNSUPPORTED if above 16 MiB: one L = 18,
 * M = 180 configuration fits, two do not), n <= 64, and the handle's device
 * to be current
 * (DQMC_ESTATE otherwise).  Calls no device allocation routine.  Every call
 * on one GPU shares the array: calls that overlap on one GPU (several
 * threads or handles) race.  Synchronises the handle's stream. */
dqmc_status dqmc_net_logits_noalloc(dqmc_handle h, const int8_t* host_fields, int32_t n, int32_t L, int32_t M,
                                    float* host_out);

/* Loss and gradient (host, DQMC_NET_NPARAM floats) over a batch of n <= 64
 * samples.  window = 0: whole configurations (n x M x N) with targets for
 * every site (n x M x N floats).  window = 1: 7-slice windows (n x 7 x N,
 * M = 7) with targets of the centre slice only (n x N floats), evaluated as
 * the sampler and the trainer do.  Synchronises. */
dqmc_status dqmc_net_grad(dqmc_handle h, void* dev_ws, size_t bytes, const int8_t* host_fields,
                          const float* host_targets, int32_t n, int32_t L, int32_t M, int32_t window,
                          float* host_loss, float* host_grad);

/* Device scratch for dqmc_net_train with minibatches of `batch` samples. */
dqmc_status dqmc_net_train_workspace_size(dqmc_handle h, int32_t batch, size_t* bytes);

/* steps Adam steps (lr; beta1 0.9, beta2 0.999, eps 1e-8) on the window
 * loss of minibatches of `batch` samples drawn with replacement from the
 * filled ring slots by a generator seeded with seed.  host_loss (nullable)
 * receives the minibatch loss of every step.  The sampler uses the new
 * parameters from its next launch on.  DQMC_ESTATE if no sample has been
 * collected.  Synchronises. */
dqmc_status dqmc_net_train(dqmc_handle h, void* dev_ws, size_t bytes, int32_t steps, int32_t batch, float lr,
                           uint64_t seed, float* host_loss);

/* Flush rank k of every instance (1 <= k <= max(n_delay, 128) of the
 * creation descriptors).  The rank changes when the buffered rank-1 terms
 * are applied, never the sequence of G's or decisions.  Synchronises. */
dqmc_status dqmc_set_delay(dqmc_handle h, int32_t k);

/* Flush kernel: 0 = one wave per 32 x 32 block of G with fragments read
 * straight from memory, 1 = 64 x 64 tiles per workgroup with X and Y staged
 * through LDS, 2 = persistent workgroups taking 64 x 64 tiles of all
 * instances from device work queues (one per XCD), the G block loaded behind
 * the products.  Mixed precision always uses its FP32 kernel.  dqmc_flush_test
 * runs the selected kernel. */
dqmc_status dqmc_set_flush_kernel(dqmc_handle h, int32_t variant);

/* Autotuner of the flush rank and kernel: for each of the n_cand candidate
 * ranks and each of the three flush kernels, run `steps` slice steps (a
 * multiple of n_stab; the chains advance as in a sweep, without estimators),
 * time them with HIP events, and keep the fastest pair (best[0] = rank,
 * best[1] = kernel; ms_per_step[3 q + v], nullable, gets the time per step
 * of rank q with kernel v, 0 where not tried).  The chains then take the
 * steps (at most one sweep) that bring the instances of the largest M back
 * to the start of a sweep.  Synchronises. */
dqmc_status dqmc_autotune(dqmc_handle h, int32_t steps, const int32_t* cand, int32_t n_cand, int32_t* best,
                          double* ms_per_step);

/* FFT tiles of the register-line wrap kernel (L <= 24 with a compile-time
 * plan): vectors (columns, or rows) per workgroup, per L and side (0 columns,
 * 1 rows): tile 0 = as many as 256 threads cover (2 L threads per vector),
 * 1 = half as many (half the LDS, more workgroups per CU), 2 = eight (rows of
 * complex G read as 128-byte segments; the wide tile where eight vectors
 * would need more than 96 KB of LDS).  Single-precision wraps always use
 * tile 0.  The tile only changes the grouping of independent vectors, never
 * the result.  DQMC_EINVAL if no instance of the handle has this L. */
dqmc_status dqmc_set_fft_tile(dqmc_handle h, int32_t L, int32_t side, int32_t tile);
/* Distinct lattice sizes with a compile-time FFT plan (n, and Ls[0..n) if
 * Ls is not null, at most 16), in the order of dqmc_autotune_fft's output. */
dqmc_status dqmc_fft_plan_count(dqmc_handle h, int32_t* n, int32_t* Ls);
/* FFT tile autotuner: for every plan L (dqmc_fft_plan_count order q), side
 * and tile, time `reps` wrap transforms of a scratch matrix of every
 * instance with HIP events and keep the fastest tile per (L, side).
 * tiles_out[2 q + side] (nullable) receives the choice, us_out[(2 q + side)
 * * 3 + tile] (nullable) the microseconds per transform.  The chains are not
 * advanced.  Synchronises. */
dqmc_status dqmc_autotune_fft(dqmc_handle h, int32_t reps, int32_t* tiles_out, double* us_out);

/* Instance groups: groups in [1, 4] (default: 3 for 24 or more instances, 2
 * for 8 or more, else 1).  The instances are split into that many contiguous groups of
 * about equal work (fewer if there are fewer instances), group 0 running on
 * the call's stream and the others on streams of the handle, so that the
 * latency-bound kernels of one group overlap the others'; the call's stream
 * waits for all of them before the call returns.  1 runs every instance in
 * the same launches.  Live timing (dqmc_set_timing) runs one group.
 * DQMC_EINVAL for groups outside [1, 4]. */
dqmc_status dqmc_set_streams(dqmc_handle h, int32_t groups);

/* HIP graphs (default on): sweeps replay one captured block of n_stab slice
 * steps (captured on first use and again after a setting that changes the
 * launches: proposals, collection, flush kernel or rank, groups, replay,
 * measure).  Live timing and step counts that are not whole blocks run
 * eagerly.  The captured block contains kernel launches only. */
dqmc_status dqmc_set_graphs(dqmc_handle h, int32_t on);

/* Matrix dimension N, slices M and whether G is complex, for instance inst. */
dqmc_status dqmc_shape(dqmc_handle h, int32_t inst, int32_t* N, int32_t* M, int32_t* is_complex);

const char* dqmc_status_string(dqmc_status s);
const char* dqmc_last_error(dqmc_handle h);

#ifdef __cplusplus
}
#endif
#endif /* DQMC_H */
