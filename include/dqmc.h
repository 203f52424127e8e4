/*
 * dqmc.h -- C ABI of the MI355X DQMC sweep library (libdqmc.so).
 *
 * Finite-temperature determinant QMC for the half-filled honeycomb Hubbard
 * model, H = -t sum_<ij>s (c^+_is c_js + h.c.) + U sum_i (n_iu n_id - (n_iu + n_id)/2)
 * (Sec. II A, eq. HubbModel), with the Hubbard-Stratonovich transformation in
 * the spin-s^z channel, cosh(lambda) = exp(dtau U / 2) (eqs. SzHS, coupling).
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
 * errors return without side effects.  DQMC_ENUMERIC reports a non-finite or
 * zero acceptance ratio seen on the device; the handle remains usable for
 * dqmc_get_stats and dqmc_destroy.  dqmc_last_error gives a message.
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
 * estimators stay FP64.  The accumulated single-precision error is reported
 * as the drift max |G_wrap - G_scratch| at each recomputation (dqmc_stats). */
typedef enum { DQMC_FP64 = 0, DQMC_MIXED = 1 } dqmc_precision;

/* One Markov chain.  All instances of a handle share n_stab, and every
 * beta/dtau must be a multiple of n_stab.  L in [2, 45] with prime factors in
 * {2, 3, 5, 7, 11, 13}. */
typedef struct {
  int32_t L;            /* unit cells per side */
  double t, U;          /* hopping and Hubbard U */
  double beta, dtau;    /* M = beta/dtau must be an integer within 1e-9 */
  double theta1, theta2;/* twist Theta_1, Theta_2 in radians along a1, a2; both 0 = periodic (real path) */
  int32_t n_delay;      /* flush rank k: flush once at least k accepted flips are pending, 1 <= k <= 192 */
  int32_t n_stab;       /* slices between recomputations of G (stabilisation) */
  int32_t precision;    /* dqmc_precision, the same for all instances of a handle */
  int32_t sym_measure;  /* 1: estimators on exp(-dtau K/2) G exp(+dtau K/2) */
  uint64_t seed;        /* Philox key */
} dqmc_instance_desc;

/* Means over all measurements since creation or the last dqmc_reset_obs. */
typedef struct {
  double n, D, ekin, e, Szz_G, Szz_dk, m2, Rm2, phase_cos, phase_sin;
  int64_t n_meas;
} dqmc_obs;

typedef struct {
  int64_t proposals, accepted, flushes, sweeps;
  double drift_max, drift_last;
  int32_t numeric_err;
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

/* n_sweeps full sweeps of every instance; estimators are accumulated at every
 * recomputation of G when measure != 0.  Asynchronous on the stream. */
dqmc_status dqmc_sweep(dqmc_handle h, int32_t n_sweeps, int32_t measure, void* stream);

/* Replay mode: the Metropolis decision for proposal n of instance i is
 * dev_bits[i * bits_per_inst + n] (1 = accept) instead of u < R; proposals
 * are numbered in visiting order over the replayed sweeps, starting at 0.
 * dev_ratios (nullable, same layout, doubles) receives R of each proposal.
 * Both are device pointers owned by the caller; bits_per_inst must cover
 * n_sweeps * 2 * M * N proposals of the largest instance.  Synchronises. */
dqmc_status dqmc_replay(dqmc_handle h, const uint8_t* dev_bits, int64_t bits_per_inst,
                        double* dev_ratios, int32_t n_sweeps, int32_t measure, void* stream);

/* G of instance inst, spin 0 (up) or 1 (down: P (1 - G_up^dagger) P with
 * P = diag(+1 on A, -1 on B)), row-major; synchronises. */
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
 * precision; synchronises. */
dqmc_status dqmc_flush_test(dqmc_handle h, int32_t inst, const double* host_X,
                            const double* host_Y, int32_t k);

dqmc_status dqmc_measure(dqmc_handle h, int32_t inst, dqmc_obs* out);  /* synchronises */
dqmc_status dqmc_reset_obs(dqmc_handle h);
/* Per-sweep means of the estimators in the order of dqmc_obs (10 doubles per
 * sweep), most recent max_sweeps at most, oldest first; *n_out = sweeps written. */
dqmc_status dqmc_get_series(dqmc_handle h, int32_t inst, double* host_out, int32_t max_sweeps,
                            int32_t* n_out);
dqmc_status dqmc_get_stats(dqmc_handle h, int32_t inst, dqmc_stats* out);  /* synchronises */

/* Live kernel timing with HIP events on the handle's stream.  While enabled,
 * every launch of the classes below is bracketed by an event pair; times are
 * summed when dqmc_get_timing synchronises.  Algorithmic work per class:
 * flush = sum over flushes of c N^2 k (c = 2 real, 8 complex; k = rank),
 * wrap = 2 N^2 s bytes per instance per side-pass (one read and one write of
 * G, s = bytes per element). */
typedef enum { DQMC_T_WRAP = 0, DQMC_T_WINDOW, DQMC_T_EXPAND, DQMC_T_FLUSH, DQMC_T_STAB, DQMC_T_MEASURE,
               DQMC_T_COUNT } dqmc_timing_class;
typedef struct {
  int64_t launches[DQMC_T_COUNT];
  double ms[DQMC_T_COUNT];
  double flush_flops;   /* algorithmic FP64 flops of all timed flushes */
  double wrap_bytes;    /* algorithmic HBM bytes of all timed wrap passes */
} dqmc_timing;
dqmc_status dqmc_set_timing(dqmc_handle h, int32_t on);   /* on: 1 enable (and reset), 0 disable */
dqmc_status dqmc_get_timing(dqmc_handle h, dqmc_timing* out);  /* synchronises */

/* Matrix dimension N, slices M and whether G is complex, for instance inst. */
dqmc_status dqmc_shape(dqmc_handle h, int32_t inst, int32_t* N, int32_t* M, int32_t* is_complex);

const char* dqmc_status_string(dqmc_status s);
const char* dqmc_last_error(dqmc_handle h);

#ifdef __cplusplus
}
#endif
#endif /* DQMC_H */
