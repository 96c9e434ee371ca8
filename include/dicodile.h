/*
 * dicodile.h -- C ABI of the MI355X (gfx950) convolutional sparse coding
 * library built on the CSC step of DiCoDiLe (Moreau & Gramfort,
 * "Distributed Convolutional Dictionary Learning (DiCoDiLe): Pattern
 * Discovery in Large Images and Signals", arXiv:1901.09235).
 *
 * Problem (Sec. 2, eq. csc):  Z* = argmin_Z 1/2 ||X - Z*D||_2^2 + lambda ||Z||_1,
 * optionally with Z >= 0.  Solver: locally greedy coordinate descent (Alg. 1)
 * on a grid of workers with the soft-lock rule (Alg. 3, eq. soft_lock); one
 * worker is one GPU workgroup.
 *
 * Conventions shared by every call (0-based, row-major, contiguous):
 *   d = 1 (signals): X (P, T),      D (K, P, L),      Z (K, T - L + 1)
 *   d = 2 (images):  X (P, T1, T2), D (K, P, L1, L2), Z (K, T1-L1+1, T2-L2+1)
 *   Z lives on the "valid" domain, so that every shifted atom keeps the norm
 *   ||D_k||_2^2 that the closed-form update of eq. pb_coord divides by.
 *   (Z*D)_p[x] = sum_k sum_t Z_k[x - t] D_{k,p}[t]               (eq. model)
 *   corr(R, D)_k[w] = sum_p sum_t D_{k,p}[t] R_p[w + t]  (the paper's R * D~_k)
 *
 * Memory: every array argument is a caller-owned DEVICE pointer (memory of
 * the current HIP device, e.g. a torch tensor's data_ptr()), in the dtype
 * given by the call, unless stated otherwise.  The library never frees caller
 * memory.  It keeps a per-device workspace that grows on demand and is
 * released by dicodile_release().
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 * stream).  Every call enqueues its work on that stream and returns after the
 * work has completed (the calls fill host-side results).
 *
 * Errors: every call returns a dcdl_status.  On an error (< 0) no caller
 * buffer is written, except where stated; dicodile_last_error() returns a
 * message for the calling thread.  Concurrent calls on the same device are
 * serialised by the library.
 */
#ifndef DICODILE_MI355X_H
#define DICODILE_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DCDL_OK = 0,
  DCDL_NOT_CONVERGED = 1, /* stopped on max_updates / max_rounds / timeout; z holds the iterate */
  DCDL_PENDING = 2,       /* dicodile_server_poll / _wait: the request has not finished yet */
  DCDL_EINVAL = -1,       /* bad shape, dtype, option or pointer */
  DCDL_ENOMEM = -2,       /* device memory or HBM budget exhausted */
  DCDL_EHIP = -3,         /* a HIP runtime call failed */
  DCDL_EDIVERGED = -4,    /* divergence guard: ||Z||_inf exceeded opts.div_guard */
  DCDL_ETIMEOUT = -5,     /* a worker waited on a neighbour past the internal limit */
  DCDL_ENODEV = -6        /* no gfx950 device, or the call needs a capability it lacks */
} dcdl_status;

typedef enum { DCDL_F32 = 0, DCDL_F64 = 1 } dcdl_dtype;

/* Precision of the dense correlation corr(R, D) (beta initialisation,
 * dicodile_corr).  The matrix-core paths need (P * L1 * L2 small enough that a
 * staged window fits 64 KB of LDS: P up to 8 x L2 up to ~700 for signals);
 * otherwise DIRECT is used. */
typedef enum {
  DCDL_CORR_AUTO = 0,    /* FP32 data: BF16X3; FP64 data: F64 */
  DCDL_CORR_F64 = 1,     /* v_mfma_f64_16x16x4: FP64 products and sums */
  DCDL_CORR_BF16 = 2,    /* v_mfma_f32_16x16x32_bf16: BF16 operands, FP32 sums (FP32 data only) */
  DCDL_CORR_BF16X3 = 3,  /* the same on hi/lo BF16 splits (hi*hi + hi*lo + lo*hi), about FP32
                            accuracy (FP32 data only) */
  DCDL_CORR_DIRECT = 4,  /* vector FMA in the data's precision, no matrix cores */
  DCDL_CORR_F64_FFT = 5  /* FP64 by FFT (the correlation theorem over the powers of two covering
                            T1 x T2): images whose padded sizes lie in [64, 8192] with P <= 8;
                            otherwise, or if its workspace (about 16 (K P + P + K) N1 N2 / 2
                            bytes) does not fit in 60% of free device memory, F64 */
} dcdl_corr_prec;

/* Coordinate-selection rule of the solve (dcdl_csc_opts.strategy).  Sec. 3
 * names the cyclic, random and greedy rules and builds the locally greedy one
 * between them; Sec. 5 compares greedy, randomized and locally greedy CD.
 * Every rule runs inside the same worker grid, soft-lock and stopping
 * certificate (no move scoring >= tol anywhere). */
typedef enum {
  DCDL_SELECT_LGCD = 0,    /* greedy within sub-domains of opts->tile (Alg. 1) */
  DCDL_SELECT_GREEDY = 1,  /* one sub-domain per worker: the worker's whole domain (GCD) */
  DCDL_SELECT_CYCLIC = 2,  /* one-position sub-domains visited in raster order: cyclic CD over
                              positions, greedy over the K atoms of a position */
  DCDL_SELECT_RANDOM = 3   /* one coordinate (position and atom) per round, drawn uniformly from the
                              worker's domain with the counter-based SplitMix64 generator: worker w's
                              n-th draw is SplitMix64 of opts->seed at counter n + w 2^40, and
                              j = draw mod (K |S_w|) picks position j / K (raster order in S_w) and
                              atom j mod K.  A worker checks its whole domain once per |S_w| draws
                              for the stopping certificate */
} dcdl_select;

/* Problem shape.  ndim = 1: T[0] = T, L[0] = L (T[1], L[1] ignored).
 * ndim = 2: T = (T1, T2), L = (L1, L2).  Requires 1 <= L_i <= T_i, P >= 1,
 * 1 <= K <= 1024, T1 T2 < 2^31, and (the round kernel's 32-bit offsets into
 * the update table of eq. beta_update) K (2 L1 - 1)(2 L2 - 1) K4 +
 * (T1 + 2 L1 - 1)(2 L2 - 1) K4 + (T2 + 2 L2 - 1) K4 < 2^31 with K4 = K
 * rounded up to a multiple of 4; DCDL_EINVAL otherwise. */
typedef struct {
  int32_t ndim;
  int32_t P;
  int32_t K;
  int32_t reserved;
  int64_t T[2];
  int32_t L[2];
} dcdl_shape;

/* Solver options (dicodile_csc).  Zero-initialise, then set lambda and tol. */
typedef struct {
  double lambda;          /* absolute lambda > 0 (Sec. 2: set as a fraction of lambda_max) */
  double tol;             /* epsilon >= 0 on |Delta Z| (Alg. 1 stopping rule) */
  int32_t positive;       /* 1: constrain Z >= 0 (one-sided soft-thresholding) */
  int32_t certify;        /* 1 (recommended): support- or sign-changing moves score at
                             least tol, so exit bounds the strict KKT violation by
                             max_k ||D_k||^2 tol; 0: the paper's plain |Delta Z| rule */
  dcdl_dtype dtype;       /* precision of X, D, z_out and of the incremental beta/Z */
  int32_t no_soft_lock;   /* 1: disable the soft-lock test of eq. soft_lock (ablation of
                             Sec. 5 only; pair it with div_guard) */
  int32_t threads;        /* threads per worker workgroup: 64, 128, 192, 256, 512 or 1024; 0 -> 256,
                             or for images 1024 (512) when the worker grid fits the device with one
                             (two) workgroups per CU */
  int32_t tile[2];        /* sub-domain size C_m per dimension; 0 -> 2 L_i (Sec. 3) */
  int32_t grid[2];        /* worker grid W_1 x W_2; 0 -> chosen by the library: ceil(extent / tile)
                             workers per axis, each at least L long, scaled down to the
                             workgroups that fit on the device together */
  int32_t warm_start;     /* 1: z_out holds the initial iterate on entry */
  int32_t refresh_every;  /* rebuild beta from its FP64 definition every this many sweeps of rounds
                             (periodic drift correction); 0 -> only after a failed final check.
                             A failed check rebuilds beta from the same FP64 contraction */
  int32_t max_polish;     /* extra solve passes after a failed final check; 0 -> 2 */
  int32_t inner;          /* sub-domain visits per worker per round; 0 -> 1 */
  int32_t beta_prec;      /* dcdl_corr_prec of the contraction that initialises beta from X
                             (0 -> FP32: BF16X3 matrix cores; FP64: FP64 matrix cores).  Every
                             later recomputation (periodic or after a failed check) and the final
                             check are FP64 whatever this is */
  int64_t max_rounds;     /* cap on worker rounds (0 -> unlimited) */
  double div_guard;       /* stop with DCDL_EDIVERGED if |Z| exceeds this (0 -> off) */
  double timeout_s;       /* wall-clock cap for the whole call (0 -> none) */
  double kkt_target;      /* final strict-KKT acceptance, in units of lambda; 0 -> 1e-4 */
  int32_t strategy;       /* dcdl_select; 0 -> LGCD.  GREEDY and CYCLIC override tile, RANDOM
                             ignores tile and inner.  Only dicodile_csc (and dicodile_cdl's CSC
                             steps) accept a rule other than LGCD */
  int32_t refresh_limit;  /* at most this many periodic drift corrections (0 -> no limit); with
                             refresh_every = S and refresh_limit = 1 the solve corrects beta once,
                             after S sweeps, and then runs to the certificate */
  uint64_t seed;          /* seed of the RANDOM rule's generator */
  uint64_t *audit;        /* optional device buffer (dicodile_csc only; NULL = off) of audit_rounds x
                             W1 x W2 records of the first launch's rounds, for checking the soft-lock
                             (Prop. A.2): record [r][w] is 0 if worker w (row-major in the worker grid
                             info->grid) published no candidate in round r; otherwise bit 63 is set,
                             bit 62 is set if the candidate passed the soft-lock test and was applied,
                             bits 32..47 hold its atom and bits 0..31 its position h W + w on the valid
                             domain.  Rounds the launch did not reach keep the caller's contents */
  int32_t audit_rounds;   /* rounds recorded (from round 0 of the first launch) */
  int32_t fp64_method;    /* how the FP64 contractions (drift corrections, checks, warm start) run:
                             0 -> by FFT where DCDL_CORR_F64_FFT applies and its estimated time is
                             below the FP64 matrix cores', 1 -> FP64 matrix cores only, 2 -> by FFT
                             wherever it applies.  The arithmetic is FP64 either way */
} dcdl_csc_opts;

/* Filled by dicodile_csc when `info` is not NULL (host memory). */
typedef struct {
  int64_t n_updates;      /* accepted coordinate updates */
  int64_t n_candidates;   /* candidates with score >= tol */
  int64_t n_softlocked;   /* candidates rejected by the soft-lock test */
  int64_t n_rounds;       /* rounds of the busiest worker */
  int64_t n_sweeps;       /* completed sweeps (every sub-domain visited once) */
  int64_t n_nonzero;      /* non-zeros of the returned Z */
  double objective;       /* FP64 F(Z) of the returned Z */
  double kkt;             /* FP64 strict KKT violation of the returned Z, / lambda */
  double lambda_max;      /* FP64 ||corr(X, D)||_inf (one-sided if positive) */
  double t_total_s;       /* wall time of the call */
  double t_init_s;        /* DtD, beta init */
  double t_cd_s;          /* coordinate-descent rounds */
  double t_check_s;       /* final FP64 objective / KKT check (and refreshes) */
  int32_t converged;      /* 1: exit certificate met and final check passed */
  int32_t grid[2];        /* worker grid used */
  int32_t tile[2];        /* sub-domain size used */
  int32_t n_passes;       /* solve passes (1 + polish passes) */
  int32_t n_fft64;        /* FP64 contractions that ran by FFT (the initialisation included) */
  int64_t n_visits;       /* sub-domain visits (worker rounds with a sub-domain to scan) */
  int64_t n_checked;      /* positions read by soft-lock tests */
  int64_t n_patched;      /* positions of beta patched by accepted updates */
  double t_worker_wait_s;    /* per-worker average time waiting on neighbours' progress */
  double t_worker_select_s;  /* ... selecting, soft-lock testing and publishing candidates */
  double t_worker_collect_s; /* ... waiting for the neighbours' candidates */
  double t_worker_apply_s;   /* ... applying accepted updates to beta, z and the move cache */
  double beta_drift;         /* at the first FP64 check: max |beta kept by the rounds - (corr(X - Z*D, D)
                                + n z) in FP64|, / lambda: the error of the incremental beta against
                                its FP64 definition (NaN if no check ran) */
  double t_init_corr_s;      /* HIP-event time of the contraction that initialised beta (0 after a
                                warm start, whose beta comes from an FP64 contraction counted below) */
  double t_corr64_s;         /* HIP-event time of the FP64 contractions: every check, drift correction
                                and warm start, summed */
  int32_t n_corr64;          /* number of those FP64 contractions */
  int32_t init_prec;         /* dcdl_corr_prec the initialisation ran at (AUTO and fallbacks resolved) */
  double t_check_inc_s;      /* HIP-event time of the incremental FP64 checks: after a dense FP64
                                contraction, a later check carries its FP64 gradient and residual
                                forward over the coordinates changed since (eq. beta_update in FP64)
                                instead of contracting again, while that is the cheaper path */
  int32_t n_check_inc;       /* number of those incremental checks */
  int32_t n_changed;         /* coordinates carried forward by the last incremental check */
} dcdl_csc_info;

/* Library version string (static storage). */
const char *dicodile_version(void);

/* Message of the last error on the calling thread ("" if none). */
const char *dicodile_last_error(void);

/* Release the library's own device resources on every device it has used:
 * each device is synchronised, its workspace buffers are freed and the
 * library-owned stream is destroyed; the caller's current device is kept.
 * Servers are not touched (dicodile_server_destroy).  Call it before the HIP
 * runtime is torn down (the Python binding does so at interpreter exit); the
 * next call re-creates what it needs.  DCDL_EHIP if a HIP call fails (the
 * remaining resources are still released). */
int dicodile_release(void);

/* DtD (Sec. 3, the kernel of eq. beta_update):
 *   dtd[k0][k][tau + L - 1] = sum_p sum_t D_{k0,p}[t] D_{k,p}[t + tau],
 *   tau in Phi = [-L+1, L-1]^d.
 * D: (K, P, L...) device, dtype.  dtd_out: (K, K, 2L1-1[, 2L2-1]) device, dtype.
 * Computed in FP64 on the matrix cores (one correlation of D with an image of
 * the atoms laid side by side, zero-padded), or by direct FP64 loops for
 * atoms whose staged windows exceed the matrix-core LDS budget; rounded once
 * to dtype. */
int dicodile_dtd(const dcdl_shape *shape, dcdl_dtype dtype, const void *D, void *dtd_out,
                 void *stream);

/* lambda_max = max_{k,w} |corr(X, D)_k[w]| (Sec. 2, CSC paragraph: for
 * lambda >= lambda_max the zero activation is optimal).  positive = 1 gives
 * the one-sided bound max(max corr, 0).  Computed in FP64 whatever dtype X
 * and D have.  out: host double. */
int dicodile_lambda_max(const dcdl_shape *shape, dcdl_dtype dtype, const void *X, const void *D,
                        int32_t positive, double *out, void *stream);

/* Solve eq. csc with LGCD + soft-lock on a grid of workgroups (Alg. 1, Alg. 3).
 * X: (P, T...) device, opts->dtype.  D: (K, P, L...) device, opts->dtype.
 * z_out: (K, T-L+1 ...) device, opts->dtype; read first if opts->warm_start.
 * info: host, may be NULL.
 * Returns DCDL_OK when the sweep certificate (no move scoring >= tol) and the
 * FP64 final check (strict KKT <= kkt_target) both hold; DCDL_NOT_CONVERGED
 * with the current iterate in z_out when a cap stopped it.  The incremental
 * beta and Z are kept in opts->dtype; the final objective/KKT are FP64. */
int dicodile_csc(const dcdl_shape *shape, const void *X, const void *D,
                 const dcdl_csc_opts *opts, void *z_out, dcdl_csc_info *info, void *stream);

/* Size of the fixed device scratch of dicodile_csc_noalloc: 64 MiB. */
#define DCDL_NOALLOC_SCRATCH_BYTES (64ull << 20)

/* dicodile_csc for callers that cannot allocate device memory: serving loops
 * and harnesses that forbid hipMalloc (the solve reads its convergence state
 * on the host between passes, so it cannot be recorded into a HIP graph).
 * Same arguments, kernels and results as dicodile_csc.  Every workspace (beta,
 * z, the move cache, the update table, DtD, the worker protocol state, the
 * packed dictionaries, the FP64 residual) is carved from a fixed
 * DCDL_NOALLOC_SCRATCH_BYTES array in device memory that each device holds for
 * the life of the process; the call makes no hipMalloc, hipFree or other
 * allocating call (its first call on a device looks the array's address up
 * and creates the seven timing events it reuses; dicodile_release drops
 * them).  The workspace of a solve is about 2 HW KS s + HW (s + 4) +
 * K (2L1-1)(2L2-1)(K + KS) s + 8 P T1 T2 bytes (s = 4 or 8 bytes, KS = K
 * rounded up to 16 bytes of atoms): for example 1-D signals of T = 5000 with
 * K = 5 atoms, or images up to about 480x480 with K = 25 atoms of 16x16 in
 * FP32.  DCDL_EINVAL, before any device access, when the solve needs more.
 * The scratch keeps the last call's contents; every call initialises what it
 * reads.  Calls on one device share the array: two that overlapped would
 * race, but the library serialises its calls on a device and each returns
 * after its work has completed. */
int dicodile_csc_noalloc(const dcdl_shape *shape, const void *X, const void *D,
                         const dcdl_csc_opts *opts, void *z_out, dcdl_csc_info *info, void *stream);

/* Dense correlation G = corr(X, D) (Sec. 2: the paper's X * D~_k; beta at
 * Z = 0, and the gradient -G of the data term):
 *   G[k][w] = sum_p sum_t D_{k,p}[t] X_p[w + t],  w on the valid domain.
 * X: (P, T...) device, dtype.  D: (K, P, L...) device, dtype.
 * out: (K, T-L+1 ...) device, dtype.  prec: dcdl_corr_prec (the BF16 paths
 * need dtype F32).  For measuring the matrix-core contraction and its error. */
int dicodile_corr(const dcdl_shape *shape, dcdl_dtype dtype, const void *X, const void *D, void *out,
                  int32_t prec, void *stream);

/* FP64 objective F(Z) = 1/2||X - Z*D||^2 + lambda ||Z||_1 and strict KKT
 * violation / lambda (with g = corr(X - Z*D, D): max(|g| - lambda, 0) on
 * zeros, |g - lambda sign Z| on the support; one-sided if positive).
 * X, D, z: device, dtype.  objective, kkt: host doubles (either may be NULL). */
int dicodile_objective_kkt(const dcdl_shape *shape, dcdl_dtype dtype, const void *X,
                           const void *D, const void *z, double lambda, int32_t positive,
                           double *objective, double *kkt, void *stream);

/* Sufficient statistics of the dictionary update (Sec. 4.2, eq. phi):
 *   ztz[k][k'][tau + L - 1] = sum_w Z_k[w] Z_k'[w + tau],  tau in Phi
 *   ztX[k][p][t]            = sum_w Z_k[w] X_p[w + t],     t in Theta
 * z: (K, T-L+1 ...) device, dtype.  X: (P, T...) device, dtype.
 * ztz_out: (K, K, 2L-1 ...) device, dtype.  ztX_out: (K, P, L...) device, dtype.
 * Accumulation is in FP64 over the non-zeros of z. */
int dicodile_dict_stats(const dcdl_shape *shape, dcdl_dtype dtype, const void *z, const void *X,
                        void *ztz_out, void *ztX_out, void *stream);

/* ------------------------------------------------------- dictionary update */

/* Options of dicodile_dict_update.  Zero-initialise for defaults. */
typedef struct {
  int32_t max_iter;   /* projected-gradient iterations at most; 0 -> 500 */
  int32_t reserved;
  double tol;         /* stop when an iteration decreases F by less than tol * max(1, F); 0 -> 1e-10 */
  double c1;          /* Armijo sufficient-decrease constant in (0, 1); 0 -> 1e-4 */
} dcdl_dict_opts;

/* Filled by dicodile_dict_update when not NULL (host memory). */
typedef struct {
  int32_t iterations;   /* accepted projected-gradient steps */
  int32_t backtracks;   /* halvings of the step over all iterations */
  double cost_initial;  /* F(D) = 1/2 ||X - Z*D||^2 at the projected input D */
  double cost;          /* F at the returned D */
  double t_s;           /* wall time of the call */
} dcdl_dict_info;

/* Dictionary update of eq. dict_update (Sec. 4.2):
 *   D = argmin_{||D_k||_2 <= 1} 1/2 ||X - Z*D||^2
 * from the sufficient statistics of eq. phi alone (no signal-size work):
 *   F(D) = 1/2 ||X||^2 - <D, ztX> + 1/2 <D, Q(D)>,  grad F = Q(D) - ztX,
 *   Q(D)_{k,p}[t] = sum_{k'} sum_{t'} ztz[k][k'][t - t' + L - 1] D_{k',p}[t'].
 * Projected gradient descent with an Armijo backtracking line search along the
 * projection arc (the paper's PGD + Armijo): the trial D(a) = Proj(D - a grad F)
 * is accepted when F(D(a)) <= F(D) + c1 <grad F(D), D(a) - D>; a starts at twice
 * the last accepted step (the first at 1 / max_k sum_{k', tau} |ztz[k][k'][tau]|,
 * an upper bound of the largest eigenvalue of the quadratic form) and halves on
 * rejection.  Proj scales atoms of norm above 1 back to the unit sphere.
 * dict_shape: ndim, P, K, L of D (T is ignored).  ztz (K, K, 2L-1 ...) and
 * ztX (K, P, L ...): device, dtype, as dicodile_dict_stats writes them.
 * x_sq: ||X||^2 (host; it only shifts the reported costs).  D_inout: (K, P, L ...)
 * device, dtype: the start on entry, the result on return.  All arithmetic is
 * FP64.  Needs |Theta| <= 2048 taps. */
int dicodile_dict_update(const dcdl_shape *dict_shape, dcdl_dtype dtype, const void *ztz, const void *ztX,
                         double x_sq, void *D_inout, const dcdl_dict_opts *opts, dcdl_dict_info *info,
                         void *stream);

/* Options of dicodile_cdl.  Zero-initialise for defaults. */
typedef struct {
  double lambda_frac;     /* lambda = lambda_frac * lambda_max(X, D_start), fixed for the run; 0 -> 0.1 */
  double nu;              /* stop when an outer iteration lowers the objective by less than nu times
                             its previous value; 0 -> 1e-4 */
  int32_t max_outer;      /* outer iterations at most; 0 -> 20 (at most 64) */
  int32_t no_warm_start;  /* 1: every CSC step starts from Z = 0 (default: from the previous Z) */
  double tol_rel;         /* CSC tolerance in units of lambda; 0 -> 1e-5 */
  dcdl_csc_opts csc;      /* the CSC step's other options (lambda, tol, dtype, warm_start are set here) */
  dcdl_dict_opts dict;    /* the dictionary update's options */
} dcdl_cdl_opts;

/* Filled by dicodile_cdl when not NULL (host memory). */
typedef struct {
  int32_t outer;             /* outer iterations run */
  int32_t converged;         /* 1: stopped by nu */
  double lambda;             /* the lambda used */
  double objective[64];      /* 1/2 ||X - Z*D||^2 + lambda ||Z||_1 after each dictionary update */
  double objective_z[64];    /* ... after each CSC step (FP64 check) */
  double t_total_s, t_csc_s, t_stats_s, t_dict_s;
  int64_t n_updates;         /* coordinate updates over all CSC steps */
} dcdl_cdl_info;

/* Convolutional dictionary learning, Alg. 2: alternate the CSC step
 * (dicodile_csc with lambda fixed as above; warm-started from the previous Z),
 * the statistics of eq. phi and the dictionary update, until the relative
 * decrease of the objective over one outer iteration is below nu.
 * X: (P, T ...) device, dtype.  D_inout: (K, P, L ...) device, dtype: the start
 * (projected onto the feasible set) on entry, the learned dictionary on return.
 * z_out: (K, T-L+1 ...) device, dtype: the last CSC step's Z.  Returns DCDL_OK
 * when stopped by nu, DCDL_NOT_CONVERGED at max_outer. */
int dicodile_cdl(const dcdl_shape *shape, dcdl_dtype dtype, const void *X, void *D_inout, void *z_out,
                 const dcdl_cdl_opts *opts, dcdl_cdl_info *info, void *stream);

/* Batch-level options of dicodile_csc_batch.  Zero-initialise for defaults. */
typedef struct {
  int32_t no_graph;     /* 1: enqueue the per-instance set-up and check kernels directly
                           instead of recording them as HIP graphs */
  int32_t workers;      /* workgroups spread over the instances; 0 -> every co-resident slot */
  int32_t threads;      /* threads per worker workgroup (64, 128, 192, 256, 512, 1024); 0 -> 256 */
  int32_t tile[2];      /* sub-domain size; 0 -> 2 L_i (Sec. 3) */
  int32_t max_polish;   /* extra passes for instances failing the final check; 0 -> 2 */
  int32_t inner;        /* sub-domain visits per worker per round; 0 -> 1 */
  int32_t reserved;
} dcdl_batch_opts;

/* Filled by dicodile_csc_batch when not NULL (host memory). */
typedef struct {
  double t_total_s;     /* wall time of the call */
  double t_setup_s;     /* DtD, beta init and move caches of every instance */
  double t_rounds_s;    /* the persistent round launch(es) */
  double t_check_s;     /* FP64 checks and output transposes */
  int64_t n_updates;    /* summed over instances */
  int64_t workers;      /* workgroups of the first launch */
  int32_t n_converged;  /* instances that passed the sweep certificate and the KKT target */
  int32_t n_passes;     /* launches of the round kernel */
  int32_t used_graph;   /* 1 if the set-up and check passes ran as HIP graphs */
  int32_t reserved;
} dcdl_batch_info;

/* Solve n independent instances of eq. csc that share the dictionary D, in one
 * persistent launch of the round kernel whose workgroups are spread over the
 * instances (each instance runs its own worker grid, soft-lock rounds and
 * stopping consensus, Alg. 3).  All shapes share ndim, P, K and L; only T
 * differs.  X and z_out are host arrays of n device pointers; D is one device
 * pointer; opts holds n per-instance options (lambda, tol, positive, certify,
 * dtype, kkt_target, timeout_s as a wall-clock cap on each round launch of
 * that instance; dtype must agree; the first instance's beta_prec applies to
 * all); infos (host, may be NULL) receives n
 * records.  Returns DCDL_OK if every instance converged, DCDL_NOT_CONVERGED if
 * some hit a cap (their z holds the iterate).  For callers that hold many
 * small or medium solves at once: batching fills the chip where one solve at
 * a time would not. */
int dicodile_csc_batch(int32_t n, const dcdl_shape *shapes, const void *const *X, const void *D,
                       const dcdl_csc_opts *opts, void *const *z_out, dcdl_csc_info *infos,
                       const dcdl_batch_opts *bopts, dcdl_batch_info *binfo, void *stream);

/* Filled by dicodile_csc_batch_autotune when not NULL (host memory). */
typedef struct {
  int32_t n_trials;     /* candidate configurations timed */
  int32_t n_sample;     /* instances in the timing sample */
  double t_tune_s;      /* wall time of the call */
  double trial_budget_s;/* round-launch time budget of one trial */
  double obj_default;   /* summed FP64 objective of the sample after one trial budget with tile
                           2 L, 256 threads and every co-resident workgroup (mean of two runs) */
  double obj_best;      /* ... with the chosen configuration (<= obj_default); a configuration
                           other than the default is chosen only when it is lower by more than
                           3 obj_spread */
  int32_t cached;       /* 1: answered from the per-process cache, nothing timed */
  int32_t reserved;
  double obj_spread;    /* |difference| of the default's two runs: the run-to-run noise */
} dcdl_tune_info;

/* Autotuner of dicodile_csc_batch.  Runs candidate configurations on a
 * sample of up to 12 instances spread over the batch's size range, with the
 * worker budget scaled to the sample's share of the area (so that every
 * sampled instance gets the worker grid it gets in the whole batch), each for
 * the same short time budget, and keeps the one whose sample reaches the
 * lowest summed FP64 objective (the most progress in equal time):
 * sub-domain tiles of 1.5, 2, 3 and 4 L_i, then 128 vs 256 threads per
 * worker, then the whole vs half the co-resident budget (fewer, larger
 * workers per instance).  Writes the winner into *best (the other fields of
 * *base are kept; base may be NULL).  Arguments as dicodile_csc_batch, without
 * outputs: the sample's solutions go to a library workspace.  Results are
 * cached for the process per (ndim, P, K, L, dtype, mean size class, count
 * class); a cached answer times nothing. */
int dicodile_csc_batch_autotune(int32_t n, const dcdl_shape *shapes, const void *const *X, const void *D,
                                const dcdl_csc_opts *opts, const dcdl_batch_opts *base,
                                dcdl_batch_opts *best, dcdl_tune_info *info, void *stream);

/* ------------------------------------------------------------------ serving
 * A server solves a stream of eq. csc requests that share one dictionary,
 * with continuous batching: requests are admitted while others run, as lanes
 * and HBM free up, and every launch of the round kernel runs up to
 * slice_rounds rounds of every admitted request that is ready (each on its
 * own worker grid, with its own soft-lock rounds and stopping consensus,
 * Alg. 3).  Between launches finished requests leave and new ones join; a
 * request's stopping state carries over from one launch to the next.  Set-up
 * (beta, move cache), the FP64 final check, drift-corrected polish passes and
 * the output transpose of one request run on a second stream while the rounds
 * of the others run.  The dictionary, its DtD table, beta, z and the cache of
 * every admitted request stay resident in HBM.
 *
 * Threading: the server runs its own host thread; submit, poll and wait may
 * be called from any thread.  A server holds device memory until destroyed. */
typedef struct dcdl_server dcdl_server;

/* Server options.  Zero-initialise for defaults. */
typedef struct {
  int64_t hbm_budget_bytes; /* device memory reserved for the working sets of admitted requests
                               (beta, z, move cache: about 2 K s + 8 bytes per position, s the
                               element size); 0 -> half of the free device memory */
  int64_t max_len;          /* positions T (d = 1) or T1*T2 (d = 2) of the largest request; sizes
                               the shared FP64 residual of the checks; 0 -> 2^20 */
  int32_t max_workers;      /* workgroups of one request at most; 0 -> 128 */
  int32_t slice_rounds;     /* rounds per launch between admissions; 0 -> 64 */
  int32_t max_active;       /* admitted requests at most; 0 -> 256 */
  int32_t threads;          /* threads per worker workgroup (64, 128, 192, 256); 0 -> 256 */
  int32_t tile[2];          /* sub-domain size; 0 -> 2 L_i (d = 1: tile[0] is the length) */
  int32_t max_polish;       /* extra passes for requests failing the final check; 0 -> 2 */
  int32_t admit_workers;    /* admission stops while the admitted requests' workgroups would exceed
                               this (the first request is always admitted); 0 -> the co-resident
                               capacity of one launch, so the admitted set advances together in
                               one launch; -1 -> no bound (only lanes and memory limit admission).
                               Launch slots go to the oldest ready requests first */
} dcdl_server_opts;

/* Counters of a server since its creation (host memory). */
typedef struct {
  int64_t n_submitted;
  int64_t n_done;
  int64_t n_launches;       /* launches of the round kernel */
  int64_t peak_active;      /* most requests admitted at once */
  int64_t peak_bytes;       /* most HBM budget in use at once */
  int64_t peak_workers;     /* most workgroups in one launch */
  double t_rounds_s;        /* summed duration of the round launches (HIP events) */
  double t_busy_s;          /* host time with at least one admitted request */
} dcdl_server_stats;

/* Create a server on the current device.  dict_shape gives ndim, P, K and L of
 * the dictionary (T is ignored); D: (K, P, L...) device, dtype; the server
 * keeps its own copy.  *out receives the handle. */
int dicodile_server_create(const dcdl_shape *dict_shape, dcdl_dtype dtype, const void *D,
                           const dcdl_server_opts *opts, dcdl_server **out);

/* Queue one request.  shape: ndim, P, K, L as the server's dictionary, any T.
 * X: (P, T...) device, opts->dtype, complete (synchronised) before the call;
 * z_out: (K, T-L+1 ...) device, opts->dtype.  Both must stay valid until the
 * request has finished (poll or wait returned something other than
 * DCDL_PENDING).  opts: as dicodile_csc (lambda, tol, positive, certify,
 * dtype = the server's, kkt_target, max_rounds, timeout_s; warm_start is not
 * supported).  *ticket identifies the request.  DCDL_ENOMEM if its working
 * set exceeds the whole HBM budget. */
int dicodile_server_submit(dcdl_server *sv, const dcdl_shape *shape, const void *X,
                           const dcdl_csc_opts *opts, void *z_out, uint64_t *ticket);

/* DCDL_PENDING while the request runs.  Otherwise its result as dicodile_csc
 * returns it, with info (host, may be NULL) filled; info->t_total_s is the
 * time from submit to z_out ready and info->t_init_s the time spent queued
 * before admission.  A finished ticket is forgotten after this call. */
int dicodile_server_poll(dcdl_server *sv, uint64_t ticket, dcdl_csc_info *info);

/* As poll, blocking until the request finishes or timeout_s (> 0) passes
 * (then DCDL_PENDING). */
int dicodile_server_wait(dcdl_server *sv, uint64_t ticket, double timeout_s, dcdl_csc_info *info);

/* Counters since creation. */
int dicodile_server_stats(dcdl_server *sv, dcdl_server_stats *stats);

/* Finish every queued and running request, stop the server thread and free
 * the server's device memory.  Unretrieved results are dropped. */
int dicodile_server_destroy(dcdl_server *sv);

/* Streaming copy dst = src of `bytes` bytes (16-byte aligned, a multiple of
 * 16), `repeats` times; *seconds (host, may be NULL) receives the average time
 * of one copy measured with HIP events.  Reads + writes 2*bytes of HBM per
 * copy: the achievable-bandwidth reference of the roofline figures and the
 * calibration kernel of the traffic counters. */
int dicodile_copy_probe(void *dst, const void *src, size_t bytes, int32_t repeats, double *seconds,
                        void *stream);

#ifdef __cplusplus
}
#endif

#endif /* DICODILE_MI355X_H */
