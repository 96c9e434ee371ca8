/*
 * csc_oracle.c -- sequential FP64 reference for the convolutional sparse
 * coding (CSC) step of DiCoDiLe (Moreau & Gramfort, "Distributed
 * Convolutional Dictionary Learning (DiCoDiLe): Pattern Discovery in Large
 * Images and Signals", arXiv:1901.09235).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this file.  It shares no code,
 * header, table or helper with the GPU library, and the GPU library never
 * calls it.
 *
 * Every routine is a plain, single-threaded loop nest in double precision
 * that writes out the definition it cites, with no blocking, fusion or
 * reordering beyond what the definition states.
 *
 * Conventions (0-based; 1-D signals are the case T1 = 1, L1 = 1):
 *   X  (P, T1, T2)               observation, Sec. 2 "Convolutional Linear Model"
 *   D  (K, P, L1, L2)            dictionary, atoms on Theta = [0,L1[ x [0,L2[
 *   Z  (K, H, W)                 activations on the valid domain
 *                                H = T1 - L1 + 1, W = T2 - L2 + 1
 *   (Z*D)_p[x] = sum_k sum_t Z_k[x - t] D_{k,p}[t]     (Sec. 2, eq. model)
 *   corr(R, D)_k[w] = sum_p sum_t D_{k,p}[t] R_p[w + t] (the paper's R * D~_k)
 *   C[k0][k][tau + L - 1] = sum_p sum_t D_{k0,p}[t] D_{k,p}[t + tau],
 *                           tau in [-L+1, L-1]          (Sec. 3, eq. beta_update)
 *   beta = corr(X - Z*D, D) + n (.) Z,  n_k = ||D_k||^2  (Sec. 3, definition of beta)
 *
 * The reading that Z lives on the valid domain (so that every shifted atom
 * has squared norm n_k, as Prop. A.1 uses) and the other readings of the
 * paper are listed in the design notes of the repository.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define IDX3(a, b, c, B, C) ((((int64_t)(a)) * (B) + (b)) * (C) + (c))
#define IDX4(a, b, c, d, B, C, Dd) (((((int64_t)(a)) * (B) + (b)) * (C) + (c)) * (Dd) + (d))

static double now_s(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/* n_k = ||D_k||_2^2 (the denominator of eq. pb_coord). */
void orc_atom_norms(int K, int P, int L1, int L2, const double *D, double *n) {
  for (int k = 0; k < K; ++k) {
    double s = 0.0;
    for (int p = 0; p < P; ++p)
      for (int t1 = 0; t1 < L1; ++t1)
        for (int t2 = 0; t2 < L2; ++t2) {
          double d = D[IDX4(k, p, t1, t2, P, L1, L2)];
          s += d * d;
        }
    n[k] = s;
  }
}

/* DtD: C[k0][k][tau] = (D_k0 * D~_k) restricted to Phi = [-L+1, L-1]
 * (Sec. 3, the kernel of eq. beta_update), stored at tau + L - 1. */
void orc_dtd(int K, int P, int L1, int L2, const double *D, double *C) {
  const int U1 = 2 * L1 - 1, U2 = 2 * L2 - 1;
  for (int k0 = 0; k0 < K; ++k0)
    for (int k = 0; k < K; ++k)
      for (int tau1 = -(L1 - 1); tau1 <= L1 - 1; ++tau1)
        for (int tau2 = -(L2 - 1); tau2 <= L2 - 1; ++tau2) {
          double s = 0.0;
          for (int p = 0; p < P; ++p)
            for (int t1 = 0; t1 < L1; ++t1)
              for (int t2 = 0; t2 < L2; ++t2) {
                int s1 = t1 + tau1, s2 = t2 + tau2;
                if (s1 < 0 || s1 >= L1 || s2 < 0 || s2 >= L2) continue;
                s += D[IDX4(k0, p, t1, t2, P, L1, L2)] * D[IDX4(k, p, s1, s2, P, L1, L2)];
              }
          C[IDX4(k0, k, tau1 + L1 - 1, tau2 + L2 - 1, K, U1, U2)] = s;
        }
}

/* G_k[w] = corr(R, D)_k[w] = sum_p sum_t D_{k,p}[t] R_p[w + t] for w on the
 * valid domain.  With R = X this is the initial beta of Alg. 1 and the
 * quantity whose sup-norm is lambda_max (Sec. 2, CSC paragraph). */
void orc_corr(int P, int64_t T1, int64_t T2, int K, int L1, int L2,
              const double *R, const double *D, double *G) {
  const int64_t H = T1 - L1 + 1, W = T2 - L2 + 1;
  for (int k = 0; k < K; ++k)
    for (int64_t w1 = 0; w1 < H; ++w1)
      for (int64_t w2 = 0; w2 < W; ++w2) {
        double s = 0.0;
        for (int p = 0; p < P; ++p)
          for (int t1 = 0; t1 < L1; ++t1)
            for (int t2 = 0; t2 < L2; ++t2)
              s += D[IDX4(k, p, t1, t2, P, L1, L2)] * R[IDX3(p, w1 + t1, w2 + t2, T1, T2)];
        G[IDX3(k, w1, w2, H, W)] = s;
      }
}

/* out = Z*D (eq. model without noise): out_p[x] = sum_k sum_t Z_k[x-t] D_{k,p}[t].
 * Terms with Z_k[w] = 0 contribute nothing and are skipped. */
void orc_reconstruct(int P, int64_t T1, int64_t T2, int K, int L1, int L2,
                     const double *Z, const double *D, double *out) {
  const int64_t H = T1 - L1 + 1, W = T2 - L2 + 1;
  memset(out, 0, sizeof(double) * (size_t)(P * T1 * T2));
  for (int k = 0; k < K; ++k)
    for (int64_t w1 = 0; w1 < H; ++w1)
      for (int64_t w2 = 0; w2 < W; ++w2) {
        double z = Z[IDX3(k, w1, w2, H, W)];
        if (z == 0.0) continue;
        for (int p = 0; p < P; ++p)
          for (int t1 = 0; t1 < L1; ++t1)
            for (int t2 = 0; t2 < L2; ++t2)
              out[IDX3(p, w1 + t1, w2 + t2, T1, T2)] += z * D[IDX4(k, p, t1, t2, P, L1, L2)];
      }
}

static void residual(int P, int64_t T1, int64_t T2, int K, int L1, int L2,
                     const double *X, const double *D, const double *Z, double *R) {
  orc_reconstruct(P, T1, T2, K, L1, L2, Z, D, R);
  for (int64_t i = 0; i < (int64_t)P * T1 * T2; ++i) R[i] = X[i] - R[i];
}

/* lambda_max = ||corr(X, D)||_inf (Sec. 2, CSC paragraph).  For the
 * non-negative variant the first-order condition at 0 only bounds the
 * positive side, so lambda_max = max(max corr, 0). */
double orc_lambda_max(int P, int64_t T1, int64_t T2, int K, int L1, int L2,
                      const double *X, const double *D, int positive) {
  const int64_t H = T1 - L1 + 1, W = T2 - L2 + 1, n = (int64_t)K * H * W;
  double *G = (double *)malloc(sizeof(double) * (size_t)n);
  orc_corr(P, T1, T2, K, L1, L2, X, D, G);
  double m = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double v = positive ? G[i] : fabs(G[i]);
    if (v > m) m = v;
  }
  free(G);
  return m;
}

/* F(Z) = 1/2 ||X - Z*D||_2^2 + lambda ||Z||_1 (Sec. 2, eq. csc). */
double orc_objective(int P, int64_t T1, int64_t T2, int K, int L1, int L2,
                     const double *X, const double *D, const double *Z, double lambda) {
  const int64_t H = T1 - L1 + 1, W = T2 - L2 + 1;
  double *R = (double *)malloc(sizeof(double) * (size_t)(P * T1 * T2));
  residual(P, T1, T2, K, L1, L2, X, D, Z, R);
  double f = 0.0, l1 = 0.0;
  for (int64_t i = 0; i < (int64_t)P * T1 * T2; ++i) f += R[i] * R[i];
  for (int64_t i = 0; i < (int64_t)K * H * W; ++i) l1 += fabs(Z[i]);
  free(R);
  return 0.5 * f + lambda * l1;
}

/* Strict KKT violation of eq. csc, divided by lambda.  With g = corr(X-Z*D, D)
 * (the negative gradient of the smooth part), optimality reads g in
 * lambda * d|Z|: |g| <= lambda where Z = 0 and g = lambda sign(Z) elsewhere.
 * Non-negative variant: g <= lambda where Z = 0 and g = lambda where Z > 0. */
double orc_kkt(int P, int64_t T1, int64_t T2, int K, int L1, int L2,
               const double *X, const double *D, const double *Z, double lambda,
               int positive) {
  const int64_t H = T1 - L1 + 1, W = T2 - L2 + 1, n = (int64_t)K * H * W;
  double *R = (double *)malloc(sizeof(double) * (size_t)(P * T1 * T2));
  double *G = (double *)malloc(sizeof(double) * (size_t)n);
  residual(P, T1, T2, K, L1, L2, X, D, Z, R);
  orc_corr(P, T1, T2, K, L1, L2, R, D, G);
  double worst = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double g = G[i], z = Z[i], v;
    if (z == 0.0)
      v = positive ? fmax(g - lambda, 0.0) : fmax(fabs(g) - lambda, 0.0);
    else
      v = fabs(g - lambda * (z > 0.0 ? 1.0 : -1.0));
    if (v > worst) worst = v;
  }
  free(R);
  free(G);
  return worst / lambda;
}

/* Soft-thresholding ST(u, lambda) = sign(u) max(|u| - lambda, 0) (Sec. 2,
 * Notations); its one-sided form for the non-negative variant. */
static double soft_threshold(double u, double lambda, int positive) {
  if (positive) return u > lambda ? u - lambda : 0.0;
  if (u > lambda) return u - lambda;
  if (u < -lambda) return u + lambda;
  return 0.0;
}

/* Coordinate update of eq. pb_coord: Z' = ST(beta, lambda) / ||D_k||^2. */
static double coord_target(double beta, double nk, double lambda, int positive) {
  return soft_threshold(beta, lambda, positive) / nk;
}

/* Selection score of a move Z -> Zn.  The paper selects and stops on
 * |Delta Z| (Alg. 1).  With certify = 1 a move that changes the support or
 * the sign of a non-zero coordinate scores at least tol, so it is never left
 * pending at exit; the remaining moves then all have |Delta Z| < tol with an
 * unchanged sign pattern, which bounds the strict KKT violation by
 * max_k n_k * tol (see orc_kkt). */
static double move_score(double z, double zn, double tol, int certify) {
  double dz = fabs(zn - z);
  if (certify && z != 0.0 && (zn == 0.0 || ((zn > 0.0) != (z > 0.0))))
    return dz > tol ? dz : tol;
  return dz;
}

/* Cost decrease of one coordinate update, Prop. A.1. */
static double delta_cost(double nk, double beta, double z, double zn, double lambda) {
  return 0.5 * nk * (z * z - zn * zn) - beta * (z - zn) + lambda * (fabs(z) - fabs(zn));
}

/* beta = corr(X - Z*D, D) + n (.) Z, the definition of beta in Sec. 3. */
void orc_beta(int P, int64_t T1, int64_t T2, int K, int L1, int L2,
              const double *X, const double *D, const double *Z, double *beta) {
  const int64_t H = T1 - L1 + 1, W = T2 - L2 + 1;
  double *n = (double *)malloc(sizeof(double) * (size_t)K);
  double *R = (double *)malloc(sizeof(double) * (size_t)(P * T1 * T2));
  orc_atom_norms(K, P, L1, L2, D, n);
  residual(P, T1, T2, K, L1, L2, X, D, Z, R);
  orc_corr(P, T1, T2, K, L1, L2, R, D, beta);
  for (int k = 0; k < K; ++k)
    for (int64_t i = 0; i < H * W; ++i) beta[(int64_t)k * H * W + i] += n[k] * Z[(int64_t)k * H * W + i];
  free(n);
  free(R);
}

/* Incremental beta update of eq. beta_update after Z_k0[w0] += delta:
 * beta_k[w] -= C[k0][k][w0 - w] * delta for every (k, w) != (k0, w0) with
 * w in V(w0) intersected with the valid domain. */
static void beta_patch(int K, int L1, int L2, int64_t H, int64_t W, const double *C,
                       int k0, int64_t a1, int64_t a2, double delta, double *beta) {
  const int U1 = 2 * L1 - 1, U2 = 2 * L2 - 1;
  int64_t lo1 = a1 - (L1 - 1), hi1 = a1 + L1, lo2 = a2 - (L2 - 1), hi2 = a2 + L2;
  if (lo1 < 0) lo1 = 0;
  if (lo2 < 0) lo2 = 0;
  if (hi1 > H) hi1 = H;
  if (hi2 > W) hi2 = W;
  for (int k = 0; k < K; ++k)
    for (int64_t w1 = lo1; w1 < hi1; ++w1)
      for (int64_t w2 = lo2; w2 < hi2; ++w2) {
        if (k == k0 && w1 == a1 && w2 == a2) continue;
        int u1 = (int)(a1 - w1) + L1 - 1, u2 = (int)(a2 - w2) + L2 - 1;
        beta[IDX3(k, w1, w2, H, W)] -= C[IDX4(k0, k, u1, u2, K, U1, U2)] * delta;
      }
}

typedef struct {
  int64_t n_updates;   /* coordinate updates applied */
  int64_t n_sweeps;    /* full passes over the M sub-domains */
  int32_t converged;   /* 1 if the last sweep applied no update */
  int32_t pad;
  double cost_decrease;   /* sum over updates of Prop. A.1's Delta E */
  double max_drift;       /* max |beta_incremental - beta_fresh| at checks */
  double t_solve_s;       /* wall time of the sweeps (checks excluded) */
  double t_kkt_s;         /* wall time at which the KKT target was first met, -1 if never */
  int64_t sweeps_kkt;     /* sweep count at that point, -1 if never */
} orc_lgcd_info;

/* Locally greedy coordinate descent, Alg. 1 (Sec. 3).
 *
 * Omega_Z is split into sub-domains C_m of tile1 x tile2 positions in raster
 * order, the last block of each dimension taking the remainder.  A sweep
 * visits m = 0..M-1 in order (cyclic rule).  In each C_m the coordinate with
 * the largest score is chosen (ties: lowest raster position, then lowest
 * atom index), and applied only if its score >= tol and Delta Z != 0.  The
 * score is |Delta Z| (the paper's rule) or, with certify = 1, the
 * move_score above.  The run stops after a sweep that applied no update,
 * which certifies ||Delta Z||_inf < tol at exit, or after max_sweeps
 * sweeps.
 *
 * warm_start = 1 takes Z as the initial iterate; otherwise Z starts at 0.
 * beta0, when not NULL, is beta of that initial iterate (its definition in
 * Sec. 3, computed by the caller) and replaces the direct computation.
 * check_every > 0 recomputes beta from its definition every check_every
 * sweeps and records the drift of the incremental beta (beta itself is not
 * replaced).  kkt_every > 0 evaluates the strict KKT violation every
 * kkt_every sweeps and records when it first drops to kkt_target or below.
 * Returns 0 on success, -1 on bad arguments or allocation failure. */
int orc_lgcd(int P, int64_t T1, int64_t T2, int K, int L1, int L2,
             const double *X, const double *D, double lambda, double tol,
             int positive, int tile1, int tile2, int64_t max_sweeps,
             int warm_start, int certify, int check_every, int kkt_every,
             double kkt_target, const double *beta0, double *Z, orc_lgcd_info *info) {
  if (P < 1 || K < 1 || L1 < 1 || L2 < 1 || T1 < L1 || T2 < L2 || tile1 < 1 || tile2 < 1 ||
      !(lambda > 0.0) || tol < 0.0)
    return -1;
  const int64_t H = T1 - L1 + 1, W = T2 - L2 + 1, nz = (int64_t)K * H * W;
  const int U1 = 2 * L1 - 1, U2 = 2 * L2 - 1;
  double *n = (double *)malloc(sizeof(double) * (size_t)K);
  double *C = (double *)malloc(sizeof(double) * (size_t)K * K * U1 * U2);
  double *beta = (double *)malloc(sizeof(double) * (size_t)nz);
  double *fresh = check_every > 0 ? (double *)malloc(sizeof(double) * (size_t)nz) : NULL;
  if (!n || !C || !beta || (check_every > 0 && !fresh)) {
    free(n); free(C); free(beta); free(fresh);
    return -1;
  }
  orc_atom_norms(K, P, L1, L2, D, n);
  orc_dtd(K, P, L1, L2, D, C);
  if (!warm_start) memset(Z, 0, sizeof(double) * (size_t)nz);
  if (beta0)
    memcpy(beta, beta0, sizeof(double) * (size_t)nz);
  else
    orc_beta(P, T1, T2, K, L1, L2, X, D, Z, beta);

  memset(info, 0, sizeof(*info));
  info->t_kkt_s = -1.0;
  info->sweeps_kkt = -1;
  const int64_t nb1 = (H + tile1 - 1) / tile1, nb2 = (W + tile2 - 1) / tile2;
  double t_run = 0.0;
  int64_t sweep = 0;
  int converged = 0;
  while (sweep < max_sweeps) {
    double t0 = now_s();
    int64_t applied = 0;
    for (int64_t m = 0; m < nb1 * nb2; ++m) {
      int64_t b1 = m / nb2, b2 = m % nb2;
      int64_t s1 = b1 * tile1, e1 = s1 + tile1 < H ? s1 + tile1 : H;
      int64_t s2 = b2 * tile2, e2 = s2 + tile2 < W ? s2 + tile2 : W;
      double best = -1.0, best_new = 0.0;
      int64_t a1 = -1, a2 = -1;
      int k0 = -1;
      for (int64_t w1 = s1; w1 < e1; ++w1)
        for (int64_t w2 = s2; w2 < e2; ++w2)
          for (int k = 0; k < K; ++k) {
            int64_t i = IDX3(k, w1, w2, H, W);
            double zn = coord_target(beta[i], n[k], lambda, positive);
            double sc = move_score(Z[i], zn, tol, certify);
            if (sc > best) {
              best = sc;
              best_new = zn;
              a1 = w1; a2 = w2; k0 = k;
            }
          }
      if (k0 < 0 || best < tol) continue;
      int64_t i0 = IDX3(k0, a1, a2, H, W);
      double z = Z[i0], delta = best_new - z;
      if (delta == 0.0) continue;
      info->cost_decrease += delta_cost(n[k0], beta[i0], z, best_new, lambda);
      beta_patch(K, L1, L2, H, W, C, k0, a1, a2, delta, beta);
      Z[i0] = best_new;
      ++applied;
    }
    t_run += now_s() - t0;
    ++sweep;
    info->n_updates += applied;
    if (check_every > 0 && sweep % check_every == 0) {
      orc_beta(P, T1, T2, K, L1, L2, X, D, Z, fresh);
      for (int64_t i = 0; i < nz; ++i) {
        double e = fabs(fresh[i] - beta[i]);
        if (e > info->max_drift) info->max_drift = e;
      }
    }
    if (kkt_every > 0 && info->sweeps_kkt < 0 && sweep % kkt_every == 0) {
      if (orc_kkt(P, T1, T2, K, L1, L2, X, D, Z, lambda, positive) <= kkt_target) {
        info->sweeps_kkt = sweep;
        info->t_kkt_s = t_run;
      }
    }
    if (applied == 0) {
      converged = 1;
      break;
    }
  }
  info->n_sweeps = sweep;
  info->converged = converged;
  info->t_solve_s = t_run;
  free(n); free(C); free(beta); free(fresh);
  return 0;
}

/* Counter-based generator of the randomized selection rule: SplitMix64
 * (Steele, Lea and Flood, "Fast splittable pseudorandom number generators",
 * OOPSLA 2014).  Its n-th output from the seed s is the mixing function
 *   z <- (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9
 *   z <- (z ^ (z >> 27)) * 0x94d049bb133111eb
 *   z <- z ^ (z >> 31)
 * applied to z = s + (n + 1) * 0x9e3779b97f4a7c15 (mod 2^64).  Stream j (one
 * per worker) uses the counter n + j * 2^40, so stream 0 is the plain
 * SplitMix64 sequence of s. */
uint64_t orc_draw(uint64_t seed, uint64_t stream, uint64_t n) {
  uint64_t z = seed + ((stream << 40) + n + 1) * 0x9e3779b97f4a7c15ULL;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

/* Randomized coordinate descent: the random selection rule Sec. 3 names
 * beside the cyclic and greedy ones, the "RCD" of the comparison in Sec. 5.
 *
 * Draw n = 0, 1, ... takes j = orc_draw(seed, 0, n) mod (K H W), the position
 * p = j / K of Omega_Z in raster order and the atom k = j mod K, and moves
 * Z_k[p] to its closed-form target (eq. pb_coord) when the move scores at
 * least tol and Delta Z != 0 (score as in orc_lgcd).  An epoch is H W draws;
 * after each one every coordinate is scored, and the run stops when none
 * scores >= tol with a non-zero move (the certificate of orc_lgcd's sweep
 * rule), or after max_epochs epochs.  info->n_sweeps counts epochs.
 * Returns 0 on success, -1 on bad arguments or allocation failure. */
int orc_rcd(int P, int64_t T1, int64_t T2, int K, int L1, int L2,
            const double *X, const double *D, double lambda, double tol,
            int positive, uint64_t seed, int64_t max_epochs, int certify,
            double *Z, orc_lgcd_info *info) {
  if (P < 1 || K < 1 || L1 < 1 || L2 < 1 || T1 < L1 || T2 < L2 || !(lambda > 0.0) || tol < 0.0)
    return -1;
  const int64_t H = T1 - L1 + 1, W = T2 - L2 + 1, HW = H * W, nz = (int64_t)K * HW;
  const int U1 = 2 * L1 - 1, U2 = 2 * L2 - 1;
  double *n = (double *)malloc(sizeof(double) * (size_t)K);
  double *C = (double *)malloc(sizeof(double) * (size_t)K * K * U1 * U2);
  double *beta = (double *)malloc(sizeof(double) * (size_t)nz);
  if (!n || !C || !beta) {
    free(n); free(C); free(beta);
    return -1;
  }
  orc_atom_norms(K, P, L1, L2, D, n);
  orc_dtd(K, P, L1, L2, D, C);
  memset(Z, 0, sizeof(double) * (size_t)nz);
  orc_beta(P, T1, T2, K, L1, L2, X, D, Z, beta);
  memset(info, 0, sizeof(*info));
  info->t_kkt_s = -1.0;
  info->sweeps_kkt = -1;
  const double t0 = now_s();
  uint64_t draw = 0;
  int converged = 0;
  int64_t epoch = 0;
  while (epoch < max_epochs) {
    for (int64_t q = 0; q < HW; ++q, ++draw) {
      const uint64_t j = orc_draw(seed, 0, draw) % (uint64_t)nz;
      const int64_t p = (int64_t)(j / (uint64_t)K);
      const int k = (int)(j % (uint64_t)K);
      const int64_t a1 = p / W, a2 = p % W;
      const int64_t i = IDX3(k, a1, a2, H, W);
      const double z = Z[i], zn = coord_target(beta[i], n[k], lambda, positive);
      if (move_score(z, zn, tol, certify) < tol || zn == z) continue;
      info->cost_decrease += delta_cost(n[k], beta[i], z, zn, lambda);
      beta_patch(K, L1, L2, H, W, C, k, a1, a2, zn - z, beta);
      Z[i] = zn;
      ++info->n_updates;
    }
    ++epoch;
    int moves = 0;
    for (int k = 0; k < K && !moves; ++k)
      for (int64_t p = 0; p < HW && !moves; ++p) {
        const int64_t i = IDX3(k, p / W, p % W, H, W);
        const double zn = coord_target(beta[i], n[k], lambda, positive);
        moves = move_score(Z[i], zn, tol, certify) >= tol && zn != Z[i];
      }
    if (!moves) {
      converged = 1;
      break;
    }
  }
  info->n_sweeps = epoch;
  info->converged = converged;
  info->t_solve_s = now_s() - t0;
  free(n); free(C); free(beta);
  return 0;
}

typedef struct {
  int64_t n_rounds;        /* bulk-synchronous rounds executed */
  int64_t n_sweeps;        /* sweeps (M_max rounds each) */
  int64_t n_candidates;    /* candidates with |Delta Z| >= tol */
  int64_t n_updates;       /* accepted and applied */
  int64_t n_softlocked;    /* rejected by the soft-lock test */
  int64_t n_interfering;   /* accepted pairs (w, w') with w' in V(w): must stay 0 with soft-locks */
  int32_t converged;
  int32_t diverged;        /* divergence guard tripped */
} orc_dz_info;

/* Balanced split of [0, N[ into Wn contiguous parts: part j starts at
 * floor(j N / Wn). */
static int64_t part_start(int64_t j, int64_t N, int64_t Wn) { return (j * N) / Wn; }

static int64_t part_owner(int64_t x, int64_t N, int64_t Wn) { return ((x + 1) * Wn - 1) / N; }

/* DiCoDiLe-Z, Alg. 3 (Sec. 4.1), executed on one core in bulk-synchronous
 * rounds: in each round every worker proposes its locally greedy candidate
 * (eq. gcd_candidate) from the same beta, the soft-lock test of eq. soft_lock
 * is evaluated against that same beta, and the accepted updates are then
 * applied with eq. beta_update.
 *
 * Workers form a W1 x W2 grid over Omega_Z (balanced split, row-major worker
 * index).  Worker w's domain S_w is cut into sub-domains of tile1 x tile2;
 * round r visits sub-domain (r mod M_max) of every worker, where M_max is the
 * largest sub-domain count, and a worker with fewer sub-domains idles.  A
 * sweep is M_max rounds; the run stops after a sweep with no candidate of
 * |Delta Z| >= tol anywhere (accepted or not).
 *
 * Soft-lock (eq. soft_lock): a candidate at w0 with V(w0) not inside S_w is
 * accepted iff its score is larger than the score of every (k, w) with w in
 * V(w0), in the valid domain and outside S_w; on equality the candidate of
 * the lower worker index wins.  The score is |Delta Z| or, with certify = 1,
 * move_score; selection and test use the same one, which is what makes two
 * workers agree on which of two mutually close candidates goes ahead.  soft_lock = 0 accepts every
 * candidate (the ablation of Sec. 5 "Impact of 2D grid partitioning"), with
 * the divergence guard ||Z||_inf > div_guard stopping the run.
 *
 * round_log, if not NULL, receives for each of the first log_rounds rounds
 * and each worker: k0, w0_1, w0_2, accepted (4 int64 per worker). */
int orc_dicodile_z(int P, int64_t T1, int64_t T2, int K, int L1, int L2,
                   const double *X, const double *D, double lambda, double tol,
                   int positive, int certify, int W1, int W2, int tile1, int tile2,
                   int soft_lock, double div_guard, int64_t max_rounds, double *Z, orc_dz_info *info,
                   int64_t *round_log, int64_t log_rounds) {
  const int64_t H = T1 - L1 + 1, W = T2 - L2 + 1, nz = (int64_t)K * H * W;
  if (P < 1 || K < 1 || L1 < 1 || L2 < 1 || T1 < L1 || T2 < L2 || W1 < 1 || W2 < 1 ||
      W1 > H || W2 > W || tile1 < 1 || tile2 < 1 || !(lambda > 0.0) || tol < 0.0)
    return -1;
  const int U1 = 2 * L1 - 1, U2 = 2 * L2 - 1;
  const int NW = W1 * W2;
  double *n = (double *)malloc(sizeof(double) * (size_t)K);
  double *C = (double *)malloc(sizeof(double) * (size_t)K * K * U1 * U2);
  double *beta = (double *)malloc(sizeof(double) * (size_t)nz);
  int64_t *ck = (int64_t *)malloc(sizeof(int64_t) * (size_t)NW * 3);
  double *cnew = (double *)malloc(sizeof(double) * (size_t)NW * 2);
  int *acc = (int *)malloc(sizeof(int) * (size_t)NW);
  if (!n || !C || !beta || !ck || !cnew || !acc) {
    free(n); free(C); free(beta); free(ck); free(cnew); free(acc);
    return -1;
  }
  orc_atom_norms(K, P, L1, L2, D, n);
  orc_dtd(K, P, L1, L2, D, C);
  memset(Z, 0, sizeof(double) * (size_t)nz);
  orc_beta(P, T1, T2, K, L1, L2, X, D, Z, beta);
  memset(info, 0, sizeof(*info));

  int64_t mmax = 0;
  for (int i = 0; i < W1; ++i)
    for (int j = 0; j < W2; ++j) {
      int64_t h = part_start(i + 1, H, W1) - part_start(i, H, W1);
      int64_t w = part_start(j + 1, W, W2) - part_start(j, W, W2);
      int64_t m = ((h + tile1 - 1) / tile1) * ((w + tile2 - 1) / tile2);
      if (m > mmax) mmax = m;
    }

  int64_t r = 0;
  int active_in_sweep = 0;
  while (r < max_rounds) {
    /* Selection: every worker picks its candidate from the same beta. */
    for (int wi = 0; wi < W1; ++wi)
      for (int wj = 0; wj < W2; ++wj) {
        int w = wi * W2 + wj;
        acc[w] = 0;
        ck[3 * w] = -1;
        int64_t l1 = part_start(wi, H, W1), u1 = part_start(wi + 1, H, W1);
        int64_t l2 = part_start(wj, W, W2), u2 = part_start(wj + 1, W, W2);
        int64_t nb2 = (u2 - l2 + tile2 - 1) / tile2;
        int64_t nb1 = (u1 - l1 + tile1 - 1) / tile1;
        int64_t m = r % mmax;
        if (m >= nb1 * nb2) continue;
        int64_t s1 = l1 + (m / nb2) * tile1, e1 = s1 + tile1 < u1 ? s1 + tile1 : u1;
        int64_t s2 = l2 + (m % nb2) * tile2, e2 = s2 + tile2 < u2 ? s2 + tile2 : u2;
        double best = -1.0, best_new = 0.0;
        int64_t a1 = -1, a2 = -1;
        int k0 = -1;
        for (int64_t w1 = s1; w1 < e1; ++w1)
          for (int64_t w2 = s2; w2 < e2; ++w2)
            for (int k = 0; k < K; ++k) {
              int64_t i = IDX3(k, w1, w2, H, W);
              double zn = coord_target(beta[i], n[k], lambda, positive);
              double sc = move_score(Z[i], zn, tol, certify);
              if (sc > best) {
                best = sc; best_new = zn; a1 = w1; a2 = w2; k0 = k;
              }
            }
        if (k0 < 0 || best < tol || best_new == Z[IDX3(k0, a1, a2, H, W)]) continue;
        active_in_sweep = 1;
        info->n_candidates++;
        ck[3 * w] = k0; ck[3 * w + 1] = a1; ck[3 * w + 2] = a2;
        cnew[2 * w] = best_new; cnew[2 * w + 1] = best;
        int ok = 1;
        if (soft_lock) {
          /* Soft-lock test over V(w0) \ S_w, read from the same beta. */
          int64_t lo1 = a1 - (L1 - 1), hi1 = a1 + L1, lo2 = a2 - (L2 - 1), hi2 = a2 + L2;
          if (lo1 < 0) lo1 = 0;
          if (lo2 < 0) lo2 = 0;
          if (hi1 > H) hi1 = H;
          if (hi2 > W) hi2 = W;
          for (int64_t w1 = lo1; w1 < hi1 && ok; ++w1)
            for (int64_t w2 = lo2; w2 < hi2 && ok; ++w2) {
              if (w1 >= l1 && w1 < u1 && w2 >= l2 && w2 < u2) continue;
              int owner = (int)(part_owner(w1, H, W1) * W2 + part_owner(w2, W, W2));
              for (int k = 0; k < K; ++k) {
                int64_t i = IDX3(k, w1, w2, H, W);
                double zn = coord_target(beta[i], n[k], lambda, positive);
                double sc = move_score(Z[i], zn, tol, certify);
                if (sc > best || (sc == best && owner < w)) {
                  ok = 0;
                  break;
                }
              }
            }
        }
        acc[w] = ok;
        if (!ok) info->n_softlocked++;
      }
    if (round_log && r < log_rounds)
      for (int w = 0; w < NW; ++w) {
        int64_t *e = round_log + (r * NW + w) * 4;
        e[0] = ck[3 * w]; e[1] = ck[3 * w + 1]; e[2] = ck[3 * w + 2]; e[3] = acc[w];
      }
    /* Interference audit (Prop. A.2): accepted pairs with w' in V(w). */
    for (int w = 0; w < NW; ++w) {
      if (!acc[w]) continue;
      for (int v = w + 1; v < NW; ++v) {
        if (!acc[v]) continue;
        int64_t d1 = ck[3 * w + 1] - ck[3 * v + 1], d2 = ck[3 * w + 2] - ck[3 * v + 2];
        if (d1 < 0) d1 = -d1;
        if (d2 < 0) d2 = -d2;
        if (d1 < L1 && d2 < L2) info->n_interfering++;
      }
    }
    /* Apply the accepted updates with eq. beta_update. */
    int diverged = 0;
    for (int w = 0; w < NW; ++w) {
      if (!acc[w]) continue;
      int k0 = (int)ck[3 * w];
      int64_t a1 = ck[3 * w + 1], a2 = ck[3 * w + 2];
      int64_t i0 = IDX3(k0, a1, a2, H, W);
      double delta = cnew[2 * w] - Z[i0];
      beta_patch(K, L1, L2, H, W, C, k0, a1, a2, delta, beta);
      Z[i0] = cnew[2 * w];
      info->n_updates++;
      if (div_guard > 0.0 && fabs(Z[i0]) > div_guard) diverged = 1;
    }
    ++r;
    if (diverged) {
      info->diverged = 1;
      break;
    }
    if (r % mmax == 0) {
      info->n_sweeps++;
      if (!active_in_sweep) {
        info->converged = 1;
        break;
      }
      active_in_sweep = 0;
    }
  }
  info->n_rounds = r;
  free(n); free(C); free(beta); free(ck); free(cnew); free(acc);
  return 0;
}

/* Sufficient statistics of the dictionary update, eq. phi (Sec. 4.2):
 *   phi[k][k'][tau + L - 1] = sum_w Z_k[w] Z_k'[w + tau],  tau in Phi
 *   psi[k][p][t]            = sum_w Z_k[w] X_p[w + t],     t in Theta
 * Terms with Z_k[w] = 0 contribute nothing and are skipped. */
void orc_dict_stats(int P, int64_t T1, int64_t T2, int K, int L1, int L2,
                    const double *Z, const double *X, double *phi, double *psi) {
  const int64_t H = T1 - L1 + 1, W = T2 - L2 + 1;
  const int U1 = 2 * L1 - 1, U2 = 2 * L2 - 1;
  memset(phi, 0, sizeof(double) * (size_t)K * K * U1 * U2);
  memset(psi, 0, sizeof(double) * (size_t)K * P * L1 * L2);
  for (int k = 0; k < K; ++k)
    for (int64_t w1 = 0; w1 < H; ++w1)
      for (int64_t w2 = 0; w2 < W; ++w2) {
        double z = Z[IDX3(k, w1, w2, H, W)];
        if (z == 0.0) continue;
        for (int kk = 0; kk < K; ++kk)
          for (int tau1 = -(L1 - 1); tau1 <= L1 - 1; ++tau1)
            for (int tau2 = -(L2 - 1); tau2 <= L2 - 1; ++tau2) {
              int64_t v1 = w1 + tau1, v2 = w2 + tau2;
              if (v1 < 0 || v1 >= H || v2 < 0 || v2 >= W) continue;
              double zz = Z[IDX3(kk, v1, v2, H, W)];
              if (zz == 0.0) continue;
              phi[IDX4(k, kk, tau1 + L1 - 1, tau2 + L2 - 1, K, U1, U2)] += z * zz;
            }
        for (int p = 0; p < P; ++p)
          for (int t1 = 0; t1 < L1; ++t1)
            for (int t2 = 0; t2 < L2; ++t2)
              psi[IDX4(k, p, t1, t2, P, L1, L2)] += z * X[IDX3(p, w1 + t1, w2 + t2, T1, T2)];
      }
}
