// dcdl_kernels.h -- gfx950 kernels around the round kernel: DtD, correlation
// (beta initialisation, drift correction, FP64 check, lambda_max), residual,
// layout changes, reductions and the dictionary statistics of Sec. 4.2.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dcdl_device.h"

namespace dcdl {

struct Geom {
  int P, K, L1, L2, U1, U2;
  int T1, T2, H, W;
  int KS;  // atom stride of position-major arrays (>= K)
};

// Non-negative doubles order like their bit patterns as unsigned integers.
__device__ __forceinline__ void atomic_max_nonneg(double *addr, double v) {
  atomicMax(reinterpret_cast<unsigned long long *>(addr), (unsigned long long)__double_as_longlong(v));
}

__device__ __forceinline__ void atomic_add_f64(double *addr, double v) { unsafeAtomicAdd(addr, v); }

template <int NT>
__device__ __forceinline__ double block_sum(double v, double *sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < NT / 64; ++q) s += sh[q];
  __syncthreads();
  return s;
}

template <int NT>
__device__ __forceinline__ double block_max(double v, double *sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = sh[0];
#pragma unroll
  for (int q = 1; q < NT / 64; ++q) s = fmax(s, sh[q]);
  __syncthreads();
  return s;
}

// --------------------------------------------------------------------- DtD
// One workgroup per (k0, k): dtd[k0][k][u] = sum_p sum_t D[k0,p,t] D[k,p,t+tau],
// tau = u - (L - 1), accumulated in FP64.  Also writes the apply table
// A[k0][U1-1-u1][U2-1-u2][k] (the same value, indexed by the offset of the
// patched position from the update; atom stride KS, padding left as set by the
// caller) and 1/||D_k||^2.
template <class R>
__global__ __launch_bounds__(256) void dtd_kernel(Geom g, const R *__restrict__ D, R *__restrict__ dtd,
                                                  R *__restrict__ A, R *__restrict__ inv_n) {
  extern __shared__ unsigned char smem_raw[];
  R *d0 = reinterpret_cast<R *>(smem_raw);
  const int PL = g.P * g.L1 * g.L2;
  R *d1 = d0 + PL;
  const int k0 = blockIdx.x / g.K, k = blockIdx.x - k0 * g.K;
  for (int i = threadIdx.x; i < PL; i += blockDim.x) {
    d0[i] = D[(long long)k0 * PL + i];
    d1[i] = D[(long long)k * PL + i];
  }
  __syncthreads();
  const int nU = g.U1 * g.U2;
  for (int u = threadIdx.x; u < nU; u += blockDim.x) {
    const int u1 = u / g.U2, u2 = u - (u / g.U2) * g.U2;
    const int tau1 = u1 - (g.L1 - 1), tau2 = u2 - (g.L2 - 1);
    const int t1lo = max(0, -tau1), t1hi = min(g.L1, g.L1 - tau1);
    const int t2lo = max(0, -tau2), t2hi = min(g.L2, g.L2 - tau2);
    double s = 0.0;
    for (int p = 0; p < g.P; ++p)
      for (int t1 = t1lo; t1 < t1hi; ++t1) {
        const R *a = d0 + (p * g.L1 + t1) * g.L2;
        const R *b = d1 + (p * g.L1 + t1 + tau1) * g.L2 + tau2;
        for (int t2 = t2lo; t2 < t2hi; ++t2) s += (double)a[t2] * (double)b[t2];
      }
    dtd[((long long)blockIdx.x) * nU + u] = (R)s;
    A[(((long long)k0 * g.U1 + (g.U1 - 1 - u1)) * g.U2 + (g.U2 - 1 - u2)) * g.KS + k] = (R)s;
    if (k == k0 && tau1 == 0 && tau2 == 0) inv_n[k] = (R)(1.0 / s);
  }
}

// ------------------------------------------------ DtD on the matrix cores
// DtD is itself a correlation with D.  Lay the atoms side by side along the
// second axis, atom k0 at columns k0 U2 + L2 - 1 ... k0 U2 + 2 L2 - 2 and rows
// L1 - 1 ... 2 L1 - 2, zeros elsewhere (the L - 1 zeros between neighbours
// serve both); this image has 3 L1 - 2 rows and K U2 + L2 - 1 columns.  Its
// valid correlation with D (U1 rows, K U2 columns) is, at row a1 and column
// k0 U2 + a2, sum_t D_k[t] D_k0[t + (a1, a2) - (L - 1)]: the apply-table entry
// A[k0][a1][a2][k], i.e. dtd[k0][k] at lag (L - 1) - (a1, a2).
template <class R>
__global__ __launch_bounds__(256) void dtd_image(Geom gi, const R *__restrict__ D, double *__restrict__ img,
                                                 long long n) {
  for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    const int a2 = (int)(i % gi.T2);
    const long long q = i / gi.T2;
    const int a1 = (int)(q % gi.T1), p = (int)(q / gi.T1);
    const int t1 = a1 - (gi.L1 - 1), c = a2 - (gi.L2 - 1);
    double v = 0.0;
    if (t1 >= 0 && t1 < gi.L1 && c >= 0) {
      const int k0 = c / gi.U2, t2 = c - k0 * gi.U2;
      if (k0 < gi.K && t2 < gi.L2) v = (double)D[(((long long)k0 * gi.P + p) * gi.L1 + t1) * gi.L2 + t2];
    }
    img[i] = v;
  }
}

// dtd, the apply table (atom stride g.KS, padding left as set by the caller)
// and 1/||D_k||^2 from G = corr(dtd_image, D) stored (U1, K U2, K).
template <class R>
__global__ __launch_bounds__(256) void dtd_gather(Geom g, const double *__restrict__ G, R *__restrict__ dtd,
                                                  R *__restrict__ A, R *__restrict__ inv_n, long long n) {
  for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    const int k = (int)(i % g.K);
    long long q = i / g.K;
    const int a2 = (int)(q % g.U2);
    q /= g.U2;
    const int a1 = (int)(q % g.U1), k0 = (int)(q / g.U1);
    const double v = G[(((long long)a1 * g.K + k0) * g.U2 + a2) * g.K + k];
    A[(((long long)k0 * g.U1 + a1) * g.U2 + a2) * g.KS + k] = (R)v;
    dtd[(((long long)k0 * g.K + k) * g.U1 + (g.U1 - 1 - a1)) * g.U2 + (g.U2 - 1 - a2)] = (R)v;
    if (k == k0 && a1 == g.L1 - 1 && a2 == g.L2 - 1) inv_n[k] = (R)(1.0 / v);
  }
}

// ------------------------------------------------------------- correlation
// G[pos][k] = sum_p sum_t D[k,p,t] X[p, pos + t] on the valid domain, computed
// directly: one thread per output position, KC atoms at a time, the slice
// D[k-chunk, p, t1, :] staged in LDS.  Tile: TH rows x 256/TH columns of
// positions (TH = 1 for signals, 8 for images).
enum CorrMode { CORR_BETA = 0, CORR_KKT = 1, CORR_ABSMAX = 2 };

struct CorrOut {
  void *beta;          // CORR_BETA: (H, W, KS) in the output type, padding written as 0.
                       // CORR_KKT, optional: also receives beta = G + n z (needs nrm); it may
                       // alias beta_cmp (each element is compared before the same thread
                       // overwrites it), which makes the check a drift correction as well
  const void *zpm;     // z (H, W, KS) in the working type: + n_k z (BETA) or the KKT test
  const double *nrm;   // n_k in FP64 (CORR_BETA with zpm)
  double lambda;       // CORR_KKT
  int positive;        // CORR_KKT / CORR_ABSMAX
  double *result;      // CORR_KKT: max violation; CORR_ABSMAX: max |G| (one-sided if positive)
  const void *beta_cmp;  // CORR_KKT, optional: a maintained beta (H, W, KS) in Rz compared with
  double *result2;       //   G + n z (needs nrm); result2 receives the max absolute difference
  double *g64;           // CORR_KKT and CORR_BETA, optional: G in FP64, (H, W, KS), atoms < K only
  const uint32_t *meta;  // optional, one word per position whose high 16 bits count the non-zeros
                         // of zpm there: the FFT epilogue reads z only where that count is not 0
};

template <class Rin, class Racc, class Rz, int MODE, int KC, int TH>
__global__ __launch_bounds__(256) void corr_kernel(Geom g, const Rin *__restrict__ X, const Rin *__restrict__ D,
                                                   CorrOut o) {
  constexpr int TW = 256 / TH;
  extern __shared__ unsigned char smem_raw[];
  Racc *ds = reinterpret_cast<Racc *>(smem_raw);  // [L2][KC]
  __shared__ double sh_red[4];
  const int tx = threadIdx.x % TW, ty = threadIdx.x / TW;
  const int h = blockIdx.y * TH + ty, w = blockIdx.x * TW + tx;
  const bool valid = h < g.H && w < g.W;
  const long long plane = (long long)g.T1 * g.T2;
  const long long pos = (long long)h * g.W + w;
  double red = 0.0, red2 = 0.0;
  for (int kb = 0; kb < g.K; kb += KC) {
    const int kc = min(KC, g.K - kb);
    Racc acc[KC];
#pragma unroll
    for (int q = 0; q < KC; ++q) acc[q] = Racc(0);
    for (int p = 0; p < g.P; ++p)
      for (int t1 = 0; t1 < g.L1; ++t1) {
        __syncthreads();
        for (int i = threadIdx.x; i < g.L2 * KC; i += blockDim.x) {
          const int t2 = i / KC, q = i - (i / KC) * KC;
          ds[i] = q < kc ? (Racc)D[(((long long)(kb + q) * g.P + p) * g.L1 + t1) * g.L2 + t2] : Racc(0);
        }
        __syncthreads();
        if (valid) {
          const Rin *xr = X + p * plane + (long long)(h + t1) * g.T2 + w;
          for (int t2 = 0; t2 < g.L2; ++t2) {
            const Racc x = (Racc)xr[t2];
            const Racc *dr = ds + t2 * KC;
#pragma unroll
            for (int q = 0; q < KC; ++q) acc[q] += dr[q] * x;
          }
        }
      }
    if (valid) {
#pragma unroll
      for (int q = 0; q < KC; ++q) {
        if (q >= kc) break;
        const int k = kb + q;
        if (MODE != CORR_ABSMAX && o.g64) o.g64[pos * g.KS + k] = (double)acc[q];
        if (MODE == CORR_BETA) {
          double v = (double)acc[q];
          if (o.zpm) v += o.nrm[k] * (double)reinterpret_cast<const Rz *>(o.zpm)[pos * g.KS + k];
          reinterpret_cast<Rz *>(o.beta)[pos * g.KS + k] = (Rz)v;
        } else if (MODE == CORR_KKT) {
          const double gv = (double)acc[q];
          const double z = (double)reinterpret_cast<const Rz *>(o.zpm)[pos * g.KS + k];
          double v;
          if (z == 0.0)
            v = o.positive ? fmax(gv - o.lambda, 0.0) : fmax(fabs(gv) - o.lambda, 0.0);
          else
            v = fabs(gv - (z > 0.0 ? o.lambda : -o.lambda));
          red = fmax(red, v);
          if (o.beta_cmp)
            red2 = fmax(red2, fabs(gv + o.nrm[k] * z - (double)reinterpret_cast<const Rz *>(o.beta_cmp)[pos * g.KS + k]));
          if (o.beta) reinterpret_cast<Rz *>(o.beta)[pos * g.KS + k] = (Rz)(gv + o.nrm[k] * z);
        } else {
          const double gv = (double)acc[q];
          red = fmax(red, o.positive ? gv : fabs(gv));
        }
      }
    }
  }
  if (MODE == CORR_BETA && valid)
    for (int k = g.K; k < g.KS; ++k) reinterpret_cast<Rz *>(o.beta)[pos * g.KS + k] = Rz(0);
  if (MODE != CORR_BETA) {
    red = block_max<256>(red, sh_red);
    if (threadIdx.x == 0) atomic_max_nonneg(o.result, fmax(red, 0.0));
    if (MODE == CORR_KKT && o.beta_cmp) {
      __syncthreads();
      red2 = block_max<256>(red2, sh_red);
      if (threadIdx.x == 0) atomic_max_nonneg(o.result2, red2);
    }
  }
}

// ------------------------------------------------------- best-move cache
// Best move of every position (the cache the round kernel keeps): score and
// atom of the largest move score over the K atoms (lowest atom on ties), and
// the position's count of non-zero coordinates.  A position's 16-byte atom
// groups are read by a segment of S lanes (S the power of two covering them,
// at most a wave), so a wave reads contiguous memory, and the segment reduces
// with shuffles; each wave takes U groups of positions per step with all
// their loads issued first.  z = NULL stands for z = 0 (a cold start), which
// is not read.  nz_known, when given, holds counts known to match z (the
// high 16 bits of a meta word; it may be meta itself, each word read before
// it is rewritten): z is then read only where the count is not 0.
template <class R>
__global__ __launch_bounds__(256) void init_moves(int HW, int K, int KS, const R *__restrict__ beta,
                                                  const R *__restrict__ z, const R *__restrict__ inv_n, R lambda,
                                                  R tol, int positive, int certify, R *__restrict__ score,
                                                  uint32_t *meta, const uint32_t *nz_known) {
  typedef typename Vec<R>::T V;
  constexpr int VE = Vec<R>::N;
  constexpr int U = 4;  // position groups per wave and step, their loads in flight together
  const int G = KS / VE;
  int S = 1;
  while (S < G && S < 64) S <<= 1;
  const int lane = threadIdx.x & 63, seg = lane / S, sl = lane - seg * S;
  const long long per_wave = 64 / S;
  const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const long long nwave = ((long long)gridDim.x * blockDim.x) >> 6;
  for (long long p0 = wave * per_wave * U; p0 < HW; p0 += nwave * per_wave * U) {
    R best[U];
    int bk[U], nz[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      best[u] = R(-1);
      bk[u] = 0x7fffffff;
      nz[u] = 0;
    }
    for (int q = sl; q < G; q += S) {
      V b[U], zv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const long long pos = p0 + u * per_wave + seg;
        b[u] = Vec<R>::zero();
        zv[u] = Vec<R>::zero();
        if (pos < HW) {
          b[u] = *reinterpret_cast<const V *>(beta + pos * KS + q * VE);
          if (z && (!nz_known || (nz_known[pos] >> 16) != 0)) zv[u] = *reinterpret_cast<const V *>(z + pos * KS + q * VE);
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int e = 0; e < VE; ++e) {
          const int k = q * VE + e;
          if (k >= K) break;
          const R zk = Vec<R>::get(zv[u], e);
          nz[u] += zk != R(0);
          const R sc = move_score(zk, st_target(Vec<R>::get(b[u], e), lambda, inv_n[k], positive), tol, certify);
          if (sc > best[u] || (sc == best[u] && k < bk[u])) {
            best[u] = sc;
            bk[u] = k;
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      for (int off = S >> 1; off > 0; off >>= 1) {
        const R ob = __shfl_xor(best[u], off, 64);
        const int ok = __shfl_xor(bk[u], off, 64);
        nz[u] += __shfl_xor(nz[u], off, 64);
        if (ob > best[u] || (ob == best[u] && ok < bk[u])) {
          best[u] = ob;
          bk[u] = ok;
        }
      }
      const long long pos = p0 + u * per_wave + seg;
      if (sl == 0 && pos < HW) {
        score[pos] = best[u];
        meta[pos] = (uint32_t)bk[u] | ((uint32_t)nz[u] << 16);
      }
    }
  }
}

template <class R>
inline void launch_init_moves(hipStream_t st, long long HW, int K, int KS, const R *beta, const R *z, const R *inv_n,
                              R lambda, R tol, int positive, int certify, R *score, uint32_t *meta,
                              const uint32_t *nz_known = nullptr) {
  int G = KS / Vec<R>::N, S = 1;
  while (S < G && S < 64) S <<= 1;
  const long long waves = (HW + 4 * (64 / S) - 1) / (4 * (64 / S));  // four position groups per wave
  const long long blocks = (waves + 3) / 4;
  hipLaunchKernelGGL(init_moves<R>, dim3((unsigned)(blocks < 16384 ? blocks : 16384)), dim3(256), 0, st, (int)HW, K,
                     KS, beta, z, inv_n, lambda, tol, positive, certify, score, meta, nz_known);
}

// ---------------------------------------------------------------- layouts
// user (K, H*W) <-> position-major (H*W, KS) with zero padding, and a type
// change: LDS-tiled transposes of 64 positions x 64 atoms, both sides of the
// copy coalesced.
template <class Rs, class Rd>
__global__ __launch_bounds__(256) void to_position_major(int HW, int K, int KS, const Rs *__restrict__ src,
                                                         Rd *__restrict__ dst) {
  __shared__ Rd tile[64][65];
  const long long p0 = (long long)blockIdx.x * 64;
  const int k0 = blockIdx.y * 64;
  const int pn = (int)min(64ll, HW - p0), kn = min(64, KS - k0);
  Rd v[16];  // a thread's 16 reads of the tile, issued together
#pragma unroll
  for (int ii = 0; ii < 16; ++ii) {
    const int i = threadIdx.x + 256 * ii, kk = i >> 6, pp = i & 63, k = k0 + kk;
    v[ii] = kk < kn && pp < pn && k < K ? (Rd)src[(long long)k * HW + p0 + pp] : Rd(0);
  }
#pragma unroll
  for (int ii = 0; ii < 16; ++ii) {
    const int i = threadIdx.x + 256 * ii;
    tile[i >> 6][i & 63] = v[ii];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < pn * kn; i += 256) {
    const int pp = i / kn, kk = i - pp * kn;
    dst[(p0 + pp) * KS + k0 + kk] = tile[kk][pp];
  }
}

template <class Rs, class Rd>
__global__ __launch_bounds__(256) void to_atom_major(int HW, int K, int KS, const Rs *__restrict__ src,
                                                     Rd *__restrict__ dst) {
  __shared__ Rd tile[64][65];
  const long long p0 = (long long)blockIdx.x * 64;
  const int k0 = blockIdx.y * 64;
  const int pn = (int)min(64ll, HW - p0), kn = min(64, K - k0);
  Rd v[16];  // a thread's reads of the tile, issued together
#pragma unroll
  for (int ii = 0; ii < 16; ++ii) {
    const int i = threadIdx.x + 256 * ii, pp = i / kn, kk = i - pp * kn;
    v[ii] = i < pn * kn ? (Rd)src[(p0 + pp) * KS + k0 + kk] : Rd(0);
  }
#pragma unroll
  for (int ii = 0; ii < 16; ++ii) {
    const int i = threadIdx.x + 256 * ii, pp = i / kn, kk = i - pp * kn;
    if (i < pn * kn) tile[kk][pp] = v[ii];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 64 * 64; i += 256) {
    const int kk = i >> 6, pp = i & 63;
    if (kk < kn && pp < pn) dst[(long long)(k0 + kk) * HW + p0 + pp] = tile[kk][pp];
  }
}

template <class Rs, class Rd>
inline void launch_to_position_major(hipStream_t st, long long HW, int K, int KS, const Rs *src, Rd *dst) {
  hipLaunchKernelGGL((to_position_major<Rs, Rd>), dim3((unsigned)((HW + 63) / 64), (unsigned)((KS + 63) / 64)),
                     dim3(256), 0, st, (int)HW, K, KS, src, dst);
}

template <class Rs, class Rd>
inline void launch_to_atom_major(hipStream_t st, long long HW, int K, int KS, const Rs *src, Rd *dst) {
  hipLaunchKernelGGL((to_atom_major<Rs, Rd>), dim3((unsigned)((HW + 63) / 64), (unsigned)((K + 63) / 64)),
                     dim3(256), 0, st, (int)HW, K, KS, src, dst);
}

// The non-zeros of a position-major z written into an atom-major (K, H*W)
// output that already holds zeros: one thread per position, and only the
// positions whose count in `meta` (high 16 bits) is not 0 are read.
template <class R>
__global__ __launch_bounds__(256) void scatter_atom_major(int HW, int K, int KS, const R *__restrict__ zpm,
                                                          const uint32_t *__restrict__ meta, R *__restrict__ dst) {
  for (long long pos = blockIdx.x * 256ll + threadIdx.x; pos < HW; pos += (long long)gridDim.x * 256) {
    if ((meta[pos] >> 16) == 0) continue;
    for (int k = 0; k < K; ++k) {
      const R v = zpm[pos * KS + k];
      if (v != R(0)) dst[(long long)k * HW + pos] = v;
    }
  }
}

template <class Rs, class Rd>
__global__ __launch_bounds__(256) void convert_kernel(long long n, const Rs *__restrict__ src, Rd *__restrict__ dst) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    dst[i] = (Rd)src[i];
}

// ------------------------------------------------ non-zero entries and sums
struct NzEntry {
  int pos;
  int k;
  double z;
};

__global__ __launch_bounds__(256) void sum_squares(long long n, const double *__restrict__ x, double *out) {
  __shared__ double sh[4];
  double a = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    a += x[i] * x[i];
  a = block_sum<256>(a, sh);
  if (threadIdx.x == 0) atomic_add_f64(out, a);
}

// res -= Z*D for a position-major z (atom stride KS), one wave per position:
// the lanes find the non-zero atoms of the position, then scatter each one's
// shifted atom (eq. model) with FP64 atomics.  A wave loads the atom rows of
// RP positions at once (RP independent loads in flight) before it scans them.
// With `meta` (one word per position, the high 16 bits counting the non-zeros
// of z there) a wave instead reads the words of 64 positions in one load and
// visits only the positions whose count is not 0: z itself is read where it
// has non-zeros.  Also accumulates sum |z| and the non-zero count into acc[0],
// acc[1] (doubles).  No host round trip.
template <class R, class Rd>
__device__ __forceinline__ void residual_patch(const Geom &g, long long pos, int kb, R v, const Rd *__restrict__ D,
                                                 double *__restrict__ res, double &l1, double &cnt) {
  const int lane = threadIdx.x & 63;
  unsigned long long m = __ballot(v != R(0));
  if (!m) return;
  if (v != R(0)) {
    l1 += fabs((double)v);
    cnt += 1.0;
  }
  const int PL = g.P * g.L1 * g.L2, LL = g.L1 * g.L2;
  const long long plane = (long long)g.T1 * g.T2;
  const int h = (int)(pos / g.W), w = (int)(pos - (pos / g.W) * g.W);
  while (m) {
    const int src = __ffsll((long long)m) - 1;
    m &= m - 1;
    const double zv = (double)__shfl(v, src, 64);
    const Rd *dk = D + (long long)(kb + src) * PL;
    for (int i = lane; i < PL; i += 64) {
      const int p = i / LL, r = i - p * LL;
      const int t1 = r / g.L2, t2 = r - (r / g.L2) * g.L2;
      atomic_add_f64(res + p * plane + (long long)(h + t1) * g.T2 + (w + t2), -zv * (double)dk[i]);
    }
  }
}

template <class R, class Rd>
__global__ __launch_bounds__(256) void residual_dense(Geom g, const R *__restrict__ z, const Rd *__restrict__ D,
                                                      double *__restrict__ res, double *__restrict__ acc,
                                                      const uint32_t *__restrict__ meta) {
  constexpr int RP = 8;
  __shared__ double sh[4];
  const int lane = threadIdx.x & 63;
  const long long HW = (long long)g.H * g.W;
  double l1 = 0.0, cnt = 0.0;
  const long long wave = (long long)blockIdx.x * 4 + (threadIdx.x >> 6), nwaves = (long long)gridDim.x * 4;
  if (meta) {
    for (long long c0 = wave * 64; c0 < HW; c0 += nwaves * 64) {
      const long long mine = c0 + lane;
      unsigned long long pm = __ballot(mine < HW && (meta[mine] >> 16) != 0);
      while (pm) {
        const long long pos = c0 + (__ffsll((long long)pm) - 1);
        pm &= pm - 1;
        for (int kb = 0; kb < g.K; kb += 64) {
          const int k = kb + lane;
          const R v = k < g.K ? z[pos * g.KS + k] : R(0);
          residual_patch<R, Rd>(g, pos, kb, v, D, res, l1, cnt);
        }
      }
    }
  } else {
    for (long long pos0 = wave * RP; pos0 < HW; pos0 += nwaves * RP) {
      for (int kb = 0; kb < g.K; kb += 64) {
        const int k = kb + lane;
        R v[RP];
#pragma unroll
        for (int q = 0; q < RP; ++q) v[q] = (k < g.K && pos0 + q < HW) ? z[(pos0 + q) * g.KS + k] : R(0);
#pragma unroll
        for (int q = 0; q < RP; ++q) residual_patch<R, Rd>(g, pos0 + q, kb, v[q], D, res, l1, cnt);
      }
    }
  }
  l1 = block_sum<256>(l1, sh);
  cnt = block_sum<256>(cnt, sh);
  if (threadIdx.x == 0) {
    atomic_add_f64(acc, l1);
    atomic_add_f64(acc + 1, cnt);
  }
}

// Fills n 32-bit words with a value (a kernel, so it may sit in a captured graph).
__global__ __launch_bounds__(256) void fill_u32(long long n, uint32_t v, uint32_t *__restrict__ dst) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    dst[i] = v;
}

// ------------------------------------------------------- dictionary stats
// psi[k][p][t] += sum over the non-zeros of atom k in [beg, end) of z X_p[pos + t].
// One workgroup per chunk; every chunk holds non-zeros of a single atom.
struct Chunk {
  int k;
  int beg;
  int end;
  int pad;
};

template <class Rin>
__global__ __launch_bounds__(256) void psi_kernel(Geom g, const Chunk *__restrict__ chunks, const NzEntry *__restrict__ list,
                                                  const Rin *__restrict__ X, double *__restrict__ psi) {
  __shared__ NzEntry sh_nz[128];
  const Chunk c = chunks[blockIdx.x];
  const int PL = g.P * g.L1 * g.L2, LL = g.L1 * g.L2;
  const long long plane = (long long)g.T1 * g.T2;
  const int n = c.end - c.beg;
  for (int i = threadIdx.x; i < n; i += blockDim.x) sh_nz[i] = list[c.beg + i];
  __syncthreads();
  for (int e = threadIdx.x; e < PL; e += blockDim.x) {
    const int p = e / LL, r = e - p * LL;
    const int t1 = r / g.L2, t2 = r - (r / g.L2) * g.L2;
    const Rin *xp = X + p * plane + (long long)t1 * g.T2 + t2;
    double acc = 0.0;
    for (int j = 0; j < n; ++j) {
      const int pos = sh_nz[j].pos;
      const int h = pos / g.W, w = pos - (pos / g.W) * g.W;
      acc += sh_nz[j].z * (double)xp[(long long)h * g.T2 + w];
    }
    atomic_add_f64(psi + (long long)c.k * PL + e, acc);
  }
}

// phi[k][k'][tau + L - 1] += z_k[w] z_k'[w + tau] for every listed non-zero
// (k, w).  Its window w + Phi is scanned row by row in the bitmap of
// non-empty positions (bit pos of nzbits: at most three words per window
// row), and only the atoms of the set positions are read from the
// position-major copy of z.
template <class R>
__global__ __launch_bounds__(256) void phi_kernel(Geom g, const NzEntry *__restrict__ list, long long nnz,
                                                  const R *__restrict__ zpm, const uint32_t *__restrict__ nzbits,
                                                  double *__restrict__ phi) {
  const int nU = g.U1 * g.U2;
  const int nwr = (g.U2 + 31) / 32 + 1;  // words one window row spans at most
  for (long long e = blockIdx.x; e < nnz; e += gridDim.x) {
    const NzEntry nz = list[e];
    const int h = nz.pos / g.W, w = nz.pos - (nz.pos / g.W) * g.W;
    const int wlo = max(0, w - (g.L2 - 1)), whi = min(g.W, w + g.L2);  // window columns [wlo, whi)
    for (int it = threadIdx.x; it < g.U1 * nwr; it += blockDim.x) {
      const int u1 = it / nwr, wi = it - u1 * nwr;
      const int hh = h + u1 - (g.L1 - 1);
      if (hh < 0 || hh >= g.H) continue;
      const long long row = (long long)hh * g.W;
      const long long b0 = row + wlo, b1 = row + whi;  // bits [b0, b1)
      const long long lo = ((b0 >> 5) + wi) << 5;       // first bit of this thread's word
      if (lo >= b1) continue;
      uint32_t m = nzbits[lo >> 5];
      if (b0 > lo) m &= ~0u << (int)(b0 - lo);
      if (b1 < lo + 32) m &= (1u << (int)(b1 - lo)) - 1u;
      while (m) {
        const int bit = __ffs(m) - 1;
        m &= m - 1;
        const long long pos2 = lo + bit;
        const int u = u1 * g.U2 + (int)(pos2 - row) - w + (g.L2 - 1);
        const R *zr = zpm + pos2 * g.KS;
        for (int k2 = 0; k2 < g.K; ++k2) {
          const R v = zr[k2];
          if (v != R(0)) atomic_add_f64(phi + ((long long)nz.k * g.K + k2) * nU + u, nz.z * (double)v);
        }
      }
    }
  }
}

// to_position_major for the dictionary statistics: also counts the non-zeros
// of every position into nzc and of every atom into cnt, and sets the bit of
// every non-empty position in nzbits (all zeroed by the caller), from the
// transposed tile.  When one tile holds every atom (KS <= 64) the rows of
// positions without non-zeros are not written: the statistics read z only
// where nzc or nzbits mark a non-zero.
template <class R>
__global__ __launch_bounds__(256) void to_position_major_counts(int HW, int K, int KS, const R *__restrict__ src,
                                                                R *__restrict__ dst, int *__restrict__ nzc,
                                                                unsigned int *__restrict__ cnt,
                                                                uint32_t *__restrict__ nzbits) {
  __shared__ R tile[64][65];
  __shared__ int pnz[64];
  const long long p0 = (long long)blockIdx.x * 64;
  const int k0 = blockIdx.y * 64;
  const int pn = (int)min(64ll, HW - p0), kn = min(64, KS - k0);
  R v[16];  // a thread's 16 reads of the tile, issued together
#pragma unroll
  for (int ii = 0; ii < 16; ++ii) {
    const int i = threadIdx.x + 256 * ii, kk = i >> 6, pp = i & 63, k = k0 + kk;
    v[ii] = kk < kn && pp < pn && k < K ? src[(long long)k * HW + p0 + pp] : R(0);
  }
#pragma unroll
  for (int ii = 0; ii < 16; ++ii) {
    const int i = threadIdx.x + 256 * ii;
    tile[i >> 6][i & 63] = v[ii];
  }
  __syncthreads();
  const int ka = min(kn, K - k0);  // real atoms of the tile
  if (threadIdx.x < 64) {
    const int pp = threadIdx.x;
    int c = 0;
    if (pp < pn)
      for (int kk = 0; kk < ka; ++kk) c += tile[kk][pp] != R(0);
    pnz[pp] = c;
    if (c) atomicAdd(&nzc[p0 + pp], c);
    // the tile's 64 positions are two whole words of the bitmap (p0 is a multiple of 64)
    const unsigned long long bits = __ballot(c != 0);
    if (pp == 0 && bits) {
      atomicOr(&nzbits[p0 >> 5], (uint32_t)bits);
      if (bits >> 32) atomicOr(&nzbits[(p0 >> 5) + 1], (uint32_t)(bits >> 32));
    }
  } else if (threadIdx.x < 128) {
    const int kk = threadIdx.x - 64;
    unsigned int c = 0;
    if (kk < ka)
      for (int pp = 0; pp < pn; ++pp) c += tile[kk][pp] != R(0);
    if (c) atomicAdd(&cnt[k0 + kk], c);
  }
  __syncthreads();
  const bool skip_empty = gridDim.y == 1;
  for (int i = threadIdx.x; i < pn * kn; i += 256) {
    const int pp = i / kn, kk = i - pp * kn;
    if (skip_empty && pnz[pp] == 0) continue;
    dst[(p0 + pp) * KS + k0 + kk] = tile[kk][pp];
  }
}

// Lists the non-zeros of a position-major z grouped by atom (cursor[k] starts
// at the atom's offset in the list), reading z only at positions whose
// non-zero count is positive.
template <class R>
__global__ __launch_bounds__(256) void list_from_position_major(int HW, int K, int KS, const R *__restrict__ zpm,
                                                                const int *__restrict__ nzc,
                                                                unsigned int *__restrict__ cursor,
                                                                NzEntry *__restrict__ list) {
  for (int pos = blockIdx.x * blockDim.x + threadIdx.x; pos < HW; pos += gridDim.x * blockDim.x) {
    if (nzc[pos] == 0) continue;
    for (int k = 0; k < K; ++k) {
      const R v = zpm[(long long)pos * KS + k];
      if (v != R(0)) {
        const unsigned int slot = atomicAdd(&cursor[k], 1u);
        NzEntry e;
        e.pos = pos;
        e.k = k;
        e.z = (double)v;
        list[slot] = e;
      }
    }
  }
}

// ------------------------------------------------------- bandwidth probe
// dst = src, 16 bytes per thread per step: a plain streaming copy used to
// measure achievable HBM bandwidth and to calibrate traffic counters.
// Streaming copy of n16 16-byte words, one word per thread over a full grid
// (no grid stride): on gfx950 this form measured 6.2 TB/s for 1 GiB, above
// grid-stride loops with one to eight words in flight per thread (4.0 to
// 5.7 TB/s) and non-temporal variants.
__global__ __launch_bounds__(256) void copy_probe(long long n16, const uint4 *__restrict__ src, uint4 *__restrict__ dst) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < n16) dst[i] = src[i];
}

}  // namespace dcdl
