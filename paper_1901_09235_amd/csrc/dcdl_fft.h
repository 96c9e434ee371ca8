// dcdl_fft.h -- the dense FP64 correlation G = corr(R, D) of an image by FFT.
//
// G_k = sum_p corr(R_p, D_kp) on the valid domain (the contraction behind beta
// = corr(X - Z*D, D) + n z of Sec. 3 and the optimality check of eq. csc) is,
// by the correlation theorem, the inverse transform of
// sum_p Rhat_p conj(Dhat_kp) over N1 x N2 points, the powers of two covering
// T1 x T2: a valid output w reads R at w + t <= T - 1, so nothing wraps.  The
// arithmetic is FP64 throughout.  Its work is O((P + K) N1 N2 log(N1 N2))
// against the direct contraction's 2 K P L1 L2 H W (for 3 x 4096^2 and 25
// atoms of 32 x 32: about 50 times fewer flops), so every pass is bound by
// HBM traffic:
//
//   rows      the N2-point FFT of each real row, as the N2/2-point complex FFT
//             of z[n] = x[2n] + i x[2n+1] (radix-8 Stockham stages in LDS,
//             natural order) split into the half spectrum X[0 .. N2/2];
//   columns   N1-point FFTs of the half-spectrum columns, 16 columns per
//             workgroup (every row segment read or written is 256 bytes), in
//             two passes of N1 = A B: A-point transforms at row stride B with
//             a twiddle, then B-point transforms of contiguous row blocks.  The
//             result stays in digit-swapped row order (row k1 + B k2 holds
//             frequency k2 + A k1), which the inverse passes take as it is:
//             the spectral products are elementwise, so the order never
//             matters.  N1 <= 128 takes one pass;
//   product   Shat_k = sum_p Rhat_p conj(Dhat_kp);
//   inverse   the column passes reversed, then the complex-to-real rows,
//             cropped to the valid domain and scaled by 1 / (N1 N2 / 2);
//   epilogue  the outputs of the matrix-core contraction (beta, KKT, max |G|,
//             G in FP64), position-major, through an LDS transpose.
//
// An atom has L1 non-zero rows: when L1 <= B its first column pass reduces to
// a twiddle of the row transforms, which the second pass applies as it loads
// them (sparse input), so a dictionary spectrum costs one write.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dcdl_kernels.h"

namespace dcdl {

struct FftGeom {
  int N1, N2, M2;   // transform size (powers of two), M2 = N2 / 2
  int F2p;          // half-spectrum columns M2 + 1, padded to a multiple of 16
  int A, B;         // N1 = A B with B = 64 (two column passes), or A = N1, B = 1 (one)
  long long plane;  // complex values of one spectrum, N1 F2p
};

__device__ __forceinline__ double2 c_add(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 c_sub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 c_mul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a conj(b)
__device__ __forceinline__ double2 c_mulc(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ double2 c_conj(double2 a) { return make_double2(a.x, -a.y); }

// tw[m] = exp(-2 pi i m / N), m < N (N a power of two, so m / N is exact).
__global__ __launch_bounds__(256) void fft_twiddles(int N, double2 *__restrict__ tw) {
  const int m = blockIdx.x * 256 + threadIdx.x;
  if (m >= N) return;
  double s, c;
  sincospi(-2.0 * (double)m / (double)N, &s, &c);
  tw[m] = make_double2(c, s);
}

// Threads of the row-transform workgroups.
constexpr int kRowThreads = 512;

// R-point DFT (R = 2, 4, 8) of v in place, natural order; the inverse uses
// the conjugate roots (unnormalised).
template <int R>
__device__ __forceinline__ void dft_r(double2 *v, bool inverse) {
  if constexpr (R == 2) {
    const double2 t = v[0];
    v[0] = c_add(t, v[1]);
    v[1] = c_sub(t, v[1]);
  } else if constexpr (R == 4) {
    const double2 a0 = c_add(v[0], v[2]), a1 = c_sub(v[0], v[2]);
    const double2 a2 = c_add(v[1], v[3]), a3 = c_sub(v[1], v[3]);
    // -i a3 forward, +i a3 inverse
    const double2 r3 = inverse ? make_double2(-a3.y, a3.x) : make_double2(a3.y, -a3.x);
    v[0] = c_add(a0, a2);
    v[2] = c_sub(a0, a2);
    v[1] = c_add(a1, r3);
    v[3] = c_sub(a1, r3);
  } else {
    double2 e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
    dft_r<4>(e, inverse);
    dft_r<4>(o, inverse);
    constexpr double h = 0.70710678118654752440;  // sqrt(1/2)
    const double s = inverse ? 1.0 : -1.0;         // sign of the imaginary part of the root
    // w^k o[k] for w = exp(-+2 pi i / 8): k = 1: (h, s h); k = 2: (0, s); k = 3: (-h, s h)
    const double2 o1 = c_mul(o[1], make_double2(h, s * h));
    const double2 o2 = make_double2(-s * o[2].y, s * o[2].x);
    const double2 o3 = c_mul(o[3], make_double2(-h, s * h));
    v[0] = c_add(e[0], o[0]);
    v[4] = c_sub(e[0], o[0]);
    v[1] = c_add(e[1], o1);
    v[5] = c_sub(e[1], o1);
    v[2] = c_add(e[2], o2);
    v[6] = c_sub(e[2], o2);
    v[3] = c_add(e[3], o3);
    v[7] = c_sub(e[3], o3);
  }
}

// The twiddles w^r, r < R, of a radix-R butterfly from w^1, w^2 and w^4 read
// from the table (index m1 = the table index of w^1): at most two products
// each, so their error stays within a few FP64 ulps.
template <int R>
__device__ __forceinline__ void stage_twiddles(double2 *w, const double2 *__restrict__ tw, long long m1, bool inverse) {
  w[0] = make_double2(1.0, 0.0);
  w[1] = tw[m1];
  if constexpr (R >= 4) {
    w[2] = tw[2 * m1];
    w[3] = c_mul(w[1], w[2]);
  }
  if constexpr (R == 8) {
    w[4] = tw[4 * m1];
    w[5] = c_mul(w[1], w[4]);
    w[6] = c_mul(w[2], w[4]);
    w[7] = c_mul(w[3], w[4]);
  }
  if (inverse) {
#pragma unroll
    for (int r = 1; r < R; ++r) w[r].y = -w[r].y;
  }
}

// One radix-R stage of the Stockham FFT (decimation in time, natural order
// in and out) of n points in LDS buffer a, span Ns: butterfly j reads
// a[j + r n / R], twiddles them by exp(-+2 pi i r (j mod Ns) / (Ns R)), takes
// the R-point DFT and writes a[(j / Ns) Ns R + (j mod Ns) + r Ns].  In place:
// every read precedes a barrier before the writes.  At most 512 butterflies,
// one per thread of the 512-thread row workgroups.  tw[m tws] =
// exp(-2 pi i m / n).
template <int R>
__device__ __forceinline__ void lds_stage(double2 *a, int n, int Ns, const double2 *__restrict__ tw, int tws,
                                          bool inverse) {
  constexpr int Q = 512 / kRowThreads;
  const int nb = n / R;
  double2 v[Q][R];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int j = threadIdx.x + q * blockDim.x;
    if (j < nb) {
      const int jm = j & (Ns - 1);
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = a[j + r * nb];
      if (jm > 0) {
        double2 w[R];
        stage_twiddles<R>(w, tw, (long long)jm * (n / (Ns * R)) * tws, inverse);
#pragma unroll
        for (int r = 1; r < R; ++r) v[q][r] = c_mul(v[q][r], w[r]);
      }
      dft_r<R>(v[q], inverse);
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int j = threadIdx.x + q * blockDim.x;
    if (j < nb) {
      const int idx = (j / Ns) * Ns * R + (j & (Ns - 1));
#pragma unroll
      for (int r = 0; r < R; ++r) a[idx + r * Ns] = v[q][r];
    }
  }
  __syncthreads();
}

// Stockham FFT of n <= 4096 points (a power of two) in LDS buffer a, natural
// order in and out, in radix-8 stages (a last radix-4 or -2 stage when log2 n
// is not a multiple of 3).  Every thread of the kRowThreads takes part.
__device__ void lds_fft(double2 *a, int n, const double2 *__restrict__ tw, int tws, bool inverse) {
  for (int Ns = 1; Ns < n;) {
    const int rem = n / Ns;
    if (rem % 8 == 0) {
      lds_stage<8>(a, n, Ns, tw, tws, inverse);
      Ns *= 8;
    } else if (rem % 4 == 0) {
      lds_stage<4>(a, n, Ns, tw, tws, inverse);
      Ns *= 4;
    } else {
      lds_stage<2>(a, n, Ns, tw, tws, inverse);
      Ns *= 2;
    }
  }
}

// One row per workgroup (blockIdx.x), one input per blockIdx.y: the half
// spectrum X[0 .. M2] of the real row x (zero beyond `cols`), written with
// zero padding up to F2p.  LDS: M2 complex values.
template <class Rin>
__global__ __launch_bounds__(kRowThreads) void fft_rows_r2c(FftGeom f, const Rin *__restrict__ x, long long xb, int xp,
                                                    int cols, const double2 *__restrict__ tw2,
                                                    double2 *__restrict__ out, long long ob) {
  extern __shared__ double2 fsm[];
  double2 *a = fsm;
  const Rin *xr = x + blockIdx.y * xb + (long long)blockIdx.x * xp;
  for (int n = threadIdx.x; n < f.M2; n += blockDim.x) {
    const int c0 = 2 * n, c1 = 2 * n + 1;
    a[n] = make_double2(c0 < cols ? (double)xr[c0] : 0.0, c1 < cols ? (double)xr[c1] : 0.0);
  }
  __syncthreads();
  // exp(-2 pi i m / M2) = tw2[2 m]
  lds_fft(a, f.M2, tw2, 2, false);
  const double2 *Z = a;
  double2 *o = out + blockIdx.y * ob + (long long)blockIdx.x * f.F2p;
  for (int k = threadIdx.x; k < f.F2p; k += blockDim.x) {
    double2 X = make_double2(0.0, 0.0);
    if (k <= f.M2) {
      // X[k] = (Z[k] + conj Z[M2-k]) / 2 - i w^k (Z[k] - conj Z[M2-k]) / 2, w = exp(-2 pi i / N2)
      const double2 zk = Z[k == f.M2 ? 0 : k], zm = c_conj(Z[k == 0 ? 0 : f.M2 - k]);
      const double2 s = c_add(zk, zm), t = c_mul(tw2[k], c_sub(zk, zm));
      X = make_double2(0.5 * (s.x + t.y), 0.5 * (s.y - t.x));
    }
    o[k] = X;
  }
}

// One output row h < H per workgroup (blockIdx.x), one spectrum per
// blockIdx.y: the real row whose half spectrum is row h of S, times `scale`,
// written for columns < W into G (row pitch W, batch stride gb).
__global__ __launch_bounds__(kRowThreads) void fft_rows_c2r(FftGeom f, const double2 *__restrict__ S, long long sb,
                                                    const double2 *__restrict__ tw2, double *__restrict__ G,
                                                    long long gb, int W, double scale) {
  extern __shared__ double2 fsm[];
  double2 *a = fsm;
  const double2 *X = S + blockIdx.y * sb + (long long)blockIdx.x * f.F2p;
  // Z[k] = E[k] + i O[k] with E = (X[k] + conj X[M2-k]) / 2 and
  // O = conj(w^k) (X[k] - conj X[M2-k]) / 2, the transforms of the even and
  // odd samples; one thread forms Z[k] and Z[M2-k] from the same two reads
  for (int k = threadIdx.x; k <= f.M2 / 2; k += blockDim.x) {
    const double2 xk = X[k], xm = X[f.M2 - k];
    {
      const double2 xb = c_conj(xm);
      const double2 s = c_add(xk, xb), t = c_mul(c_conj(tw2[k]), c_sub(xk, xb));
      a[k] = make_double2(0.5 * (s.x - t.y), 0.5 * (s.y + t.x));
    }
    if (k > 0 && k < f.M2 - k) {
      const double2 xb = c_conj(xk);
      const double2 s = c_add(xm, xb), t = c_mul(c_conj(tw2[f.M2 - k]), c_sub(xm, xb));
      a[f.M2 - k] = make_double2(0.5 * (s.x - t.y), 0.5 * (s.y + t.x));
    }
  }
  __syncthreads();
  lds_fft(a, f.M2, tw2, 2, true);
  const double2 *z = a;
  double *g = G + blockIdx.y * gb + (long long)blockIdx.x * W;
  for (int n = threadIdx.x; n < f.M2; n += blockDim.x) {
    const int c0 = 2 * n, c1 = 2 * n + 1;
    if (c0 < W) g[c0] = z[n].x * scale;
    if (c1 < W) g[c1] = z[n].y * scale;
  }
}

// M-point FFTs along the columns of the spectra S (row pitch F2p, batch
// stride sb, blockIdx.z): group g holds rows g gmul + i stride, i < M;
// 16 columns (blockIdx.x) and 128 / M groups (blockIdx.y) per workgroup.
// Rows >= rows_valid read as zero; rows >= rows_store are not written.  With
// `twiddle`, output i of group g is multiplied by exp(-+2 pi i g i / N1).
// With E (sparse input, eb per spectrum): the input of group g at i is
// E[i] exp(-2 pi i g i / N1) for i < e_rows, else zero.
struct ColArgs {
  FftGeom f;
  double2 *S;
  int ngroups, gmul, stride, rows_valid, rows_store, inverse, twiddle;
  const double2 *tw1;
  const double2 *E;
  long long eb;
  int e_rows;
};

__device__ __forceinline__ double2 col_load(const ColArgs &ca, int g, int i, int col) {
  double2 v = make_double2(0.0, 0.0);
  if (g >= ca.ngroups) return v;
  if (ca.E) {
    if (i < ca.e_rows) v = c_mul(ca.E[blockIdx.z * ca.eb + (long long)i * ca.f.F2p + col], ca.tw1[(long long)i * g]);
  } else {
    const int row = g * ca.gmul + i * ca.stride;
    if (row < ca.rows_valid) v = ca.S[blockIdx.z * ca.f.plane + (long long)row * ca.f.F2p + col];
  }
  return v;
}

__device__ __forceinline__ void col_store(const ColArgs &ca, long long plane, int g, int i, int col, double2 v) {
  if (g >= ca.ngroups) return;
  const int row = g * ca.gmul + i * ca.stride;
  if (row >= ca.rows_store) return;
  if (ca.twiddle) {
    double2 w = ca.tw1[(long long)g * i];
    if (ca.inverse) w.y = -w.y;
    v = c_mul(v, w);
  }
  ca.S[plane * ca.f.plane + (long long)row * ca.f.F2p + col] = v;
}

// The plain input of a column pass: spectrum blockIdx.z of S (or E).
struct ColLoadPlain {
  __device__ __forceinline__ double2 operator()(const ColArgs &ca, int, int g, int i, int col) const {
    return col_load(ca, g, i, col);
  }
};

// Radix-R stage of span Ns of the M-point Stockham FFTs of a workgroup's 16 x
// (128 / M) sequences (element i of sequence (gs, c) at buf[(gs M + i) 16 + c]
// between stages): the first stage loads from the spectra, the last stores to
// them, so M <= 8 never touches LDS and M = 64 crosses it once.
template <int M, int Ns, class Load>
__device__ __forceinline__ void col_stages(const ColArgs &ca, double2 *buf, const Load &load, long long out_plane) {
  constexpr int R = (M / Ns) % 8 == 0 ? 8 : ((M / Ns) % 4 == 0 ? 4 : 2);
  constexpr int Q = 2048 / R / 256;  // butterflies per thread
  constexpr bool FIRST = Ns == 1, LAST = Ns * R == M;
  constexpr int GPW = 128 / M;
  const int c0 = blockIdx.x * 16, g0 = blockIdx.y * GPW, tws = ca.f.N1 / M;
  double2 v[Q][R];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int b = threadIdx.x + 256 * q;
    const int c = b & 15, rest = b >> 4, gs = rest / (M / R), j = rest % (M / R);
    const int jm = j & (Ns - 1);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = j + r * (M / R);
      if constexpr (FIRST)
        v[q][r] = load(ca, q * R + r, g0 + gs, i, c0 + c);
      else
        v[q][r] = buf[(gs * M + i) * 16 + c];
    }
    if (!FIRST && jm > 0) {
      double2 w[R];
      stage_twiddles<R>(w, ca.tw1, (long long)jm * (M / (Ns * R)) * tws, ca.inverse);
#pragma unroll
      for (int r = 1; r < R; ++r) v[q][r] = c_mul(v[q][r], w[r]);
    }
    dft_r<R>(v[q], ca.inverse);
  }
  if constexpr (!LAST) {
    if constexpr (!FIRST) __syncthreads();
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int b = threadIdx.x + 256 * q;
      const int c = b & 15, rest = b >> 4, gs = rest / (M / R), j = rest % (M / R);
      const int idx = (j / Ns) * Ns * R + (j & (Ns - 1));
#pragma unroll
      for (int r = 0; r < R; ++r) buf[(gs * M + idx + r * Ns) * 16 + c] = v[q][r];
    }
    __syncthreads();
    col_stages<M, Ns * R>(ca, buf, load, out_plane);
  } else {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int b = threadIdx.x + 256 * q;
      const int c = b & 15, rest = b >> 4, gs = rest / (M / R), j = rest % (M / R);
      const int idx = (j / Ns) * Ns * R + (j & (Ns - 1));
#pragma unroll
      for (int r = 0; r < R; ++r) col_store(ca, out_plane, g0 + gs, idx + r * Ns, c0 + c, v[q][r]);
    }
  }
}

template <int M>
__global__ __launch_bounds__(256) void fft_cols(ColArgs ca) {
  __shared__ double2 buf[M > 8 ? 2048 : 1];
  col_stages<M, 1>(ca, buf, ColLoadPlain(), blockIdx.z);
}

// The first inverse column pass fused with the spectral product: the input
// of spectrum kk is sum_p Rhat_p conj(Dhat_(k0+kk),p) at each element, for
// kk < nk in turn, with the workgroup's Rhat values (P <= 4 channels, the
// eight first-stage elements of each thread) held in registers across the
// atoms.
// Dhat is stored [k][p]; the outputs go to planes kk of ca.S.
template <int P>
struct ColLoadProduct {
  const double2 (*rr)[8];
  const double2 *dk;  // Dhat of atom k, channel 0
  __device__ __forceinline__ double2 operator()(const ColArgs &ca, int e8, int g, int i, int col) const {
    if (g >= ca.ngroups) return make_double2(0.0, 0.0);
    const long long e = (long long)(g * ca.gmul + i * ca.stride) * ca.f.F2p + col;
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int p = 0; p < P; ++p) acc = c_add(acc, c_mulc(rr[p][e8], dk[p * ca.f.plane + e]));
    return acc;
  }
};

template <int M, int P>
__global__ __launch_bounds__(256) void fft_cols_product(ColArgs ca, const double2 *__restrict__ Rh,
                                                        const double2 *__restrict__ Dh, int k0, int nk) {
  __shared__ double2 buf[M > 8 ? 2048 : 1];
  constexpr int R0 = M % 8 == 0 ? 8 : (M % 4 == 0 ? 4 : 2), Q0 = 2048 / R0 / 256;
  static_assert(Q0 * R0 == 8, "eight first-stage elements per thread");
  constexpr int GPW = 128 / M;
  const int c0 = blockIdx.x * 16, g0 = blockIdx.y * GPW;
  double2 rr[P][8];
#pragma unroll
  for (int q = 0; q < Q0; ++q) {
    const int b = threadIdx.x + 256 * q;
    const int c = b & 15, rest = b >> 4, gs = rest / (M / R0), j = rest % (M / R0);
    const int g = g0 + gs;
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      const int i = j + r * (M / R0);
      const long long e = (long long)(g * ca.gmul + i * ca.stride) * ca.f.F2p + c0 + c;
#pragma unroll
      for (int p = 0; p < P; ++p) rr[p][q * R0 + r] = g < ca.ngroups ? Rh[p * ca.f.plane + e] : make_double2(0.0, 0.0);
    }
  }
  for (int kk = 0; kk < nk; ++kk) {
    __syncthreads();  // the previous atom's last reads of buf are done
    const ColLoadProduct<P> load{rr, Dh + (long long)(k0 + kk) * P * ca.f.plane};
    col_stages<M, 1>(ca, buf, load, kk);
  }
}

// Shat_kk = sum_p Rhat_p conj(Dhat_(k0+kk),p) for kk < nk at every element of
// the spectra (P <= 8; Dhat stored [k][p]).
__global__ __launch_bounds__(256) void fft_product(long long plane, int P, int k0, int nk,
                                                   const double2 *__restrict__ Rh, const double2 *__restrict__ Dh,
                                                   double2 *__restrict__ Sh) {
  for (long long e = blockIdx.x * 256ll + threadIdx.x; e < plane; e += (long long)gridDim.x * 256) {
    double2 r[8];
#pragma unroll
    for (int p = 0; p < 8; ++p)
      if (p < P) r[p] = Rh[p * plane + e];
    for (int kk = 0; kk < nk; ++kk) {
      const double2 *d = Dh + (long long)(k0 + kk) * P * plane + e;
      double2 acc = make_double2(0.0, 0.0);
#pragma unroll
      for (int p = 0; p < 8; ++p)
        if (p < P) acc = c_add(acc, c_mulc(r[p], d[p * plane]));
      Sh[kk * plane + e] = acc;
    }
  }
}

// The contraction's outputs from G (K, H, W) in FP64, as corr_mfma's epilogue
// writes them: 64 positions per tile, atoms in chunks of 32 through LDS, so
// that both G's rows and the position-major outputs are read and written in
// contiguous runs.
template <int MODE, class Rz>
__global__ __launch_bounds__(256) void fft_epilogue(Geom g, const double *__restrict__ G, CorrOut o) {
  __shared__ double t[32][65];
  __shared__ double sh_red[4];
  const long long HW = (long long)g.H * g.W;
  const int KW = MODE == CORR_BETA ? g.KS : g.K;  // BETA also zeroes the padding atoms
  double red = 0.0, red2 = 0.0;
  for (long long pos0 = blockIdx.x * 64ll; pos0 < HW; pos0 += (long long)gridDim.x * 64) {
    for (int k0 = 0; k0 < KW; k0 += 32) {
      __syncthreads();
      {
        // the chunk's eight G reads of a thread are issued together
        constexpr int NJ = 32 * 64 / 256;
        double gl[NJ];
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj) {
          const int j = threadIdx.x + 256 * jj, kk = j >> 6, pp = j & 63;
          const int k = k0 + kk;
          const long long pos = pos0 + pp;
          gl[jj] = (k < g.K && pos < HW) ? G[k * HW + pos] : 0.0;
        }
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj) {
          const int j = threadIdx.x + 256 * jj;
          t[j >> 6][j & 63] = gl[jj];
        }
      }
      __syncthreads();
      for (int j = threadIdx.x; j < 32 * 64; j += 256) {
        const int kk = j & 31, pp = j >> 5;
        const int k = k0 + kk;
        const long long pos = pos0 + pp;
        if (pos >= HW || k >= KW) continue;
        const double gv = t[kk][pp];
        if (MODE != CORR_ABSMAX && o.g64 && k < g.K) o.g64[pos * g.KS + k] = gv;
        const bool zread = !o.meta || (o.meta[pos] >> 16) != 0;  // z is 0 at positions without non-zeros
        if (MODE == CORR_BETA) {
          double bv = gv;
          if (o.zpm && k < g.K && zread) bv += o.nrm[k] * (double)reinterpret_cast<const Rz *>(o.zpm)[pos * g.KS + k];
          reinterpret_cast<Rz *>(o.beta)[pos * g.KS + k] = k < g.K ? (Rz)bv : Rz(0);
        } else if (MODE == CORR_KKT) {
          const double z = zread ? (double)reinterpret_cast<const Rz *>(o.zpm)[pos * g.KS + k] : 0.0;
          double vv;
          if (z == 0.0)
            vv = o.positive ? fmax(gv - o.lambda, 0.0) : fmax(fabs(gv) - o.lambda, 0.0);
          else
            vv = fabs(gv - (z > 0.0 ? o.lambda : -o.lambda));
          red = fmax(red, vv);
          if (o.beta_cmp)
            red2 = fmax(red2, fabs(gv + o.nrm[k] * z -
                                   (double)reinterpret_cast<const Rz *>(o.beta_cmp)[pos * g.KS + k]));
          if (o.beta) reinterpret_cast<Rz *>(o.beta)[pos * g.KS + k] = (Rz)(gv + o.nrm[k] * z);
        } else {
          red = fmax(red, o.positive ? gv : fabs(gv));
        }
      }
    }
  }
  if (MODE != CORR_BETA) {
    __syncthreads();
    red = block_max<256>(red, sh_red);
    if (threadIdx.x == 0) atomic_max_nonneg(o.result, fmax(red, 0.0));
    if (MODE == CORR_KKT && o.beta_cmp) {
      red2 = block_max<256>(red2, sh_red);
      if (threadIdx.x == 0) atomic_max_nonneg(o.result2, red2);
    }
  }
}

}  // namespace dcdl
