// dcdl_check.h -- the FP64 objective/KKT check of a solve, carried forward
// from an earlier FP64 contraction instead of recomputed densely.
//
// The negative gradient g = corr(X - Z*D, D) is linear in Z, so from an
// iterate z_ref whose g_ref and residual r_ref = X - z_ref*D are known in FP64
// (the output of a dense FP64 contraction), the current iterate z has
//   g_k[w] = g_ref,k[w] - sum over changed coordinates (k0, w0) of
//            C[k0][k][w0 - w] (z - z_ref)_k0[w0],   w in V(w0)
//   r      = r_ref - sum over changed coordinates of (z - z_ref)_k0[w0] e_w0 * D_k0
// (Sec. 3, eq. beta_update, here in FP64 and for g rather than beta).  The
// work is proportional to the number of changed coordinates times
// K (2L1-1)(2L2-1), against K P L1 L2 per position for the dense contraction.
//
//   diff_changes    lists (position, atom, z - z_ref) of every changed
//                   coordinate (wave-aggregated append), with sum |z| and the
//                   non-zero count of z;
//   residual_scatter  r -= dz e_w0 * D_k0, FP64 atomics;
//   bin_count / bin_scan / bin_fill
//                   CSR lists of the changes whose V(w0) meets each output
//                   tile of TH x TW positions;
//   g_update_kkt    one workgroup per tile, two-atom pieces spread over the
//                   threads: g from g_ref and the tile's changes, the strict KKT violation,
//                   the drift of the maintained beta, beta = g + n z for a
//                   polish pass, and the new reference (g_ref <- g, z_ref <- z).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dcdl_kernels.h"

namespace dcdl {

struct Change {
  int32_t pos;  // h W + w on the valid domain
  int32_t k;
  double delta;
};

constexpr int kChkTH = 8, kChkTW = 32;  // output tile of g_update_kkt (256 positions)

// acc[0] += sum |z|, acc[1] += nnz(z); changes appended while *count < cap
// (the count keeps growing past cap so the host sees the true number).
template <class R>
__global__ __launch_bounds__(256) void diff_changes(long long HW, int K, int KS, const R *__restrict__ z,
                                                    const R *__restrict__ zref, Change *__restrict__ out,
                                                    unsigned long long *count, long long cap, double *acc) {
  __shared__ double sh[4];
  double l1 = 0.0, nnz = 0.0;
  const long long n = HW * KS;
  const int lane = threadIdx.x & 63;
  for (long long base = (long long)blockIdx.x * 256; base < n; base += (long long)gridDim.x * 256) {
    const long long e = base + threadIdx.x;
    bool ch = false;
    double d = 0.0;
    int pos = 0, k = 0;
    if (e < n) {
      pos = (int)(e / KS);
      k = (int)(e - (long long)pos * KS);
      if (k < K) {
        const double zv = (double)z[e], zr = (double)zref[e];
        l1 += fabs(zv);
        nnz += zv != 0.0 ? 1.0 : 0.0;
        d = zv - zr;
        ch = d != 0.0;
      }
    }
    const unsigned long long m = __ballot(ch);
    if (m) {
      unsigned long long first = 0;
      const int leader = __ffsll((long long)m) - 1;
      if (lane == leader) first = atomicAdd(count, (unsigned long long)__popcll(m));
      first = __shfl(first, leader, 64);
      if (ch) {
        const unsigned long long idx = first + __popcll(m & ((1ull << lane) - 1ull));
        if ((long long)idx < cap) {
          Change c;
          c.pos = pos;
          c.k = k;
          c.delta = d;
          out[idx] = c;
        }
      }
    }
  }
  l1 = block_sum<256>(l1, sh);
  nnz = block_sum<256>(nnz, sh);
  if (threadIdx.x == 0) {
    atomicAdd(acc, l1);
    atomicAdd(acc + 1, nnz);
  }
}

// r_p[w0 + t] -= dz D_k0,p[t] for every listed change (one workgroup per
// change at a time).
__global__ __launch_bounds__(256) void residual_scatter(Geom g, const Change *__restrict__ ch, long long n,
                                                        const double *__restrict__ D64, double *__restrict__ res) {
  const int PL = g.P * g.L1 * g.L2, LL = g.L1 * g.L2;
  const long long plane = (long long)g.T1 * g.T2;
  for (long long j = blockIdx.x; j < n; j += gridDim.x) {
    const Change c = ch[j];
    const int h0 = c.pos / g.W, w0 = c.pos - (c.pos / g.W) * g.W;
    const double *d = D64 + (long long)c.k * PL;
    for (int i = threadIdx.x; i < PL; i += 256) {
      const int p = i / LL, t = i - p * LL;
      const int t1 = t / g.L2, t2 = t - (t / g.L2) * g.L2;
      atomicAdd(res + p * plane + (long long)(h0 + t1) * g.T2 + (w0 + t2), -c.delta * d[i]);
    }
  }
}

// Tiles (rows [tr TH, tr TH + TH), columns [tc TW, tc TW + TW)) that V(w0)
// of a change meets.
__device__ __forceinline__ void change_tiles(const Geom &g, int pos, int *r0, int *r1, int *c0, int *c1) {
  const int h0 = pos / g.W, w0 = pos - (pos / g.W) * g.W;
  *r0 = max(0, h0 - g.L1 + 1) / kChkTH;
  *r1 = min(g.H - 1, h0 + g.L1 - 1) / kChkTH;
  *c0 = max(0, w0 - g.L2 + 1) / kChkTW;
  *c1 = min(g.W - 1, w0 + g.L2 - 1) / kChkTW;
}

__global__ __launch_bounds__(256) void bin_count(Geom g, const Change *__restrict__ ch, long long n, int ntc,
                                                 unsigned *__restrict__ cnt) {
  for (long long j = (long long)blockIdx.x * 256 + threadIdx.x; j < n; j += (long long)gridDim.x * 256) {
    int r0, r1, c0, c1;
    change_tiles(g, ch[j].pos, &r0, &r1, &c0, &c1);
    for (int r = r0; r <= r1; ++r)
      for (int c = c0; c <= c1; ++c) atomicAdd(cnt + (long long)r * ntc + c, 1u);
  }
}

// Exclusive scan of n counts into off[0..n] (one workgroup of 1024 threads),
// and the fill cursors reset to the offsets.
__global__ __launch_bounds__(1024) void bin_scan(const unsigned *__restrict__ cnt, long long n,
                                                 unsigned *__restrict__ off, unsigned *__restrict__ cur) {
  __shared__ unsigned long long part[1024];
  const long long per = (n + 1023) / 1024;
  const long long b = threadIdx.x * per, e = min(n, b + per);
  unsigned long long s = 0;
  for (long long i = b; i < e; ++i) s += cnt[i];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long run = 0;
    for (int t = 0; t < 1024; ++t) {
      const unsigned long long v = part[t];
      part[t] = run;
      run += v;
    }
    off[n] = (unsigned)run;
  }
  __syncthreads();
  unsigned long long run = part[threadIdx.x];
  for (long long i = b; i < e; ++i) {
    off[i] = (unsigned)run;
    cur[i] = (unsigned)run;
    run += cnt[i];
  }
}

__global__ __launch_bounds__(256) void bin_fill(Geom g, const Change *__restrict__ ch, long long n, int ntc,
                                                unsigned *__restrict__ cur, unsigned *__restrict__ list) {
  for (long long j = (long long)blockIdx.x * 256 + threadIdx.x; j < n; j += (long long)gridDim.x * 256) {
    int r0, r1, c0, c1;
    change_tiles(g, ch[j].pos, &r0, &r1, &c0, &c1);
    for (int r = r0; r <= r1; ++r)
      for (int c = c0; c <= c1; ++c) list[atomicAdd(cur + (long long)r * ntc + c, 1u)] = (unsigned)j;
  }
}

struct IncOut {
  double lambda;
  int positive;
  const double *nrm;  // n_k in FP64
  double *result;     // [0] max strict-KKT violation, [1] max |beta - (g + n z)| (if beta_cmp)
  const void *beta_cmp;  // the maintained beta (HW, KS) in R, optional
  void *beta;            // receives g + n z in R (may alias beta_cmp), optional
};

// One workgroup per output tile of TH x TW = 256 positions.  The tile's
// values are cut into pieces of two atoms (16 bytes of FP64) for up to 32
// atoms at a time, NPc pieces per position; piece P = t + 256 j (j < NPc) is
// held by thread t, so consecutive lanes hold consecutive pieces and a change's
// update-table reads for a tile row (consecutive positions, KS64 atoms each)
// are contiguous 16-byte loads across the wave.  A64[k0][d1][d2][k] =
// C[k0][k][-tau] at d = tau + L - 1 (atom stride KS64, even), as the round
// kernel's update table.
template <class R>
__global__ __launch_bounds__(256) void g_update_kkt(Geom g, const Change *__restrict__ ch,
                                                    const unsigned *__restrict__ off,
                                                    const unsigned *__restrict__ list,
                                                    const double *__restrict__ A64, int KS64, int ntc,
                                                    double *__restrict__ gref, const R *__restrict__ z,
                                                    R *__restrict__ zref, IncOut o) {
  constexpr int NPMAX = 16;  // pieces per thread: 32 atoms per pass
  __shared__ double sh[4];
  const int tile = blockIdx.x;
  const int tr = tile / ntc, tc = tile - (tile / ntc) * ntc;
  const unsigned lb = off[tile], le = off[tile + 1];
  double red = 0.0, red2 = 0.0;
  for (int kb = 0; kb < g.K; kb += 2 * NPMAX) {
    const int npc = min(NPMAX, (min(g.K - kb, 2 * NPMAX) + 1) / 2);  // pieces per position
    int ph[NPMAX], pw[NPMAX], pk[NPMAX];
    double2 acc[NPMAX];
#pragma unroll
    for (int j = 0; j < NPMAX; ++j) {
      ph[j] = -1;
      acc[j] = make_double2(0.0, 0.0);
      if (j >= npc) continue;
      const int P = threadIdx.x + 256 * j;
      const int pl = P / npc, a = P - (P / npc) * npc;
      const int h = tr * kChkTH + pl / kChkTW, w = tc * kChkTW + pl % kChkTW;
      pk[j] = kb + 2 * a;
      if (h < g.H && w < g.W) {
        ph[j] = h;
        pw[j] = w;
        const double *gp = gref + ((long long)h * g.W + w) * g.KS + pk[j];
        acc[j].x = gp[0];
        acc[j].y = pk[j] + 1 < g.K ? gp[1] : 0.0;
      }
    }
    for (unsigned li = lb; li < le; ++li) {
      const Change c = ch[list[li]];
      const int h0 = c.pos / g.W, w0 = c.pos - (c.pos / g.W) * g.W;
      const double *base = A64 + (long long)c.k * g.U1 * g.U2 * KS64;
#pragma unroll
      for (int j = 0; j < NPMAX; ++j) {
        if (ph[j] < 0) continue;
        const int d1 = ph[j] - h0 + g.L1 - 1, d2 = pw[j] - w0 + g.L2 - 1;
        if (d1 < 0 || d1 >= g.U1 || d2 < 0 || d2 >= g.U2) continue;
        const double2 t = *reinterpret_cast<const double2 *>(base + ((long long)d1 * g.U2 + d2) * KS64 + pk[j]);
        acc[j].x -= t.x * c.delta;
        acc[j].y -= t.y * c.delta;
      }
    }
#pragma unroll
    for (int j = 0; j < NPMAX; ++j) {
      if (ph[j] < 0) continue;
      const long long e0 = ((long long)ph[j] * g.W + pw[j]) * g.KS + pk[j];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int k = pk[j] + q;
        if (k >= g.K) break;
        const long long e = e0 + q;
        const double gv = q == 0 ? acc[j].x : acc[j].y, zv = (double)z[e];
        gref[e] = gv;
        zref[e] = z[e];
        double v;
        if (zv == 0.0)
          v = o.positive ? fmax(gv - o.lambda, 0.0) : fmax(fabs(gv) - o.lambda, 0.0);
        else
          v = fabs(gv - (zv > 0.0 ? o.lambda : -o.lambda));
        red = fmax(red, v);
        const double bn = gv + o.nrm[k] * zv;
        if (o.beta_cmp) red2 = fmax(red2, fabs(bn - (double)reinterpret_cast<const R *>(o.beta_cmp)[e]));
        if (o.beta) reinterpret_cast<R *>(o.beta)[e] = (R)bn;
      }
    }
  }
  red = block_max<256>(red, sh);
  if (threadIdx.x == 0) atomic_max_nonneg(o.result, red);
  if (o.beta_cmp) {
    red2 = block_max<256>(red2, sh);
    if (threadIdx.x == 0) atomic_max_nonneg(o.result + 1, red2);
  }
}

}  // namespace dcdl
