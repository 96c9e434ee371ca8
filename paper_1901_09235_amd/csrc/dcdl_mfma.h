// dcdl_mfma.h -- the dense correlation G = corr(R, D) on the CDNA matrix cores.
//
// G_k[pos] = sum_p sum_t D_{k,p}[t] R_p[pos + t] (the paper's R * D~_k, used by
// beta = corr(X - Z*D, D) + n z of Sec. 3 and by the optimality check) is a
// product of the atom matrix D (K x P|Theta|) with the windows of R: rows are
// atoms, columns are positions, the reduction runs over (t1, channel chunk,
// t2, channel).  One workgroup computes TR rows x TC columns of positions for
// up to 64 atoms; each of its four waves owns NTW 16-position column tiles.
//
//   * the atom operand comes from a packed copy of D laid out so that every
//     lane's fragment of one MFMA step is one coalesced load;
//   * the window operand is staged in LDS as [row][column][channel] for one t1
//     and one chunk of PC channels, so a lane's fragment (consecutive
//     reduction indices) is contiguous in LDS;
//   * F64: v_mfma_f64_16x16x4 (FP64 products and sums, the precision of the
//     final check and the drift correction);  BF16: v_mfma_f32_16x16x32_bf16
//     (BF16 operands, FP32 accumulation);  BF16X3: the same instruction on
//     hi/lo BF16 splits of both operands (hi*hi + hi*lo + lo*hi), close to
//     FP32 accuracy at three BF16 products.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dcdl_kernels.h"

namespace dcdl {

typedef double mf_d4 __attribute__((ext_vector_type(4)));
typedef float mf_f4 __attribute__((ext_vector_type(4)));
typedef __bf16 mf_bf8 __attribute__((ext_vector_type(8)));

enum MfPrec { MF_F64 = 0, MF_BF16 = 1, MF_BF16X3 = 2 };

template <int PREC> struct MfT;
template <> struct MfT<MF_F64> {
  using In = double;   // operand element
  using Acc = double;  // accumulator element
  using C4 = mf_d4;
  static constexpr int KK = 4;      // reduction length of one instruction
  static constexpr int NCOPY = 1;   // operand copies (hi, lo)
};
template <> struct MfT<MF_BF16> {
  using In = __bf16;
  using Acc = float;
  using C4 = mf_f4;
  static constexpr int KK = 32;
  static constexpr int NCOPY = 1;
};
template <> struct MfT<MF_BF16X3> {
  using In = __bf16;
  using Acc = float;
  using C4 = mf_f4;
  static constexpr int KK = 32;
  static constexpr int NCOPY = 2;
};

// Layout of the packed dictionary and of the reduction.
struct MfPlan {
  int PC;    // channels per chunk (FP64: 1 ... 8; BF16: 1, 2, 4 or 8)
  int NPC;   // channel chunks
  int L2p;   // t2 extent padded so that L2p * PC is a multiple of the instruction's reduction
  int SPS;   // instruction steps per (t1, chunk) stage = L2p * PC / KK
  int MTT;   // 16-atom tiles in total = ceil(K / 16)
};

// Packed atom operand: for stage (t1, chunk), step s, atom tile m and lane l,
// the KK/4 values D[16 m + l % 16][p][t1][t2] at reduction indices
// rl = s KK + (l / 16) (KK / 4) + e, (t2, pp) = divmod(rl, PC), p = chunk PC + pp;
// zero outside the atoms, channels and taps.  Copy 1 (BF16X3) holds the low
// halves d - bf16(d).
template <int PREC, class Rd>
__global__ __launch_bounds__(256) void mf_pack_dict(Geom g, MfPlan pl, const Rd *__restrict__ D,
                                                    typename MfT<PREC>::In *__restrict__ out, long long n) {
  using T = MfT<PREC>;
  constexpr int VPL = T::KK / 4;
  for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    const int e = (int)(i % VPL);
    long long q = i / VPL;
    const int lane = (int)(q % 64);
    q /= 64;
    const int m = (int)(q % pl.MTT);
    q /= pl.MTT;
    const int s = (int)(q % pl.SPS);
    q /= pl.SPS;
    const int pc = (int)(q % pl.NPC);
    const int t1 = (int)(q / pl.NPC);
    const int rl = s * T::KK + (lane / 16) * VPL + e;
    const int t2 = rl / pl.PC, pp = rl - (rl / pl.PC) * pl.PC;
    const int k = 16 * m + lane % 16, p = pc * pl.PC + pp;
    double v = 0.0;
    if (k < g.K && p < g.P && t2 < g.L2) v = (double)D[(((long long)k * g.P + p) * g.L1 + t1) * g.L2 + t2];
    if constexpr (PREC == MF_F64) {
      out[i] = (typename T::In)v;
    } else {
      const __bf16 hi = (__bf16)(float)v;
      out[i] = hi;
      if constexpr (T::NCOPY == 2) out[n + i] = (__bf16)((float)v - (float)hi);
    }
  }
}

template <int PREC>
__device__ __forceinline__ typename MfT<PREC>::C4 mf_step(typename MfT<PREC>::C4 c, const void *a, const void *b);

template <>
__device__ __forceinline__ mf_d4 mf_step<MF_F64>(mf_d4 c, const void *a, const void *b) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(*reinterpret_cast<const double *>(a),
                                              *reinterpret_cast<const double *>(b), c, 0, 0, 0);
}
template <>
__device__ __forceinline__ mf_f4 mf_step<MF_BF16>(mf_f4 c, const void *a, const void *b) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(*reinterpret_cast<const mf_bf8 *>(a),
                                                 *reinterpret_cast<const mf_bf8 *>(b), c, 0, 0, 0);
}

// A lane's window fragment: KK/4 consecutive elements at an alignment of
// PC elements (a whole fragment when PC * size >= 16 bytes).
template <int PREC, int PC>
__device__ __forceinline__ void mf_load_b(const typename MfT<PREC>::In *p, typename MfT<PREC>::In *dst) {
  using In = typename MfT<PREC>::In;
  constexpr int VPL = MfT<PREC>::KK / 4;
  if constexpr (VPL == 1) {
    dst[0] = p[0];
  } else {
    constexpr int CH = PC * (int)sizeof(In) >= 16 ? VPL : PC;  // elements per aligned piece
#pragma unroll
    for (int c = 0; c < VPL; c += CH) {
      if (CH * sizeof(In) == 16)
        *reinterpret_cast<uint4 *>(dst + c) = *reinterpret_cast<const uint4 *>(p + c);
      else if (CH * sizeof(In) == 8)
        *reinterpret_cast<uint2 *>(dst + c) = *reinterpret_cast<const uint2 *>(p + c);
      else if (CH * sizeof(In) == 4)
        *reinterpret_cast<uint32_t *>(dst + c) = *reinterpret_cast<const uint32_t *>(p + c);
      else
        *reinterpret_cast<uint16_t *>(dst + c) = *reinterpret_cast<const uint16_t *>(p + c);
    }
  }
}

// BF16 window staging, one (row, column) cell per thread and step: the PC
// channels of the chunk are read (coalesced along the row for each channel)
// and written to LDS as one PC-element store.  Eight cells' loads are issued
// before the first is converted, so a thread has 8 PC reads in flight; the
// cell index advances by 256 without a division per element.  Copy 1
// (NCOPY = 2) holds v - bf16(v).
template <int NCOPY, int PC, class Rin>
__device__ __forceinline__ void mf_stage_cells(const Geom &g, const Rin *__restrict__ X, int pc, int hbase, int w0,
                                               int nrows, int TCX, int copy_elems, __bf16 *xs) {
  constexpr int NB = 8;
  const long long plane = (long long)g.T1 * g.T2;
  const int tid = threadIdx.x, cells = nrows * TCX;
  const int rstep = 256 / TCX, cstep = 256 - rstep * TCX;
  int r = tid / TCX, c = tid - r * TCX;
  for (int e0 = tid; e0 < cells; e0 += 256 * NB) {
    float v[NB][PC];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int hh = hbase + r, ww = w0 + c;
      const bool in = e0 + 256 * b < cells && hh < g.T1 && ww < g.T2;
      const Rin *src = X + (long long)hh * g.T2 + ww;
#pragma unroll
      for (int pp = 0; pp < PC; ++pp) {
        const int p = pc * PC + pp;
        v[b][pp] = in && p < g.P ? (float)src[p * plane] : 0.0f;
      }
      r += rstep;
      c += cstep;
      if (c >= TCX) {
        c -= TCX;
        ++r;
      }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int e = e0 + 256 * b;
      if (e >= cells) break;
      __bf16 hi[PC], lo[PC];
#pragma unroll
      for (int pp = 0; pp < PC; ++pp) {
        hi[pp] = (__bf16)v[b][pp];
        lo[pp] = (__bf16)(v[b][pp] - (float)hi[pp]);
      }
      __bf16 *dst = xs + (long long)e * PC;
#pragma unroll
      for (int cp = 0; cp < NCOPY; ++cp) {
        const __bf16 *hs = cp == 0 ? hi : lo;
        __bf16 *d = dst + cp * copy_elems;
        if constexpr (PC == 8)
          *reinterpret_cast<uint4 *>(d) = *reinterpret_cast<const uint4 *>(hs);
        else if constexpr (PC == 4)
          *reinterpret_cast<uint2 *>(d) = *reinterpret_cast<const uint2 *>(hs);
        else if constexpr (PC == 2)
          *reinterpret_cast<uint32_t *>(d) = *reinterpret_cast<const uint32_t *>(hs);
        else
          d[0] = hs[0];
      }
    }
  }
}

// TR x (4 NTW 16 / TR) positions per workgroup: TR = 1 for signals (the four
// waves side by side along the row), TR = 4 for images (one row per wave).
// PC = 0 takes the channel chunk from the plan (FP64, one element per lane).
// TALL: the window of every t1 is staged once per channel chunk, TR + L1 - 1
// rows (row wr + t1 serves wave wr at tap row t1), instead of TR rows per t1;
// the steps of consecutive t1 then run without a barrier between them.
// SPSC > 0 fixes the steps per stage at compile time: the step loop unrolls
// and window fragments that two (column tile, step) pairs share (the tile
// 16 columns to the right, 16 / (KK / PC) steps earlier) are read once.
template <int PREC, int MODE, int TR, int NTW, int MT, int PC, bool TALL, class Rin, class Rz, int SPSC = 0>
__global__ __launch_bounds__(256) void corr_mfma(Geom g, MfPlan pl, const Rin *__restrict__ X,
                                                 const typename MfT<PREC>::In *__restrict__ Dpk, long long npk,
                                                 int m0, CorrOut o) {
  using T = MfT<PREC>;
  using In = typename T::In;
  using Acc = typename T::Acc;
  constexpr int VPL = T::KK / 4;
  constexpr int TC = (4 / TR) * NTW * 16;  // positions per row
  extern __shared__ __align__(16) unsigned char mf_smem[];
  In *xs = reinterpret_cast<In *>(mf_smem);
  const int pcs = PC > 0 ? PC : pl.PC;
  const int TCX = TC + pl.L2p;  // staged columns
  const int row_elems = TCX * pcs;
  const int nrows = TALL ? TR + g.L1 - 1 : TR;  // staged rows
  const int copy_elems = nrows * row_elems;
  __shared__ double sh_red[4];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int h0 = blockIdx.y * TR, w0 = blockIdx.x * TC;
  const int wr = TR == 1 ? 0 : wave;                      // row of this wave in the tile
  const int wc = TR == 1 ? wave * NTW * 16 : 0;           // first column of this wave
  const long long plane = (long long)g.T1 * g.T2;

  typename T::C4 acc[MT][NTW];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int n = 0; n < NTW; ++n) acc[m][n] = typename T::C4{0, 0, 0, 0};

  for (int pcq = 0; pcq < pl.NPC; ++pcq)
    for (int t1q = 0; t1q < g.L1; ++t1q) {
      // the non-TALL order is (t1, chunk); TALL runs every t1 of a chunk
      const int t1 = TALL ? t1q : (pcq * g.L1 + t1q) / pl.NPC;
      const int pc = TALL ? pcq : (pcq * g.L1 + t1q) % pl.NPC;
      if (!TALL || t1 == 0) {
        __syncthreads();
        // stage rows h0 + (TALL ? 0 : t1) + r, columns w0 + c, channels pc PC + pp
        const int hbase = h0 + (TALL ? 0 : t1);
        if constexpr (PREC != MF_F64 && PC > 0) {
          mf_stage_cells<T::NCOPY, PC>(g, X, pc, hbase, w0, nrows, TCX, copy_elems, xs);
        } else
        for (int e = tid; e < copy_elems; e += 256) {
          const int c = e % TCX, rest = e / TCX;
          const int pp = rest % pcs, r = rest / pcs;
          const int p = pc * pcs + pp, hh = hbase + r, ww = w0 + c;
          double v = 0.0;
          if (p < g.P && hh < g.T1 && ww < g.T2) v = (double)X[p * plane + (long long)hh * g.T2 + ww];
          const int li = r * row_elems + c * pcs + pp;
          if constexpr (PREC == MF_F64) {
            xs[li] = (In)v;
          } else {
            const __bf16 hi = (__bf16)(float)v;
            xs[li] = hi;
            if constexpr (T::NCOPY == 2) xs[copy_elems + li] = (__bf16)((float)v - (float)hi);
          }
        }
        __syncthreads();
      }
      const long long sbase = ((long long)(t1 * pl.NPC + pc) * pl.SPS) * pl.MTT;
      const In *xrow = xs + (wr + (TALL ? t1 : 0)) * row_elems;
      const In *arow = Dpk + ((sbase + m0) * 64 + lane) * VPL;  // step 0, tile m0 of this stage
      const long long astep = (long long)pl.MTT * 64 * VPL;
      auto step = [&](int s) {
        In a[T::NCOPY][MT][VPL];
#pragma unroll
        for (int m = 0; m < MT; ++m) {
          const In *ap = arow + s * astep + m * 64 * VPL;
#pragma unroll
          for (int cp = 0; cp < T::NCOPY; ++cp) {
            if constexpr (VPL == 1)
              a[cp][m][0] = ap[cp * npk];
            else
              *reinterpret_cast<uint4 *>(a[cp][m]) = *reinterpret_cast<const uint4 *>(ap + cp * npk);
          }
        }
        const int rl = s * T::KK + (lane >> 4) * VPL;  // first reduction index of this lane
#pragma unroll
        for (int n = 0; n < NTW; ++n) {
          const int col = wc + n * 16 + (lane & 15);
          In b[T::NCOPY][VPL];
#pragma unroll
          for (int cp = 0; cp < T::NCOPY; ++cp) mf_load_b<PREC, PC>(xrow + cp * copy_elems + col * pcs + rl, b[cp]);
#pragma unroll
          for (int m = 0; m < MT; ++m) {
            if constexpr (PREC == MF_F64) {
              acc[m][n] = mf_step<MF_F64>(acc[m][n], a[0][m], b[0]);
            } else {
              acc[m][n] = mf_step<MF_BF16>(acc[m][n], a[0][m], b[0]);
              if constexpr (T::NCOPY == 2) {
                acc[m][n] = mf_step<MF_BF16>(acc[m][n], a[0][m], b[1]);
                acc[m][n] = mf_step<MF_BF16>(acc[m][n], a[1][m], b[0]);
              }
            }
          }
        }
      };
      if constexpr (SPSC > 0) {
#pragma unroll
        for (int s = 0; s < SPSC; ++s) step(s);
      } else {
        for (int s = 0; s < pl.SPS; ++s) step(s);
      }
    }

  // epilogue: register v of a lane holds position column (lane % 16) and, in
  // the 16-atom tile, row (lane / 16) + 4 v for the FP64 instruction and row
  // 4 (lane / 16) + v for the BF16 one
  double red = 0.0, red2 = 0.0;
  const int hh = h0 + wr;
#pragma unroll
  for (int n = 0; n < NTW; ++n) {
    const int ww = w0 + wc + n * 16 + (lane & 15);
    if (hh >= g.H || ww >= g.W) continue;
    const long long pos = (long long)hh * g.W + ww;
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = 16 * (m0 + m) + (PREC == MF_F64 ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v);
        const double gv = (double)acc[m][n][v];
        if (MODE != CORR_ABSMAX && o.g64 && k < g.K) o.g64[pos * g.KS + k] = gv;
        if (MODE == CORR_BETA) {
          if (k < g.K) {
            double bv = gv;
            if (o.zpm) bv += o.nrm[k] * (double)reinterpret_cast<const Rz *>(o.zpm)[pos * g.KS + k];
            reinterpret_cast<Rz *>(o.beta)[pos * g.KS + k] = (Rz)bv;
          } else if (k < g.KS) {
            reinterpret_cast<Rz *>(o.beta)[pos * g.KS + k] = Rz(0);
          }
        } else if (k < g.K) {
          if (MODE == CORR_KKT) {
            const double z = (double)reinterpret_cast<const Rz *>(o.zpm)[pos * g.KS + k];
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
    red = block_max<256>(red, sh_red);
    if (tid == 0) atomic_max_nonneg(o.result, fmax(red, 0.0));
    if (MODE == CORR_KKT && o.beta_cmp) {
      __syncthreads();
      red2 = block_max<256>(red2, sh_red);
      if (tid == 0) atomic_max_nonneg(o.result2, red2);
    }
  }
}

}  // namespace dcdl
