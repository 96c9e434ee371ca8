// dcdl_device.h -- gfx950 device code of the DiCoDiLe CSC library.
//
// Internal layout (all on the device):
//   beta, z : position-major (H, W, KS), the atom index innermost and padded
//             to KS = K rounded up to a 16-byte vector (4 floats or 2 doubles;
//             padding entries stay 0).  The beta patch of one update (Sec. 3,
//             eq. beta_update) is (2L1-1) contiguous, 16-byte aligned runs of
//             (2L2-1)*KS values, read and written as vectors.
//   score   : per position, the best move score over its K atoms (Alg. 1's
//             selection key); read by neighbouring workers, so it is accessed
//             with coherent atomics.
//   meta    : per position, the atom of that best move (low 16 bits) and the
//             number of non-zero atoms (high 16 bits); private to the owner.
//   A       : apply table A[k0][d1][d2][k] = DtD[k][k0][d1][d2] (k padded to KS):
//             the row of eq. beta_update for an update of atom k0, indexed by
//             the offset d = w - w0 + L - 1 of the patched position w.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dcdl {

template <class R> struct Vec;
template <> struct Vec<float> {
  typedef float4 T;
  static constexpr int N = 4;
  static __device__ __forceinline__ float get(const float4 &v, int e) {
    return e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w;
  }
  static __device__ __forceinline__ float4 fma_neg(float4 b, float4 a, float d) {
    return make_float4(b.x - a.x * d, b.y - a.y * d, b.z - a.z * d, b.w - a.w * d);
  }
  static __device__ __forceinline__ float4 zero() { return make_float4(0.f, 0.f, 0.f, 0.f); }
  static __device__ __forceinline__ void set(float4 &v, int e, float x) {
    if (e == 0) v.x = x;
    else if (e == 1) v.y = x;
    else if (e == 2) v.z = x;
    else v.w = x;
  }
};
template <> struct Vec<double> {
  typedef double2 T;
  static constexpr int N = 2;
  static __device__ __forceinline__ double get(const double2 &v, int e) { return e == 0 ? v.x : v.y; }
  static __device__ __forceinline__ double2 fma_neg(double2 b, double2 a, double d) {
    return make_double2(b.x - a.x * d, b.y - a.y * d);
  }
  static __device__ __forceinline__ double2 zero() { return make_double2(0.0, 0.0); }
  static __device__ __forceinline__ void set(double2 &v, int e, double x) {
    if (e == 0) v.x = x;
    else v.y = x;
  }
};

// Padded atom stride: K rounded up to a whole vector.
__host__ __device__ inline int atom_stride(int K, int elem_bytes) {
  const int ve = 16 / elem_bytes;
  return (K + ve - 1) / ve * ve;
}

// Per-instance control block, followed in memory by a ring of kRing 64-bit
// per-round counters (completions in the low word, quiet workers in the high
// word).
struct Ctl {
  int32_t converged;
  int32_t stop;
  int32_t status;  // 0 ok, 1 round cap, 2 diverged, 3 neighbour wait timed out
  int32_t max_round;
  int32_t sweeps_done;
  int32_t pad[3];
  unsigned long long n_updates, n_candidates, n_softlocked;
  unsigned long long n_visits;        // rounds in which a worker scanned a sub-domain
  unsigned long long n_checked;       // positions read by soft-lock tests
  unsigned long long n_patched;       // positions of beta patched (summed over workers)
  unsigned long long tk_wait, tk_select, tk_collect, tk_apply;  // clock ticks summed over workers
};
constexpr int kRing = 4096;

// Everything one instance of eq. csc needs inside the round kernel.
template <class R> struct Inst {
  int K, KS, L1, L2, U1, U2;
  int H, W;
  int W1, W2, tile1, tile2, mmax, wg_base;
  int inner;  // sub-domain visits per round (at most Mw); 0 -> 1
  int positive, certify, soft_lock;
  int strategy;  // dcdl_select: 0 LGCD, 1 greedy, 2 cyclic (both through tile1/tile2), 3 random
  R lambda, tol, div_guard;
  long long max_rounds;
  long long budget_ticks;  // wall-clock cap of one launch, 100 MHz clock ticks
  unsigned long long seed;  // generator seed of the random rule
  R *beta, *z;
  R *score;        // shared: coherent accesses only
  uint32_t *meta;  // private to the owning worker
  const R *A, *inv_n;
  unsigned long long *cand;  // 2 words per worker
  int *prog;
  Ctl *ctl;
  int *ring;  // kRing 64-bit slots: completions (low word) and quiet workers (high word) of a round
  // optional, 2 per worker: visits so far and the quiet count, loaded at the
  // start of a launch and stored at its end, so that a solve split over
  // several launches (each capped by max_rounds) keeps its stopping state
  long long *wstate;
  // optional round log: for rounds r < audit_rounds, audit[r * W1 W2 + w]
  // records worker w's published candidate (audit_record)
  unsigned long long *audit;
  int audit_rounds;
};

// A worker's published candidate of one round: 0 when it had none; otherwise
// bit 63 set, bit 62 set if it passed the soft-lock test (and was applied),
// the atom in bits 32..47 and the position (row-major in the valid domain)
// in bits 0..31.
__device__ __forceinline__ unsigned long long audit_record(bool has, bool accepted, int k0, int pos) {
  if (!has) return 0ull;
  return (1ull << 63) | ((accepted ? 1ull : 0ull) << 62) | ((unsigned long long)(k0 & 0xffff) << 32) |
         (unsigned long long)(unsigned)pos;
}

// ----------------------------------------------------------------- arithmetic

// Closed-form coordinate target of eq. pb_coord: ST(b, lambda) / ||D_k||^2,
// one-sided when positive.  The product is rounded on its own (no
// contraction into a later subtraction): the move score |zn - z| must be that
// of the value z takes, or a coordinate at its target keeps a score of the
// size of zn's rounding error and a tolerance below it is never certified.
template <class R>
__device__ __forceinline__ R st_target(R b, R lam, R inv_n, int positive) {
#pragma clang fp contract(off)
  R u;
  if (positive)
    u = b > lam ? b - lam : R(0);
  else
    u = b > lam ? b - lam : (b < -lam ? b + lam : R(0));
  return u * inv_n;
}

// Selection score of the move z -> zn: |zn - z|, raised to at least tol for a
// move that changes the support or the sign when certify is set.
template <class R>
__device__ __forceinline__ R move_score(R z, R zn, R tol, int certify) {
  R dz = zn > z ? zn - z : z - zn;
  if (certify && z != R(0) && (zn == R(0) || ((zn > R(0)) != (z > R(0)))))
    dz = dz > tol ? dz : tol;
  return dz;
}

// Counter-based draw of the random selection rule: SplitMix64 (Steele, Lea
// and Flood, OOPSLA 2014).  Its n-th output from seed s mixes
// s + (n + 1) * 0x9e3779b97f4a7c15 with two xor-shift-multiply steps and a
// final xor-shift; worker w draws at counter n + w * 2^40.
__device__ __forceinline__ unsigned long long sm64_draw(unsigned long long seed, unsigned long long w,
                                                        unsigned long long n) {
  unsigned long long x = seed + ((w << 40) + n + 1ull) * 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}

__device__ __forceinline__ int part_start(int j, int N, int Wn) {
  return (int)(((long long)j * N) / Wn);
}
__device__ __forceinline__ int part_owner(int x, int N, int Wn) {
  return (int)((((long long)x + 1) * Wn - 1) / N);
}

// ------------------------------------------------------------ synchronisation
//
// Workers exchange three kinds of data: the cached best move of positions on
// their borders (read by the soft-lock test of a neighbour), the candidate of
// each round and a progress counter.  These are read and written only with
// relaxed agent-scope atomics, which are coherent across the chip's L2
// caches; a writer waits for its atomic stores to complete (vmcnt 0) before it
// publishes the progress counter or the tag of a candidate, and a reader
// issues its reads after it observed that counter or tag.  beta, z and the
// DtD table are only ever touched by one workgroup during a launch and stay
// in ordinary cached memory, so no cache write-back or invalidation is
// needed between rounds.

__device__ __forceinline__ unsigned long long ld_shared_u64(const unsigned long long *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_shared_u64(unsigned long long *p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_shared_i32(const int *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_shared_i32(int *p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Wait until every vector memory operation this wave issued has completed.
__device__ __forceinline__ void wait_vm() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0), expcnt/lgkmcnt untouched
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Shared best-move scores, accessed atomically.
__device__ __forceinline__ float score_ld(const float *p) {
  return __uint_as_float(__hip_atomic_load(reinterpret_cast<const unsigned *>(p), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ double score_ld(const double *p) {
  return __longlong_as_double((long long)ld_shared_u64(reinterpret_cast<const unsigned long long *>(p)));
}
__device__ __forceinline__ void score_st(float *p, float v) {
  __hip_atomic_store(reinterpret_cast<unsigned *>(p), __float_as_uint(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void score_st(double *p, double v) {
  st_shared_u64(reinterpret_cast<unsigned long long *>(p), (unsigned long long)__double_as_longlong(v));
}
__device__ __forceinline__ uint32_t meta_pack(int argk, int nzc) { return (uint32_t)argk | ((uint32_t)nzc << 16); }
__device__ __forceinline__ int meta_argk(uint32_t m) { return (int)(m & 0xffffu); }
__device__ __forceinline__ int meta_nzc(uint32_t m) { return (int)(m >> 16); }

// A candidate is two 64-bit words: the delta (word 1) and a tag word (word 0)
// holding the round (22 bits), the atom (10 bits) and the position (32 bits;
// all ones for "no accepted candidate").  Word 1 is stored and completed
// before word 0.
constexpr unsigned kNoPos = 0xffffffffu;
constexpr int kRoundBits = 22;
__device__ __forceinline__ unsigned long long cand_tag(int r, int k0, unsigned pos) {
  return ((unsigned long long)(r & ((1 << kRoundBits) - 1)) << 42) | ((unsigned long long)(k0 & 0x3ff) << 32) |
         (unsigned long long)pos;
}
__device__ __forceinline__ int tag_round(unsigned long long t) { return (int)(t >> 42); }
__device__ __forceinline__ int tag_k0(unsigned long long t) { return (int)((t >> 32) & 0x3ff); }
__device__ __forceinline__ unsigned tag_pos(unsigned long long t) { return (unsigned)(t & 0xffffffffull); }

template <class R> __device__ __forceinline__ unsigned long long delta_bits(R d);
template <> __device__ __forceinline__ unsigned long long delta_bits<float>(float d) { return __float_as_uint(d); }
template <> __device__ __forceinline__ unsigned long long delta_bits<double>(double d) {
  return (unsigned long long)__double_as_longlong(d);
}
template <class R> __device__ __forceinline__ R bits_delta(unsigned long long v);
template <> __device__ __forceinline__ float bits_delta<float>(unsigned long long v) { return __uint_as_float((unsigned)v); }
template <> __device__ __forceinline__ double bits_delta<double>(unsigned long long v) {
  return __longlong_as_double((long long)v);
}

// Progress counters of the workers in `nbr` must reach `target`.  Returns
// false after `timeout_ticks` of the 100 MHz clock.
__device__ __forceinline__ bool wait_progress(const int *prog, const int *sh_nbr, int nn, int self, int target,
                                              long long timeout_ticks, int *sh_ok) {
  // lanes 0..nn-1 of the first wave each watch one neighbour, so the polls of
  // all neighbours are in flight together
  const int q = threadIdx.x;
  if (q < nn) {
    int ok = 1;
    const int n = sh_nbr[q];
    if (n != self) {
      const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
      while (ld_shared_i32(prog + n) < target) {
        __builtin_amdgcn_s_sleep(1);
        if ((long long)(__builtin_amdgcn_s_memrealtime() - t0) > timeout_ticks) {
          ok = 0;
          break;
        }
      }
    }
    sh_ok[q] = ok;
  }
  __syncthreads();
  int ok = 1;
  for (int k = 0; k < nn; ++k) ok &= sh_ok[k];
  return ok != 0;
}

// ------------------------------------------------------------ block reductions

// Largest (score, -pos): larger score wins, equal scores go to the lower pos.
template <class R, int NT>
__device__ __forceinline__ void block_argmax(R &s, int &pos, R *sh_s, int *sh_p) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    R os = __shfl_xor(s, off, 64);
    int op = __shfl_xor(pos, off, 64);
    if (os > s || (os == s && op < pos)) {
      s = os;
      pos = op;
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    sh_s[wave] = s;
    sh_p[wave] = pos;
  }
  __syncthreads();
  s = sh_s[0];
  pos = sh_p[0];
#pragma unroll
  for (int q = 1; q < NT / 64; ++q) {
    R os = sh_s[q];
    int op = sh_p[q];
    if (os > s || (os == s && op < pos)) {
      s = os;
      pos = op;
    }
  }
  __syncthreads();
}

template <int NT>
__device__ __forceinline__ int block_or(int v, int *sh) {
  v = __any(v) ? 1 : 0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  int r = 0;
#pragma unroll
  for (int q = 0; q < NT / 64; ++q) r |= sh[q];
  __syncthreads();
  return r;
}

// ------------------------------------------------------------- the round kernel

// Items (position, atom-group pair) one LDS block of a patch holds: 24 KB of
// best-move staging for FP32 and 20 KB for FP64, so that four FP32 or three
// FP64 workers share a CU.
template <class R> struct PatchBuf {
  static constexpr int N = sizeof(R) == 4 ? 4096 : 2048;
};

// Words of the LDS bitmask that marks the positions of S_w holding a non-zero
// coordinate (workers of up to 32 * kNzWords positions keep one).
constexpr int kNzWords = 1024;

// Rows and columns of one patch block whose cover masks (the updates whose
// patch covers that row or column) are tabulated in LDS.
constexpr int kMaskRows = 128, kMaskCols = 512;

template <class R, int NT> struct PatchCtx {
  R *sh_ps;
  uint16_t *sh_pk;
  uint32_t *rowm, *colm;  // cover masks of a block's rows and columns
  const R *sh_inv_n;
  uint32_t *nzb;    // bit (h - a1) * ext2 + (w - a2) set when position (h, w) of S_w has a non-zero;
                    // null for larger workers, whose patches read z everywhere
  int G;            // 16-byte atom groups per position
  int a1, a2, ext2;  // origin and width of S_w
};

__device__ __forceinline__ void nzb_put(uint32_t *nzb, int t, bool on) {
  if (on)
    nzb[t >> 5] |= 1u << (t & 31);
  else
    nzb[t >> 5] &= ~(1u << (t & 31));
}

// An accepted update as the apply phase uses it: atom k0 at (ch, cw0), change
// delta, and the rows [r1, r2) x columns [c1, c2) of this worker's region it
// patches.
template <class R> struct UCand {
  int k0, ch, cw0, r1, r2, c1, c2;
  int aoff;  // element offset in A of (row 0, column 0) for this update: ((k0 U1 - ch + L1 - 1) U2 - cw0 + L2 - 1) KS
  R delta;
};

// Applies every update of `uc` to this worker's region in one pass over the
// bounding box [R1, R2) x [C1, C2) of their patches: each position reads beta
// once, subtracts the contributions of the updates whose patch covers it
// (eq. beta_update; the updated coordinate of each update keeps its value from
// before that update), writes beta once and recomputes its best-move cache
// once.  Positions no update covers are left untouched.  The sum runs over
// the updates in increasing worker order, as applying them one after another
// would.  Every thread of the workgroup takes part.
//
// The box is cut into blocks of at most LBUF items (a position and a pair of
// its atom groups), each block with LDS tables of the updates covering its
// rows and its columns.  A thread runs one item per pass with all its reads
// in flight before any is used: beta, the DtD row and, where the worker's LDS
// bitmask marks a non-zero coordinate, z.  The items' best moves meet in LDS,
// and a last pass reduces them per position into the score cache and the
// atom half of meta.

// n / d for 0 <= n < 8192 and 1 <= d <= 8192, with m = rcp_of(d): a
// multiply-high by floor((2^32 - 1) / d) + 1, exact in that range (checked
// over all of it); d = 1, whose reciprocal does not fit 32 bits, is passed through.
__device__ __forceinline__ unsigned rcp_of(int d) { return d > 1 ? 0xffffffffu / (unsigned)d + 1u : 0u; }
__device__ __forceinline__ int div_rcp(int n, int d, unsigned m) { return d > 1 ? (int)__umulhi((unsigned)n, m) : n; }

// A patch item is a position and a pair of its 16-byte atom groups (2 q2 and,
// if it exists, 2 q2 + 1): the row, column, cover and address work of an item
// serves eight FP32 (four FP64) atoms, and its six vector reads are in flight
// together.
template <class R> struct PItem {
  typename Vec<R>::T b0, b1, a0, a1, z0, z1;
  int q2, rr, cc;
  unsigned m;  // updates covering the item's position, the first one's DtD row in a0/a1
  bool two;    // the second group exists (an odd group count leaves the last pair half)
};

// Item `it` of a block of rows [rr0, ...) x columns [cc0, cc0 + ng / G2): its
// row, column and group pair from two multiply-high divisions (div_rcp with
// the block's reciprocals mng of ng and mg of G2), its cover mask from the
// block's row and column tables, then its memory reads.
template <class R, int NT>
__device__ __forceinline__ void pitem_load(const Inst<R> &I, const PatchCtx<R, NT> &P, const UCand<R> *uc, int it,
                                           int nit, int rr0, int cc0, int ng, int G2, unsigned mng, unsigned mg,
                                           int rowstride, PItem<R> &x) {
  typedef typename Vec<R>::T V;
  constexpr int VE = Vec<R>::N;
  x.m = 0;
  if (it >= nit) return;
  const int tr = div_rcp(it, ng, mng);
  const int rem = it - tr * ng;
  const int pl = div_rcp(rem, G2, mg);
  x.q2 = rem - pl * G2;
  x.rr = rr0 + tr;
  x.cc = cc0 + pl;
  x.m = P.rowm[tr] & P.colm[pl];
  if (!x.m) return;
  x.two = 2 * x.q2 + 1 < P.G;
  const long long e = ((long long)x.rr * I.W + x.cc) * I.KS + 2 * x.q2 * VE;
  const long long ea = uc[__ffs(x.m) - 1].aoff + x.rr * rowstride + x.cc * I.KS + 2 * x.q2 * VE;
  x.b0 = *reinterpret_cast<const V *>(I.beta + e);
  x.b1 = x.two ? *reinterpret_cast<const V *>(I.beta + e + VE) : Vec<R>::zero();
  x.a0 = *reinterpret_cast<const V *>(I.A + ea);
  x.a1 = x.two ? *reinterpret_cast<const V *>(I.A + ea + VE) : Vec<R>::zero();
  bool nz = true;
  if (P.nzb) {
    const int lt = (x.rr - P.a1) * P.ext2 + (x.cc - P.a2);
    nz = (P.nzb[lt >> 5] >> (lt & 31)) & 1u;
  }
  x.z0 = nz ? *reinterpret_cast<const V *>(I.z + e) : Vec<R>::zero();
  x.z1 = nz && x.two ? *reinterpret_cast<const V *>(I.z + e + VE) : Vec<R>::zero();
}

template <class R, int NT>
__device__ __forceinline__ void pitem_apply(const Inst<R> &I, const PatchCtx<R, NT> &P, const UCand<R> *uc, int it,
                                            int rowstride, PItem<R> &x) {
  typedef typename Vec<R>::T V;
  constexpr int VE = Vec<R>::N;
  if (!x.m) return;
  V b0 = x.b0, b1 = x.b1;
  unsigned m = x.m;
  bool first = true;
  while (m) {
    const int c = __ffs(m) - 1;
    m &= m - 1;
    const UCand<R> &u = uc[c];
    V av0 = x.a0, av1 = x.a1;
    if (!first) {
      const long long ea = u.aoff + x.rr * rowstride + x.cc * I.KS + 2 * x.q2 * VE;
      av0 = *reinterpret_cast<const V *>(I.A + ea);
      av1 = x.two ? *reinterpret_cast<const V *>(I.A + ea + VE) : Vec<R>::zero();
    }
    first = false;
    const V bold0 = b0, bold1 = b1;
    b0 = Vec<R>::fma_neg(b0, av0, u.delta);
    b1 = Vec<R>::fma_neg(b1, av1, u.delta);
    if (x.rr == u.ch && x.cc == u.cw0) {  // the updated coordinate itself keeps its value
      const int kq = u.k0 / VE, ke = u.k0 % VE;
      if (kq == 2 * x.q2) Vec<R>::set(b0, ke, Vec<R>::get(bold0, ke));
      if (kq == 2 * x.q2 + 1) Vec<R>::set(b1, ke, Vec<R>::get(bold1, ke));
    }
  }
  const long long e = ((long long)x.rr * I.W + x.cc) * I.KS + 2 * x.q2 * VE;
  *reinterpret_cast<V *>(I.beta + e) = b0;
  if (x.two) *reinterpret_cast<V *>(I.beta + e + VE) = b1;
  R best = R(-1);
  int bk = 0;
  const int k0 = 2 * x.q2 * VE;
  const V in0 = *reinterpret_cast<const V *>(P.sh_inv_n + k0);
  const V in1 = x.two ? *reinterpret_cast<const V *>(P.sh_inv_n + k0 + VE) : Vec<R>::zero();
#pragma unroll
  for (int e2 = 0; e2 < 2 * VE; ++e2) {
    const int k = k0 + e2;
    const R bv = e2 < VE ? Vec<R>::get(b0, e2) : Vec<R>::get(b1, e2 - VE);
    const R zv = e2 < VE ? Vec<R>::get(x.z0, e2) : Vec<R>::get(x.z1, e2 - VE);
    const R zn = st_target(bv, I.lambda, e2 < VE ? Vec<R>::get(in0, e2) : Vec<R>::get(in1, e2 - VE), I.positive);
    const R sc = k < I.K ? move_score(zv, zn, I.tol, I.certify) : R(-1);
    if (sc > best) {
      best = sc;
      bk = k;
    }
  }
  P.sh_ps[it] = best;
  P.sh_pk[it] = (uint16_t)bk;
}

template <class R, int NT>
__device__ __forceinline__ void patch_union(const Inst<R> &I, const PatchCtx<R, NT> &P, const UCand<R> *uc, int nc,
                                            int R1, int R2, int C1, int C2) {
  constexpr int LBUF = PatchBuf<R>::N;
  const int tid = threadIdx.x;
  const int W = I.W, G2 = (P.G + 1) / 2;
  const int rowstride = I.U2 * I.KS;
  const int ncol = C2 - C1;
  const int cw = min(min(ncol, LBUF / G2), kMaskCols);
  const int rc = max(1, min(kMaskRows, LBUF / (cw * G2)));
  for (int rr0 = R1; rr0 < R2; rr0 += rc) {
    const int rr1 = min(rr0 + rc, R2);
    for (int cc0 = C1; cc0 < C2; cc0 += cw) {
      const int ccw = min(cw, C2 - cc0);
      const int nrow = rr1 - rr0, npos = nrow * ccw;
      for (int j = tid; j < nrow + ccw; j += NT) {
        unsigned mk = 0;
        if (j < nrow) {
          for (int c = 0; c < nc; ++c)
            if (rr0 + j >= uc[c].r1 && rr0 + j < uc[c].r2) mk |= 1u << c;
          P.rowm[j] = mk;
        } else {
          for (int c = 0; c < nc; ++c)
            if (cc0 + j - nrow >= uc[c].c1 && cc0 + j - nrow < uc[c].c2) mk |= 1u << c;
          P.colm[j - nrow] = mk;
        }
      }
      __syncthreads();
      const int ng = ccw * G2, nit = npos * G2;
      const unsigned mng = rcp_of(ng), mg = rcp_of(G2), rcw = rcp_of(ccw);
#pragma unroll 1
      for (int it = tid; it < nit; it += NT) {
        PItem<R> x;
        pitem_load<R, NT>(I, P, uc, it, nit, rr0, cc0, ng, G2, mng, mg, rowstride, x);
        if (!x.m) P.sh_ps[it] = R(-2);  // no update covers this position: its cache stays
        pitem_apply<R, NT>(I, P, uc, it, rowstride, x);
      }
      __syncthreads();
      for (int t = tid; t < npos; t += NT) {
        const R *pp = P.sh_ps + t * G2;
        if (pp[0] == R(-2)) continue;
        const int tr = div_rcp(t, ccw, rcw);
        const int pos = (rr0 + tr) * W + cc0 + (t - tr * ccw);
        const uint16_t *pk = P.sh_pk + t * G2;
        R best = pp[0];
        int bk = pk[0];
        for (int g = 1; g < G2; ++g)
          if (pp[g] > best) {
            best = pp[g];
            bk = pk[g];
          }
        score_st(I.score + pos, best);
        reinterpret_cast<uint16_t *>(I.meta + pos)[0] = (uint16_t)bk;  // the atom half of meta
      }
      __syncthreads();
    }
  }
}

// One workgroup is one worker of Alg. 3 (DiCoDiLe-Z).  Worker w of an instance
// owns S_w, a block of a W1 x W2 balanced split of the valid domain, cut into
// Mw balanced sub-domains of about tile1 x tile2 positions that it visits
// cyclically.
//
// Neighbours read the scores of S_w's border band (positions within L_i - 1
// of a side shared with a neighbour) in their soft-lock tests.  A round runs:
//   A  visit `inner` sub-domains (Alg. 1's local greedy choice).  Candidates
//      whose patch stays clear of the band concern no other worker
//      (eq. soft_lock only applies near the border): they are applied at once.
//      The first band-reaching candidate is held; it is tested against the
//      other workers' scores in V(w0) when V(w0) leaves S_w (eq. soft_lock,
//      lower worker index wins a tie) and published, tagged with the round;
//   B  every worker applies, to the part of beta, z and the cache it owns, the
//      accepted published candidates of itself and of its grid neighbours
//      whose neighbourhood meets S_w (eq. beta_update), in increasing worker
//      order, then publishes progress r + 1.
// Phase A of round r reads the band of S_w's neighbours, which only they
// write, in their phase B: it starts once each neighbour's progress is >= r.
// A neighbour starts its phase B of round r only after reading this worker's
// round-r candidate, published after this worker's phase A reads.  Worker
// sizes of at least L_i keep every interaction between grid neighbours.
//
// Stopping: a worker is quiet once its last Mw visits found no move scoring
// >= tol and no patch touched S_w since (random rule: once the scan at the
// end of its last epoch found none and no patch touched S_w since).  When
// every worker reports quiet at the end of the same round, every
// coordinate's move is below tol and no further update can happen: all
// workers exit.
//
// Under the random rule a candidate's score is that of its drawn coordinate,
// at most the cached best of its position, so of two interacting candidates
// the soft-lock test still rejects at least one: each sees the other's
// position holding a score >= its own (ties go to the lower worker index).
template <class R, int NT> struct RoundSmem {
  static constexpr int LBUF = PatchBuf<R>::N;
  R ps[LBUF];
  uint16_t pk[LBUF];
  uint32_t nzb[kNzWords];
  uint32_t rowm[kMaskRows], colm[kMaskCols];
  R inv_n[1024];
  R rs[NT / 64];
  int ri[NT / 64];
  int exit_f, cok;
  int wok[9];  // per-neighbour result of the progress wait
  int ck0;       // the held candidate's atom, current value and target
  R czc, czn;
  uint32_t cmeta;  // ... and its position's meta word (LGCD rules)
  UCand<R> ui;  // an interior candidate applied within phase A
  int nbr[9];
  UCand<R> uc[9];
  int nuc, ub[4];  // updates touching S_w and the bounding box of their patches
  int ub_union;    // 1: apply them in one pass over the bounding box
};

// Runs worker w of instance I until its instance converges or stops.  Every
// thread of the workgroup calls it.
template <class R, int NT>
__device__ void run_worker(const Inst<R> &I, const int w, const long long timeout_ticks, RoundSmem<R, NT> &sm) {
  constexpr int VE = Vec<R>::N;
  R *const sh_inv_n = sm.inv_n;
  R *const sh_rs = sm.rs;
  int *const sh_ri = sm.ri;
  int &sh_exit = sm.exit_f;
  int &sh_cok = sm.cok;
  int *const sh_nbr = sm.nbr;
  const int tid = threadIdx.x;
  const int nW = I.W1 * I.W2;
  const int wi = w / I.W2, wj = w - wi * I.W2;
  const int K = I.K, H = I.H, W = I.W;
  const int a1 = part_start(wi, H, I.W1), b1 = part_start(wi + 1, H, I.W1);
  const int a2 = part_start(wj, W, I.W2), b2 = part_start(wj + 1, W, I.W2);
  // sub-domains: about extent / tile per axis, balanced (sizes differ by <= 1)
  const int ext1 = b1 - a1, ext2 = b2 - a2;
  const int nb1 = max(1, (ext1 + I.tile1 / 2) / I.tile1), nb2 = max(1, (ext2 + I.tile2 / 2) / I.tile2);
  const int Mw = nb1 * nb2;
  // random rule: one drawn coordinate per round; a scan of S_w every npw
  // draws (an epoch) decides whether the worker is quiet
  const bool rnd = I.strategy == 3;
  const int npw = ext1 * ext2;
  const int inner = rnd ? 1 : (I.inner > 0 ? min(I.inner, Mw) : 1);
  const int qthr = rnd ? 1 : Mw;  // quiet count of a worker with no pending move
  // candidates at w0 in [in_lo, in_hi[ patch nothing of the band neighbours read
  const int in_lo1 = wi > 0 ? a1 + 2 * (I.L1 - 1) : a1, in_hi1 = wi < I.W1 - 1 ? b1 - 2 * (I.L1 - 1) : b1;
  const int in_lo2 = wj > 0 ? a2 + 2 * (I.L2 - 1) : a2, in_hi2 = wj < I.W2 - 1 ? b2 - 2 * (I.L2 - 1) : b2;

  PatchCtx<R, NT> P;
  P.sh_ps = sm.ps;
  P.sh_pk = sm.pk;
  P.sh_inv_n = sh_inv_n;
  P.rowm = sm.rowm;
  P.colm = sm.colm;
  P.G = I.KS / VE;
  P.a1 = a1;
  P.a2 = a2;
  P.ext2 = ext2;
  P.nzb = npw <= 32 * kNzWords ? sm.nzb : nullptr;
  if (P.nzb)
    for (int wd = tid; wd < (npw + 31) / 32; wd += NT) {
      uint32_t m = 0;
      for (int b = 0; b < 32; ++b) {
        const int t = wd * 32 + b;
        if (t < npw && meta_nzc(I.meta[(a1 + t / ext2) * W + a2 + t % ext2])) m |= 1u << b;
      }
      sm.nzb[wd] = m;
    }

  __syncthreads();
  for (int k = tid; k < I.KS; k += NT) sh_inv_n[k] = k < K ? I.inv_n[k] : R(0);
  if (tid == 0) {
    int nn = 0;
    for (int di = -1; di <= 1; ++di)
      for (int dj = -1; dj <= 1; ++dj) {
        const int ni = wi + di, nj = wj + dj;
        if (ni >= 0 && ni < I.W1 && nj >= 0 && nj < I.W2) sh_nbr[nn++] = ni * I.W2 + nj;
      }
    for (int q = nn; q < 9; ++q) sh_nbr[q] = -1;
  }
  __syncthreads();
  int nn = 0;
#pragma unroll
  for (int q = 0; q < 9; ++q) nn += sh_nbr[q] >= 0;

  unsigned long long my_upd = 0, my_cand = 0, my_lock = 0, my_visit = 0, my_chk = 0, my_patch = 0;
  unsigned long long tk_wait = 0, tk_sel = 0, tk_col = 0, tk_app = 0, tk_mark = 0;
  long long cursor = I.wstate ? I.wstate[2 * w] : 0;         // visits so far
  int quiet = I.wstate ? (int)I.wstate[2 * w + 1] : 0;  // consecutive visits with no move >= tol and no patch of S_w
  const unsigned long long t_launch = __builtin_amdgcn_s_memrealtime();
  int r = 0;
  int exit_status = 0;
  int next_exit = 0;  // thread 0: exit flags read at the end of the previous round
  for (;; ++r) {
    // ---- exit conditions
    if (tid == 0) {
      int f = r == 0 ? (ld_shared_i32(&I.ctl->converged) | ld_shared_i32(&I.ctl->stop)) : next_exit;
      // every worker runs exactly max_rounds rounds: all moves of the last
      // round are then applied everywhere and the launch can be resumed
      if (!f && I.max_rounds > 0 && r >= I.max_rounds) {
        atomicCAS(&I.ctl->status, 0, 1);
        f = 1;
      }
      if (!f && (long long)(__builtin_amdgcn_s_memrealtime() - t_launch) > I.budget_ticks) {
        st_shared_i32(&I.ctl->stop, 1);
        atomicCAS(&I.ctl->status, 0, 4);
        f = 1;
      }
      sh_exit = f;
      sh_cok = 1;
      tk_mark = __builtin_amdgcn_s_memrealtime();
    }
    __syncthreads();
    if (sh_exit) break;

    // ---- phase A: `inner` visits.  Interior candidates are applied at once;
    // the first band-reaching candidate is held for the protocol, and later
    // interior candidates are applied only if neither lies in the other's
    // V (they cannot interact); other candidates wait for the next cycle.
    R bs = R(-1);
    int bp = 0x7fffffff, bk = 0;
    bool has = false;
    int hh0 = 0, hw0 = 0;
    long long restart = -1;  // first visit whose candidate had to wait: next round starts there
    for (int v = 0; v < inner; ++v) {
      const long long visit = cursor;
      const int m = (int)(cursor % Mw);
      ++cursor;
      ++my_visit;
      if (rnd) {
        const unsigned long long u = sm64_draw(I.seed, (unsigned long long)w, (unsigned long long)visit);
        const unsigned long long j = u % ((unsigned long long)npw * (unsigned long long)K);
        const unsigned long long jp = j / (unsigned long long)K;
        const int k = (int)(j - jp * (unsigned long long)K);
        const int hh = a1 + (int)jp / ext2, ww = a2 + (int)jp % ext2;
        const int pos = hh * W + ww;
        if (tid == 0) {
          const long long i0 = (long long)pos * I.KS + k;
          const R zc = I.z[i0];
          const R zn = st_target(I.beta[i0], I.lambda, sh_inv_n[k], I.positive);
          sm.ck0 = k;
          sm.czc = zc;
          sm.czn = zn;
          sh_rs[0] = move_score(zc, zn, I.tol, I.certify);
        }
        __syncthreads();
        const R sc = sh_rs[0];
        __syncthreads();
        if (!(sc >= I.tol && sc > R(0))) continue;
        quiet = 0;
        ++my_cand;
        has = true;
        bs = sc;
        bp = pos;
        bk = k;
        hh0 = hh;
        hw0 = ww;
        continue;
      }
      const int bi = m / nb2, bj = m - (m / nb2) * nb2;
      const int s1 = a1 + part_start(bi, ext1, nb1), e1 = a1 + part_start(bi + 1, ext1, nb1);
      const int s2 = a2 + part_start(bj, ext2, nb2), e2 = a2 + part_start(bj + 1, ext2, nb2);
      const int bw = e2 - s2, np = (e1 - s1) * bw;
      R vs = R(-1);
      int vp = 0x7fffffff;
      {
        // four positions per pass with their loads in flight together; the
        // (row, column) of position t steps by NT each time
        const int dh = NT / bw, dw = NT - dh * bw;
        int th = tid / bw, tw = tid - th * bw;
        for (int t = tid; t < np; t += 4 * NT) {
          R sc[4];
          int ps[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            ps[u] = (s1 + th) * W + s2 + tw;
            sc[u] = t + u * NT < np ? score_ld(I.score + ps[u]) : R(-1);
            tw += dw;
            th += dh;
            if (tw >= bw) {
              tw -= bw;
              ++th;
            }
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (sc[u] > vs || (sc[u] == vs && ps[u] < vp)) {
              vs = sc[u];
              vp = ps[u];
            }
        }
      }
      // with one visit per round each thread whose own best could be the
      // candidate (a position of the sub-domain scoring >= tol) fetches its
      // meta word while the block reduces, so the winning thread reads the
      // candidate's z and beta one dependent load earlier
      const int lp = vp;
      const bool lok = inner == 1 && vs >= I.tol && vs > R(0);
      const uint32_t lmeta = lok ? I.meta[lp] : 0u;
      block_argmax<R, NT>(vs, vp, sh_rs, sh_ri);
      if (!(vs >= I.tol && vs > R(0))) {
        ++quiet;
        continue;
      }
      quiet = 0;
      ++my_cand;
      const int h0 = vp / W, w0 = vp - (vp / W) * W;
      // with one visit per round every candidate takes the published path, so
      // its patch runs in phase B beside the neighbours' ones
      const bool interior = inner > 1 && h0 >= in_lo1 && h0 < in_hi1 && w0 >= in_lo2 && w0 < in_hi2;
      if (!interior) {
        if (!has) {
          has = true;
          bs = vs;
          bp = vp;
          hh0 = h0;
          hw0 = w0;
          if (lok && lp == vp) {
            const int k0 = meta_argk(lmeta);
            const long long i0 = (long long)vp * I.KS + k0;
            sm.ck0 = k0;
            sm.cmeta = lmeta;
            sm.czc = I.z[i0];
            sm.czn = st_target(I.beta[i0], I.lambda, sh_inv_n[k0], I.positive);
          }
        } else if (restart < 0) {
          restart = visit;  // a second band-reaching candidate waits for the next round
        }
        continue;
      }
      if (has && abs(h0 - hh0) < I.L1 && abs(w0 - hw0) < I.L2) {  // would interact with the held one
        if (restart < 0) restart = visit;
        continue;
      }
      if (tid == 0) {
        const int k0 = meta_argk(I.meta[vp]);
        const long long i0 = (long long)vp * I.KS + k0;
        const R zc = I.z[i0];
        const R zn = st_target(I.beta[i0], I.lambda, sh_inv_n[k0], I.positive);
        I.z[i0] = zn;
        const uint32_t mt = I.meta[vp];
        const int nzc = meta_nzc(mt) + (zn != R(0)) - (zc != R(0));
        I.meta[vp] = meta_pack(meta_argk(mt), nzc);
        if (P.nzb) nzb_put(P.nzb, (h0 - a1) * ext2 + (w0 - a2), nzc != 0);
        UCand<R> &u = sm.ui;
        u.k0 = k0;
        u.ch = h0;
        u.cw0 = w0;
        u.r1 = max(h0 - I.L1 + 1, a1);
        u.r2 = min(h0 + I.L1, b1);
        u.c1 = max(w0 - I.L2 + 1, a2);
        u.c2 = min(w0 + I.L2, b2);
        u.aoff = ((k0 * I.U1 - h0 + I.L1 - 1) * I.U2 - w0 + I.L2 - 1) * I.KS;
        u.delta = zn - zc;
        if (I.div_guard > R(0) && (zn > I.div_guard || -zn > I.div_guard)) {
          st_shared_i32(&I.ctl->stop, 1);
          atomicCAS(&I.ctl->status, 0, 2);
        }
        wait_vm();
      }
      __syncthreads();
      ++my_upd;
      my_patch += (unsigned long long)(sm.ui.r2 - sm.ui.r1) * (sm.ui.c2 - sm.ui.c1);
      patch_union<R, NT>(I, P, &sm.ui, 1, sm.ui.r1, sm.ui.r2, sm.ui.c1, sm.ui.c2);
    }
    if (restart >= 0) cursor = restart;
    int h0 = 0, w0 = 0;
    if (has) {
      h0 = bp / W;
      w0 = bp - h0 * W;
    }
    // The visits above read only S_w, which this worker alone writes and
    // finished patching in its last phase B; so do the candidate's reads
    // (in the visit with one visit per round, below with several).  Only the soft-lock test (the neighbours' scores of round r - 1)
    // and the reuse of the candidate slot (read by the neighbours in round
    // r - 1) need the neighbours' progress.
    if (tid == 0) {
      if (has && inner != 1) {
        const uint32_t mt = I.meta[bp];
        const int k0 = meta_argk(mt);
        const long long i0 = (long long)bp * I.KS + k0;
        sm.ck0 = k0;
        sm.cmeta = mt;
        sm.czc = I.z[i0];
        sm.czn = st_target(I.beta[i0], I.lambda, sh_inv_n[k0], I.positive);
      }
      const unsigned long long t = __builtin_amdgcn_s_memrealtime();
      tk_sel += t - tk_mark;
      tk_mark = t;
    }
    if (!wait_progress(I.prog, sh_nbr, nn, w, r, timeout_ticks, sm.wok)) {
      exit_status = 3;
      break;
    }
    if (tid == 0) {
      const unsigned long long t = __builtin_amdgcn_s_memrealtime();
      tk_wait += t - tk_mark;
      tk_mark = t;
    }
    int locked = 0;
    if (has && I.soft_lock &&
        (h0 - I.L1 + 1 < a1 || h0 + I.L1 > b1 || w0 - I.L2 + 1 < a2 || w0 + I.L2 > b2)) {
      // soft-lock test over V(w0), inside the valid domain, outside S_w
      const int v1 = max(h0 - I.L1 + 1, 0), u1 = min(h0 + I.L1, H);
      const int v2 = max(w0 - I.L2 + 1, 0), u2 = min(w0 + I.L2, W);
      const int vw = u2 - v2, nv = (u1 - v1) * vw;
      my_chk += nv;
      int lk = 0;
      {
        const int dh = NT / vw, dw = NT - dh * vw;
        int th = tid / vw, tw = tid - th * vw;
        for (int t = tid; t < nv; t += 4 * NT) {
          R sc[4];
          int hq[4], wq[4];
          bool use[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            hq[u] = v1 + th;
            wq[u] = v2 + tw;
            use[u] = t + u * NT < nv && !(hq[u] >= a1 && hq[u] < b1 && wq[u] >= a2 && wq[u] < b2);
            sc[u] = use[u] ? score_ld(I.score + hq[u] * W + wq[u]) : R(-1);
            tw += dw;
            th += dh;
            if (tw >= vw) {
              tw -= vw;
              ++th;
            }
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            if (!use[u]) continue;
            if (sc[u] > bs) {
              lk = 1;
            } else if (sc[u] == bs) {
              const int owner = part_owner(hq[u], H, I.W1) * I.W2 + part_owner(wq[u], W, I.W2);
              if (owner < w) lk = 1;
            }
          }
        }
      }
      locked = block_or<NT>(lk, sh_ri);
    }
    // the band reads above are complete before the candidate becomes visible
    wait_vm();
    __syncthreads();
    if (tid == 0) {
      unsigned long long tag = cand_tag(r, 0, kNoPos);
      unsigned long long dbits = 0;
      if (has) {
        if (locked) {
          ++my_lock;
        } else {
          const int k0 = sm.ck0;
          const long long i0 = (long long)bp * I.KS + k0;
          const R zc = sm.czc;
          const R zn = sm.czn;
          // z and its non-zero count change now; beta and the cache in phase B
          I.z[i0] = zn;
          // the meta word read with the candidate: nothing writes it since
          const uint32_t mt = rnd ? I.meta[bp] : sm.cmeta;
          const int nzc = meta_nzc(mt) + (zn != R(0)) - (zc != R(0));
          I.meta[bp] = meta_pack(meta_argk(mt), nzc);
          if (P.nzb) nzb_put(P.nzb, (h0 - a1) * ext2 + (w0 - a2), nzc != 0);
          dbits = delta_bits<R>(zn - zc);
          tag = cand_tag(r, k0, (unsigned)bp);
          ++my_upd;
          if (I.div_guard > R(0) && (zn > I.div_guard || -zn > I.div_guard)) {
            st_shared_i32(&I.ctl->stop, 1);
            atomicCAS(&I.ctl->status, 0, 2);
          }
        }
      }
      if (I.audit && r < I.audit_rounds)
        I.audit[(long long)r * nW + w] = audit_record(has, has && !locked, sm.ck0, bp);
      st_shared_u64(I.cand + 2 * w + 1, dbits);
      wait_vm();
      st_shared_u64(I.cand + 2 * w, tag);
      const unsigned long long t = __builtin_amdgcn_s_memrealtime();
      tk_sel += t - tk_mark;
      tk_mark = t;
    }

    // ---- collect this round's candidates of the 3x3 neighbourhood; lane q
    // also clips neighbour q's update to S_w for phase B
    bool uval = false;
    int uk0 = 0, uch = 0, ucw = 0, ur1 = 0, ur2 = 0, uc1 = 0, uc2 = 0;
    R udl = R(0);
    if (tid < nn) {
      const int n = sh_nbr[tid];
      unsigned long long t = 0;
      int ok = 1;
      const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
      const int rtag = r & ((1 << kRoundBits) - 1);
      for (;;) {
        // the tag and the progress word are read together, one round trip
        // per poll
        t = ld_shared_u64(I.cand + 2 * n);
        const int pg = ld_shared_i32(I.prog + n);
        if (tag_round(t) == rtag) break;
        if (pg == 0x7fffffff) {
          // the neighbour has left; it stored its last tag before its
          // progress word, so a tag of this round is seen by a reread
          t = ld_shared_u64(I.cand + 2 * n);
          if (tag_round(t) != rtag) t = cand_tag(r, 0, kNoPos);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
        if ((long long)(__builtin_amdgcn_s_memrealtime() - t0) > timeout_ticks) {
          ok = 0;
          t = cand_tag(r, 0, kNoPos);
          break;
        }
      }
      const unsigned cpos = tag_pos(t);
      if (cpos != kNoPos) {
        udl = bits_delta<R>(ld_shared_u64(I.cand + 2 * n + 1));
        uk0 = tag_k0(t);
        uch = (int)(cpos / (unsigned)W);
        ucw = (int)(cpos - (unsigned)uch * (unsigned)W);
        ur1 = max(uch - I.L1 + 1, a1);
        ur2 = min(uch + I.L1, b1);
        uc1 = max(ucw - I.L2 + 1, a2);
        uc2 = min(ucw + I.L2, b2);
        uval = ur1 < ur2 && uc1 < uc2;
      }
      if (!ok) sh_cok = 0;
    }
    if (tid < 64) {
      // the touching updates in neighbour order, their bounding box and the
      // patched area, over the first wave's lanes
      const unsigned long long bal = __ballot(uval);
      if (uval) {
        UCand<R> &u = sm.uc[__popcll(bal & ((1ull << tid) - 1ull))];
        u.k0 = uk0;
        u.ch = uch;
        u.cw0 = ucw;
        u.r1 = ur1;
        u.r2 = ur2;
        u.c1 = uc1;
        u.c2 = uc2;
        u.aoff = ((uk0 * I.U1 - uch + I.L1 - 1) * I.U2 - ucw + I.L2 - 1) * I.KS;
        u.delta = udl;
      }
      int x1 = uval ? ur1 : b1, x2 = uval ? ur2 : a1, y1 = uval ? uc1 : b2, y2 = uval ? uc2 : a2;
      unsigned pa = uval ? (unsigned)((ur2 - ur1) * (uc2 - uc1)) : 0u;
#pragma unroll
      for (int off = 8; off > 0; off >>= 1) {
        x1 = min(x1, __shfl_xor(x1, off, 16));
        x2 = max(x2, __shfl_xor(x2, off, 16));
        y1 = min(y1, __shfl_xor(y1, off, 16));
        y2 = max(y2, __shfl_xor(y2, off, 16));
        pa += __shfl_xor(pa, off, 16);
      }
      if (tid == 0) {
        const int nu = __popcll(bal);
        sm.nuc = nu;
        sm.ub[0] = x1;
        sm.ub[1] = x2;
        sm.ub[2] = y1;
        sm.ub[3] = y2;
        my_patch += pa;
        // One pass over the bounding box pays for small patches, whose cost is
        // mostly per-update latency (positions no update covers cost no loads).
        // Large patches (over 1024 positions) are bandwidth-bound and go one by
        // one: measured on 32x32 atoms (3969-position patches) the single pass
        // costs 15-20% of the rounds' time.
        sm.ub_union = nu > 1 && (long long)I.U1 * I.U2 <= 1024;
      }
    }
    __syncthreads();
    if (!sh_cok) {
      exit_status = 3;
      break;
    }
    if (tid == 0) {
      const unsigned long long t = __builtin_amdgcn_s_memrealtime();
      tk_col += t - tk_mark;
      tk_mark = t;
    }

    // ---- phase B: apply the accepted candidates that touch S_w (eq. beta_update),
    // all in one pass over the bounding box of their patches
    if (sm.nuc > 0) {
      quiet = 0;
      if (sm.ub_union || sm.nuc == 1) {
        patch_union<R, NT>(I, P, sm.uc, sm.nuc, sm.ub[0], sm.ub[1], sm.ub[2], sm.ub[3]);
      } else {
        for (int c = 0; c < sm.nuc; ++c)
          patch_union<R, NT>(I, P, sm.uc + c, 1, sm.uc[c].r1, sm.uc[c].r2, sm.uc[c].c1, sm.uc[c].c2);
      }
    }
    // cache stores complete before the progress counter moves
    wait_vm();
    __syncthreads();
    if (rnd && cursor % npw == 0) {
      // end of an epoch: the worker is quiet if no position of S_w holds a
      // move scoring >= tol (every later patch of S_w clears it again)
      R mx = R(-1);
      int mp = 0;
      for (int t = tid; t < npw; t += NT) {
        const R sc = score_ld(I.score + (a1 + t / ext2) * W + a2 + t % ext2);
        if (sc > mx) mx = sc;
      }
      block_argmax<R, NT>(mx, mp, sh_rs, sh_ri);
      quiet = (mx >= I.tol && mx > R(0)) ? 0 : 1;
    }
    if (tid == 0) {
      st_shared_i32(I.prog + w, r + 1);
      tk_app += __builtin_amdgcn_s_memrealtime() - tk_mark;
      // ---- stopping consensus of round r: one 64-bit counter per ring slot,
      // completions in the low word and quiet workers in the high word.  The
      // exit flags for the next round are read while the add is in flight; a
      // flag raised later in this round is seen one round later, which only
      // costs an empty round.
      const int slot = r % kRing;
      unsigned long long *ring = reinterpret_cast<unsigned long long *>(I.ring);
      const unsigned long long q = quiet >= qthr ? 1ull : 0ull;
      const unsigned long long old =
          __hip_atomic_fetch_add(&ring[slot], 1ull + (q << 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      int f = ld_shared_i32(&I.ctl->converged) | ld_shared_i32(&I.ctl->stop);
      if ((old & 0xffffffffull) == (unsigned long long)(nW - 1)) {
        st_shared_u64(&ring[slot], 0ull);
        if ((old >> 32) + q == (unsigned long long)nW) {
          st_shared_i32(&I.ctl->converged, 1);
          f = 1;
        }
      }
      next_exit = f;
    }
  }
  // ---- leave: neighbours must never wait on a finished worker
  wait_vm();
  __syncthreads();
  if (tid == 0) {
    if (exit_status) {
      st_shared_i32(&I.ctl->stop, 1);
      atomicCAS(&I.ctl->status, 0, exit_status);
    }
    atomicAdd(&I.ctl->n_updates, my_upd);
    atomicAdd(&I.ctl->n_candidates, my_cand);
    atomicAdd(&I.ctl->n_softlocked, my_lock);
    atomicAdd(&I.ctl->n_visits, my_visit);
    atomicAdd(&I.ctl->n_checked, my_chk);
    atomicAdd(&I.ctl->n_patched, my_patch);
    atomicAdd(&I.ctl->tk_wait, tk_wait);
    atomicAdd(&I.ctl->tk_select, tk_sel);
    atomicAdd(&I.ctl->tk_collect, tk_col);
    atomicAdd(&I.ctl->tk_apply, tk_app);
    atomicMax(&I.ctl->max_round, r);
    atomicMax(&I.ctl->sweeps_done, (int)(cursor / (rnd ? npw : Mw)));
    if (I.wstate) {
      I.wstate[2 * w] = cursor;
      I.wstate[2 * w + 1] = quiet;
    }
    st_shared_i32(I.prog + w, 0x7fffffff);
  }
}

// Four 256-thread FP32 workers per CU (at most 128 VGPRs): the co-resident
// worker count sets how finely an image can be split.
template <class R, int NT> struct RoundWaves {
  static constexpr int value = sizeof(R) == 4 ? (NT <= 256 ? NT / 64 : 4) : 1;
};

template <class R, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(RoundWaves<R, NT>::value))) void lgcd_rounds(const Inst<R> *__restrict__ insts,
                                                   const int *__restrict__ wg_inst,
                                                   long long timeout_ticks) {
  __shared__ RoundSmem<R, NT> sm;
  const int ii = wg_inst[blockIdx.x];
  const Inst<R> I = insts[ii];
  run_worker<R, NT>(I, blockIdx.x - I.wg_base, timeout_ticks, sm);
}

}  // namespace dcdl
