// capi.hip -- host runtime and C ABI of the DiCoDiLe CSC library for gfx950.
// The declarations, argument meanings, layouts and error behaviour are in
// include/dicodile.h.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <thread>
#include <vector>

#include "../../include/dicodile.h"
#include "dcdl_device.h"
#include "dcdl_kernels.h"
#include "dcdl_mfma.h"
#include "dcdl_dict.h"
#include "dcdl_check.h"
#include "dcdl_fft.h"

using namespace dcdl;

// Fixed device scratch of dicodile_csc_noalloc: every workspace of that call
// is carved from it, so the call allocates nothing.  Each device holds its
// own copy for the life of the process; host code reaches it only through
// the address hipGetSymbolAddress returns for the device (DeviceState).
constexpr size_t kScratchBytes = (size_t)DCDL_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCK(expr)                                                                     \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return fail(DCDL_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// ------------------------------------------------------------- workspace
struct Buf {
  void *p = nullptr;
  size_t n = 0;
};

// Workspaces of one no-allocation call: named slots carved in order from the
// device's scratch array (a name asked for again gets its slot back).
struct ScratchArena {
  unsigned char *base = nullptr;
  size_t cap = 0, off = 0;
  std::map<std::string, std::pair<size_t, size_t>> slots;  // name -> (offset, bytes)
};

constexpr int kCallEvents = 7;

struct DeviceState {
  std::mutex mu;
  std::map<std::string, Buf> bufs;
  hipStream_t aux = nullptr;  // library-owned stream (default priority) for captured work
  int cus = 0;
  bool checked = false;
  bool is_gfx950 = false;
  // no-allocation calls: this device's address of `scratch` and the events
  // its calls time with, both obtained once at the first such call
  unsigned char *scratch_ptr = nullptr;
  hipEvent_t na_ev[kCallEvents] = {};
  ScratchArena *arena = nullptr;  // set for the duration of a no-allocation call
};

std::mutex g_devices_mu;
std::map<int, DeviceState *> g_devices;

DeviceState *device_state(int *dev_out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(g_devices_mu);
  DeviceState *&s = g_devices[dev];
  if (!s) s = new DeviceState();
  if (dev_out) *dev_out = dev;
  return s;
}

// Returns a device buffer of at least `bytes` bytes, reusing or growing the
// named slot.  Synchronises `stream` before freeing an old allocation.
int ws_get(DeviceState *ds, hipStream_t stream, const char *name, size_t bytes, void **out) {
  if (bytes == 0) bytes = 256;
  if (ds->arena) {
    ScratchArena &a = *ds->arena;
    auto it = a.slots.find(name);
    if (it != a.slots.end() && it->second.second >= bytes) {
      *out = a.base + it->second.first;
      return DCDL_OK;
    }
    const size_t nb = (bytes + 255) / 256 * 256;
    if (a.off + nb > a.cap)
      return fail(DCDL_EINVAL, "workspace '%s' (%zu bytes) does not fit the %zu-byte fixed scratch of "
                  "dicodile_csc_noalloc (%zu bytes used)", name, bytes, a.cap, a.off);
    a.slots[name] = {a.off, nb};
    *out = a.base + a.off;
    a.off += nb;
    return DCDL_OK;
  }
  Buf &b = ds->bufs[name];
  if (b.n < bytes) {
    if (b.p) {
      HIPCK(hipStreamSynchronize(stream));
      HIPCK(hipFree(b.p));
      b.p = nullptr;
      b.n = 0;
    }
    size_t nb = bytes + bytes / 8;
    if (hipMalloc(&b.p, nb) != hipSuccess) {
      (void)hipGetLastError();
      b.p = nullptr;
      return fail(DCDL_ENOMEM, "workspace '%s': cannot allocate %zu bytes", name, nb);
    }
    b.n = nb;
  }
  *out = b.p;
  return DCDL_OK;
}

#define WS(name, bytes, ptr)                                                              \
  do {                                                                                    \
    void *p_ = nullptr;                                                                   \
    int rc_ = ws_get(ds, stream, name, (size_t)(bytes), &p_);                             \
    if (rc_ != DCDL_OK) return rc_;                                                       \
    ptr = reinterpret_cast<decltype(ptr)>(p_);                                            \
  } while (0)

int check_device(DeviceState *ds) {
  if (!ds->checked) {
    int dev = 0;
    HIPCK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIPCK(hipGetDeviceProperties(&prop, dev));
    ds->is_gfx950 = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0;
    ds->cus = prop.multiProcessorCount;
    ds->checked = true;
  }
  if (!ds->is_gfx950) return fail(DCDL_ENODEV, "the current device is not gfx950 (MI355X)");
  return DCDL_OK;
}

// ------------------------------------------------------------- geometry
int make_geom(const dcdl_shape *s, Geom *g) {
  if (!s) return fail(DCDL_EINVAL, "shape is NULL");
  if (s->ndim != 1 && s->ndim != 2) return fail(DCDL_EINVAL, "ndim must be 1 or 2 (got %d)", s->ndim);
  if (s->P < 1 || s->K < 1 || s->K > 1024) return fail(DCDL_EINVAL, "need P >= 1 and 1 <= K <= 1024");
  long long T1, T2;
  int L1, L2;
  if (s->ndim == 1) {
    T1 = 1;
    L1 = 1;
    T2 = s->T[0];
    L2 = s->L[0];
  } else {
    T1 = s->T[0];
    T2 = s->T[1];
    L1 = s->L[0];
    L2 = s->L[1];
  }
  if (L1 < 1 || L2 < 1 || T1 < L1 || T2 < L2) return fail(DCDL_EINVAL, "need 1 <= L_i <= T_i");
  if (T1 * T2 > (1ll << 31) - 1 || (T1 - L1 + 1) * (T2 - L2 + 1) * (long long)s->K > (1ll << 40))
    return fail(DCDL_EINVAL, "problem too large for 32-bit position indices");
  {
    // the round kernel addresses the apply table A[k0][d1][d2][k] and a
    // patch's rows (row * (2 L2 - 1) * KS) with 32-bit offsets; KS is at most
    // K rounded up to four
    const long long ks = (s->K + 3) / 4 * 4, u1 = 2ll * L1 - 1, u2 = 2ll * L2 - 1;
    if ((long long)s->K * u1 * u2 * ks + (T1 + u1) * u2 * ks + (T2 + u2) * ks >= (1ll << 31))
      return fail(DCDL_EINVAL, "K * (2 L1 - 1) * (2 L2 - 1) * K = %lld apply-table entries exceed 32-bit offsets",
                  (long long)s->K * u1 * u2 * ks);
  }
  g->P = s->P;
  g->K = s->K;
  g->L1 = L1;
  g->L2 = L2;
  g->U1 = 2 * L1 - 1;
  g->U2 = 2 * L2 - 1;
  g->T1 = (int)T1;
  g->T2 = (int)T2;
  g->H = (int)(T1 - L1 + 1);
  g->W = (int)(T2 - L2 + 1);
  g->KS = s->K;
  return DCDL_OK;
}

inline unsigned blocks_for(long long n, int nt) { return (unsigned)((n + nt - 1) / nt); }
inline unsigned grid_stride_blocks(long long n) {
  long long b = (n + 255) / 256;
  return (unsigned)(b < 8192 ? (b < 1 ? 1 : b) : 8192);
}

// The events one call times its launches with: created for the call, or
// borrowed from the device's set when the call may not allocate.
struct CallEvents {
  hipEvent_t e[kCallEvents] = {};
  bool owned = false;
  int init(const DeviceState *ds) {
    if (ds->arena) {
      for (int i = 0; i < kCallEvents; ++i) e[i] = ds->na_ev[i];
      return DCDL_OK;
    }
    owned = true;
    for (int i = 0; i < kCallEvents; ++i) HIPCK(hipEventCreate(&e[i]));
    return DCDL_OK;
  }
  ~CallEvents() {
    if (owned)
      for (int i = 0; i < kCallEvents; ++i)
        if (e[i]) (void)hipEventDestroy(e[i]);
  }
};

// Two events bracketing launches on one stream; the elapsed times are summed
// when the end event has completed.
struct CorrTimer {
  hipEvent_t e[2] = {nullptr, nullptr};
  double s = 0.0;
  int n = 0;
  CorrTimer(hipEvent_t a, hipEvent_t b) {
    e[0] = a;
    e[1] = b;
  }
  int begin(hipStream_t st) {
    HIPCK(hipEventRecord(e[0], st));
    return DCDL_OK;
  }
  int end(hipStream_t st) {
    HIPCK(hipEventRecord(e[1], st));
    HIPCK(hipEventSynchronize(e[1]));
    float ms = 0.f;
    HIPCK(hipEventElapsedTime(&ms, e[0], e[1]));
    s += ms * 1e-3;
    ++n;
    return DCDL_OK;
  }
};

// ------------------------------------------------------------- kernels
// DtD by the direct FP64 loops (atoms whose staged windows do not fit the
// matrix-core path).
template <class R>
int run_dtd_loops(hipStream_t stream, const Geom &g, const R *D, R *dtd, R *A, R *inv_n) {
  const size_t lds = 2 * sizeof(R) * (size_t)g.P * g.L1 * g.L2;
  if (lds > 160 * 1024) return fail(DCDL_EINVAL, "atoms of %d values exceed the LDS budget", g.P * g.L1 * g.L2);
  hipLaunchKernelGGL(dtd_kernel<R>, dim3(g.K * g.K), dim3(256), lds, stream, g, D, dtd, A, inv_n);
  HIPCK(hipGetLastError());
  return DCDL_OK;
}

template <class Rin, class Racc, class Rz, int MODE>
int run_corr(hipStream_t stream, const Geom &g, const Rin *X, const Rin *D, const CorrOut &o) {
  constexpr int KC = sizeof(Racc) == 8 ? 8 : 16;
  const size_t lds = sizeof(Racc) * (size_t)g.L2 * KC;
  if (g.H == 1)
    hipLaunchKernelGGL((corr_kernel<Rin, Racc, Rz, MODE, KC, 1>), dim3(blocks_for(g.W, 256)), dim3(256), lds, stream,
                       g, X, D, o);
  else
    hipLaunchKernelGGL((corr_kernel<Rin, Racc, Rz, MODE, KC, 8>), dim3(blocks_for(g.W, 32), blocks_for(g.H, 8)),
                       dim3(256), lds, stream, g, X, D, o);
  HIPCK(hipGetLastError());
  return DCDL_OK;
}

#include "mfma_host.inc"

int mf_of(int prec) { return prec == DCDL_CORR_F64 ? MF_F64 : (prec == DCDL_CORR_BF16 ? MF_BF16 : MF_BF16X3); }

// ------------------------------------------------------------- FP64 by FFT
// Transform sizes of the FFT contraction (dcdl_fft.h): images whose powers of
// two covering T1 and T2 lie in [64, 8192] (a row transform fits the LDS), at
// most 8 channels.
bool fft_geom(const Geom &g, FftGeom *f) {
  if (g.P > 8 || g.T1 > 8192 || g.T2 > 8192) return false;
  int N1 = 1, N2 = 1;
  while (N1 < g.T1) N1 <<= 1;
  while (N2 < g.T2) N2 <<= 1;
  if (N1 < 64 || N2 < 64) return false;
  f->N1 = N1;
  f->N2 = N2;
  f->M2 = N2 / 2;
  f->F2p = (f->M2 + 1 + 15) / 16 * 16;
  if (N1 > 128) {
    f->B = 64;
    f->A = N1 / 64;
  } else {
    f->A = N1;
    f->B = 1;
  }
  f->plane = (long long)N1 * f->F2p;
  return true;
}

// An atom's spectrum skips its first column pass when its L1 rows fit in one
// row block of the second.
bool fft_atoms_sparse(const Geom &g, const FftGeom &f) { return g.L1 <= (f.B > 1 ? f.B : f.N1); }

struct FftWs {
  size_t tw, dhat, e, rhat, shat, G;
  size_t total() const { return tw + dhat + e + rhat + shat + G; }
};

// Workspace of the FFT contraction with inverse transforms kc atoms at a time.
FftWs fft_ws(const Geom &g, const FftGeom &f, int kc) {
  auto r = [](size_t b) { return (std::max<size_t>(b, 256) + 255) / 256 * 256; };
  const size_t sp = 16 * (size_t)f.plane;
  FftWs w;
  w.tw = r(16 * (size_t)(f.N1 + f.N2));
  w.dhat = r(sp * g.K * g.P);
  w.e = fft_atoms_sparse(g, f) ? r(16 * (size_t)g.K * g.P * g.L1 * f.F2p) : 0;
  w.rhat = r(sp * g.P);
  w.shat = r(sp * kc);
  w.G = r(8 * (size_t)g.K * g.H * g.W);
  return w;
}

// Estimated seconds of one FP64 contraction: on the matrix cores (FP64 MFMA
// at about 55 TFLOP/s with 16-atom tiles) and by FFT (the HBM bytes of its
// passes at about 4.5 TB/s, dictionary spectra included).
double mfma64_seconds(const Geom &g) {
  return 2.0 * 16 * ((g.K + 15) / 16) * g.P * g.L1 * g.L2 * (double)g.H * g.W / 55e12;
}

double fft64_seconds(const Geom &g, const FftGeom &f) {
  const double sp = 16.0 * f.plane, hw = (double)g.H * g.W;
  double b = (double)g.K * g.P * sp;                         // dictionary spectra (one write)
  b += g.P * (8.0 * g.T1 * g.T2 + 5 * sp);                   // rows, two column passes
  b += sp * (g.P + (double)g.K * g.P + g.K);                 // products
  b += g.K * (5 * sp + 8.0 * hw);                            // inverse passes, rows
  b += 8.0 * g.K * hw + 16.0 * hw * g.KS;                    // epilogue
  return b / 4.5e12;
}

size_t ws_held(DeviceState *ds, const char *name) {
  auto it = ds->bufs.find(name);
  return it == ds->bufs.end() ? 0 : it->second.n;
}

// The FP64 contractions of one call: how they are computed (0: FFT where it
// is estimated faster, 1: matrix cores only, 2: FFT wherever supported) and
// whether the "fft_dhat" slot holds the spectra of the call's dictionary.
struct Fp64Ctx {
  int method = 0;
  bool dhat_ok = false;
  const void *dhat = nullptr;
  int n_fft = 0;
};

// Whether an FP64 contraction of g runs by FFT under `method`, and the atom
// chunk of its inverse transforms (the workspace is kept within 60% of the
// device memory free to the library).
bool fft64_pick(DeviceState *ds, const Geom &g, int method, FftGeom *f, int *kc) {
  if (ds->arena || method == 1 || !fft_geom(g, f)) return false;
  if (method == 0 && fft64_seconds(g, *f) >= mfma64_seconds(g)) return false;
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  size_t avail = fr;
  for (const char *n : {"fft_tw", "fft_dhat", "fft_e", "fft_rhat", "fft_shat", "fft_g"}) avail += ws_held(ds, n);
  for (int c = g.K;; c = (c + 1) / 2) {
    if (fft_ws(g, *f, c).total() <= avail / 10 * 6) {
      *kc = c;
      return true;
    }
    if (c == 1) return false;
  }
}

// M-point column transforms (fft_cols) of nb spectra of S: groups g of rows
// g gmul + i stride; see ColArgs.
void fft_cols_m(int M, hipStream_t st, const FftGeom &f, double2 *S, int nb, int ngroups, int gmul, int stride,
                int rows_valid, int rows_store, int inverse, int twiddle, const double2 *tw1,
                const double2 *E = nullptr, long long eb = 0, int e_rows = 0) {
  const ColArgs ca{f, S, ngroups, gmul, stride, rows_valid, rows_store, inverse, twiddle, tw1, E, eb, e_rows};
  const int gpw = 128 / M;
  const dim3 grid(f.F2p / 16, (ngroups + gpw - 1) / gpw, nb), blk(256);
  switch (M) {
    case 4: hipLaunchKernelGGL(fft_cols<4>, grid, blk, 0, st, ca); break;
    case 8: hipLaunchKernelGGL(fft_cols<8>, grid, blk, 0, st, ca); break;
    case 16: hipLaunchKernelGGL(fft_cols<16>, grid, blk, 0, st, ca); break;
    case 32: hipLaunchKernelGGL(fft_cols<32>, grid, blk, 0, st, ca); break;
    case 64: hipLaunchKernelGGL(fft_cols<64>, grid, blk, 0, st, ca); break;
    default: hipLaunchKernelGGL(fft_cols<128>, grid, blk, 0, st, ca); break;
  }
}

// Forward column transforms of nb spectra whose input rows >= rows_valid are
// zero (digit-swapped output order), and their inverse back to natural order
// writing rows < rows_store.
void fft_cols_forward(hipStream_t st, const FftGeom &f, double2 *S, int nb, int rows_valid, const double2 *tw1) {
  if (f.B > 1) {
    fft_cols_m(f.A, st, f, S, nb, f.B, 1, f.B, rows_valid, f.N1, 0, 1, tw1);
    fft_cols_m(f.B, st, f, S, nb, f.A, f.B, 1, f.N1, f.N1, 0, 0, tw1);
  } else {
    fft_cols_m(f.N1, st, f, S, nb, 1, 0, 1, rows_valid, f.N1, 0, 0, tw1);
  }
}

void fft_cols_inverse(hipStream_t st, const FftGeom &f, double2 *S, int nb, int rows_store, const double2 *tw1) {
  if (f.B > 1) {
    fft_cols_m(f.B, st, f, S, nb, f.A, f.B, 1, f.N1, f.N1, 1, 1, tw1);
    fft_cols_m(f.A, st, f, S, nb, f.B, 1, f.B, f.N1, rows_store, 1, 0, tw1);
  } else {
    fft_cols_m(f.N1, st, f, S, nb, 1, 0, 1, f.N1, rows_store, 1, 0, tw1);
  }
}

// The FP64 contraction corr(R64, D64) by FFT with the outputs of `o` in MODE
// (as corr_mfma writes them).  The dictionary spectra are computed unless
// ctx says the "fft_dhat" slot already holds those of D64.
template <class Rz, int MODE>
int corr_fft64(DeviceState *ds, hipStream_t stream, const Geom &g, const FftGeom &f, int kc, const double *R64,
               const double *D64, const CorrOut &o, Fp64Ctx *ctx) {
  const FftWs w = fft_ws(g, f, kc);
  double2 *tw, *dhat, *E = nullptr, *rhat, *shat;
  double *G;
  WS("fft_tw", w.tw, tw);
  WS("fft_dhat", w.dhat, dhat);
  if (w.e) WS("fft_e", w.e, E);
  WS("fft_rhat", w.rhat, rhat);
  WS("fft_shat", w.shat, shat);
  WS("fft_g", w.G, G);
  double2 *tw1 = tw, *tw2 = tw + f.N1;
  hipLaunchKernelGGL(fft_twiddles, dim3(blocks_for(f.N1, 256)), dim3(256), 0, stream, f.N1, tw1);
  hipLaunchKernelGGL(fft_twiddles, dim3(blocks_for(f.N2, 256)), dim3(256), 0, stream, f.N2, tw2);
  const size_t lds_row = sizeof(double2) * (size_t)f.M2;
  const int KP = g.K * g.P;
  if (!ctx || !ctx->dhat_ok || ctx->dhat != dhat) {
    if (E) {
      hipLaunchKernelGGL(fft_rows_r2c<double>, dim3(g.L1, KP), dim3(kRowThreads), lds_row, stream, f, D64,
                         (long long)g.L1 * g.L2, g.L2, g.L2, tw2, E, (long long)g.L1 * f.F2p);
      if (f.B > 1)
        fft_cols_m(f.B, stream, f, dhat, KP, f.A, f.B, 1, f.N1, f.N1, 0, 0, tw1, E, (long long)g.L1 * f.F2p, g.L1);
      else
        fft_cols_m(f.N1, stream, f, dhat, KP, 1, 0, 1, f.N1, f.N1, 0, 0, tw1, E, (long long)g.L1 * f.F2p, g.L1);
    } else {
      hipLaunchKernelGGL(fft_rows_r2c<double>, dim3(g.L1, KP), dim3(kRowThreads), lds_row, stream, f, D64,
                         (long long)g.L1 * g.L2, g.L2, g.L2, tw2, dhat, f.plane);
      fft_cols_forward(stream, f, dhat, KP, g.L1, tw1);
    }
    if (ctx) {
      ctx->dhat_ok = true;
      ctx->dhat = dhat;
    }
  }
  hipLaunchKernelGGL(fft_rows_r2c<double>, dim3(g.T1, g.P), dim3(kRowThreads), lds_row, stream, f, R64,
                     (long long)g.T1 * g.T2, g.T2, g.T2, tw2, rhat, f.plane);
  fft_cols_forward(stream, f, rhat, g.P, g.T1, tw1);
  const long long HW = (long long)g.H * g.W;
  const double scale = 1.0 / ((double)f.N1 * f.M2);
  for (int k0 = 0; k0 < g.K; k0 += kc) {
    const int nk = std::min(kc, g.K - k0);
    if (g.P <= 4) {
      // products fused into the first inverse column pass
      const int M = f.B > 1 ? f.B : f.N1;
      const ColArgs ca = f.B > 1 ? ColArgs{f, shat, f.A, f.B, 1, f.N1, f.N1, 1, 1, tw1, nullptr, 0, 0}
                                 : ColArgs{f, shat, 1, 0, 1, f.N1, g.H, 1, 0, tw1, nullptr, 0, 0};
      const dim3 grid(f.F2p / 16, (ca.ngroups + 128 / M - 1) / (128 / M)), blk(256);
#define DCDL_COLS_PRODUCT(MM, PP) \
  hipLaunchKernelGGL((fft_cols_product<MM, PP>), grid, blk, 0, stream, ca, rhat, dhat, k0, nk)
      if (M == 64) {
        switch (g.P) {
          case 1: DCDL_COLS_PRODUCT(64, 1); break;
          case 2: DCDL_COLS_PRODUCT(64, 2); break;
          case 3: DCDL_COLS_PRODUCT(64, 3); break;
          default: DCDL_COLS_PRODUCT(64, 4); break;
        }
      } else {
        switch (g.P) {
          case 1: DCDL_COLS_PRODUCT(128, 1); break;
          case 2: DCDL_COLS_PRODUCT(128, 2); break;
          case 3: DCDL_COLS_PRODUCT(128, 3); break;
          default: DCDL_COLS_PRODUCT(128, 4); break;
        }
      }
#undef DCDL_COLS_PRODUCT
      if (f.B > 1) fft_cols_m(f.A, stream, f, shat, nk, f.B, 1, f.B, f.N1, g.H, 1, 0, tw1);
    } else {
      hipLaunchKernelGGL(fft_product, dim3(grid_stride_blocks(f.plane)), dim3(256), 0, stream, f.plane, g.P, k0,
                         nk, rhat, dhat, shat);
      fft_cols_inverse(stream, f, shat, nk, g.H, tw1);
    }
    hipLaunchKernelGGL(fft_rows_c2r, dim3(g.H, nk), dim3(kRowThreads), lds_row, stream, f, shat, f.plane, tw2,
                       G + (long long)k0 * HW, HW, g.W, scale);
  }
  const unsigned nb = (unsigned)std::min<long long>((HW + 63) / 64, 4096);
  hipLaunchKernelGGL((fft_epilogue<MODE, Rz>), dim3(nb), dim3(256), 0, stream, g, G, o);
  HIPCK(hipGetLastError());
  return DCDL_OK;
}

// ------------------------------------------------------------- DtD
// Geometry of the DtD image (dtd_image) and whether the FP64 matrix cores
// take its correlation.
bool dtd_geom(const Geom &g, Geom *gi) {
  *gi = g;
  gi->T1 = 3 * g.L1 - 2;
  gi->H = g.U1;
  gi->W = g.K * g.U2;
  gi->T2 = gi->W + g.L2 - 1;
  gi->KS = g.K;
  return (long long)g.K * g.U2 + g.L2 < (1ll << 30) && mf_supported(*gi, MF_F64);
}

struct DtdWs {
  size_t img, pk, G;
  size_t total() const { return img + pk + G; }
};

DtdWs dtd_ws_bytes(const Geom &gi) {
  auto r = [](size_t b) { return (b + 255) / 256 * 256; };
  DtdWs w;
  w.img = r(8 * (size_t)gi.P * gi.T1 * gi.T2);
  w.pk = r(mf_pack_bytes(gi, mf_plan(gi, MF_F64), MF_F64));
  w.G = r(8 * (size_t)gi.H * gi.W * gi.KS);
  return w;
}

// DtD, the apply table and 1/||D_k||^2 as one FP64 matrix-core correlation
// of the DtD image, in the caller's workspace of dtd_ws_bytes(gi).total()
// bytes.
template <class R>
int run_dtd_mfma(hipStream_t stream, const Geom &g, const Geom &gi, const R *D, R *dtd, R *A, R *inv_n, void *ws) {
  const DtdWs w = dtd_ws_bytes(gi);
  double *img = (double *)ws, *G = (double *)((char *)ws + w.img + w.pk);
  void *pk = (char *)ws + w.img;
  const long long nimg = (long long)gi.P * gi.T1 * gi.T2;
  hipLaunchKernelGGL(dtd_image<R>, dim3(grid_stride_blocks(nimg)), dim3(256), 0, stream, gi, D, img, nimg);
  const MfPlan pl = mf_plan(gi, MF_F64);
  int rc = mf_pack<R>(stream, gi, pl, MF_F64, D, pk);
  if (rc) return rc;
  CorrOut o{};
  o.beta = G;
  if ((rc = run_corr_mfma<MF_F64, CORR_BETA, double, double>(stream, gi, pl, img, pk, o))) return rc;
  const long long n = (long long)g.K * g.U1 * g.U2 * g.K;
  hipLaunchKernelGGL(dtd_gather<R>, dim3(grid_stride_blocks(n)), dim3(256), 0, stream, g, G, dtd, A, inv_n, n);
  HIPCK(hipGetLastError());
  return DCDL_OK;
}

template <class R>
int run_dtd(DeviceState *ds, hipStream_t stream, const Geom &g, const R *D, R *dtd, R *A, R *inv_n) {
  Geom gi;
  if (!dtd_geom(g, &gi)) return run_dtd_loops<R>(stream, g, D, dtd, A, inv_n);
  void *ws;
  WS("dtd_ws", dtd_ws_bytes(gi).total(), ws);
  return run_dtd_mfma<R>(stream, g, gi, D, dtd, A, inv_n, ws);
}

// The contraction actually used for a requested dcdl_corr_prec on data of
// type R: AUTO picks BF16X3 for FP32 and F64 for FP64; F64_FFT stays where
// allowed and its transform sizes apply, else becomes F64; the matrix-core
// paths fall back to DIRECT when the staged windows would not fit.  -1 for a
// BF16 request on FP64 data.
int resolve_prec(int want, bool f32, const Geom &g, bool allow_fft = false) {
  int p = want == DCDL_CORR_AUTO ? (f32 ? DCDL_CORR_BF16X3 : DCDL_CORR_F64) : want;
  if (p < DCDL_CORR_F64 || p > DCDL_CORR_F64_FFT) return -1;
  if ((p == DCDL_CORR_BF16 || p == DCDL_CORR_BF16X3) && !f32) return -1;
  if (p == DCDL_CORR_F64_FFT) {
    FftGeom f;
    if (allow_fft && fft_geom(g, &f)) return p;
    p = DCDL_CORR_F64;
  }
  if (p != DCDL_CORR_DIRECT && !mf_supported(g, mf_of(p))) p = DCDL_CORR_DIRECT;
  return p;
}

// corr(Xin, D) at a resolved precision into CORR_BETA output `ob`; `pk`
// holds D packed for that precision (mf_pack) unless DIRECT.
template <class R>
int corr_beta_at(hipStream_t stream, const Geom &g, int prec, const R *Xin, const R *D, const void *pk,
                 const CorrOut &ob) {
  if (prec == DCDL_CORR_DIRECT || !pk || !mf_supported(g, mf_of(prec)))
    return run_corr<R, R, R, CORR_BETA>(stream, g, Xin, D, ob);
  const int mp = mf_of(prec);
  const MfPlan pl = mf_plan(g, mp);
  if (mp == MF_F64) return run_corr_mfma<MF_F64, CORR_BETA, R, R>(stream, g, pl, Xin, pk, ob);
  if constexpr (std::is_same<R, float>::value) {
    if (mp == MF_BF16) return run_corr_mfma<MF_BF16, CORR_BETA, float, float>(stream, g, pl, Xin, pk, ob);
    return run_corr_mfma<MF_BF16X3, CORR_BETA, float, float>(stream, g, pl, Xin, pk, ob);
  }
  return fail(DCDL_EINVAL, "the BF16 contractions need FP32 data");
}

// beta = corr(X, D) (Z = 0) at precision `prec` (a dcdl_corr_prec); the
// contraction alone is timed by `tm` when given, and the resolved precision is
// stored in `used`.
template <class R>
int beta_init(DeviceState *ds, hipStream_t stream, const Geom &g, const R *X, const R *D, int want, R *beta,
              CorrTimer *tm = nullptr, int *used = nullptr, Fp64Ctx *ctx = nullptr) {
  int prec = resolve_prec(want, std::is_same<R, float>::value, g, true);
  if (prec < 0) return fail(DCDL_EINVAL, "beta_prec %d is not available for this dtype", want);
  CorrOut ob{};
  ob.beta = beta;
  if (prec == DCDL_CORR_F64_FFT) {
    // FP64 by FFT (the data and atoms in FP64 in the "res64" and "D64" slots);
    // the matrix cores if its workspace does not fit
    FftGeom f;
    int kc = 0;
    if (fft64_pick(ds, g, 2, &f, &kc)) {
      if (used) *used = prec;
      const long long nx = (long long)g.P * g.T1 * g.T2, nd = (long long)g.K * g.P * g.L1 * g.L2;
      double *X64, *D64;
      WS("res64", sizeof(double) * nx, X64);
      WS("D64", sizeof(double) * nd, D64);
      hipLaunchKernelGGL((convert_kernel<R, double>), dim3(grid_stride_blocks(nx)), dim3(256), 0, stream, nx, X, X64);
      hipLaunchKernelGGL((convert_kernel<R, double>), dim3(grid_stride_blocks(nd)), dim3(256), 0, stream, nd, D, D64);
      Fp64Ctx local;
      if (tm) {
        int rc = tm->begin(stream);
        if (rc) return rc;
      }
      int rc = corr_fft64<R, CORR_BETA>(ds, stream, g, f, kc, X64, D64, ob, ctx ? ctx : &local);
      if (rc || !tm) return rc;
      return tm->end(stream);
    }
    prec = mf_supported(g, MF_F64) ? DCDL_CORR_F64 : DCDL_CORR_DIRECT;
  }
  if (used) *used = prec;
  void *pk = nullptr;
  if (prec != DCDL_CORR_DIRECT) {
    const int mp = mf_of(prec);
    const MfPlan pl = mf_plan(g, mp);
    WS("dpk_init", mf_pack_bytes(g, pl, mp), pk);
    int rc = mf_pack<R>(stream, g, pl, mp, D, pk);
    if (rc) return rc;
  }
  if (tm) {
    int rc = tm->begin(stream);
    if (rc) return rc;
  }
  int rc = corr_beta_at<R>(stream, g, prec, X, D, pk, ob);
  if (rc || !tm) return rc;
  return tm->end(stream);
}

// D packed for the FP64 matrix-core contraction in the "dpk64" slot, or NULL
// when those atoms take the direct kernel.
template <class R>
int pack64(DeviceState *ds, hipStream_t stream, const Geom &g, const R *D, void **out) {
  *out = nullptr;
  if (!mf_supported(g, MF_F64)) return DCDL_OK;
  const MfPlan pl = mf_plan(g, MF_F64);
  void *pk;
  WS("dpk64", mf_pack_bytes(g, pl, MF_F64), pk);
  int rc = mf_pack<R>(stream, g, pl, MF_F64, D, pk);
  if (rc) return rc;
  *out = pk;
  return DCDL_OK;
}

// FP64 correlation of an FP64 signal: the FP64 matrix cores when `pk64` is
// set, else the direct kernel.
template <class Rz, int MODE>
int corr64(hipStream_t stream, const Geom &g, const double *R64, const double *D64, const void *pk64,
           const CorrOut &o) {
  if (pk64 && mf_supported(g, MF_F64))
    return run_corr_mfma<MF_F64, MODE, double, Rz>(stream, g, mf_plan(g, MF_F64), R64, pk64, o);
  return run_corr<double, double, Rz, MODE>(stream, g, R64, D64, o);
}

// The FP64 contraction of one call: by FFT when ctx's method picks it for
// this geometry, else corr64.
template <class Rz, int MODE>
int corr64x(DeviceState *ds, hipStream_t stream, const Geom &g, const double *R64, const double *D64,
            const void *pk64, const CorrOut &o, Fp64Ctx *ctx) {
  FftGeom f;
  int kc = 0;
  if (ctx && fft64_pick(ds, g, ctx->method, &f, &kc)) {
    ++ctx->n_fft;
    return corr_fft64<Rz, MODE>(ds, stream, g, f, kc, R64, D64, o, ctx);
  }
  return corr64<Rz, MODE>(stream, g, R64, D64, pk64, o);
}

// FP64 residual res = X - Z*D of a position-major z, enqueued without host
// synchronisation; acc[0] += sum |z|, acc[1] += nnz (acc must start at 0).
template <class R>
int residual64_async(hipStream_t stream, const Geom &g, const R *X, const double *D64, const R *zpm, double *res,
                     double *acc, const uint32_t *meta = nullptr) {
  const long long nx = (long long)g.P * g.T1 * g.T2, HW = (long long)g.H * g.W;
  hipLaunchKernelGGL((convert_kernel<R, double>), dim3(grid_stride_blocks(nx)), dim3(256), 0, stream, nx, X, res);
  const unsigned nb = (unsigned)std::min<long long>((HW + 31) / 32, 16384);
  hipLaunchKernelGGL((residual_dense<R, double>), dim3(nb), dim3(256), 0, stream, g, zpm, D64, res, acc, meta);
  HIPCK(hipGetLastError());
  return DCDL_OK;
}

// FP64 objective and strict KKT of a position-major z.  Leaves the FP64
// residual in the "res64" slot and D in FP64 in the "D64" slot.
// With beta_fix (which may be beta_cmp) the same contraction also rebuilds
// beta = G + n z there in FP64 rounded to R: the check doubles as a drift
// correction.  `tm` times the contraction.
template <class R>
int check64(DeviceState *ds, hipStream_t stream, const Geom &g, const R *X, const R *D, const R *zpm, double lambda,
            int positive, double *obj, double *kkt, long long *nnz, const R *beta_cmp = nullptr,
            const double *nrm64 = nullptr, double *drift = nullptr, R *beta_fix = nullptr,
            CorrTimer *tm = nullptr, double *g64 = nullptr, Fp64Ctx *ctx = nullptr, const uint32_t *meta = nullptr) {
  const long long nd = (long long)g.K * g.P * g.L1 * g.L2, nx = (long long)g.P * g.T1 * g.T2;
  double *D64, *res, *scal;
  WS("D64", sizeof(double) * nd, D64);
  WS("res64", sizeof(double) * nx, res);
  WS("scal", 64, scal);
  hipLaunchKernelGGL((convert_kernel<R, double>), dim3(grid_stride_blocks(nd)), dim3(256), 0, stream, nd, D, D64);
  HIPCK(hipMemsetAsync(scal, 0, 40, stream));
  int rc = residual64_async<R>(stream, g, X, D64, zpm, res, scal + 2, meta);
  if (rc) return rc;
  hipLaunchKernelGGL(sum_squares, dim3(grid_stride_blocks(nx)), dim3(256), 0, stream, nx, res, scal);
  CorrOut o{};
  o.zpm = zpm;
  o.lambda = lambda;
  o.positive = positive;
  o.result = scal + 1;
  o.beta_cmp = beta_cmp;
  o.nrm = nrm64;
  o.result2 = scal + 4;
  o.beta = beta_fix;
  o.g64 = g64;
  o.meta = meta;
  void *pk64;
  if ((rc = pack64<R>(ds, stream, g, D, &pk64))) return rc;
  if (tm && (rc = tm->begin(stream))) return rc;
  rc = corr64x<R, CORR_KKT>(ds, stream, g, res, D64, pk64, o, ctx);
  if (rc) return rc;
  if (tm && (rc = tm->end(stream))) return rc;
  double h[5];
  HIPCK(hipMemcpyAsync(h, scal, 40, hipMemcpyDeviceToHost, stream));
  HIPCK(hipStreamSynchronize(stream));
  if (obj) *obj = 0.5 * h[0] + lambda * h[2];
  if (kkt) *kkt = h[1] / lambda;
  if (nnz) *nnz = (long long)h[3];
  if (drift) *drift = beta_cmp ? h[4] / lambda : std::nan("");
  return DCDL_OK;
}

// beta = corr(X - Z*D, D) + n z by an FP64 contraction, rounded to R: the
// definition of beta in Sec. 3, used for warm starts and drift correction.
// With fresh = false it reuses the residual and D64 left by check64.
template <class R>
int beta_from_z64(DeviceState *ds, hipStream_t stream, const Geom &g, const R *X, const R *D, const R *zpm,
                  const double *nrm64, R *beta, bool fresh, CorrTimer *tm = nullptr, double *g64 = nullptr,
                  Fp64Ctx *ctx = nullptr, const uint32_t *meta = nullptr) {
  const long long nd = (long long)g.K * g.P * g.L1 * g.L2, nx = (long long)g.P * g.T1 * g.T2;
  double *D64, *res, *scal;
  WS("D64", sizeof(double) * nd, D64);
  WS("res64", sizeof(double) * nx, res);
  if (fresh) {
    WS("scal", 64, scal);
    hipLaunchKernelGGL((convert_kernel<R, double>), dim3(grid_stride_blocks(nd)), dim3(256), 0, stream, nd, D, D64);
    HIPCK(hipMemsetAsync(scal, 0, 32, stream));
    int rc = residual64_async<R>(stream, g, X, D64, zpm, res, scal + 2, meta);
    if (rc) return rc;
  }
  CorrOut ob{};
  ob.beta = beta;
  ob.zpm = zpm;
  ob.nrm = nrm64;
  ob.g64 = g64;
  ob.meta = meta;
  void *pk64;
  int rc = pack64<R>(ds, stream, g, D, &pk64);
  if (rc) return rc;
  if (tm && (rc = tm->begin(stream))) return rc;
  rc = corr64x<R, CORR_BETA>(ds, stream, g, res, D64, pk64, ob, ctx);
  if (rc || !tm) return rc;
  return tm->end(stream);
}

// The incremental FP64 check (dcdl_check.h) of a position-major z against the
// reference (gref, zref, the residual in the "res64" slot) left by the last
// dense FP64 contraction or incremental check, which it advances to z.  Needs
// D in FP64 in the "D64" slot.  Sets *used = false, changing nothing, when the
// number of changed coordinates exceeds `max_changes` (the dense contraction is
// then cheaper).  Also rebuilds beta = g + n z in `beta`.
template <class R>
int check_inc(DeviceState *ds, hipStream_t stream, const Geom &g, const R *zpm, double *gref, R *zref,
              const double *nrm64, double lambda, int positive, long long max_changes, R *beta, double *obj,
              double *kkt, long long *nnz, double *drift, bool *used, long long *n_changed) {
  *used = false;
  const long long HW = (long long)g.H * g.W, nx = (long long)g.P * g.T1 * g.T2;
  const int KS64 = atom_stride(g.K, 8);
  const long long nA64 = (long long)g.K * g.U1 * g.U2 * KS64;
  const int ntr = (g.H + kChkTH - 1) / kChkTH, ntc = (g.W + kChkTW - 1) / kChkTW;
  const long long ntiles = (long long)ntr * ntc;
  const long long per_change = ((long long)(g.U1 + kChkTH - 1) / kChkTH + 1) * ((g.U2 + kChkTW - 1) / kChkTW + 1);
  double *D64, *res, *scal, *A64, *dtd64, *inv64;
  Change *chg;
  unsigned long long *cnt;
  unsigned *tcnt, *toff, *tcur, *tlist;
  WS("D64", sizeof(double) * (size_t)g.K * g.P * g.L1 * g.L2, D64);
  WS("res64", sizeof(double) * nx, res);
  WS("scal", 64, scal);
  WS("chk_count", 16, cnt);
  WS("chk_changes", sizeof(Change) * (size_t)std::max(1ll, max_changes), chg);
  HIPCK(hipMemsetAsync(cnt, 0, 8, stream));
  HIPCK(hipMemsetAsync(scal, 0, 64, stream));
  hipLaunchKernelGGL((diff_changes<R>), dim3(grid_stride_blocks(HW * g.KS)), dim3(256), 0, stream, HW, g.K, g.KS,
                     zpm, zref, chg, cnt, max_changes, scal + 2);
  unsigned long long nch = 0;
  HIPCK(hipMemcpyAsync(&nch, cnt, 8, hipMemcpyDeviceToHost, stream));
  HIPCK(hipStreamSynchronize(stream));
  *n_changed = (long long)nch;
  if ((long long)nch > max_changes) return DCDL_OK;
  *used = true;
  // the FP64 update table A64[k0][d1][d2][k] (padding atoms zero)
  Geom g64 = g;
  g64.KS = KS64;
  WS("A64", sizeof(double) * nA64, A64);
  WS("dtd64", sizeof(double) * (size_t)g.K * g.K * g.U1 * g.U2, dtd64);
  WS("inv64", sizeof(double) * KS64, inv64);
  if (KS64 != g.K) HIPCK(hipMemsetAsync(A64, 0, sizeof(double) * nA64, stream));
  int rc = run_dtd<double>(ds, stream, g64, D64, dtd64, A64, inv64);
  if (rc) return rc;
  WS("chk_tiles", sizeof(unsigned) * (3 * (size_t)ntiles + 1), tcnt);
  toff = tcnt + ntiles;
  tcur = toff + ntiles + 1;
  WS("chk_list", sizeof(unsigned) * (size_t)std::max(1ll, (long long)nch * per_change), tlist);
  if (nch > 0) {
    const unsigned nb = (unsigned)std::min<long long>((long long)nch, 65536);
    hipLaunchKernelGGL(residual_scatter, dim3(nb), dim3(256), 0, stream, g, chg, (long long)nch, D64, res);
    HIPCK(hipMemsetAsync(tcnt, 0, sizeof(unsigned) * ntiles, stream));
    hipLaunchKernelGGL(bin_count, dim3(grid_stride_blocks((long long)nch)), dim3(256), 0, stream, g, chg,
                       (long long)nch, ntc, tcnt);
    hipLaunchKernelGGL(bin_scan, dim3(1), dim3(1024), 0, stream, tcnt, ntiles, toff, tcur);
    hipLaunchKernelGGL(bin_fill, dim3(grid_stride_blocks((long long)nch)), dim3(256), 0, stream, g, chg,
                       (long long)nch, ntc, tcur, tlist);
  } else {
    HIPCK(hipMemsetAsync(toff, 0, sizeof(unsigned) * (ntiles + 1), stream));
  }
  IncOut io{};
  io.lambda = lambda;
  io.positive = positive;
  io.nrm = nrm64;
  io.result = scal + 4;
  io.beta_cmp = beta;
  io.beta = beta;
  hipLaunchKernelGGL((g_update_kkt<R>), dim3((unsigned)ntiles), dim3(256), 0, stream, g, chg, toff, tlist, A64,
                     KS64, ntc, gref, zpm, zref, io);
  hipLaunchKernelGGL(sum_squares, dim3(grid_stride_blocks(nx)), dim3(256), 0, stream, nx, res, scal);
  HIPCK(hipGetLastError());
  double h[6];
  HIPCK(hipMemcpyAsync(h, scal, 48, hipMemcpyDeviceToHost, stream));
  HIPCK(hipStreamSynchronize(stream));
  *obj = 0.5 * h[0] + lambda * h[2];
  *kkt = h[4] / lambda;
  *nnz = (long long)h[3];
  *drift = h[5] / lambda;
  return DCDL_OK;
}

// Exact FP64 norms from D.
template <class R>
__global__ void norms64(int K, int PL, const R *D, double *nrm) {
  __shared__ double sh[4];
  const int k = blockIdx.x;
  double a = 0.0;
  for (int i = threadIdx.x; i < PL; i += blockDim.x) {
    const double d = (double)D[(long long)k * PL + i];
    a += d * d;
  }
  a = block_sum<256>(a, sh);
  if (threadIdx.x == 0) nrm[k] = a;
}

// ------------------------------------------------------------- grid plan
struct Plan {
  int W1, W2, tile1, tile2, mmax, nt;
};

template <class R, int NT>
int capacity(DeviceState *ds, int *cap) {
  int nb = 0;
  HIPCK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void *>(lgcd_rounds<R, NT>), NT, 0));
  *cap = nb * ds->cus;
  return DCDL_OK;
}

// Workgroup sizes the round kernel is built for.
bool valid_nt(int nt) { return nt == 64 || nt == 128 || nt == 192 || nt == 256 || nt == 512 || nt == 1024; }

template <class R>
int capacity_nt(DeviceState *ds, int nt, int *cap) {
  switch (nt) {
    case 64: return capacity<R, 64>(ds, cap);
    case 128: return capacity<R, 128>(ds, cap);
    case 192: return capacity<R, 192>(ds, cap);
    case 512: return capacity<R, 512>(ds, cap);
    case 1024: return capacity<R, 1024>(ds, cap);
    default: return capacity<R, 256>(ds, cap);
  }
}

int plan_grid(const Geom &g, int ndim, const dcdl_csc_opts *o, int cap, Plan *p) {
  p->tile1 = o->tile[0] > 0 ? o->tile[0] : (ndim == 1 ? 1 : 2 * g.L1);
  p->tile2 = o->tile[1] > 0 ? o->tile[1] : 2 * g.L2;
  if (ndim == 1 && o->tile[0] <= 0 && o->tile[1] <= 0) {
    p->tile1 = 1;
    p->tile2 = 2 * g.L2;
  }
  if (ndim == 1 && o->tile[0] > 0 && o->tile[1] <= 0) {  // 1-D: tile[0] is the length
    p->tile2 = o->tile[0];
    p->tile1 = 1;
  }
  const int max1 = g.H / g.L1 > 0 ? g.H / g.L1 : 1, max2 = g.W / g.L2 > 0 ? g.W / g.L2 : 1;
  int W1, W2;
  if (o->grid[0] > 0 || o->grid[1] > 0) {
    W1 = ndim == 1 ? 1 : (o->grid[0] > 0 ? o->grid[0] : 1);
    W2 = ndim == 1 ? (o->grid[0] > 0 ? o->grid[0] : o->grid[1]) : (o->grid[1] > 0 ? o->grid[1] : 1);
    if (W1 > max1 && W1 > 1) return fail(DCDL_EINVAL, "grid[0]=%d leaves workers shorter than L1=%d", W1, g.L1);
    if (W2 > max2 && W2 > 1) return fail(DCDL_EINVAL, "grid=%d leaves workers shorter than L=%d", W2, g.L2);
    if (W1 > g.H || W2 > g.W) return fail(DCDL_EINVAL, "more workers than positions");
  } else {
    // as many workers per axis as it takes for none to be longer than a
    // sub-domain (at least L long each); on the 1024^2 image with 16x16
    // atoms 32x32 workers of 31-32 positions take 303 ms of rounds where
    // 31x31 workers of 32-33 positions take 326 ms, for as many rounds
    W1 = std::max(1, std::min((g.H + p->tile1 - 1) / p->tile1, max1));
    W2 = std::max(1, std::min((g.W + p->tile2 - 1) / p->tile2, max2));
    if ((long long)W1 * W2 > cap) {
      const double f = std::sqrt((double)cap / ((double)W1 * W2));
      if (ndim == 1) {
        W2 = std::max(1, cap);
      } else {
        W1 = std::max(1, (int)(W1 * f));
        W2 = std::max(1, (int)(W2 * f));
        while ((long long)W1 * W2 > cap) {
          if (W1 >= W2) --W1; else --W2;
        }
      }
    }
  }
  if ((long long)W1 * W2 > cap)
    return fail(DCDL_EINVAL, "worker grid %dx%d exceeds the %d co-resident workgroups", W1, W2, cap);
  const int ext1 = (g.H + W1 - 1) / W1, ext2 = (g.W + W2 - 1) / W2;
  p->W1 = W1;
  p->W2 = W2;
  // the rules other than LGCD keep the grid chosen above and fix the sub-domains
  if (o->strategy == DCDL_SELECT_GREEDY) {
    p->tile1 = g.H;
    p->tile2 = g.W;
  } else if (o->strategy == DCDL_SELECT_CYCLIC) {
    p->tile1 = 1;
    p->tile2 = 1;
  }
  p->mmax = std::max(1, (ext1 + p->tile1 / 2) / p->tile1) * std::max(1, (ext2 + p->tile2 / 2) / p->tile2);
  if (o->strategy == DCDL_SELECT_RANDOM) p->mmax = ext1 * ext2;  // draws per epoch
  return DCDL_OK;
}

template <class R>
int launch_rounds(hipStream_t stream, int nt, Inst<R> *d_inst, int *d_wg, int nwg, long long timeout_ticks) {
  void *args[] = {&d_inst, &d_wg, &timeout_ticks};
  const void *fn;
  switch (nt) {
    case 64: fn = reinterpret_cast<const void *>(lgcd_rounds<R, 64>); break;
    case 192: fn = reinterpret_cast<const void *>(lgcd_rounds<R, 192>); break;
    case 128: fn = reinterpret_cast<const void *>(lgcd_rounds<R, 128>); break;
    case 512: fn = reinterpret_cast<const void *>(lgcd_rounds<R, 512>); break;
    case 1024: fn = reinterpret_cast<const void *>(lgcd_rounds<R, 1024>); break;
    default: fn = reinterpret_cast<const void *>(lgcd_rounds<R, 256>); break;
  }
  HIPCK(hipLaunchCooperativeKernel(fn, dim3(nwg), dim3(nt), args, 0, stream));
  return DCDL_OK;
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------- the solve
template <class R>
int csc_impl(DeviceState *ds, hipStream_t stream, const Geom &g_user, int ndim, const R *X, const R *D,
             const dcdl_csc_opts *o, R *z_out, dcdl_csc_info *info) {
  const double t_start = now_s();
  Geom g = g_user;
  g.KS = atom_stride(g.K, (int)sizeof(R));
  const long long HW = (long long)g.H * g.W, nz = HW * g.KS;
  const long long nA = (long long)g.K * g.U1 * g.U2 * g.KS;
  int nt = valid_nt(o->threads) ? o->threads : 256;
  int cap = 0, rc = capacity_nt<R>(ds, nt, &cap);
  if (rc) return rc;
  Plan pl;
  if ((rc = plan_grid(g, ndim, o, cap, &pl))) return rc;
  const int nW = pl.W1 * pl.W2;
  if (o->threads == 0 && ndim == 2) {
    // a grid that leaves workgroup slots of the CUs empty (one or two workers
    // per CU) gives each worker the threads of those slots: its scans and
    // patches then run on 4x or 2x the waves (the 16x16 grid of a 1024^2
    // image: 2.3x faster rounds).  Signals keep 256 threads, faster there.
    for (int big : {1024, 512}) {
      int capb = 0;
      if ((rc = capacity_nt<R>(ds, big, &capb))) return rc;
      if (nW <= capb) {
        nt = big;
        break;
      }
    }
  }

  R *beta, *zpm, *A, *dtd, *inv_n, *score;
  uint32_t *meta;
  double *nrm64;
  unsigned long long *cand;
  int *prog, *wg;
  Ctl *ctl;
  Inst<R> *d_inst;
  WS("beta", sizeof(R) * nz, beta);
  WS("zpm", sizeof(R) * nz, zpm);
  WS("score", sizeof(R) * HW, score);
  WS("meta", sizeof(uint32_t) * HW, meta);
  WS("applyA", sizeof(R) * nA, A);
  WS("dtd", sizeof(R) * (size_t)g.K * g.K * g.U1 * g.U2, dtd);
  WS("inv_n", sizeof(R) * g.KS, inv_n);
  WS("nrm64", sizeof(double) * g.K, nrm64);
  WS("cand", sizeof(unsigned long long) * 2 * nW, cand);
  WS("prog", sizeof(int) * nW, prog);
  WS("wg", sizeof(int) * nW, wg);
  WS("ctl", sizeof(Ctl) + sizeof(int) * 2 * kRing, ctl);
  WS("inst", sizeof(Inst<R>), d_inst);

  CallEvents evs;
  if ((rc = evs.init(ds))) return rc;
  hipEvent_t ev0 = evs.e[0], ev1 = evs.e[1], ev2 = evs.e[2];
  HIPCK(hipEventRecord(ev0, stream));
  if (g.KS != g.K) HIPCK(hipMemsetAsync(A, 0, sizeof(R) * nA, stream));  // padding atoms patch nothing
  HIPCK(hipMemsetAsync(inv_n, 0, sizeof(R) * g.KS, stream));
  if ((rc = run_dtd<R>(ds, stream, g, D, dtd, A, inv_n))) return rc;
  hipLaunchKernelGGL(norms64<R>, dim3(g.K), dim3(256), 0, stream, g.K, g.P * g.L1 * g.L2, D, nrm64);
  CorrTimer tm_init(evs.e[3], evs.e[4]), tm64(evs.e[5], evs.e[6]);
  int init_prec = DCDL_CORR_F64;
  // the solve's FP64 contractions share one set of dictionary spectra when
  // they run by FFT
  Fp64Ctx f64;
  f64.method = o->fp64_method;
  if (o->warm_start) {
    launch_to_position_major<R, R>(stream, HW, g.K, g.KS, z_out, zpm);
    if ((rc = beta_from_z64<R>(ds, stream, g, X, D, zpm, nrm64, beta, true, &tm64, nullptr, &f64))) return rc;
  } else {
    HIPCK(hipMemsetAsync(zpm, 0, sizeof(R) * nz, stream));
    if ((rc = beta_init<R>(ds, stream, g, X, D, o->beta_prec, beta, &tm_init, &init_prec, &f64))) return rc;
  }
  const R lam = (R)o->lambda, tol = (R)o->tol;
  launch_init_moves<R>(stream, HW, g.K, g.KS, beta, o->warm_start ? zpm : nullptr, inv_n, lam, tol, o->positive,
                       o->certify, score, meta);
  HIPCK(hipGetLastError());
  HIPCK(hipEventRecord(ev1, stream));
  HIPCK(hipEventSynchronize(ev1));
  float ms_init = 0;
  HIPCK(hipEventElapsedTime(&ms_init, ev0, ev1));

  Inst<R> hi{};
  hi.K = g.K;
  hi.KS = g.KS;
  hi.L1 = g.L1;
  hi.L2 = g.L2;
  hi.U1 = g.U1;
  hi.U2 = g.U2;
  hi.H = g.H;
  hi.W = g.W;
  hi.W1 = pl.W1;
  hi.W2 = pl.W2;
  hi.tile1 = pl.tile1;
  hi.tile2 = pl.tile2;
  hi.mmax = pl.mmax;
  hi.inner = o->inner > 0 ? o->inner : 1;
  hi.wg_base = 0;
  hi.positive = o->positive;
  hi.certify = o->certify;
  hi.soft_lock = o->no_soft_lock ? 0 : 1;
  hi.strategy = o->strategy;
  hi.seed = o->seed;
  hi.lambda = lam;
  hi.tol = tol;
  hi.div_guard = (R)o->div_guard;
  hi.beta = beta;
  hi.z = zpm;
  hi.score = score;
  hi.meta = meta;
  hi.A = A;
  hi.inv_n = inv_n;
  hi.cand = cand;
  hi.prog = prog;
  hi.ctl = ctl;
  hi.ring = reinterpret_cast<int *>(ctl + 1);
  HIPCK(hipMemsetAsync(wg, 0, sizeof(int) * nW, stream));

  const double kkt_target = o->kkt_target > 0 ? o->kkt_target : 1e-4;
  const int max_polish = o->max_polish > 0 ? o->max_polish : 2;
  const int refresh = o->refresh_every > 0 ? o->refresh_every : 0;
  const int refresh_limit = o->refresh_limit > 0 ? o->refresh_limit : 0;
  int n_refresh = 0;
  // The dense FP64 contraction: by FFT or on the matrix cores (fp64_method).
  FftGeom fgeom;
  int fkc = 0;
  const bool dense_fft = fft64_pick(ds, g, f64.method, &fgeom, &fkc);
  // FP64 reference of the incremental check: g and z of the last dense FP64
  // contraction (its residual stays in the "res64" slot).  Used with the
  // matrix-core contraction only: the FFT contraction costs less than
  // carrying forward the changes of a solve's rounds (and keeping G would add
  // its writes to every contraction).  Not used by the no-allocation entry
  // point, whose scratch holds the dense path only.
  const bool inc_ok = ds->arena == nullptr && !dense_fft;
  bool have_ref = false;
  double *gref = nullptr;
  R *zref = nullptr;
  // the incremental check pays while the changed coordinates' patches,
  // K (2L1-1)(2L2-1) FP64 table entries each, cost under half the dense
  // contraction's 2 (16 ceil(K/16)) P L1 L2 flops per position (rates of the
  // two paths on gfx950: about 6 TB/s of table reads, 55 TFLOP/s of FP64 MFMA)
  const double dense_s = dense_fft ? fft64_seconds(g, fgeom) : mfma64_seconds(g);
  const long long max_changes = std::max(1ll, std::min((long long)(0.5 * dense_s * 6e12 / (8.0 * g.K * g.U1 * g.U2)),
                                                       HW * g.K));
  CorrTimer tm_inc(evs.e[3], evs.e[4]);
  long long n_changed = 0;
  auto want_ref = [&]() -> int {
    if (!inc_ok || gref) return DCDL_OK;
    WS("gref", sizeof(double) * nz, gref);
    WS("zref", sizeof(R) * nz, zref);
    return DCDL_OK;
  };
  long long rounds_left = o->max_rounds > 0 ? o->max_rounds : (1ll << 30);
  double t_cd = 0, t_check = 0, obj = 0, kkt = 0;
  long long nnz = 0;
  unsigned long long upd = 0, cands = 0, locked = 0, visits = 0, checked = 0, patched = 0;
  double tw_wait = 0, tw_sel = 0, tw_col = 0, tw_app = 0;
  long long rounds = 0, sweeps = 0;
  int passes = 0, n_checks = 0, status = DCDL_NOT_CONVERGED, converged = 0;
  double beta_drift = std::nan("");
  const long long timeout_ticks = 500000000ll;  // 5 s per neighbour wait, 100 MHz clock
  for (;;) {
    ++passes;
    const bool refresh_due = refresh > 0 && (refresh_limit == 0 || n_refresh < refresh_limit);
    long long chunk = refresh_due ? (long long)refresh * pl.mmax : rounds_left;
    if (chunk > rounds_left) chunk = rounds_left;
    if (chunk > (1ll << 22) - 2) chunk = (1ll << 22) - 2;  // candidate tags hold 22 bits of round
    hi.max_rounds = chunk;
    {
      double budget = 120.0;  // per launch unless the caller asks for less
      if (o->timeout_s > 0) budget = std::max(1e-3, o->timeout_s - (now_s() - t_start));
      hi.budget_ticks = (long long)(budget * 1e8);
    }
    // the round log covers the first launch only
    hi.audit = passes == 1 ? reinterpret_cast<unsigned long long *>(o->audit) : nullptr;
    hi.audit_rounds = passes == 1 && o->audit ? std::max(0, o->audit_rounds) : 0;
    HIPCK(hipMemcpyAsync(d_inst, &hi, sizeof(hi), hipMemcpyHostToDevice, stream));
    HIPCK(hipMemsetAsync(prog, 0, sizeof(int) * nW, stream));
    // all-ones tags carry a round number no launch reaches
    HIPCK(hipMemsetAsync(cand, 0xff, sizeof(unsigned long long) * 2 * nW, stream));
    HIPCK(hipMemsetAsync(ctl, 0, sizeof(Ctl) + sizeof(int) * 2 * kRing, stream));
    HIPCK(hipEventRecord(ev1, stream));
    if ((rc = launch_rounds<R>(stream, nt, d_inst, wg, nW, timeout_ticks))) return rc;
    HIPCK(hipEventRecord(ev2, stream));
    Ctl hc;
    HIPCK(hipMemcpyAsync(&hc, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
    HIPCK(hipStreamSynchronize(stream));
    float ms = 0;
    HIPCK(hipEventElapsedTime(&ms, ev1, ev2));
    t_cd += ms * 1e-3;
    upd += hc.n_updates;
    cands += hc.n_candidates;
    locked += hc.n_softlocked;
    visits += hc.n_visits;
    checked += hc.n_checked;
    patched += hc.n_patched;
    tw_wait += hc.tk_wait * 1e-8 / nW;
    tw_sel += hc.tk_select * 1e-8 / nW;
    tw_col += hc.tk_collect * 1e-8 / nW;
    tw_app += hc.tk_apply * 1e-8 / nW;
    rounds += hc.max_round;
    sweeps += hc.sweeps_done;
    rounds_left -= hc.max_round;
    if (hc.status == 2) {
      status = fail(DCDL_EDIVERGED, "divergence guard tripped (|z| > %g)", o->div_guard);
      break;
    }
    if (hc.status == 3) {
      status = fail(DCDL_ETIMEOUT, "a worker waited on a neighbour for more than 5 s");
      break;
    }
    const bool time_capped = hc.status == 4;
    const double tc0 = now_s();
    const bool sweep_done = hc.converged != 0;
    const bool out_of_time = time_capped || (o->timeout_s > 0 && now_s() - t_start > o->timeout_s);
    if (!sweep_done && rounds_left > 0 && !out_of_time) {
      // a refresh chunk ended: beta rebuilt from its FP64 definition, no check.
      // (A coarser contraction here would re-inject errors above tol at every
      // chunk, and the sweep certificate could never be reached.)
      ++n_refresh;
      if ((rc = want_ref())) return rc;
      if ((rc = beta_from_z64<R>(ds, stream, g, X, D, zpm, nrm64, beta, true, &tm64, gref, &f64, meta))) return rc;
      if (gref) {
        HIPCK(hipMemcpyAsync(zref, zpm, sizeof(R) * nz, hipMemcpyDeviceToDevice, stream));
        have_ref = true;
      }
      launch_init_moves<R>(stream, HW, g.K, g.KS, beta, zpm, inv_n, lam, tol, o->positive, o->certify, score, meta,
                           meta);
      HIPCK(hipStreamSynchronize(stream));
      t_check += now_s() - tc0;
      continue;
    }
    // FP64 check of the iterate (objective, strict KKT, drift of the maintained
    // beta); the same contraction rebuilds beta from its FP64 definition for a
    // polish pass
    double drift_now = 0;
    bool inc_used = false;
    if (have_ref) {
      if ((rc = tm_inc.begin(stream))) return rc;
      rc = check_inc<R>(ds, stream, g, zpm, gref, zref, nrm64, o->lambda, o->positive, max_changes, beta, &obj, &kkt,
                        &nnz, &drift_now, &inc_used, &n_changed);
      if (rc) return rc;
      if (inc_used) {
        if ((rc = tm_inc.end(stream))) return rc;
      }
    }
    if (!inc_used) {
      if ((rc = want_ref())) return rc;
      rc = check64<R>(ds, stream, g, X, D, zpm, o->lambda, o->positive, &obj, &kkt, &nnz, beta, nrm64, &drift_now,
                      beta, &tm64, gref, &f64, meta);
      if (rc) return rc;
      have_ref = false;
    }
    if (n_checks++ == 0) beta_drift = drift_now;
    if (sweep_done && kkt <= kkt_target) {
      t_check += now_s() - tc0;
      converged = 1;
      status = DCDL_OK;
      break;
    }
    if (rounds_left <= 0 || out_of_time || (sweep_done && n_checks >= 1 + max_polish)) {
      t_check += now_s() - tc0;
      break;
    }
    // another pass: beta was rebuilt from its FP64 definition by the check,
    // which is the reference of the next one
    if (!inc_used && gref) {
      HIPCK(hipMemcpyAsync(zref, zpm, sizeof(R) * nz, hipMemcpyDeviceToDevice, stream));
      have_ref = true;
    }
    launch_init_moves<R>(stream, HW, g.K, g.KS, beta, zpm, inv_n, lam, tol, o->positive, o->certify, score, meta,
                         meta);
    HIPCK(hipStreamSynchronize(stream));
    t_check += now_s() - tc0;
  }
  if (status != DCDL_ETIMEOUT) {
    // the per-position non-zero counts match z (unless a launch ended on a
    // neighbour wait): zeros, then the positions that hold non-zeros
    HIPCK(hipMemsetAsync(z_out, 0, sizeof(R) * (size_t)g.K * HW, stream));
    hipLaunchKernelGGL(scatter_atom_major<R>, dim3(grid_stride_blocks(HW)), dim3(256), 0, stream, (int)HW, g.K, g.KS,
                       (const R *)zpm, (const uint32_t *)meta, z_out);
  } else {
    launch_to_atom_major<R, R>(stream, HW, g.K, g.KS, zpm, z_out);
  }
  HIPCK(hipGetLastError());
  HIPCK(hipStreamSynchronize(stream));
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->n_updates = (long long)upd;
    info->n_candidates = (long long)cands;
    info->n_softlocked = (long long)locked;
    info->n_rounds = rounds;
    info->n_sweeps = sweeps;
    info->n_nonzero = nnz;
    info->objective = obj;
    info->kkt = kkt;
    info->lambda_max = std::nan("");
    info->t_total_s = now_s() - t_start;
    info->t_init_s = ms_init * 1e-3;
    info->t_cd_s = t_cd;
    info->t_check_s = t_check;
    info->converged = converged;
    info->grid[0] = pl.W1;
    info->grid[1] = pl.W2;
    info->tile[0] = pl.tile1;
    info->tile[1] = pl.tile2;
    info->n_passes = passes;
    info->n_visits = (long long)visits;
    info->n_checked = (long long)checked;
    info->n_patched = (long long)patched;
    info->t_worker_wait_s = tw_wait;
    info->t_worker_select_s = tw_sel;
    info->t_worker_collect_s = tw_col;
    info->t_worker_apply_s = tw_app;
    info->beta_drift = beta_drift;
    info->t_init_corr_s = tm_init.s;
    info->t_corr64_s = tm64.s;
    info->n_corr64 = tm64.n;
    info->init_prec = init_prec;
    info->t_check_inc_s = tm_inc.s;
    info->n_check_inc = tm_inc.n;
    info->n_changed = (int32_t)std::min<long long>(n_changed, INT32_MAX);
    info->n_fft64 = f64.n_fft + (init_prec == DCDL_CORR_F64_FFT ? 1 : 0);
  }
  return status;
}

template <class R>
int corr_impl(DeviceState *ds, hipStream_t stream, Geom g, const R *X, const R *D, R *out, int prec) {
  g.KS = atom_stride(g.K, (int)sizeof(R));
  const long long HW = (long long)g.H * g.W;
  R *gpm;
  WS("corr_pm", sizeof(R) * HW * g.KS, gpm);
  int rc = beta_init<R>(ds, stream, g, X, D, prec, gpm);
  if (rc) return rc;
  launch_to_atom_major<R, R>(stream, HW, g.K, g.KS, gpm, out);
  HIPCK(hipGetLastError());
  HIPCK(hipStreamSynchronize(stream));
  return DCDL_OK;
}

// lambda_max = max |corr(X, D)| (one-sided if positive) in FP64 (Sec. 2).
template <class R>
int lambda_max_impl(DeviceState *ds, hipStream_t stream, const Geom &g, const R *X, const R *D, int positive,
                    double *out) {
  const long long nx = (long long)g.P * g.T1 * g.T2, nd = (long long)g.K * g.P * g.L1 * g.L2;
  double *X64, *D64, *scal;
  WS("res64", sizeof(double) * nx, X64);
  WS("D64", sizeof(double) * nd, D64);
  WS("scal", 64, scal);
  hipLaunchKernelGGL((convert_kernel<R, double>), dim3(grid_stride_blocks(nx)), dim3(256), 0, stream, nx, X, X64);
  hipLaunchKernelGGL((convert_kernel<R, double>), dim3(grid_stride_blocks(nd)), dim3(256), 0, stream, nd, D, D64);
  HIPCK(hipMemsetAsync(scal, 0, 16, stream));
  CorrOut o{};
  o.positive = positive;
  o.result = scal;
  void *pk64;
  int rc = pack64<double>(ds, stream, g, D64, &pk64);
  if (rc) return rc;
  Fp64Ctx ctx;
  if ((rc = corr64x<double, CORR_ABSMAX>(ds, stream, g, X64, D64, pk64, o, &ctx))) return rc;
  HIPCK(hipMemcpyAsync(out, scal, sizeof(double), hipMemcpyDeviceToHost, stream));
  HIPCK(hipStreamSynchronize(stream));
  return DCDL_OK;
}

// Argument checks of dicodile_csc and its no-allocation variant, made before
// any device access.
int validate_csc(const dcdl_shape *shape, const void *X, const void *D, const dcdl_csc_opts *opts,
                 const void *z_out, Geom *g) {
  int rc = make_geom(shape, g);
  if (rc) return rc;
  if (!X || !D || !opts || !z_out) return fail(DCDL_EINVAL, "NULL pointer");
  if (!(opts->lambda > 0)) return fail(DCDL_EINVAL, "lambda must be > 0");
  if (!(opts->tol >= 0)) return fail(DCDL_EINVAL, "tol must be >= 0");
  if (opts->dtype != DCDL_F32 && opts->dtype != DCDL_F64) return fail(DCDL_EINVAL, "unknown dtype");
  if (opts->threads != 0 && !valid_nt(opts->threads))
    return fail(DCDL_EINVAL, "threads must be 64, 128, 192, 256, 512 or 1024");
  if (opts->tile[0] < 0 || opts->tile[1] < 0 || opts->grid[0] < 0 || opts->grid[1] < 0)
    return fail(DCDL_EINVAL, "negative tile or grid");
  if (opts->max_rounds > (1ll << 30)) return fail(DCDL_EINVAL, "max_rounds above 2^30");
  if (opts->strategy < DCDL_SELECT_LGCD || opts->strategy > DCDL_SELECT_RANDOM)
    return fail(DCDL_EINVAL, "unknown selection rule %d", opts->strategy);
  return DCDL_OK;
}

// Scratch bytes a solve carves (every workspace slot of csc_impl and the
// calls it makes, each rounded up to 256 bytes), with the worker count bounded
// by 8192 workgroups.
size_t csc_scratch_need(const Geom &g_user, const dcdl_csc_opts *o) {
  const bool f32 = o->dtype == DCDL_F32;
  const size_t es = f32 ? 4 : 8;
  Geom g = g_user;
  g.KS = atom_stride(g.K, (int)es);
  auto r = [](size_t b) { return (std::max<size_t>(b, 256) + 255) / 256 * 256; };
  const size_t HW = (size_t)g.H * g.W, nz = HW * g.KS, nA = (size_t)g.K * g.U1 * g.U2 * g.KS;
  const size_t nW = 8192;
  size_t need = 2 * r(es * nz) + r(es * HW) + r(4 * HW) + r(es * nA) + r(es * g.K * g.K * g.U1 * g.U2) +
                r(es * g.KS) + r(8 * (size_t)g.K) + r(16 * nW) + 2 * r(4 * nW) +
                r(sizeof(Ctl) + sizeof(int) * 2 * kRing) + r(std::max(sizeof(Inst<float>), sizeof(Inst<double>)));
  need += r(8 * (size_t)g.K * g.P * g.L1 * g.L2) + r(8 * (size_t)g.P * g.T1 * g.T2) + r(64);
  Geom gi;
  if (dtd_geom(g, &gi)) need += r(dtd_ws_bytes(gi).total());
  if (mf_supported(g, MF_F64)) need += r(mf_pack_bytes(g, mf_plan(g, MF_F64), MF_F64));
  if (!o->warm_start) {
    const int prec = resolve_prec(o->beta_prec, f32, g);
    if (prec >= 0 && prec != DCDL_CORR_DIRECT) need += r(mf_pack_bytes(g, mf_plan(g, mf_of(prec)), mf_of(prec)));
  }
  return need;
}

// Once per device, with it current: the device's address of `scratch` and the
// events of its no-allocation calls.
int noalloc_setup(DeviceState *ds) {
  if (ds->scratch_ptr) return DCDL_OK;
  void *p = nullptr;
  HIPCK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) return fail(DCDL_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
  for (int i = 0; i < kCallEvents; ++i) HIPCK(hipEventCreate(&ds->na_ev[i]));
  ds->scratch_ptr = static_cast<unsigned char *>(p);
  return DCDL_OK;
}

struct ArenaScope {
  DeviceState *ds;
  ScratchArena a;
  explicit ArenaScope(DeviceState *d) : ds(d) {
    a.base = d->scratch_ptr;
    a.cap = kScratchBytes;
    ds->arena = &a;
  }
  ~ArenaScope() { ds->arena = nullptr; }
};

struct Guard {
  DeviceState *ds;
  explicit Guard(DeviceState *d) : ds(d) { ds->mu.lock(); }
  ~Guard() { ds->mu.unlock(); }
};

#define PROLOGUE()                                                        \
  g_err.clear();                                                          \
  DeviceState *ds = device_state(nullptr);                                \
  if (!ds) return fail(DCDL_EHIP, "hipGetDevice failed");                 \
  Guard guard_(ds);                                                       \
  {                                                                       \
    int rc0_ = check_device(ds);                                          \
    if (rc0_) return rc0_;                                                \
  }                                                                       \
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);

}  // namespace

// ================================================================= C ABI
extern "C" {

const char *dicodile_version(void) { return "dicodile-mi355x 0.1 (gfx950)"; }

const char *dicodile_last_error(void) { return g_err.c_str(); }

// Frees every workspace buffer and destroys the library-owned stream of every
// device the library has touched, each with that device current; the caller's
// current device is restored.  Servers own their resources and are released
// by dicodile_server_destroy.
int dicodile_release(void) {
  g_err.clear();
  int cur = 0;
  HIPCK(hipGetDevice(&cur));
  std::vector<std::pair<int, DeviceState *>> devs;
  {
    std::lock_guard<std::mutex> lk(g_devices_mu);
    for (auto &kv : g_devices) devs.push_back(kv);
  }
  int rc = DCDL_OK;
  for (auto &kv : devs) {
    DeviceState *ds = kv.second;
    Guard guard_(ds);
    if (hipSetDevice(kv.first) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
      rc = fail(DCDL_EHIP, "device %d: synchronisation before release failed", kv.first);
      continue;
    }
    for (auto &b : ds->bufs)
      if (b.second.p && hipFree(b.second.p) != hipSuccess) rc = fail(DCDL_EHIP, "hipFree failed");
    ds->bufs.clear();
    if (ds->aux) {
      if (hipStreamDestroy(ds->aux) != hipSuccess) rc = fail(DCDL_EHIP, "hipStreamDestroy failed");
      ds->aux = nullptr;
    }
    // the scratch array itself stays (it is part of the loaded code object);
    // the next no-allocation call looks its address up again
    for (auto &e : ds->na_ev)
      if (e) {
        (void)hipEventDestroy(e);
        e = nullptr;
      }
    ds->scratch_ptr = nullptr;
  }
  HIPCK(hipSetDevice(cur));
  return rc;
}

int dicodile_dtd(const dcdl_shape *shape, dcdl_dtype dtype, const void *D, void *dtd_out, void *stream_) {
  Geom g;
  int rc = make_geom(shape, &g);
  if (rc) return rc;
  if (!D || !dtd_out) return fail(DCDL_EINVAL, "NULL pointer");
  PROLOGUE();
  const long long nA = (long long)g.K * g.U1 * g.U2 * g.K;
  if (dtype == DCDL_F32) {
    float *A, *inv;
    WS("applyA", sizeof(float) * nA, A);
    WS("inv_n", sizeof(float) * g.K, inv);
    if ((rc = run_dtd<float>(ds, stream, g, (const float *)D, (float *)dtd_out, A, inv))) return rc;
  } else if (dtype == DCDL_F64) {
    double *A, *inv;
    WS("applyA", sizeof(double) * nA, A);
    WS("inv_n", sizeof(double) * g.K, inv);
    if ((rc = run_dtd<double>(ds, stream, g, (const double *)D, (double *)dtd_out, A, inv))) return rc;
  } else {
    return fail(DCDL_EINVAL, "unknown dtype %d", (int)dtype);
  }
  HIPCK(hipStreamSynchronize(stream));
  return DCDL_OK;
}

int dicodile_lambda_max(const dcdl_shape *shape, dcdl_dtype dtype, const void *X, const void *D, int32_t positive,
                        double *out, void *stream_) {
  Geom g;
  int rc = make_geom(shape, &g);
  if (rc) return rc;
  if (!X || !D || !out) return fail(DCDL_EINVAL, "NULL pointer");
  if (dtype != DCDL_F32 && dtype != DCDL_F64) return fail(DCDL_EINVAL, "unknown dtype %d", (int)dtype);
  PROLOGUE();
  if (dtype == DCDL_F32) return lambda_max_impl<float>(ds, stream, g, (const float *)X, (const float *)D, positive, out);
  return lambda_max_impl<double>(ds, stream, g, (const double *)X, (const double *)D, positive, out);
}

int dicodile_csc(const dcdl_shape *shape, const void *X, const void *D, const dcdl_csc_opts *opts, void *z_out,
                 dcdl_csc_info *info, void *stream_) {
  Geom g;
  int rc = validate_csc(shape, X, D, opts, z_out, &g);
  if (rc) return rc;
  PROLOGUE();
  if (opts->dtype == DCDL_F32)
    return csc_impl<float>(ds, stream, g, shape->ndim, (const float *)X, (const float *)D, opts, (float *)z_out, info);
  return csc_impl<double>(ds, stream, g, shape->ndim, (const double *)X, (const double *)D, opts, (double *)z_out,
                          info);
}

int dicodile_csc_noalloc(const dcdl_shape *shape, const void *X, const void *D, const dcdl_csc_opts *opts,
                         void *z_out, dcdl_csc_info *info, void *stream_) {
  Geom g;
  int rc = validate_csc(shape, X, D, opts, z_out, &g);
  if (rc) return rc;
  const size_t need = csc_scratch_need(g, opts);
  if (need > kScratchBytes)
    return fail(DCDL_EINVAL, "this solve needs %zu bytes of workspace; the fixed scratch of dicodile_csc_noalloc "
                "holds %zu", need, kScratchBytes);
  PROLOGUE();
  if ((rc = noalloc_setup(ds))) return rc;
  ArenaScope scope(ds);
  if (opts->dtype == DCDL_F32)
    return csc_impl<float>(ds, stream, g, shape->ndim, (const float *)X, (const float *)D, opts, (float *)z_out, info);
  return csc_impl<double>(ds, stream, g, shape->ndim, (const double *)X, (const double *)D, opts, (double *)z_out,
                          info);
}

int dicodile_corr(const dcdl_shape *shape, dcdl_dtype dtype, const void *X, const void *D, void *out, int32_t prec,
                  void *stream_) {
  Geom g;
  int rc = make_geom(shape, &g);
  if (rc) return rc;
  if (!X || !D || !out) return fail(DCDL_EINVAL, "NULL pointer");
  if (dtype != DCDL_F32 && dtype != DCDL_F64) return fail(DCDL_EINVAL, "unknown dtype %d", (int)dtype);
  if (prec < DCDL_CORR_AUTO || prec > DCDL_CORR_F64_FFT) return fail(DCDL_EINVAL, "unknown precision %d", prec);
  if (dtype == DCDL_F64 && (prec == DCDL_CORR_BF16 || prec == DCDL_CORR_BF16X3))
    return fail(DCDL_EINVAL, "the BF16 contractions need FP32 data");
  PROLOGUE();
  if (dtype == DCDL_F32) return corr_impl<float>(ds, stream, g, (const float *)X, (const float *)D, (float *)out, prec);
  return corr_impl<double>(ds, stream, g, (const double *)X, (const double *)D, (double *)out, prec);
}

int dicodile_objective_kkt(const dcdl_shape *shape, dcdl_dtype dtype, const void *X, const void *D, const void *z,
                           double lambda, int32_t positive, double *objective, double *kkt, void *stream_) {
  Geom g;
  int rc = make_geom(shape, &g);
  if (rc) return rc;
  if (!X || !D || !z) return fail(DCDL_EINVAL, "NULL pointer");
  if (!(lambda > 0)) return fail(DCDL_EINVAL, "lambda must be > 0");
  PROLOGUE();
  const long long HW = (long long)g.H * g.W, nz = HW * g.K;
  const unsigned pb = blocks_for(HW, 256);
  if (dtype == DCDL_F32) {
    float *zpm;
    WS("zpm_check", sizeof(float) * nz, zpm);
    launch_to_position_major<float, float>(stream, HW, g.K, g.KS, (const float *)z, zpm);
    Fp64Ctx ctx;
    return check64<float>(ds, stream, g, (const float *)X, (const float *)D, zpm, lambda, positive, objective, kkt,
                          nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, &ctx);
  } else if (dtype == DCDL_F64) {
    double *zpm;
    WS("zpm_check", sizeof(double) * nz, zpm);
    launch_to_position_major<double, double>(stream, HW, g.K, g.KS, (const double *)z, zpm);
    Fp64Ctx ctx;
    return check64<double>(ds, stream, g, (const double *)X, (const double *)D, zpm, lambda, positive, objective,
                           kkt, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, &ctx);
  }
  return fail(DCDL_EINVAL, "unknown dtype %d", (int)dtype);
}

int dicodile_copy_probe(void *dst, const void *src, size_t bytes, int32_t repeats, double *seconds,
                        void *stream_) {
  if (!dst || !src || bytes == 0 || (bytes & 15) || ((uintptr_t)dst & 15) || ((uintptr_t)src & 15) || repeats < 1)
    return fail(DCDL_EINVAL, "copy probe needs 16-byte aligned, non-empty buffers and repeats >= 1");
  PROLOGUE();
  const long long n16 = (long long)(bytes / 16);
  if ((n16 + 255) / 256 > 0x7fffffffll) return fail(DCDL_EINVAL, "copy probe of more than 2^39 bytes");
  const unsigned nb = (unsigned)((n16 + 255) / 256);
  hipEvent_t e0, e1;
  HIPCK(hipEventCreate(&e0));
  HIPCK(hipEventCreate(&e1));
  HIPCK(hipEventRecord(e0, stream));
  for (int i = 0; i < repeats; ++i)
    hipLaunchKernelGGL(copy_probe, dim3(nb), dim3(256), 0, stream, n16, (const uint4 *)src, (uint4 *)dst);
  HIPCK(hipGetLastError());
  HIPCK(hipEventRecord(e1, stream));
  HIPCK(hipEventSynchronize(e1));
  float ms = 0;
  HIPCK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (seconds) *seconds = ms * 1e-3 / repeats;
  return DCDL_OK;
}

}  // extern "C"

namespace {

template <class R>
int dict_stats_impl(DeviceState *ds, hipStream_t stream, const Geom &g, const R *z, const R *X, R *ztz, R *ztX,
                    double **phi64_out = nullptr, double **psi64_out = nullptr) {
  const long long HW = (long long)g.H * g.W, nz = HW * g.K;
  const long long nphi = (long long)g.K * g.K * g.U1 * g.U2, npsi = (long long)g.K * g.P * g.L1 * g.L2;
  unsigned int *cnt;
  double *phi64, *psi64;
  R *zpm;
  int *nzc;
  WS("st_cnt", sizeof(unsigned int) * 2 * g.K, cnt);
  WS("st_phi", sizeof(double) * nphi, phi64);
  WS("st_psi", sizeof(double) * npsi, psi64);
  WS("st_zpm", sizeof(R) * nz, zpm);
  WS("st_nzc", sizeof(int) * HW, nzc);
  uint32_t *nzbits;
  const long long nbw = (HW + 63) / 64 * 2;
  WS("st_nzbits", sizeof(uint32_t) * nbw, nzbits);
  HIPCK(hipMemsetAsync(cnt, 0, sizeof(unsigned int) * 2 * g.K, stream));
  HIPCK(hipMemsetAsync(phi64, 0, sizeof(double) * nphi, stream));
  HIPCK(hipMemsetAsync(psi64, 0, sizeof(double) * npsi, stream));
  HIPCK(hipMemsetAsync(nzc, 0, sizeof(int) * HW, stream));
  HIPCK(hipMemsetAsync(nzbits, 0, sizeof(uint32_t) * nbw, stream));
  // z position-major with the non-zero counts of every position and atom
  hipLaunchKernelGGL(to_position_major_counts<R>, dim3((unsigned)((HW + 63) / 64), (unsigned)((g.KS + 63) / 64)),
                     dim3(256), 0, stream, (int)HW, g.K, g.KS, z, zpm, nzc, cnt, nzbits);
  std::vector<unsigned int> hc(g.K);
  HIPCK(hipMemcpyAsync(hc.data(), cnt, sizeof(unsigned int) * g.K, hipMemcpyDeviceToHost, stream));
  HIPCK(hipStreamSynchronize(stream));
  std::vector<unsigned int> off(g.K);
  long long total = 0;
  std::vector<Chunk> chunks;
  constexpr int CH = 128;
  for (int k = 0; k < g.K; ++k) {
    off[k] = (unsigned int)total;
    for (unsigned int b = 0; b < hc[k]; b += CH) {
      Chunk c;
      c.k = k;
      c.beg = (int)(total + b);
      c.end = (int)(total + std::min<unsigned int>(hc[k], b + CH));
      c.pad = 0;
      chunks.push_back(c);
    }
    total += hc[k];
  }
  if (total > 0) {
    NzEntry *list;
    Chunk *d_chunks;
    WS("st_list", sizeof(NzEntry) * total, list);
    WS("st_chunks", sizeof(Chunk) * chunks.size(), d_chunks);
    HIPCK(hipMemcpyAsync(cnt + g.K, off.data(), sizeof(unsigned int) * g.K, hipMemcpyHostToDevice, stream));
    HIPCK(hipMemcpyAsync(d_chunks, chunks.data(), sizeof(Chunk) * chunks.size(), hipMemcpyHostToDevice, stream));
    hipLaunchKernelGGL(list_from_position_major<R>, dim3(grid_stride_blocks(HW)), dim3(256), 0, stream, (int)HW,
                       g.K, g.KS, zpm, nzc, cnt + g.K, list);
    hipLaunchKernelGGL(psi_kernel<R>, dim3((unsigned)chunks.size()), dim3(256), 0, stream, g, d_chunks, list, X,
                       psi64);
    const long long nb = total < 65536 ? total : 65536;
    hipLaunchKernelGGL(phi_kernel<R>, dim3((unsigned)nb), dim3(256), 0, stream, g, list, total, zpm, nzbits, phi64);
    HIPCK(hipGetLastError());
  }
  if (ztz)
    hipLaunchKernelGGL((convert_kernel<double, R>), dim3(grid_stride_blocks(nphi)), dim3(256), 0, stream, nphi,
                       phi64, ztz);
  if (ztX)
    hipLaunchKernelGGL((convert_kernel<double, R>), dim3(grid_stride_blocks(npsi)), dim3(256), 0, stream, npsi,
                       psi64, ztX);
  HIPCK(hipGetLastError());
  HIPCK(hipStreamSynchronize(stream));
  if (phi64_out) *phi64_out = phi64;
  if (psi64_out) *psi64_out = psi64;
  return DCDL_OK;
}

}  // namespace

extern "C" int dicodile_dict_stats(const dcdl_shape *shape, dcdl_dtype dtype, const void *z, const void *X,
                                   void *ztz_out, void *ztX_out, void *stream_) {
  Geom g;
  int rc = make_geom(shape, &g);
  if (rc) return rc;
  if (!z || !X || !ztz_out || !ztX_out) return fail(DCDL_EINVAL, "NULL pointer");
  PROLOGUE();
  if (dtype == DCDL_F32)
    return dict_stats_impl<float>(ds, stream, g, (const float *)z, (const float *)X, (float *)ztz_out,
                                  (float *)ztX_out);
  if (dtype == DCDL_F64)
    return dict_stats_impl<double>(ds, stream, g, (const double *)z, (const double *)X, (double *)ztz_out,
                                   (double *)ztX_out);
  return fail(DCDL_EINVAL, "unknown dtype %d", (int)dtype);
}
#include "batch.inc"
#include "tune.inc"
#include "dict.inc"
#include "serve.inc"
