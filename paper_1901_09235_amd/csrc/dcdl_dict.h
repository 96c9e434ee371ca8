// dcdl_dict.h -- kernels of the dictionary update (Sec. 4.2, eq. dict_update).
//
// With the sufficient statistics phi (K, K, 2L-1...) and psi (K, P, L...) of
// eq. phi, the data term of eq. dict_update and its gradient are
//   F(D)      = 1/2 ||X||^2 - <D, psi> + 1/2 <D, Q(D)>
//   grad F(D) = Q(D) - psi,   Q(D)_{k,p}[t] = sum_{k'} sum_{t'} phi[k, k', t - t'] D_{k',p}[t']
// (Q is the quadratic form's matrix applied to D; the signal size does not
// enter).  Everything here runs in FP64: the problem is K P |Theta| values.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dcdl_kernels.h"

namespace dcdl {

constexpr int kDictMaxTaps = 2048;  // |Theta| handled by one phi_matvec workgroup (8 outputs per thread)

// Q = phi applied to D.  One workgroup per (k, p); for each k' the row
// phi[k, k', :] and the atom D[k', p, :] are staged in LDS.
__global__ __launch_bounds__(256) void phi_matvec(Geom g, const double *__restrict__ phi,
                                                  const double *__restrict__ D, double *__restrict__ Q) {
  extern __shared__ double dsm[];
  const int n = g.L1 * g.L2, m = g.U1 * g.U2;
  double *sd = dsm, *sp = dsm + n;
  const int k = blockIdx.x, p = blockIdx.y, tid = threadIdx.x;
  double acc[kDictMaxTaps / 256];
#pragma unroll
  for (int i = 0; i < kDictMaxTaps / 256; ++i) acc[i] = 0.0;
  for (int kk = 0; kk < g.K; ++kk) {
    __syncthreads();
    for (int i = tid; i < n; i += 256) sd[i] = D[((long long)kk * g.P + p) * n + i];
    for (int i = tid; i < m; i += 256) sp[i] = phi[((long long)k * g.K + kk) * m + i];
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kDictMaxTaps / 256; ++s) {
      const int t = tid + 256 * s;
      if (t >= n) break;
      const int t1 = t / g.L2, t2 = t - (t / g.L2) * g.L2;
      double a = 0.0;
      for (int u1 = 0; u1 < g.L1; ++u1) {
        const double *prow = sp + (t1 - u1 + g.L1 - 1) * g.U2 + t2 + g.L2 - 1;
        const double *drow = sd + u1 * g.L2;
        for (int u2 = 0; u2 < g.L2; ++u2) a += prow[-u2] * drow[u2];
      }
      acc[s] += a;
    }
  }
#pragma unroll
  for (int s = 0; s < kDictMaxTaps / 256; ++s) {
    const int t = tid + 256 * s;
    if (t >= n) break;
    Q[((long long)k * g.P + p) * n + t] = acc[s];
  }
}

// One projected-gradient trial: Dn = Proj(D - step G), one workgroup per atom.
// Proj scales an atom whose norm exceeds 1 back to the unit sphere.
__global__ __launch_bounds__(256) void pgd_trial(int per_atom, const double *__restrict__ D,
                                                 const double *__restrict__ G, double step, double *__restrict__ Dn) {
  __shared__ double sh[4];
  const long long base = (long long)blockIdx.x * per_atom;
  double a = 0.0;
  for (int i = threadIdx.x; i < per_atom; i += 256) {
    const double v = D[base + i] - step * G[base + i];
    Dn[base + i] = v;
    a += v * v;
  }
  a = block_sum<256>(a, sh);
  if (a > 1.0) {
    const double s = 1.0 / sqrt(a);
    for (int i = threadIdx.x; i < per_atom; i += 256) Dn[base + i] *= s;
  }
}

// out[0] += <Dn, psi>, out[1] += <Dn, Qn>, out[2] += <G, Dn - D> (D, G may be NULL).
__global__ __launch_bounds__(256) void trial_dots(long long n, const double *__restrict__ Dn,
                                                  const double *__restrict__ D, const double *__restrict__ psi,
                                                  const double *__restrict__ Qn, const double *__restrict__ G,
                                                  double *out) {
  __shared__ double sh[4];
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    const double d = Dn[i];
    a0 += d * psi[i];
    a1 += d * Qn[i];
    if (G) a2 += G[i] * (d - D[i]);
  }
  a0 = block_sum<256>(a0, sh);
  a1 = block_sum<256>(a1, sh);
  a2 = block_sum<256>(a2, sh);
  if (threadIdx.x == 0) {
    atomic_add_f64(out, a0);
    atomic_add_f64(out + 1, a1);
    atomic_add_f64(out + 2, a2);
  }
}

// G = Q - psi.
__global__ __launch_bounds__(256) void grad_from_q(long long n, const double *__restrict__ Q,
                                                   const double *__restrict__ psi, double *__restrict__ G) {
  for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (long long)gridDim.x * 256) G[i] = Q[i] - psi[i];
}

// out = max_k sum_{k', tau} |phi[k, k', tau]|: an upper bound of every row sum
// of the quadratic form's matrix, hence of its largest eigenvalue (Gershgorin).
__global__ __launch_bounds__(256) void phi_row_bound(int K, int m, const double *__restrict__ phi, double *out) {
  __shared__ double sh[4];
  const int k = blockIdx.x;
  double a = 0.0;
  for (long long i = threadIdx.x; i < (long long)K * m; i += 256) a += fabs(phi[(long long)k * K * m + i]);
  a = block_sum<256>(a, sh);
  if (threadIdx.x == 0) atomic_max_nonneg(out, a);
}

}  // namespace dcdl
