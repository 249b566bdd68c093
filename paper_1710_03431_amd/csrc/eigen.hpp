// Workgroup-level FP64 dense symmetric eigensolver (device functions).
//
// A symmetric N x N matrix in global memory is reduced to tridiagonal form by
// Householder reflections (each reflection maps the part of a row right of
// the diagonal onto a multiple of the first unit vector, applied from both
// sides to the trailing block as a rank-2 update), the tridiagonal matrix is
// diagonalised by implicit symmetric QR steps with the Wilkinson shift (a
// Givens rotation seeded by the shifted leading column, then chased down the
// band), and the eigenvectors are obtained by applying the reflections to the
// accumulated rotations.  Textbook algorithms (Householder 1958; Francis QR
// with Wilkinson's shift), restated for a 256-thread workgroup:
//   * the reflection is built with two block reductions, the trailing block
//     is updated by all threads with accesses contiguous along rows;
//   * one thread computes the rotation sequence of a QR sweep on the band
//     (O(N) scalar work) and publishes it in LDS, then every thread applies
//     the whole sequence to its own rows of Z (column-major, so the updates
//     of a column pair are contiguous across threads);
//   * eigenvalues are ranked in parallel into a stable ascending order.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace aqt {

constexpr int kEigThreads = 256;
constexpr int kEigMaxN = 1024;

// LDS state of the solver for matrices of order up to MaxN.
template <int MaxN>
struct EigSharedN {
  static constexpr int kMax = MaxN;
  double v[MaxN];     // Householder vector / scratch
  double w[MaxN];     // p, then w
  double d[MaxN];     // band diagonal
  double e[MaxN];     // band off-diagonal
  double beta[MaxN];  // reflection coefficients
  double c[MaxN];     // rotation cosines of one sweep
  double s[MaxN];     // rotation sines of one sweep
  double red[kEigThreads / kWave];
  int lo, hi, done, fail;
};
using EigShared = EigSharedN<kEigMaxN>;

__device__ __forceinline__ double block_sum(double v, double* red) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < kEigThreads / kWave; ++i) t += red[i];
  return t;
}

// Reduce symmetric A (row-major, leading dimension lda) to tridiagonal form.
// On exit sh.d/sh.e hold the band, sh.beta the reflection coefficients and row
// j of A, right of the diagonal, the Householder vector of step j.  Per step the
// product with the Householder vector and the rank-2 update of the whole trailing
// block, reading both triangles: for matrices that stay in the caches.
template <class Sh>
__device__ void wg_tridiagonalize(double* A, int N, int lda, Sh& sh) {
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1), wave = tid >> 6;
  for (int j = 0; j + 2 < N; ++j) {
    const int L = N - j - 1;
    double* row = A + static_cast<size_t>(j) * lda + j + 1;
    double part = 0.0;
    for (int i = tid + 1; i < L; i += kEigThreads) part += row[i] * row[i];
    const double tail = block_sum(part, sh.red);
    const double x0 = row[0];
    if (tid == 0) sh.d[j] = A[static_cast<size_t>(j) * lda + j];
    if (tail == 0.0) {
      if (tid == 0) {
        sh.e[j] = x0;
        sh.beta[j] = 0.0;
      }
      __syncthreads();
      continue;
    }
    const double sigma = sqrt(x0 * x0 + tail);
    const double alpha = (x0 >= 0.0) ? -sigma : sigma;
    const double v0 = x0 - alpha;
    const double beta = 2.0 / (v0 * v0 + tail);
    for (int i = tid; i < L; i += kEigThreads) sh.v[i] = (i == 0) ? v0 : row[i];
    __syncthreads();
    // p = beta * S v, S the trailing block; one wavefront per row
    for (int i = wave; i < L; i += kEigThreads / kWave) {
      const double* Si = A + static_cast<size_t>(j + 1 + i) * lda + j + 1;
      double acc = 0.0;
      for (int k = lane; k < L; k += kWave) acc += Si[k] * sh.v[k];
      acc = wave_sum(acc);
      if (lane == 0) sh.w[i] = beta * acc;
    }
    __syncthreads();
    part = 0.0;
    for (int i = tid; i < L; i += kEigThreads) part += sh.v[i] * sh.w[i];
    const double Kc = 0.5 * beta * block_sum(part, sh.red);
    for (int i = tid; i < L; i += kEigThreads) sh.w[i] -= Kc * sh.v[i];
    __syncthreads();
    const size_t tot = static_cast<size_t>(L) * L;
    for (size_t f = tid; f < tot; f += kEigThreads) {
      const int i = static_cast<int>(f / L), k = static_cast<int>(f - static_cast<size_t>(i) * L);
      A[static_cast<size_t>(j + 1 + i) * lda + j + 1 + k] -= sh.v[i] * sh.w[k] + sh.w[i] * sh.v[k];
    }
    for (int i = tid; i < L; i += kEigThreads) row[i] = sh.v[i];
    if (tid == 0) {
      sh.e[j] = alpha;
      sh.beta[j] = beta;
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (N >= 2) {
      sh.d[N - 2] = A[static_cast<size_t>(N - 2) * lda + N - 2];
      sh.e[N - 2] = A[static_cast<size_t>(N - 2) * lda + N - 1];
      sh.beta[N - 2] = 0.0;
    }
    sh.d[N - 1] = A[static_cast<size_t>(N - 1) * lda + N - 1];
    sh.e[N - 1] = 0.0;
    sh.beta[N - 1] = 0.0;
  }
  __syncthreads();
}

// wg_tridiagonalize for a matrix too large for the caches, where the reduction is
// bound by HBM bandwidth (same results on exit; the rest of A is overwritten).
// Only the lower triangle is read.  The rank-2 updates (v w^T + w v^T) are held back
// -- up to two, in sh.c / sh.s (free until the QR sweep) and in pend (2 MaxN
// doubles) -- and written into A every other step, in the pass that forms that
// step's symmetric product from the updated entries; the steps between read the
// stale lower triangle and correct the product by the held-back updates (two dot
// products each).  The product: row sums by wavefront reductions, the transposed
// half accumulated per lane and combined across wavefronts in a fixed order.  Per
// two steps one read-write and one read-only pass over the lower triangle: a quarter
// of the traffic of wg_tridiagonalize (which reads the full matrix for the product
// and reads and writes it for the update, every step).
template <class Sh>
__device__ void wg_tridiagonalize_streamed(double* A, int N, int lda, Sh& sh, double* pend) {
  constexpr int NT = (Sh::kMax + kWave - 1) / kWave;   // column slots per lane
  constexpr int NW = kEigThreads / kWave;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1), wave = tid >> 6;
  // held-back updates r = 0, 1: the trailing block is A - sum_r (pv_r pw_r^T + pw_r pv_r^T)
  double* pv0 = sh.c;
  double* pw0 = sh.s;
  double* pv1 = pend;
  double* pw1 = pend + Sh::kMax;
  for (int i = tid; i < N; i += kEigThreads) {
    pv0[i] = 0.0;
    pw0[i] = 0.0;
    pv1[i] = 0.0;
    pw1[i] = 0.0;
  }
  __syncthreads();
  int npend = 0;   // held-back updates in use (slots 0 .. npend - 1)
  for (int j = 0; j + 2 < N; ++j) {
    const int c0 = j + 1;
    const double pv0j = pv0[j], pw0j = pw0[j], pv1j = pv1[j], pw1j = pw1[j];
    // column j below the diagonal, updated
    double part = 0.0;
    for (int i = c0 + tid; i < N; i += kEigThreads) {
      const double x = A[static_cast<size_t>(i) * lda + j] - (pv0[i] * pw0j + pw0[i] * pv0j) -
                       (pv1[i] * pw1j + pw1[i] * pv1j);
      sh.v[i] = x;
      if (i > c0) part += x * x;
    }
    const double tail = block_sum(part, sh.red);
    const double x0 = sh.v[c0];
    const bool refl = tail != 0.0;
    const double sigma = sqrt(x0 * x0 + tail);
    const double alpha = (x0 >= 0.0) ? -sigma : sigma;
    const double v0 = x0 - alpha;
    const double bet = refl ? 2.0 / (v0 * v0 + tail) : 0.0;
    __syncthreads();   // every thread has read x0
    if (tid == 0) {
      sh.d[j] = A[static_cast<size_t>(j) * lda + j] - 2.0 * (pv0j * pw0j + pv1j * pw1j);
      sh.e[j] = refl ? alpha : x0;
      sh.beta[j] = bet;
      if (refl) sh.v[c0] = v0;
    }
    __syncthreads();
    if (refl)
      for (int i = c0 + tid; i < N; i += kEigThreads) A[static_cast<size_t>(j) * lda + i] = sh.v[i];
    const bool flush = npend == 2;   // this pass writes both held-back updates into A
    if (!flush && !refl) continue;   // nothing to write, nothing to multiply
    double q[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) q[t] = 0.0;
    for (int i = c0 + wave; i < N; i += NW) {
      double* row = A + static_cast<size_t>(i) * lda;
      const double pv0i = pv0[i], pw0i = pw0[i], pv1i = pv1[i], pw1i = pw1[i];
      const double vi = refl ? sh.v[i] : 0.0;
      double a[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int k = c0 + lane + kWave * t;
        a[t] = (c0 + kWave * t <= i && k <= i) ? row[k] : 0.0;
      }
      double acc = 0.0;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int k = c0 + lane + kWave * t;
        if (c0 + kWave * t <= i && k <= i) {
          double x = a[t];
          if (flush) {
            x -= (pv0i * pw0[k] + pw0i * pv0[k]) + (pv1i * pw1[k] + pw1i * pv1[k]);
            row[k] = x;
          }
          if (refl) {
            acc += x * sh.v[k];
            if (k < i) q[t] += x * vi;
          }
        }
      }
      if (refl) {
        acc = wave_sum(acc);
        if (lane == 0) sh.w[i] = acc;
      }
    }
    __syncthreads();   // pass done: row sums in sh.w
    if (refl) {
      for (int r = 0; r < NW; ++r) {
        if (wave == r) {
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            const int k = c0 + lane + kWave * t;
            if (k < N) sh.w[k] += q[t];
          }
        }
        __syncthreads();
      }
      if (!flush && npend > 0) {
        // the pass read the stale block: subtract the held-back updates' product with v
        double d00 = 0.0, d01 = 0.0, d10 = 0.0, d11 = 0.0;
        for (int i = c0 + tid; i < N; i += kEigThreads) {
          const double vv = sh.v[i];
          d00 += pw0[i] * vv;
          d01 += pv0[i] * vv;
          d10 += pw1[i] * vv;
          d11 += pv1[i] * vv;
        }
        d00 = block_sum(d00, sh.red);
        d01 = block_sum(d01, sh.red);
        d10 = block_sum(d10, sh.red);
        d11 = block_sum(d11, sh.red);
        for (int i = c0 + tid; i < N; i += kEigThreads)
          sh.w[i] -= (pv0[i] * d00 + pw0[i] * d01) + (pv1[i] * d10 + pw1[i] * d11);
      }
      double pp = 0.0;
      for (int i = c0 + tid; i < N; i += kEigThreads) {
        const double wi = bet * sh.w[i];
        sh.w[i] = wi;
        pp += sh.v[i] * wi;
      }
      const double Kc = 0.5 * bet * block_sum(pp, sh.red);
      // the new update goes to slot 0 after a flush (slot 1 cleared), else to slot npend
      const int slot = flush ? 0 : npend;
      double* nv = slot ? pv1 : pv0;
      double* nw = slot ? pw1 : pw0;
      for (int i = c0 + tid; i < N; i += kEigThreads) {
        nv[i] = sh.v[i];
        nw[i] = sh.w[i] - Kc * sh.v[i];
        if (flush) {
          pv1[i] = 0.0;
          pw1[i] = 0.0;
        }
      }
      npend = slot + 1;
    } else {
      // a flush without a reflection: both slots are written into A
      for (int i = c0 + tid; i < N; i += kEigThreads) {
        pv0[i] = 0.0;
        pw0[i] = 0.0;
        pv1[i] = 0.0;
        pw1[i] = 0.0;
      }
      npend = 0;
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (N >= 2) {
      const int a = N - 2, b = N - 1;
      sh.d[a] = A[static_cast<size_t>(a) * lda + a] - 2.0 * (pv0[a] * pw0[a] + pv1[a] * pw1[a]);
      sh.e[a] = A[static_cast<size_t>(b) * lda + a] - (pv0[b] * pw0[a] + pw0[b] * pv0[a]) -
                (pv1[b] * pw1[a] + pw1[b] * pv1[a]);
      sh.beta[a] = 0.0;
    }
    sh.d[N - 1] = A[static_cast<size_t>(N - 1) * lda + N - 1] -
                  2.0 * (pv0[N - 1] * pw0[N - 1] + pv1[N - 1] * pw1[N - 1]);
    sh.e[N - 1] = 0.0;
    sh.beta[N - 1] = 0.0;
  }
  __syncthreads();
}

// Implicit symmetric QR on the band in sh.d/sh.e; rotations accumulated into
// Z (column-major N x N, leading dimension ldz), which is initialised to I here
// unless from_z is set (then Z's columns are rotated as given: starting from the
// reflection product, Z ends up holding the eigenvectors of the full matrix).
// Returns false if the iteration budget is exhausted.
template <class Sh>
__device__ bool wg_band_qr(double* Z, int N, int ldz, Sh& sh, bool from_z = false) {
  const int tid = threadIdx.x;
  if (!from_z)
    for (int c = 0; c < N; ++c)
      for (int r = tid; r < N; r += kEigThreads) Z[static_cast<size_t>(c) * ldz + r] = (r == c) ? 1.0 : 0.0;
  if (tid == 0) {
    sh.done = 0;
    sh.fail = 0;
    sh.hi = N - 1;
  }
  __syncthreads();
  const long budget = 64L * N + 64;
  for (long sweep = 0;; ++sweep) {
    if (tid < kWave) {
      // wavefront 0: deflation.  Negligible off-diagonal entries below hi are zeroed;
      // the window [l, m] is the unreduced block that ends at the highest nonzero e.
      const int m0 = sh.hi;
      for (int k = tid; k < m0; k += kWave)
        if (fabs(sh.e[k]) <= 2.220446049250313e-16 * (fabs(sh.d[k]) + fabs(sh.d[k + 1]))) sh.e[k] = 0.0;
      int m = 0;
      for (int c = (m0 - 1) / kWave; c >= 0 && m0 > 0; --c) {
        const int k = c * kWave + tid;
        const unsigned long long nz = __ballot(k < m0 && sh.e[k] != 0.0);
        if (nz) {
          m = c * kWave + (63 - __clzll(nz)) + 1;
          break;
        }
      }
      int l = 0;
      for (int c = (m - 2) / kWave; c >= 0 && m >= 2; --c) {
        const int k = c * kWave + tid;
        const unsigned long long zr = __ballot(k < m - 1 && sh.e[k] == 0.0);
        if (zr) {
          l = c * kWave + (63 - __clzll(zr)) + 1;
          break;
        }
      }
      const bool have = m > 0;
      if (tid == 0) {
        sh.hi = m;
        if (!have || sweep >= budget) {
          sh.done = 1;
          sh.fail = have ? 1 : 0;
        } else {
          // Wilkinson shift from the trailing 2x2 block of the window [l, m]
          const double delta = 0.5 * (sh.d[m - 1] - sh.d[m]);
          const double bb = sh.e[m - 1];
          const double den = delta + copysign(hypot(delta, bb), delta >= 0.0 ? 1.0 : -1.0);
          const double mu = sh.d[m] - bb * bb / den;
          // bulge chase; the running diagonal (dk), the scaled off-diagonal (bk) and the
          // untouched next diagonal (dn) stay in registers, the next band entries are
          // loaded one rotation ahead.  1/r by Newton's iteration for the reciprocal
          // square root (two steps from the hardware estimate), squares in range.
          double x = sh.d[l] - mu, z = sh.e[l];
          double dk = sh.d[l], bk = sh.e[l], dn = sh.d[l + 1];
          double ek = 0.0;
          for (int k = l; k < m; ++k) {
            const bool more = k + 1 < m;
            const double en = more ? sh.e[k + 1] : 0.0;
            const double dnn = more ? sh.d[k + 2] : 0.0;
            const double q = fma(x, x, z * z);
            double r, ri;
            if (q > 1e-300 && q < 1e300) {
              double y = __builtin_amdgcn_rsq(q);
              const double hq = 0.5 * q;
              y = y * fma(-hq * y, y, 1.5);
              y = y * fma(-hq * y, y, 1.5);
              ri = y;
              r = q * y;
            } else {
              r = hypot(x, z);
              ri = 1.0 / r;
            }
            const double c = x * ri, s = z * ri;
            if (k > l) sh.e[k - 1] = r;
            const double a = dk, b = bk, cc = dn;
            sh.d[k] = c * c * a + 2.0 * c * s * b + s * s * cc;
            dk = s * s * a - 2.0 * c * s * b + c * c * cc;
            ek = c * s * (cc - a) + (c * c - s * s) * b;
            if (more) {
              z = s * en;
              bk = c * en;
              dn = dnn;
            }
            x = ek;
            sh.c[k] = c;
            sh.s[k] = s;
          }
          sh.d[m] = dk;
          sh.e[m - 1] = ek;
          sh.lo = l;
        }
      }
    }
    __syncthreads();
    if (sh.done) break;
    const int l = sh.lo, m = sh.hi;
    for (int r = tid; r < N; r += kEigThreads) {
      double zk = Z[static_cast<size_t>(l) * ldz + r];
      int k = l;
      // eight columns loaded ahead of their rotations: each column is read before the
      // rotation that rewrites it, and the loads are in flight together
      for (; k + 8 <= m; k += 8) {
        double z1[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) z1[u] = Z[static_cast<size_t>(k + 1 + u) * ldz + r];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const double c = sh.c[k + u], s = sh.s[k + u];
          Z[static_cast<size_t>(k + u) * ldz + r] = c * zk + s * z1[u];
          zk = -s * zk + c * z1[u];
        }
      }
      for (; k < m; ++k) {
        const double zk1 = Z[static_cast<size_t>(k + 1) * ldz + r];
        const double c = sh.c[k], s = sh.s[k];
        Z[static_cast<size_t>(k) * ldz + r] = c * zk + s * zk1;
        zk = -s * zk + c * zk1;
      }
      Z[static_cast<size_t>(m) * ldz + r] = zk;
    }
    __syncthreads();
  }
  const bool ok = !sh.fail;
  __syncthreads();
  return ok;
}

// Apply the stored reflections to the columns of Z listed in cols[0..ncols-1]
// (column-major), turning band eigenvectors into eigenvectors of A.  Per
// reflection one pass for the dot products with the columns and one for their
// update: for matrices that stay in the caches.
template <class Sh>
__device__ void wg_back_transform(const double* A, int N, int lda, double* Z, int ldz, const int* cols, int ncols,
                                  Sh& sh) {
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1), wave = tid >> 6;
  for (int j = N - 3; j >= 0; --j) {
    const double beta = sh.beta[j];
    if (beta == 0.0) continue;
    const int L = N - j - 1;
    const double* vrow = A + static_cast<size_t>(j) * lda + j + 1;
    for (int i = tid; i < L; i += kEigThreads) sh.v[i] = vrow[i];
    __syncthreads();
    for (int q = wave; q < ncols; q += kEigThreads / kWave) {
      const double* zc = Z + static_cast<size_t>(cols[q]) * ldz + j + 1;
      double acc = 0.0;
      for (int i = lane; i < L; i += kWave) acc += sh.v[i] * zc[i];
      acc = wave_sum(acc);
      if (lane == 0) sh.w[q] = beta * acc;
    }
    __syncthreads();
    const size_t tot = static_cast<size_t>(ncols) * L;
    for (size_t f = tid; f < tot; f += kEigThreads) {
      const int q = static_cast<int>(f / L), i = static_cast<int>(f - static_cast<size_t>(q) * L);
      Z[static_cast<size_t>(cols[q]) * ldz + j + 1 + i] -= sh.w[q] * sh.v[i];
    }
    __syncthreads();
  }
}

// wg_back_transform for matrices too large for the caches: each wavefront holds a
// group of kBtCols columns of Z in registers (row lane + 64 t in slot t) while every
// reflection is applied to them, so Z is read and written once and each reflection
// is read once per group (wg_back_transform moves Z three times per reflection).
constexpr int kBtCols = 2;
template <class Sh>
__device__ void wg_back_transform_streamed(const double* A, int N, int lda, double* Z, int ldz, const int* cols,
                                           int ncols, Sh& sh) {
  constexpr int NT = (Sh::kMax + kWave - 1) / kWave;
  constexpr int NW = kEigThreads / kWave;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6;
  const int ngrp = (ncols + kBtCols - 1) / kBtCols;
  for (int gi = wave; gi < ngrp; gi += NW) {
    double* zc[kBtCols];
    double z[kBtCols][NT];
#pragma unroll
    for (int c = 0; c < kBtCols; ++c) {
      const int q = gi * kBtCols + c;
      zc[c] = (q < ncols) ? Z + static_cast<size_t>(cols[q]) * ldz : nullptr;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int r = lane + kWave * t;
        z[c][t] = (zc[c] != nullptr && r < N) ? zc[c][r] : 0.0;
      }
    }
    for (int j = N - 3; j >= 0; --j) {
      const double beta = sh.beta[j];
      if (beta == 0.0) continue;
      const double* vrow = A + static_cast<size_t>(j) * lda;   // v_j at rows j+1 .. N-1
      double v[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int r = lane + kWave * t;
        v[t] = (r > j && r < N) ? vrow[r] : 0.0;
      }
      double dot[kBtCols];
#pragma unroll
      for (int c = 0; c < kBtCols; ++c) {
        double acc = 0.0;
#pragma unroll
        for (int t = 0; t < NT; ++t) acc = fma(v[t], z[c][t], acc);
        dot[c] = acc;
      }
#pragma unroll
      for (int c = 0; c < kBtCols; ++c) dot[c] = beta * wave_sum(dot[c]);
#pragma unroll
      for (int c = 0; c < kBtCols; ++c)
#pragma unroll
        for (int t = 0; t < NT; ++t) z[c][t] = fma(-dot[c], v[t], z[c][t]);
    }
#pragma unroll
    for (int c = 0; c < kBtCols; ++c)
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int r = lane + kWave * t;
        if (zc[c] != nullptr && r < N) zc[c][r] = z[c][t];
      }
  }
  __syncthreads();
}

// Stable ascending rank of the eigenvalues: perm[rank] = index.  A NaN ranks as
// +infinity (ties by index), so perm is a permutation for any input and every
// index read through it stays in range.
__device__ __forceinline__ double rank_key(double v) { return (v == v) ? v : __builtin_huge_val(); }
__device__ void wg_rank_ascending(const double* d, int N, int* perm) {
  for (int i = threadIdx.x; i < N; i += kEigThreads) {
    const double di = rank_key(d[i]);
    int rank = 0;
    for (int j = 0; j < N; ++j) {
      const double dj = rank_key(d[j]);
      rank += (dj < di) || (dj == di && j < i);
    }
    perm[rank] = i;
  }
  __syncthreads();
}


// ---- small matrices resident in LDS (order N <= kEigThreads) -------------------
// One thread per row (or column) walks it serially: no block reductions in the
// inner loops, and a leading dimension that is odd in doubles keeps the threads of
// a wavefront on different banks.

// sum_k a[k] b[k] over k < L, eight independent loads and partial sums in flight
__device__ __forceinline__ double lds_dot(const double* a, const double* b, int L) {
  double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int k = 0;
  for (; k + 8 <= L; k += 8) {
    double x[8], y[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      x[u] = a[k + u];
      y[u] = b[k + u];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] = fma(x[u], y[u], acc[u]);
  }
  for (; k < L; ++k) acc[0] = fma(a[k], b[k], acc[0]);
  return ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
}

// y[k] -= alpha * x[k] + beta * z[k] over k < L, eight entries per batch
__device__ __forceinline__ void lds_axpy2(double* y, double alpha, const double* x, double beta, const double* z,
                                          int L) {
  int k = 0;
  for (; k + 8 <= L; k += 8) {
    double yy[8], xx[8], zz[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      yy[u] = y[k + u];
      xx[u] = x[k + u];
      zz[u] = z[k + u];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) y[k + u] = yy[u] - (alpha * xx[u] + beta * zz[u]);
  }
  for (; k < L; ++k) y[k] -= alpha * x[k] + beta * z[k];
}

// Householder tridiagonalisation as wg_tridiagonalize, A row-major in LDS.
template <class Sh>
__device__ void lds_tridiagonalize(double* A, int N, int lda, Sh& sh) {
  const int tid = threadIdx.x;
  for (int j = 0; j + 2 < N; ++j) {
    const int L = N - j - 1;
    double* row = A + j * lda + j + 1;
    if (tid < kWave) {
      double part = 0.0;
      for (int i = tid + 1; i < L; i += kWave) part += row[i] * row[i];
      part = wave_sum(part);
      if (tid == 0) sh.red[j & 1] = part;   // alternating slot: readers of step j-1 may lag
    }
    __syncthreads();
    const double tail = sh.red[j & 1];
    const double x0 = row[0];
    if (tid == 0) sh.d[j] = A[j * lda + j];
    if (tail == 0.0) {
      if (tid == 0) {
        sh.e[j] = x0;
        sh.beta[j] = 0.0;
      }
      __syncthreads();
      continue;
    }
    const double sigma = sqrt(x0 * x0 + tail);
    const double alpha = (x0 >= 0.0) ? -sigma : sigma;
    const double v0 = x0 - alpha;
    const double beta = 2.0 / (v0 * v0 + tail);
    for (int i = tid; i < L; i += blockDim.x) sh.v[i] = (i == 0) ? v0 : row[i];
    __syncthreads();
    // p = beta * S v, one thread per row of the trailing block S
    for (int i = tid; i < L; i += blockDim.x) sh.w[i] = beta * lds_dot(A + (j + 1 + i) * lda + j + 1, sh.v, L);
    __syncthreads();
    // Kc = beta/2 v.p (every thread, broadcast reads); with w = p - Kc v the update is
    // S_ik -= v_i w_k + w_i v_k = v_i p_k + (w_i - Kc v_i) v_k
    const double Kc = 0.5 * beta * lds_dot(sh.v, sh.w, L);
    for (int i = tid; i < L; i += blockDim.x) {
      const double vi = sh.v[i], wi = sh.w[i] - Kc * vi;
      lds_axpy2(A + (j + 1 + i) * lda + j + 1, vi, sh.w, wi - Kc * vi, sh.v, L);
      row[i] = vi;
    }
    if (tid == 0) {
      sh.e[j] = alpha;
      sh.beta[j] = beta;
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (N >= 2) {
      sh.d[N - 2] = A[(N - 2) * lda + N - 2];
      sh.e[N - 2] = A[(N - 2) * lda + N - 1];
      sh.beta[N - 2] = 0.0;
    }
    sh.d[N - 1] = A[(N - 1) * lda + N - 1];
    sh.e[N - 1] = 0.0;
    sh.beta[N - 1] = 0.0;
  }
  __syncthreads();
}

// Z = H_0 H_1 ... H_{N-3}, the product of the reflections of lds_tridiagonalize
// (vectors in Hv, row j right of the diagonal, leading dimension ldh; coefficients in
// sh.beta), column-major in LDS (leading dimension ldz), one thread per column.
// Columns q <= j are still unit vectors when H_j is applied, so only q > j are touched.
template <class Sh>
__device__ void lds_form_q(const double* Hv, int ldh, int N, double* Z, int ldz, Sh& sh) {
  const int tid = threadIdx.x;
  for (int f = tid; f < N * N; f += blockDim.x) {
    const int c = f / N, r = f - c * N;
    Z[c * ldz + r] = (r == c) ? 1.0 : 0.0;
  }
  for (int j = N - 3; j >= 0; --j) {
    const double beta = sh.beta[j];
    if (beta == 0.0) continue;
    const int L = N - j - 1;
    const double* vrow = Hv + static_cast<size_t>(j) * ldh + j + 1;
    __syncthreads();   // previous step's readers of sh.v are done (and Z's first fill)
    for (int i = tid; i < L; i += blockDim.x) sh.v[i] = vrow[i];
    __syncthreads();
    for (int q = j + 1 + tid; q < N; q += blockDim.x) {
      double* zc = Z + q * ldz + j + 1;
      const double w = beta * lds_dot(sh.v, zc, L);
      lds_axpy2(zc, w, sh.v, 0.0, sh.v, L);
    }
  }
  __syncthreads();
}

// ---- lowest eigenpairs of the band without the full rotation product --------
// Number of eigenvalues of the symmetric tridiagonal (d, e) below x (Sturm count
// of the LDL^T pivots; a zero pivot is replaced by -tiny).
__device__ __forceinline__ int sturm_count(const double* d, const double* e, int N, double x, double tiny) {
  int cnt = 0;
  double q = d[0] - x;
  cnt += q < 0.0;
  for (int i = 1; i < N; ++i) {
    const double den = (q != 0.0) ? q : -tiny;
    q = (d[i] - x) - e[i - 1] * e[i - 1] / den;
    cnt += q < 0.0;
  }
  return cnt;
}

// k-th smallest eigenvalue (0-based) of the band by bisection inside [lo, hi].
__device__ double band_bisect(const double* d, const double* e, int N, int k, double lo, double hi, double tiny) {
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (!(mid > lo && mid < hi)) break;
    if (hi - lo <= 4.440892098500626e-16 * fmax(fabs(lo), fabs(hi)) + tiny) break;
    if (sturm_count(d, e, N, mid, tiny) > k) hi = mid;
    else lo = mid;
  }
  return 0.5 * (lo + hi);
}

// Inverse iteration for eigenvalue lam of the band: LU of (T - lam I) with partial
// pivoting (a zero pivot becomes tiny), three solves from a fixed start vector, each
// normalised.  ws: 4N doubles plus N bytes of pivot flags; x: N doubles.
__device__ void band_inverse_iteration(const double* d, const double* e, int N, double lam, double tiny,
                                       unsigned seed, double* ws, unsigned char* piv, double* x) {
  double* dl = ws;
  double* dd = ws + N;
  double* du = ws + 2 * N;
  double* du2 = ws + 3 * N;
  for (int i = 0; i < N; ++i) {
    dd[i] = d[i] - lam;
    if (i + 1 < N) {
      dl[i] = e[i];
      du[i] = e[i];
    }
    du2[i] = 0.0;
  }
  for (int i = 0; i + 1 < N; ++i) {
    if (fabs(dd[i]) >= fabs(dl[i])) {
      piv[i] = 0;
      if (dd[i] == 0.0) dd[i] = tiny;
      const double f = dl[i] / dd[i];
      dl[i] = f;
      dd[i + 1] -= f * du[i];
    } else {
      piv[i] = 1;
      const double f = dd[i] / dl[i];
      dd[i] = dl[i];
      dl[i] = f;
      const double t = du[i];
      du[i] = dd[i + 1];
      dd[i + 1] = t - f * dd[i + 1];
      if (i + 2 < N) {
        du2[i] = du[i + 1];
        du[i + 1] = -f * du[i + 1];
      }
    }
  }
  if (dd[N - 1] == 0.0) dd[N - 1] = tiny;
  uint32_t h = seed * 2654435761u + 12345u;
  for (int i = 0; i < N; ++i) {
    h ^= h << 13;
    h ^= h >> 17;
    h ^= h << 5;
    x[i] = static_cast<double>(h & 0xffffff) * (1.0 / 16777216.0) - 0.5;
  }
  for (int it = 0; it < 3; ++it) {
    for (int i = 0; i + 1 < N; ++i) {
      if (piv[i] == 0) {
        x[i + 1] -= dl[i] * x[i];
      } else {
        const double t = x[i];
        x[i] = x[i + 1];
        x[i + 1] = t - dl[i] * x[i];
      }
    }
    x[N - 1] /= dd[N - 1];
    if (N >= 2) x[N - 2] = (x[N - 2] - du[N - 2] * x[N - 1]) / dd[N - 2];
    for (int i = N - 3; i >= 0; --i) x[i] = (x[i] - du[i] * x[i + 1] - du2[i] * x[i + 2]) / dd[i];
    double nn = 0.0;
    for (int i = 0; i < N; ++i) nn += x[i] * x[i];
    const double inv = (nn > 0.0 && nn < 1e300) ? 1.0 / sqrt(nn) : 0.0;
    for (int i = 0; i < N; ++i) x[i] *= inv;
  }
}

}  // namespace aqt
