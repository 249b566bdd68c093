// GPU precompute of the instantaneous eigensystem and the AME tables (FP64).
//
// Per grid point s_g (Sec. II eq. Lindblad2 needs the eigenpairs of H_S(t)):
//   k_build_dense  H(s_g) = A(s_g) H_X + B(s_g) diag(e_Z)  (Sec. V eq. H_S)
//   k_dense_eig    workgroup eigensolver (eigen.hpp), eigenvalues ranked
//   k_canon        clusters of levels closer than deg_tol rotated to the
//                  eigenbasis of the projected diagonal operator diag(x)
//                  (energies become Rayleigh quotients); column signs fixed
//                  so that the first entry within 1e-9 of the column's largest
//                  magnitude is positive; truncation to the n lowest levels
//   k_gemm_f64     MFMA (16x16x4 FP64) products V_g V_{g-1}^T (overlaps) and
//                  V_g diag(sz_i) V_g^T (matrix elements <a|sz_i|b>)
//   k_polar        polar factor of the truncated overlap via the eigen-
//                  decomposition of M^T M; leakage 1 - sigma_min^2
//   (2^n_qubits > 1024: Chebyshev-filtered subspace iteration with a
//   matrix-free H replaces k_build_dense and k_dense_eig; see below)
//   k_rates        R[i][b][a] = gamma(e_b - e_a) z_ab^2 (a != b),
//                  gamma(0) z_bb^2 (a == b), Ohmic gamma (Sec. V), and zdiag
// The ground state of H(s_0) (must be non-degenerate) is expressed in the
// grid-1 basis and normalised: the initial state of every trajectory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"
#include "ctx.hpp"
#include "eigen.hpp"

namespace aqt {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

inline unsigned nblk(int64_t count, int threads = 256) {
  return static_cast<unsigned>((count + threads - 1) / threads);
}

__global__ void k_ising_diag(const double* __restrict__ h, const double* __restrict__ J, int nq,
                             double* __restrict__ eZ) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= (1 << nq)) return;
  double e = 0.0;
  for (int i = 0; i < nq; ++i) {
    const double si = ((x >> i) & 1) ? -1.0 : 1.0;
    e += h[i] * si;
    for (int j = i + 1; j < nq; ++j) {
      const double sj = ((x >> j) & 1) ? -1.0 : 1.0;
      e += J[i * nq + j] * si * sj;
    }
  }
  eZ[x] = e;
}

__global__ void k_build_dense(const double* __restrict__ eZ, int nq, const double* __restrict__ Ag,
                              const double* __restrict__ Bg, int g0, int count, double* __restrict__ H) {
  const int N = 1 << nq;
  const int64_t per = static_cast<int64_t>(N) * N;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= per * count) return;
  const int c = static_cast<int>(idx / per);
  const int64_t r = idx - c * per;
  const int x = static_cast<int>(r / N), y = static_cast<int>(r - static_cast<int64_t>(x) * N);
  const int g = g0 + c;
  double v = 0.0;
  if (x == y) v = Bg[g] * eZ[x];
  else if (__popc(static_cast<unsigned>(x ^ y)) == 1) v = -Ag[g];
  H[idx] = v;
}

// One workgroup per matrix: eigenvalues (ascending, stable) and eigenvectors.
// Z is column-major: Z[col * N + row]; perm[a] is the column of level a.
// STREAMED: the order is at least kStreamedEigMin, so the matrix lives in HBM
// rather than the caches, and the reduction and back transform take their
// bandwidth-saving forms (a separate instantiation, as their register needs
// would lower the occupancy of the cached form).
constexpr int kStreamedEigMin = 512;
template <bool STREAMED>
__global__ __launch_bounds__(kEigThreads) void k_dense_eig(double* H, double* Z, int N, int ncols, int partial,
                                                           double* __restrict__ Eraw, int* __restrict__ perm,
                                                           int* __restrict__ status) {
  __shared__ EigShared sh;
  __shared__ int s_perm[kEigMaxN];
  __shared__ double s_lo, s_hi;
  __shared__ double s_pend[STREAMED ? 2 * kEigMaxN : 1];   // second held-back update of the reduction
  const int c = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* A = H + static_cast<size_t>(c) * N * N;
  double* Zc = Z + static_cast<size_t>(c) * N * N;
  if (STREAMED) wg_tridiagonalize_streamed(A, N, N, sh, s_pend);
  else wg_tridiagonalize(A, N, N, sh);
  if (!partial) {
    const bool ok = wg_band_qr(Zc, N, N, sh);
    wg_rank_ascending(sh.d, N, s_perm);
    if (STREAMED) wg_back_transform_streamed(A, N, N, Zc, N, s_perm, ncols, sh);
    else wg_back_transform(A, N, N, Zc, N, s_perm, ncols, sh);
    for (int a = tid; a < N; a += blockDim.x) {
      perm[static_cast<size_t>(c) * N + a] = s_perm[a];
      Eraw[static_cast<size_t>(c) * N + a] = sh.d[s_perm[a]];
    }
    if (tid == 0) status[c] = ok ? 0 : 1;
    return;
  }
  // Lowest ncols pairs only: bisection for the eigenvalues of the band, inverse
  // iteration for its eigenvectors, one orthonormalisation and a Rayleigh-Ritz step
  // on the band inside their span, then the Householder back-transform.  Columns
  // ncols.. of Zc serve as workspace.
  const int nc = ncols;
  double* X = Zc;                                        // band eigenvectors, column-major
  double* Dsv = Zc + static_cast<size_t>(nc) * N;        // band diagonal
  double* Esv = Dsv + N;                                 // band off-diagonal
  double* Bsv = Esv + N;                                 // reflection coefficients
  double* lam = Bsv + N;                                 // nc
  double* Tc = lam + nc;                                 // nc x nc
  double* Zs = Tc + static_cast<size_t>(nc) * nc;        // nc x nc
  double* Wt = Zs + static_cast<size_t>(nc) * nc;        // nc x N
  double* lu = Wt + static_cast<size_t>(nc) * N;         // 4 N per vector
  unsigned char* piv = reinterpret_cast<unsigned char*>(lu + 4 * static_cast<size_t>(nc) * N);
  for (int i = tid; i < N; i += blockDim.x) {
    Dsv[i] = sh.d[i];
    Esv[i] = sh.e[i];
    Bsv[i] = sh.beta[i];
  }
  if (tid == 0) {
    double lo = 1e300, hi = -1e300;
    for (int i = 0; i < N; ++i) {
      const double r = ((i > 0) ? fabs(sh.e[i - 1]) : 0.0) + ((i + 1 < N) ? fabs(sh.e[i]) : 0.0);
      lo = fmin(lo, sh.d[i] - r);
      hi = fmax(hi, sh.d[i] + r);
    }
    const double pad = 1e-12 * fmax(fabs(lo), fabs(hi)) + 1e-300;
    s_lo = lo - pad;
    s_hi = hi + pad;
  }
  __syncthreads();
  const double tiny = 2.220446049250313e-16 * fmax(fabs(s_lo), fabs(s_hi)) + 1e-300;
  for (int t = tid; t < nc; t += blockDim.x) {
    lam[t] = band_bisect(sh.d, sh.e, N, t, s_lo, s_hi, tiny);
    band_inverse_iteration(sh.d, sh.e, N, lam[t], tiny, static_cast<unsigned>(t + 1), lu + 4 * static_cast<size_t>(t) * N,
                           piv + static_cast<size_t>(t) * N, X + static_cast<size_t>(t) * N);
  }
  __syncthreads();
  // modified Gram-Schmidt, two passes per vector
  for (int j = 0; j < nc; ++j) {
    double* xj = X + static_cast<size_t>(j) * N;
    for (int pass = 0; pass < 2; ++pass) {
      for (int i = 0; i < j; ++i) {
        const double* xi = X + static_cast<size_t>(i) * N;
        double part = 0.0;
        for (int k = tid; k < N; k += blockDim.x) part += xi[k] * xj[k];
        const double dot = block_sum(part, sh.red);
        for (int k = tid; k < N; k += blockDim.x) xj[k] -= dot * xi[k];
        __syncthreads();
      }
    }
    double part = 0.0;
    for (int k = tid; k < N; k += blockDim.x) part += xj[k] * xj[k];
    const double nn = block_sum(part, sh.red);
    const double inv = (nn > 0.0) ? 1.0 / sqrt(nn) : 0.0;
    for (int k = tid; k < N; k += blockDim.x) xj[k] *= inv;
    __syncthreads();
  }
  // Rayleigh-Ritz with the band inside span(X)
  for (size_t f = tid; f < static_cast<size_t>(nc) * N; f += blockDim.x) {
    const int j = static_cast<int>(f / N), k = static_cast<int>(f - static_cast<size_t>(j) * N);
    const double* xj = X + static_cast<size_t>(j) * N;
    double v = Dsv[k] * xj[k];
    if (k > 0) v += Esv[k - 1] * xj[k - 1];
    if (k + 1 < N) v += Esv[k] * xj[k + 1];
    Wt[f] = v;
  }
  __syncthreads();
  for (int p = wave; p < nc * nc; p += kEigThreads / kWave) {
    const int i = p / nc, j = p - i * nc;
    const double* xi = X + static_cast<size_t>(i) * N;
    const double* wj = Wt + static_cast<size_t>(j) * N;
    double acc = 0.0;
    for (int k = lane; k < N; k += kWave) acc += xi[k] * wj[k];
    acc = wave_sum(acc);
    if (lane == 0) Tc[p] = acc;
  }
  __syncthreads();
  for (int p = tid; p < nc * nc; p += blockDim.x) {
    const int i = p / nc, j = p - i * nc;
    if (i < j) {
      const double m = 0.5 * (Tc[i * nc + j] + Tc[j * nc + i]);
      Tc[i * nc + j] = m;
      Tc[j * nc + i] = m;
    }
  }
  __syncthreads();
  wg_tridiagonalize(Tc, nc, nc, sh);
  const bool ok = wg_band_qr(Zs, nc, nc, sh);
  wg_rank_ascending(sh.d, nc, s_perm);
  wg_back_transform(Tc, nc, nc, Zs, nc, s_perm, nc, sh);
  for (int a = tid; a < nc; a += blockDim.x) lam[a] = sh.d[s_perm[a]];
  for (size_t f = tid; f < static_cast<size_t>(nc) * N; f += blockDim.x) {
    const int a = static_cast<int>(f / N), k = static_cast<int>(f - static_cast<size_t>(a) * N);
    const double* q = Zs + static_cast<size_t>(s_perm[a]) * nc;
    double acc = 0.0;
    for (int i = 0; i < nc; ++i) acc += q[i] * X[static_cast<size_t>(i) * N + k];
    Wt[f] = acc;
  }
  __syncthreads();
  for (size_t f = tid; f < static_cast<size_t>(nc) * N; f += blockDim.x) X[f] = Wt[f];
  for (int i = tid; i < N; i += blockDim.x) sh.beta[i] = Bsv[i];
  for (int a = tid; a < nc; a += blockDim.x) s_perm[a] = a;
  __syncthreads();
  if (STREAMED) wg_back_transform_streamed(A, N, N, X, N, s_perm, nc, sh);
  else wg_back_transform(A, N, N, X, N, s_perm, nc, sh);
  for (int a = tid; a < N; a += blockDim.x) {
    perm[static_cast<size_t>(c) * N + a] = a;
    Eraw[static_cast<size_t>(c) * N + a] = (a < nc) ? lam[a] : 0.0;
  }
  if (tid == 0) status[c] = ok ? 0 : 1;
}

// Canonical basis, signs and truncation.  Reads level a (< ncols) as column
// perm[a] of Z; writes V[a][x] (a < n) row-major, E[g][a] (padded to NP), gs[g].
// Workspace per matrix: G and its eigenvectors (ncols^2 each), and ncols*N
// doubles holding the cluster's old vectors.
__global__ __launch_bounds__(kEigThreads) void k_canon(const double* __restrict__ Z, const int* __restrict__ perm,
                                                       const double* __restrict__ Eraw, int N, int ncols, int n,
                                                       int NP, double tol, int g0, double* __restrict__ Vout,
                                                       double* __restrict__ Etab, int* __restrict__ gstab,
                                                       double* __restrict__ ws, int* __restrict__ status) {
  __shared__ EigShared sh;
  __shared__ double s_E[kEigMaxN];
  __shared__ int s_cs[kEigMaxN + 1];
  __shared__ int s_ncl;
  __shared__ int s_perm2[kEigMaxN];
  const int c = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid >> 6;
  const double* Zc = Z + static_cast<size_t>(c) * N * N;
  const int* pc = perm + static_cast<size_t>(c) * N;
  double* V = Vout + static_cast<size_t>(c) * ncols * N;   // canonical vectors, ncols rows
  double* G = ws + static_cast<size_t>(c) * (2 * static_cast<size_t>(ncols) * ncols + static_cast<size_t>(ncols) * N);
  double* ZG = G + static_cast<size_t>(ncols) * ncols;
  double* old = ZG + static_cast<size_t>(ncols) * ncols;
  for (int a = tid; a < ncols; a += blockDim.x) s_E[a] = Eraw[static_cast<size_t>(c) * N + a];
  for (size_t f = tid; f < static_cast<size_t>(ncols) * N; f += blockDim.x) {
    const int a = static_cast<int>(f / N), x = static_cast<int>(f - static_cast<size_t>(a) * N);
    V[f] = Zc[static_cast<size_t>(pc[a]) * N + x];
  }
  __syncthreads();
  if (tid == 0) {
    int k = 0;
    s_cs[k++] = 0;
    for (int a = 1; a < ncols; ++a)
      if (s_E[a] - s_E[a - 1] >= tol) s_cs[k++] = a;
    s_cs[k] = ncols;
    s_ncl = k;
  }
  __syncthreads();
  const int ncl = s_ncl;
  bool ok = true;
  for (int q = 0; q < ncl; ++q) {
    const int a0 = s_cs[q], a1 = s_cs[q + 1], cs = a1 - a0;
    if (cs < 2) continue;
    // G[i][j] = sum_x x V[a0+i][x] V[a0+j][x]
    for (int p = wave; p < cs * cs; p += kEigThreads / kWave) {
      const int i = p / cs, j = p - i * cs;
      const double* vi = V + static_cast<size_t>(a0 + i) * N;
      const double* vj = V + static_cast<size_t>(a0 + j) * N;
      double acc = 0.0;
      for (int x = lane; x < N; x += kWave) acc += static_cast<double>(x) * vi[x] * vj[x];
      acc = wave_sum(acc);
      if (lane == 0) G[i * cs + j] = acc;
    }
    __syncthreads();
    wg_tridiagonalize(G, cs, cs, sh);
    ok = wg_band_qr(ZG, cs, cs, sh) && ok;
    wg_rank_ascending(sh.d, cs, s_perm2);
    wg_back_transform(G, cs, cs, ZG, cs, s_perm2, cs, sh);
    // rotate: new_j = sum_i Q[i][j] old_i, Q[i][j] = ZG[perm2[j]][i]
    for (size_t f = tid; f < static_cast<size_t>(cs) * N; f += blockDim.x) old[f] = V[static_cast<size_t>(a0) * N + f];
    __syncthreads();
    for (size_t f = tid; f < static_cast<size_t>(cs) * N; f += blockDim.x) {
      const int j = static_cast<int>(f / N), x = static_cast<int>(f - static_cast<size_t>(j) * N);
      const double* qj = ZG + static_cast<size_t>(s_perm2[j]) * cs;
      double acc = 0.0;
      for (int i = 0; i < cs; ++i) acc += qj[i] * old[static_cast<size_t>(i) * N + x];
      V[static_cast<size_t>(a0 + j) * N + x] = acc;
    }
    for (int j = tid; j < cs; j += blockDim.x) {
      const double* qj = ZG + static_cast<size_t>(s_perm2[j]) * cs;
      double e = 0.0;
      for (int i = 0; i < cs; ++i) e += qj[i] * qj[i] * s_E[a0 + i];
      sh.w[j] = e;
    }
    __syncthreads();
    for (int j = tid; j < cs; j += blockDim.x) s_E[a0 + j] = sh.w[j];
    __syncthreads();
  }
  // signs: first entry within 1e-9 of the largest magnitude is made positive
  for (int a = wave; a < n; a += kEigThreads / kWave) {
    double* va = V + static_cast<size_t>(a) * N;
    double mx = 0.0;
    for (int x = lane; x < N; x += kWave) mx = fmax(mx, fabs(va[x]));
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, kWave));
    int first = N;
    for (int x = lane; x < N; x += kWave)
      if (fabs(va[x]) >= (1.0 - 1e-9) * mx) {
        first = x;
        break;
      }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) first = min(first, __shfl_xor(first, o, kWave));
    if (first >= N) first = 0;   // no entry qualified (non-finite vector): stay in range
    const bool flip = va[first] < 0.0;
    if (flip)
      for (int x = lane; x < N; x += kWave) va[x] = -va[x];
  }
  __syncthreads();
  const int g = g0 + c;
  for (int a = tid; a < NP; a += blockDim.x) Etab[static_cast<size_t>(g) * NP + a] = (a < n) ? s_E[a] : 0.0;
  if (tid == 0) {
    gstab[g] = min(n, ncl > 1 ? s_cs[1] : ncols);
    if (!ok) status[c] |= 2;
  }
}

// C[b][i][j] (+)= sum_x w(x) A[i][x] B[j][x] for rows i < ra, j < rb: 64x64 tile
// per workgroup, x staged through LDS in chunks of 32, 16x16x4 FP64 MFMAs.
// wmode 0: w = 1; 1: w = sz of qubit (bz % nq) (operands of batch bz / nq); 2: w = x;
// 3: w = wvec[x]; 4: w = wvec[(bz % nq) K + x] (channel weights; operands of batch bz / nq).  bdiv > 1: operand B of batch bz is B + sB * (bz / bdiv);
// adiv > 1: operand A of batch bz is A + sA * (bz / adiv).
// sub_eye: subtract the identity (stores O - I).
struct GemmArgs {
  const double* A;
  const double* B;
  double* C;
  int64_t sA, sB, sC;
  int ra, rb, K, lda, ldb, ldc;
  int wmode, nq, sub_eye;
  int ksplit = 1;   // > 1: blockIdx.z = batch * ksplit + part, each part sums x in its
  int kspan = 0;    // span of kspan and writes a compact [ra][rb] partial at C + sC * blockIdx.z
  const double* wvec = nullptr;
  int bdiv = 1;
  int adiv = 1;
  const int* bmask = nullptr;   // non-null: batch bz is computed only where bmask[bz] != 0
};

__global__ __launch_bounds__(256) void k_gemm_f64(GemmArgs p) {
  __shared__ double As[64][33];
  __shared__ double Bs[64][33];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int bz = blockIdx.z / p.ksplit;
  if (p.bmask && !p.bmask[bz]) return;
  const int kpart = blockIdx.z - bz * p.ksplit;
  const int xbeg = (p.ksplit > 1) ? kpart * p.kspan : 0;
  const int xend = (p.ksplit > 1) ? min(p.K, xbeg + p.kspan) : p.K;
  const int opb = (p.wmode == 1 || p.wmode == 4) ? bz / p.nq : bz;
  const int qubit = (p.wmode == 1 || p.wmode == 4) ? bz % p.nq : 0;
  const double* A = p.A + p.sA * ((p.adiv > 1) ? bz / p.adiv : opb);
  const double* B = p.B + p.sB * ((p.bdiv > 1) ? bz / p.bdiv : opb);
  double* C = p.C + p.sC * blockIdx.z;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
  d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  for (int x0 = xbeg; x0 < xend; x0 += 32) {
    for (int f = tid; f < 64 * 32; f += 256) {
      const int r = f >> 5, k = f & 31, x = x0 + k;
      double w = 1.0;
      if (p.wmode == 1) w = ((x >> qubit) & 1) ? -1.0 : 1.0;
      else if (p.wmode == 2) w = static_cast<double>(x);
      else if (p.wmode == 3 && x < xend) w = p.wvec[x];
      else if (p.wmode == 4 && x < xend) w = p.wvec[static_cast<size_t>(qubit) * p.K + x];
      As[r][k] = (i0 + r < p.ra && x < xend) ? w * A[static_cast<size_t>(i0 + r) * p.lda + x] : 0.0;
      Bs[r][k] = (j0 + r < p.rb && x < xend) ? B[static_cast<size_t>(j0 + r) * p.ldb + x] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      const int k = 4 * kk + (lane >> 4);
      double av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = As[wi + 16 * a + (lane & 15)][k];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = Bs[wj + 16 * b + (lane & 15)][k];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
  // FP64 16x16x4 accumulator: lane l, element e holds row l/16 + 4e, column l%16
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = i0 + wi + 16 * a + (lane >> 4) + 4 * e;
        const int j = j0 + wj + 16 * b + (lane & 15);
        if (i < p.ra && j < p.rb) {
          double v = acc[a][b][e];
          if (p.ksplit > 1) {
            C[static_cast<size_t>(i) * p.rb + j] = v;   // compact partial
          } else {
            if (p.sub_eye && i == j) v -= 1.0;
            C[static_cast<size_t>(i) * p.ldc + j] = v;
          }
        }
      }
}

// out[b][i][j] (ld ldo) = sum over parts of partial[b * ksplit + part][i][j] (- I if sub_eye).
__global__ void k_splitk_reduce(const double* __restrict__ part, int ksplit, int ra, int rb, int nbatch,
                                double* __restrict__ out, int64_t s_out, int ldo, int sub_eye) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t per = static_cast<int64_t>(ra) * rb;
  if (idx >= per * nbatch) return;
  const int b = static_cast<int>(idx / per);
  const int64_t e = idx - b * per;
  const int i = static_cast<int>(e / rb), j = static_cast<int>(e - static_cast<int64_t>(i) * rb);
  double acc = 0.0;
  for (int k = 0; k < ksplit; ++k) acc += part[(static_cast<int64_t>(b) * ksplit + k) * per + e];
  if (sub_eye && i == j) acc -= 1.0;
  out[b * s_out + static_cast<int64_t>(i) * ldo + j] = acc;
}

// Canonical orthonormal basis of the range of the projector P (n x n, rank k):
// eigenvectors of P diag(1..n) P for its k largest eigenvalues (ascending), each
// with the column sign rule.  Writes k columns into out (column-major, ld n).
__device__ void wg_canonical_range(const double* P, int n, int k, double* K, double* Z, int* perm, double* out,
                                   EigShared& sh) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int f = tid; f < n * n; f += blockDim.x) {
    const int i = f / n, j = f - i * n;
    double acc = 0.0;
    for (int m = 0; m < n; ++m) acc += P[i * n + m] * static_cast<double>(m + 1) * P[m * n + j];
    K[f] = acc;
  }
  __syncthreads();
  wg_tridiagonalize(K, n, n, sh);
  wg_band_qr(Z, n, n, sh);
  wg_rank_ascending(sh.d, n, perm);
  wg_back_transform(K, n, n, Z, n, perm, n, sh);
  for (int q = wave; q < k; q += kEigThreads / kWave) {
    const double* v = Z + static_cast<size_t>(perm[n - k + q]) * n;
    double mx = 0.0;
    for (int x = lane; x < n; x += kWave) mx = fmax(mx, fabs(v[x]));
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, kWave));
    int first = n;
    for (int x = lane; x < n; x += kWave)
      if (fabs(v[x]) >= (1.0 - 1e-9) * mx) {
        first = x;
        break;
      }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) first = min(first, __shfl_xor(first, o, kWave));
    if (first >= n) first = 0;   // no entry qualified (non-finite vector): stay in range
    const double sgn = (v[first] < 0.0) ? -1.0 : 1.0;
    for (int x = lane; x < n; x += kWave) out[static_cast<size_t>(q) * n + x] = sgn * v[x];
  }
  __syncthreads();
}

// Polar factor of the truncated overlap M = O (stored as Delta = M - I in dlt):
// M^T M = U S^2 U^T, polar(M) = sum_{s_a > tau} (M u_a / s_a) u_a^T.  Directions
// with s_a <= tau = 1e-4 (lost by the truncation) are mapped onto the left
// directions that the others leave free, both in the canonical basis of
// wg_canonical_range, so the factor stays orthogonal.  Leakage 1 - min S^2.
__global__ __launch_bounds__(kEigThreads) void k_polar(double* dlt, int NP, int n, int g0, double* leak,
                                                       double* ws, int* status) {
  __shared__ EigShared sh;
  __shared__ int s_perm[kEigMaxN];
  __shared__ int s_bad[kEigMaxN];
  __shared__ int s_nbad;
  const int c = blockIdx.x;
  const int g = g0 + c;
  const int tid = threadIdx.x;
  const size_t nn = static_cast<size_t>(n) * n;
  double* D = dlt + static_cast<size_t>(g) * NP * NP;
  double* Mm = ws + static_cast<size_t>(c) * 9 * nn;   // M
  double* Gm = Mm + nn;                                 // M^T M, then reflectors
  double* U = Gm + nn;                                  // eigenvectors (column-major)
  double* T = U + nn;                                   // M U S^-1 (row-major [i][a])
  double* P = T + nn;                                   // projector scratch
  double* K = P + nn;                                   // canonical-range scratch
  double* ZK = K + nn;
  double* Rb = ZK + nn;                                 // right lost basis (column-major)
  double* Lb = Rb + nn;                                 // left completion (column-major)
  for (size_t f = tid; f < nn; f += blockDim.x) {
    const int i = static_cast<int>(f / n), j = static_cast<int>(f - static_cast<size_t>(i) * n);
    Mm[f] = D[static_cast<size_t>(i) * NP + j] + (i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  for (size_t f = tid; f < nn; f += blockDim.x) {
    const int i = static_cast<int>(f / n), j = static_cast<int>(f - static_cast<size_t>(i) * n);
    double acc = 0.0;
    for (int k = 0; k < n; ++k) acc += Mm[k * n + i] * Mm[k * n + j];
    Gm[f] = acc;
  }
  __syncthreads();
  wg_tridiagonalize(Gm, n, n, sh);
  const bool ok = wg_band_qr(U, n, n, sh);
  for (int a = tid; a < n; a += blockDim.x) s_perm[a] = a;   // all columns, any order
  __syncthreads();
  wg_back_transform(Gm, n, n, U, n, s_perm, n, sh);
  const double tau2 = 1e-8;   // tau^2
  if (tid == 0) {
    int k = 0;
    for (int a = 0; a < n; ++a)
      if (!(sh.d[a] > tau2)) s_bad[k++] = a;
    s_nbad = k;
  }
  __syncthreads();
  const int nbad = s_nbad;
  double smin = 1e300;
  for (int a = 0; a < n; ++a) smin = fmin(smin, sh.d[a]);
  // T[:, a] = M u_a / s_a for the kept directions, 0 for the lost ones
  for (size_t f = tid; f < nn; f += blockDim.x) {
    const int i = static_cast<int>(f / n), a = static_cast<int>(f - static_cast<size_t>(i) * n);
    double acc = 0.0;
    if (sh.d[a] > tau2) {
      for (int k = 0; k < n; ++k) acc += Mm[i * n + k] * U[static_cast<size_t>(a) * n + k];
      acc /= sqrt(sh.d[a]);
    }
    T[f] = acc;
  }
  __syncthreads();
  if (nbad > 0) {
    // right: projector onto the lost right directions
    for (size_t f = tid; f < nn; f += blockDim.x) {
      const int i = static_cast<int>(f / n), j = static_cast<int>(f - static_cast<size_t>(i) * n);
      double acc = 0.0;
      for (int q = 0; q < nbad; ++q) {
        const double* u = U + static_cast<size_t>(s_bad[q]) * n;
        acc += u[i] * u[j];
      }
      P[f] = acc;
    }
    __syncthreads();
    wg_canonical_range(P, n, nbad, K, ZK, s_perm, Rb, sh);
    // left: complement of the kept left directions
    for (size_t f = tid; f < nn; f += blockDim.x) {
      const int i = static_cast<int>(f / n), j = static_cast<int>(f - static_cast<size_t>(i) * n);
      double acc = (i == j) ? 1.0 : 0.0;
      for (int a = 0; a < n; ++a) acc -= T[i * n + a] * T[j * n + a];
      P[f] = acc;
    }
    __syncthreads();
    wg_canonical_range(P, n, nbad, K, ZK, s_perm, Lb, sh);
  }
  // the factor, into Mm (M is no longer needed)
  for (size_t f = tid; f < nn; f += blockDim.x) {
    const int i = static_cast<int>(f / n), j = static_cast<int>(f - static_cast<size_t>(i) * n);
    double acc = 0.0;
    for (int a = 0; a < n; ++a) acc += T[i * n + a] * U[static_cast<size_t>(a) * n + j];
    for (int q = 0; q < nbad; ++q) acc += Lb[static_cast<size_t>(q) * n + i] * Rb[static_cast<size_t>(q) * n + j];
    Mm[f] = acc;
  }
  __syncthreads();
  // One Newton-Schulz step, O <- O - O (O^T O - I) / 2: the kept directions come from
  // the eigenvectors of M^T M, so with singular values near tau the factor is orthogonal
  // only to about eps / tau^2; the step squares that error.
  for (size_t f = tid; f < nn; f += blockDim.x) {
    const int i = static_cast<int>(f / n), j = static_cast<int>(f - static_cast<size_t>(i) * n);
    double acc = 0.0;
    for (int k = 0; k < n; ++k) acc += Mm[k * n + i] * Mm[k * n + j];
    P[f] = acc - (i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  for (size_t f = tid; f < nn; f += blockDim.x) {
    const int i = static_cast<int>(f / n), j = static_cast<int>(f - static_cast<size_t>(i) * n);
    double acc = 0.0;
    for (int k = 0; k < n; ++k) acc += Mm[i * n + k] * P[k * n + j];
    D[static_cast<size_t>(i) * NP + j] = (Mm[f] - 0.5 * acc) - (i == j ? 1.0 : 0.0);
  }
  if (tid == 0) {
    leak[g] = 1.0 - smin;
    if (!ok) status[c] |= 4;
  }
}

// Full spectrum: M is orthogonal up to rounding; leakage from column norms.
__global__ void k_leak_columns(const double* dlt, int NP, int n, int g0, int count, double* leak) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= count) return;
  const int g = g0 + c;
  const double* D = dlt + static_cast<size_t>(g) * NP * NP;
  double worst = 0.0;
  for (int b = 0; b < n; ++b) {
    double s = 0.0;
    for (int a = 0; a < n; ++a) {
      const double o = D[static_cast<size_t>(a) * NP + b] + (a == b ? 1.0 : 0.0);
      s += o * o;
    }
    worst = fmax(worst, 1.0 - s);
  }
  leak[g] = worst;
}

__device__ double gamma_ohmic(double w, double eta, double wc, double T) {
  if (w == 0.0) return 2.0 * M_PI * eta * T;
  return 2.0 * M_PI * eta * w * exp(-fabs(w) / wc) / (-expm1(-w / T));
}

// R[g][i][b][a] and zdiag[g][i][b] from z (row-major [g-local][i][a][b], ld n); channel i's
// rate has cutoff wc[i].
__global__ void k_rates(const double* __restrict__ z, const double* __restrict__ E, int n, int NP, int nq, int g0,
                        int count, double eta, const double* __restrict__ wc, double T, double* __restrict__ R,
                        double* __restrict__ zdiag) {
  const int64_t per = static_cast<int64_t>(nq) * NP * NP;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= per * count) return;
  const int c = static_cast<int>(idx / per);
  int64_t r = idx - c * per;
  const int i = static_cast<int>(r / (static_cast<int64_t>(NP) * NP));
  r -= static_cast<int64_t>(i) * NP * NP;
  const int b = static_cast<int>(r / NP), a = static_cast<int>(r - static_cast<int64_t>(b) * NP);
  const int g = g0 + c;
  double val = 0.0;
  if (a < n && b < n) {
    const double zab = z[((static_cast<size_t>(c) * nq + i) * n + a) * n + b];
    const double w = (a == b) ? 0.0 : E[static_cast<size_t>(g) * NP + b] - E[static_cast<size_t>(g) * NP + a];
    val = gamma_ohmic(w, eta, wc[i], T) * zab * zab;
    if (a == b) zdiag[(static_cast<size_t>(g) * nq + i) * NP + b] = zab;
  } else if (a == b) {
    zdiag[(static_cast<size_t>(g) * nq + i) * NP + b] = 0.0;
  }
  R[((static_cast<size_t>(g) * nq + i) * NP + b) * NP + a] = val;
}

// Initial state: ground state of H(s_0) (row 0 of V0) in the grid-1 basis.
__global__ void k_cinit(const double* __restrict__ V0, const double* __restrict__ V1, int N, int n, int NP,
                        double* __restrict__ cinit, double* __restrict__ leak) {
  __shared__ double s_c[kEigMaxN];
  __shared__ double red[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int a = wave; a < n; a += 4) {
    double acc = 0.0;
    for (int x = lane; x < N; x += 64) acc += V1[static_cast<size_t>(a) * N + x] * V0[x];
    acc = wave_sum(acc);
    if (lane == 0) s_c[a] = acc;
  }
  __syncthreads();
  double part = 0.0;
  for (int a = tid; a < n; a += blockDim.x) part += s_c[a] * s_c[a];
  part = wave_sum(part);
  if (lane == 0) red[wave] = part;
  __syncthreads();
  const double nn = red[0] + red[1] + red[2] + red[3];
  const double inv = 1.0 / sqrt(nn);
  for (int a = tid; a < NP; a += blockDim.x) cinit[a] = (a < n) ? s_c[a] * inv : 0.0;
  if (tid == 0) leak[1] = 1.0 - nn;
}

// ---- Lamb shift (Sec. II eq. ME2-H) -------------------------------------------------
// H_LS = sum_i sum_w S(w) A_i,w^dag A_i,w is diagonal in the eigenbasis: level b gets
// sum_i [sum_{a != b} S(e_b - e_a) z_ab^2 + S(0) z_bb^2].  S(w) = (1/2pi) P int gamma(w') /
// (w - w') dw' = (1/2pi) int_0^inf [gamma(w - u) - gamma(w + u)] / u du, tabulated once per
// precompute on nodes w_k = W sinh(sigma x_k) / sinh(sigma), x_k uniform in [-1, 1] (fine
// near w = 0, where S has a w log|w| term from the kink of gamma), by composite 16-point
// Gauss-Legendre panels that start at the kink u = |w| and double in width up to wc / 2.
constexpr int kLambNodes = 16385;
constexpr double kLambSigma = 10.0;

struct LambTable {
  const double* S;   // [tables][kLambNodes], one table per distinct channel cutoff
  double W;          // largest |w| covered
  const int* tix;    // [channels] table of each channel (null: table 0)
};

// The S table of jump channel i.
__device__ inline LambTable lamb_channel(const LambTable& t, int i) {
  return LambTable{t.S + static_cast<size_t>(t.tix ? t.tix[i] : 0) * kLambNodes, t.W, nullptr};
}

__device__ double lamb_integrand_panel(double w, double lo, double hi, double eta, double wc, double T,
                                       const double* __restrict__ glx, const double* __restrict__ glw) {
  const double c = 0.5 * (hi + lo), h = 0.5 * (hi - lo);
  double s = 0.0;
  for (int q = 0; q < 16; ++q) {
    const double u = c + h * glx[q];
    s += glw[q] * (gamma_ohmic(w - u, eta, wc, T) - gamma_ohmic(w + u, eta, wc, T)) / u;
  }
  return h * s;
}

__global__ void k_lamb_table(double W, double eta, double wc, double T, const double* __restrict__ glx,
                             const double* __restrict__ glw, double* __restrict__ S) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= kLambNodes) return;
  const double x = -1.0 + 2.0 * k / (kLambNodes - 1);
  const double w = W * sinh(kLambSigma * x) / sinh(kLambSigma);
  const double a = fabs(w);
  const double h0 = fmin(T, wc) / 8.0, hmax = 0.5 * wc;
  const double U = a + 40.0 * T + 60.0 * wc;
  double sum = 0.0, lo = a, hw = h0;
  while (lo < U) {
    const double hi = fmin(lo + hw, U);
    sum += lamb_integrand_panel(w, lo, hi, eta, wc, T, glx, glw);
    lo = hi;
    hw = fmin(2.0 * hw, hmax);
  }
  double hi = a;
  hw = h0;
  while (hi > 0.0) {
    const double l2 = fmax(hi - hw, 0.0);
    sum += lamb_integrand_panel(w, l2, hi, eta, wc, T, glx, glw);
    hi = l2;
    hw = fmin(2.0 * hw, hmax);
  }
  S[k] = sum / (2.0 * M_PI);
}

// S(w) by cubic Lagrange interpolation in x (|w| <= W).
__device__ double lamb_S(const LambTable& t, double w) {
  const double x = asinh(w * sinh(kLambSigma) / t.W) / kLambSigma;
  const double dx = 2.0 / (kLambNodes - 1);
  int k = static_cast<int>(floor((x + 1.0) / dx)) - 1;
  k = min(max(k, 0), kLambNodes - 4);
  const double u = (x + 1.0) / dx - k;   // position in node units from node k
  const double l0 = -(u - 1.0) * (u - 2.0) * (u - 3.0) / 6.0;
  const double l1 = u * (u - 2.0) * (u - 3.0) / 2.0;
  const double l2 = -u * (u - 1.0) * (u - 3.0) / 2.0;
  const double l3 = u * (u - 1.0) * (u - 2.0) / 6.0;
  return l0 * t.S[k] + l1 * t.S[k + 1] + l2 * t.S[k + 2] + l3 * t.S[k + 3];
}

// shift[g][b] from z (chunk-local [c][i][a][b], ld n) for grid points zg0 .. zg0 + zcnt - 1.
// dS/dw of the interpolant: the cubic's derivative in x times dx/dw.
__device__ double lamb_dS(const LambTable& t, double w) {
  const double sg = sinh(kLambSigma) / t.W;
  const double y = w * sg;
  const double x = asinh(y) / kLambSigma;
  const double dxdw = sg / (kLambSigma * sqrt(1.0 + y * y));
  const double dx = 2.0 / (kLambNodes - 1);
  int k = static_cast<int>(floor((x + 1.0) / dx)) - 1;
  k = min(max(k, 0), kLambNodes - 4);
  const double u = (x + 1.0) / dx - k;
  const double d0 = -((u - 2.0) * (u - 3.0) + (u - 1.0) * (u - 3.0) + (u - 1.0) * (u - 2.0)) / 6.0;
  const double d1 = ((u - 2.0) * (u - 3.0) + u * (u - 3.0) + u * (u - 2.0)) / 2.0;
  const double d2 = -((u - 1.0) * (u - 3.0) + u * (u - 3.0) + u * (u - 1.0)) / 2.0;
  const double d3 = ((u - 1.0) * (u - 2.0) + u * (u - 2.0) + u * (u - 1.0)) / 6.0;
  return (d0 * t.S[k] + d1 * t.S[k + 1] + d2 * t.S[k + 2] + d3 * t.S[k + 3]) / dx * dxdw;
}

// Derivative of the Lamb shift of level b (k_lamb_shift's sum) for both directions:
// dshift[g][dir][b] = sum_i [sum_{a != b} (S'(w_ab) (de_b - de_a) z_ab^2 + 2 S(w_ab) z_ab dz_ab)
//                            + 2 S(0) z_bb dz_bb],  w_ab = e_b - e_a, dz_i = -(Q + Q^T).
__global__ void k_lamb_dshift(const double* __restrict__ z, const double* __restrict__ Q,
                              const double* __restrict__ E, const double* __restrict__ dE, int n, int NP, int nq,
                              int zg0, int zcnt, LambTable tab, double* __restrict__ dshift) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<int64_t>(zcnt) * 2 * NP) return;
  const int c = static_cast<int>(idx / (2 * NP));
  const int dir = static_cast<int>((idx / NP) & 1);
  const int b = static_cast<int>(idx % NP);
  const int g = zg0 + c;
  const size_t gd = static_cast<size_t>(g) * 2 + dir;
  double acc = 0.0;
  if (b < n) {
    const double* e = E + static_cast<size_t>(g) * NP;
    const double* de = dE + gd * NP;
    for (int i = 0; i < nq; ++i) {
      const LambTable ti = lamb_channel(tab, i);
      const double s0 = lamb_S(ti, 0.0);
      const double* zi = z + (static_cast<size_t>(c) * nq + i) * n * n;
      const double* Qi = Q + ((static_cast<size_t>(dir) * zcnt + c) * nq + i) * n * n;
      for (int a = 0; a < n; ++a) {
        const double zab = zi[a * n + b];
        const double dz = -(Qi[a * n + b] + Qi[b * n + a]);
        if (a == b) {
          acc += 2.0 * s0 * zab * dz;
        } else {
          const double w = e[b] - e[a];
          acc += lamb_dS(ti, w) * (de[b] - de[a]) * zab * zab + 2.0 * lamb_S(ti, w) * zab * dz;
        }
      }
    }
  }
  dshift[gd * NP + b] = acc;
}

__global__ void k_lamb_shift(const double* __restrict__ z, const double* __restrict__ E, int n, int NP, int nq,
                             int zg0, int zcnt, LambTable tab, double* __restrict__ shift) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<int64_t>(zcnt) * NP) return;
  const int c = static_cast<int>(idx / NP), b = static_cast<int>(idx % NP);
  const int g = zg0 + c;
  double acc = 0.0;
  if (b < n) {
    const double* e = E + static_cast<size_t>(g) * NP;
    for (int i = 0; i < nq; ++i) {
      const LambTable ti = lamb_channel(tab, i);
      const double s0 = lamb_S(ti, 0.0);
      const double* zi = z + (static_cast<size_t>(c) * nq + i) * n * n;
      for (int a = 0; a < n; ++a) {
        const double zab = zi[a * n + b];
        acc += ((a == b) ? s0 : lamb_S(ti, e[b] - e[a])) * zab * zab;
      }
    }
  }
  shift[static_cast<size_t>(g) * NP + b] = acc;
}

// ---- derivative tables of the gradient (full spectrum, n = 2^n_qubits) ----------
// Directions: 0 = A(s_g) (operator H_X = -sum_i sx_i), 1 = B(s_g) (operator
// diag(e_Z)).  First-order perturbation theory of the symmetric eigenproblem:
// de_a = <a|H'|a>, dv_b = sum_a v_a X_ab with X_ab = <a|H'|b> / (e_b - e_a) for
// levels in different clusters and 0 inside a cluster (the canonical in-cluster
// basis is held fixed), so X is antisymmetric and dz_i = z_i X - X z_i.

// Y[c][k][b][x] = (O_k v_b)[x] for channel operators O_k = diag(wz_k) + sum_a cx[k][a] sx_a
// (sx_a v)[x] = v[x ^ 2^a], for the n rows of cnt grid points.
__global__ void k_channel_rows(const double* __restrict__ V, int64_t vstride, int N, int nq, int n, int cnt,
                               int nch, const double* __restrict__ wz, const double* __restrict__ cx,
                               double* __restrict__ Y) {
  const int64_t per = static_cast<int64_t>(n) * N;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= per * nch * cnt) return;
  const int ck = static_cast<int>(idx / per);
  const int c = ck / nch, k = ck - c * nch;
  const int64_t r = idx - ck * per;
  const int b = static_cast<int>(r / N), x = static_cast<int>(r - static_cast<int64_t>(b) * N);
  const double* v = V + c * vstride + static_cast<int64_t>(b) * N;
  double acc = wz[static_cast<size_t>(k) * N + x] * v[x];
  for (int a = 0; a < nq; ++a) {
    const double w = cx[k * nq + a];
    if (w != 0.0) acc += w * v[x ^ (1 << a)];
  }
  Y[idx] = acc;
}

// W[c][b][x] = (H_X v_b)[x] = -sum_i v_b[x ^ 2^i] for the n rows of cnt grid points.
__global__ void k_hx_rows(const double* __restrict__ V, int64_t vstride, int N, int nq, int n, int cnt,
                          double* __restrict__ W) {
  const int64_t per = static_cast<int64_t>(n) * N;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= per * cnt) return;
  const int c = static_cast<int>(idx / per);
  const int64_t r = idx - c * per;
  const int b = static_cast<int>(r / N), x = static_cast<int>(r - static_cast<int64_t>(b) * N);
  const double* v = V + c * vstride + static_cast<int64_t>(b) * N;
  double acc = 0.0;
  for (int i = 0; i < nq; ++i) acc -= v[x ^ (1 << i)];
  W[idx] = acc;
}

// X[g][dir] (NP x NP, zero padded) and de[g][dir] from Hd[c][dir] = V H' V^T (n x n).
__global__ void k_xmat(const double* __restrict__ Hd, int n, int NP, const double* __restrict__ E, int g0,
                       double tol, double* __restrict__ Xd, double* __restrict__ dE) {
  __shared__ int cl[256];
  const int c = blockIdx.x, dir = blockIdx.y, g = g0 + c;
  const double* e = E + static_cast<size_t>(g) * NP;
  if (threadIdx.x == 0) {
    int id = 0;
    cl[0] = 0;
    for (int a = 1; a < n; ++a) {
      if (e[a] - e[a - 1] >= tol) ++id;
      cl[a] = id;
    }
  }
  __syncthreads();
  const double* H = Hd + (static_cast<size_t>(c) * 2 + dir) * n * n;
  double* X = Xd + (static_cast<size_t>(g) * 2 + dir) * NP * NP;
  for (int f = threadIdx.x; f < NP * NP; f += blockDim.x) {
    const int x = f / NP, y = f - x * NP;
    double v = 0.0;
    if (x < n && y < n && cl[x] != cl[y]) v = H[x * n + y] / (e[y] - e[x]);
    X[f] = v;
  }
  for (int x = threadIdx.x; x < NP; x += blockDim.x)
    dE[(static_cast<size_t>(g) * 2 + dir) * NP + x] = (x < n) ? H[x * n + x] : 0.0;
}

// d log gamma / d w of the Ohmic rate (w != 0 form; series below |w/T| = 1e-3).
__device__ double dlog_gamma(double w, double wc, double T) {
  const double x = w / T;
  const double h = (fabs(x) < 1e-3) ? 0.5 - x / 12.0 + x * x * x / 720.0 : 1.0 / x - 1.0 / expm1(x);
  const double sg = (w > 0.0) ? 1.0 : ((w < 0.0) ? -1.0 : 0.0);
  return h / T - sg / wc;
}

// Per jump channel i (rate cutoff wc[i]; any fixed coupling operator, so z_i = V^T O_i V
// and dz_i = z_i X - X z_i), from z_i (chunk-local [c][i][a][b], ld n) and
// Q[dir][c][i] = z_i X^T (row products):
// dz_i = -(Q + Q^T);  dzd[g][dir][i][b] = dz_i[b][b];
// dll[g][dir][i][b][a] = d log |l_i,ab| = (1/2) dlog_gamma(w_ab) (de_b - de_a) + dz_ab / z_ab
// for a != b (l = sqrt(gamma(w_ab)) z_ab, the b -> a operator), 0 on the diagonal;
// dGam[g][dir][b] = d Gamma_b = sum_i [sum_{a != b} dR_i,ab + 2 gamma(0) z_bb dz_bb].
__global__ void k_dtables(const double* __restrict__ z, const double* __restrict__ Q, const double* __restrict__ E,
                          const double* __restrict__ dE, int n, int NP, int nq, int zg0, int zcnt, double eta,
                          const double* __restrict__ wc, double T, double* __restrict__ dGam, double* __restrict__ dzd,
                          double* __restrict__ dll) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<int64_t>(zcnt) * 2 * NP) return;
  const int c = static_cast<int>(idx / (2 * NP));
  const int dir = static_cast<int>((idx / NP) & 1);
  const int b = static_cast<int>(idx % NP);
  const int g = zg0 + c;
  const size_t gd = static_cast<size_t>(g) * 2 + dir;
  const double* e = E + static_cast<size_t>(g) * NP;
  const double* de = dE + gd * NP;
  const double g0 = 2.0 * M_PI * eta * T;
  double dG = 0.0;
  for (int i = 0; i < nq; ++i) {
    double* dl = dll + ((gd * nq + i) * NP + b) * NP;
    if (b >= n) {
      for (int a = 0; a < NP; ++a) dl[a] = 0.0;
      dzd[(gd * nq + i) * NP + b] = 0.0;
      continue;
    }
    const double* zi = z + (static_cast<size_t>(c) * nq + i) * n * n;
    const double* Qi = Q + ((static_cast<size_t>(dir) * zcnt + c) * nq + i) * n * n;
    for (int a = 0; a < NP; ++a) {
      if (a >= n) {
        dl[a] = 0.0;
        continue;
      }
      const double zab = zi[a * n + b];
      const double dz = -(Qi[a * n + b] + Qi[b * n + a]);
      if (a == b) {
        dzd[(gd * nq + i) * NP + b] = dz;
        dG += 2.0 * g0 * zab * dz;
        dl[a] = 0.0;
        continue;
      }
      const double w = e[b] - e[a];
      const double gam = gamma_ohmic(w, eta, wc[i], T);
      const double lg = (w == 0.0) ? 0.5 / T : dlog_gamma(w, wc[i], T);
      const double dw = de[b] - de[a];
      dG += gam * (lg * dw * zab * zab + 2.0 * zab * dz);
      dl[a] = (zab != 0.0) ? 0.5 * lg * dw + dz / zab : 0.0;
    }
  }
  dGam[gd * NP + b] = (b < n) ? dG : 0.0;
}

// dcin[dir] = V_1 dv_0: derivative of the initial state (ground state of H(s_0)) in the
// grid-1 basis through grid 0's eigenvectors, dv_0 = sum_y v_y X_0[y][0].
__global__ __launch_bounds__(256) void k_dcinit(const double* __restrict__ V0, const double* __restrict__ V1,
                                                const double* __restrict__ X0, int N, int n, int NP,
                                                double* __restrict__ dcin) {
  __shared__ double u[kEigMaxN];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int dir = 0; dir < 2; ++dir) {
    const double* X = X0 + static_cast<size_t>(dir) * NP * NP;
    for (int x = tid; x < N; x += blockDim.x) {
      double acc = 0.0;
      for (int y = 0; y < n; ++y) acc += X[static_cast<size_t>(y) * NP] * V0[static_cast<size_t>(y) * N + x];
      u[x] = acc;
    }
    __syncthreads();
    for (int a = wave; a < NP; a += 4) {
      double acc = 0.0;
      if (a < n)
        for (int x = lane; x < N; x += 64) acc += V1[static_cast<size_t>(a) * N + x] * u[x];
      acc = wave_sum(acc);
      if (lane == 0) dcin[dir * NP + a] = acc;
    }
    __syncthreads();
  }
}

aqt_status launch_gemm(aqt_ctx* ctx, const GemmArgs& g, int batch) {
  dim3 grid(static_cast<unsigned>((g.rb + 63) / 64), static_cast<unsigned>((g.ra + 63) / 64),
            static_cast<unsigned>(batch));
  hipLaunchKernelGGL(k_gemm_f64, grid, dim3(256), 0, ctx->stream, g);
  AQT_HIP(ctx, hipGetLastError());
  return AQT_OK;
}

// ------------------------------------------------------------------------
// Lowest eigenpairs of large H(s) (2^n_qubits > 1024): Chebyshev-filtered
// subspace iteration on a block of KB vectors with Rayleigh-Ritz steps
// (Zhou and Saad's filtered subspace iteration), each grid point warm-started
// from the Ritz vectors of the grid point before it.  H is applied matrix-free:
// (H v)[x] = -A sum_i v[x ^ 2^i] + B e_Z[x] v[x].  Vectors are rows of length N.
//
// The grid is cut into contiguous chains of grid points, one per block slot.
// The slots iterate in lock step: each kernel below takes the slot as a grid
// dimension, so one launch serves every chain, and a slot whose solve has
// converged (or that has no grid point at this step) is masked out.

constexpr int kHxChunk = 4096;        // x per workgroup of the block product (LDS-resident)
constexpr int kSmallEigMax = 128;     // block size of the subspace iteration, at most
constexpr int kMaxFilterDegree = 256;  // Chebyshev filter degree, at most
constexpr int kMaxChains = 16;         // block slots of the lock-step chains, at most

// Per-slot coefficients of one block product.
struct HxCoef {
  double A, B;                 // H = A H_X + B diag(e_Z)
  double alpha, beta, gamma;   // Y = alpha H X + beta X + gamma Z
  int active;
  int pad;
};

// Y_j = alpha (H X_j) + beta X_j + gamma Z_j for the KB rows j of every active
// slot (a slot is KB*N doubles of each buffer; Z may be null).  One workgroup per
// (row, chunk of CH entries); the chunk is staged in LDS for the flips of its low
// bits, flips of higher bits read the row's other chunks.  Workgroups are handed to
// the 8 XCDs round-robin by index, so the index is decoded such that all chunks of
// a row land on one XCD, one after another, and those reads hit that XCD's L2.
__global__ __launch_bounds__(256) void k_hx_block(const double* __restrict__ X, const double* __restrict__ Zin,
                                                  double* __restrict__ Y, const double* __restrict__ eZ, int nq,
                                                  int KB, const HxCoef* __restrict__ coef) {
  const int N = 1 << nq;
  const int CH = N < kHxChunk ? N : kHxChunk;
  const int nchunk = N / CH;
  const int id = blockIdx.x;
  const int local = id >> 3;                              // rows (KB * slots) are a multiple of 8
  const int r = (local / nchunk) * 8 + (id & 7);          // row over all slots
  const int slot = r / KB;
  const HxCoef cf = coef[slot];
  if (!cf.active) return;
  __shared__ double sx[kHxChunk];
  const int lch = 31 - __clz(CH);
  const size_t row = static_cast<size_t>(r) * N;
  const int x0 = (local % nchunk) * CH;
  const double* v = X + row;
  for (int t = threadIdx.x; t < CH; t += blockDim.x) sx[t] = v[x0 + t];
  __syncthreads();
  const int nlow = nq < lch ? nq : lch;
  const int nfar = nq - nlow;   // flips of bits beyond the chunk
  // four entries per thread and pass, their global loads (e_Z, Z, far flips) issued
  // together, the far flips four bits per batch
  for (int t0 = threadIdx.x; t0 < CH; t0 += 4 * 256) {
    double own[4], fl[4], ez[4], zz[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int t = t0 + 256 * u;
      own[u] = fl[u] = ez[u] = zz[u] = 0.0;
      if (t < CH) {
        const int x = x0 + t;
        ez[u] = eZ[x];
        if (Zin) zz[u] = Zin[row + x];
        own[u] = sx[t];
        double f = 0.0;
#pragma unroll 4
        for (int i = 0; i < nlow; ++i) f += sx[t ^ (1 << i)];
        fl[u] = f;
      }
    }
    for (int k0 = 0; k0 < nfar; k0 += 4) {
      double a[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const int t = t0 + 256 * u, k = k0 + kk;
          a[u][kk] = (t < CH && k < nfar) ? v[(x0 + t) ^ (1 << (lch + k))] : 0.0;
        }
#pragma unroll
      for (int u = 0; u < 4; ++u) fl[u] += (a[u][0] + a[u][1]) + (a[u][2] + a[u][3]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int t = t0 + 256 * u;
      if (t < CH) {
        double out = cf.alpha * (cf.B * ez[u] * own[u] - cf.A * fl[u]) + cf.beta * own[u];
        if (Zin) out += cf.gamma * zz[u];
        Y[row + x0 + t] = out;
      }
    }
  }
}

// Y_j = sum_i C[i][j] X_i (C row-major KB x KB) in every slot (blockIdx.y): the
// block times a small matrix, on FP64 MFMAs.  C is staged in LDS (rows padded by 16
// doubles, so the four k-rows a wavefront reads at once start 128 bytes apart); each
// wavefront owns 16 columns x of the workgroup's 128 and all KB rows j, and reads its
// X columns once, as the B operand.  A masked slot is skipped, or copied (Y = X) when
// copy_masked is set.
constexpr int kCombineCols = 128;   // columns x per workgroup (8 wavefronts x 16)
template <int KB>
__global__ __launch_bounds__(512) void k_combine(const double* __restrict__ X, const double* __restrict__ C,
                                                 double* __restrict__ Y, int N, const int* __restrict__ act,
                                                 int copy_masked) {
  constexpr int LDC = KB + 16;
  constexpr int T = KB / 16;   // 16-row output tiles per wavefront
  const int b = blockIdx.y;
  const size_t off = static_cast<size_t>(b) * KB * N;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int x0 = blockIdx.x * kCombineCols;
  if (!act[b]) {
    if (copy_masked)
      for (int f = tid; f < KB * kCombineCols; f += blockDim.x) {
        const int r = f / kCombineCols, x = x0 + f % kCombineCols;
        if (x < N) Y[off + static_cast<size_t>(r) * N + x] = X[off + static_cast<size_t>(r) * N + x];
      }
    return;
  }
  __shared__ double sC[KB * LDC];
  const double* Cb = C + static_cast<size_t>(b) * KB * KB;
  for (int f = tid; f < KB * KB; f += blockDim.x) sC[(f / KB) * LDC + f % KB] = Cb[f];
  __syncthreads();
  const int xw = x0 + 16 * wave;
  if (xw >= N) return;   // N >= 64 and a power of two: a wavefront's 16 columns are all in range or all out
  const int col = lane & 15, kq = lane >> 4;
  // FP64 16x16x4 operands: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]
  const double* xb = X + off + xw + col;
  d4 acc[T];
#pragma unroll
  for (int t = 0; t < T; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
  for (int i0 = 0; i0 < KB; i0 += 4) {
    const int i = i0 + kq;
    const double bv = xb[static_cast<size_t>(i) * N];
#pragma unroll
    for (int t = 0; t < T; ++t)
      acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(sC[i * LDC + 16 * t + col], bv, acc[t], 0, 0, 0);
  }
  // accumulator: lane l, element e holds row l/16 + 4e, column l%16 of the tile
#pragma unroll
  for (int t = 0; t < T; ++t)
#pragma unroll
    for (int e = 0; e < 4; ++e) Y[off + static_cast<size_t>(16 * t + kq + 4 * e) * N + xw + col] = acc[t][e];
}

// Deterministic start block: entries in [-1, 1) from a counter hash.
__global__ void k_random_block(double* X, int64_t count) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= count) return;
  uint64_t z = static_cast<uint64_t>(idx) * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  X[idx] = static_cast<double>(z >> 11) * 0x1.0p-52 - 1.0;
}

// One workgroup per unmasked slot (blockIdx.x), KB x KB symmetric S (row-major,
// symmetrised here):
//   mode 0 (Rayleigh-Ritz): C = eigenvectors of S as columns, ascending; theta.
//   mode 1 (orthonormalisation of a Gram matrix): with D = diag(S)^(1/2) and
//     D^-1 S D^-1 = U L U^T, C = D^-1 U L^-1/2 so that X C has orthonormal rows;
//   mode 2: the same by Cholesky, D^-1 S D^-1 = L L^T and C = D^-1 L^-T, with
//     mode 1 as the fallback for a small pivot.
// Per slot: S, C KB^2 doubles, theta KB, ws 2 KB^2, status one int (bit 1:
// eigensolver failed, bit 2: non-finite input).
__global__ __launch_bounds__(kEigThreads) void k_small_eig(const double* __restrict__ S, int KB, int mode,
                                                           double* __restrict__ C, double* __restrict__ theta,
                                                           double* __restrict__ ws, int* __restrict__ status,
                                                           const int* __restrict__ act) {
  const int b = blockIdx.x;
  if (!act[b]) return;
  // the matrix lives in LDS (KB <= kSmallEigMax, rows padded to an odd length); ws
  // holds the reflection vectors of the eigen route
  constexpr int LDS_LD = kSmallEigMax + 1;
  __shared__ EigSharedN<kSmallEigMax> sh;
  __shared__ double sA[kSmallEigMax * LDS_LD];
  __shared__ int s_perm[kSmallEigMax];
  __shared__ double s_dinv[kSmallEigMax];
  S += static_cast<size_t>(b) * KB * KB;
  C += static_cast<size_t>(b) * KB * KB;
  theta += static_cast<size_t>(b) * KB;
  ws += static_cast<size_t>(b) * 2 * KB * KB;
  status += b;
  const int lda = KB + 1;
  double* A = sA;
  for (int a = threadIdx.x; a < KB; a += blockDim.x)
    s_dinv[a] = (mode >= 1) ? 1.0 / sqrt(fmax(S[a * KB + a], 1e-300)) : 1.0;
  __syncthreads();
  for (int f = threadIdx.x; f < KB * KB; f += blockDim.x) {
    const int i = f / KB, j = f - i * KB;
    A[i * lda + j] = 0.5 * (S[f] + S[j * KB + i]) * s_dinv[i] * s_dinv[j];
  }
  __syncthreads();
  if (mode == 2) {
    // Cholesky A = L L^T of the column-scaled Gram matrix; C = D^-1 L^-T.  Falls back
    // to the eigen route (mode 1) when a pivot is small (ill-conditioned block).
    bool okc = true;
    for (int k = 0; k < KB; ++k) {
      const double piv = A[k * lda + k];
      if (!(piv > 1e-10)) {
        okc = false;
        break;
      }
      const double lkk = sqrt(piv);
      __syncthreads();
      for (int i = k + threadIdx.x; i < KB; i += blockDim.x) A[i * lda + k] = (i == k) ? lkk : A[i * lda + k] / lkk;
      __syncthreads();
      // trailing update, one thread per row, eight column entries loaded per batch
      for (int i = k + 1 + threadIdx.x; i < KB; i += blockDim.x) {
        const double lik = A[i * lda + k];
        double* Ai = A + i * lda;
        int j = k + 1;
        for (; j + 8 <= i + 1; j += 8) {
          double ajk[8], aij[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            ajk[u] = A[(j + u) * lda + k];
            aij[u] = Ai[j + u];
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) Ai[j + u] = aij[u] - lik * ajk[u];
        }
        for (; j <= i; ++j) Ai[j] -= lik * A[j * lda + k];
      }
      __syncthreads();
    }
    if (okc) {
      // L^-1 in place, columns right to left: with x = L[j+1:, j], column j of the inverse
      // is 1/L_jj on the diagonal and -(1/L_jj) Linv[j+1:, j+1:] x below it
      for (int j = KB - 1; j >= 0; --j) {
        for (int i = j + 1 + threadIdx.x; i < KB; i += blockDim.x) sh.v[i] = A[i * lda + j];
        __syncthreads();
        const double djj = 1.0 / A[j * lda + j];
        for (int i = j + 1 + threadIdx.x; i < KB; i += blockDim.x)
          A[i * lda + j] = -djj * lds_dot(A + i * lda + j + 1, sh.v + j + 1, i - j);
        __syncthreads();
        if (threadIdx.x == 0) A[j * lda + j] = djj;
      }
      __syncthreads();
      // C = D^-1 L^-T
      for (int f = threadIdx.x; f < KB * KB; f += blockDim.x) {
        const int i = f / KB, j = f - i * KB;
        C[f] = (j >= i) ? s_dinv[i] * A[j * lda + i] : 0.0;
      }
      return;
    }
    __syncthreads();
    for (int f = threadIdx.x; f < KB * KB; f += blockDim.x) {
      const int i = f / KB, j = f - i * KB;
      A[i * lda + j] = 0.5 * (S[f] + S[j * KB + i]) * s_dinv[i] * s_dinv[j];
    }
    __syncthreads();
  }
  lds_tridiagonalize(A, KB, lda, sh);
  // the reflection vectors (rows j right of the diagonal) go to ws; the LDS matrix then
  // becomes the reflection product Q (column-major), and the QR rotations are applied to
  // Q itself, which leaves the eigenvectors of the full matrix in LDS
  double* Hv = ws;
  for (int f = threadIdx.x; f < KB * KB; f += blockDim.x) {
    const int i = f / KB, j = f - i * KB;
    Hv[f] = A[i * lda + j];
  }
  __syncthreads();
  lds_form_q(Hv, KB, KB, A, lda, sh);
  const bool ok = wg_band_qr(A, KB, lda, sh, true);
  wg_rank_ascending(sh.d, KB, s_perm);
  double lmax = 0.0, lmin = 1e300;
  bool finite = true;
  for (int a = 0; a < KB; ++a) {
    finite = finite && (sh.d[a] - sh.d[a] == 0.0);
    lmax = fmax(lmax, sh.d[a]);
    lmin = fmin(lmin, sh.d[a]);
  }
  // a failed step reports and writes the identity, so the block stays finite until
  // the host sees the status; Gram eigenvalues are floored at 1e-15 of the largest
  // (directions lost to rounding come back rescaled, the next pass normalises them)
  const bool bad = !ok || !finite || (mode >= 1 && !(lmax > 0.0));
  const double floor_l = 1e-15 * lmax;
  for (int f = threadIdx.x; f < KB * KB; f += blockDim.x) {
    const int i = f / KB, j = f - i * KB;   // C[i][j] = component i of vector j
    const double zij = A[s_perm[j] * lda + i];
    if (bad) C[f] = (i == j) ? 1.0 : 0.0;
    else C[f] = (mode >= 1) ? s_dinv[i] * zij / sqrt(fmax(sh.d[s_perm[j]], floor_l)) : zij;
  }
  if (mode == 0)
    for (int a = threadIdx.x; a < KB; a += blockDim.x) theta[a] = sh.d[s_perm[a]];
  if (threadIdx.x == 0 && bad) atomicOr(status, ok ? 2 : 1);
}

// res_j = |W_j - theta_j X_j| for the KB rows j (blockIdx.x) of every unmasked
// slot (blockIdx.y).
__global__ __launch_bounds__(256) void k_resid(const double* __restrict__ X, const double* __restrict__ W,
                                               const double* __restrict__ theta, int N, int KB,
                                               const int* __restrict__ act, double* __restrict__ res) {
  const int b = blockIdx.y;
  if (!act[b]) return;
  __shared__ double red[4];
  const int j = blockIdx.x;
  const size_t row = (static_cast<size_t>(b) * KB + j) * N;
  const double th = theta[static_cast<size_t>(b) * KB + j];
  const double* xj = X + row;
  const double* wj = W + row;
  double acc = 0.0;
  for (int x = threadIdx.x; x < N; x += blockDim.x) {
    const double r = wj[x] - th * xj[x];
    acc += r * r;
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) res[static_cast<size_t>(b) * KB + j] = sqrt(red[0] + red[1] + red[2] + red[3]);
}

// Canonical basis of a converged Ritz block, in three launches over all slots
// whose info entry (chunk index c, grid point g) has c >= 0.  The levels a < ncols
// (Ritz values theta, ascending) form clusters where consecutive values differ by
// less than tol; within a cluster of two or more levels the vectors are rotated to
// the eigenvectors of diag(x) (ascending), then every level a < n gets the sign rule.

// Cluster rotations, one workgroup per slot.  Gfull: <v_i| diag(x) |v_j> over the
// ncols levels (ld ncols).  Writes R (row-major, ld ncols: new_j = sum_i R[j][i]
// old_i, the identity outside clusters), cl (per level: cluster start, then at +KB
// its size), E[g] (level energies, padded to NP with zeros), gs[g] (levels of the
// lowest cluster, at most n) and status[c] bit 2 if a cluster eigensolve failed.
__global__ __launch_bounds__(kEigThreads) void k_canon_rot(const double* __restrict__ Gfull, int KB,
                                                           const double* __restrict__ theta, int ncols, int n,
                                                           int NP, double tol, const int* __restrict__ info,
                                                           double* __restrict__ Etab, int* __restrict__ gstab,
                                                           double* __restrict__ R, int* __restrict__ cl,
                                                           double* __restrict__ ws, int* __restrict__ status) {
  const int b = blockIdx.x;
  const int c = info[2 * b], g = info[2 * b + 1];
  if (c < 0) return;
  __shared__ EigShared sh;
  __shared__ double s_E[kEigMaxN];
  __shared__ int s_cs[kEigMaxN + 1];
  __shared__ int s_ncl;
  __shared__ int s_perm2[kEigMaxN];
  const int tid = threadIdx.x;
  Gfull += static_cast<size_t>(b) * KB * KB;
  theta += static_cast<size_t>(b) * KB;
  R += static_cast<size_t>(b) * KB * KB;
  cl += static_cast<size_t>(b) * 2 * KB;
  ws += static_cast<size_t>(b) * 2 * KB * KB;
  for (int a = tid; a < ncols; a += blockDim.x) s_E[a] = theta[a];
  for (int f = tid; f < ncols * ncols; f += blockDim.x) R[f] = (f / ncols == f % ncols) ? 1.0 : 0.0;
  __syncthreads();
  if (tid == 0) {
    int k = 0;
    s_cs[k++] = 0;
    for (int a = 1; a < ncols; ++a)
      if (s_E[a] - s_E[a - 1] >= tol) s_cs[k++] = a;
    s_cs[k] = ncols;
    s_ncl = k;
  }
  __syncthreads();
  const int ncl = s_ncl;
  for (int q = tid; q < ncl; q += blockDim.x)
    for (int a = s_cs[q]; a < s_cs[q + 1]; ++a) {
      cl[a] = s_cs[q];
      cl[KB + a] = s_cs[q + 1] - s_cs[q];
    }
  bool ok = true;
  for (int q = 0; q < ncl; ++q) {
    const int a0 = s_cs[q], cs = s_cs[q + 1] - a0;
    if (cs < 2) continue;
    double* G = ws;
    double* ZG = ws + static_cast<size_t>(cs) * cs;
    for (int p = tid; p < cs * cs; p += blockDim.x) {
      const int i = p / cs, j = p - i * cs;
      G[p] = Gfull[static_cast<size_t>(a0 + i) * ncols + a0 + j];
    }
    __syncthreads();
    wg_tridiagonalize(G, cs, cs, sh);
    ok = wg_band_qr(ZG, cs, cs, sh) && ok;
    wg_rank_ascending(sh.d, cs, s_perm2);
    wg_back_transform(G, cs, cs, ZG, cs, s_perm2, cs, sh);
    // new_j = sum_i Q[i][j] old_i with Q[i][j] = ZG[perm2[j]][i]
    for (int p = tid; p < cs * cs; p += blockDim.x) {
      const int j = p / cs, i = p - j * cs;
      R[static_cast<size_t>(a0 + j) * ncols + a0 + i] = ZG[static_cast<size_t>(s_perm2[j]) * cs + i];
    }
    for (int j = tid; j < cs; j += blockDim.x) {
      const double* qj = ZG + static_cast<size_t>(s_perm2[j]) * cs;
      double e = 0.0;
      for (int i = 0; i < cs; ++i) e += qj[i] * qj[i] * s_E[a0 + i];
      sh.w[j] = e;
    }
    __syncthreads();
    for (int j = tid; j < cs; j += blockDim.x) s_E[a0 + j] = sh.w[j];
    __syncthreads();
  }
  for (int a = tid; a < NP; a += blockDim.x) Etab[static_cast<size_t>(g) * NP + a] = (a < n) ? s_E[a] : 0.0;
  if (tid == 0) {
    gstab[g] = min(n, ncl > 1 ? s_cs[1] : ncols);
    if (!ok) status[c] |= 2;
  }
}

// V_j = sum_i R[j][i] X_i over the cluster of level j (blockIdx.y < ncols), x in
// blockIdx.x, slot in blockIdx.z; written as row j of chunk entry c of Vout.
__global__ __launch_bounds__(256) void k_canon_apply(const double* __restrict__ X, size_t blk,
                                                     const double* __restrict__ R, int KB,
                                                     const int* __restrict__ cl, const int* __restrict__ info,
                                                     int ncols, int N, double* __restrict__ Vout, size_t Vstride) {
  const int b = blockIdx.z;
  const int c = info[2 * b];
  if (c < 0) return;
  const int j = blockIdx.y;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= N) return;
  const int a0 = cl[static_cast<size_t>(b) * 2 * KB + j], cs = cl[static_cast<size_t>(b) * 2 * KB + KB + j];
  const double* Rj = R + static_cast<size_t>(b) * KB * KB + static_cast<size_t>(j) * ncols + a0;
  const double* Xb = X + static_cast<size_t>(b) * blk + static_cast<size_t>(a0) * N + x;
  double acc = 0.0;
  for (int i = 0; i < cs; ++i) acc += Rj[i] * Xb[static_cast<size_t>(i) * N];
  Vout[static_cast<size_t>(c) * Vstride + static_cast<size_t>(j) * N + x] = acc;
}

// Sign rule for level blockIdx.x of every slot's canonical rows (blockIdx.y): the
// first entry within 1e-9 of the largest magnitude is made positive.
__global__ __launch_bounds__(256) void k_canon_signs(double* __restrict__ Vout, size_t Vstride,
                                                     const int* __restrict__ info, int N) {
  const int b = blockIdx.y;
  const int c = info[2 * b];
  if (c < 0) return;
  __shared__ double s_mx[4];
  __shared__ int s_first[4];
  __shared__ int s_flip;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* va = Vout + static_cast<size_t>(c) * Vstride + static_cast<size_t>(blockIdx.x) * N;
  double mx = 0.0;
  for (int x = tid; x < N; x += blockDim.x) mx = fmax(mx, fabs(va[x]));
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  if (lane == 0) s_mx[wave] = mx;
  __syncthreads();
  mx = fmax(fmax(s_mx[0], s_mx[1]), fmax(s_mx[2], s_mx[3]));
  int first = N;
  for (int x = tid; x < N; x += blockDim.x)
    if (fabs(va[x]) >= (1.0 - 1e-9) * mx) {
      first = x;
      break;
    }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) first = min(first, __shfl_xor(first, o, 64));
  if (lane == 0) s_first[wave] = first;
  __syncthreads();
  if (tid == 0) {
    int f = min(min(s_first[0], s_first[1]), min(s_first[2], s_first[3]));
    if (f >= N) f = 0;   // no entry qualified (non-finite vector): stay in range
    s_flip = va[f] < 0.0;
  }
  __syncthreads();
  if (s_flip)
    for (int x = tid; x < N; x += blockDim.x) va[x] = -va[x];
}

struct Chfsi {
  int nq = 0, N = 0, KB = 0, ksplit = 1;
  int nb = 1;        // block slots (chains advanced together)
  size_t blk = 0;    // doubles per slot of X, Y1, Y2, W (KB * N)
  DevBuf X, Y1, Y2, W, part, S, C, theta, res, ws, status, act, coef, info, cl;
  std::vector<double> h_theta, h_res;
  std::vector<int> h_status, h_act, h_info;
  std::vector<HxCoef> h_coef;
  std::vector<char> warm;   // per slot: X holds the Ritz block of a nearby grid point
  std::vector<char> far;    // per slot: ... of a grid point a chain length away (chain heads)
  double hub = 0.0;         // upper bound of the spectrum (Gershgorin)
  double* at(const DevBuf& b, int j) const { return b.as<double>() + static_cast<size_t>(j) * blk; }
};

// Control data for the next launches (host buffers are reused: wait for the copy).
aqt_status chfsi_upload(aqt_ctx* ctx, void* dst, const void* src, size_t bytes) {
  AQT_HIP(ctx, hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, ctx->stream));
  AQT_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return AQT_OK;
}

aqt_status chfsi_set_mask(aqt_ctx* ctx, Chfsi& c, const std::vector<int>& m) {
  c.h_act = m;
  return chfsi_upload(ctx, c.act.p, c.h_act.data(), static_cast<size_t>(c.nb) * 4);
}

// S_b = P_b Q_b^T (rows x rows, weight w(x) of GEMM mode wmode) over x in every
// unmasked slot, split over x; stored compact (ld rows) at slot b of c.S.
aqt_status chfsi_gram(aqt_ctx* ctx, Chfsi& c, const double* P, const double* Q, int rows, int wmode) {
  const int kspan = (c.N + c.ksplit - 1) / c.ksplit;
  GemmArgs ga{P, Q, c.part.as<double>(), static_cast<int64_t>(c.blk), static_cast<int64_t>(c.blk),
              static_cast<int64_t>(rows) * rows, rows, rows, c.N, c.N, c.N, rows, wmode, c.nq, 0, c.ksplit, kspan};
  ga.bmask = c.act.as<int>();
  aqt_status st = launch_gemm(ctx, ga, c.nb * c.ksplit);
  if (st != AQT_OK) return st;
  hipLaunchKernelGGL(k_splitk_reduce, dim3(nblk(static_cast<int64_t>(rows) * rows * c.nb)), dim3(256), 0,
                     ctx->stream, c.part.as<double>(), c.ksplit, rows, rows, c.nb, c.S.as<double>(),
                     static_cast<int64_t>(c.KB) * c.KB, rows, 0);
  AQT_HIP(ctx, hipGetLastError());
  return AQT_OK;
}

aqt_status chfsi_combine(aqt_ctx* ctx, Chfsi& c, const double* in, double* out, int copy_masked) {
  const dim3 grid(static_cast<unsigned>((c.N + kCombineCols - 1) / kCombineCols), static_cast<unsigned>(c.nb));
  if (c.KB == 64)
    hipLaunchKernelGGL(k_combine<64>, grid, dim3(512), 0, ctx->stream, in, c.C.as<double>(), out, c.N,
                       c.act.as<int>(), copy_masked);
  else
    hipLaunchKernelGGL(k_combine<128>, grid, dim3(512), 0, ctx->stream, in, c.C.as<double>(), out, c.N,
                       c.act.as<int>(), copy_masked);
  AQT_HIP(ctx, hipGetLastError());
  return AQT_OK;
}

aqt_status chfsi_hx(aqt_ctx* ctx, Chfsi& c, const double* eZ, const HxCoef* coef, const double* in, const double* z,
                    double* out) {
  const int CH = std::min(c.N, kHxChunk);
  // one workgroup per (row, chunk); the decode in the kernel needs KB * nb % 8 == 0
  const int64_t wgs = static_cast<int64_t>(c.N / CH) * c.KB * c.nb;
  hipLaunchKernelGGL(k_hx_block, dim3(static_cast<unsigned>(wgs)), dim3(256), 0, ctx->stream, in, z, out, eZ, c.nq,
                     c.KB, coef);
  AQT_HIP(ctx, hipGetLastError());
  return AQT_OK;
}

aqt_status chfsi_small_eig(aqt_ctx* ctx, Chfsi& c, int mode) {
  hipLaunchKernelGGL(k_small_eig, dim3(c.nb), dim3(kEigThreads), 0, ctx->stream, c.S.as<double>(), c.KB, mode,
                     c.C.as<double>(), c.theta.as<double>(), c.ws.as<double>(), c.status.as<int>(),
                     c.act.as<int>());
  AQT_HIP(ctx, hipGetLastError());
  return AQT_OK;
}

// Orthonormalise, in every unmasked slot, the rows of `in` into c.X (column
// scaling, then the inverse square root of the Gram matrix, twice).
aqt_status chfsi_orth(aqt_ctx* ctx, Chfsi& c, double* in) {
  double* src = in;
  for (int pass = 0; pass < 2; ++pass) {
    aqt_status st = chfsi_gram(ctx, c, src, src, c.KB, 0);
    if (st == AQT_OK) st = chfsi_small_eig(ctx, c, 2);
    if (st != AQT_OK) return st;
    double* dst = (pass == 0) ? c.Y2.as<double>() : c.X.as<double>();
    if (dst == src) dst = c.W.as<double>();
    if ((st = chfsi_combine(ctx, c, src, dst, 0)) != AQT_OK) return st;
    src = dst;
  }
  if (src != c.X.as<double>())
    for (int j = 0; j < c.nb; ++j)
      if (c.h_act[j])
        AQT_HIP(ctx, hipMemcpyAsync(c.at(c.X, j), src + static_cast<size_t>(j) * c.blk, c.blk * 8,
                                    hipMemcpyDeviceToDevice, ctx->stream));
  return AQT_OK;
}

// Converge, in every slot j with nconv[j] > 0, the lowest nconv[j] Ritz pairs of
// H(s_g) = A_g H_X + B_g diag(e_Z), g = gidx[j], to residual <= tol * hub.  On
// return slot j of c.X holds its KB Ritz vectors (ascending Ritz values in slot j
// of c.theta); the other slots keep their contents.
aqt_status chfsi_solve(aqt_ctx* ctx, Chfsi& c, const double* eZ, const std::vector<double>& Ag,
                       const std::vector<double>& Bg, const std::vector<int>& gidx, const std::vector<int>& nconv,
                       double tol) {
  hipStream_t st = ctx->stream;
  const int nb = c.nb, KB = c.KB;
  std::vector<int> live(nb, 0), cold(nb, 0), iters(nb, 0), maxit(nb, 0), degree(nb, 0);
  bool anycold = false;
  for (int j = 0; j < nb; ++j) {
    live[j] = nconv[j] > 0;
    cold[j] = live[j] && !c.warm[j];
    anycold = anycold || cold[j];
    // a start from the neighbouring grid point converges in a few iterations; a chain head
    // starts from the previous head, a chain length away, where the spectrum near the cut
    // may have rearranged, and gets the budget of a cold start twice over
    maxit[j] = !c.warm[j] ? 150 : (c.far[j] ? 300 : 80);
  }
  auto where = [&](int j) { return "at grid point " + std::to_string(gidx[j]); };
  AQT_HIP(ctx, hipMemsetAsync(c.status.p, 0, static_cast<size_t>(nb) * 4, st));
  aqt_status s = AQT_OK;
  if (anycold) {
    for (int j = 0; j < nb; ++j)
      if (cold[j]) {
        hipLaunchKernelGGL(k_random_block, dim3(nblk(static_cast<int64_t>(c.blk))), dim3(256), 0, st, c.at(c.X, j),
                           static_cast<int64_t>(c.blk));
        AQT_HIP(ctx, hipGetLastError());
      }
    if ((s = chfsi_set_mask(ctx, c, cold)) != AQT_OK || (s = chfsi_orth(ctx, c, c.X.as<double>())) != AQT_OK) return s;
  }
  for (;;) {
    // Rayleigh-Ritz in every live slot
    if ((s = chfsi_set_mask(ctx, c, live)) != AQT_OK) return s;
    c.h_coef.assign(nb, HxCoef{0.0, 0.0, 1.0, 0.0, 0.0, 0, 0});
    for (int j = 0; j < nb; ++j)
      if (live[j]) {
        c.h_coef[j].A = Ag[gidx[j]];
        c.h_coef[j].B = Bg[gidx[j]];
        c.h_coef[j].active = 1;
      }
    if ((s = chfsi_upload(ctx, c.coef.p, c.h_coef.data(), nb * sizeof(HxCoef))) != AQT_OK) return s;
    const HxCoef* drr = c.coef.as<HxCoef>();
    if ((s = chfsi_hx(ctx, c, eZ, drr, c.X.as<double>(), nullptr, c.W.as<double>())) != AQT_OK) return s;
    if ((s = chfsi_gram(ctx, c, c.X.as<double>(), c.W.as<double>(), KB, 0)) != AQT_OK) return s;
    if ((s = chfsi_small_eig(ctx, c, 0)) != AQT_OK) return s;
    // masked slots are copied, so that the buffer swap keeps their blocks
    if ((s = chfsi_combine(ctx, c, c.X.as<double>(), c.Y1.as<double>(), 1)) != AQT_OK) return s;
    if ((s = chfsi_combine(ctx, c, c.W.as<double>(), c.Y2.as<double>(), 1)) != AQT_OK) return s;
    std::swap(c.X.p, c.Y1.p);
    std::swap(c.W.p, c.Y2.p);
    hipLaunchKernelGGL(k_resid, dim3(KB, nb), dim3(256), 0, st, c.X.as<double>(), c.W.as<double>(),
                       c.theta.as<double>(), c.N, KB, c.act.as<int>(), c.res.as<double>());
    AQT_HIP(ctx, hipGetLastError());
    AQT_HIP(ctx, hipMemcpyAsync(c.h_theta.data(), c.theta.p, static_cast<size_t>(nb) * KB * 8, hipMemcpyDeviceToHost, st));
    AQT_HIP(ctx, hipMemcpyAsync(c.h_res.data(), c.res.p, static_cast<size_t>(nb) * KB * 8, hipMemcpyDeviceToHost, st));
    AQT_HIP(ctx, hipMemcpyAsync(c.h_status.data(), c.status.p, static_cast<size_t>(nb) * 4, hipMemcpyDeviceToHost, st));
    AQT_HIP(ctx, hipStreamSynchronize(st));
    bool any = false;
    for (int j = 0; j < nb; ++j) {
      if (!live[j]) continue;
      if (c.h_status[j]) return ctx->fail(AQT_ENUMERIC, "subspace iteration: small eigensolver failed " + where(j));
      const double* res = c.h_res.data() + static_cast<size_t>(j) * KB;
      double worst = 0.0;
      for (int a = 0; a < nconv[j]; ++a) worst = std::max(worst, res[a]);
      if (!(worst == worst)) return ctx->fail(AQT_ENUMERIC, "subspace iteration produced NaN " + where(j));
      if (worst <= tol * c.hub) {
        live[j] = 0;
        continue;
      }
      if (iters[j] >= maxit[j])
        return ctx->fail(AQT_ENUMERIC, "subspace iteration did not converge " + where(j) + " (residual " +
                                           std::to_string(worst / c.hub) + " of |H|)");
      ++iters[j];
      any = true;
    }
    if (!any) break;
    // Chebyshev filter damping [theta_last, hub], scaled at theta_0, per live slot; the
    // degree makes the slowest wanted level gain about 10^3 over the damped interval
    int dmax = 0;
    std::vector<double> fe(nb), fcen(nb), fsig(nb);
    for (int j = 0; j < nb; ++j) {
      degree[j] = 0;
      if (!live[j]) continue;
      const double* th = c.h_theta.data() + static_cast<size_t>(j) * KB;
      const double lo = th[0], cut = th[KB - 1];
      const double e = 0.5 * (c.hub - cut), cen = 0.5 * (c.hub + cut);
      const double xw = std::fabs((th[nconv[j] - 1] - cen) / e);
      const double xl = std::fabs((lo - cen) / e);
      int d = 256;
      if (xw > 1.0 + 1e-12) d = static_cast<int>(std::ceil(std::acosh(1e3) / std::acosh(xw)));
      // amplification of the lowest level over the damped interval, T_d(x_lo) ~ e^{d acosh x_lo},
      // kept below 1e10: beyond that the filtered block loses the directions it amplifies
      // least to rounding (its Gram matrix becomes numerically singular)
      if (xl > 1.0) d = std::min(d, static_cast<int>(std::log(1e10) / std::acosh(xl)));
      degree[j] = std::max(2, std::min(kMaxFilterDegree, d));
      dmax = std::max(dmax, degree[j]);
      fe[j] = e;
      fcen[j] = cen;
      fsig[j] = e / (lo - cen);
    }
    // three-term recurrence coefficients, row k-1 for step k; a slot past its degree is masked
    c.h_coef.assign(static_cast<size_t>(dmax) * nb, HxCoef{0.0, 0.0, 0.0, 0.0, 0.0, 0, 0});
    for (int j = 0; j < nb; ++j) {
      if (!live[j]) continue;
      const double e = fe[j], cen = fcen[j];
      double sigma = fsig[j];
      const double tau = 2.0 / sigma;
      for (int k = 1; k <= degree[j]; ++k) {
        HxCoef& h = c.h_coef[static_cast<size_t>(k - 1) * nb + j];
        h.A = Ag[gidx[j]];
        h.B = Bg[gidx[j]];
        h.active = 1;
        if (k == 1) {
          h.alpha = sigma / e;
          h.beta = -cen * sigma / e;
        } else {
          const double sn = 1.0 / (tau - sigma);
          h.alpha = 2.0 * sn / e;
          h.beta = -2.0 * cen * sn / e;
          h.gamma = -sigma * sn;
          sigma = sn;
        }
      }
    }
    HxCoef* dfc = c.coef.as<HxCoef>() + nb;
    if ((s = chfsi_upload(ctx, dfc, c.h_coef.data(), c.h_coef.size() * sizeof(HxCoef))) != AQT_OK) return s;
    double* const P[3] = {c.X.as<double>(), c.Y1.as<double>(), c.Y2.as<double>()};
    double* x0 = P[0];
    double* y1 = P[1];
    double* y2 = P[2];
    if ((s = chfsi_hx(ctx, c, eZ, dfc, x0, nullptr, y1)) != AQT_OK) return s;
    for (int k = 2; k <= dmax; ++k) {
      if ((s = chfsi_hx(ctx, c, eZ, dfc + static_cast<size_t>(k - 1) * nb, y1, x0, y2)) != AQT_OK) return s;
      double* t = x0;
      x0 = y1;
      y1 = y2;
      y2 = t;
    }
    // step k writes buffer P[k % 3]: gather every slot's filtered block into Y1, then
    // orthonormalise into X (Y2 and W are the scratch of the orthonormalisation)
    for (int j = 0; j < nb; ++j)
      if (live[j] && degree[j] % 3 != 1)
        AQT_HIP(ctx, hipMemcpyAsync(c.at(c.Y1, j), P[degree[j] % 3] + static_cast<size_t>(j) * c.blk, c.blk * 8,
                                    hipMemcpyDeviceToDevice, st));
    if ((s = chfsi_orth(ctx, c, c.Y1.as<double>())) != AQT_OK) return s;
  }
  for (int j = 0; j < nb; ++j)
    if (nconv[j] > 0) {
      c.warm[j] = 1;
      c.far[j] = 0;
    }
  return AQT_OK;
}

// Canonical vectors, energies and ground-state multiplicities of the slots with
// gidx[j] >= 0 (grid point gidx[j], chunk entry gidx[j] - g0 of Vout).
aqt_status chfsi_canon(aqt_ctx* ctx, Chfsi& c, const std::vector<int>& gidx, int g0, int ncols, int n, int NP,
                       double tol, double* Vout, size_t Vstride, int* status) {
  hipStream_t st = ctx->stream;
  const int nb = c.nb;
  std::vector<int> m(nb);
  c.h_info.assign(2 * static_cast<size_t>(nb), -1);
  for (int j = 0; j < nb; ++j) {
    m[j] = gidx[j] >= 0;
    if (m[j]) {
      c.h_info[2 * j] = gidx[j] - g0;
      c.h_info[2 * j + 1] = gidx[j];
    }
  }
  aqt_status s = chfsi_set_mask(ctx, c, m);
  if (s == AQT_OK) s = chfsi_upload(ctx, c.info.p, c.h_info.data(), c.h_info.size() * 4);
  // Gram matrix of diag(x) over the ncols Ritz vectors (cluster rotations)
  if (s == AQT_OK) s = chfsi_gram(ctx, c, c.X.as<double>(), c.X.as<double>(), ncols, 2);
  if (s != AQT_OK) return s;
  hipLaunchKernelGGL(k_canon_rot, dim3(nb), dim3(kEigThreads), 0, st, c.S.as<double>(), c.KB, c.theta.as<double>(),
                     ncols, n, NP, tol, c.info.as<int>(), ctx->E.as<double>(), ctx->gs.as<int>(), c.C.as<double>(),
                     c.cl.as<int>(), c.ws.as<double>(), status);
  AQT_HIP(ctx, hipGetLastError());
  hipLaunchKernelGGL(k_canon_apply, dim3(nblk(c.N), ncols, nb), dim3(256), 0, st, c.X.as<double>(), c.blk,
                     c.C.as<double>(), c.KB, c.cl.as<int>(), c.info.as<int>(), ncols, c.N, Vout, Vstride);
  AQT_HIP(ctx, hipGetLastError());
  hipLaunchKernelGGL(k_canon_signs, dim3(n, nb), dim3(256), 0, st, Vout, Vstride, c.info.as<int>(), c.N);
  AQT_HIP(ctx, hipGetLastError());
  return AQT_OK;
}

constexpr int kChainMinRun = 8;   // grid points per chain, at least

// Eigenpairs and canonical vectors of grid points g0 .. g0+cnt-1 (chunk entries
// 0 .. cnt-1 of Vout).  The run is cut into up to c.nb contiguous chains.  The
// chain heads are solved one after another, each warm-started from the head before
// it (the first from the last grid point solved before), then the chains advance
// one grid point per step in lock step.
aqt_status chfsi_chunk(aqt_ctx* ctx, Chfsi& c, const double* eZ, const std::vector<double>& Ag,
                       const std::vector<double>& Bg, int g0, int cnt, int ncols, int n, int NP, double tol,
                       double* Vout, size_t Vstride, int* status) {
  const int nb = c.nb;
  const int nc = std::max(1, std::min(nb, cnt / kChainMinRun));
  std::vector<int> head(nc + 1);
  for (int j = 0; j <= nc; ++j) head[j] = g0 + static_cast<int>(static_cast<int64_t>(j) * cnt / nc);
  // grid 0 only supplies the initial state (its ground state, checked to be
  // non-degenerate); H(0) is typically highly degenerate, so only the two lowest
  // levels are converged there
  auto nconv_at = [&](int g) { return (g == 0) ? std::min(2, ncols) : ncols; };
  std::vector<int> gidx(nb, -1), nconv(nb, 0);
  aqt_status s = AQT_OK;
  for (int j = 0; j < nc; ++j) {
    if (j > 0) {
      AQT_HIP(ctx, hipMemcpyAsync(c.at(c.X, j), c.at(c.X, j - 1), c.blk * 8, hipMemcpyDeviceToDevice, ctx->stream));
      c.warm[j] = 1;
      c.far[j] = 1;
    }
    std::fill(gidx.begin(), gidx.end(), -1);
    std::fill(nconv.begin(), nconv.end(), 0);
    gidx[j] = head[j];
    nconv[j] = nconv_at(head[j]);
    if ((s = chfsi_solve(ctx, c, eZ, Ag, Bg, gidx, nconv, 1e-12)) != AQT_OK) return s;
    // at s = 0 only the lowest levels converged: the next solve from this block starts
    // nearly cold
    if (head[j] == 0) c.far[j] = 1;
  }
  std::fill(gidx.begin(), gidx.end(), -1);
  int len = 0;
  for (int j = 0; j < nc; ++j) {
    gidx[j] = head[j];
    len = std::max(len, head[j + 1] - head[j]);
  }
  if ((s = chfsi_canon(ctx, c, gidx, g0, ncols, n, NP, tol, Vout, Vstride, status)) != AQT_OK) return s;
  for (int t = 1; t < len; ++t) {
    for (int j = 0; j < nb; ++j) {
      const bool on = j < nc && head[j] + t < head[j + 1];
      gidx[j] = on ? head[j] + t : -1;
      nconv[j] = on ? nconv_at(gidx[j]) : 0;
    }
    if ((s = chfsi_solve(ctx, c, eZ, Ag, Bg, gidx, nconv, 1e-12)) != AQT_OK) return s;
    if ((s = chfsi_canon(ctx, c, gidx, g0, ncols, n, NP, tol, Vout, Vstride, status)) != AQT_OK) return s;
  }
  // the next chunk starts from the last grid point of this one
  if (nc > 1) {
    AQT_HIP(ctx, hipMemcpyAsync(c.at(c.X, 0), c.at(c.X, nc - 1), c.blk * 8, hipMemcpyDeviceToDevice, ctx->stream));
    c.warm[0] = 1;
  }
  return AQT_OK;
}

}  // namespace

aqt_status precompute_tables(aqt_ctx* ctx, int M, int n, double tol, int method, bool grad) {
  const int nq = ctx->nq;
  const int N = 1 << nq;
  const int nch = ctx->nch();   // jump channels (nq for independent or constant-correlation baths)
  ctx->have_grad = false;
  ctx->gpk_prec = -1;
  if (grad && n != N) return ctx->fail(AQT_EINVAL, "gradient tables need the full spectrum (n_levels = 2^n_qubits)");
  const bool iterative = (method == AQT_EIG_ITERATIVE) || (method == AQT_EIG_AUTO && N > kEigMaxN);
  const int ncols = std::min(N, n + 16);   // levels solved for: n plus a guard for clusters at the cut
  int KB = 0;                              // block size of the subspace iteration
  if (iterative) {
    if (n >= N) return ctx->fail(AQT_EINVAL, "the iterative eigensolver computes truncated spectra (n_levels < 2^n_qubits)");
    // dense spectra of large spaces need the filter's cut well above the wanted levels
    KB = (ncols + 8 <= 64 && N < 4096) ? 64 : 128;
    if (ncols + 8 > KB || KB > N) return ctx->fail(AQT_EINVAL, "iterative eigensolver: n_levels too large for 2^n_qubits");
  } else {
    if (N > kEigMaxN) return ctx->fail(AQT_EINVAL, "dense eigensolver path needs 2^n_qubits <= 1024");
    if (n < N && n > 128) return ctx->fail(AQT_EINVAL, "truncated spectra are limited to n <= 128 levels");
  }
  const int NP = padded_levels(n);
  if (nch > std::min(NP, 64))
    return ctx->fail(AQT_EINVAL, "more jump channels than min(64, padded levels): keep more levels or fewer bath terms");
  hipStream_t st = ctx->stream;
  // dense path with ncols << N: bisection and inverse iteration instead of the full
  // rotation product, when the workspace (columns ncols.. of the N x N eigenvector
  // buffer) holds it
  bool partial = false;
  if (!iterative && ncols < N) {
    const size_t c = ncols, NN = N;
    const size_t need = 3 * NN + c + 2 * c * c + c * NN + 4 * c * NN + (c * NN + 7) / 8;
    partial = need <= (NN - c) * NN;
  }

  // ---- schedule samples and Ising diagonal
  if (!ctx->sgrid.empty() && static_cast<int>(ctx->sgrid.size()) != M)
    return ctx->fail(AQT_EINVAL, "n_grid differs from the point count of aqt_set_grid");
  std::vector<double> Ag(M), Bg(M);
  const int nc = static_cast<int>(ctx->A_ctrl.size());
  for (int g = 0; g < M; ++g) {
    const double s = ctx->sgrid.empty() ? static_cast<double>(g) / (M - 1) : ctx->sgrid[g];
    const double u = s * (nc - 1);
    int j = std::min(static_cast<int>(std::floor(u)), nc - 2);
    const double f = u - j;
    Ag[g] = ctx->A_ctrl[j] * (1.0 - f) + ctx->A_ctrl[j + 1] * f;
    Bg[g] = ctx->B_ctrl[j] * (1.0 - f) + ctx->B_ctrl[j + 1] * f;
  }
  ctx->sched_A = Ag;
  ctx->sched_B = Bg;
  DevBuf dA, dB, dh, dJ, eZ;
  if (dA.reserve(M * 8) || dB.reserve(M * 8) || dh.reserve(nq * 8) || dJ.reserve(nq * nq * 8) || eZ.reserve(N * 8))
    return ctx->fail(AQT_ENOMEM, "precompute allocation failed");
  AQT_HIP(ctx, hipMemcpyAsync(dA.p, Ag.data(), M * 8, hipMemcpyHostToDevice, st));
  AQT_HIP(ctx, hipMemcpyAsync(dB.p, Bg.data(), M * 8, hipMemcpyHostToDevice, st));
  AQT_HIP(ctx, hipMemcpyAsync(dh.p, ctx->h.data(), nq * 8, hipMemcpyHostToDevice, st));
  AQT_HIP(ctx, hipMemcpyAsync(dJ.p, ctx->J.data(), nq * nq * 8, hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_ising_diag, dim3(nblk(N)), dim3(256), 0, st, dh.as<double>(), dJ.as<double>(), nq,
                     eZ.as<double>());
  AQT_HIP(ctx, hipGetLastError());

  // ---- tables
  ctx->M = M;
  ctx->n = n;
  ctx->NP = NP;
  ctx->tab_nch = nch;
  ctx->dt = ctx->t_f / (M - 1);
  const size_t sNP = static_cast<size_t>(NP);
  if (ctx->E.reserve(M * sNP * 8) || ctx->gs.reserve(M * 4) || ctx->dlt.reserve(M * sNP * sNP * 8) ||
      ctx->cinit.reserve(sNP * 8) || ctx->R.reserve(static_cast<size_t>(M) * nch * sNP * sNP * 8) ||
      ctx->zdiag.reserve(static_cast<size_t>(M) * nch * sNP * 8) || ctx->leak.reserve(M * 8) ||
      ctx->shift.reserve(M * sNP * 8))
    return ctx->fail(AQT_ENOMEM, "table allocation failed");
  AQT_HIP(ctx, hipMemsetAsync(ctx->dlt.p, 0, M * sNP * sNP * 8, st));
  AQT_HIP(ctx, hipMemsetAsync(ctx->R.p, 0, static_cast<size_t>(sNP) * sNP * nch * 8, st));       // g = 0 unused
  AQT_HIP(ctx, hipMemsetAsync(ctx->zdiag.p, 0, static_cast<size_t>(sNP) * nch * 8, st));
  AQT_HIP(ctx, hipMemsetAsync(ctx->leak.p, 0, M * 8, st));
  AQT_HIP(ctx, hipMemsetAsync(ctx->shift.p, 0, M * sNP * 8, st));
  // jump-channel couplings: sz of each qubit, or for correlated baths gamma_ab(w) =
  // sum_m C_m[a][b] gamma(w; omega_c,m) with C_m = F_m F_m^T the channels sum_a F_m[a][k] sz_a,
  // each with its term's cutoff (Sec. II eq. ME2-L); chan holds the F columns
  DevBuf chw, wcv;
  if (!ctx->chan.empty()) {
    std::vector<double> w(static_cast<size_t>(nch) * N);
    for (int k = 0; k < nch; ++k)
      for (int x = 0; x < N; ++x) {
        double acc = 0.0;
        for (int a = 0; a < nq; ++a) acc += ctx->chan[static_cast<size_t>(k) * nq + a] * (((x >> a) & 1) ? -1.0 : 1.0);
        w[static_cast<size_t>(k) * N + x] = acc;
      }
    if (chw.reserve(w.size() * 8)) return ctx->fail(AQT_ENOMEM, "channel weight allocation failed");
    AQT_HIP(ctx, hipMemcpyAsync(chw.p, w.data(), w.size() * 8, hipMemcpyHostToDevice, st));
  }
  // sx parts of the channel operators (general couplings): applied as row permutations
  const bool sx = !ctx->chan_x.empty();
  DevBuf cxv;
  if (sx) {
    if (cxv.reserve(ctx->chan_x.size() * 8)) return ctx->fail(AQT_ENOMEM, "channel coupling allocation failed");
    AQT_HIP(ctx, hipMemcpyAsync(cxv.p, ctx->chan_x.data(), ctx->chan_x.size() * 8, hipMemcpyHostToDevice, st));
  }
  std::vector<double> wch(nch, ctx->omega_c);
  for (int k = 0; k < nch && k < static_cast<int>(ctx->chan_wc.size()); ++k)
    if (ctx->chan_wc[k] != 0.0) wch[k] = ctx->chan_wc[k];
  if (wcv.reserve(nch * 8)) return ctx->fail(AQT_ENOMEM, "channel cutoff allocation failed");
  AQT_HIP(ctx, hipMemcpyAsync(wcv.p, wch.data(), nch * 8, hipMemcpyHostToDevice, st));
  // Lamb-shift function table over every Bohr frequency (Gershgorin bound on |e|)
  DevBuf lambS, gl, tixd;
  LambTable ltab{nullptr, 0.0, nullptr};
  if (ctx->lamb) {
    double hsum = 0.0;
    for (double v : ctx->h) hsum += std::fabs(v);
    for (int i = 0; i < nq; ++i)
      for (int j = i + 1; j < nq; ++j) hsum += std::fabs(ctx->J[i * nq + j]);
    double amax = 0.0, bmax = 0.0;
    for (int g = 0; g < M; ++g) {
      amax = std::max(amax, std::fabs(Ag[g]));
      bmax = std::max(bmax, std::fabs(Bg[g]));
    }
    ltab.W = 2.0 * (amax * nq + bmax * hsum) * 1.01 + 1.0;
    // 16-point Gauss-Legendre nodes (Newton on P_16) and weights
    std::vector<double> glh(32);
    for (int q = 0; q < 16; ++q) {
      double x = std::cos(M_PI * (q + 0.75) / 16.5), dp = 1.0;
      for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = x;
        for (int l = 2; l <= 16; ++l) {
          const double p2 = ((2.0 * l - 1.0) * x * p1 - (l - 1.0) * p0) / l;
          p0 = p1;
          p1 = p2;
        }
        dp = 16.0 * (x * p1 - p0) / (x * x - 1.0);
        const double dx = p1 / dp;
        x -= dx;
        if (std::fabs(dx) < 1e-16) break;
      }
      glh[q] = x;
      glh[16 + q] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    // one S table per distinct channel cutoff
    std::vector<double> cut;
    std::vector<int> tix(nch);
    for (int k = 0; k < nch; ++k) {
      const auto it = std::find(cut.begin(), cut.end(), wch[k]);
      tix[k] = static_cast<int>(it - cut.begin());
      if (it == cut.end()) cut.push_back(wch[k]);
    }
    if (lambS.reserve(cut.size() * kLambNodes * 8) || gl.reserve(32 * 8) || tixd.reserve(nch * 4))
      return ctx->fail(AQT_ENOMEM, "Lamb-shift table allocation failed");
    AQT_HIP(ctx, hipMemcpyAsync(gl.p, glh.data(), 32 * 8, hipMemcpyHostToDevice, st));
    AQT_HIP(ctx, hipMemcpyAsync(tixd.p, tix.data(), nch * 4, hipMemcpyHostToDevice, st));
    for (size_t m = 0; m < cut.size(); ++m) {
      hipLaunchKernelGGL(k_lamb_table, dim3(nblk(kLambNodes, 64)), dim3(64), 0, st, ltab.W, ctx->eta, cut[m],
                         ctx->T, gl.as<double>(), gl.as<double>() + 16, lambS.as<double>() + m * kLambNodes);
      AQT_HIP(ctx, hipGetLastError());
    }
    ltab.S = lambS.as<double>();
    ltab.tix = tixd.as<int>();
  }

  // ---- chunked workspace
  const size_t per_grid = (iterative ? 0 : 2 * static_cast<size_t>(N) * N)   // H, Z (dense path)
                          + static_cast<size_t>(ncols) * N            // canonical V
                          + (iterative ? 0 : 2 * static_cast<size_t>(ncols) * ncols + static_cast<size_t>(ncols) * N)  // canon ws
                          + static_cast<size_t>(nch) * n * n          // z
                          + (sx ? static_cast<size_t>(nch) * n * N : 0)   // channel operators on V
                          + 9 * static_cast<size_t>(n) * n            // polar ws
                          + N                                         // Eraw
                          + (grad ? static_cast<size_t>(n) * N + 2 * static_cast<size_t>(n) * n +
                                        2 * static_cast<size_t>(nch) * n * n
                                  : 0);                               // H_X rows, V H' V^T, z X^T
  const size_t budget = size_t(24) << 30;   // of 288 GB HBM: all grid points of a 10-qubit instance in one chunk
  int Gc = static_cast<int>(std::max<size_t>(1, std::min<size_t>(M, budget / (per_grid * 8))));
  Gc = std::max(1, std::min(Gc, 65535 / std::max(nch, 2 * nq)));   // batched products: grid z <= 65535
  DevBuf H, Z, Vc, Vprev, cws, zws, pws, Eraw, perm, status;
  if ((!iterative && (H.reserve(static_cast<size_t>(Gc) * N * N * 8) || Z.reserve(static_cast<size_t>(Gc) * N * N * 8))) ||
      Vc.reserve(static_cast<size_t>(Gc) * ncols * N * 8) || Vprev.reserve(static_cast<size_t>(ncols) * N * 8) ||
      (!iterative && cws.reserve(static_cast<size_t>(Gc) * (2 * static_cast<size_t>(ncols) * ncols + static_cast<size_t>(ncols) * N) * 8)) ||
      zws.reserve(static_cast<size_t>(Gc) * nch * n * n * 8) || pws.reserve(static_cast<size_t>(Gc) * 9 * n * n * 8) ||
      Eraw.reserve(static_cast<size_t>(Gc) * N * 8) || perm.reserve(static_cast<size_t>(Gc) * N * 4) ||
      status.reserve(static_cast<size_t>(Gc) * 4))
    return ctx->fail(AQT_ENOMEM, "precompute workspace allocation failed");
  DevBuf Yc;
  if (sx && Yc.reserve(static_cast<size_t>(Gc) * nch * n * N * 8))
    return ctx->fail(AQT_ENOMEM, "precompute workspace allocation failed");
  DevBuf Wx, Hd, Qz;
  if (grad) {
    const size_t sn = n, sN = N, snp = NP;
    if (Wx.reserve(Gc * sn * sN * 8) || Hd.reserve(Gc * 2 * sn * sn * 8) || Qz.reserve(Gc * 2 * nch * sn * sn * 8) ||
        ctx->Xd.reserve(M * 2 * snp * snp * 8) || ctx->dE.reserve(M * 2 * snp * 8) ||
        ctx->dGam.reserve(M * 2 * snp * 8) || ctx->dzd.reserve(M * 2 * nch * snp * 8) ||
        ctx->dll.reserve(M * 2 * nch * snp * snp * 8) || ctx->dcin.reserve(2 * snp * 8) ||
        ctx->dshift.reserve(M * 2 * snp * 8))
      return ctx->fail(AQT_ENOMEM, "gradient table allocation failed");
    AQT_HIP(ctx, hipMemsetAsync(ctx->dGam.p, 0, 2 * snp * 8, st));          // g = 0 unused
    AQT_HIP(ctx, hipMemsetAsync(ctx->dzd.p, 0, 2 * nch * snp * 8, st));
    AQT_HIP(ctx, hipMemsetAsync(ctx->dll.p, 0, 2 * nch * snp * snp * 8, st));
    AQT_HIP(ctx, hipMemsetAsync(ctx->dshift.p, 0, M * 2 * snp * 8, st));   // stays zero without the Lamb shift
  }
  std::vector<int> hstat(Gc);
  const size_t Vstride = static_cast<size_t>(ncols) * N;
  Chfsi ch;
  if (iterative) {
    ch.nq = nq;
    ch.N = N;
    ch.KB = KB;
    ch.ksplit = std::max(1, std::min(256, N / 256));
    ch.blk = static_cast<size_t>(KB) * N;
    const size_t kk = static_cast<size_t>(KB) * KB;
    // slots (chains solved together): up to kMaxChains, within 8 GiB of workspace
    const size_t per_slot = (4 * ch.blk + static_cast<size_t>(ch.ksplit) * kk + 5 * kk + 2 * KB) * 8;
    ch.nb = static_cast<int>(std::max<size_t>(1, std::min<size_t>(kMaxChains, (size_t(8) << 30) / per_slot)));
    const size_t nb = ch.nb;
    if (ch.X.reserve(nb * ch.blk * 8) || ch.Y1.reserve(nb * ch.blk * 8) || ch.Y2.reserve(nb * ch.blk * 8) ||
        ch.W.reserve(nb * ch.blk * 8) || ch.part.reserve(nb * ch.ksplit * kk * 8) || ch.S.reserve(nb * kk * 8) ||
        ch.C.reserve(nb * kk * 8) || ch.theta.reserve(nb * KB * 8) || ch.res.reserve(nb * KB * 8) ||
        ch.ws.reserve(nb * 2 * kk * 8) || ch.status.reserve(nb * 4) || ch.act.reserve(nb * 4) ||
        ch.coef.reserve(nb * (1 + kMaxFilterDegree) * sizeof(HxCoef)) || ch.info.reserve(nb * 2 * 4) ||
        ch.cl.reserve(nb * 2 * KB * 4))
      return ctx->fail(AQT_ENOMEM, "subspace iteration workspace allocation failed");
    ch.h_theta.resize(nb * KB);
    ch.h_res.resize(nb * KB);
    ch.h_status.resize(nb);
    ch.warm.assign(nb, 0);
    ch.far.assign(nb, 0);
    std::vector<double> hz(N);
    AQT_HIP(ctx, hipMemcpyAsync(hz.data(), eZ.p, N * 8, hipMemcpyDeviceToHost, st));
    AQT_HIP(ctx, hipStreamSynchronize(st));
    double zmax = 0.0;
    for (double v : hz) zmax = std::max(zmax, std::fabs(v));
    double amax = 0.0, bmax = 0.0;
    for (int g = 0; g < M; ++g) {
      amax = std::max(amax, std::fabs(Ag[g]));
      bmax = std::max(bmax, std::fabs(Bg[g]));
    }
    ch.hub = amax * nq + bmax * zmax;   // Gershgorin bound on every H(s_g)
  }

  for (int g0 = 0; g0 < M; g0 += Gc) {
    const int cnt = std::min(Gc, M - g0);
    if (!iterative) {
      hipLaunchKernelGGL(k_build_dense, dim3(nblk(static_cast<int64_t>(N) * N * cnt)), dim3(256), 0, st,
                         eZ.as<double>(), nq, dA.as<double>(), dB.as<double>(), g0, cnt, H.as<double>());
      AQT_HIP(ctx, hipGetLastError());
      if (N >= kStreamedEigMin)
        hipLaunchKernelGGL(k_dense_eig<true>, dim3(cnt), dim3(kEigThreads), 0, st, H.as<double>(), Z.as<double>(), N,
                           ncols, partial ? 1 : 0, Eraw.as<double>(), perm.as<int>(), status.as<int>());
      else
        hipLaunchKernelGGL(k_dense_eig<false>, dim3(cnt), dim3(kEigThreads), 0, st, H.as<double>(), Z.as<double>(), N,
                           ncols, partial ? 1 : 0, Eraw.as<double>(), perm.as<int>(), status.as<int>());
      AQT_HIP(ctx, hipGetLastError());
      hipLaunchKernelGGL(k_canon, dim3(cnt), dim3(kEigThreads), 0, st, Z.as<double>(), perm.as<int>(),
                         Eraw.as<double>(), N, ncols, n, NP, tol, g0, Vc.as<double>(), ctx->E.as<double>(),
                         ctx->gs.as<int>(), cws.as<double>(), status.as<int>());
      AQT_HIP(ctx, hipGetLastError());
    } else {
      AQT_HIP(ctx, hipMemsetAsync(status.p, 0, cnt * 4, st));
      aqt_status s = chfsi_chunk(ctx, ch, eZ.as<double>(), Ag, Bg, g0, cnt, ncols, n, NP, tol, Vc.as<double>(),
                                 Vstride, status.as<int>());
      if (s != AQT_OK) return s;
    }
    AQT_HIP(ctx, hipMemcpyAsync(hstat.data(), status.p, cnt * 4, hipMemcpyDeviceToHost, st));
    AQT_HIP(ctx, hipStreamSynchronize(st));
    for (int c = 0; c < cnt; ++c)
      if (hstat[c]) return ctx->fail(AQT_ENUMERIC, "eigensolver did not converge at grid point " + std::to_string(g0 + c));
    if (g0 == 0) {
      int gs0 = 0;
      AQT_HIP(ctx, hipMemcpy(&gs0, ctx->gs.p, 4, hipMemcpyDeviceToHost));
      if (gs0 != 1) return ctx->fail(AQT_ENUMERIC, "ground state of H(s=0) is degenerate; initial state undefined");
    }
    // overlaps into grid g from g-1 (g >= 2); the first grid of a chunk pairs with Vprev
    for (int c = 0; c < cnt; ++c) {
      const int g = g0 + c;
      const double* Vg = Vc.as<double>() + c * Vstride;
      const double* Vp = (c == 0) ? Vprev.as<double>() : Vc.as<double>() + (c - 1) * Vstride;
      if (g == 1) {
        hipLaunchKernelGGL(k_cinit, dim3(1), dim3(256), 0, st, Vp, Vg, N, n, NP, ctx->cinit.as<double>(),
                           ctx->leak.as<double>());
        AQT_HIP(ctx, hipGetLastError());
      }
      if (g >= 2 && c == 0) {
        GemmArgs ga{Vg, Vp, ctx->dlt.as<double>() + static_cast<size_t>(g) * NP * NP, 0, 0, 0, n, n, N, N, N, NP, 0, nq, 1};
        aqt_status s = launch_gemm(ctx, ga, 1);
        if (s != AQT_OK) return s;
      }
    }
    {
      // batched overlaps for the grid points whose predecessor is in the chunk
      const int first = std::max(1, (g0 == 0) ? 2 : 1);   // chunk-local index
      const int count = cnt - first;
      if (count > 0) {
        GemmArgs ga{Vc.as<double>() + first * Vstride, Vc.as<double>() + (first - 1) * Vstride,
                    ctx->dlt.as<double>() + static_cast<size_t>(g0 + first) * NP * NP, static_cast<int64_t>(Vstride),
                    static_cast<int64_t>(Vstride), static_cast<int64_t>(NP) * NP, n, n, N, N, N, NP, 0, nq, 1};
        aqt_status s = launch_gemm(ctx, ga, count);
        if (s != AQT_OK) return s;
      }
    }
    const int pg0 = std::max(g0, 2), pcnt = g0 + cnt - pg0;
    if (pcnt > 0) {
      if (n < N) {
        hipLaunchKernelGGL(k_polar, dim3(pcnt), dim3(kEigThreads), 0, st, ctx->dlt.as<double>(), NP, n, pg0,
                           ctx->leak.as<double>(), pws.as<double>(), status.as<int>() + (pg0 - g0));
      } else {
        hipLaunchKernelGGL(k_leak_columns, dim3(nblk(pcnt, 64)), dim3(64), 0, st, ctx->dlt.as<double>(), NP, n,
                           pg0, pcnt, ctx->leak.as<double>());
      }
      AQT_HIP(ctx, hipGetLastError());
    }
    // matrix elements z_i = V diag(sz_i) V^T and rate tables for g >= 1
    const int zg0 = std::max(g0, 1), zcnt = g0 + cnt - zg0;
    if (zcnt > 0) {
      const int off = zg0 - g0;
      aqt_status s = AQT_OK;
      if (sx) {
        // z_k = V^T (O_k V): the operands O_k V, then one product per (grid point, channel)
        hipLaunchKernelGGL(k_channel_rows, dim3(nblk(static_cast<int64_t>(zcnt) * nch * n * N)), dim3(256), 0, st,
                           Vc.as<double>() + off * Vstride, static_cast<int64_t>(Vstride), N, nq, n, zcnt, nch,
                           chw.as<double>(), cxv.as<double>(), Yc.as<double>());
        AQT_HIP(ctx, hipGetLastError());
        GemmArgs ga{Vc.as<double>() + off * Vstride, Yc.as<double>(), zws.as<double>(),
                    static_cast<int64_t>(Vstride), static_cast<int64_t>(n) * N, static_cast<int64_t>(n) * n,
                    n, n, N, N, N, n, 0, nch, 0};
        ga.adiv = nch;
        s = launch_gemm(ctx, ga, zcnt * nch);
      } else {
        GemmArgs ga{Vc.as<double>() + off * Vstride, Vc.as<double>() + off * Vstride, zws.as<double>(),
                    static_cast<int64_t>(Vstride), static_cast<int64_t>(Vstride), static_cast<int64_t>(n) * n,
                    n, n, N, N, N, n, chw.p ? 4 : 1, nch, 0};
        ga.wvec = chw.as<double>();
        s = launch_gemm(ctx, ga, zcnt * nch);
      }
      if (s != AQT_OK) return s;
      hipLaunchKernelGGL(k_rates, dim3(nblk(static_cast<int64_t>(nch) * NP * NP * zcnt)), dim3(256), 0, st,
                         zws.as<double>(), ctx->E.as<double>(), n, NP, nch, zg0, zcnt, ctx->eta, wcv.as<double>(),
                         ctx->T, ctx->R.as<double>(), ctx->zdiag.as<double>());
      AQT_HIP(ctx, hipGetLastError());
      if (ctx->lamb) {
        hipLaunchKernelGGL(k_lamb_shift, dim3(nblk(static_cast<int64_t>(zcnt) * NP)), dim3(256), 0, st,
                           zws.as<double>(), ctx->E.as<double>(), n, NP, nch, zg0, zcnt, ltab, ctx->shift.as<double>());
        AQT_HIP(ctx, hipGetLastError());
      }
    }
    if (grad) {
      // V H' V^T for both directions at every grid point of the chunk, then X and de
      const int64_t nn = static_cast<int64_t>(n) * n;
      hipLaunchKernelGGL(k_hx_rows, dim3(nblk(static_cast<int64_t>(cnt) * n * N)), dim3(256), 0, st, Vc.as<double>(),
                         static_cast<int64_t>(Vstride), N, nq, n, cnt, Wx.as<double>());
      AQT_HIP(ctx, hipGetLastError());
      GemmArgs gx{Vc.as<double>(), Wx.as<double>(), Hd.as<double>(), static_cast<int64_t>(Vstride),
                  static_cast<int64_t>(n) * N, 2 * nn, n, n, N, N, N, n, 0, nq, 0};
      aqt_status s = launch_gemm(ctx, gx, cnt);
      if (s != AQT_OK) return s;
      GemmArgs gz{Vc.as<double>(), Vc.as<double>(), Hd.as<double>() + nn, static_cast<int64_t>(Vstride),
                  static_cast<int64_t>(Vstride), 2 * nn, n, n, N, N, N, n, 3, nq, 0};
      gz.wvec = eZ.as<double>();
      if ((s = launch_gemm(ctx, gz, cnt)) != AQT_OK) return s;
      hipLaunchKernelGGL(k_xmat, dim3(cnt, 2), dim3(256), 0, st, Hd.as<double>(), n, NP, ctx->E.as<double>(), g0, tol,
                         ctx->Xd.as<double>(), ctx->dE.as<double>());
      AQT_HIP(ctx, hipGetLastError());
      if (g0 <= 1 && g0 + cnt > 1) {
        const int c1 = 1 - g0;
        const double* V1 = Vc.as<double>() + c1 * Vstride;
        const double* V0 = (c1 == 0) ? Vprev.as<double>() : Vc.as<double>() + (c1 - 1) * Vstride;
        hipLaunchKernelGGL(k_dcinit, dim3(1), dim3(256), 0, st, V0, V1, ctx->Xd.as<double>(), N, n, NP,
                           ctx->dcin.as<double>());
        AQT_HIP(ctx, hipGetLastError());
      }
      if (zcnt > 0) {
        for (int dir = 0; dir < 2; ++dir) {
          GemmArgs gq{zws.as<double>(), ctx->Xd.as<double>() + (static_cast<size_t>(zg0) * 2 + dir) * NP * NP,
                      Qz.as<double>() + static_cast<size_t>(dir) * zcnt * nch * nn, nn,
                      2 * static_cast<int64_t>(NP) * NP, nn, n, n, n, n, NP, n, 0, nch, 0};
          gq.bdiv = nch;
          if ((s = launch_gemm(ctx, gq, zcnt * nch)) != AQT_OK) return s;
        }
        hipLaunchKernelGGL(k_dtables, dim3(nblk(static_cast<int64_t>(zcnt) * 2 * NP)), dim3(256), 0, st,
                           zws.as<double>(), Qz.as<double>(), ctx->E.as<double>(), ctx->dE.as<double>(), n, NP, nch,
                           zg0, zcnt, ctx->eta, wcv.as<double>(), ctx->T, ctx->dGam.as<double>(), ctx->dzd.as<double>(),
                           ctx->dll.as<double>());
        AQT_HIP(ctx, hipGetLastError());
        if (ctx->lamb) {
          hipLaunchKernelGGL(k_lamb_dshift, dim3(nblk(static_cast<int64_t>(zcnt) * 2 * NP)), dim3(256), 0, st,
                             zws.as<double>(), Qz.as<double>(), ctx->E.as<double>(), ctx->dE.as<double>(), n, NP, nch,
                             zg0, zcnt, ltab, ctx->dshift.as<double>());
          AQT_HIP(ctx, hipGetLastError());
        }
      }
    }
    AQT_HIP(ctx, hipMemcpyAsync(Vprev.p, Vc.as<double>() + (cnt - 1) * Vstride, Vstride * 8, hipMemcpyDeviceToDevice, st));
    AQT_HIP(ctx, hipMemcpyAsync(hstat.data(), status.p, cnt * 4, hipMemcpyDeviceToHost, st));
    AQT_HIP(ctx, hipStreamSynchronize(st));
    for (int c = 0; c < cnt; ++c)
      if (hstat[c]) return ctx->fail(AQT_ENUMERIC, "polar factor eigensolver failed at grid " + std::to_string(g0 + c));
  }
  ctx->have_grad = grad;
  return AQT_OK;
}

}  // namespace aqt
