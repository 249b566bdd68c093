// Tile products shared by the sweep kernels (gradient, fixed-step unraveling): a
// workgroup of kGW wavefronts holds TT trajectories as an LDS tile [NP][LD] (columns
// 2t, 2t + 1 = re, im of trajectory t) and multiplies it by NP x NP operands read from
// global memory on MFMA (FP32 or FP64 16x16x4).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace aqt {
namespace tile {

constexpr int kGW = 8;              // wavefronts per workgroup
constexpr int kGThreads = kGW * 64;

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));

template <class T> struct Mfma;
template <> struct Mfma<float> {
  using acc_t = f4;
  __device__ static acc_t zero() { return f4{0.f, 0.f, 0.f, 0.f}; }
  __device__ static acc_t step(float a, float b, acc_t c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  // element e of lane l holds output row 4 (l / 16) + e, column l % 16
  __device__ static int row(int lane, int e) { return 4 * (lane >> 4) + e; }
};
template <> struct Mfma<double> {
  using acc_t = d4;
  __device__ static acc_t zero() { return d4{0.0, 0.0, 0.0, 0.0}; }
  __device__ static acc_t step(double a, double b, acc_t c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  // element e of lane l holds output row l / 16 + 4 e, column l % 16
  __device__ static int row(int lane, int e) { return (lane >> 4) + 4 * e; }
};

// Operand A of the products below: an NP x NP row-major matrix in the state precision
// (packed copies of O_g - I, its transpose and X_g), read straight into registers.  Each
// wave owns whole 16-row tiles; lane (r, q) of the 16 x 4 fragment grid loads VW
// consecutive entries A[row][k..k+VW) with one 16-byte load, so one MFMA step takes
// k = 4 VW j + VW q + e (e < VW) from lane q: any bijection of k onto (step, lane
// group) is a valid contraction as long as A and B use the same one.
template <class T> struct Vec;
template <> struct Vec<float> { using t = float __attribute__((ext_vector_type(4))); static constexpr int W = 4; };
template <> struct Vec<double> { using t = double __attribute__((ext_vector_type(2))); static constexpr int W = 2; };

// acc[b][ct] += A[rows of tile rt][:] * B_b[:, columns of tile ct] for NB LDS operands.
template <int NP, int NC, int LD, class T, int NB>
__device__ __forceinline__ void panel_mma(const T* __restrict__ A, int rt, const T* const (&B)[NB],
                                          typename Mfma<T>::acc_t (&acc)[NB][NC / 16]) {
  constexpr int VW = Vec<T>::W;
  constexpr int NJ = NP / (4 * VW);                // vector loads per lane for the whole panel
  // loads kept in flight: the whole FP32 panel row at 256 levels (one workgroup per CU
  // leaves little else to hide their latency), 8 in FP64 (no gain there, more registers)
  constexpr int JMAX = (sizeof(T) == 4) ? 16 : 8;
  constexpr int JCH = (NJ < JMAX) ? NJ : JMAX;
  using V = typename Vec<T>::t;
  const int lane = threadIdx.x & 63, q = lane >> 4, c = lane & 15;
  const V* arow = reinterpret_cast<const V*>(A + static_cast<size_t>(rt * 16 + c) * NP) + q;
#pragma unroll 1
  for (int j0 = 0; j0 < NJ; j0 += JCH) {
    V av[JCH];
#pragma unroll
    for (int u = 0; u < JCH; ++u) av[u] = arow[(j0 + u) * 4];
#pragma unroll
    for (int u = 0; u < JCH; ++u)
#pragma unroll
      for (int e = 0; e < VW; ++e) {
        const int k = (j0 + u) * 4 * VW + q * VW + e;
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
          for (int ct = 0; ct < NC / 16; ++ct)
            acc[b][ct] = Mfma<T>::step(av[u][e], B[b][k * LD + ct * 16 + c], acc[b][ct]);
      }
  }
}

// Y = (I + A) B over NP x NC (A = O_g - I or its transpose); B and Y in LDS, Y != B.
template <int NP, int NC, int LD, class T>
__device__ void gemm_kick(const T* __restrict__ A, const T* B, T* Y) {
  constexpr int RT = NP / 16, CT = NC / 16;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, c = lane & 15;
  const T* const Bs[1] = {B};
  for (int rt = wave; rt < RT; rt += kGW) {
    typename Mfma<T>::acc_t acc[1][CT];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[0][ct] = Mfma<T>::zero();
    panel_mma<NP, NC, LD, T, 1>(A, rt, Bs, acc);
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = rt * 16 + Mfma<T>::row(lane, e), col = ct * 16 + c;
        Y[r * LD + col] = acc[0][ct][e] + B[r * LD + col];
      }
  }
}

// Y1 = (I + A) B1 and Y2 = (I + A) B2 with one pass over A (the panel loads are shared);
// each product is accumulated in the same order as gemm_kick's.
template <int NP, int NC, int LD, class T>
__device__ void gemm_kick2(const T* __restrict__ A, const T* B1, T* Y1, const T* B2, T* Y2) {
  constexpr int RT = NP / 16, CT = NC / 16;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, c = lane & 15;
  const T* const Bs[2] = {B1, B2};
  for (int rt = wave; rt < RT; rt += kGW) {
    typename Mfma<T>::acc_t acc[2][CT];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) acc[b][ct] = Mfma<T>::zero();
    panel_mma<NP, NC, LD, T, 2>(A, rt, Bs, acc);
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = rt * 16 + Mfma<T>::row(lane, e), col = ct * 16 + c;
        Y1[r * LD + col] = acc[0][ct][e] + B1[r * LD + col];
        Y2[r * LD + col] = acc[1][ct][e] + B2[r * LD + col];
      }
  }
}

// Copies between an LDS state tile (leading dimension LD) and a dense [NP][NC] block.
template <int NP, int NC, int LD, class T>
__device__ void tile_store(const T* src, T* __restrict__ dst) {
  for (int f = threadIdx.x; f < NP * NC; f += kGThreads) dst[f] = src[(f / NC) * LD + (f % NC)];
}
template <int NP, int NC, int LD, class T>
__device__ void tile_load(const T* __restrict__ src, T* dst) {
  for (int f = threadIdx.x; f < NP * NC; f += kGThreads) dst[(f / NC) * LD + (f % NC)] = src[f];
}

}  // namespace tile
}  // namespace aqt
