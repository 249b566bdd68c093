// Derived tables and MFMA operand packing for the trajectory kernel.
//
// finish_tables: Gamma_b = sum_{i,a} R[i][b][a], the diagonal of
//   sum_i A_i^dag A_i (Sec. III eq. Heff with the rates absorbed, eq. Aired),
//   with, per (qubit, source level), the row sum, the partial sum below the
//   diagonal and the diagonal element kept for the two-stage channel draw,
//   and d_b = exp(-i e_b dt - Gamma_b dt / 2), the no-jump propagator over one
//   step of the diagonal effective Hamiltonian (Sec. III eq. detun).
// pack_for_precision: Delta = O - I rearranged into 16x16 MFMA A-operand
//   fragments (64 lanes contiguous) in the state precision; for BF16 two
//   fragment sets (hi, lo) with Delta ~ hi + lo (K = 32 fragments, or K = 16
//   fragments when only 16 levels are kept).
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "common.hpp"
#include "ctx.hpp"

namespace aqt {
namespace {

__global__ void k_gamma_phase(const double* __restrict__ E, const double* __restrict__ shift,
                              const double* __restrict__ R, int M, int NP, int n,
                              int nq, const double* __restrict__ tlen, double* __restrict__ Gamma,
                              double* __restrict__ Rcol,
                              double* __restrict__ ehalf, double* __restrict__ dre, double* __restrict__ dim) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<int64_t>(M) * NP) return;
  const int g = static_cast<int>(idx / NP);
  const int b = static_cast<int>(idx - static_cast<int64_t>(g) * NP);
  const double dt = tlen[g];   // length of the step into grid g
  double G = 0.0;
  for (int i = 0; i < nq; ++i) {
    double rs = 0.0, lo = 0.0, dg = 0.0;
    if (b < n) {
      const double* row = R + ((static_cast<size_t>(g) * nq + i) * NP + b) * NP;
      for (int a = 0; a < n; ++a) {
        if (a == b) {
          lo = rs;
          dg = row[a];
        }
        rs += row[a];
      }
    }
    double* out = Rcol + ((static_cast<size_t>(g) * nq + i) * NP + b) * 4;
    out[0] = rs;
    out[1] = lo;
    out[2] = dg;
    out[3] = 0.0;
    G += rs;
  }
  Gamma[idx] = G;
  if (b < n) {
    double sn, cs;
    sincos((E[idx] + shift[idx]) * dt, &sn, &cs);   // phases of H_S + H_LS
    const double mag = exp(-0.5 * G * dt);
    dre[idx] = mag * cs;
    dim[idx] = -mag * sn;
    ehalf[idx] = exp(0.5 * G * dt);
  } else {
    dre[idx] = 0.0;
    dim[idx] = 0.0;
    ehalf[idx] = 0.0;
  }
}

template <class T>
__global__ void k_pack_k4(const double* __restrict__ dlt, int M, int NP, T* __restrict__ out) {
  // out[((g*NRT + rt)*(NP/4) + kc)*64 + l] = Delta[g][16 rt + l%16][4 kc + l/16]
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t per_g = static_cast<int64_t>(NP) * NP;
  if (idx >= per_g * M) return;
  const int g = static_cast<int>(idx / per_g);
  int64_t r = idx - g * per_g;
  const int l = static_cast<int>(r & 63);
  r >>= 6;
  const int kc = static_cast<int>(r % (NP / 4));
  const int rt = static_cast<int>(r / (NP / 4));
  const int row = 16 * rt + (l & 15);
  const int col = 4 * kc + (l >> 4);
  out[idx] = static_cast<T>(dlt[(static_cast<size_t>(g) * NP + row) * NP + col]);
}

__device__ __forceinline__ uint32_t bf16_rne_bits(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}

__global__ void k_pack_bf16(const double* __restrict__ dlt, int M, int NP, uint4* __restrict__ hi,
                            uint4* __restrict__ lo) {
  // fragment (g, rt, kc, l) holds Delta[g][16 rt + l%16][32 kc + 8 (l/16) + j], j = 0..7
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t per_g = static_cast<int64_t>(NP) * NP / 8;
  if (idx >= per_g * M) return;
  const int g = static_cast<int>(idx / per_g);
  int64_t r = idx - g * per_g;
  const int l = static_cast<int>(r & 63);
  r >>= 6;
  const int kc = static_cast<int>(r % (NP / 32));
  const int rt = static_cast<int>(r / (NP / 32));
  const int row = 16 * rt + (l & 15);
  const int col0 = 32 * kc + 8 * (l >> 4);
  uint32_t h[4], w[4];
  for (int j = 0; j < 4; ++j) {
    uint32_t hb[2], lb[2];
    for (int e = 0; e < 2; ++e) {
      const double x = dlt[(static_cast<size_t>(g) * NP + row) * NP + col0 + 2 * j + e];
      const uint32_t hh = bf16_rne_bits(static_cast<float>(x));
      const double rest = x - static_cast<double>(__uint_as_float(hh << 16));
      hb[e] = hh;
      lb[e] = bf16_rne_bits(static_cast<float>(rest));
    }
    h[j] = hb[0] | (hb[1] << 16);
    w[j] = lb[0] | (lb[1] << 16);
  }
  hi[idx] = make_uint4(h[0], h[1], h[2], h[3]);
  lo[idx] = make_uint4(w[0], w[1], w[2], w[3]);
}

__global__ void k_pack_bf16_k16(const double* __restrict__ dlt, int M, int NP, uint2* __restrict__ hi,
                                uint2* __restrict__ lo) {
  // fragment (g, rt, kc, l) holds Delta[g][16 rt + l%16][16 kc + 4 (l/16) + j], j = 0..3
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t per_g = static_cast<int64_t>(NP) * NP / 4;
  if (idx >= per_g * M) return;
  const int g = static_cast<int>(idx / per_g);
  int64_t r = idx - g * per_g;
  const int l = static_cast<int>(r & 63);
  r >>= 6;
  const int kc = static_cast<int>(r % (NP / 16));
  const int rt = static_cast<int>(r / (NP / 16));
  const int row = 16 * rt + (l & 15);
  const int col0 = 16 * kc + 4 * (l >> 4);
  uint32_t h[2], w[2];
  for (int j = 0; j < 2; ++j) {
    uint32_t hb[2], lb[2];
    for (int e = 0; e < 2; ++e) {
      const double x = dlt[(static_cast<size_t>(g) * NP + row) * NP + col0 + 2 * j + e];
      const uint32_t hh = bf16_rne_bits(static_cast<float>(x));
      const double rest = x - static_cast<double>(__uint_as_float(hh << 16));
      hb[e] = hh;
      lb[e] = bf16_rne_bits(static_cast<float>(rest));
    }
    h[j] = hb[0] | (hb[1] << 16);
    w[j] = lb[0] | (lb[1] << 16);
  }
  hi[idx] = make_uint2(h[0], h[1]);
  lo[idx] = make_uint2(w[0], w[1]);
}

__global__ void k_to_f32(const double* __restrict__ in, float* __restrict__ out, int64_t count) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx < count) out[idx] = static_cast<float>(in[idx]);
}

inline unsigned blocks_for(int64_t count, int threads = 256) {
  return static_cast<unsigned>((count + threads - 1) / threads);
}

}  // namespace

// Largest Gamma_b dt_g over all grid points g >= 1 and levels (one workgroup; Gamma >= 0,
// so the maximum of the bit patterns is the maximum of the values).
// The jump handler's per-channel numbers in the FP32 state precision, one 16-byte
// entry per (grid, channel, level): row sum of R, its part below the diagonal, the
// diagonal, and the dephasing factor z_bb.
__global__ void k_pack_chan(const double* __restrict__ Rcol, const double* __restrict__ zdiag, int64_t count,
                            float4* __restrict__ out) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= count) return;
  const double* c = Rcol + idx * 4;
  out[idx] = make_float4(static_cast<float>(c[0]), static_cast<float>(c[1]), static_cast<float>(c[2]),
                         static_cast<float>(zdiag[idx]));
}

__global__ void k_max_gdt(const double* __restrict__ Gamma, const double* __restrict__ tlen, int M, int NP,
                          double* __restrict__ out) {
  __shared__ double red[256];
  double v = 0.0;
  for (int64_t i = static_cast<int64_t>(NP) + threadIdx.x; i < static_cast<int64_t>(M) * NP; i += blockDim.x)
    v = fmax(v, Gamma[i] * tlen[i / NP]);
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

aqt_status check_step_decay(aqt_ctx* ctx, int precision) {
  const double lim = precision == AQT_FP64 ? 500.0 : 50.0;
  if (!(ctx->max_gdt <= lim))
    return ctx->fail(AQT_ENUMERIC, "a level decays by Gamma dt = " + std::to_string(ctx->max_gdt) +
                                       " within one step, beyond the " + std::to_string(lim) +
                                       " this precision carries; use more grid points");
  return AQT_OK;
}

aqt_status finish_tables(aqt_ctx* ctx) {
  const int M = ctx->M;
  const int64_t cnt = static_cast<int64_t>(M) * ctx->NP;
  // grid points and steps: s_g = g / (M - 1) with steps t_f / (M - 1) starting at (g - 1) dt,
  // or the grid of aqt_set_grid, where the step of grid point g has length (h_g + h_{g+1}) / 2,
  // h_g = t_f (s_g - s_{g-1}), and starts at t_f (s_{g-1} + s_g - s_1) / 2
  if (!ctx->sgrid.empty() && static_cast<int>(ctx->sgrid.size()) != M)
    return ctx->fail(AQT_EINVAL, "the grid of aqt_set_grid has a different number of points");
  std::vector<double> sg(M), tb(M, 0.0), tl(M, 0.0);
  for (int g = 0; g < M; ++g) {
    if (ctx->sgrid.empty()) {
      sg[g] = static_cast<double>(g) / (M - 1);
      if (g > 0) tb[g] = (g - 1) * ctx->dt, tl[g] = ctx->dt;
    } else {
      // grid point g's factor covers half of each neighbouring step (the last point also
      // the half step the first leaves out): a symmetric splitting of every step
      sg[g] = ctx->sgrid[g];
      if (g > 0) {
        const double s_next = (g < M - 1) ? ctx->sgrid[g + 1] : 1.0 + ctx->sgrid[1];
        tb[g] = 0.5 * ctx->t_f * (ctx->sgrid[g - 1] + ctx->sgrid[g] - ctx->sgrid[1]);
        tl[g] = 0.5 * ctx->t_f * (s_next - ctx->sgrid[g - 1]);
      }
    }
  }
  if (ctx->sgd.reserve(M * sizeof(double)) != hipSuccess || ctx->tbeg.reserve(M * sizeof(double)) != hipSuccess ||
      ctx->tlen.reserve(M * sizeof(double)) != hipSuccess)
    return ctx->fail(AQT_ENOMEM, "table allocation failed");
  AQT_HIP(ctx, hipMemcpy(ctx->sgd.p, sg.data(), M * sizeof(double), hipMemcpyHostToDevice));
  AQT_HIP(ctx, hipMemcpy(ctx->tbeg.p, tb.data(), M * sizeof(double), hipMemcpyHostToDevice));
  AQT_HIP(ctx, hipMemcpy(ctx->tlen.p, tl.data(), M * sizeof(double), hipMemcpyHostToDevice));
  if (ctx->Gamma.reserve(cnt * sizeof(double)) != hipSuccess || ctx->dre.reserve(cnt * sizeof(double)) != hipSuccess ||
      ctx->dim.reserve(cnt * sizeof(double)) != hipSuccess ||
      ctx->Rcol.reserve(cnt * ctx->tab_nch * 4 * sizeof(double)) != hipSuccess ||
      ctx->ehalf.reserve(cnt * sizeof(double)) != hipSuccess)
    return ctx->fail(AQT_ENOMEM, "table allocation failed");
  hipLaunchKernelGGL(k_gamma_phase, dim3(blocks_for(cnt)), dim3(256), 0, ctx->stream, ctx->E.as<double>(),
                     ctx->shift.as<double>(), ctx->R.as<double>(), ctx->M, ctx->NP, ctx->n, ctx->tab_nch, ctx->tlen.as<double>(), ctx->Gamma.as<double>(),
                     ctx->Rcol.as<double>(), ctx->ehalf.as<double>(), ctx->dre.as<double>(), ctx->dim.as<double>());
  AQT_HIP(ctx, hipGetLastError());
  {
    DevBuf mx;
    if (mx.reserve(sizeof(double)) != hipSuccess) return ctx->fail(AQT_ENOMEM, "table allocation failed");
    hipLaunchKernelGGL(k_max_gdt, dim3(1), dim3(256), 0, ctx->stream, ctx->Gamma.as<double>(), ctx->tlen.as<double>(),
                       ctx->M, ctx->NP, mx.as<double>());
    AQT_HIP(ctx, hipGetLastError());
    AQT_HIP(ctx, hipMemcpyAsync(&ctx->max_gdt, mx.p, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    AQT_HIP(ctx, hipStreamSynchronize(ctx->stream));
  }
  ctx->packed_for = -1;
  ctx->fix_prec = -1;
  return AQT_OK;
}

aqt_status pack_for_precision(aqt_ctx* ctx, int precision) {
  if (ctx->packed_for == precision) return AQT_OK;
  const int64_t nd = static_cast<int64_t>(ctx->M) * ctx->NP * ctx->NP;
  const int64_t nv = static_cast<int64_t>(ctx->M) * ctx->NP;
  ctx->pk_a.release();
  ctx->pk_b.release();
  ctx->pk_dre.release();
  ctx->pk_dim.release();
  ctx->pk_ch.release();
  if (precision == AQT_FP64) {
    if (ctx->pk_a.reserve(nd * 8) != hipSuccess || ctx->pk_dre.reserve(nv * 8) != hipSuccess ||
        ctx->pk_dim.reserve(nv * 8) != hipSuccess)
      return ctx->fail(AQT_ENOMEM, "operand allocation failed");
    hipLaunchKernelGGL(k_pack_k4<double>, dim3(blocks_for(nd)), dim3(256), 0, ctx->stream, ctx->dlt.as<double>(),
                       ctx->M, ctx->NP, ctx->pk_a.as<double>());
    AQT_HIP(ctx, hipMemcpyAsync(ctx->pk_dre.p, ctx->dre.p, nv * 8, hipMemcpyDeviceToDevice, ctx->stream));
    AQT_HIP(ctx, hipMemcpyAsync(ctx->pk_dim.p, ctx->dim.p, nv * 8, hipMemcpyDeviceToDevice, ctx->stream));
  } else {
    if (ctx->pk_dre.reserve(nv * 4) != hipSuccess || ctx->pk_dim.reserve(nv * 4) != hipSuccess)
      return ctx->fail(AQT_ENOMEM, "operand allocation failed");
    if (precision == AQT_FP32) {
      if (ctx->pk_a.reserve(nd * 4) != hipSuccess) return ctx->fail(AQT_ENOMEM, "operand allocation failed");
      hipLaunchKernelGGL(k_pack_k4<float>, dim3(blocks_for(nd)), dim3(256), 0, ctx->stream, ctx->dlt.as<double>(),
                         ctx->M, ctx->NP, ctx->pk_a.as<float>());
      if (ctx->NP >= 128) {   // the level counts whose FP32 kernels stage the channel entries
        const int64_t nc = nv * ctx->tab_nch;
        if (ctx->pk_ch.reserve(nc * sizeof(float4)) != hipSuccess)
          return ctx->fail(AQT_ENOMEM, "operand allocation failed");
        hipLaunchKernelGGL(k_pack_chan, dim3(blocks_for(nc)), dim3(256), 0, ctx->stream, ctx->Rcol.as<double>(),
                           ctx->zdiag.as<double>(), nc, ctx->pk_ch.as<float4>());
      }
    } else if (precision == AQT_BF16) {
      if (ctx->pk_a.reserve(nd * 2) != hipSuccess || ctx->pk_b.reserve(nd * 2) != hipSuccess)
        return ctx->fail(AQT_ENOMEM, "operand allocation failed");
      if (ctx->NP == 16)
        hipLaunchKernelGGL(k_pack_bf16_k16, dim3(blocks_for(nd / 4)), dim3(256), 0, ctx->stream,
                           ctx->dlt.as<double>(), ctx->M, ctx->NP, ctx->pk_a.as<uint2>(), ctx->pk_b.as<uint2>());
      else
        hipLaunchKernelGGL(k_pack_bf16, dim3(blocks_for(nd / 8)), dim3(256), 0, ctx->stream,
                           ctx->dlt.as<double>(), ctx->M, ctx->NP, ctx->pk_a.as<uint4>(), ctx->pk_b.as<uint4>());
    } else {
      return ctx->fail(AQT_EINVAL, "unknown precision");
    }
    AQT_HIP(ctx, hipGetLastError());
    hipLaunchKernelGGL(k_to_f32, dim3(blocks_for(nv)), dim3(256), 0, ctx->stream, ctx->dre.as<double>(),
                       ctx->pk_dre.as<float>(), nv);
    hipLaunchKernelGGL(k_to_f32, dim3(blocks_for(nv)), dim3(256), 0, ctx->stream, ctx->dim.as<double>(),
                       ctx->pk_dim.as<float>(), nv);
  }
  AQT_HIP(ctx, hipGetLastError());
  ctx->packed_for = precision;
  return AQT_OK;
}

}  // namespace aqt
