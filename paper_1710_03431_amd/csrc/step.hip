// Persistent trajectory kernel: batched quantum-jump stepping in the
// instantaneous eigenbasis (Sec. IV waiting-time procedure; App. C validity;
// jump-type law App. B eq. Pi(t); jump update Sec. III eq. jump).
//
// One workgroup (4 waves) owns a tile of TT = 16*TQ trajectories for the whole
// anneal; their amplitudes stay in LDS.  Per grid step g (from s_{g-1} to s_g):
//   1. C <- O_g C on MFMA, written as C + Delta_g C (identity split) so the
//      accumulator starts from C.  Real Delta times complex C is one real GEMM
//      on the re and im column tiles.
//   2. C' = d_g o C with d_b = exp(-i e_b dt - Gamma_b dt / 2): the no-jump
//      propagator of the diagonal H_eff (Sec. III eq. Heff), fused into the
//      GEMM epilogue together with the per-trajectory squared norm.
//   3. A trajectory whose squared norm falls to its threshold r crosses: a
//      wavefront takes it, finds the crossing time (Newton on the log of
//      sum_b |c_b|^2 e^{-Gamma_b tau}), draws the source level with weight
//      q_b Gamma_b and the (qubit, target) with weight R[i][b][a], applies the
//      jump, renormalises, records it and draws a new threshold; repeated
//      until the step's time is used up.  FP64 arithmetic in every mode.
//   4. Ground-cluster population per trajectory; per-tile sums go to a
//      [tile][g] buffer reduced afterwards in a fixed order.
// Phases of the whole step are applied in step 2; the jump path only applies
// real factors (decays, omega = 0 elements, normalisation) or collapses to a
// single level whose phase is that of d_a, which equals applying the step's
// phases at its end.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.hpp"
#include "ctx.hpp"
#include "philox.hpp"

namespace aqt {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Accumulator layouts of the 16x16 MFMAs (lane l, accumulator element i -> row;
// the column is always l % 16): the FP64 16x16x4 interleaves rows by 4, the FP32
// and BF16 variants keep four consecutive rows per lane.
struct ModeF64 {
  using T = double;
  using Acc = d4;
  static constexpr int KC = 4;
  __device__ static constexpr int row(int lane, int i) { return (lane >> 4) + 4 * i; }
};
struct ModeF32 {
  using T = float;
  using Acc = f4;
  static constexpr int KC = 4;
  __device__ static constexpr int row(int lane, int i) { return 4 * (lane >> 4) + i; }
};
struct ModeBF16 {
  using T = float;
  using Acc = f4;
  static constexpr int KC = 32;
  __device__ static constexpr int row(int lane, int i) { return 4 * (lane >> 4) + i; }
};

struct StepArgs {
  int M, n, nq;
  double dt;
  int64_t K;
  uint64_t seed, iid, traj0;
  int cap;
  const void* dlt_a;     // Delta fragments (hi for BF16)
  const void* dlt_b;     // Delta lo fragments (BF16 only)
  const void* dre;       // [M][NP] state precision
  const void* dim;
  const double* cinit;   // [NP]
  const double* Gamma;   // [M][NP]
  const double* d64re;   // [M][NP]
  const double* d64im;
  const double* R;       // [M][nq][NP][NP]
  const double* zdiag;   // [M][nq][NP]
  const double* E;       // [M][NP]
  const int* gs;         // [M]
  double* partial;       // [tiles][M][2]
  int64_t* jump_totals;
  int32_t* jump_count;
  aqt_jump* jumps;
  int32_t* net_gs;
  int64_t* net_hist;
  int hist_lo, hist_hi;
  double* final_state;
};

__device__ __forceinline__ d4 mfma_k4(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma_k4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Round-to-nearest-even FP32 -> BF16 bits (inputs are finite).
__device__ __forceinline__ uint32_t bf16_bits(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}

// hi/lo BF16 split of 8 floats: x ~ hi + lo with |x - hi - lo| <= 2^-17 |x|.
__device__ __forceinline__ void split8(const float* x, bf16x8& hi, bf16x8& lo) {
  uint32_t h[4], l[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    uint32_t h0 = bf16_bits(x[2 * j]), h1 = bf16_bits(x[2 * j + 1]);
    float r0 = x[2 * j] - __uint_as_float(h0 << 16);
    float r1 = x[2 * j + 1] - __uint_as_float(h1 << 16);
    h[j] = h0 | (h1 << 16);
    l[j] = bf16_bits(r0) | (bf16_bits(r1) << 16);
  }
  uint4 hv = make_uint4(h[0], h[1], h[2], h[3]);
  uint4 lv = make_uint4(l[0], l[1], l[2], l[3]);
  hi = __builtin_bit_cast(bf16x8, hv);
  lo = __builtin_bit_cast(bf16x8, lv);
}

// ----------------------------------------------------------- jump handler --
// One wavefront finishes step g for trajectory column t of the tile whose
// amplitudes after step 2 are in S.  Works in FP64.
template <int NP, int TQ, class T>
__device__ void finish_crossing(const StepArgs& a, int g, int t, int64_t jloc, T (*S)[TQ][NP][16],
                                double* s_r, int* s_m, int* s_cnt, int* s_net, double* s_p,
                                int* s_kind) {
  constexpr int PL = (NP + kWave - 1) / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int q = t >> 4, col = t & 15;
  const double dt = a.dt;
  const uint64_t traj = a.traj0 + static_cast<uint64_t>(jloc);   // Philox counter word 0
  const double* Gam = a.Gamma + static_cast<size_t>(g) * NP;
  double cr[PL], ci[PL], G[PL];
#pragma unroll
  for (int j = 0; j < PL; ++j) {
    const int x = lane + kWave * j;
    if (x < NP) {
      G[j] = Gam[x];
      // undo the full-step decay of step 2: keep the phases, restore magnitudes
      const double up = exp(fmin(0.5 * G[j] * dt, 700.0));
      cr[j] = static_cast<double>(S[0][q][x][col]) * up;
      ci[j] = static_cast<double>(S[1][q][x][col]) * up;
    } else {
      G[j] = 0.0;
      cr[j] = ci[j] = 0.0;
    }
  }
  double r = s_r[t];
  int m = s_m[t];
  int cnt = s_cnt[t];
  int net = s_net[t];
  const int gsz = a.gs[g];
  const double tk = (g - 1) * dt;
  double tau_e = 0.0;
  for (int guard = 0; guard < 4096; ++guard) {   // jumps within one step
    const double rem = dt - tau_e;
    double part = 0.0;
#pragma unroll
    for (int j = 0; j < PL; ++j) part += (cr[j] * cr[j] + ci[j] * ci[j]) * exp(-G[j] * rem);
    const double nu_end = wave_sum(part);
    if (nu_end > r) {
#pragma unroll
      for (int j = 0; j < PL; ++j) {
        const double f = exp(-0.5 * G[j] * rem);
        cr[j] *= f;
        ci[j] *= f;
      }
      break;
    }
    // crossing time: Newton on log sum_b w_b e^{-G_b tau} = log r from tau = 0
    double w[PL];
#pragma unroll
    for (int j = 0; j < PL; ++j) w[j] = cr[j] * cr[j] + ci[j] * ci[j];
    double tau = 0.0;
    const double logr = log(r);
    for (int it = 0; it < 100; ++it) {
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int j = 0; j < PL; ++j) {
        const double e = w[j] * exp(-G[j] * tau);
        s0 += e;
        s1 += G[j] * e;
      }
      s0 = wave_sum(s0);
      s1 = wave_sum(s1);
      const double f = log(s0) - logr;
      const double fp = -s1 / s0;
      if (fp == 0.0) {
        tau = rem;
        break;
      }
      const double stp = -f / fp;
      if (!(stp > 0.0)) break;
      const double tn = fmin(tau + stp, rem);
      if (tn - tau <= 1e-15 * dt) {
        tau = tn;
        break;
      }
      tau = tn;
      if (tau >= rem) break;
    }
#pragma unroll
    for (int j = 0; j < PL; ++j) {
      const double f = exp(-0.5 * G[j] * tau);
      cr[j] *= f;
      ci[j] *= f;
    }
    tau_e += tau;
    const double u1 = draw_uniform(a.seed, a.iid, traj, 3ull * m + 1);
    const double u2 = draw_uniform(a.seed, a.iid, traj, 3ull * m + 2);
    // source level b: first index whose running sum of q_b Gamma_b exceeds u1 * total
    int b = -1;
    {
      double wq[PL], carry = 0.0;
#pragma unroll
      for (int j = 0; j < PL; ++j) wq[j] = (cr[j] * cr[j] + ci[j] * ci[j]) * G[j];
      double tot = 0.0;
#pragma unroll
      for (int j = 0; j < PL; ++j) tot += wq[j];
      tot = wave_sum(tot);
      const double thr = u1 * tot;
      int lastpos = -1;
#pragma unroll
      for (int j = 0; j < PL; ++j) {
        const double cum = wave_inclusive_scan(wq[j]) + carry;
        carry = __shfl(cum, kWave - 1, kWave);
        const uint64_t hit = __ballot(cum > thr);
        if (b < 0 && hit) b = first_set_lane(hit) + kWave * j;
        const uint64_t pos = __ballot(wq[j] > 0.0);
        if (pos) lastpos = last_set_lane(pos) + kWave * j;
      }
      if (b < 0) b = lastpos;
    }
    if (b < 0) {
      // no populated level decays (a rounding-level crossing): nothing can jump
#pragma unroll
      for (int j = 0; j < PL; ++j) {
        const double f = exp(-0.5 * G[j] * (dt - tau_e));
        cr[j] *= f;
        ci[j] *= f;
      }
      break;
    }
    // qubit i and target a: running sum over R[g][i][b][a], i-major, a-minor
    int qi = 0, ta = b;
    {
      const int nf = a.nq * NP;
      const double* Rg = a.R + static_cast<size_t>(g) * a.nq * NP * NP;
      double tot = 0.0;
      for (int f = lane; f < nf; f += kWave) {
        const int i = f / NP, x = f - i * NP;
        tot += Rg[(static_cast<size_t>(i) * NP + b) * NP + x];
      }
      tot = wave_sum(tot);
      const double thr = u2 * tot;
      double carry = 0.0;
      int hitf = -1, lastpos = -1;
      for (int f0 = 0; f0 < nf; f0 += kWave) {
        const int f = f0 + lane;
        double v = 0.0;
        if (f < nf) {
          const int i = f / NP, x = f - i * NP;
          v = Rg[(static_cast<size_t>(i) * NP + b) * NP + x];
        }
        const double cum = wave_inclusive_scan(v) + carry;
        carry = __shfl(cum, kWave - 1, kWave);
        const uint64_t pos = __ballot(v > 0.0);
        if (pos) lastpos = f0 + last_set_lane(pos);
        const uint64_t hit = __ballot(cum > thr);
        if (hit) {
          hitf = f0 + first_set_lane(hit);
          break;
        }
      }
      if (hitf < 0) hitf = lastpos;
      if (hitf < 0) hitf = b;   // empty row cannot happen when q_b Gamma_b > 0; stay in range anyway
      qi = hitf / NP;
      ta = hitf - qi * NP;
    }
    int kind;
    if (ta != b) {
      // collapse to level ta, carrying the step phase e^{-i e_a dt}
      const double pr = a.d64re[static_cast<size_t>(g) * NP + ta];
      const double pim = a.d64im[static_cast<size_t>(g) * NP + ta];
      const double inv = 1.0 / sqrt(pr * pr + pim * pim);
#pragma unroll
      for (int j = 0; j < PL; ++j) {
        const int x = lane + kWave * j;
        cr[j] = (x == ta) ? pr * inv : 0.0;
        ci[j] = (x == ta) ? pim * inv : 0.0;
      }
      const double* Eg = a.E + static_cast<size_t>(g) * NP;
      kind = (Eg[ta] <= Eg[b]) ? AQT_KIND_RELAX : AQT_KIND_EXCITE;
      if (ta < gsz && b >= gsz) ++net;
      else if (b < gsz && ta >= gsz) --net;
    } else {
      const double* zd = a.zdiag + (static_cast<size_t>(g) * a.nq + qi) * NP;
#pragma unroll
      for (int j = 0; j < PL; ++j) {
        const int x = lane + kWave * j;
        const double z = (x < NP) ? zd[x] : 0.0;
        cr[j] *= z;
        ci[j] *= z;
      }
      kind = AQT_KIND_DEPHASE;
    }
    double nrm = 0.0;
#pragma unroll
    for (int j = 0; j < PL; ++j) nrm += cr[j] * cr[j] + ci[j] * ci[j];
    nrm = wave_sum(nrm);
    const double inv = 1.0 / sqrt(nrm);
#pragma unroll
    for (int j = 0; j < PL; ++j) {
      cr[j] *= inv;
      ci[j] *= inv;
    }
    if (lane == 0) {
      if (cnt < a.cap && a.jumps) {
        aqt_jump rec;
        rec.t = tk + tau_e;
        rec.step = g - 1;
        rec.qubit = static_cast<int16_t>(qi);
        rec.kind = static_cast<int16_t>(kind);
        rec.from_level = b;
        rec.to_level = ta;
        a.jumps[jloc * a.cap + cnt] = rec;
      }
      atomicAdd(&s_kind[kind], 1);
    }
    ++cnt;
    ++m;
    r = draw_uniform(a.seed, a.iid, traj, 3ull * m);
  }
  double pg = 0.0, pt = 0.0;
#pragma unroll
  for (int j = 0; j < PL; ++j) {
    const int x = lane + kWave * j;
    const double w2 = cr[j] * cr[j] + ci[j] * ci[j];
    pt += w2;
    if (x < gsz) pg += w2;
    if (x < NP) {
      S[0][q][x][col] = static_cast<T>(cr[j]);
      S[1][q][x][col] = static_cast<T>(ci[j]);
    }
  }
  pg = wave_sum(pg);
  pt = wave_sum(pt);
  if (lane == 0) {
    s_p[t] = pg / pt;
    s_r[t] = r;
    s_m[t] = m;
    s_cnt[t] = cnt;
    s_net[t] = net;
  }
}

// --------------------------------------------------------------- kernel ----
template <int NP, int TQ, class Mode>
__global__ __launch_bounds__(256) void k_trajectories(StepArgs a) {
  using T = typename Mode::T;
  using Acc = typename Mode::Acc;
  constexpr int NRT = NP / 16;
  constexpr int TT = 16 * TQ;
  constexpr int QG = (NRT >= 4) ? TQ : 1;          // column groups per work unit
  constexpr int NUNITS = NRT * (TQ / QG);
  constexpr int UPW = (NUNITS + 3) / 4;            // units per wave
  static_assert(TT <= kWave, "tile must fit one wavefront for the decision pass");

  __shared__ T S[2][TQ][NP][16];
  __shared__ T s_nu[NRT][TT];
  __shared__ T s_gw[NRT][TT];
  __shared__ double s_r[TT];
  __shared__ double s_p[TT];
  __shared__ int s_m[TT], s_cnt[TT], s_net[TT];
  __shared__ int s_list[TT];
  __shared__ int s_nlist;
  __shared__ int s_kind[3];

  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = tid >> 6;
  const int64_t tile = blockIdx.x;
  const int64_t tb = tile * TT;

  if (tid < TT) {
    const int64_t j = tb + tid;
    s_r[tid] = (j < a.K) ? draw_uniform(a.seed, a.iid, a.traj0 + j, 0) : 2.0;
    s_m[tid] = 0;
    s_cnt[tid] = 0;
    s_net[tid] = 0;
  }
  if (tid < 3) s_kind[tid] = 0;

  Acc acc[UPW][QG][2];
  const int lc = lane & 15;         // output column (trajectory) within a column tile

  for (int g = 1; g < a.M; ++g) {
    const int gsz = a.gs[g];
    // ---- 1. C + Delta C (or the initial state at g = 1)
#pragma unroll
    for (int u = 0; u < UPW; ++u) {
      const int unit = wave + 4 * u;
      if (unit >= NUNITS) break;
      const int rt = unit % NRT;
      const int q0 = (unit / NRT) * QG;
#pragma unroll
      for (int qq = 0; qq < QG; ++qq) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = rt * 16 + Mode::row(lane, i);
          if (g == 1) {
            acc[u][qq][0][i] = static_cast<T>(a.cinit[row]);
            acc[u][qq][1][i] = T(0);
          } else {
            acc[u][qq][0][i] = S[0][q0 + qq][row][lc];
            acc[u][qq][1][i] = S[1][q0 + qq][row][lc];
          }
        }
      }
      if (g > 1) {
        if constexpr (Mode::KC == 4) {
          const T* A = static_cast<const T*>(a.dlt_a) +
                       ((static_cast<size_t>(g) * NRT + rt) * (NP / 4)) * kWave + lane;
#pragma unroll 4
          for (int kc = 0; kc < NP / 4; ++kc) {
            const T av = A[kc * kWave];
            const int krow = 4 * kc + (lane >> 4);
#pragma unroll
            for (int qq = 0; qq < QG; ++qq) {
              acc[u][qq][0] = mfma_k4(av, S[0][q0 + qq][krow][lc], acc[u][qq][0]);
              acc[u][qq][1] = mfma_k4(av, S[1][q0 + qq][krow][lc], acc[u][qq][1]);
            }
          }
        } else {
          const uint4* Ah = static_cast<const uint4*>(a.dlt_a) +
                            ((static_cast<size_t>(g) * NRT + rt) * (NP / 32)) * kWave + lane;
          const uint4* Al = static_cast<const uint4*>(a.dlt_b) +
                            ((static_cast<size_t>(g) * NRT + rt) * (NP / 32)) * kWave + lane;
#pragma unroll 2
          for (int kc = 0; kc < NP / 32; ++kc) {
            const bf16x8 ah = __builtin_bit_cast(bf16x8, Ah[kc * kWave]);
            const bf16x8 al = __builtin_bit_cast(bf16x8, Al[kc * kWave]);
            const int k0 = 32 * kc + 8 * (lane >> 4);
#pragma unroll
            for (int qq = 0; qq < QG; ++qq) {
#pragma unroll
              for (int part = 0; part < 2; ++part) {
                float xv[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) xv[j] = S[part][q0 + qq][k0 + j][lc];
                bf16x8 bh, bl;
                split8(xv, bh, bl);
                Acc c = acc[u][qq][part];
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
                acc[u][qq][part] = c;
              }
            }
          }
        }
      }
    }
    __syncthreads();   // every wave has finished reading S
    // ---- 2. C' = d o C, squared norms and ground-cluster weights per row tile
    {
      const T* dr = static_cast<const T*>(a.dre) + static_cast<size_t>(g) * NP;
      const T* di = static_cast<const T*>(a.dim) + static_cast<size_t>(g) * NP;
#pragma unroll
      for (int u = 0; u < UPW; ++u) {
        const int unit = wave + 4 * u;
        if (unit >= NUNITS) break;
        const int rt = unit % NRT;
        const int q0 = (unit / NRT) * QG;
        T drv[4], div[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          drv[i] = dr[rt * 16 + Mode::row(lane, i)];
          div[i] = di[rt * 16 + Mode::row(lane, i)];
        }
#pragma unroll
        for (int qq = 0; qq < QG; ++qq) {
          T nrm = T(0), gw = T(0);
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int row = rt * 16 + Mode::row(lane, i);
            const T yr = acc[u][qq][0][i], yi = acc[u][qq][1][i];
            const T cr = drv[i] * yr - div[i] * yi;
            const T ci = drv[i] * yi + div[i] * yr;
            S[0][q0 + qq][row][lc] = cr;
            S[1][q0 + qq][row][lc] = ci;
            const T w2 = cr * cr + ci * ci;
            nrm += w2;
            if (row < gsz) gw += w2;
          }
          nrm += __shfl_xor(nrm, 16, kWave);
          nrm += __shfl_xor(nrm, 32, kWave);
          gw += __shfl_xor(gw, 16, kWave);
          gw += __shfl_xor(gw, 32, kWave);
          if (lane < 16) {
            s_nu[rt][(q0 + qq) * 16 + lane] = nrm;
            s_gw[rt][(q0 + qq) * 16 + lane] = gw;
          }
        }
      }
    }
    if (tid == 0) s_nlist = 0;
    __syncthreads();
    // ---- 3. threshold test
    if (tid < TT) {
      const bool valid = tb + tid < a.K;
      double nu = 0.0, gw = 0.0;
#pragma unroll
      for (int rt = 0; rt < NRT; ++rt) {
        nu += static_cast<double>(s_nu[rt][tid]);
        gw += static_cast<double>(s_gw[rt][tid]);
      }
      if (valid) {
        if (nu <= s_r[tid]) {
          s_list[atomicAdd(&s_nlist, 1)] = tid;
        } else {
          s_p[tid] = gw / nu;
        }
      } else {
        s_p[tid] = 0.0;
      }
    }
    __syncthreads();
    const int ncross = s_nlist;
    for (int e = wave; e < ncross; e += 4) {
      const int t = s_list[e];
      finish_crossing<NP, TQ, T>(a, g, t, tb + t, S, s_r, s_m, s_cnt, s_net, s_p, s_kind);
    }
    __syncthreads();
    // ---- 4. per-tile observable sums (wave 0)
    if (wave == 0) {
      const double p = (lane < TT) ? s_p[lane] : 0.0;
      const double sp = wave_sum(p);
      const double sq = wave_sum(p * p);
      if (lane == 0) {
        double* dst = a.partial + (static_cast<size_t>(tile) * a.M + g) * 2;
        dst[0] = sp;
        dst[1] = sq;
      }
    }
  }
  // ---- per-trajectory results
  if (tid < TT && tb + tid < a.K) {
    const int64_t j = tb + tid;
    if (a.jump_count) a.jump_count[j] = s_cnt[tid];
    if (a.net_gs) a.net_gs[j] = s_net[tid];
    if (a.net_hist) {
      int v = s_net[tid];
      v = v < a.hist_lo ? a.hist_lo : (v > a.hist_hi ? a.hist_hi : v);
      atomicAdd(reinterpret_cast<unsigned long long*>(&a.net_hist[v - a.hist_lo]), 1ull);
    }
  }
  if (a.final_state) {
    for (int e = tid; e < TT * a.n; e += blockDim.x) {
      const int t = e / a.n, x = e - t * a.n;
      const int64_t j = tb + t;
      if (j < a.K) {
        a.final_state[(j * a.n + x) * 2 + 0] = static_cast<double>(S[0][t >> 4][x][t & 15]);
        a.final_state[(j * a.n + x) * 2 + 1] = static_cast<double>(S[1][t >> 4][x][t & 15]);
      }
    }
  }
  if (a.jump_totals && tid < 3 && s_kind[tid])
    atomicAdd(reinterpret_cast<unsigned long long*>(&a.jump_totals[tid]),
              static_cast<unsigned long long>(s_kind[tid]));
}

__global__ void k_reduce_partials(const double* __restrict__ partial, int64_t tiles, int M, double K,
                                  double* __restrict__ sum, double* __restrict__ sumsq) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= M) return;
  double s = 0.0, q = 0.0;
  if (g == 0) {
    s = K;   // every trajectory starts in the ground state of H(0)
    q = K;
  } else {
    for (int64_t t = 0; t < tiles; ++t) {
      s += partial[(t * M + g) * 2];
      q += partial[(t * M + g) * 2 + 1];
    }
  }
  if (sum) sum[g] = s;
  if (sumsq) sumsq[g] = q;
}

template <int NP, int TQ, class Mode>
hipError_t launch_np(const StepArgs& a, int64_t tiles, hipStream_t st) {
  hipLaunchKernelGGL((k_trajectories<NP, TQ, Mode>), dim3(static_cast<unsigned>(tiles)), dim3(256), 0, st, a);
  return hipGetLastError();
}

template <class Mode>
hipError_t launch_mode(int NP, int TQ, const StepArgs& a, int64_t tiles, hipStream_t st) {
#define AQT_CASE(np, tq) \
  if (NP == np && TQ == tq) return launch_np<np, tq, Mode>(a, tiles, st);
  if constexpr (Mode::KC == 4) {
    AQT_CASE(16, 1) AQT_CASE(16, 2) AQT_CASE(16, 4)
  }
  AQT_CASE(32, 1) AQT_CASE(32, 2) AQT_CASE(32, 4)
  AQT_CASE(64, 1) AQT_CASE(64, 2) AQT_CASE(64, 4)
  AQT_CASE(128, 1) AQT_CASE(128, 2)
  AQT_CASE(256, 1) AQT_CASE(256, 2)
#undef AQT_CASE
  return hipErrorInvalidValue;
}

}  // namespace

int default_tq(int NP, int precision, int64_t K) {
  // Largest column-group count that still spreads the tiles over the chip.
  int tq = (NP >= 128) ? 2 : 4;
  if (precision == AQT_FP64 && NP >= 256) tq = 1;
  while (tq > 1 && (K + 16 * tq - 1) / (16 * tq) < 512) tq >>= 1;
  return tq;
}

aqt_status launch_run(aqt_ctx* ctx, const aqt_run_params* p, const aqt_outputs* o) {
  const int prec = p->precision;
  const int NP_run = (prec == AQT_BF16 && ctx->NP < 32) ? 32 : ctx->NP;
  if (NP_run != ctx->NP) return ctx->fail(AQT_EINVAL, "BF16 stepping needs at least 17 levels (pad n to 32)");
  aqt_status s = pack_for_precision(ctx, prec);
  if (s != AQT_OK) return s;
  int tq = p->tile ? p->tile / 16 : default_tq(ctx->NP, prec, p->n_traj);
  if (p->tile && (p->tile % 16 || tq < 1 || tq > 4 || (tq == 3)))
    return ctx->fail(AQT_EINVAL, "tile must be 16, 32 or 64 trajectories");
  if (ctx->NP >= 128 && tq > 2) return ctx->fail(AQT_EINVAL, "tile of 64 needs n <= 64");
  const int64_t TT = 16 * tq;
  const int64_t tiles = (p->n_traj + TT - 1) / TT;
  const size_t need = static_cast<size_t>(tiles) * ctx->M * 2 * sizeof(double);
  if (ctx->partial.reserve(need) != hipSuccess) return ctx->fail(AQT_ENOMEM, "workspace allocation failed");

  StepArgs a{};
  a.M = ctx->M;
  a.n = ctx->n;
  a.nq = ctx->nq;
  a.dt = ctx->dt;
  a.K = p->n_traj;
  a.seed = p->seed;
  a.iid = p->instance_id;
  a.traj0 = p->traj_offset;
  a.cap = p->record_capacity;
  a.dlt_a = ctx->pk_a.p;
  a.dlt_b = ctx->pk_b.p;
  a.dre = ctx->pk_dre.p;
  a.dim = ctx->pk_dim.p;
  a.cinit = ctx->cinit.as<double>();
  a.Gamma = ctx->Gamma.as<double>();
  a.d64re = ctx->dre.as<double>();
  a.d64im = ctx->dim.as<double>();
  a.R = ctx->R.as<double>();
  a.zdiag = ctx->zdiag.as<double>();
  a.E = ctx->E.as<double>();
  a.gs = ctx->gs.as<int>();
  a.partial = ctx->partial.as<double>();
  a.jump_totals = o->jump_totals;
  a.jump_count = o->jump_count;
  a.jumps = o->jumps;
  a.net_gs = o->net_gs;
  a.net_hist = o->net_hist;
  a.hist_lo = o->hist_lo;
  a.hist_hi = o->hist_hi;
  a.final_state = o->final_state;

  hipError_t e;
  if (prec == AQT_FP64) e = launch_mode<ModeF64>(ctx->NP, tq, a, tiles, ctx->stream);
  else if (prec == AQT_FP32) e = launch_mode<ModeF32>(ctx->NP, tq, a, tiles, ctx->stream);
  else e = launch_mode<ModeBF16>(ctx->NP, tq, a, tiles, ctx->stream);
  if (e != hipSuccess) return ctx->fail(AQT_EHIP, std::string("trajectory kernel launch: ") + hipGetErrorString(e));
  if (o->pgs_sum || o->pgs_sumsq) {
    hipLaunchKernelGGL(k_reduce_partials, dim3((ctx->M + 255) / 256), dim3(256), 0, ctx->stream,
                       ctx->partial.as<double>(), tiles, ctx->M, static_cast<double>(p->n_traj), o->pgs_sum,
                       o->pgs_sumsq);
    e = hipGetLastError();
    if (e != hipSuccess) return ctx->fail(AQT_EHIP, std::string("reduction launch: ") + hipGetErrorString(e));
  }
  return AQT_OK;
}

}  // namespace aqt
