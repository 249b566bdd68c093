// Fixed-step quantum-jump unraveling (App. B, "to jump or not to jump"), the second
// unraveling beside the waiting-time procedure of step.hip.
//
// Each grid step of length dt (generator frozen at the grid point, basis change O_g at
// its start, as in the waiting-time kernel) is cut into S sub-steps of length h.  Per
// sub-step the normalised state has jump probability dp = h sum_b |c_b|^2 Gamma_b
// (eq. lambda).  A uniform eps decides: eps >= dp evolves every component by
// exp(-i e_b h - Gamma_b h / 2) and renormalises; eps < dp applies the jump operator
// drawn with probability proportional to <A_i^dag A_i> (eq. Pi(t): source level b with
// weight |c_b|^2 Gamma_b, then channel i and target a by R[i][b][a]) and renormalises.
// The scheme is first order in h; its mean approaches the master equation as h -> 0.
// The kernel carries the no-jump evolution unnormalised within a grid step (dp and the
// jump draws are ratios, dp = h sum |c|^2 Gamma / sum |c|^2) and normalises at its end.
//
// Draws: sub-step u = (g - 1) S + s of trajectory j uses Philox draws 3u (eps), 3u + 1
// (source) and 3u + 2 (channel and target).  Jump records carry the sub-step's start.
//
// One workgroup (8 wavefronts) owns TT = 16 trajectories: the basis change is an MFMA
// product on the LDS tile (tilegemm.hpp); the sub-steps run on one wavefront per
// trajectory with lanes over levels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"
#include "ctx.hpp"
#include "philox.hpp"
#include "tilegemm.hpp"

namespace aqt {
namespace {

using namespace tile;

struct FixArgs {
  const void* pD;        // [M][NP][NP] O_g - I in the state precision
  const double* cinit;   // [NP]
  const double* E;       // [M][NP]
  const double* shift;   // [M][NP] Lamb shift (phases use E + shift)
  const double* Gam;     // [M][NP]
  const double* R;       // [M][nq][NP(b)][NP(a)]
  const double* Rcol;    // [M][nq][NP][4] (row sum first)
  const double* zdiag;   // [M][nq][NP]
  const int* gs;         // [M]
  double* partial;       // [tiles][M][2]
  int64_t* jump_totals;  // [3] (may be null)
  int32_t* jump_count;   // [K] (may be null)
  aqt_jump* jumps;       // [K][cap] (may be null)
  int32_t* net_gs;       // [K] (may be null)
  double* final_state;   // [K][n][2] (may be null)
  int cap;
  int* flags;            // AQT_RUN_* flags of the context (OR-ed)
  int M, n, nq, S;
  const double* tbeg;    // [M] start time of the step into grid g
  const double* tlen;    // [M] its length
  int64_t K;
  uint64_t seed, iid, traj0;
};

// First index of the running sum of the NP weights w (one per lane slot x = lane + 64 r)
// that exceeds target; ties and rounding as a left-to-right sum.  Returns -1 if none.
template <int NR>
__device__ int first_exceeding(const double (&w)[NR], double target) {
  const int lane = threadIdx.x & 63;
  double base = 0.0;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const double inc = wave_inclusive_scan(w[r]);
    const uint64_t hit = __ballot(base + inc > target);
    if (hit) return 64 * r + first_set_lane(hit);
    base += __shfl(inc, 63, 64);
  }
  (void)lane;
  return -1;
}

template <int NP, int TT, class T>
__global__ __launch_bounds__(kGThreads) void k_fixed_step(FixArgs a) {
  constexpr int NC = 2 * TT;
  constexpr int LD = (sizeof(T) == 4 && NC == 32) ? 36 : NC + 1;
  constexpr int NR = (NP + 63) / 64;
  __shared__ T PA[NP * LD];
  __shared__ T PB[NP * LD];
  __shared__ double s_p[TT][2];
  __shared__ int s_kind[3];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t tile = blockIdx.x;
  if (tid < 3) s_kind[tid] = 0;
  for (int f = tid; f < NP * LD; f += kGThreads) PB[f] = static_cast<T>(0);
  // per-trajectory registers of the handling wave (trajectories t = wave + kGW k)
  constexpr int TPW = (TT + kGW - 1) / kGW;
  int cnt[TPW], net[TPW];
#pragma unroll
  for (int k = 0; k < TPW; ++k) cnt[k] = net[k] = 0;
  __syncthreads();

  for (int g = 1; g < a.M; ++g) {
    const double h = a.tlen[g] / a.S;   // sub-step length
    if (g == 1) {
      for (int f = tid; f < NP * NC; f += kGThreads) {
        const int x = f / NC, col = f % NC;
        const bool act = tile * TT + (col >> 1) < a.K;
        PA[x * LD + col] = (!(col & 1) && act) ? static_cast<T>(a.cinit[x]) : static_cast<T>(0);
      }
    } else {
      gemm_kick<NP, NC, LD, T>(static_cast<const T*>(a.pD) + static_cast<size_t>(g) * NP * NP, PB, PA);
    }
    __syncthreads();
    const size_t gN = static_cast<size_t>(g) * NP;
    // sub-step propagator and rates of this grid point, per level slot
    double dr[NR], di[NR], G[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int x = lane + 64 * r;
      dr[r] = di[r] = G[r] = 0.0;
      if (x < a.n) {
        G[r] = a.Gam[gN + x];
        double sn, cs;
        sincos((a.E[gN + x] + a.shift[gN + x]) * h, &sn, &cs);
        const double mag = exp(-0.5 * G[r] * h);
        dr[r] = mag * cs;
        di[r] = -mag * sn;
      }
    }
#pragma unroll
    for (int k = 0; k < TPW; ++k) {
      const int t = wave + kGW * k;
      if (t >= TT) continue;
      const int64_t j = tile * TT + t;
      if (j >= a.K) {
        if (lane < 2) s_p[t][lane] = 0.0;
        continue;
      }
      const uint64_t tj = a.traj0 + static_cast<uint64_t>(j);
      double cr[NR], ci[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const int x = lane + 64 * r;
        cr[r] = (x < NP) ? static_cast<double>(PA[x * LD + 2 * t]) : 0.0;
        ci[r] = (x < NP) ? static_cast<double>(PA[x * LD + 2 * t + 1]) : 0.0;
      }
      // the decision draws of up to 64 sub-steps at once, one Philox evaluation per lane
      double eps_l = 0.0;
      for (int s = 0; s < a.S; ++s) {
        const uint64_t u = static_cast<uint64_t>(g - 1) * a.S + s;
        if ((s & 63) == 0 && lane < a.S - s) eps_l = draw_uniform(a.seed, a.iid, tj, 3 * (u + lane));
        const double eps = __shfl(eps_l, s & 63, 64);
        double nn = 0.0, rate = 0.0;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const double q = cr[r] * cr[r] + ci[r] * ci[r];
          nn += q;
          rate += q * G[r];
        }
        nn = wave_sum(nn);
        rate = wave_sum(rate);
        const double dp = h * rate / nn;
        if (!(eps < dp)) {
          // no jump: the decayed state stays unnormalised until the end of the grid step
          // (dp and the jump draws use ratios; the decay over S sub-steps is bounded)
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            const double xr = dr[r] * cr[r] - di[r] * ci[r], xi = dr[r] * ci[r] + di[r] * cr[r];
            cr[r] = xr;
            ci[r] = xi;
          }
          continue;
        }
        // jump: source level, then channel and target (eq. Pi(t))
        const double u1 = draw_uniform(a.seed, a.iid, tj, 3 * u + 1);
        const double u2 = draw_uniform(a.seed, a.iid, tj, 3 * u + 2);
        double wsrc[NR];
        double tot = 0.0;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          wsrc[r] = (cr[r] * cr[r] + ci[r] * ci[r]) * G[r];
          tot += wsrc[r];
        }
        tot = wave_sum(tot);
        int b = first_exceeding<NR>(wsrc, u1 * tot);
        if (b < 0) {   // rounding at the top end: the last level with weight
          int last = -1;
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            const int l = last_set_lane(__ballot(wsrc[r] > 0.0));
            if (l >= 0) last = 64 * r + l;
          }
          b = last;
        }
        // channel rows in order, then the target within the row
        const double target = u2 * a.Gam[gN + b];
        double before = 0.0, before_last = 0.0;
        int qi = -1, last_row = 0;
        for (int i = 0; i < a.nq; ++i) {
          const double rs = a.Rcol[((static_cast<size_t>(g) * a.nq + i) * NP + b) * 4];
          if (rs > 0.0) {
            last_row = i;
            before_last = before;
          }
          if (before + rs > target) {
            qi = i;
            break;
          }
          before += rs;
        }
        if (qi < 0) {   // rounding at the top end: the last channel with weight
          qi = last_row;
          before = before_last;
        }
        const double* row = a.R + ((static_cast<size_t>(g) * a.nq + qi) * NP + b) * NP;
        double wr[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const int x = lane + 64 * r;
          wr[r] = (x < a.n) ? row[x] : 0.0;
        }
        int ta = first_exceeding<NR>(wr, target - before);
        if (ta < 0) {
          int last = -1;
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            const int l = last_set_lane(__ballot(wr[r] > 0.0));
            if (l >= 0) last = 64 * r + l;
          }
          ta = last;
        }
        int kind;
        if (ta != b) {
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            cr[r] = (lane + 64 * r == ta) ? 1.0 : 0.0;
            ci[r] = 0.0;
          }
          kind = (a.E[gN + ta] <= a.E[gN + b]) ? AQT_KIND_RELAX : AQT_KIND_EXCITE;
          const int gsz = a.gs[g];
          if (ta < gsz && b >= gsz) ++net[k];
          else if (b < gsz && ta >= gsz) --net[k];
        } else {
          const double* z = a.zdiag + (static_cast<size_t>(g) * a.nq + qi) * NP;
          double n2 = 0.0;
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            const int x = lane + 64 * r;
            const double zz = (x < NP) ? z[x] : 0.0;
            cr[r] *= zz;
            ci[r] *= zz;
            n2 += cr[r] * cr[r] + ci[r] * ci[r];
          }
          const double inv = 1.0 / sqrt(wave_sum(n2));
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            cr[r] *= inv;
            ci[r] *= inv;
          }
          kind = AQT_KIND_DEPHASE;
        }
        if (lane == 0) {
          if (a.jumps && cnt[k] >= a.cap) atomicOr(a.flags, AQT_RUN_RECORDS_TRUNCATED);
          if (a.jumps && cnt[k] < a.cap) {
            aqt_jump rec;
            rec.t = a.tbeg[g] + s * h;
            rec.step = g - 1;
            rec.qubit = static_cast<int16_t>(qi);
            rec.kind = static_cast<int16_t>(kind);
            rec.from_level = b;
            rec.to_level = ta;
            a.jumps[j * a.cap + cnt[k]] = rec;
          }
          atomicAdd(&s_kind[kind], 1);
        }
        ++cnt[k];
      }
      // end of the step: ground-cluster population, then the normalised state for the
      // next basis change
      double pg = 0.0, nn = 0.0;
      const int gsz = a.gs[g];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const int x = lane + 64 * r;
        const double q = cr[r] * cr[r] + ci[r] * ci[r];
        nn += q;
        if (x < gsz) pg += q;
      }
      nn = wave_sum(nn);
      pg = wave_sum(pg);
      const double inv = 1.0 / sqrt(nn);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const int x = lane + 64 * r;
        cr[r] *= inv;
        ci[r] *= inv;
        if (x < NP) {
          PB[x * LD + 2 * t] = static_cast<T>(cr[r]);
          PB[x * LD + 2 * t + 1] = static_cast<T>(ci[r]);
        }
      }
      if (lane == 0) {
        const double p = pg / nn;
        s_p[t][0] = p;
        s_p[t][1] = p * p;
      }
      if (g == a.M - 1 && a.final_state) {
        for (int x = lane; x < a.n; x += 64) {
          int r = x >> 6;
          double vr = 0.0, vi = 0.0;
#pragma unroll
          for (int rr = 0; rr < NR; ++rr)
            if (rr == r) {
              vr = cr[rr];
              vi = ci[rr];
            }
          a.final_state[(j * a.n + x) * 2] = vr;
          a.final_state[(j * a.n + x) * 2 + 1] = vi;
        }
      }
    }
    __syncthreads();
    if (tid == 0) {
      double s1 = 0.0, s2 = 0.0;
      for (int t = 0; t < TT; ++t) {
        s1 += s_p[t][0];
        s2 += s_p[t][1];
      }
      a.partial[(tile * a.M + g) * 2] = s1;
      a.partial[(tile * a.M + g) * 2 + 1] = s2;
    }
  }
  // per-trajectory counters and this tile's jump totals
#pragma unroll
  for (int k = 0; k < TPW; ++k) {
    const int t = wave + kGW * k;
    const int64_t j = tile * TT + t;
    if (t < TT && j < a.K && lane == 0) {
      if (a.jump_count) a.jump_count[j] = cnt[k];
      if (a.net_gs) a.net_gs[j] = net[k];
    }
  }
  __syncthreads();
  if (tid < 3 && a.jump_totals) atomicAdd(reinterpret_cast<unsigned long long*>(a.jump_totals + tid),
                                          static_cast<unsigned long long>(s_kind[tid]));
}

// pgs_sum[g], pgs_sumsq[g] = fixed-order sums over tiles (g = 0: the initial ground state).
__global__ void k_fixed_reduce(const double* __restrict__ partial, int64_t tiles, int M, double K,
                               double* __restrict__ sum, double* __restrict__ sumsq) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= M) return;
  double s = K, q = K;
  if (g > 0) {
    s = q = 0.0;
    for (int64_t t = 0; t < tiles; ++t) {
      s += partial[(t * M + g) * 2];
      q += partial[(t * M + g) * 2 + 1];
    }
  }
  if (sum) sum[g] = s;
  if (sumsq) sumsq[g] = q;
}

template <class T>
__global__ void k_pack_delta(const double* __restrict__ dlt, int64_t count, T* __restrict__ D) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    D[i] = static_cast<T>(dlt[i]);
}

}  // namespace

aqt_status launch_fixed_step(aqt_ctx* ctx, const aqt_run_params* p, int substeps, const aqt_outputs* o) {
  {
    const aqt_status s = check_step_decay(ctx, p->precision);
    if (s != AQT_OK) return s;
  }
  const int NP = ctx->NP;
  const bool f64 = p->precision == AQT_FP64;
  constexpr int TT = 16;
  const int64_t tiles = (p->n_traj + TT - 1) / TT;
  hipStream_t st = ctx->stream;
  const size_t el = f64 ? 8 : 4, per = static_cast<size_t>(NP) * NP * ctx->M;
  if (ctx->fix_prec != p->precision) {
    if (ctx->fix_D.reserve(per * el) != hipSuccess) return ctx->fail(AQT_ENOMEM, "operand allocation failed");
    const unsigned blocks = static_cast<unsigned>(std::min<size_t>(65536, (per + 255) / 256));
    if (f64)
      hipLaunchKernelGGL(k_pack_delta<double>, dim3(blocks), dim3(256), 0, st, ctx->dlt.as<double>(),
                         static_cast<int64_t>(per), ctx->fix_D.as<double>());
    else
      hipLaunchKernelGGL(k_pack_delta<float>, dim3(blocks), dim3(256), 0, st, ctx->dlt.as<double>(),
                         static_cast<int64_t>(per), ctx->fix_D.as<float>());
    AQT_HIP(ctx, hipGetLastError());
    ctx->fix_prec = p->precision;
  }
  if (ctx->partial.reserve(static_cast<size_t>(tiles) * ctx->M * 2 * sizeof(double)) != hipSuccess)
    return ctx->fail(AQT_ENOMEM, "workspace allocation failed");
  FixArgs fa{};
  fa.pD = ctx->fix_D.p;
  fa.cinit = ctx->cinit.as<double>();
  fa.E = ctx->E.as<double>();
  fa.shift = ctx->shift.as<double>();
  fa.Gam = ctx->Gamma.as<double>();
  fa.R = ctx->R.as<double>();
  fa.Rcol = ctx->Rcol.as<double>();
  fa.zdiag = ctx->zdiag.as<double>();
  fa.gs = ctx->gs.as<int>();
  fa.partial = ctx->partial.as<double>();
  fa.jump_totals = o->jump_totals;
  fa.jump_count = o->jump_count;
  fa.jumps = (p->record_capacity > 0) ? o->jumps : nullptr;
  fa.net_gs = o->net_gs;
  fa.final_state = o->final_state;
  fa.cap = p->record_capacity;
  fa.flags = ctx->run_flags.as<int>();
  fa.M = ctx->M;
  fa.n = ctx->n;
  fa.nq = ctx->tab_nch;   // jump channels
  fa.S = substeps;
  fa.tbeg = ctx->tbeg.as<double>();
  fa.tlen = ctx->tlen.as<double>();
  fa.K = p->n_traj;
  fa.seed = p->seed;
  fa.iid = p->instance_id;
  fa.traj0 = p->traj_offset;
#define AQT_FIX(np, T) \
  hipLaunchKernelGGL((k_fixed_step<np, TT, T>), dim3(static_cast<unsigned>(tiles)), dim3(kGThreads), 0, st, fa)
  switch (NP) {
    case 16: if (f64) AQT_FIX(16, double); else AQT_FIX(16, float); break;
    case 32: if (f64) AQT_FIX(32, double); else AQT_FIX(32, float); break;
    case 64: if (f64) AQT_FIX(64, double); else AQT_FIX(64, float); break;
    case 128: if (f64) AQT_FIX(128, double); else AQT_FIX(128, float); break;
    case 256: if (f64) AQT_FIX(256, double); else AQT_FIX(256, float); break;
    default: return ctx->fail(AQT_EINVAL, "unsupported level count");
  }
#undef AQT_FIX
  AQT_HIP(ctx, hipGetLastError());
  if (o->pgs_sum || o->pgs_sumsq) {
    hipLaunchKernelGGL(k_fixed_reduce, dim3((ctx->M + 255) / 256), dim3(256), 0, st, ctx->partial.as<double>(), tiles,
                       ctx->M, static_cast<double>(p->n_traj), o->pgs_sum, o->pgs_sumsq);
    AQT_HIP(ctx, hipGetLastError());
  }
  return AQT_OK;
}

}  // namespace aqt
