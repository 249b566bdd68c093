// Adjoint gradient of the trajectory average of the final ground-cluster population
// with respect to the schedule control points and the bath coupling eta.
//
// A trajectory of the waiting-time procedure (Sec. IV) is a path: its jump times
// and channels.  Paths have density |psi~|^2 with respect to a measure that does
// not depend on the parameters (Lebesgue measure on times, counting measure on
// channels), psi~ being the unnormalised amplitude built from the no-jump
// propagators (Sec. III eq. Heff), the basis changes O_g and the jump operators
// sqrt(gamma) A (Sec. III eq. jump, App. B).  So E[P_GS] is the integral over paths
// of <psi~|Pi|psi~>, and each trajectory gives the unbiased estimate
//
//   g = 2 Re <psi~|Pi| d psi~> / |psi~|^2,
//
// the sum of a pathwise term (derivative of the normalised final population along
// the fixed path) and a score-function term (derivative of the path density) for the
// jump times and channels.  d psi~ is a sum over the factors F of psi~; with the
// adjoint lambda propagated backward (lambda_before = F^H lambda_after / rho, rho the
// forward renormalisation of that factor, lambda_final = Pi psi / |psi|^2) a factor
// contributes 2 Re <lambda_after| dF |psi_before> / rho.  <lambda|psi> = f (the
// trajectory's final ground-cluster population) at every point of the path.
//
// Factors per step g (from s_{g-1} to s_g; generator frozen at s_g) and what they give:
//   basis change O_g = V_g^T V_{g-1}: with dV_g = V_g X_g (first-order perturbation
//     theory; X antisymmetric), grid g collects -2 Re <lambda_A|X_g|psi_A> (just after
//     O_g) and +2 Re <lambda_B|X_g|psi_B> (just before O_{g+1}); grid 0 acts through
//     the initial state, 2 Re <lambda_A|V_1 dv_0> at step 1.  These are MFMA products
//     X_g [psi_A psi_B] contracted with the adjoints.  H(s_g) = A(s_g) H_X + B(s_g) H_Z is
//     diagonal in its own eigenbasis, so the off-diagonal parts of V^T H_X V and V^T H_Z V
//     are proportional (A <.>_X + B <.>_Z = 0 off the diagonal), and so are X^A_g and X^B_g:
//     one product per point serves both directions, scaled per grid point.
//   no-jump propagation exp(-i e tau - Gamma tau / 2) (diagonal): per component
//     P_x = conj(lambda_x) psi_x is constant between a != b jumps; a step without one
//     gives 2 dt sum de_x Im P_x - dt sum dGamma_x Re P_x.
//   jump b -> a (a != b), operator sqrt(gamma(e_b - e_a)) z_ab |a><b|: the state
//     collapses, so every factor of the step is single-component and contributes
//     through f alone: 2 f d log|l_ab| per such jump and -f tau dGamma_c for each
//     stretch spent in component c.
//   omega = 0 operator sqrt(gamma(0)) diag(z_i): 2 Re <lambda_after| diag(dz_i) |psi_before>
//     / |diag(z_i) psi_before| (gamma(0) cancels).
// eta scales every rate: dGamma = Gamma / eta, d log l = 1 / (2 eta), no basis change;
// it scales the Lamb shift too (phases exp(-i (e + shift) dt)), whose derivative with
// respect to the schedule is tabulated beside de.
// Controls enter through A(s_g) and B(s_g) with the hat-function weights of the
// piecewise-linear schedule.
//
// The same sweep carries a second adjoint with the identity in place of Pi: it gives
// s = d log |psi~|^2, the score of the path density (mean zero), used as a control
// variate.  Both adjoints share the replayed states and the X_g products.
//
// The forward paths come from the trajectory kernel (its jump records); one
// workgroup owns TT trajectories for the whole sweep: a forward replay that stores
// the state every C steps, then per segment of C steps (last first) a replay that
// keeps every post-kick state, followed by the backward steps of that segment.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"
#include "ctx.hpp"
#include "tilegemm.hpp"

namespace aqt {
namespace {

using namespace tile;

constexpr int kMaxJ = 32;           // omega = 0 jumps of one trajectory within one step

struct GradArgs {
  const void* pD;        // [M][NP][NP] O_g - I in the state precision
  const void* pDT;       // [M][NP][NP] its transpose
  const void* pX;        // [M][NP][NP] X_g in the state precision (X^A_g = xc[0] X_g, X^B_g = xc[1] X_g)
  const double* xc;      // [M][3]
  const double* cinit;   // [NP]
  const double* E;       // [M][NP]
  const double* Gam;     // [M][NP]
  const double* zdiag;   // [M][nq][NP]
  const double* dre;     // [M][NP] Re exp(-i e dt - Gamma dt / 2)
  const double* dim;
  const double* dE;      // [M][2][NP]
  const double* dGam;    // [M][2][NP]
  const double* dzd;     // [M][2][nq][NP]
  const double* dll;     // [M][2][nq][NP][NP]
  const double* dcin;    // [2][NP]
  const double* shift;   // [M][NP] Lamb shift (zeros when off): the phases use E + shift
  const double* dshift;  // [M][2][NP] its derivative (zeros when off)
  int lamb;              // the Lamb shift is on (else both tables are skipped)
  const aqt_jump* jumps; // [K][cap]
  const int32_t* jcount; // [K]
  int cap;
  void* ckpt;            // [tiles][S][NP][NC] states after steps sC
  int* ckcur;            // [tiles][S][TT] record cursors there
  void* seg;             // [tiles][C][NP][NC] post-kick states of the segment
  int* scur;             // [tiles][C][TT] record cursor at the start of each step of the segment
  double* out;           // row j at out + j * ostride: f, then dP/dA_j, dP/dB_j, dP/deta
  int ostride;
  int proj;              // levels of the final projector: the ground cluster, or all (path-density score)
  int* status;           // bit 0: more than kMaxJ omega = 0 jumps in one step
  int M, nq, nctrl, C, S;
  double eta;
  const double* tbeg;    // [M] start time of the step into grid g
  const double* tlen;    // [M] its length
  const double* sg;      // [M] grid points s_g (hat-function weights of the controls)
  int64_t K, tile0;
};

// part1[t] += Re <L1_t | Y_t> and part2[t] += Re <L2_t | Y_t> for the 16-row tile rt of a
// product Y held in MFMA accumulators (columns 2t, 2t + 1 = re, im); each wave adds to
// its own part rows.
template <int NP, int NC, int LD, class T>
__device__ __forceinline__ void dot2_tile(const typename Mfma<T>::acc_t (&acc)[NC / 16], int rt, const T* L1,
                                          const T* L2, double* part1, double* part2) {
  constexpr int CT = NC / 16;
  const int lane = threadIdx.x & 63, c = lane & 15;
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    double s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = rt * 16 + Mfma<T>::row(lane, e), col = ct * 16 + c;
      const double y = static_cast<double>(acc[ct][e]);
      s1 += static_cast<double>(L1[r * LD + col]) * y;
      s2 += static_cast<double>(L2[r * LD + col]) * y;
    }
    s1 += __shfl_xor(s1, 16, 64);
    s1 += __shfl_xor(s1, 32, 64);
    s1 += __shfl_xor(s1, 1, 64);
    s2 += __shfl_xor(s2, 16, 64);
    s2 += __shfl_xor(s2, 32, 64);
    s2 += __shfl_xor(s2, 1, 64);
    if (lane < 16 && !(lane & 1)) {
      part1[(ct * 16 + lane) >> 1] += s1;
      part2[(ct * 16 + lane) >> 1] += s2;
    }
  }
}

// part1[t] += Re <L1_t | X | B_t> and part2[t] += Re <L2_t | X | B_t>: one product, two adjoints.
template <int NP, int NC, int LD, class T>
__device__ void gemm_dot2(const T* __restrict__ X, const T* B, const T* L1, const T* L2, double* part1,
                          double* part2) {
  constexpr int RT = NP / 16, CT = NC / 16;
  const int wave = threadIdx.x >> 6;
  const T* const Bs[1] = {B};
  for (int rt = wave; rt < RT; rt += kGW) {
    typename Mfma<T>::acc_t acc[1][CT];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[0][ct] = Mfma<T>::zero();
    panel_mma<NP, NC, LD, T, 1>(X, rt, Bs, acc);
    dot2_tile<NP, NC, LD, T>(acc[0], rt, L1, L2, part1, part2);
  }
}

// Row tiles of an NP-row product per wave.
template <int NP>
constexpr int rows_per_wave() { return (NP / 16 + kGW - 1) / kGW; }

// Both X_g products of a step in one pass over X_g: X B (end of the step) contracted
// with L1, L2 now (when dotB), X A (just after the basis change) left in accA for
// gemm_dot2_finish once the adjoints have been carried back through the step.
template <int NP, int NC, int LD, class T>
__device__ void gemm_dot2_pair(const T* __restrict__ X, const T* B, const T* A, const T* L1, const T* L2,
                               double* part1, double* part2, bool dotB,
                               typename Mfma<T>::acc_t (&accA)[rows_per_wave<NP>()][NC / 16]) {
  constexpr int RT = NP / 16, CT = NC / 16;
  const int wave = threadIdx.x >> 6;
  const T* const Bs[2] = {B, A};
  int i = 0;
  for (int rt = wave; rt < RT; rt += kGW, ++i) {
    typename Mfma<T>::acc_t acc[2][CT];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) acc[b][ct] = Mfma<T>::zero();
    panel_mma<NP, NC, LD, T, 2>(X, rt, Bs, acc);
    if (dotB) dot2_tile<NP, NC, LD, T>(acc[0], rt, L1, L2, part1, part2);
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) accA[i][ct] = acc[1][ct];
  }
}

template <int NP, int NC, int LD, class T>
__device__ void gemm_dot2_finish(const typename Mfma<T>::acc_t (&accA)[rows_per_wave<NP>()][NC / 16], const T* L1,
                                 const T* L2, double* part1, double* part2) {
  constexpr int RT = NP / 16;
  const int wave = threadIdx.x >> 6;
  int i = 0;
  for (int rt = wave; rt < RT; rt += kGW, ++i) dot2_tile<NP, NC, LD, T>(accA[i], rt, L1, L2, part1, part2);
}

template <int NP, int TT, class T>
struct GradShared {
  static constexpr int NC = 2 * TT;
  // FP32: 4 LD = 16 (mod 64) puts the four k rows of an MFMA operand read in disjoint bank
  // ranges; FP64 keeps the smallest odd stride (LDS budget at 256 levels)
  static constexpr int LD = (sizeof(T) == 4 && NC == 32) ? 36 : NC + 1;
  // four state tiles whose roles rotate: the post-kick state, the end-of-step state and the
  // two adjoints (ground-cluster projector; identity, for the path-density score)
  T buf[4][NP * LD];
  int cur[TT];                   // running record cursor
  double f[TT];                  // final ground-cluster population
  double S[TT][6];               // handler terms of the current grid point: (A, B, eta) per adjoint
  double part[kGW][4][TT];       // X-term partial sums [point][adjoint]
  double rho[TT][kMaxJ];         // |diag(z) psi| of the omega = 0 jumps of one trajectory-step
};

// Records of trajectory j's step g (record step g - 1) start at m0; returns the end.
__device__ inline int step_end(const aqt_jump* rec, int cnt, int m0, int g) {
  int m = m0;
  while (m < cnt && rec[m].step == g - 1) ++m;
  return m;
}

// Replays step g of trajectory t: PA columns -> PB columns.  Between jumps the
// components decay by exp(-Gamma tau / 2); an a != b jump leaves e_a; an omega = 0
// jump multiplies by z_i and renormalises (rho[k] receives the norm before it); the
// phases exp(-i e dt) are applied at the end of the step.
template <int NP, int LD, class T>
__device__ void replay_step(const GradArgs& a, int g, const aqt_jump* rec, int m0, int m1, const T* PA, T* PB, int t,
                            double* rho) {
  constexpr int NR = (NP + 63) / 64;
  const int lane = threadIdx.x & 63;
  const size_t gN = static_cast<size_t>(g) * NP;
  double pr[NR], pi[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int x = lane + 64 * r;
    pr[r] = (x < NP) ? static_cast<double>(PA[x * LD + 2 * t]) : 0.0;
    pi[r] = (x < NP) ? static_cast<double>(PA[x * LD + 2 * t + 1]) : 0.0;
  }
  if (m1 == m0) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int x = lane + 64 * r;
      if (x < NP) {
        const double dr = a.dre[gN + x], di = a.dim[gN + x];
        PB[x * LD + 2 * t] = static_cast<T>(dr * pr[r] - di * pi[r]);
        PB[x * LD + 2 * t + 1] = static_cast<T>(dr * pi[r] + di * pr[r]);
      }
    }
    return;
  }
  const double tk = a.tbeg[g], dt = a.tlen[g];
  double tau_e = 0.0;
  for (int m = m0; m < m1; ++m) {
    const aqt_jump J = rec[m];
    const double tau = J.t - tk;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int x = lane + 64 * r;
      if (x < NP) {
        const double dec = exp(-0.5 * a.Gam[gN + x] * (tau - tau_e));
        pr[r] *= dec;
        pi[r] *= dec;
      }
    }
    tau_e = tau;
    if (J.from_level != J.to_level) {
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        pr[r] = (lane + 64 * r == J.to_level) ? 1.0 : 0.0;
        pi[r] = 0.0;
      }
    } else {
      const double* z = a.zdiag + (static_cast<size_t>(g) * a.nq + J.qubit) * NP;
      double nrm = 0.0;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const int x = lane + 64 * r;
        const double zz = (x < NP) ? z[x] : 0.0;
        pr[r] *= zz;
        pi[r] *= zz;
        nrm += pr[r] * pr[r] + pi[r] * pi[r];
      }
      nrm = wave_sum(nrm);
      const double rn = sqrt(nrm);
      if (rho && m - m0 < kMaxJ) rho[m - m0] = rn;   // every lane writes (and later reads) the same value
      const double inv = 1.0 / rn;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        pr[r] *= inv;
        pi[r] *= inv;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int x = lane + 64 * r;
    if (x < NP) {
      const double dec = exp(-0.5 * a.Gam[gN + x] * (dt - tau_e));
      double sn, cs;
      sincos((a.E[gN + x] + (a.lamb ? a.shift[gN + x] : 0.0)) * dt, &sn, &cs);
      const double ur = pr[r] * dec, ui = pi[r] * dec;
      PB[x * LD + 2 * t] = static_cast<T>(cs * ur + sn * ui);       // times exp(-i e dt)
      PB[x * LD + 2 * t + 1] = static_cast<T>(cs * ui - sn * ur);
    }
  }
}

// Backward through step g for trajectory t (wave-uniform): adds the decay, phase and
// jump terms of grid g to S[3] (directions A, B and eta) and writes lambda_A into LA.
template <int NP, int LD, class T>
__device__ void adjoint_step(const GradArgs& a, int g, const aqt_jump* rec, int m0, int m1, const T* PA, const T* PB,
                             const T* LB, T* LA, int t, double f, const double* rho, double S[3]) {
  constexpr int NR = (NP + 63) / 64;
  const int lane = threadIdx.x & 63;
  const size_t gN = static_cast<size_t>(g) * NP;
  const double* dE0 = a.dE + (static_cast<size_t>(g) * 2) * NP;
  const double* dE1 = dE0 + NP;
  const double* dG0 = a.dGam + (static_cast<size_t>(g) * 2) * NP;
  const double* dG1 = dG0 + NP;
  const double* dS0 = a.dshift + (static_cast<size_t>(g) * 2) * NP;
  const double* dS1 = dS0 + NP;
  const double dt = a.tlen[g], ieta = 1.0 / a.eta;
  bool has_ab = false;
  int b1 = 0;
  for (int m = m0; m < m1; ++m)
    if (rec[m].from_level != rec[m].to_level) {
      has_ab = true;
      b1 = rec[m].from_level;
      break;
    }
  if (has_ab) {
    // every factor of the step acts on one component: terms through f alone
    const double tk = a.tbeg[g];
    int c = b1;
    double tp = 0.0, s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int m = m0; m < m1; ++m) {
      const aqt_jump J = rec[m];
      const double tau = J.t - tk, dur = tau - tp;
      s0 -= f * dur * dG0[c];
      s1 -= f * dur * dG1[c];
      s2 -= f * dur * a.Gam[gN + c] * ieta;
      tp = tau;
      const size_t gi = (static_cast<size_t>(g) * 2) * a.nq + J.qubit;   // [g][dir = 0][i]
      const size_t dstride = static_cast<size_t>(a.nq);                     // dir 1 is nq rows further
      if (J.from_level != J.to_level) {
        const size_t o = (gi * NP + J.from_level) * NP + J.to_level;
        s0 += 2.0 * f * a.dll[o];
        s1 += 2.0 * f * a.dll[o + dstride * NP * NP];
        c = J.to_level;
      } else {
        const double zc = a.zdiag[(static_cast<size_t>(g) * a.nq + J.qubit) * NP + c];
        s0 += 2.0 * f * a.dzd[gi * NP + c] / zc;
        s1 += 2.0 * f * a.dzd[(gi + dstride) * NP + c] / zc;
      }
      s2 += f * ieta;
    }
    const double dur = dt - tp;
    s0 -= f * dur * dG0[c];
    s1 -= f * dur * dG1[c];
    s2 -= f * dur * a.Gam[gN + c] * ieta;
    S[0] += s0;
    S[1] += s1;
    S[2] += s2;
    // lambda_A = f psi_A,b1 / |psi_A,b1|^2 e_b1
    const double ar = static_cast<double>(PA[b1 * LD + 2 * t]), ai = static_cast<double>(PA[b1 * LD + 2 * t + 1]);
    const double sc = f / (ar * ar + ai * ai);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int x = lane + 64 * r;
      if (x < NP) {
        LA[x * LD + 2 * t] = static_cast<T>(x == b1 ? sc * ar : 0.0);
        LA[x * LD + 2 * t + 1] = static_cast<T>(x == b1 ? sc * ai : 0.0);
      }
    }
    return;
  }
  // no collapse: P_x = conj(lambda_B,x) psi_B,x is constant through the step
  const int nj = m1 - m0;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  double fr[NR], fi[NR];   // total step factor F_x = d_x prod_k z_k,x / rho_k
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int x = lane + 64 * r;
    fr[r] = fi[r] = 0.0;
    if (x >= NP) continue;
    const double lr = static_cast<double>(LB[x * LD + 2 * t]), li = static_cast<double>(LB[x * LD + 2 * t + 1]);
    const double br = static_cast<double>(PB[x * LD + 2 * t]), bi = static_cast<double>(PB[x * LD + 2 * t + 1]);
    const double Pr = lr * br + li * bi, Pi = lr * bi - li * br;
    // phases exp(-i (e + shift) dt), decay exp(-Gamma dt / 2); shift and Gamma scale with eta
    double de0 = dE0[x], de1 = dE1[x], sh = 0.0;
    if (a.lamb) {
      de0 += dS0[x];
      de1 += dS1[x];
      sh = a.shift[gN + x];
    }
    s0 += 2.0 * dt * de0 * Pi - dt * dG0[x] * Pr;
    s1 += 2.0 * dt * de1 * Pi - dt * dG1[x] * Pr;
    s2 += 2.0 * dt * ieta * sh * Pi - dt * ieta * a.Gam[gN + x] * Pr;
    double pr = 1.0;
    for (int k = 0; k < nj && k < kMaxJ; ++k)
      pr *= a.zdiag[(static_cast<size_t>(g) * a.nq + rec[m0 + k].qubit) * NP + x] / rho[k];
    fr[r] = a.dre[gN + x] * pr;
    fi[r] = a.dim[gN + x] * pr;
  }
  for (int k = 0; k < nj && k < kMaxJ; ++k) {
    // 2 Re <lambda_after| diag(dz) |psi_before> / rho_k, with
    // conj(lambda_after,x) psi_before,x = d_x prod_{k' != k} (z_k',x / rho_k') conj(lambda_B,x) psi_A,x
    const int qi = rec[m0 + k].qubit;
    const size_t gi = (static_cast<size_t>(g) * 2) * a.nq + qi;
    double c0 = 0.0, c1 = 0.0;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int x = lane + 64 * r;
      if (x >= NP) continue;
      double pr = 1.0;
      for (int k2 = 0; k2 < nj && k2 < kMaxJ; ++k2)
        if (k2 != k) pr *= a.zdiag[(static_cast<size_t>(g) * a.nq + rec[m0 + k2].qubit) * NP + x] / rho[k2];
      const double lr = static_cast<double>(LB[x * LD + 2 * t]), li = static_cast<double>(LB[x * LD + 2 * t + 1]);
      const double ar = static_cast<double>(PA[x * LD + 2 * t]), ai = static_cast<double>(PA[x * LD + 2 * t + 1]);
      const double qr = lr * ar + li * ai, qm = lr * ai - li * ar;   // conj(lambda_B) psi_A
      const double re = (a.dre[gN + x] * qr - a.dim[gN + x] * qm) * pr;
      c0 += a.dzd[gi * NP + x] * re;
      c1 += a.dzd[(gi + a.nq) * NP + x] * re;
    }
    s0 += 2.0 * c0 / rho[k];
    s1 += 2.0 * c1 / rho[k];
    if (lane == 0) s2 += f * ieta;   // summed over lanes below
  }
  S[0] += wave_sum(s0);
  S[1] += wave_sum(s1);
  S[2] += wave_sum(s2);
  // lambda_A = conj(F) lambda_B
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int x = lane + 64 * r;
    if (x >= NP) continue;
    const double lr = static_cast<double>(LB[x * LD + 2 * t]), li = static_cast<double>(LB[x * LD + 2 * t + 1]);
    LA[x * LD + 2 * t] = static_cast<T>(fr[r] * lr + fi[r] * li);
    LA[x * LD + 2 * t + 1] = static_cast<T>(fr[r] * li - fi[r] * lr);
  }
}

template <int NP, int TT, class T>
__global__ __launch_bounds__(kGThreads) void k_grad(GradArgs a) {
  using SH = GradShared<NP, TT, T>;
  constexpr int NC = SH::NC, LD = SH::LD;
  __shared__ SH sh;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t tile = a.tile0 + blockIdx.x;
  const int64_t lt = blockIdx.x;   // tile within this launch (workspace index)
  const int P = 2 * a.nctrl + 1;
  T* ck = static_cast<T*>(a.ckpt) + lt * a.S * NP * NC;
  int* ckc = a.ckcur + lt * a.S * TT;
  T* sg = static_cast<T*>(a.seg) + lt * a.C * NP * NC;
  int* scur = a.scur + lt * a.C * TT;
  auto traj = [&](int t) { return tile * TT + t; };
  auto active = [&](int t) { return traj(t) < a.K; };
  auto recs = [&](int t) { return a.jumps + traj(t) * a.cap; };
  auto count = [&](int t) { return a.jcount[traj(t)]; };
  // roles of the four LDS tiles (workgroup-uniform): post-kick state, end-of-step state,
  // adjoint of the projector, adjoint of the identity
  int iA = 0, iB = 1, iL = 2, iM = 3;

  auto kick = [&](int g) {   // A = O_g B (g >= 2) or the initial state (g = 1)
    T* PA = sh.buf[iA];
    if (g == 1) {
      for (int f = tid; f < NP * NC; f += kGThreads) {
        const int x = f / NC, col = f % NC;
        PA[x * LD + col] = (!(col & 1) && active(col >> 1)) ? static_cast<T>(a.cinit[x]) : static_cast<T>(0);
      }
    } else {
      gemm_kick<NP, NC, LD, T>(static_cast<const T*>(a.pD) + static_cast<size_t>(g) * NP * NP, sh.buf[iB], PA);
    }
  };
  auto forward = [&](int g) {   // B = step g (A); advances the cursors
    for (int t = wave; t < TT; t += kGW) {
      if (!active(t)) continue;
      const int m0 = sh.cur[t];
      const int m1 = step_end(recs(t), count(t), m0, g);
      replay_step<NP, LD, T>(a, g, recs(t), m0, m1, sh.buf[iA], sh.buf[iB], t, nullptr);
      if (lane == 0) sh.cur[t] = m1;
    }
  };

  // ---- forward replay with checkpoints (not needed when one segment spans the anneal)
  for (int t = tid; t < TT; t += kGThreads) sh.cur[t] = 0;
  for (int f = tid; f < NP * LD; f += kGThreads) {
    sh.buf[iB][f] = static_cast<T>(0);
    sh.buf[iL][f] = static_cast<T>(0);
    sh.buf[iM][f] = static_cast<T>(0);
  }
  __syncthreads();
  for (int g = 1; a.S > 1 && g < a.M; ++g) {
    kick(g);
    __syncthreads();
    forward(g);
    __syncthreads();
    if (g % a.C == 0 && g < a.M - 1) {
      const int s = g / a.C;
      tile_store<NP, NC, LD, T>(sh.buf[iB], ck + static_cast<size_t>(s) * NP * NC);
      for (int t = tid; t < TT; t += kGThreads) ckc[s * TT + t] = sh.cur[t];
      __syncthreads();
    }
  }

  // ---- backward, one segment at a time (last first)
  for (int s = a.S - 1; s >= 0; --s) {
    const int glo = s * a.C + 1, ghi = std::min((s + 1) * a.C, a.M - 1);
    if (s > 0) tile_load<NP, NC, LD, T>(ck + static_cast<size_t>(s) * NP * NC, sh.buf[iB]);
    for (int t = tid; t < TT; t += kGThreads) sh.cur[t] = (s > 0) ? ckc[s * TT + t] : 0;
    __syncthreads();
    for (int g = glo; g <= ghi; ++g) {
      kick(g);
      for (int t = tid; t < TT; t += kGThreads) scur[(g - glo) * TT + t] = sh.cur[t];
      __syncthreads();
      tile_store<NP, NC, LD, T>(sh.buf[iA], sg + static_cast<size_t>(g - glo) * NP * NC);
      if (g < ghi) forward(g);
      __syncthreads();
    }
    for (int g = ghi; g >= glo; --g) {
      T* PA = sh.buf[iA];
      T* PB = sh.buf[iB];
      T* LP = sh.buf[iL];
      T* LI = sh.buf[iM];
      tile_load<NP, NC, LD, T>(sg + static_cast<size_t>(g - glo) * NP * NC, PA);
      for (int f = tid; f < kGW * 4 * TT; f += kGThreads) (&sh.part[0][0][0])[f] = 0.0;
      __syncthreads();
      // end-of-step state (and the adjoints' final condition at the last grid point)
      for (int t = wave; t < TT; t += kGW) {
        if (!active(t)) continue;
        const aqt_jump* rec = recs(t);
        const int m0 = scur[(g - glo) * TT + t];
        const int m1 = step_end(rec, count(t), m0, g);
        if (m1 - m0 > kMaxJ && lane == 0) a.status[0] = 1;
        replay_step<NP, LD, T>(a, g, rec, m0, m1, PA, PB, t, sh.rho[t]);
        if (g == a.M - 1) {
          // lambda = Pi psi / |psi|^2 (Pi: ground cluster of the last grid point) and psi / |psi|^2
          const int gsz = a.proj;
          double nn = 0.0, pg = 0.0;
          for (int x = lane; x < NP; x += 64) {
            const double br = static_cast<double>(PB[x * LD + 2 * t]), bi = static_cast<double>(PB[x * LD + 2 * t + 1]);
            nn += br * br + bi * bi;
            if (x < gsz) pg += br * br + bi * bi;
          }
          nn = wave_sum(nn);
          pg = wave_sum(pg);
          for (int x = lane; x < NP; x += 64) {
            const double br = static_cast<double>(PB[x * LD + 2 * t]), bi = static_cast<double>(PB[x * LD + 2 * t + 1]);
            const double w = (x < gsz) ? 1.0 / nn : 0.0;
            LP[x * LD + 2 * t] = static_cast<T>(w * br);
            LP[x * LD + 2 * t + 1] = static_cast<T>(w * bi);
            LI[x * LD + 2 * t] = static_cast<T>(br / nn);
            LI[x * LD + 2 * t + 1] = static_cast<T>(bi / nn);
          }
          if (lane == 0) sh.f[t] = pg / nn;
        }
      }
      __syncthreads();
      // basis-change terms at the end of the step (the point before O_{g+1}); in FP64 the
      // product for the point just after O_g comes from the same pass over X_g and is held
      // in registers through the backward step (in FP32 holding it spills: a second pass)
      constexpr bool kFusedX = sizeof(T) == 8;
      const T* Xg = static_cast<const T*>(a.pX) + static_cast<size_t>(g) * NP * NP;
      typename Mfma<T>::acc_t xa[kFusedX ? rows_per_wave<NP>() : 1][NC / 16];
      if constexpr (kFusedX)
        gemm_dot2_pair<NP, NC, LD, T>(Xg, PB, PA, LP, LI, &sh.part[wave][2][0], &sh.part[wave][3][0], g < a.M - 1,
                                      xa);
      else if (g < a.M - 1)
        gemm_dot2<NP, NC, LD, T>(Xg, PB, LP, LI, &sh.part[wave][2][0], &sh.part[wave][3][0]);
      __syncthreads();
      // backward through the step, both adjoints in place
      for (int t = wave; t < TT; t += kGW) {
        if (!active(t)) {
          if (lane < 6) sh.S[t][lane] = 0.0;
          continue;
        }
        const aqt_jump* rec = recs(t);
        const int m0 = scur[(g - glo) * TT + t];
        const int m1 = step_end(rec, count(t), m0, g);
        double S1[3] = {0.0, 0.0, 0.0}, S2[3] = {0.0, 0.0, 0.0};
        adjoint_step<NP, LD, T>(a, g, rec, m0, m1, PA, PB, LP, LP, t, sh.f[t], sh.rho[t], S1);
        adjoint_step<NP, LD, T>(a, g, rec, m0, m1, PA, PB, LI, LI, t, 1.0, sh.rho[t], S2);
        if (g == 1) {
          // grid 0 through the initial state: 2 Re <lambda_A | dcin>
          double c[4] = {0.0, 0.0, 0.0, 0.0};
          for (int x = lane; x < NP; x += 64) {
            const double l1 = static_cast<double>(LP[x * LD + 2 * t]), l2 = static_cast<double>(LI[x * LD + 2 * t]);
            c[0] += l1 * a.dcin[x];
            c[1] += l1 * a.dcin[NP + x];
            c[2] += l2 * a.dcin[x];
            c[3] += l2 * a.dcin[NP + x];
          }
          for (int q = 0; q < 4; ++q) c[q] = wave_sum(c[q]);
          if (lane == 0) {
            double* o = a.out + traj(t) * a.ostride;
            o[1] += 2.0 * c[0];            // grid 0: s = 0, weight 1 on control 0
            o[1 + a.nctrl] += 2.0 * c[1];
            o[P + 2] += 2.0 * c[2];
            o[P + 2 + a.nctrl] += 2.0 * c[3];
          }
        }
        if (lane == 0)
          for (int q = 0; q < 3; ++q) {
            sh.S[t][q] = S1[q];
            sh.S[t][3 + q] = S2[q];
          }
      }
      __syncthreads();
      // basis-change terms just after O_g
      if constexpr (kFusedX)
        gemm_dot2_finish<NP, NC, LD, T>(xa, LP, LI, &sh.part[wave][0][0], &sh.part[wave][1][0]);
      else
        gemm_dot2<NP, NC, LD, T>(Xg, PA, LP, LI, &sh.part[wave][0][0], &sh.part[wave][1][0]);
      __syncthreads();
      for (int t = tid; t < TT; t += kGThreads) {
        if (!active(t)) continue;
        const double u = a.sg[g] * (a.nctrl - 1);
        const int j = std::min(static_cast<int>(floor(u)), a.nctrl - 2);
        const double fr = u - j;
        for (int adj = 0; adj < 2; ++adj) {
          double pa = 0.0, pb = 0.0;
          for (int w = 0; w < kGW; ++w) {
            pa += sh.part[w][adj][t];
            pb += sh.part[w][2 + adj][t];
          }
          double xa[2];
          for (int dir = 0; dir < 2; ++dir) xa[dir] = sh.S[t][3 * adj + dir] + 2.0 * a.xc[3 * g + dir] * (pb - pa);
          double* o = a.out + traj(t) * a.ostride + adj * (P + 1);
          o[1 + j] += (1.0 - fr) * xa[0];
          o[2 + j] += fr * xa[0];
          o[1 + a.nctrl + j] += (1.0 - fr) * xa[1];
          o[2 + a.nctrl + j] += fr * xa[1];
          o[P] += sh.S[t][3 * adj + 2];
          if (g == a.M - 1) o[0] = adj ? 1.0 : sh.f[t];
        }
      }
      // adjoints before the kick, lambda_B(g - 1) = O_g^T lambda_A(g), into the two state
      // tiles of this step; the tiles then swap roles
      if (g >= 2) {
        const T* DT = static_cast<const T*>(a.pDT) + static_cast<size_t>(g) * NP * NP;
        gemm_kick2<NP, NC, LD, T>(DT, LP, PB, LI, PA);
        int tmp = iL;
        iL = iB;
        iB = tmp;
        tmp = iM;
        iM = iA;
        iA = tmp;
      }
      __syncthreads();
    }
  }
}

// Per column c < half of out[K][2 half]: sums of v = out[j][c], v^2, w = out[j][c + half],
// w^2 and v w (one workgroup per column, fixed order).
__global__ __launch_bounds__(256) void k_colstats(const double* __restrict__ out, int64_t K, int half,
                                                  double* __restrict__ stats) {
  __shared__ double r[5][4];
  const int c = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t j = tid; j < K; j += 256) {
    const double v = out[j * 2 * half + c], w = out[j * 2 * half + half + c];
    acc[0] += v;
    acc[1] += v * v;
    acc[2] += w;
    acc[3] += w * w;
    acc[4] += v * w;
  }
  for (int q = 0; q < 5; ++q) {
    const double t = wave_sum(acc[q]);
    if (lane == 0) r[q][wave] = t;
  }
  __syncthreads();
  if (tid < 5) stats[5 * c + tid] = r[tid][0] + r[tid][1] + r[tid][2] + r[tid][3];
}

// State-precision copies of O_g - I, its transpose and X_g (the direction xc[g][2] of the
// FP64 tables) for the sweep's products.
template <class T>
__global__ void k_grad_pack(const double* __restrict__ dlt, const double* __restrict__ Xd,
                            const double* __restrict__ xc, int M, int NP, T* __restrict__ D, T* __restrict__ DT,
                            T* __restrict__ X) {
  const int64_t per = static_cast<int64_t>(NP) * NP;
  const int64_t tot = per * M;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < tot;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t g = i / per, r = i - g * per;
    const int a = static_cast<int>(r / NP), b = static_cast<int>(r - static_cast<int64_t>(a) * NP);
    D[i] = static_cast<T>(dlt[i]);
    DT[i] = static_cast<T>(dlt[g * per + static_cast<int64_t>(b) * NP + a]);
    const int dir = (xc[3 * g + 2] != 0.0) ? 1 : 0;
    X[i] = static_cast<T>(Xd[(2 * g + dir) * per + r]);
  }
}

// Segment length: the whole anneal (every post-kick state kept, no checkpoint pass)
// when that fits the workspace budget for at least one CU-full of tiles; else about
// sqrt(M - 1) steps with checkpoints.  Launches take whole CU-fulls of tiles.
template <int NP, int TT, class T>
aqt_status launch_sweep(aqt_ctx* ctx, GradArgs& ga, int64_t tiles, int cus, int seg_req) {
  constexpr int NC = 2 * TT;
  const size_t budget = size_t(40) << 30;   // of 288 GB HBM
  auto per_tile = [&](int C, int S) {
    return (static_cast<size_t>(S) + C) * NP * NC * sizeof(T) + (static_cast<size_t>(S) + C) * TT * 4;
  };
  const int steps = ga.M - 1;
  const int64_t want = std::min<int64_t>(tiles, cus);
  if (seg_req > 0) {
    ga.C = std::min(seg_req, steps);
  } else if (static_cast<int64_t>(budget / per_tile(steps, 1)) >= want) {
    ga.C = steps;
  } else {
    ga.C = std::max(1, static_cast<int>(std::ceil(std::sqrt(static_cast<double>(steps)))));
  }
  ga.S = (steps + ga.C - 1) / ga.C;
  const size_t pt = per_tile(ga.C, ga.S);
  int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(tiles, static_cast<int64_t>(budget / pt)));
  if (chunk < tiles && chunk >= cus) chunk = (chunk / cus) * cus;
  DevBuf ws;
  if (ws.reserve(pt * chunk) != hipSuccess) return ctx->fail(AQT_ENOMEM, "gradient workspace allocation failed");
  char* base = static_cast<char*>(ws.p);
  const size_t st = static_cast<size_t>(chunk) * NP * NC * sizeof(T);
  ga.ckpt = base;
  ga.seg = base + st * ga.S;
  ga.ckcur = reinterpret_cast<int*>(base + st * (ga.S + ga.C));
  ga.scur = ga.ckcur + static_cast<size_t>(chunk) * ga.S * TT;
  for (int64_t t0 = 0; t0 < tiles; t0 += chunk) {
    ga.tile0 = t0;
    const int64_t nt = std::min(chunk, tiles - t0);
    hipLaunchKernelGGL((k_grad<NP, TT, T>), dim3(static_cast<unsigned>(nt)), dim3(kGThreads), 0, ctx->stream, ga);
    AQT_HIP(ctx, hipGetLastError());
  }
  AQT_HIP(ctx, hipStreamSynchronize(ctx->stream));   // the workspace is freed on return
  return AQT_OK;
}

}  // namespace

aqt_status launch_grad(aqt_ctx* ctx, const aqt_run_params* p, double* value, double* value_se, double* grad,
                       double* grad_se, double* per_traj) {
  const int64_t K = p->n_traj;
  const int nctrl = static_cast<int>(ctx->A_ctrl.size());
  if (nctrl < 2) return ctx->fail(AQT_EINVAL, "the gradient needs at least two control points");
  {
    const aqt_status s = check_step_decay(ctx, p->precision);
    if (s != AQT_OK) return s;
  }
  const int P = 2 * nctrl + 1;
  const int NP = ctx->NP;
  hipStream_t st = ctx->stream;

  // forward paths from the trajectory kernel, every jump recorded
  DevBuf jc, jr, outb, stats, status;
  if (jc.reserve(K * 4) || status.reserve(4) || stats.reserve(5 * (P + 1) * 8))
    return ctx->fail(AQT_ENOMEM, "gradient allocation failed");
  int cap = 32;
  for (int attempt = 0; attempt < 2; ++attempt) {
    if (jr.reserve(static_cast<size_t>(K) * cap * sizeof(aqt_jump)) != hipSuccess)
      return ctx->fail(AQT_ENOMEM, "jump record allocation failed");
    aqt_run_params rp = *p;
    rp.record_capacity = cap;
    aqt_outputs o{};
    o.jump_count = jc.as<int32_t>();
    o.jumps = jr.as<aqt_jump>();
    aqt_status s = launch_run(ctx, &rp, &o);
    if (s != AQT_OK) return s;
    std::vector<int32_t> cnt(K);
    AQT_HIP(ctx, hipMemcpyAsync(cnt.data(), jc.p, K * 4, hipMemcpyDeviceToHost, st));
    AQT_HIP(ctx, hipStreamSynchronize(st));
    const int mx = cnt.empty() ? 0 : *std::max_element(cnt.begin(), cnt.end());
    if (mx <= cap) break;
    if (attempt == 1) return ctx->fail(AQT_ENUMERIC, "jump counts changed between identical runs");
    cap = mx;
  }

  // per trajectory: [f, g (P)] for the ground-cluster projector, then [1, s (P)] for the
  // identity (s = d log |psi~|^2, the path-density score: mean zero, a control variate)
  double* out = per_traj;
  const size_t rowb = 2 * static_cast<size_t>(P + 1) * 8;
  if (!out) {
    if (outb.reserve(static_cast<size_t>(K) * rowb) != hipSuccess)
      return ctx->fail(AQT_ENOMEM, "gradient output allocation failed");
    out = outb.as<double>();
  }
  AQT_HIP(ctx, hipMemsetAsync(out, 0, static_cast<size_t>(K) * rowb, st));
  int gs_last = 1;
  AQT_HIP(ctx, hipMemcpy(&gs_last, ctx->gs.as<int>() + (ctx->M - 1), 4, hipMemcpyDeviceToHost));
  AQT_HIP(ctx, hipMemsetAsync(status.p, 0, 4, st));

  GradArgs ga{};
  ga.cinit = ctx->cinit.as<double>();
  ga.E = ctx->E.as<double>();
  ga.Gam = ctx->Gamma.as<double>();
  ga.zdiag = ctx->zdiag.as<double>();
  ga.dre = ctx->dre.as<double>();
  ga.dim = ctx->dim.as<double>();
  ga.dE = ctx->dE.as<double>();
  ga.dGam = ctx->dGam.as<double>();
  ga.dzd = ctx->dzd.as<double>();
  ga.dll = ctx->dll.as<double>();
  ga.dcin = ctx->dcin.as<double>();
  ga.shift = ctx->shift.as<double>();
  ga.dshift = ctx->dshift.as<double>();
  ga.lamb = ctx->lamb ? 1 : 0;
  ga.jumps = jr.as<aqt_jump>();
  ga.jcount = jc.as<int32_t>();
  ga.cap = cap;
  ga.out = out;
  ga.ostride = 2 * (P + 1);
  ga.status = status.as<int>();
  ga.M = ctx->M;
  ga.nq = ctx->tab_nch;   // jump channels
  ga.nctrl = nctrl;
  ga.tbeg = ctx->tbeg.as<double>();
  ga.tlen = ctx->tlen.as<double>();
  ga.sg = ctx->sgd.as<double>();
  ga.eta = ctx->eta;
  ga.K = K;
  if (!(ga.eta > 0.0)) return ctx->fail(AQT_EINVAL, "the gradient needs eta > 0");

  const bool f64 = p->precision == AQT_FP64;
  const int cus = ctx->cus > 0 ? ctx->cus : 256;
  if (ctx->gpk_prec != p->precision) {
    const int M = ctx->M;
    if (static_cast<int>(ctx->sched_A.size()) != M || static_cast<int>(ctx->sched_B.size()) != M)
      return ctx->fail(AQT_ESTATE, "schedule samples missing; call aqt_precompute");
    // A X^A + B X^B = 0 at every grid point: X_g holds X^B when |A| >= |B| (then
    // X^A = -(B / A) X^B), else X^A; the other direction is a scaling of magnitude <= 1
    std::vector<double> xc(3 * static_cast<size_t>(M));
    for (int g = 0; g < M; ++g) {
      const double A = ctx->sched_A[g], B = ctx->sched_B[g];
      double* c = &xc[3 * static_cast<size_t>(g)];
      if (A == 0.0 && B == 0.0) {
        c[0] = 1.0, c[1] = 0.0, c[2] = 0.0;
      } else if (std::fabs(A) >= std::fabs(B)) {
        c[0] = -B / A, c[1] = 1.0, c[2] = 1.0;
      } else {
        c[0] = 1.0, c[1] = -A / B, c[2] = 0.0;
      }
    }
    const size_t el = f64 ? 8 : 4, per = static_cast<size_t>(NP) * NP * M;
    if (ctx->gpk_D.reserve(per * el) || ctx->gpk_DT.reserve(per * el) || ctx->gpk_X.reserve(per * el) ||
        ctx->gpk_xc.reserve(xc.size() * 8))
      return ctx->fail(AQT_ENOMEM, "gradient operand allocation failed");
    AQT_HIP(ctx, hipMemcpyAsync(ctx->gpk_xc.p, xc.data(), xc.size() * 8, hipMemcpyHostToDevice, st));
    AQT_HIP(ctx, hipStreamSynchronize(st));
    const unsigned blocks = static_cast<unsigned>(std::min<size_t>(65536, (per + 255) / 256));
    if (f64)
      hipLaunchKernelGGL(k_grad_pack<double>, dim3(blocks), dim3(256), 0, st, ctx->dlt.as<double>(),
                         ctx->Xd.as<double>(), ctx->gpk_xc.as<double>(), M, NP, ctx->gpk_D.as<double>(),
                         ctx->gpk_DT.as<double>(), ctx->gpk_X.as<double>());
    else
      hipLaunchKernelGGL(k_grad_pack<float>, dim3(blocks), dim3(256), 0, st, ctx->dlt.as<double>(),
                         ctx->Xd.as<double>(), ctx->gpk_xc.as<double>(), M, NP, ctx->gpk_D.as<float>(),
                         ctx->gpk_DT.as<float>(), ctx->gpk_X.as<float>());
    AQT_HIP(ctx, hipGetLastError());
    ctx->gpk_prec = p->precision;
  }
  ga.pD = ctx->gpk_D.p;
  ga.pDT = ctx->gpk_DT.p;
  ga.pX = ctx->gpk_X.p;
  ga.xc = ctx->gpk_xc.as<double>();
  aqt_status s = AQT_OK;
#define AQT_SWEEP(np, tt, T) s = launch_sweep<np, tt, T>(ctx, ga, (K + (tt) - 1) / (tt), cus, p->segment)
  {
    ga.out = out;
    ga.proj = gs_last;
    switch (NP) {
      case 16: if (f64) AQT_SWEEP(16, 16, double); else AQT_SWEEP(16, 16, float); break;
      case 32: if (f64) AQT_SWEEP(32, 16, double); else AQT_SWEEP(32, 16, float); break;
      case 64: if (f64) AQT_SWEEP(64, 16, double); else AQT_SWEEP(64, 16, float); break;
      case 128: if (f64) AQT_SWEEP(128, 16, double); else AQT_SWEEP(128, 16, float); break;
      case 256: if (f64) AQT_SWEEP(256, 8, double); else AQT_SWEEP(256, 16, float); break;
      default: return ctx->fail(AQT_EINVAL, "unsupported level count");
    }
    if (s != AQT_OK) return s;
  }
#undef AQT_SWEEP
  int hstat = 0;
  AQT_HIP(ctx, hipMemcpy(&hstat, status.p, 4, hipMemcpyDeviceToHost));
  if (hstat) return ctx->fail(AQT_ECAPACITY, "more than 32 omega = 0 jumps of one trajectory within one step");

  hipLaunchKernelGGL(k_colstats, dim3(P + 1), dim3(256), 0, st, out, K, P + 1, stats.as<double>());
  AQT_HIP(ctx, hipGetLastError());
  std::vector<double> hs(5 * (P + 1));
  AQT_HIP(ctx, hipMemcpyAsync(hs.data(), stats.p, hs.size() * 8, hipMemcpyDeviceToHost, st));
  AQT_HIP(ctx, hipStreamSynchronize(st));
  const double Kd = static_cast<double>(K);
  {
    const double mu = hs[0] / Kd, var = std::max(0.0, (hs[1] - Kd * mu * mu) / (Kd - 1));
    if (value) *value = mu;
    if (value_se) *value_se = std::sqrt(var / Kd);
  }
  // control variate: mean(g) - c mean(s), c = Cov(g, s) / Var(s) from the same sample
  for (int c = 1; c <= P; ++c) {
    const double* h = &hs[5 * c];
    const double mg = h[0] / Kd, ms = h[2] / Kd;
    const double vg = std::max(0.0, (h[1] - Kd * mg * mg) / (Kd - 1));
    const double vs = std::max(0.0, (h[3] - Kd * ms * ms) / (Kd - 1));
    const double cv = (h[4] - Kd * mg * ms) / (Kd - 1);
    const double cc = (vs > 0.0) ? cv / vs : 0.0;
    const double var = std::max(0.0, vg - cc * cv);
    if (grad) grad[c - 1] = mg - cc * ms;
    if (grad_se) grad_se[c - 1] = std::sqrt(var / Kd);
  }
  return AQT_OK;
}

}  // namespace aqt
