// Time-step bound of App. B (eq. B7) and an s-grid that follows it.
//
// The bound at time t is min{ |H_eff| / |dH_eff/dt|, 1 / |H_eff|, |lambda / (lambda^2 -
// dlambda/dt)| } with operator norms, H_eff = H - (i/2) sum_k A_k^dag A_k the non-Hermitian
// generator of the no-jump evolution (Sec. III eq. Heff) and lambda the jump rate.  In the
// instantaneous eigenbasis H_eff = diag(h), h_b = e_b - i Gamma_b / 2 (the decay is diagonal
// there), so |H_eff| = max_b |h_b|; lambda depends on the trajectory's state and is taken at
// its largest value, max_b Gamma_b.  dH_eff/dt is a finite difference over equidistant probe
// points s_p: central inside, one-sided at the ends.  The operator norm is basis-invariant,
// so the difference is formed in the eigenbasis of probe p from the tables of a
// full-spectrum precompute on the probe points: with O_p the overlap V_p^T V_{p-1},
//   H_eff(s_{p+1}) = O_{p+1}^T diag(h_{p+1}) O_{p+1},  H_eff(s_{p-1}) = O_p diag(h_{p-1}) O_p^T,
// and |D|_2 follows from a power iteration on D^H D.  The grid equidistributes the density
// 1 / bound(s): F(s) = int_0^s ds' / bound(s') by the trapezoid rule on the probes,
// s_g = F^{-1}(g F(1) / (M - 1)) by linear interpolation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <limits>
#include <string>
#include <vector>

#include "common.hpp"
#include "ctx.hpp"

namespace aqt {
namespace {

constexpr int kDnThreads = 256;
constexpr int kDnMaxN = 256;

struct CVec {
  double* re;
  double* im;
};

// y = M x or y = M^T x for M = I + Delta (row-major NP x NP), complex x, n <= blockDim.x.
// Every thread owns row r of y; the transposed product reads Delta column-wise (coalesced).
__device__ void cmatvec(const double* __restrict__ dlt, int NP, int n, bool trans, CVec x, CVec y) {
  const int r = threadIdx.x;
  double yr = 0.0, yi = 0.0;
  if (r < n) {
    yr = x.re[r];
    yi = x.im[r];
    for (int c = 0; c < n; ++c) {
      const double m = trans ? dlt[static_cast<size_t>(c) * NP + r] : dlt[static_cast<size_t>(r) * NP + c];
      yr = fma(m, x.re[c], yr);
      yi = fma(m, x.im[c], yi);
    }
  }
  __syncthreads();   // x may alias y
  if (r < n) {
    y.re[r] = yr;
    y.im[r] = yi;
  }
  __syncthreads();
}

// Workgroup-wide sum (every thread receives it).
__device__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  const double s = red[0];
  __syncthreads();
  return s;
}

// y = D x for the finite difference at probe p (grid index g = p + 1 of the tables, whose
// index 0 duplicates s = 0): D = (X_+ - X_-) / span with X_+ = O_{g+1}^T diag(h_{g+1}) O_{g+1},
// X_- = O_g diag(h_{g-1}) O_g^T, or diag(h_g) in place of the missing side at the ends.
// conj_h applies conj(D) instead (D is complex symmetric, so D^H = conj(D)).
__device__ void apply_d(const double* __restrict__ dlt, const double* __restrict__ E, const double* __restrict__ Gam,
                        int NP, int n, int g, int gmax, double span, bool conj_h, CVec x, CVec y, CVec t1, CVec t2,
                        double* red) {
  (void)red;
  const int r = threadIdx.x;
  const double sgn = conj_h ? 1.0 : -1.0;   // Im h = -Gamma / 2 (conj: + Gamma / 2)
  // X_+ x
  if (g + 1 <= gmax) {
    const double* O1 = dlt + static_cast<size_t>(g + 1) * NP * NP;
    cmatvec(O1, NP, n, false, x, t1);
    if (r < n) {
      const double er = E[static_cast<size_t>(g + 1) * NP + r], ei = sgn * 0.5 * Gam[static_cast<size_t>(g + 1) * NP + r];
      const double a = t1.re[r], b = t1.im[r];
      t1.re[r] = er * a - ei * b;
      t1.im[r] = er * b + ei * a;
    }
    __syncthreads();
    cmatvec(O1, NP, n, true, t1, t1);
  } else if (r < n) {
    const double er = E[static_cast<size_t>(g) * NP + r], ei = sgn * 0.5 * Gam[static_cast<size_t>(g) * NP + r];
    t1.re[r] = er * x.re[r] - ei * x.im[r];
    t1.im[r] = er * x.im[r] + ei * x.re[r];
  }
  __syncthreads();
  // X_- x
  if (g - 1 >= 1) {
    const double* O0 = dlt + static_cast<size_t>(g) * NP * NP;
    cmatvec(O0, NP, n, true, x, t2);
    if (r < n) {
      const double er = E[static_cast<size_t>(g - 1) * NP + r], ei = sgn * 0.5 * Gam[static_cast<size_t>(g - 1) * NP + r];
      const double a = t2.re[r], b = t2.im[r];
      t2.re[r] = er * a - ei * b;
      t2.im[r] = er * b + ei * a;
    }
    __syncthreads();
    cmatvec(O0, NP, n, false, t2, t2);
  } else if (r < n) {
    const double er = E[static_cast<size_t>(g) * NP + r], ei = sgn * 0.5 * Gam[static_cast<size_t>(g) * NP + r];
    t2.re[r] = er * x.re[r] - ei * x.im[r];
    t2.im[r] = er * x.im[r] + ei * x.re[r];
  }
  __syncthreads();
  if (r < n) {
    y.re[r] = (t1.re[r] - t2.re[r]) / span;
    y.im[r] = (t1.im[r] - t2.im[r]) / span;
  }
  __syncthreads();
}

// |dH_eff/dt|_2 at every probe p = blockIdx.x (power iteration on D^H D from a fixed
// start vector until the Rayleigh quotient settles to 1e-13 relative or max_it steps).
__global__ __launch_bounds__(kDnThreads) void k_heff_dnorm(const double* __restrict__ dlt,
                                                           const double* __restrict__ E,
                                                           const double* __restrict__ Gam,
                                                           const double* __restrict__ tp, int NP, int n, int P,
                                                           int max_it, double* __restrict__ out) {
  __shared__ double buf[8][kDnMaxN];
  __shared__ double red[kDnThreads];
  const int p = blockIdx.x;
  const int g = p + 1, gmax = P;
  const double span = (p == 0) ? tp[1] - tp[0] : (p == P - 1 ? tp[P - 1] - tp[P - 2] : tp[p + 1] - tp[p - 1]);
  CVec v{buf[0], buf[1]}, w{buf[2], buf[3]}, t1{buf[4], buf[5]}, t2{buf[6], buf[7]};
  const int r = threadIdx.x;
  if (r < n) {
    v.re[r] = 1.0 + 0.25 * sin(1.0 + r);
    v.im[r] = 0.25 * cos(2.0 + 3.0 * r);
  }
  __syncthreads();
  double nv = block_sum(r < n ? v.re[r] * v.re[r] + v.im[r] * v.im[r] : 0.0, red);
  double mu = 0.0;
  for (int it = 0; it < max_it; ++it) {
    // w = D v, mu = |w|^2 / |v|^2, then v <- D^H w = conj(D) w (D is complex symmetric)
    apply_d(dlt, E, Gam, NP, n, g, gmax, span, false, v, w, t1, t2, red);
    const double nw = block_sum(r < n ? w.re[r] * w.re[r] + w.im[r] * w.im[r] : 0.0, red);
    const double mu_new = nw / nv;
    apply_d(dlt, E, Gam, NP, n, g, gmax, span, true, w, v, t1, t2, red);
    nv = block_sum(r < n ? v.re[r] * v.re[r] + v.im[r] * v.im[r] : 0.0, red);
    if (!(nv > 0.0)) {
      mu = mu_new;
      break;
    }
    const double inv = 1.0 / sqrt(nv);
    if (r < n) {
      v.re[r] *= inv;
      v.im[r] *= inv;
    }
    __syncthreads();
    nv = 1.0;
    const bool done = it > 8 && fabs(mu_new - mu) <= 1e-13 * mu_new;
    mu = mu_new;
    if (done) break;
  }
  if (r == 0) out[p] = sqrt(mu);
}

}  // namespace

// Full-spectrum tables on the probe points s_p = p / (P - 1) in a scratch context (the
// caller's tables stay untouched), then the bound at every probe.
aqt_status step_bound(aqt_ctx* ctx, int P, double deg_tol, std::vector<double>& bound) {
  const int N = 1 << ctx->nq;
  if (N > kDnMaxN) return ctx->fail(AQT_EINVAL, "the step bound needs the full spectrum: at most 256 basis states");
  if (P < 3) return ctx->fail(AQT_EINVAL, "n_probe must be >= 3");
  aqt_ctx tmp;
  tmp.device = ctx->device;
  tmp.stream = ctx->stream;
  tmp.cus = ctx->cus;
  tmp.nq = ctx->nq;
  tmp.h = ctx->h;
  tmp.J = ctx->J;
  tmp.have_h = true;
  tmp.t_f = ctx->t_f;
  tmp.A_ctrl = ctx->A_ctrl;
  tmp.B_ctrl = ctx->B_ctrl;
  tmp.have_sched = true;
  tmp.eta = ctx->eta;
  tmp.omega_c = ctx->omega_c;
  tmp.T = ctx->T;
  tmp.have_bath = true;
  tmp.chan = ctx->chan;
  tmp.chan_wc = ctx->chan_wc;
  tmp.chan_x = ctx->chan_x;
  // table index 0 repeats s = 0, so that index p + 1 (which carries rates) is probe p
  tmp.sgrid.resize(P + 1);
  tmp.sgrid[0] = 0.0;
  for (int p = 0; p < P; ++p) tmp.sgrid[p + 1] = static_cast<double>(p) / (P - 1);
  aqt_status s = precompute_tables(&tmp, P + 1, N, deg_tol, AQT_EIG_DENSE);
  if (s == AQT_OK) s = finish_tables(&tmp);
  if (s != AQT_OK) return ctx->fail(s, "step bound: " + tmp.err);
  const int NP = tmp.NP, n = tmp.n;
  std::vector<double> tp(P);
  for (int p = 0; p < P; ++p) tp[p] = ctx->t_f * static_cast<double>(p) / (P - 1);
  DevBuf dtp, dn;
  if (dtp.reserve(P * sizeof(double)) || dn.reserve(P * sizeof(double)))
    return ctx->fail(AQT_ENOMEM, "step bound allocation failed");
  AQT_HIP(ctx, hipMemcpyAsync(dtp.p, tp.data(), P * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  hipLaunchKernelGGL(k_heff_dnorm, dim3(P), dim3(kDnThreads), 0, ctx->stream, tmp.dlt.as<double>(), tmp.E.as<double>(),
                     tmp.Gamma.as<double>(), dtp.as<double>(), NP, n, P, 4000, dn.as<double>());
  AQT_HIP(ctx, hipGetLastError());
  std::vector<double> dnorm(P), E(static_cast<size_t>(P + 1) * NP), G(static_cast<size_t>(P + 1) * NP);
  AQT_HIP(ctx, hipMemcpyAsync(dnorm.data(), dn.p, P * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  AQT_HIP(ctx, hipMemcpyAsync(E.data(), tmp.E.p, E.size() * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  AQT_HIP(ctx, hipMemcpyAsync(G.data(), tmp.Gamma.p, G.size() * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  AQT_HIP(ctx, hipStreamSynchronize(ctx->stream));
  std::vector<double> nrm(P), lam(P), dlam(P);
  for (int p = 0; p < P; ++p) {
    double mx = 0.0, lm = 0.0;
    for (int b = 0; b < n; ++b) {
      const double e = E[static_cast<size_t>(p + 1) * NP + b], gm = G[static_cast<size_t>(p + 1) * NP + b];
      mx = std::max(mx, std::sqrt(e * e + 0.25 * gm * gm));
      lm = std::max(lm, gm);
    }
    nrm[p] = mx;
    lam[p] = lm;
  }
  for (int p = 0; p < P; ++p)
    dlam[p] = (p == 0) ? (lam[1] - lam[0]) / (tp[1] - tp[0])
                       : (p == P - 1 ? (lam[P - 1] - lam[P - 2]) / (tp[P - 1] - tp[P - 2])
                                     : (lam[p + 1] - lam[p - 1]) / (tp[p + 1] - tp[p - 1]));
  bound.assign(P, 0.0);
  for (int p = 0; p < P; ++p) {
    const double inf = std::numeric_limits<double>::infinity();
    const double b1 = dnorm[p] > 0.0 ? nrm[p] / dnorm[p] : inf;
    const double b2 = 1.0 / nrm[p];
    const double den = lam[p] * lam[p] - dlam[p];
    const double b3 = den != 0.0 ? std::fabs(lam[p] / den) : inf;
    bound[p] = std::min(std::min(b1, b2), b3);
  }
  return AQT_OK;
}

// F(s_p) = int_0^{s_p} ds / bound(s) by the trapezoid rule on the probes (units 1/ns).
static aqt_status bound_density_integral(aqt_ctx* ctx, int P, double deg_tol, std::vector<double>& sp,
                                         std::vector<double>& F) {
  std::vector<double> bound;
  aqt_status s = step_bound(ctx, P, deg_tol, bound);
  if (s != AQT_OK) return s;
  sp.assign(P, 0.0);
  F.assign(P, 0.0);
  for (int p = 0; p < P; ++p) sp[p] = static_cast<double>(p) / (P - 1);
  for (int p = 1; p < P; ++p) F[p] = F[p - 1] + 0.5 * (1.0 / bound[p] + 1.0 / bound[p - 1]) * (sp[p] - sp[p - 1]);
  if (!(F[P - 1] > 0.0) || !std::isfinite(F[P - 1])) return ctx->fail(AQT_ENUMERIC, "step bound density not integrable");
  return AQT_OK;
}

// Step control from the bound: on the bound-following grid of M points the step into
// s_g is t_f (s_g - s_{g-1}) ~ t_f F(1) bound(s_g) / (M - 1), so every step stays within
// `fraction` of the bound when M - 1 >= t_f F(1) / fraction.
aqt_status bound_grid_points(aqt_ctx* ctx, double fraction, int P, double deg_tol, int* M_out) {
  std::vector<double> sp, F;
  aqt_status s = bound_density_integral(ctx, P, deg_tol, sp, F);
  if (s != AQT_OK) return s;
  const double steps = std::ceil(ctx->t_f * F[P - 1] / fraction);
  if (!(steps <= static_cast<double>(kMaxBoundGridPoints - 1)))
    return ctx->fail(AQT_EINVAL, "the bound asks for more than " + std::to_string(kMaxBoundGridPoints) +
                                     " grid points at this fraction");
  *M_out = std::max(2, static_cast<int>(steps) + 1);
  return AQT_OK;
}

aqt_status bound_grid(aqt_ctx* ctx, int M, int P, double deg_tol, double* s_out) {
  std::vector<double> sp, F;
  aqt_status s = bound_density_integral(ctx, P, deg_tol, sp, F);
  if (s != AQT_OK) return s;
  // invert F by linear interpolation (targets are non-decreasing, so one forward pass)
  int q = 0;
  for (int g = 0; g < M; ++g) {
    const double target = F[P - 1] * static_cast<double>(g) / (M - 1);
    while (q < P - 2 && F[q + 1] < target) ++q;
    const double f0 = F[q], f1 = F[q + 1];
    const double w = (f1 > f0) ? (target - f0) / (f1 - f0) : 0.0;
    s_out[g] = sp[q] + std::min(1.0, std::max(0.0, w)) * (sp[q + 1] - sp[q]);
  }
  s_out[0] = 0.0;
  s_out[M - 1] = 1.0;
  for (int g = 1; g < M; ++g)
    if (!(s_out[g] > s_out[g - 1])) return ctx->fail(AQT_ENUMERIC, "bound grid is not increasing (too few probes)");
  return AQT_OK;
}

}  // namespace aqt
