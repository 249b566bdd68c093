// C-ABI entry points of libaqt (declared and documented in include/aqt.h).
// Argument validation, host->device staging and call-order checks live here;
// the numerical work is in tables.hip, step.hip, precompute.hip and grad.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "aqt.h"
#include "ctx.hpp"

using aqt::DevBuf;

namespace {

aqt_status set_device(aqt_ctx* ctx) {
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return ctx->fail(AQT_EHIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
  return AQT_OK;
}

bool finite_all(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

// Copies a [rows][n][n]-shaped host array into a zero-padded [rows][NP][NP] device buffer.
aqt_status upload_padded(aqt_ctx* ctx, DevBuf& dst, const double* src, size_t rows, int n, int NP, bool square) {
  const size_t inner_src = square ? static_cast<size_t>(n) * n : n;
  const size_t inner_dst = square ? static_cast<size_t>(NP) * NP : NP;
  std::vector<double> host(rows * inner_dst, 0.0);
  for (size_t r = 0; r < rows; ++r) {
    if (square) {
      for (int a = 0; a < n; ++a)
        std::memcpy(&host[r * inner_dst + static_cast<size_t>(a) * NP], &src[r * inner_src + static_cast<size_t>(a) * n],
                    n * sizeof(double));
    } else {
      std::memcpy(&host[r * inner_dst], &src[r * inner_src], n * sizeof(double));
    }
  }
  if (dst.reserve(host.size() * sizeof(double)) != hipSuccess) return ctx->fail(AQT_ENOMEM, "table allocation failed");
  AQT_HIP(ctx, hipMemcpy(dst.p, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice));
  return AQT_OK;
}

aqt_status download_unpadded(aqt_ctx* ctx, double* dst, const DevBuf& src, size_t rows, int n, int NP, bool square) {
  const size_t inner_src = square ? static_cast<size_t>(NP) * NP : NP;
  const size_t inner_dst = square ? static_cast<size_t>(n) * n : n;
  std::vector<double> host(rows * inner_src);
  AQT_HIP(ctx, hipMemcpy(host.data(), src.p, host.size() * sizeof(double), hipMemcpyDeviceToHost));
  for (size_t r = 0; r < rows; ++r) {
    if (square) {
      for (int a = 0; a < n; ++a)
        std::memcpy(&dst[r * inner_dst + static_cast<size_t>(a) * n], &host[r * inner_src + static_cast<size_t>(a) * NP],
                    n * sizeof(double));
    } else {
      std::memcpy(&dst[r * inner_dst], &host[r * inner_src], n * sizeof(double));
    }
  }
  return AQT_OK;
}

}  // namespace

extern "C" {

int aqt_version(void) { return 10000; }

aqt_status aqt_create(aqt_ctx** out, int device, void* hip_stream) {
  if (!out) return AQT_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return AQT_EHIP;
  if (device < 0 || device >= count) return AQT_EINVAL;
  aqt_ctx* ctx = new (std::nothrow) aqt_ctx();
  if (!ctx) return AQT_ENOMEM;
  ctx->device = device;
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  if (set_device(ctx) != AQT_OK) {
    delete ctx;
    return AQT_EHIP;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
    ctx->cus = prop.multiProcessorCount;
  if (ctx->run_flags.reserve(sizeof(int)) != hipSuccess || hipMemset(ctx->run_flags.p, 0, sizeof(int)) != hipSuccess) {
    delete ctx;
    return AQT_ENOMEM;
  }
  // address of this device's no-allocation buffer (a failure only disables aqt_run_noalloc)
  (void)aqt::setup_noalloc_scratch(ctx);
  ctx->err.clear();
  *out = ctx;
  return AQT_OK;
}

aqt_status aqt_run_status(aqt_ctx* ctx, int32_t* flags) {
  if (!ctx) return AQT_EINVAL;
  aqt_status s = set_device(ctx);
  if (s != AQT_OK) return s;
  AQT_HIP(ctx, hipStreamSynchronize(ctx->stream));
  int v = 0;
  AQT_HIP(ctx, hipMemcpy(&v, ctx->run_flags.p, sizeof(int), hipMemcpyDeviceToHost));
  AQT_HIP(ctx, hipMemset(ctx->run_flags.p, 0, sizeof(int)));
  if (flags) *flags = v;
  if (v & AQT_RUN_JUMP_LIMIT)
    return ctx->fail(AQT_ENUMERIC, "a trajectory reached the limit of jumps within one step; rates too large for the step length");
  if (v & AQT_RUN_RECORDS_TRUNCATED)
    return ctx->fail(AQT_ECAPACITY, "jump records beyond record_capacity were dropped (jump_count holds the true counts)");
  return AQT_OK;
}

void aqt_destroy(aqt_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  else (void)hipDeviceSynchronize();
  delete ctx;
}

const char* aqt_last_error(const aqt_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

aqt_status aqt_set_hamiltonian(aqt_ctx* ctx, int n_qubits, const double* h, const double* J) {
  if (!ctx) return AQT_EINVAL;
  if (n_qubits < 1 || n_qubits > 16) return ctx->fail(AQT_EINVAL, "n_qubits must be in [1, 16]");
  if (!h || !J) return ctx->fail(AQT_EINVAL, "h and J must be non-null");
  if (!finite_all(h, n_qubits) || !finite_all(J, static_cast<size_t>(n_qubits) * n_qubits))
    return ctx->fail(AQT_EINVAL, "h and J must be finite");
  if (ctx->nq != n_qubits) {   // bath correlations are per qubit count
    ctx->chan.clear();
    ctx->chan_wc.clear();
    ctx->chan_x.clear();
  }
  ctx->nq = n_qubits;
  ctx->h.assign(h, h + n_qubits);
  ctx->J.assign(J, J + static_cast<size_t>(n_qubits) * n_qubits);
  ctx->have_h = true;
  ctx->have_tables = false;
  return AQT_OK;
}

aqt_status aqt_set_schedule(aqt_ctx* ctx, double t_f, int n_ctrl, const double* A_ctrl, const double* B_ctrl) {
  if (!ctx) return AQT_EINVAL;
  if (!(t_f > 0.0) || !std::isfinite(t_f)) return ctx->fail(AQT_EINVAL, "t_f must be positive");
  if (n_ctrl < 2 || !A_ctrl || !B_ctrl) return ctx->fail(AQT_EINVAL, "need n_ctrl >= 2 control points");
  if (!finite_all(A_ctrl, n_ctrl) || !finite_all(B_ctrl, n_ctrl))
    return ctx->fail(AQT_EINVAL, "schedule must be finite");
  ctx->t_f = t_f;
  ctx->A_ctrl.assign(A_ctrl, A_ctrl + n_ctrl);
  ctx->B_ctrl.assign(B_ctrl, B_ctrl + n_ctrl);
  ctx->have_sched = true;
  ctx->have_tables = false;
  return AQT_OK;
}

aqt_status aqt_set_bath(aqt_ctx* ctx, double eta, double omega_c, double T) {
  if (!ctx) return AQT_EINVAL;
  if (!(eta >= 0.0) || !(omega_c > 0.0) || !(T > 0.0) || !std::isfinite(eta) || !std::isfinite(omega_c) ||
      !std::isfinite(T))
    return ctx->fail(AQT_EINVAL, "need eta >= 0, omega_c > 0, T > 0");
  ctx->eta = eta;
  ctx->omega_c = omega_c;
  ctx->T = T;
  ctx->have_bath = true;
  ctx->have_tables = false;
  return AQT_OK;
}

aqt_status aqt_precompute(aqt_ctx* ctx, int n_grid, int n_levels, double deg_tol) {
  return aqt_precompute_ex(ctx, n_grid, n_levels, deg_tol, AQT_EIG_AUTO);
}

aqt_status aqt_precompute_ex(aqt_ctx* ctx, int n_grid, int n_levels, double deg_tol, int method) {
  if (!ctx) return AQT_EINVAL;
  if (method != AQT_EIG_AUTO && method != AQT_EIG_DENSE && method != AQT_EIG_ITERATIVE)
    return ctx->fail(AQT_EINVAL, "unknown eigensolver method");
  if (!ctx->have_h || !ctx->have_sched || !ctx->have_bath)
    return ctx->fail(AQT_ESTATE, "set_hamiltonian, set_schedule and set_bath must come first");
  const int N = 1 << ctx->nq;
  if (n_grid < 2) return ctx->fail(AQT_EINVAL, "n_grid must be >= 2");
  if (n_levels < 1 || n_levels > 256 || n_levels > N) return ctx->fail(AQT_EINVAL, "n_levels must be in [1, min(256, 2^nq)]");
  if (!(deg_tol >= 0.0)) return ctx->fail(AQT_EINVAL, "deg_tol must be >= 0");
  aqt_status s = set_device(ctx);
  if (s != AQT_OK) return s;
  ctx->have_tables = false;
  ctx->last_from_solver = false;
  s = aqt::precompute_tables(ctx, n_grid, n_levels, deg_tol, method);
  if (s != AQT_OK) return s;
  s = aqt::finish_tables(ctx);
  if (s != AQT_OK) return s;
  AQT_HIP(ctx, hipStreamSynchronize(ctx->stream));
  ctx->have_tables = true;
  ctx->last_from_solver = true;
  ctx->last_method = method;
  ctx->last_tol = deg_tol;
  return AQT_OK;
}

aqt_status aqt_set_tables(aqt_ctx* ctx, int n_grid, int n_levels, const double* E, const int32_t* gs,
                          const double* O, const double* cinit, const double* R, const double* zdiag) {
  if (!ctx) return AQT_EINVAL;
  if (!ctx->have_h || !ctx->have_sched)
    return ctx->fail(AQT_ESTATE, "set_hamiltonian and set_schedule must come first");
  if (n_grid < 2 || n_levels < 1 || n_levels > 256) return ctx->fail(AQT_EINVAL, "bad n_grid or n_levels");
  if (!ctx->sgrid.empty() && static_cast<int>(ctx->sgrid.size()) != n_grid)
    return ctx->fail(AQT_EINVAL, "n_grid differs from the point count of aqt_set_grid");
  if (!E || !gs || !O || !cinit || !R || !zdiag) return ctx->fail(AQT_EINVAL, "all table pointers are required");
  for (int g = 0; g < n_grid; ++g)
    if (gs[g] < 1 || gs[g] > n_levels) return ctx->fail(AQT_EINVAL, "ground-cluster size out of range");
  aqt_status s = set_device(ctx);
  if (s != AQT_OK) return s;
  const int n = n_levels, NP = aqt::padded_levels(n), nq = ctx->nch();   // nq: jump channels
  if (nq > std::min(NP, 64)) return ctx->fail(AQT_EINVAL, "more jump channels than min(64, padded levels)");
  ctx->have_tables = false;
  ctx->have_grad = false;
  ctx->last_from_solver = false;
  ctx->M = n_grid;
  ctx->n = n;
  ctx->NP = NP;
  ctx->tab_nch = nq;
  ctx->dt = ctx->t_f / (n_grid - 1);
  if ((s = upload_padded(ctx, ctx->E, E, n_grid, n, NP, false)) != AQT_OK) return s;
  // Delta = O - I on the n x n block, zero elsewhere
  {
    std::vector<double> dl(static_cast<size_t>(n_grid) * n * n);
    for (int g = 0; g < n_grid; ++g)
      for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
          const size_t k = (static_cast<size_t>(g) * n + a) * n + b;
          dl[k] = (g >= 2) ? O[k] - (a == b ? 1.0 : 0.0) : 0.0;
        }
    if ((s = upload_padded(ctx, ctx->dlt, dl.data(), n_grid, n, NP, true)) != AQT_OK) return s;
  }
  if ((s = upload_padded(ctx, ctx->cinit, cinit, 1, n, NP, false)) != AQT_OK) return s;
  if ((s = upload_padded(ctx, ctx->R, R, static_cast<size_t>(n_grid) * nq, n, NP, true)) != AQT_OK) return s;
  if ((s = upload_padded(ctx, ctx->zdiag, zdiag, static_cast<size_t>(n_grid) * nq, n, NP, false)) != AQT_OK) return s;
  if (ctx->gs.reserve(n_grid * sizeof(int32_t)) != hipSuccess) return ctx->fail(AQT_ENOMEM, "table allocation failed");
  AQT_HIP(ctx, hipMemcpy(ctx->gs.p, gs, n_grid * sizeof(int32_t), hipMemcpyHostToDevice));
  if (ctx->leak.reserve(n_grid * sizeof(double)) != hipSuccess) return ctx->fail(AQT_ENOMEM, "table allocation failed");
  AQT_HIP(ctx, hipMemset(ctx->leak.p, 0, n_grid * sizeof(double)));
  // host tables carry their own energies: no Lamb shift is added to them
  if (ctx->shift.reserve(static_cast<size_t>(n_grid) * NP * sizeof(double)) != hipSuccess)
    return ctx->fail(AQT_ENOMEM, "table allocation failed");
  AQT_HIP(ctx, hipMemset(ctx->shift.p, 0, static_cast<size_t>(n_grid) * NP * sizeof(double)));
  if ((s = aqt::finish_tables(ctx)) != AQT_OK) return s;
  AQT_HIP(ctx, hipStreamSynchronize(ctx->stream));
  ctx->have_tables = true;
  return AQT_OK;
}

aqt_status aqt_get_dims(aqt_ctx* ctx, int32_t* n_grid, int32_t* n_levels, int32_t* n_qubits) {
  if (!ctx) return AQT_EINVAL;
  if (!ctx->have_tables) return ctx->fail(AQT_ESTATE, "no tables loaded");
  if (n_grid) *n_grid = ctx->M;
  if (n_levels) *n_levels = ctx->n;
  if (n_qubits) *n_qubits = ctx->nq;
  return AQT_OK;
}

aqt_status aqt_get_tables(aqt_ctx* ctx, double* E, int32_t* gs, double* O, double* cinit, double* R, double* zdiag,
                          double* Gamma, double* leak) {
  if (!ctx) return AQT_EINVAL;
  if (!ctx->have_tables) return ctx->fail(AQT_ESTATE, "no tables loaded");
  aqt_status s = set_device(ctx);
  if (s != AQT_OK) return s;
  AQT_HIP(ctx, hipStreamSynchronize(ctx->stream));
  const int M = ctx->M, n = ctx->n, NP = ctx->NP, nq = ctx->tab_nch;   // nq: jump channels
  if (E && (s = download_unpadded(ctx, E, ctx->E, M, n, NP, false)) != AQT_OK) return s;
  if (gs) AQT_HIP(ctx, hipMemcpy(gs, ctx->gs.p, M * sizeof(int32_t), hipMemcpyDeviceToHost));
  if (O) {
    if ((s = download_unpadded(ctx, O, ctx->dlt, M, n, NP, true)) != AQT_OK) return s;
    for (int g = 0; g < M; ++g)
      for (int a = 0; a < n; ++a) O[(static_cast<size_t>(g) * n + a) * n + a] += 1.0;
  }
  if (cinit && (s = download_unpadded(ctx, cinit, ctx->cinit, 1, n, NP, false)) != AQT_OK) return s;
  if (R && (s = download_unpadded(ctx, R, ctx->R, static_cast<size_t>(M) * nq, n, NP, true)) != AQT_OK) return s;
  if (zdiag && (s = download_unpadded(ctx, zdiag, ctx->zdiag, static_cast<size_t>(M) * nq, n, NP, false)) != AQT_OK)
    return s;
  if (Gamma && (s = download_unpadded(ctx, Gamma, ctx->Gamma, M, n, NP, false)) != AQT_OK) return s;
  if (leak) AQT_HIP(ctx, hipMemcpy(leak, ctx->leak.p, M * sizeof(double), hipMemcpyDeviceToHost));
  return AQT_OK;
}

aqt_status aqt_run(aqt_ctx* ctx, const aqt_run_params* p, const aqt_outputs* o) {
  if (!ctx) return AQT_EINVAL;
  if (!p || !o) return ctx->fail(AQT_EINVAL, "params and outputs are required");
  if (!ctx->have_tables) return ctx->fail(AQT_ESTATE, "precompute or set_tables must come first");
  if (p->n_traj < 1) return ctx->fail(AQT_EINVAL, "n_traj must be >= 1");
  if (p->precision < AQT_FP64 || p->precision > AQT_BF16) return ctx->fail(AQT_EINVAL, "unknown precision");
  if (p->record_capacity < 0) return ctx->fail(AQT_EINVAL, "record_capacity must be >= 0");
  if (p->record_capacity > 0 && !o->jumps) return ctx->fail(AQT_EINVAL, "record_capacity > 0 needs a jumps buffer");
  if (o->net_hist && o->hist_hi < o->hist_lo) return ctx->fail(AQT_EINVAL, "hist_hi < hist_lo");
  aqt_status s = set_device(ctx);
  if (s != AQT_OK) return s;
  return aqt::launch_run(ctx, p, o);
}

aqt_status aqt_run_noalloc(aqt_ctx* ctx, const aqt_run_params* p, const aqt_outputs* o) {
  if (!ctx) return AQT_EINVAL;
  if (!p || !o) return ctx->fail(AQT_EINVAL, "params and outputs are required");
  if (!ctx->have_tables) return ctx->fail(AQT_ESTATE, "precompute or set_tables must come first");
  if (p->n_traj < 1) return ctx->fail(AQT_EINVAL, "n_traj must be >= 1");
  if (p->precision < AQT_FP64 || p->precision > AQT_BF16) return ctx->fail(AQT_EINVAL, "unknown precision");
  if (p->record_capacity < 0) return ctx->fail(AQT_EINVAL, "record_capacity must be >= 0");
  if (p->record_capacity > 0 && !o->jumps) return ctx->fail(AQT_EINVAL, "record_capacity > 0 needs a jumps buffer");
  if (o->net_hist && o->hist_hi < o->hist_lo) return ctx->fail(AQT_EINVAL, "hist_hi < hist_lo");
  aqt_status s = set_device(ctx);
  if (s != AQT_OK) return s;
  return aqt::launch_run_noalloc(ctx, p, o);
}

aqt_status aqt_run_fixed_step(aqt_ctx* ctx, const aqt_run_params* p, int substeps, const aqt_outputs* o) {
  if (!ctx) return AQT_EINVAL;
  if (!p || !o) return ctx->fail(AQT_EINVAL, "params and outputs are required");
  if (!ctx->have_tables) return ctx->fail(AQT_ESTATE, "precompute or set_tables must come first");
  if (p->n_traj < 1) return ctx->fail(AQT_EINVAL, "n_traj must be >= 1");
  if (p->precision != AQT_FP64 && p->precision != AQT_FP32)
    return ctx->fail(AQT_EINVAL, "the fixed-step unraveling runs in AQT_FP64 or AQT_FP32");
  if (substeps < 1) return ctx->fail(AQT_EINVAL, "substeps must be >= 1");
  if (p->record_capacity < 0) return ctx->fail(AQT_EINVAL, "record_capacity must be >= 0");
  if (p->record_capacity > 0 && !o->jumps) return ctx->fail(AQT_EINVAL, "record_capacity > 0 needs a jumps buffer");
  if (o->net_hist) return ctx->fail(AQT_EINVAL, "the fixed-step unraveling does not fill net_hist");
  aqt_status s = set_device(ctx);
  if (s != AQT_OK) return s;
  return aqt::launch_fixed_step(ctx, p, substeps, o);
}

aqt_status aqt_set_bath_correlation(aqt_ctx* ctx, const double* C) {
  if (!ctx) return AQT_EINVAL;
  if (!ctx->have_h) return ctx->fail(AQT_ESTATE, "set_hamiltonian must come first");
  const int nq = ctx->nq;
  if (!C) {
    ctx->chan.clear();
    ctx->chan_wc.clear();
    ctx->chan_x.clear();
  } else {
    double scale = 0.0;
    for (int i = 0; i < nq * nq; ++i) {
      if (!std::isfinite(C[i])) return ctx->fail(AQT_EINVAL, "correlation matrix has non-finite entries");
      scale = std::max(scale, std::fabs(C[i]));
    }
    for (int i = 0; i < nq; ++i)
      for (int j = 0; j < i; ++j)
        if (std::fabs(C[i * nq + j] - C[j * nq + i]) > 1e-12 * scale)
          return ctx->fail(AQT_EINVAL, "correlation matrix is not symmetric");
    std::vector<double> L(static_cast<size_t>(nq) * nq, 0.0);
    for (int j = 0; j < nq; ++j) {
      double d = C[j * nq + j];
      for (int k = 0; k < j; ++k) d -= L[j * nq + k] * L[j * nq + k];
      if (!(d > 1e-12 * scale)) return ctx->fail(AQT_EINVAL, "correlation matrix is not positive definite");
      L[j * nq + j] = std::sqrt(d);
      for (int i = j + 1; i < nq; ++i) {
        double v = C[i * nq + j];
        for (int k = 0; k < j; ++k) v -= L[i * nq + k] * L[j * nq + k];
        L[i * nq + j] = v / L[j * nq + j];
      }
    }
    ctx->chan.assign(static_cast<size_t>(nq) * nq, 0.0);
    for (int k = 0; k < nq; ++k)
      for (int a = 0; a < nq; ++a) ctx->chan[static_cast<size_t>(k) * nq + a] = L[a * nq + k];
    ctx->chan_wc.assign(nq, 0.0);
    ctx->chan_x.clear();
  }
  ctx->have_tables = false;
  ctx->have_grad = false;
  return AQT_OK;
}

aqt_status aqt_set_bath_terms(aqt_ctx* ctx, int n_terms, const double* C, const double* omega_c) {
  if (!ctx) return AQT_EINVAL;
  if (!ctx->have_h) return ctx->fail(AQT_ESTATE, "set_hamiltonian must come first");
  const int nq = ctx->nq;
  if (n_terms == 0) {
    ctx->chan.clear();
    ctx->chan_wc.clear();
    ctx->chan_x.clear();
    ctx->have_tables = false;
    ctx->have_grad = false;
    return AQT_OK;
  }
  if (n_terms < 0 || !C || !omega_c) return ctx->fail(AQT_EINVAL, "bath terms need C and omega_c");
  std::vector<double> chan, wc;
  for (int m = 0; m < n_terms; ++m) {
    const double* Cm = C + static_cast<size_t>(m) * nq * nq;
    if (!(omega_c[m] > 0.0) || !std::isfinite(omega_c[m]))
      return ctx->fail(AQT_EINVAL, "bath term cutoff must be positive and finite");
    double scale = 0.0, dmax = 0.0;
    for (int i = 0; i < nq * nq; ++i) {
      if (!std::isfinite(Cm[i])) return ctx->fail(AQT_EINVAL, "bath term matrix has non-finite entries");
      scale = std::max(scale, std::fabs(Cm[i]));
    }
    for (int i = 0; i < nq; ++i) {
      dmax = std::max(dmax, Cm[i * nq + i]);
      for (int j = 0; j < i; ++j)
        if (std::fabs(Cm[i * nq + j] - Cm[j * nq + i]) > 1e-12 * scale)
          return ctx->fail(AQT_EINVAL, "bath term matrix is not symmetric");
    }
    // semidefinite Cholesky in natural order: a column whose pivot is at most
    // 1e-12 max(diag) is dropped (for a semidefinite matrix the rest of it vanishes)
    const double tol = 1e-12 * dmax;
    std::vector<double> L(static_cast<size_t>(nq) * nq, 0.0);
    std::vector<int> keep;
    for (int j = 0; j < nq; ++j) {
      double d = Cm[j * nq + j];
      for (int k : keep) d -= L[j * nq + k] * L[j * nq + k];
      if (d <= tol) {
        if (d < -1e-9 * std::max(dmax, 1e-300)) return ctx->fail(AQT_EINVAL, "bath term matrix is not semidefinite");
        continue;
      }
      L[j * nq + j] = std::sqrt(d);
      for (int i = j + 1; i < nq; ++i) {
        double v = Cm[i * nq + j];
        for (int k : keep) v -= L[i * nq + k] * L[j * nq + k];
        L[i * nq + j] = v / L[j * nq + j];
      }
      keep.push_back(j);
    }
    for (int k : keep) {
      for (int a = 0; a < nq; ++a) chan.push_back(L[a * nq + k]);
      wc.push_back(omega_c[m]);
    }
  }
  if (wc.empty()) return ctx->fail(AQT_EINVAL, "bath terms are all zero");
  if (wc.size() > 64) return ctx->fail(AQT_EINVAL, "more than 64 jump channels");
  ctx->chan = chan;
  ctx->chan_wc = wc;
  ctx->chan_x.clear();
  ctx->have_tables = false;
  ctx->have_grad = false;
  return AQT_OK;
}

aqt_status aqt_set_coupling(aqt_ctx* ctx, int n_channels, const double* cz, const double* cx,
                            const double* omega_c) {
  if (!ctx) return AQT_EINVAL;
  if (!ctx->have_h) return ctx->fail(AQT_ESTATE, "set_hamiltonian must come first");
  const int nq = ctx->nq;
  if (n_channels == 0) {
    ctx->chan.clear();
    ctx->chan_wc.clear();
    ctx->chan_x.clear();
    ctx->have_tables = false;
    ctx->have_grad = false;
    return AQT_OK;
  }
  if (n_channels < 0 || n_channels > 64) return ctx->fail(AQT_EINVAL, "n_channels must be in [0, 64]");
  if (!cz && !cx) return ctx->fail(AQT_EINVAL, "cz and cx cannot both be NULL");
  const size_t cnt = static_cast<size_t>(n_channels) * nq;
  std::vector<double> z(cnt, 0.0), x;
  if (cz) z.assign(cz, cz + cnt);
  if (cx) x.assign(cx, cx + cnt);
  for (double v : z)
    if (!std::isfinite(v)) return ctx->fail(AQT_EINVAL, "coupling coefficients must be finite");
  bool any_x = false;
  for (double v : x) {
    if (!std::isfinite(v)) return ctx->fail(AQT_EINVAL, "coupling coefficients must be finite");
    any_x = any_x || v != 0.0;
  }
  for (int k = 0; k < n_channels; ++k) {
    bool nz = false;
    for (int a = 0; a < nq; ++a)
      nz = nz || z[static_cast<size_t>(k) * nq + a] != 0.0 || (!x.empty() && x[static_cast<size_t>(k) * nq + a] != 0.0);
    if (!nz) return ctx->fail(AQT_EINVAL, "a channel has a zero coupling operator");
  }
  std::vector<double> wc(n_channels, 0.0);
  if (omega_c)
    for (int k = 0; k < n_channels; ++k) {
      if (!(omega_c[k] > 0.0) || !std::isfinite(omega_c[k]))
        return ctx->fail(AQT_EINVAL, "channel cutoffs must be positive and finite");
      wc[k] = omega_c[k];
    }
  ctx->chan = z;
  ctx->chan_wc = wc;
  if (any_x) ctx->chan_x = x;
  else ctx->chan_x.clear();
  ctx->have_tables = false;
  ctx->have_grad = false;
  return AQT_OK;
}

aqt_status aqt_set_grid(aqt_ctx* ctx, int n_grid, const double* s) {
  if (!ctx) return AQT_EINVAL;
  if (n_grid == 0 || !s) {
    ctx->sgrid.clear();
    ctx->have_tables = false;
    ctx->have_grad = false;
    return AQT_OK;
  }
  if (n_grid < 2) return ctx->fail(AQT_EINVAL, "a grid needs at least two points");
  if (s[0] != 0.0 || s[n_grid - 1] != 1.0) return ctx->fail(AQT_EINVAL, "grid points must run from 0 to 1");
  for (int g = 1; g < n_grid; ++g)
    if (!(s[g] > s[g - 1]) || !std::isfinite(s[g])) return ctx->fail(AQT_EINVAL, "grid points must increase");
  ctx->sgrid.assign(s, s + n_grid);
  ctx->have_tables = false;
  ctx->have_grad = false;
  return AQT_OK;
}

static aqt_status bound_checks(aqt_ctx* ctx, int n_probe) {
  if (!ctx->have_h || !ctx->have_sched || !ctx->have_bath)
    return ctx->fail(AQT_ESTATE, "set_hamiltonian, set_schedule and set_bath must come first");
  if (ctx->nq > 8) return ctx->fail(AQT_EINVAL, "the step bound needs the full spectrum: at most 8 qubits");
  if (n_probe < 3 || n_probe > 100000) return ctx->fail(AQT_EINVAL, "n_probe must be in [3, 100000]");
  return set_device(ctx);
}

aqt_status aqt_step_bound(aqt_ctx* ctx, int n_probe, double* bound) {
  if (!ctx) return AQT_EINVAL;
  if (!bound) return ctx->fail(AQT_EINVAL, "bound must not be null");
  aqt_status s = bound_checks(ctx, n_probe);
  if (s != AQT_OK) return s;
  std::vector<double> b;
  s = aqt::step_bound(ctx, n_probe, 1e-8, b);
  if (s != AQT_OK) return s;
  std::copy(b.begin(), b.end(), bound);
  return AQT_OK;
}

aqt_status aqt_bound_grid(aqt_ctx* ctx, int n_grid, int n_probe, double* sg) {
  if (!ctx) return AQT_EINVAL;
  if (!sg) return ctx->fail(AQT_EINVAL, "s must not be null");
  if (n_grid < 2) return ctx->fail(AQT_EINVAL, "n_grid must be >= 2");
  aqt_status s = bound_checks(ctx, n_probe);
  if (s != AQT_OK) return s;
  std::vector<double> out(n_grid);
  s = aqt::bound_grid(ctx, n_grid, n_probe, 1e-8, out.data());
  if (s != AQT_OK) return s;
  std::copy(out.begin(), out.end(), sg);
  return AQT_OK;
}

aqt_status aqt_bound_grid_points(aqt_ctx* ctx, double fraction, int n_probe, int32_t* n_grid) {
  if (!ctx) return AQT_EINVAL;
  if (!n_grid) return ctx->fail(AQT_EINVAL, "n_grid must not be null");
  if (!(fraction > 0.0) || !std::isfinite(fraction)) return ctx->fail(AQT_EINVAL, "fraction must be positive and finite");
  aqt_status s = bound_checks(ctx, n_probe);
  if (s != AQT_OK) return s;
  int M = 0;
  s = aqt::bound_grid_points(ctx, fraction, n_probe, 1e-8, &M);
  if (s != AQT_OK) return s;
  *n_grid = M;
  return AQT_OK;
}

aqt_status aqt_get_channel_count(aqt_ctx* ctx, int32_t* n_channels) {
  if (!ctx || !n_channels) return AQT_EINVAL;
  *n_channels = ctx->have_tables ? ctx->tab_nch : ctx->nch();
  return AQT_OK;
}

aqt_status aqt_set_lamb_shift(aqt_ctx* ctx, int enabled) {
  if (!ctx) return AQT_EINVAL;
  ctx->lamb = enabled != 0;
  ctx->have_tables = false;
  ctx->have_grad = false;
  return AQT_OK;
}

aqt_status aqt_get_lamb_shift(aqt_ctx* ctx, double* shift) {
  if (!ctx) return AQT_EINVAL;
  if (!ctx->have_tables) return ctx->fail(AQT_ESTATE, "no tables loaded");
  if (!shift) return ctx->fail(AQT_EINVAL, "shift is required");
  aqt_status s = set_device(ctx);
  if (s != AQT_OK) return s;
  AQT_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return download_unpadded(ctx, shift, ctx->shift, ctx->M, ctx->n, ctx->NP, false);
}

aqt_status aqt_grad_pgs(aqt_ctx* ctx, const aqt_run_params* p, double* value, double* value_se, double* grad,
                        double* grad_se, double* per_traj) {
  if (!ctx) return AQT_EINVAL;
  if (!p) return ctx->fail(AQT_EINVAL, "params are required");
  if (!ctx->have_tables) return ctx->fail(AQT_ESTATE, "precompute must come first");
  if (!ctx->last_from_solver)
    return ctx->fail(AQT_ESTATE, "the gradient needs tables from aqt_precompute (eigenvectors), not aqt_set_tables");
  if (ctx->n != (1 << ctx->nq))
    return ctx->fail(AQT_EINVAL, "the gradient needs the full spectrum (n_levels = 2^n_qubits)");
  if (p->n_traj < 2) return ctx->fail(AQT_EINVAL, "n_traj must be >= 2");
  if (p->precision != AQT_FP64 && p->precision != AQT_FP32)
    return ctx->fail(AQT_EINVAL, "the gradient runs in AQT_FP64 or AQT_FP32");
  if (p->segment < 0) return ctx->fail(AQT_EINVAL, "segment must be >= 0");
  aqt_status s = set_device(ctx);
  if (s != AQT_OK) return s;
  if (!ctx->have_grad) {
    ctx->have_tables = false;
    s = aqt::precompute_tables(ctx, ctx->M, ctx->n, ctx->last_tol, ctx->last_method, true);
    if (s != AQT_OK) return s;
    if ((s = aqt::finish_tables(ctx)) != AQT_OK) return s;
    AQT_HIP(ctx, hipStreamSynchronize(ctx->stream));
    ctx->have_tables = true;
  }
  return aqt::launch_grad(ctx, p, value, value_se, grad, grad_se, per_traj);
}

}  // extern "C"
