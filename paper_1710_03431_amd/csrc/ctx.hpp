// Internal state of an aqt_ctx and the host-side launchers shared between the
// C-ABI layer (api.hip) and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "aqt.h"
#include "common.hpp"

struct aqt_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;

  // ---- problem definition (host copies)
  int nq = 0;
  std::vector<double> h, J;   // J: nq*nq row-major, i<j used
  bool have_h = false;
  double t_f = 0.0;
  std::vector<double> A_ctrl, B_ctrl;
  bool have_sched = false;
  double eta = 0.0, omega_c = 0.0, T = 0.0;
  bool have_bath = false;
  bool lamb = false;    // add the Lamb shift at the next precompute
  // jump channels: coupling operator sum_a chan[k][a] sz_a and the cutoff of its Ohmic rate
  // (chan_wc[k], 0: the bath's omega_c); empty: sz of each qubit (independent baths)
  std::vector<double> chan;      // [nch][nq]
  std::vector<double> chan_wc;   // [nch]
  std::vector<double> chan_x;    // [nch][nq] sx coefficients of the channel operators (empty: none)
  int nch() const { return chan.empty() ? nq : static_cast<int>(chan.size() / nq); }
  bool single_spectrum() const {
    for (double w : chan_wc)
      if (w != 0.0) return false;
    return true;
  }

  // ---- tables (device, FP64 masters; rows padded to NP with zeros)
  bool have_tables = false;
  int M = 0;        // grid points
  int tab_nch = 0;  // jump channels of the loaded tables
  std::vector<double> sgrid;   // [M] grid points s_g of aqt_set_grid (empty: equidistant)
  aqt::DevBuf sgd;             // [M] s_g of the loaded tables
  aqt::DevBuf tbeg, tlen;      // [M] start time and length of the step into grid g (g >= 1)
  int n = 0;        // retained levels
  int NP = 0;       // padded level count: 16, 32, 64, 128 or 256
  double dt = 0.0;
  aqt::DevBuf E;        // [M][NP]
  aqt::DevBuf gs;       // [M] int32
  aqt::DevBuf dlt;      // [M][NP][NP]  Delta = O - I (row-major), zero padded; g < 2 unused
  aqt::DevBuf cinit;    // [NP]
  aqt::DevBuf R;        // [M][nq][NP(b)][NP(a)]
  aqt::DevBuf zdiag;    // [M][nq][NP]
  aqt::DevBuf Gamma;    // [M][NP]
  aqt::DevBuf Rcol;     // [M][nq][NP][4]: sum_a R[i][b][a], sum_{a<b} R[i][b][a], R[i][b][b], 0
  aqt::DevBuf ehalf;    // [M][NP] exp(+Gamma dt / 2), undoes the step's decay
  aqt::DevBuf dre, dim; // [M][NP] FP64 exp(-i e dt - Gamma dt / 2)
  aqt::DevBuf leak;     // [M]
  aqt::DevBuf shift;    // [M][NP] Lamb shift of each level (zeros when off); phases use E + shift
  double max_gdt = 0.0; // largest Gamma_b dt_g of the loaded tables (decay over one step)

  // ---- derivative tables of the gradient (direction 0 = A(s_g), 1 = B(s_g)); full spectrum only
  bool have_grad = false;
  int last_method = 0;      // eigensolver and cluster tolerance of the last aqt_precompute
  double last_tol = 0.0;
  bool last_from_solver = false;   // tables came from aqt_precompute (not aqt_set_tables)
  aqt::DevBuf Xd;       // [M][2][NP][NP] X[x][y]: dv_y = sum_x v_x X[x][y]
  aqt::DevBuf dE;       // [M][2][NP]
  aqt::DevBuf dGam;     // [M][2][NP]
  aqt::DevBuf dzd;      // [M][2][nq][NP] d z_i[x][x]
  aqt::DevBuf dll;      // [M][2][nq][NP(b)][NP(a)] d log |l_i,ab|
  aqt::DevBuf dcin;     // [2][NP] derivative of the initial state through grid 0
  aqt::DevBuf dshift;   // [M][2][NP] derivative of the Lamb shift (zeros when off)
  std::vector<double> sched_A, sched_B;   // [M] A(s_g), B(s_g) of the last aqt_precompute
  int fix_prec = -1;    // precision of the fixed-step kernel's O_g - I copy, -1 = none
  aqt::DevBuf fix_D;
  int gpk_prec = -1;    // precision of the sweep operands below, -1 = none
  aqt::DevBuf gpk_D, gpk_DT, gpk_X;   // O_g - I, its transpose, X_g in that precision
  aqt::DevBuf gpk_xc;   // [M][3] X^A_g = xc[0] X_g, X^B_g = xc[1] X_g, xc[2] = direction held in X_g

  // ---- per-precision packed operands of the step kernel (built lazily)
  int packed_for = -1;      // aqt_precision the packs below hold, -1 = none
  aqt::DevBuf pk_a, pk_b;   // Delta fragments (hi / lo for BF16)
  aqt::DevBuf pk_dre, pk_dim;  // d in the state precision
  aqt::DevBuf pk_ch;            // FP32 runs: [M][nq][NP] float4 (R row sum, sum below the diagonal, diagonal, z_bb)

  // ---- run workspace
  aqt::DevBuf partial;      // [tiles][M][2] per-tile observable sums
  aqt::DevBuf run_flags;    // int32 OR of AQT_RUN_* flags since the last aqt_run_status (allocated by aqt_create)
  int cus = 0;              // compute units of the device (queried once by aqt_create)

  aqt_status fail(aqt_status s, const std::string& msg) {
    err = msg;
    return s;
  }
};

namespace aqt {

#define AQT_HIP(ctx, expr)                                                              \
  do {                                                                                  \
    hipError_t _e = (expr);                                                             \
    if (_e != hipSuccess)                                                               \
      return (ctx)->fail(AQT_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e));  \
  } while (0)

// tables.hip: derive Gamma and d from E and R; pack the step operands.
aqt_status finish_tables(aqt_ctx* ctx);
aqt_status pack_for_precision(aqt_ctx* ctx, int precision);
// AQT_ENUMERIC if a level decays by more than the state precision carries within one step
// (max Gamma_b dt_g above 500 in FP64 runs, 50 in FP32 / BF16 runs).
aqt_status check_step_decay(aqt_ctx* ctx, int precision);

// step.hip: enqueue the trajectory kernel and the observable reduction.
aqt_status launch_run(aqt_ctx* ctx, const aqt_run_params* p, const aqt_outputs* o);
// step.hip: the same with the per-tile sums in the library's fixed device buffer (no
// allocation); setup_noalloc_scratch takes the buffer's address once per device.
aqt_status launch_run_noalloc(aqt_ctx* ctx, const aqt_run_params* p, const aqt_outputs* o);
aqt_status setup_noalloc_scratch(aqt_ctx* ctx);

// precompute.hip: GPU eigensystem and tables.
aqt_status precompute_tables(aqt_ctx* ctx, int n_grid, int n_levels, double deg_tol, int method, bool grad = false);

// grid.hip: the App. B time-step bound at n_probe equidistant points (full spectrum,
// from a scratch precompute) and the grid that equidistributes it.
aqt_status step_bound(aqt_ctx* ctx, int n_probe, double deg_tol, std::vector<double>& bound);
aqt_status bound_grid(aqt_ctx* ctx, int n_grid, int n_probe, double deg_tol, double* s_out);
constexpr int kMaxBoundGridPoints = 10000000;
aqt_status bound_grid_points(aqt_ctx* ctx, double fraction, int n_probe, double deg_tol, int* n_grid);

// mcwf.hip: fixed-step unraveling.
aqt_status launch_fixed_step(aqt_ctx* ctx, const aqt_run_params* p, int substeps, const aqt_outputs* o);

// grad.hip: adjoint gradient of the final ground-cluster population.
aqt_status launch_grad(aqt_ctx* ctx, const aqt_run_params* p, double* value, double* value_se, double* grad,
                       double* grad_se, double* per_traj);

inline int padded_levels(int n) {
  int np = 16;
  while (np < n) np *= 2;
  return np;
}

}  // namespace aqt
