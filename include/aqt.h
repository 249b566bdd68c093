/*
 * aqt.h -- C ABI of libaqt, an MI355X (gfx950) engine for quantum-jump
 * trajectories of the adiabatic master equation (AME).
 *
 * Method: Yip, Albash, Lidar, "Quantum trajectories for time-dependent
 * adiabatic master equations".  The AME in Lindblad form with operators in the
 * instantaneous eigenbasis (Sec. II, eqs. ME2-H, ME2-L, Lindblad2) is unravelled
 * into jump trajectories (Sec. III, eqs. Heff, sse, jump) and simulated with the
 * waiting-time procedure (Sec. IV; validity App. C).  Model: transverse-field
 * Ising system with independent Ohmic baths coupled through sz_i (Sec. V).
 *
 * Conventions (all calls):
 *   - Units: hbar = k_B = 1; energies, rates, temperature in rad/ns; time in ns.
 *   - H(s) = A(s) (-sum_i sx_i) + B(s) (sum_i h_i sz_i + sum_{i<j} J_ij sz_i sz_j),
 *     bit i of a basis index is qubit i, sz_i|x> = (1 - 2 bit_i(x)) |x>.
 *     (The paper's field term is -sum h sz; pass -h for that convention.)
 *   - Ohmic rates gamma(w) = 2 pi eta w e^{-|w|/wc} / (1 - e^{-w/T}), gamma(0) = 2 pi eta T.
 *   - Grid s_g = g/(M-1), g = 0..M-1, t = s t_f, dt = t_f/(M-1).  The step from
 *     s_{g-1} to s_g uses the generator frozen at s_g; the basis change between
 *     grid points is the polar factor of V_g^T V_{g-1}.
 *   - Errors: a negative aqt_status; aqt_last_error() returns a message that
 *     stays valid until the next call on the same context.  On AQT_EINVAL and
 *     AQT_ESTATE nothing is written to outputs.
 *   - Ownership: the library owns the context and every precomputed table; the
 *     caller owns every output buffer.  Host input arrays are copied during the
 *     call.  Device pointers must be on the context's device.
 *   - Stream order: device work is enqueued on the context's stream and the
 *     calls return without synchronising unless stated; the caller synchronises.
 *   - One context per host thread at a time; contexts are independent.
 */
#ifndef AQT_H
#define AQT_H

#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define AQT_API __attribute__((visibility("default")))
#else
#define AQT_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct aqt_ctx aqt_ctx;

typedef enum {
  AQT_OK = 0,
  AQT_EINVAL = -1,     /* an argument is out of range or a pointer is NULL          */
  AQT_ENOMEM = -2,     /* device or host allocation failed                          */
  AQT_ESTATE = -3,     /* call order: set_* -> precompute (or set_tables) -> run     */
  AQT_EHIP = -4,       /* a HIP runtime call failed                                 */
  AQT_ENUMERIC = -5,   /* eigensolver did not converge, degenerate initial state... */
  AQT_ECAPACITY = -6   /* jump records overflowed; observables are still valid      */
} aqt_status;

typedef enum {
  AQT_FP64 = 0,        /* FP64 state, FP64 MFMA overlap GEMM                        */
  AQT_FP32 = 1,        /* FP32 state, FP32 MFMA, FP32 accumulate                    */
  AQT_BF16 = 2         /* FP32 state; overlap GEMM on BF16 MFMA with hi/lo splits of
                          both operands (three products) and the identity split
                          O = I + Delta; FP32 accumulate                             */
} aqt_precision;

enum { AQT_KIND_RELAX = 0, AQT_KIND_EXCITE = 1, AQT_KIND_DEPHASE = 2 };

/* One recorded jump (24 bytes).  from_level b -> to_level a in the eigenbasis of
 * grid step+1; a == b is the omega = 0 operator of `qubit`.  kind: relax if
 * e_a <= e_b, excite otherwise, dephase for a == b. */
typedef struct {
  double t;            /* ns */
  int32_t step;        /* step index k: the step from s_k to s_{k+1} */
  int16_t qubit;
  int16_t kind;
  int32_t from_level;
  int32_t to_level;
} aqt_jump;

typedef struct {
  int32_t precision;        /* aqt_precision */
  int32_t record_capacity;  /* jump records kept per trajectory (0: none)            */
  int64_t n_traj;           /* K >= 1                                               */
  uint64_t seed;            /* Philox key word 0                                    */
  uint64_t instance_id;     /* Philox key word 1                                    */
  uint64_t traj_offset;     /* trajectory ids are traj_offset .. traj_offset+K-1     */
  int32_t tile;             /* trajectories per workgroup: 8, 16, 32, 40 or 64 (0: auto) */
  int32_t segment;          /* aqt_grad_pgs only: steps per checkpoint segment of the
                               adjoint sweep (0: automatic); ignored by aqt_run       */
} aqt_run_params;

/* Device output buffers of aqt_run (any pointer may be NULL to skip it). */
typedef struct {
  double* pgs_sum;          /* [M] sum over trajectories of the ground-cluster population
                               after each grid point (index 0 = initial state)        */
  double* pgs_sumsq;        /* [M] sum of squares (standard error, Sec. VI eq. stderror) */
  int64_t* jump_totals;     /* [3] relax, excite, dephase; accumulated (+=)            */
  int32_t* jump_count;      /* [K] jumps per trajectory (may exceed record_capacity)   */
  aqt_jump* jumps;          /* [K * record_capacity], trajectory-major                 */
  int32_t* net_gs;          /* [K] jumps into minus jumps out of the ground cluster    */
  int64_t* net_hist;        /* [hist_hi - hist_lo + 1] histogram of net_gs; accumulated,
                               values outside the range are clamped to the end bins   */
  int32_t hist_lo, hist_hi;
  double* final_state;      /* [K * n * 2] final amplitudes (re, im), trajectory-major  */
} aqt_outputs;

/* Create a context on HIP device `device`; `hip_stream` is a hipStream_t or NULL
 * for the default stream.  *out receives the context (NULL on failure). */
AQT_API aqt_status aqt_create(aqt_ctx** out, int device, void* hip_stream);
AQT_API void aqt_destroy(aqt_ctx* ctx);
AQT_API const char* aqt_last_error(const aqt_ctx* ctx);
AQT_API int aqt_version(void);

/* Sec. V, eq. H_S: n_qubits in [1, 16]; h[n_qubits]; J[n_qubits * n_qubits] row-major,
 * only entries with i < j are read.  Host arrays. */
AQT_API aqt_status aqt_set_hamiltonian(aqt_ctx* ctx, int n_qubits, const double* h, const double* J);

/* Annealing schedule: t_f > 0 ns; A(s), B(s) piecewise linear through n_ctrl >= 2
 * control points at s_j = j/(n_ctrl-1), rad/ns.  Host arrays. */
AQT_API aqt_status aqt_set_schedule(aqt_ctx* ctx, double t_f, int n_ctrl, const double* A_ctrl,
                            const double* B_ctrl);

/* Ohmic bath (Sec. V): eta >= 0 (the paper's g^2), omega_c > 0, T > 0, rad/ns. */
AQT_API aqt_status aqt_set_bath(aqt_ctx* ctx, double eta, double omega_c, double T);

/* FP64 eigensystem and AME tables on the GPU for grid points g = 0..n_grid-1
 * (Sec. II eq. Lindblad2, Sec. III eqs. Aired, Heff): lowest n_levels eigenpairs
 * (n_levels <= 256; == 2^n_qubits for the full spectrum), clusters closer than
 * deg_tol rotated to a canonical basis, overlaps, sz matrix elements, rates,
 * decay and phases.  Synchronises the stream.  AQT_ENUMERIC if the ground state
 * of H(0) is degenerate or the eigensolver fails. */
AQT_API aqt_status aqt_precompute(aqt_ctx* ctx, int n_grid, int n_levels, double deg_tol);

/* Eigensolver choice of aqt_precompute_ex. */
enum { AQT_EIG_AUTO = 0, AQT_EIG_DENSE = 1, AQT_EIG_ITERATIVE = 2 };

/* aqt_precompute with an explicit eigensolver (Sec. II eq. Lindblad2 needs the
 * lowest eigenpairs of H(s) at every grid point):
 *   AQT_EIG_DENSE      dense FP64 solver per grid point, 2^n_qubits <= 1024;
 *   AQT_EIG_ITERATIVE  Chebyshev-filtered subspace iteration with a matrix-free
 *                      H(s) (any 2^n_qubits; truncated spectra with
 *                      n_levels + 16 <= 120 and n_levels < 2^n_qubits), warm-
 *                      started from the previous grid point, converged to
 *                      residual <= 1e-12 of a bound on |H|;
 *   AQT_EIG_AUTO       dense when 2^n_qubits <= 1024, else iterative.
 * Both apply the same canonical cluster basis, signs and truncation.
 * AQT_EINVAL for an unknown method or sizes outside these limits; AQT_ENUMERIC
 * if the iteration does not converge.  Synchronises the stream. */
AQT_API aqt_status aqt_precompute_ex(aqt_ctx* ctx, int n_grid, int n_levels, double deg_tol, int method);

/* Load externally computed tables instead of aqt_precompute (same meaning as the
 * tables aqt_precompute builds; host arrays, FP64, row-major):
 *   E[n_grid*n]; gs[n_grid] ground-cluster sizes; O[n_grid*n*n] with O[g] the
 *   polar overlap into grid g (g >= 2, others ignored); cinit[n] initial state in
 *   the grid-1 basis; R[n_grid*nc*n*n] as R[g][i][b][a] (rate of b -> a through
 *   jump channel i, a == b the omega = 0 weight gamma(0) z_bb^2); zdiag[n_grid*nc*n].
 *   nc = aqt_get_channel_count (n_qubits unless bath terms are set); AQT_EINVAL if
 *   nc > min(64, n_levels padded to 16, 32, 64, 128 or 256).
 * Decay rates and phases are derived from them on the GPU.  Synchronises. */
AQT_API aqt_status aqt_set_tables(aqt_ctx* ctx, int n_grid, int n_levels, const double* E,
                          const int32_t* gs, const double* O, const double* cinit,
                          const double* R, const double* zdiag);

/* Copy tables back to host arrays (any may be NULL): E[M*n], gs[M], O[M*n*n],
 * cinit[n], R[M*nc*n*n], zdiag[M*nc*n], Gamma[M*n], leak[M] (nc: the tables' jump
 * channels, aqt_get_channel_count).  Synchronises. */
AQT_API aqt_status aqt_get_tables(aqt_ctx* ctx, double* E, int32_t* gs, double* O, double* cinit,
                          double* R, double* zdiag, double* Gamma, double* leak);

/* Sizes of the loaded tables: n_grid, n_levels, n_qubits (any may be NULL). */
AQT_API aqt_status aqt_get_dims(aqt_ctx* ctx, int32_t* n_grid, int32_t* n_levels, int32_t* n_qubits);

/* Run K trajectories (Sec. IV waiting-time procedure, App. B jump-type law
 * eq. Pi(t)) through all grid points; stream-ordered.  Random draws: Philox4x64-10
 * with key (seed, instance_id) and counter (trajectory id, draw >> 2, 0, 0);
 * draw 0 is the first threshold, jump m uses 3m+1, 3m+2, 3m+3.
 * Never synchronises.  Records beyond record_capacity are dropped; jump_count
 * still holds the true number of jumps of each trajectory.  AQT_ENUMERIC (nothing
 * enqueued) if some level decays within one step by more than the state precision
 * carries: Gamma_b dt_g above 500 for AQT_FP64, above 50 for AQT_FP32 and AQT_BF16
 * (the same limit holds for aqt_run_fixed_step, aqt_grad_pgs and batches). */
AQT_API aqt_status aqt_run(aqt_ctx* ctx, const aqt_run_params* params, const aqt_outputs* out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): aqt_run without any allocation.  The
 * per-tile observable sums go to a fixed buffer of AQT_NOALLOC_SCRATCH_BYTES in device
 * memory, one per device, set up by aqt_create and held until the process ends.
 * Same arguments, outputs, kernels, results and stream ordering as aqt_run; the caller
 * still provides every output buffer.  Calls no hipMalloc, hipFree or allocating
 * library routine.  Errors (nothing enqueued):
 *   AQT_ESTATE  the step operands of params->precision are not resident (aqt_run packs
 *               them on its first call in a precision after the tables were loaded);
 *   AQT_EINVAL  the run's per-tile sums, tiles x n_grid x 16 bytes with
 *               tiles = ceil(n_traj / trajectories per workgroup), exceed the buffer
 *               (the 8-qubit workload: 250 tiles x 2000 points = 8 MB in FP32);
 *   otherwise as aqt_run.
 * Every call on one device shares that device's buffer and leaves its contents from the
 * last call (every entry a run reads it writes first): calls that overlap in time on one
 * device (for instance on two streams) race, and must be serialised by the caller. */
#define AQT_NOALLOC_SCRATCH_BYTES (64 * 1024 * 1024)
AQT_API aqt_status aqt_run_noalloc(aqt_ctx* ctx, const aqt_run_params* params, const aqt_outputs* out);

/* Run-status flags (bits of the word aqt_run_status reports). */
#define AQT_RUN_RECORDS_TRUNCATED 1   /* a trajectory made more jumps than record_capacity */
#define AQT_RUN_JUMP_LIMIT 2          /* a trajectory made AQT_MAX_JUMPS_PER_STEP jumps in one
                                         step; its results are invalid (rates far too large
                                         for the step length)                               */
#define AQT_MAX_JUMPS_PER_STEP 4096

/* Status of the runs enqueued on this context since the previous aqt_run_status call
 * (aqt_run, aqt_run_fixed_step, a batch launch that includes the context).  The runs
 * are stream-ordered and never synchronise, so their overflow conditions are collected
 * in a device word of the context; this call synchronises the context's stream, stores
 * the OR of the AQT_RUN_* flags in *flags (may be NULL) and clears the word.  Returns
 * AQT_ENUMERIC if AQT_RUN_JUMP_LIMIT is set, else AQT_ECAPACITY if records were
 * truncated (observables, jump_count and jump totals remain valid: jump_count holds the
 * true counts), else AQT_OK. */
AQT_API aqt_status aqt_run_status(aqt_ctx* ctx, int32_t* flags);

/* ---- Fixed-step unraveling ------------------------------------------------------------
 * The second unraveling (App. B, "to jump or not to jump"): every grid step is cut into
 * `substeps` sub-steps of length h = dt / substeps with the same frozen generator and
 * basis changes as aqt_run.  Per sub-step the normalised state jumps with probability
 * dp = h sum_b |c_b|^2 Gamma_b (eq. lambda): a uniform eps < dp applies the jump drawn as
 * in aqt_run (source weight |c_b|^2 Gamma_b, then channel and target by R; eq. Pi(t)),
 * otherwise the sub-step's no-jump propagator is applied; the state is renormalised
 * either way.  First order in h (aqt_run's waiting-time procedure is exact within each
 * step): a cross-check of the unraveling, its mean approaching the master equation as
 * h -> 0.  Draws: sub-step u = (step) substeps + s uses draws 3u (eps), 3u + 1 (source),
 * 3u + 2 (channel and target) of the same Philox streams; jump records carry the
 * sub-step's start time.  params as aqt_run (precision AQT_FP64 or AQT_FP32; tile and
 * segment ignored: 16 trajectories per workgroup).  Writes pgs_sum, pgs_sumsq,
 * jump_totals (+=), jump_count, jumps, net_gs, final_state (each may be NULL); net_hist
 * must be NULL.  Stream-ordered; never synchronises. */
AQT_API aqt_status aqt_run_fixed_step(aqt_ctx* ctx, const aqt_run_params* params, int substeps,
                                      const aqt_outputs* out);

/* ---- Time-step bound and bound-following grids -------------------------------------------
 * The bound of App. B (eq. B7) on the step of a trajectory integrator at time t:
 *   min{ |H_eff| / |dH_eff/dt|, 1 / |H_eff|, |lambda / (lambda^2 - dlambda/dt)| },
 * operator norms, H_eff = H - (i/2) sum_k A_k^dag A_k (Sec. III eq. Heff).  Readings: in the
 * eigenbasis H_eff = diag(e - i Gamma / 2); lambda, the jump rate of a trajectory, is taken
 * at its largest value max_b Gamma_b; time derivatives are finite differences over the
 * probes (central inside, one-sided at the ends); no Lamb shift.  Evaluated from a
 * full-spectrum FP64 precompute on n_probe equidistant points s_p = p / (n_probe - 1) in a
 * scratch context (the context's own tables are left as they are), so the instance must
 * have at most 256 basis states; clusters closer than 1e-8 rad/ns take the canonical basis
 * of aqt_precompute.  Needs set_hamiltonian, set_schedule and set_bath (and the bath and
 * coupling choices, which enter Gamma).  Synchronises.
 * aqt_step_bound: bound[n_probe] (host, ns) at the probes.
 * aqt_bound_grid: s[n_grid] (host), 0 = s_0 < ... < s_{n_grid-1} = 1, with local density
 * proportional to 1 / bound: s_g solves F(s_g) = g F(1) / (n_grid - 1), F the trapezoid
 * integral of 1 / bound over the probes, inverted by linear interpolation.  Pass it to
 * aqt_set_grid before aqt_precompute.  AQT_ENUMERIC if the bound is not positive and finite
 * or the grid does not increase (use more probes).
 * aqt_bound_grid_points: the step control the paper draws from the bound (the step kept
 * below it): *n_grid (host) = the fewest points, at least 2, whose bound-following grid keeps
 * every step t_f (s_g - s_{g-1}) within `fraction` (> 0) of the bound, to the accuracy of
 * the trapezoid integral: n_grid - 1 = ceil(t_f F(1) / fraction).  AQT_EINVAL if that
 * exceeds 10^7 points or fraction is not positive and finite. */
AQT_API aqt_status aqt_step_bound(aqt_ctx* ctx, int n_probe, double* bound);
AQT_API aqt_status aqt_bound_grid(aqt_ctx* ctx, int n_grid, int n_probe, double* s);
AQT_API aqt_status aqt_bound_grid_points(aqt_ctx* ctx, double fraction, int n_probe, int32_t* n_grid);

/* ---- Correlated baths -----------------------------------------------------------------
 * Baths with gamma_ab(w) = C_ab gamma(w) (Sec. II eq. ME2-L with a frequency-independent
 * correlation between the qubits' baths; the Lamb shift, when on, uses C_ab S(w) alike).
 * C: host [n_qubits * n_qubits], row-major, symmetric positive definite (C = I: the
 * independent baths of the default; NULL restores them).  With C = L L^T (Cholesky) the
 * double sum over qubits is a sum over n_qubits jump channels with coupling operators
 * sum_a L[a][k] sz_a, each with rate gamma(w); every table, jump record ("qubit" is then
 * the channel k) and the gradient refer to these channels.  Applies from the next
 * aqt_precompute (loaded tables are invalidated); cleared by aqt_set_hamiltonian with a
 * different qubit count.  AQT_ESTATE before aqt_set_hamiltonian; AQT_EINVAL if C is not
 * finite, symmetric (1e-12 relative) or positive definite. */
AQT_API aqt_status aqt_set_bath_correlation(aqt_ctx* ctx, const double* C);

/* Frequency-dependent bath correlations (Sec. II eq. ME2-L with a general gamma_ab(w),
 * which the paper brings to diagonal form by a frequency-dependent rotation u(w)):
 *   gamma_ab(w) = sum_m C_m[a][b] gamma(w; omega_c[m]),
 * a sum of n_terms Ohmic spectral densities (the bath's eta and T, each term its own
 * cutoff omega_c[m] > 0, rad/ns), each with a symmetric positive semidefinite
 * correlation C_m (host, [n_terms][n_qubits][n_qubits] row-major).  Every C_m is
 * factored as F_m F_m^T by the Cholesky recursion in natural order, dropping a
 * column whose pivot is at most 1e-12 max(diag C_m); each kept column k gives a jump
 * channel with coupling operator sum_a F_m[a][k] sz_a and rate gamma(w; omega_c[m]),
 * channels numbered term by term.  Since sum over channels of F F^T gamma_m equals
 * gamma_ab(w) at every w, these channels give the master equation's dissipator at
 * every Bohr frequency (in place of u(w)); tables, jump records ("qubit" is the
 * channel) and aqt_get_channel_count refer to them.  n_terms = 0 restores independent
 * baths; replaces any aqt_set_bath_correlation.  Applies from the next aqt_precompute
 * (loaded tables are invalidated).  The Lamb shift and the gradient cover bath terms:
 * each channel's S(w) and rate derivative use its cutoff (one S table per cutoff).  AQT_ESTATE before
 * aqt_set_hamiltonian; AQT_EINVAL for non-finite or non-symmetric (1e-12 relative)
 * C_m, a pivot below -1e-9 max(diag C_m) (not semidefinite), a cutoff <= 0, no
 * channel at all or more than 64; aqt_precompute returns AQT_EINVAL when the channels
 * outnumber the padded level count. */
AQT_API aqt_status aqt_set_bath_terms(aqt_ctx* ctx, int n_terms, const double* C, const double* omega_c);

/* Grid points of the anneal (Sec. IV; App. B eq. B7 bounds the step and suggests
 * adapting it to the bound's instantaneous value): s[n_grid] host, s[0] = 0 <
 * s[1] < ... < s[n_grid-1] = 1.  Grid point g sits at t = t_f s_g.  Its step (the
 * basis change into g, then the no-jump propagator and jumps with g's tables) has
 * length (h_g + h_{g+1}) / 2, h_g = t_f (s_g - s_{g-1}), half of each neighbouring
 * interval, so that every interval is split symmetrically around its basis change (the
 * last point takes (h_{n_grid-1} + h_1) / 2, so the lengths add up to t_f), and starts
 * at t_f (s_{g-1} + s_g - s_1) / 2 (jump record times, the no-jump propagator and the
 * gradient's hat-function weights of the controls use them).  On equidistant points
 * this is the step t_f / (n_grid - 1) starting at (g - 1) t_f / (n_grid - 1), which is
 * what n_grid = 0 or s = NULL restores (s_g = g / (n_grid - 1)).  Applies from
 * the next aqt_precompute or aqt_set_tables, whose n_grid must then equal this one
 * (AQT_EINVAL otherwise); loaded tables are invalidated.  AQT_EINVAL for fewer than
 * two points, ends other than 0 and 1, or points that do not increase. */
AQT_API aqt_status aqt_set_grid(aqt_ctx* ctx, int n_grid, const double* s);

/* General coupling operators (Sec. II: the system operators A_a of the system-bath
 * coupling, here any real combination of single-qubit sz and sx): channel k couples
 * through O_k = sum_a (cz[k][a] sz_a + cx[k][a] sx_a) to its own bath (independent of
 * the other channels) with the Ohmic rate gamma(w; omega_c[k]) (omega_c NULL: the
 * bath's cutoff for every channel).  cz, cx: host [n_channels][n_qubits] row-major,
 * either may be NULL (zero); omega_c: host [n_channels] or NULL.  Matrix elements
 * <a|O_k|b> in the real eigenbasis are real, so tables and kernels are those of the
 * sz channels; jump records' "qubit" is the channel k.  n_channels = 0 restores the
 * default (sz of each qubit).  Replaces aqt_set_bath_correlation / aqt_set_bath_terms
 * settings and vice versa; applies from the next aqt_precompute.  The Lamb shift uses
 * each channel's cutoff in S(w); aqt_grad_pgs covers these channels (dz_k = z_k X - X z_k holds for any
 * fixed coupling operator).
 * AQT_ESTATE before aqt_set_hamiltonian; AQT_EINVAL for n_channels outside [0, 64],
 * non-finite coefficients, a channel whose operator is zero, cz and cx both NULL or a
 * cutoff <= 0. */
AQT_API aqt_status aqt_set_coupling(aqt_ctx* ctx, int n_channels, const double* cz, const double* cx,
                                    const double* omega_c);

/* Jump channels of the loaded tables (before any, of the current bath settings):
 * n_qubits for independent or constant-correlation baths; the kept factor columns of
 * bath terms; n_channels of aqt_set_coupling. */
AQT_API aqt_status aqt_get_channel_count(aqt_ctx* ctx, int32_t* n_channels);

/* ---- Lamb shift ----------------------------------------------------------------------
 * enabled != 0 adds the Lamb-shift Hamiltonian of the Ohmic bath, H_LS = sum_i sum_w S(w)
 * A_i,w^dag A_i,w (Sec. II eq. ME2-H; the operators of the Bohr-frequency grouping), with
 * S(w) = (1/2pi) P int gamma(w') / (w - w') dw', to the tables built by the next
 * aqt_precompute.  H_LS is diagonal in the eigenbasis, so only the energies that set the
 * no-jump phases move: level b gets sum_i [sum_{a != b} S(e_b - e_a) z_ab^2 + S(0) z_bb^2];
 * Bohr frequencies, rates and jump kinds keep the energies of H_S.  Off by default; tables
 * given with aqt_set_tables are used as given.  Invalidates loaded tables (precompute
 * again).  aqt_grad_pgs includes it: the shift's derivative (dS/dw of the interpolated
 * S(w) table, and 2 S z dz) enters the phase terms, and S scales with eta. */
AQT_API aqt_status aqt_set_lamb_shift(aqt_ctx* ctx, int enabled);

/* The Lamb shift of every level at every grid point (host [n_grid * n_levels], row-major;
 * zeros when off).  Synchronises. */
AQT_API aqt_status aqt_get_lamb_shift(aqt_ctx* ctx, double* shift);

/* ---- Gradient ------------------------------------------------------------------------
 * Estimate of d E[P_GS(1)] / d theta, theta = (A_ctrl[0..m-1], B_ctrl[0..m-1], eta):
 * the derivative of the trajectory average of the final ground-cluster population
 * with respect to the schedule control points of aqt_set_schedule (m of each) and
 * the coupling eta of aqt_set_bath.  Paths of the waiting-time procedure (Sec. IV)
 * have density |psi~|^2 over a parameter-free measure on jump times and channels
 * (Sec. III eqs. Heff and jump, App. B), so each trajectory contributes
 * g = 2 Re <psi~|Pi|d psi~> / |psi~|^2: a pathwise term through the no-jump
 * propagation and basis changes plus a score-function term for the jump times and
 * channels, evaluated by an adjoint sweep with checkpointed recomputation of the
 * forward steps.  Eigenvector derivatives use first-order perturbation theory with
 * the canonical in-cluster basis held fixed.
 *   params:   as aqt_run (precision AQT_FP64 or AQT_FP32, n_traj >= 2; record_capacity
 *             is ignored: the paths are recorded internally; segment > 0 forces
 *             checkpoint segments of that many steps, else the sweep keeps every
 *             post-kick state when the workspace allows, with segments of about
 *             sqrt(n_grid) steps otherwise; segment < 0 is AQT_EINVAL).  The trajectories are
 *             the ones aqt_run draws with the same params.
 *   value, value_se: host, mean and standard error of P_GS(1) (may be NULL).
 *   grad, grad_se:   host [2m+1], mean estimate and its standard error (may be NULL).
 *   per_traj: device [n_traj][2(2m+2)] or NULL: per trajectory f (final ground-cluster
 *             population) and its 2m+1 estimates g, then 1 and the 2m+1 components of
 *             s = d log |psi~|^2 (the path-density score, mean zero).
 * The reported gradient is mean(g) - c mean(s) with c = Cov(g, s) / Var(s) per component
 * (a control variate from the same trajectories: it removes the part of the score-function
 * noise that does not depend on f; its bias is O(1/n_traj)); grad_se is its standard error.
 * Needs tables from aqt_precompute with n_levels = 2^n_qubits (AQT_ESTATE after
 * aqt_set_tables, AQT_EINVAL for truncated spectra); the first call after a
 * precompute re-runs the eigensolver to add the derivative tables.  Covers every bath
 * model (aqt_set_bath_correlation, aqt_set_bath_terms, aqt_set_coupling), the Lamb shift
 * and grids of aqt_set_grid (hat weights at the grid points).  AQT_ECAPACITY if
 * one trajectory takes more than 32 omega = 0 jumps within one step.  Synchronises. */
AQT_API aqt_status aqt_grad_pgs(aqt_ctx* ctx, const aqt_run_params* params, double* value, double* value_se,
                                double* grad, double* grad_se, double* per_traj);

/* ---- Batched runs: many instances in one persistent launch --------------------------
 * Each context (with tables loaded) is one instance with its own run parameters and
 * output buffers.  One kernel launch runs every (instance, tile) work item from an
 * atomic queue, longest items first, then one fixed-order reduction writes every
 * instance's observable sums.  All contexts must be on one device and use one
 * precision.  flags: AQT_BATCH_GRAPH captures the launch sequence once into a HIP
 * graph (replayed by aqt_batch_launch); AQT_BATCH_AUTOTUNE times the supported tile
 * sizes per level count on a shortened anneal and keeps the fastest (instances
 * with a non-zero params[i].tile keep theirs).  Output pointers are bound at
 * creation.  On failure *out may still receive a batch whose aqt_batch_last_error
 * explains the failure; it must be destroyed.  Launches on the first context's
 * stream; jump_totals and net_hist accumulate across launches. */
typedef struct aqt_batch aqt_batch;
enum { AQT_BATCH_GRAPH = 1, AQT_BATCH_AUTOTUNE = 2 };
AQT_API aqt_status aqt_batch_create(aqt_batch** out, aqt_ctx* const* ctxs, int n, const aqt_run_params* params,
                                    const aqt_outputs* outs, int flags);
AQT_API aqt_status aqt_batch_launch(aqt_batch* batch);
/* Trajectories per workgroup tile chosen for each instance (host array [n]). */
AQT_API aqt_status aqt_batch_tiles(const aqt_batch* batch, int32_t* tile_per_instance);
AQT_API const char* aqt_batch_last_error(const aqt_batch* batch);
AQT_API void aqt_batch_destroy(aqt_batch* batch);

#ifdef __cplusplus
}
#endif

#endif /* AQT_H */
