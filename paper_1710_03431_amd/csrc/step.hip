// Persistent trajectory kernel: batched quantum-jump stepping in the
// instantaneous eigenbasis (Sec. IV waiting-time procedure; App. C validity;
// jump-type law App. B eq. Pi(t); jump update Sec. III eq. jump).
//
// One workgroup (WV = 4 or 8 wavefronts) owns a tile of TT = 8*TQ trajectories for the whole
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
#include <type_traits>
#include <algorithm>
#include <limits>
#include <mutex>
#include <new>
#include <string>
#include <vector>

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
// 16-level instances: BF16 16x16x16 MFMA (four BF16 per lane and operand).
struct ModeBF16K16 {
  using T = float;
  using Acc = f4;
  static constexpr int KC = 16;
  __device__ static constexpr int row(int lane, int i) { return 4 * (lane >> 4) + i; }
};
typedef short s16x4 __attribute__((ext_vector_type(4)));

struct StepArgs {
  int M, n, nq;
  int M_run;             // grid points processed (M, or fewer when autotuning)
  int NP, TQ;            // padded levels and column tiles of this instance (batched runs)
  int64_t tiles;         // workgroup tiles of this instance
  double* pgs_sum;       // [M] (batched runs reduce into these)
  double* pgs_sumsq;
  const double* tbeg;    // [M] start time of the step into grid g
  const double* tlen;    // [M] its length
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
  const double* Rcol;    // [M][nq][NP][4] row sum, sum below the diagonal, diagonal of R
  const double* ehalf;   // [M][NP] exp(+Gamma dt / 2)
  const double* zdiag;   // [M][nq][NP]
  const float4* chf;     // FP32 runs: [M][nq][NP] (row sum, sum below the diagonal, diagonal, z_bb), else null
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
  int* flags;            // AQT_RUN_* flags of the context (OR-ed)
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

// hi/lo BF16 split of 4 floats, packed as two 64-bit words.
__device__ __forceinline__ void split4(const float* x, s16x4& hi, s16x4& lo) {
  uint32_t h[2], l[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    uint32_t h0 = bf16_bits(x[2 * j]), h1 = bf16_bits(x[2 * j + 1]);
    float r0 = x[2 * j] - __uint_as_float(h0 << 16);
    float r1 = x[2 * j + 1] - __uint_as_float(h1 << 16);
    h[j] = h0 | (h1 << 16);
    l[j] = bf16_bits(r0) | (bf16_bits(r1) << 16);
  }
  hi = __builtin_bit_cast(s16x4, make_uint2(h[0], h[1]));
  lo = __builtin_bit_cast(s16x4, make_uint2(l[0], l[1]));
}

// One A-operand fragment of Delta (per lane): a value for the K = 4 MFMAs,
// hi/lo BF16 words for the K = 16 and K = 32 ones.
template <class Mode>
struct Frag {
  typename Mode::T v;
};
template <>
struct Frag<ModeBF16K16> {
  uint2 h, l;
};
template <>
struct Frag<ModeBF16> {
  uint4 h, l;
};

template <class Mode>
__device__ __forceinline__ Frag<Mode> load_frag(const StepArgs& a, size_t idx) {
  Frag<Mode> f;
  if constexpr (Mode::KC == 4) {
    f.v = static_cast<const typename Mode::T*>(a.dlt_a)[idx];
  } else if constexpr (Mode::KC == 16) {
    f.h = static_cast<const uint2*>(a.dlt_a)[idx];
    f.l = static_cast<const uint2*>(a.dlt_b)[idx];
  } else {
    f.h = static_cast<const uint4*>(a.dlt_a)[idx];
    f.l = static_cast<const uint4*>(a.dlt_b)[idx];
  }
  return f;
}

// Chunks of A fragments kept in flight: a ring of PF chunks per unit, refilled
// PF chunks ahead and, at the end of a step, with the first chunks of the next
// step, so the loads overlap the epilogue and the jump handler.
template <class Mode, int NP>
constexpr int prefetch_depth() {
  constexpr int NKC = NP / Mode::KC;
  constexpr int want = (Mode::KC == 4) ? 8 : 2;
  return NKC < want ? NKC : want;
}

// ----------------------------------------------------------- jump handler --
// Tile layout in LDS: S[q][c][row] holds column tile q (8 trajectories) column-
// major; column c = (t & 7) + 8 * part carries the real (part 0) or imaginary
// (part 1) part of local trajectory t = 8 q + (c & 7).  Columns are padded to
// NP + kPad elements so the 16 columns of an MFMA operand fall in distinct banks.
constexpr int kPad = 4;   // >= 4: the B read-ahead touches padding rows NP..NP+3
constexpr int kStepTables = 5;
// Wavefronts per workgroup.  Eight (two per SIMD) let one wave's LDS and load waits
// hide behind the other's MFMAs where each wave still has a large share of the
// GEMM (>= 128 levels, FP32/FP64 and the batched kernel); small tiles and the
// register-heavy BF16 path at 256 levels keep four.
template <int NP, class Mode>
constexpr int waves_for() {
  return (NP >= 128 && Mode::KC == 4) ? 8 : 4;
}
template <int NP, class T>
using TileCols = T[16][NP + kPad];

template <int NP, class T>
__device__ __forceinline__ T& amp(TileCols<NP, T>* S, int t, int part, int row) {
  return S[t >> 3][(t & 7) + 8 * part][row];
}

// Exchange with lane ^ 8 (the other part of the same amplitude) by DPP row
// rotation: within each row of 16 lanes, rotating by 8 maps lane i to i ^ 8.
__device__ __forceinline__ float xor8(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x128, 0xf, 0xf, false));
}
__device__ __forceinline__ double xor8(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(u & 0xffffffffu), 0x128, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(u >> 32), 0x128, 0xf, 0xf, false);
  return __builtin_bit_cast(double, (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) | static_cast<uint32_t>(lo));
}

// A crossing is handled by a segment of SEG consecutive lanes (seg_width): a
// wavefront serves 64 / SEG crossings at once.  Reductions, scans, ballots and broadcasts stay inside the segment, and
// are built from DPP row operations (rows of 16 lanes) and row-pair swaps rather
// than LDS-routed shuffles; every lane of a segment receives a bit-identical sum.
template <int CTRL, int ROWS = 0xf, bool BOUND = false>
__device__ __forceinline__ float dpp(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROWS, 0xf, BOUND));
}
template <int CTRL, int ROWS = 0xf, bool BOUND = false>
__device__ __forceinline__ double dpp(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(u & 0xffffffffu), CTRL, ROWS, 0xf, BOUND);
  const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(u >> 32), CTRL, ROWS, 0xf, BOUND);
  return __builtin_bit_cast(double, (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) | static_cast<uint32_t>(lo));
}
// v + (the same register of the partner row): rows 0+1 and 2+3 (W = 16), or the two
// halves of the wavefront (W = 32); both operands of the swap are v, so the two
// results hold the pair's values in every lane and their sum needs no select.
template <int W>
__device__ __forceinline__ float swap_add(float v) {
  const int x = __builtin_bit_cast(int, v);
  const auto s = (W == 16) ? __builtin_amdgcn_permlane16_swap(x, x, false, false)
                           : __builtin_amdgcn_permlane32_swap(x, x, false, false);
  return __builtin_bit_cast(float, static_cast<int>(s[0])) + __builtin_bit_cast(float, static_cast<int>(s[1]));
}
template <int W>
__device__ __forceinline__ double swap_add(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const int lo = static_cast<int>(u & 0xffffffffu), hi = static_cast<int>(u >> 32);
  const auto sl = (W == 16) ? __builtin_amdgcn_permlane16_swap(lo, lo, false, false)
                            : __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto sh = (W == 16) ? __builtin_amdgcn_permlane16_swap(hi, hi, false, false)
                            : __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  const double a = __builtin_bit_cast(double, (static_cast<uint64_t>(static_cast<uint32_t>(sh[0])) << 32) |
                                                  static_cast<uint32_t>(sl[0]));
  const double b = __builtin_bit_cast(double, (static_cast<uint64_t>(static_cast<uint32_t>(sh[1])) << 32) |
                                                  static_cast<uint32_t>(sl[1]));
  return a + b;
}
template <int SEG, class V>
__device__ __forceinline__ V seg_sum(V v) {
  static_assert(SEG == 16 || SEG == 32 || SEG == 64, "segments are whole rows");
  v += dpp<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dpp<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp<0x141>(v);   // row_half_mirror
  v += dpp<0x140>(v);   // row_mirror: the row total in every lane of the row
  if constexpr (SEG >= 32) v = swap_add<16>(v);
  if constexpr (SEG == 64) v = swap_add<32>(v);
  return v;
}
// Inclusive scan over the segment's lanes in lane order.
template <int SEG, class V>
__device__ __forceinline__ V seg_scan(V v) {
  static_assert(SEG == 16 || SEG == 32 || SEG == 64, "segments are whole rows");
  v += dpp<0x111, 0xf, true>(v);   // row_shr:1 (zero shifted in)
  v += dpp<0x112, 0xf, true>(v);   // row_shr:2
  v += dpp<0x114, 0xf, true>(v);   // row_shr:4
  v += dpp<0x118, 0xf, true>(v);   // row_shr:8: inclusive scan of each row
  if constexpr (SEG >= 32) v += dpp<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
  if constexpr (SEG == 64) v += dpp<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
  return v;
}
// Lanes per crossing: one 16-lane row for up to 32 levels (four crossings per
// wavefront), half a wavefront for 64 levels, the whole wavefront above.
template <int NP>
__host__ __device__ constexpr int seg_width() {
  return NP <= 32 ? 16 : (NP == 64 ? 32 : kWave);
}
template <int SEG>
__device__ __forceinline__ uint64_t seg_ballot(bool pred, int base) {
  const uint64_t m = __ballot(pred);
  return (SEG == 64) ? m : (m >> base) & ((1ull << (SEG & 63)) - 1ull);
}
// Value of segment lane `idx` (segment-uniform) in every lane of the segment.
template <int SEG>
__device__ __forceinline__ float seg_read(float v, int idx, int base) {
  if constexpr (SEG == 64) return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), idx));
  else return __shfl(v, base + idx, kWave);
}
template <int SEG>
__device__ __forceinline__ double seg_read(double v, int idx, int base) {
  if constexpr (SEG == 64) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(u & 0xffffffffu), idx));
    const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(u >> 32), idx));
    return __builtin_bit_cast(double, (static_cast<uint64_t>(hi) << 32) | lo);
  } else {
    return __shfl(v, base + idx, kWave);
  }
}
template <int SEG>
__device__ __forceinline__ uint32_t seg_read(uint32_t v, int idx, int base) {
  if constexpr (SEG == 64) return static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), idx));
  else return __shfl(v, base + idx, kWave);
}

// First index x = lane + SEG j (chunk-major order) whose running sum of w exceeds thr,
// with `start` added in front; -1 if none.  Chunk totals first (independent sums),
// then one scan of the chunk the threshold falls in (the next chunk if rounding of
// the scan keeps it below).  Also returns the last index with w > 0 in *lastpos.
template <int SEG, int PL, class H>
__device__ __forceinline__ int seg_pick(const H (&w)[PL], H thr, H start, int base, int* lastpos) {
  H tot[PL];
#pragma unroll
  for (int j = 0; j < PL; ++j) tot[j] = seg_sum<SEG>(w[j]);
  H prefix = start;
  int hit = -1, last = -1;
#pragma unroll
  for (int j = 0; j < PL; ++j) {
    if (hit < 0 && prefix + tot[j] > thr) {
      const H cum = seg_scan<SEG>(w[j]) + prefix;
      // cum is non-decreasing, so the first index exceeding thr carries weight; the
      // weight test only keeps a scan rounded below the chunk total from picking the
      // next chunk's (possibly empty) first level
      const uint64_t h = seg_ballot<SEG>(cum > thr && w[j] > H(0), base);
      if (h) hit = first_set_lane(h) + SEG * j;
    }
    prefix += tot[j];
    const uint64_t pz = seg_ballot<SEG>(w[j] > H(0), base);
    if (pz) last = last_set_lane(pz) + SEG * j;
  }
  *lastpos = last;
  return hit;
}

// Uniform draws of one trajectory served from Philox blocks computed in parallel:
// lane l of the segment holds block B0 + l (four words), so one generator
// evaluation covers the next 4 SEG draws; later draws fall back to a direct
// evaluation.
template <int SEG>
struct DrawCache {
  uint64_t B0;
  uint64_t w0, w1, w2, w3;
  uint64_t seed, iid, traj;
  int base;
  __device__ void fill(uint64_t seed_, uint64_t iid_, uint64_t traj_, uint64_t first_draw, int base_, int sl) {
    seed = seed_;
    iid = iid_;
    traj = traj_;
    base = base_;
    B0 = first_draw >> 2;
    const Philox4 r = philox4x64_10(traj, B0 + sl, 0, 0, seed, iid);
    w0 = r.w[0];
    w1 = r.w[1];
    w2 = r.w[2];
    w3 = r.w[3];
  }
  __device__ double operator()(uint64_t d) const {
    const uint64_t rel = (d >> 2) - B0;
    if (rel >= static_cast<uint64_t>(SEG)) return draw_uniform(seed, iid, traj, d);
    const unsigned k = static_cast<unsigned>(d & 3);
    const uint64_t mine = k == 0 ? w0 : (k == 1 ? w1 : (k == 2 ? w2 : w3));
    const uint32_t lo = seg_read<SEG>(static_cast<uint32_t>(mine & 0xffffffffu), static_cast<int>(rel), base);
    const uint32_t hi = seg_read<SEG>(static_cast<uint32_t>(mine >> 32), static_cast<int>(rel), base);
    return uniform_open01((static_cast<uint64_t>(hi) << 32) | lo);
  }
};

// Per-trajectory cache of Philox blocks in LDS: blocks rngb[t] and rngb[t] + 1 of
// trajectory t's stream, refreshed after each crossing to B = (3 m + 1) / 4 so that the
// draws of the next jump (3m+1, 3m+2 and the threshold 3m+3) are waiting there.  The
// refresh of the trajectories listed after a step runs on one wavefront at the start of
// the next step, off the crossing handler's path.
struct RngCache {
  uint64_t (*w)[8];
  uint64_t* b;
  int* list;
  int* n;
};

// Blocks B and B + 1, B = (3 m + 1) / 4, for n trajectories (list, or 0..n-1 when list
// is null; m = 0 when m_of is null): one wavefront, two lanes per trajectory.
__device__ void rng_refill(const StepArgs& a, int64_t tb, int n, const int* list, const int* m_of, RngCache rc,
                           int lane) {
  for (int i0 = 0; i0 < 2 * n; i0 += kWave) {
    const int i = i0 + lane;
    if (i < 2 * n) {
      const int t = list ? list[i >> 1] : (i >> 1);
      const int half = i & 1;
      const uint64_t mm = m_of ? static_cast<uint64_t>(m_of[t]) : 0ull;
      const uint64_t B = (3ull * mm + 1ull) >> 2;
      const Philox4 r = philox4x64_10(a.traj0 + static_cast<uint64_t>(tb + t), B + half, 0, 0, a.seed, a.iid);
#pragma unroll
      for (int k = 0; k < 4; ++k) rc.w[t][4 * half + k] = r.w[k];
      if (half == 0) rc.b[t] = B;
    }
  }
}

// Convergence of the crossing-time iteration: a step below tol * dt ends it.
template <class H>
__device__ constexpr H newton_tol() {
  return sizeof(H) == 8 ? H(1e-15) : H(4.0f * 1.1920929e-7f);
}

// One wavefront finishes step g for local trajectory t whose amplitudes after
// the fused propagator are in S (the threshold pass found the FP64 sum of |S|^2
// at or below r).  The handler computes in the state precision H = T: FP64 runs
// keep every step in FP64 (jump times and channels as the FP64 oracle's), mixed-
// precision runs take the crossing time, the channel scans and the renormalisation
// in FP32 (native exponentials, 32-bit shuffles).  The crossing test itself and
// the observable sums stay in FP64 in every mode.
template <int NP, class T, bool STAGED>
__device__ void finish_crossing(const StepArgs& a, int g, int t, int64_t jloc, TileCols<NP, T>* S,
                                const double* s_r, double* s_rn, int* s_m, int* s_cnt, int* s_net, double* s_p,
                                int* s_kind, RngCache rc, const double* tg, const float4* chs) {
  using H = T;
  constexpr int SEG = seg_width<NP>();
  constexpr int PL = NP / SEG;
  const int lane = threadIdx.x & (SEG - 1);                    // lane within the segment
  const int base = (threadIdx.x & (kWave - 1)) & ~(SEG - 1);   // first lane of the segment
  const double dt = a.tlen[g];
  const uint64_t traj = a.traj0 + static_cast<uint64_t>(jloc);   // Philox counter word 0
  // grid point g's Gamma, e^{G dt/2}, E and phase factors: staged in LDS (kStepTables rows
  // of NP) or read from the tables
  const size_t gofs = static_cast<size_t>(g) * NP;
  const double* Gam = STAGED ? tg : a.Gamma + gofs;
  const double* Eh = STAGED ? tg + NP : a.ehalf + gofs;
  const double* Eg = STAGED ? tg + 2 * NP : a.E + gofs;
  const double* Pre = STAGED ? tg + 3 * NP : a.d64re + gofs;
  const double* Pim = STAGED ? tg + 4 * NP : a.d64im + gofs;
  H sr[PL], si[PL], G[PL], up[PL];
#pragma unroll
  for (int j = 0; j < PL; ++j) {
    const int x = lane + SEG * j;
    const bool in = x < NP;
    G[j] = in ? static_cast<H>(Gam[x]) : H(0);
    up[j] = in ? static_cast<H>(Eh[x]) : H(0);
    sr[j] = in ? static_cast<H>(amp<NP, T>(S, t, 0, x)) : H(0);
    si[j] = in ? static_cast<H>(amp<NP, T>(S, t, 1, x)) : H(0);
  }
  double r = s_r[t];
  int m = s_m[t];
  int cnt = s_cnt[t];
  int net = s_net[t];
  const int gsz = a.gs[g];
  const double tk = a.tbeg[g];
  // the crossing test of the whole step, in FP64 as in the threshold pass:
  // sum_b |c_b|^2 e^{-G_b dt} = sum |S|^2
  double nu0 = 0.0;
#pragma unroll
  for (int j = 0; j < PL; ++j) {
    const double xr = sr[j], xi = si[j];
    nu0 = fma(xr, xr, fma(xi, xi, nu0));
  }
  nu0 = seg_sum<SEG>(nu0);
  if (nu0 > r) {
    // no crossing after all (the threshold pass summed in another order): S stays
    double pg = 0.0;
#pragma unroll
    for (int j = 0; j < PL; ++j)
      if (lane + SEG * j < gsz) pg += static_cast<double>(sr[j]) * sr[j] + static_cast<double>(si[j]) * si[j];
    pg = seg_sum<SEG>(pg);
    if (lane == 0) {
      s_p[t] = pg / nu0;
      s_rn[t] = r;
    }
    return;
  }
  // draws: the two cached blocks, else Philox blocks evaluated across the segment's lanes
  const uint64_t Bc = rc.b[t];
  DrawCache<SEG> far;
  bool far_ready = false;
  auto draw = [&](uint64_t d) -> double {
    const uint64_t rel = (d >> 2) - Bc;
    if (rel < 2) return uniform_open01(rc.w[t][4 * rel + (d & 3)]);
    if (!far_ready) {
      far.fill(a.seed, a.iid, traj, d, base, lane);
      far_ready = true;
    }
    return far(d);
  };
  // amplitudes at the start of the step's decay: undo the fused e^{-G dt / 2}
  H cr[PL], ci[PL];
#pragma unroll
  for (int j = 0; j < PL; ++j) {
    cr[j] = sr[j] * up[j];
    ci[j] = si[j] * up[j];
  }
  const double* Rc = a.Rcol + static_cast<size_t>(g) * a.nq * NP * 4;
  double tau_e = 0.0;
  int guard = 0;
  for (; guard < AQT_MAX_JUMPS_PER_STEP; ++guard) {   // jumps within one step
    const H rem = static_cast<H>(dt - tau_e);
    if (guard > 0) {
      // after a jump: does the norm reach the next threshold within the rest of the step?
      H h[PL], part = H(0);
#pragma unroll
      for (int j = 0; j < PL; ++j) {
        h[j] = exp(H(-0.5) * G[j] * rem);
        part += (cr[j] * cr[j] + ci[j] * ci[j]) * (h[j] * h[j]);
      }
      const H nu_end = seg_sum<SEG>(part);
      if (static_cast<double>(nu_end) > r) {
#pragma unroll
        for (int j = 0; j < PL; ++j) {
          cr[j] *= h[j];
          ci[j] *= h[j];
        }
        break;
      }
    }
    // crossing time: Newton on log sum_b w_b e^{-G_b tau} = log r from tau = 0
    H w[PL], hf[PL];
#pragma unroll
    for (int j = 0; j < PL; ++j) {
      w[j] = cr[j] * cr[j] + ci[j] * ci[j];
      hf[j] = H(1);
    }
    H tau = H(0);
    const H logr = static_cast<H>(log(r));
    for (int it = 0; it < 100; ++it) {
      H s0 = H(0), s1 = H(0);
#pragma unroll
      for (int j = 0; j < PL; ++j) {
        const H e = w[j] * (hf[j] * hf[j]);
        s0 += e;
        s1 += G[j] * e;
      }
      s0 = seg_sum<SEG>(s0);
      s1 = seg_sum<SEG>(s1);
      const H f = log(s0) - logr;
      // converged once the log-ratio is at rounding level: further steps only follow
      // the noise of the sums (for a slowly decaying level that noise exceeds tol dt)
      if (fabs(f) <= H(8) * std::numeric_limits<H>::epsilon()) break;
      const H fp = -s1 / s0;
      if (fp == H(0)) {
        tau = rem;
#pragma unroll
        for (int j = 0; j < PL; ++j) hf[j] = exp(H(-0.5) * G[j] * tau);
        break;
      }
      const H stp = -f / fp;
      if (!(stp > H(0))) break;
      const H tn = fmin(tau + stp, rem);
      const bool done = (tn - tau <= newton_tol<H>() * static_cast<H>(dt)) || (tn >= rem);
      tau = tn;
#pragma unroll
      for (int j = 0; j < PL; ++j) hf[j] = exp(H(-0.5) * G[j] * tau);
      if (done) break;
    }
#pragma unroll
    for (int j = 0; j < PL; ++j) {
      cr[j] *= hf[j];
      ci[j] *= hf[j];
    }
    tau_e += static_cast<double>(tau);
    const H u1 = static_cast<H>(draw(3ull * m + 1));
    const H u2 = static_cast<H>(draw(3ull * m + 2));
    // source level b: first index whose running sum of q_b Gamma_b exceeds u1 * total
    int b = -1;
    {
      H wq[PL];
#pragma unroll
      for (int j = 0; j < PL; ++j) wq[j] = (cr[j] * cr[j] + ci[j] * ci[j]) * G[j];
      H tot = H(0);
#pragma unroll
      for (int j = 0; j < PL; ++j) tot += wq[j];
      tot = seg_sum<SEG>(tot);
      int lastpos = -1;
      b = seg_pick<SEG, PL, H>(wq, u1 * tot, H(0), base, &lastpos);
      if (b < 0) b = lastpos;
    }
    if (b < 0) {
      // no populated level decays (a rounding-level crossing): nothing can jump
#pragma unroll
      for (int j = 0; j < PL; ++j) {
        const H f = exp(H(-0.5) * G[j] * static_cast<H>(dt - tau_e));
        cr[j] *= f;
        ci[j] *= f;
      }
      break;
    }
    // qubit i and target a: inverse CDF over R[g][i][b][a] in i-major, a-minor order,
    // taken in stages -- the qubit from the row sums, then the diagonal (omega = 0)
    // element from the sum below it, and only for a != b a scan of the row --
    // which selects the same (i, a) as one pass over the whole list.
    int qi = 0, ta = b;
    {
      H thr, before, lo_q, dg_q;
      if (a.nq <= SEG) {
        // one channel per lane
        H rs = H(0), rlo = H(0), rdg = H(0);
        if (lane < a.nq) {
          if (chs) {   // staged in LDS
            const float4 c4 = chs[lane * NP + b];
            rs = static_cast<H>(c4.x);
            rlo = static_cast<H>(c4.y);
            rdg = static_cast<H>(c4.z);
          } else {
            const double* c4 = Rc + (static_cast<size_t>(lane) * NP + b) * 4;
            rs = static_cast<H>(c4[0]);
            rlo = static_cast<H>(c4[1]);
            rdg = static_cast<H>(c4[2]);
          }
        }
        const H cum_i = seg_scan<SEG>(rs);
        const H tot = seg_read<SEG>(cum_i, SEG - 1, base);
        thr = u2 * tot;
        const uint64_t hit_i = seg_ballot<SEG>(cum_i > thr && lane < a.nq, base);
        const uint64_t pos_i = seg_ballot<SEG>(rs > H(0), base);
        qi = hit_i ? first_set_lane(hit_i) : last_set_lane(pos_i);
        if (qi < 0) qi = 0;
        before = (qi > 0) ? seg_read<SEG>(cum_i, qi - 1, base) : H(0);
        lo_q = seg_read<SEG>(rlo, qi, base);
        dg_q = seg_read<SEG>(rdg, qi, base);
      } else {
        // more channels than lanes: channel lane + SEG j sits in chunk j; the chosen
        // channel's diagonal bounds are read once it is known
        constexpr int CQ = kWave / SEG;
        H rs[CQ];
#pragma unroll
        for (int j = 0; j < CQ; ++j) {
          const int ch = lane + SEG * j;
          rs[j] = (ch < a.nq) ? static_cast<H>(Rc[(static_cast<size_t>(ch) * NP + b) * 4]) : H(0);
        }
        H tot = H(0);
#pragma unroll
        for (int j = 0; j < CQ; ++j) tot += seg_sum<SEG>(rs[j]);
        thr = u2 * tot;
        int lastq = -1;
        qi = seg_pick<SEG, CQ, H>(rs, thr, H(0), base, &lastq);
        if (qi < 0) qi = lastq;
        if (qi < 0) qi = 0;
        const double* c4 = Rc + (static_cast<size_t>(qi) * NP + b) * 4;
        lo_q = static_cast<H>(c4[1]);
        dg_q = static_cast<H>(c4[2]);
        before = H(0);
#pragma unroll
        for (int j = 0; j < CQ; ++j) before += seg_sum<SEG>((lane + SEG * j < qi) ? rs[j] : H(0));
      }
      const H rel = thr - before;
      if (!(rel >= lo_q && rel < lo_q + dg_q)) {
        const double* row = a.R + ((static_cast<size_t>(g) * a.nq + qi) * NP + b) * NP;
        H v[PL];
#pragma unroll
        for (int j = 0; j < PL; ++j) {
          const int x = lane + SEG * j;
          v[j] = (x < NP) ? static_cast<H>(row[x]) : H(0);
        }
        int lastpos = -1;
        const int hit = seg_pick<SEG, PL, H>(v, thr, before, base, &lastpos);
        ta = (hit >= 0) ? hit : (lastpos >= 0 ? lastpos : b);
      }
    }
    int kind;
    if (ta != b) {
      // collapse to level ta, carrying the step phase e^{-i e_a dt}
      const double pr = Pre[ta];
      const double pim = Pim[ta];
      const double inv = 1.0 / sqrt(pr * pr + pim * pim);
#pragma unroll
      for (int j = 0; j < PL; ++j) {
        const int x = lane + SEG * j;
        cr[j] = (x == ta) ? static_cast<H>(pr * inv) : H(0);
        ci[j] = (x == ta) ? static_cast<H>(pim * inv) : H(0);
      }
      kind = (Eg[ta] <= Eg[b]) ? AQT_KIND_RELAX : AQT_KIND_EXCITE;
      if (ta < gsz && b >= gsz) ++net;
      else if (b < gsz && ta >= gsz) --net;
    } else {
      const double* zd = a.zdiag + (static_cast<size_t>(g) * a.nq + qi) * NP;
      H z[PL];
      if (chs) {
#pragma unroll
        for (int j = 0; j < PL; ++j) {
          const int x = lane + SEG * j;
          z[j] = (x < NP) ? static_cast<H>(chs[qi * NP + x].w) : H(0);
        }
      } else {
#pragma unroll
        for (int j = 0; j < PL; ++j) {
          const int x = lane + SEG * j;
          z[j] = (x < NP) ? static_cast<H>(zd[x]) : H(0);
        }
      }
#pragma unroll
      for (int j = 0; j < PL; ++j) {
        cr[j] *= z[j];
        ci[j] *= z[j];
      }
      kind = AQT_KIND_DEPHASE;
    }
    H nrm = H(0);
#pragma unroll
    for (int j = 0; j < PL; ++j) nrm += cr[j] * cr[j] + ci[j] * ci[j];
    nrm = seg_sum<SEG>(nrm);
    const H inv = H(1) / sqrt(nrm);
#pragma unroll
    for (int j = 0; j < PL; ++j) {
      cr[j] *= inv;
      ci[j] *= inv;
    }
    if (lane == 0) {
      if (a.jumps && cnt >= a.cap) atomicOr(a.flags, AQT_RUN_RECORDS_TRUNCATED);
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
    r = draw(3ull * m);
  }
  if (guard == AQT_MAX_JUMPS_PER_STEP && lane == 0) atomicOr(a.flags, AQT_RUN_JUMP_LIMIT);
  double pg = 0.0, pt = 0.0;
#pragma unroll
  for (int j = 0; j < PL; ++j) {
    const int x = lane + SEG * j;
    const double xr = cr[j], xi = ci[j];
    const double w2 = xr * xr + xi * xi;
    pt += w2;
    if (x < gsz) pg += w2;
    if (x < NP) {
      amp<NP, T>(S, t, 0, x) = static_cast<T>(cr[j]);
      amp<NP, T>(S, t, 1, x) = static_cast<T>(ci[j]);
    }
  }
  pg = seg_sum<SEG>(pg);
  pt = seg_sum<SEG>(pt);
  if (lane == 0) {
    s_p[t] = pg / pt;
    s_rn[t] = r;
    s_m[t] = m;
    s_cnt[t] = cnt;
    s_net[t] = net;
    if (((3ull * static_cast<uint64_t>(m) + 1ull) >> 2) != Bc) rc.list[atomicAdd(rc.n, 1)] = t;
  }
}

// Per-grid-point tables the jump handler reads, staged in LDS each step in the FP32
// kernels: loaded from HBM/L2 ahead of the GEMM, stored after it, so a crossing finds
// them at LDS latency.  (The BF16 and FP64 kernels run out of registers holding them
// across the GEMM and read them from the tables.)
template <class Mode>
constexpr bool stage_tables() {
  return Mode::KC == 4 && sizeof(typename Mode::T) == 4;
}
// The channel entries of a grid point (per channel and level: R's row sum, its part
// below the diagonal, its diagonal, z_bb) as well, in the FP32 kernels with 128 or
// more levels when they fit kChanStage entries: the channel draw and the dephasing
// factors of a crossing then need no dependent global load.  (The smaller-level
// kernels keep their LDS for more resident workgroups.)
constexpr int kChanStage = 2048;
template <class Mode, int NP>
constexpr bool stage_channels() {
  return stage_tables<Mode>() && NP >= 128;
}

// --------------------------------------------------------------- kernel ----
// Work split of the overlap GEMM over the WV wavefronts: with WV or more row
// tiles each wave owns the row tiles rt = wave (mod WV) for every column tile
// (one A fragment feeds TQ MFMAs); with fewer, waves take (row tile, column
// tile) pairs.  The k loop is outermost so each wave keeps UPW*QG independent
// accumulator chains in flight.
template <int NP, int TQ, class Mode, int WV>
struct TileShared {
  using T = typename Mode::T;
  static constexpr int NRT = NP / 16;
  static constexpr int TT = 8 * TQ;
  static constexpr int NSLOT = (NRT >= WV) ? WV : NRT;   // partial squared norms per trajectory
  TileCols<NP, T> S[TQ];
  double nu[NSLOT][TT];   // partial squared norms, accumulated in FP64
  double r[2][TT];   // waiting-time thresholds: read from r[g & 1], written to r[(g + 1) & 1]
  double p[TT];
  int m[TT], cnt[TT], net[TT];
  int kind[3];
  uint64_t rng[TT][8];   // Philox blocks of each trajectory's next draws (RngCache)
  uint64_t rngb[TT];
  int rfl[TT];           // trajectories whose blocks are to be refreshed
  int nrfl;
  double tg[kStepTables][NP];   // the step's Gamma, e^{G dt/2}, E, phase re/im (jump handler)
  float4 chs[stage_channels<Mode, NP>() ? kChanStage : 1];   // the step's channel entries (jump handler)
};

__device__ __forceinline__ const double* step_table(const StepArgs& a, int which) {
  return which == 0 ? a.Gamma : which == 1 ? a.ehalf : which == 2 ? a.E : which == 3 ? a.d64re : a.d64im;
}

template <int NP, int TQ, class Mode, int WV>
__device__ void run_tile(const StepArgs& a, int64_t tile, TileShared<NP, TQ, Mode, WV>& sh) {
  using T = typename Mode::T;
  using Acc = typename Mode::Acc;
  constexpr int NRT = NP / 16;
  constexpr int TT = 8 * TQ;
  constexpr int QG = (NRT >= WV) ? TQ : 1;         // column tiles per work unit
  constexpr int NUNITS = NRT * (TQ / QG);
  constexpr int UPW = (NUNITS + WV - 1) / WV;      // units per wave
  constexpr int NKC = NP / Mode::KC;
  static_assert(TT <= kWave, "tile must fit one wavefront for the decision pass");

  auto& S = sh.S;
  auto& s_nu = sh.nu;
  constexpr int NSLOT = TileShared<NP, TQ, Mode, WV>::NSLOT;
  double* s_p = sh.p;
  int* s_m = sh.m;
  int* s_cnt = sh.cnt;
  int* s_net = sh.net;
  int* s_kind = sh.kind;

  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform per wave
  const int64_t tb = tile * TT;
  const int lc = lane & 15;          // MFMA output column
  const int part = (lane >> 3) & 1;  // 0: real part, 1: imaginary part

  const RngCache rc{sh.rng, sh.rngb, sh.rfl, &sh.nrfl};
  if (tid < TT) {
    const int64_t j = tb + tid;
    sh.r[1][tid] = (j < a.K) ? draw_uniform(a.seed, a.iid, a.traj0 + j, 0) : 2.0;   // read at g = 1
    s_m[tid] = 0;
    s_cnt[tid] = 0;
    s_net[tid] = 0;
  }
  if (tid < 3) s_kind[tid] = 0;
  if (tid == 0) sh.nrfl = 0;
  if (wave == WV - 1) rng_refill(a, tb, TT, nullptr, nullptr, rc, lane);   // m = 0: blocks 0 and 1

  int rt_u[UPW], q0_u[UPW];
  bool ok_u[UPW];
#pragma unroll
  for (int u = 0; u < UPW; ++u) {
    const int unit = wave + WV * u;
    ok_u[u] = (NUNITS % WV == 0) || unit < NUNITS;
    rt_u[u] = unit % NRT;
    q0_u[u] = (unit / NRT) * QG;
  }
  Acc acc[UPW][QG];
  // with >= WV row tiles every unit covers all column tiles (q0 = 0) and each wave
  // keeps one norm partial per trajectory (NSLOT = WV); otherwise units are
  // (row tile, column tile) pairs and the partials are per row tile
  constexpr bool kSharedQ = (NRT >= WV);
  static_assert(NSLOT == (kSharedQ ? WV : NRT), "norm slots follow the work split");
#define q0(u) (kSharedQ ? 0 : q0_u[u])
  // fragment (g, row tile, k chunk) lives at ((g * NRT + rt) * NKC + k) * 64 + lane
  size_t fbase[UPW];
#pragma unroll
  for (int u = 0; u < UPW; ++u) fbase[u] = static_cast<size_t>(rt_u[u]) * NKC * kWave + lane;
#define frag_index(gg, u, k) \
  (static_cast<size_t>(gg) * (NRT * NKC * kWave) + fbase[u] + static_cast<size_t>(k) * kWave)
  constexpr int PF = prefetch_depth<Mode, NP>();
  static_assert(NKC % PF == 0, "prefetch depth must divide the k chunks");
  Frag<Mode> ring[PF][UPW];
  if (a.M_run > 2) {
#pragma unroll
    for (int s2 = 0; s2 < PF; ++s2)
#pragma unroll
      for (int u = 0; u < UPW; ++u)
        if (ok_u[u]) ring[s2][u] = load_frag<Mode>(a, frag_index(2, u, s2));
  }

  // Accumulator <-> LDS: four rows of one column per lane (consecutive rows in
  // the FP32 layouts, one 16-byte access).
  auto acc_load = [&](int q, int rt, Acc& v) {
    if constexpr (sizeof(T) == 4) {
      v = *reinterpret_cast<const Acc*>(&S[q][lc][rt * 16 + 4 * (lane >> 4)]);
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) v[i] = S[q][lc][rt * 16 + Mode::row(lane, i)];
    }
  };
  auto acc_store = [&](int q, int rt, const Acc& v) {
    if constexpr (sizeof(T) == 4) {
      *reinterpret_cast<Acc*>(&S[q][lc][rt * 16 + 4 * (lane >> 4)]) = v;
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) S[q][lc][rt * 16 + Mode::row(lane, i)] = v[i];
    }
  };
  // The accumulators keep C between steps (the identity split starts from C);
  // only column tiles touched by the jump handler are reloaded from LDS.
  unsigned dirty = 0;
  // channel entries staged per step when the kernel keeps room for them and they fit
  constexpr int CHPT = stage_channels<Mode, NP>() ? (kChanStage + WV * 64 - 1) / (WV * 64) : 1;
  const int nch_e = a.nq * NP;
  const bool ch_on = stage_channels<Mode, NP>() && a.chf != nullptr && nch_e <= kChanStage;

  for (int g = 1; g < a.M_run; ++g) {
    const int gsz = a.gs[g];
    // Philox blocks for the trajectories that jumped in the previous step (their
    // handlers listed them before the last barrier; this step's handlers read the
    // blocks only after the barrier that follows the GEMM)
    if (g > 1 && wave == 0) {
      const int nr = __builtin_amdgcn_readfirstlane(sh.nrfl);
      if (nr) {
        rng_refill(a, tb, nr, sh.rfl, s_m, rc, lane);
        if (lane == 0) sh.nrfl = 0;
      }
    }
    // ---- 1. C + Delta C (or the initial state at g = 1)
    if (g == 1) {
#pragma unroll
      for (int u = 0; u < UPW; ++u) {
        if (!ok_u[u]) continue;
#pragma unroll
        for (int qq = 0; qq < QG; ++qq)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int row = rt_u[u] * 16 + Mode::row(lane, i);
            acc[u][qq][i] = part ? T(0) : static_cast<T>(a.cinit[row]);
          }
      }
    } else if (dirty) {
#pragma unroll
      for (int u = 0; u < UPW; ++u) {
        if (!ok_u[u]) continue;
#pragma unroll
        for (int qq = 0; qq < QG; ++qq)
          if ((dirty >> (q0(u) + qq)) & 1u) acc_load(q0(u) + qq, rt_u[u], acc[u][qq]);
      }
    }
    // the step's phase factors, loaded ahead of the GEMM (used by the epilogue)
    T dpre[UPW][4], dpim[UPW][4];
    {
      const T* dr = static_cast<const T*>(a.dre) + static_cast<size_t>(g) * NP;
      const T* di = static_cast<const T*>(a.dim) + static_cast<size_t>(g) * NP;
#pragma unroll
      for (int u = 0; u < UPW; ++u)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          dpre[u][i] = dr[rt_u[u] * 16 + Mode::row(lane, i)];
          dpim[u][i] = di[rt_u[u] * 16 + Mode::row(lane, i)];
        }
    }
    constexpr bool STAGED = stage_tables<Mode>();
    constexpr int NTG = kStepTables * NP, TGPT = STAGED ? (NTG + WV * 64 - 1) / (WV * 64) : 1;
    double tgv[TGPT];
#pragma unroll
    for (int k = 0; k < TGPT; ++k) {
      const int f = tid + k * WV * 64;
      tgv[k] = (STAGED && f < NTG) ? step_table(a, f / NP)[static_cast<size_t>(g) * NP + f % NP] : 0.0;
    }
    float4 chv[CHPT];
#pragma unroll
    for (int k = 0; k < CHPT; ++k) {
      const int f = tid + k * WV * 64;
      chv[k] = (ch_on && f < nch_e) ? a.chf[static_cast<size_t>(g) * nch_e + f] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    if (g > 1) {
      T bnx[QG];
      if constexpr (Mode::KC == 4 && kSharedQ) {
#pragma unroll
        for (int qq = 0; qq < QG; ++qq) bnx[qq] = S[qq][lc][lane >> 4];
      }
      // two wavefronts share each SIMD, and with equal priorities they issue so that one
      // finishes its share early and leaves the other to run the tail of the GEMM alone
      // (8% slower in FP32); one of each pair at a raised priority keeps both issuing to
      // the end.  Raising waves 0-3 (wave 0 starts the step late: it refreshes the Philox
      // caches) measured 0.6% faster than raising waves 4-7 in FP32, 0.7% in FP64 against
      // equal priorities, and wave 0 one level higher still another 0.6% in FP32.
      if (WV == 8 && wave == 0) __builtin_amdgcn_s_setprio(2);
      else if (WV == 8 && wave < 4) __builtin_amdgcn_s_setprio(1);
      for (int kc = 0; kc < NKC; kc += PF) {
#pragma unroll
        for (int s2 = 0; s2 < PF; ++s2) {
          const int k = kc + s2;
          Frag<Mode> av[UPW];
#pragma unroll
          for (int u = 0; u < UPW; ++u) av[u] = ring[s2][u];
          // refill this slot PF chunks ahead (next step's first chunks at the end)
          // (after the last step the slot reloads grid M_run - 1: in bounds, unused)
          const int kn = k + PF;
          const int gn = min(kn < NKC ? g : g + 1, a.M_run - 1);
          const int kk = kn < NKC ? kn : kn - NKC;
#pragma unroll
          for (int u = 0; u < UPW; ++u)
            if (ok_u[u]) ring[s2][u] = load_frag<Mode>(a, frag_index(gn, u, kk));
          if constexpr (Mode::KC == 4 && kSharedQ) {
            // B for this chunk was read one chunk ahead; read the next one now (on
            // the last chunk that is padding row NP + lane / 16: in bounds, unused)
            T bcur[QG];
#pragma unroll
            for (int qq = 0; qq < QG; ++qq) bcur[qq] = bnx[qq];
            const int krn = 4 * (k + 1) + (lane >> 4);
#pragma unroll
            for (int qq = 0; qq < QG; ++qq) bnx[qq] = S[qq][lc][krn];
#pragma unroll
            for (int u = 0; u < UPW; ++u)
#pragma unroll
              for (int qq = 0; qq < QG; ++qq) acc[u][qq] = mfma_k4(av[u].v, bcur[qq], acc[u][qq]);
          } else if constexpr (Mode::KC == 4) {
            const int krow = 4 * k + (lane >> 4);
            T bv[UPW][QG];
#pragma unroll
            for (int u = 0; u < UPW; ++u)
#pragma unroll
              for (int qq = 0; qq < QG; ++qq)
                bv[u][qq] = (u == 0 || !kSharedQ) ? S[q0(u) + qq][lc][krow] : bv[0][qq];
#pragma unroll
            for (int u = 0; u < UPW; ++u) {
              if (!ok_u[u]) continue;
#pragma unroll
              for (int qq = 0; qq < QG; ++qq) acc[u][qq] = mfma_k4(av[u].v, bv[u][qq], acc[u][qq]);
            }
          } else if constexpr (Mode::KC == 16) {
            const int k0 = 16 * k + 4 * (lane >> 4);
#pragma unroll
            for (int u = 0; u < UPW; ++u) {
              if (!ok_u[u]) continue;
              const s16x4 ah = __builtin_bit_cast(s16x4, av[u].h);
              const s16x4 al = __builtin_bit_cast(s16x4, av[u].l);
#pragma unroll
              for (int qq = 0; qq < QG; ++qq) {
                float xv[4];
                *reinterpret_cast<float4*>(xv) = *reinterpret_cast<const float4*>(&S[q0(u) + qq][lc][k0]);
                s16x4 bh, bl;
                split4(xv, bh, bl);
                Acc c = acc[u][qq];
                c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, c, 0, 0, 0);
                acc[u][qq] = c;
              }
            }
          } else {
            const int k0 = 32 * k + 8 * (lane >> 4);
            // B split once per column tile when every unit shares the column tiles
            bf16x8 bh[kSharedQ ? QG : 1], bl[kSharedQ ? QG : 1];
            if constexpr (kSharedQ) {
#pragma unroll
              for (int qq = 0; qq < QG; ++qq) {
                float xv[8];
                *reinterpret_cast<float4*>(xv) = *reinterpret_cast<const float4*>(&S[qq][lc][k0]);
                *reinterpret_cast<float4*>(xv + 4) = *reinterpret_cast<const float4*>(&S[qq][lc][k0 + 4]);
                split8(xv, bh[qq], bl[qq]);
              }
            }
#pragma unroll
            for (int u = 0; u < UPW; ++u) {
              if (!ok_u[u]) continue;
              const bf16x8 ah = __builtin_bit_cast(bf16x8, av[u].h);
              const bf16x8 al = __builtin_bit_cast(bf16x8, av[u].l);
#pragma unroll
              for (int qq = 0; qq < QG; ++qq) {
                bf16x8 h, l;
                if constexpr (kSharedQ) {
                  h = bh[qq];
                  l = bl[qq];
                } else {
                  float xv[8];
                  *reinterpret_cast<float4*>(xv) = *reinterpret_cast<const float4*>(&S[q0(u) + qq][lc][k0]);
                  *reinterpret_cast<float4*>(xv + 4) = *reinterpret_cast<const float4*>(&S[q0(u) + qq][lc][k0 + 4]);
                  split8(xv, h, l);
                }
                Acc c = acc[u][qq];
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, h, c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, l, c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, h, c, 0, 0, 0);
                acc[u][qq] = c;
              }
            }
          }
        }
      }
    }
    if (WV == 8) __builtin_amdgcn_s_setprio(0);
    // the step tables for this step's handlers (the previous step's handlers are done)
    if constexpr (STAGED) {
#pragma unroll
      for (int k = 0; k < TGPT; ++k) {
        const int f = tid + k * WV * 64;
        if (f < NTG) sh.tg[f / NP][f % NP] = tgv[k];
      }
    }
    if (ch_on) {
#pragma unroll
      for (int k = 0; k < CHPT; ++k) {
        const int f = tid + k * WV * 64;
        if (f < nch_e) sh.chs[f] = chv[k];
      }
    }
    __syncthreads();   // every wave has finished reading S
    // ---- 2. C' = d o C and the squared norms (partial sums per wave or row tile).
    // The squares of state-precision amplitudes are exact in FP64 and every sum of
    // them (per lane, across lanes, across slots) is taken in FP64, so the threshold
    // test sees the norm of the stored state to FP64 rounding whatever the state
    // precision: a compensated norm, not a state-precision running sum.
    {
      double nacc[QG];
#pragma unroll
      for (int qq = 0; qq < QG; ++qq) nacc[qq] = 0.0;
#pragma unroll
      for (int u = 0; u < UPW; ++u) {
        if (!ok_u[u]) continue;
        const int rt = rt_u[u];
        T drv[4], div[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          drv[i] = dpre[u][i];
          div[i] = dpim[u][i];
        }
#pragma unroll
        for (int qq = 0; qq < QG; ++qq) {
          double nrm = 0.0;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const T y = acc[u][qq][i];
            const T yp = xor8(y);       // the other part of the same amplitude
            const T yr = part ? yp : y, yi = part ? y : yp;
            const T c = part ? (drv[i] * yi + div[i] * yr) : (drv[i] * yr - div[i] * yi);
            acc[u][qq][i] = c;
            const double cd = static_cast<double>(c);
            nrm = fma(cd, cd, nrm);
          }
          acc_store(q0(u) + qq, rt, acc[u][qq]);
          if constexpr (kSharedQ) {
            nacc[qq] += nrm;
          } else {
            nrm += xor8(nrm);
            nrm = swap_add<16>(nrm);
            nrm = swap_add<32>(nrm);
            if (lane < 8) s_nu[rt][(q0(u) + qq) * 8 + lane] = nrm;
          }
        }
      }
      if constexpr (kSharedQ) {
#pragma unroll
        for (int qq = 0; qq < QG; ++qq) {
          double nrm = nacc[qq];
          nrm += xor8(nrm);
          nrm = swap_add<16>(nrm);
          nrm = swap_add<32>(nrm);
          if (lane < 8) s_nu[wave][qq * 8 + lane] = nrm;
        }
      }
    }
    __syncthreads();
    // ---- 3. threshold test.  Every wavefront takes it for all TT trajectories (lane t,
    // the same FP64 sums in the same order), so each knows the crossing set from a
    // ballot, without a list or another barrier; the thresholds it reads are not
    // written this step (the handlers write the other buffer).  Wavefront 0 records
    // the ground-cluster weight of the trajectories that do not cross and carries
    // their thresholds over.
    const double* s_r = sh.r[g & 1];
    double* s_rn = sh.r[(g + 1) & 1];
    uint64_t cmask;
    {
      bool cross = false;
      double nu = 0.0;
      const bool valid = lane < TT && tb + lane < a.K;
      if (lane < TT) {
#pragma unroll
        for (int sl = 0; sl < NSLOT; ++sl) nu += s_nu[sl][lane];
        cross = valid && nu <= s_r[lane];
      }
      cmask = __ballot(cross);
      if (wave == 0 && lane < TT && !cross) {
        double gw = 0.0;
        if (valid)
          for (int row = 0; row < gsz; ++row) {
            const double re = static_cast<double>(amp<NP, T>(S, lane, 0, row));
            const double im = static_cast<double>(amp<NP, T>(S, lane, 1, row));
            gw += re * re + im * im;
          }
        s_p[lane] = valid ? gw / nu : 0.0;
        s_rn[lane] = s_r[lane];
      }
    }
    const int ncross = __popcll(cmask);
    {
      // 64 / SEG crossings per wavefront, one per segment of SEG lanes; crossing e is
      // the trajectory of the e-th set bit of the mask
      constexpr int SEG = seg_width<NP>();
      constexpr int NSEG = kWave / SEG;
      const int seg = (tid & (kWave - 1)) / SEG;
      for (int e0 = wave * NSEG; e0 < ncross; e0 += WV * NSEG) {
        const int e = e0 + seg;
        if (e < ncross) {
          uint64_t mm = cmask;
          for (int k = 0; k < e; ++k) mm &= mm - 1;
          const int t = __builtin_ctzll(mm);
          finish_crossing<NP, T, STAGED>(a, g, t, tb + t, S, s_r, s_rn, s_m, s_cnt, s_net, s_p, s_kind, rc,
                                         &sh.tg[0][0], ch_on ? sh.chs : nullptr);
        }
      }
    }
    __syncthreads();
    // column tiles whose amplitudes the handler rewrote
    dirty = 0;
#pragma unroll
    for (int q = 0; q < TQ; ++q)
      if ((cmask >> (8 * q)) & 0xffull) dirty |= 1u << q;
    // ---- 4. per-tile observable sums (wave 0)
    if (wave == 0) {
      const double p = (lane < TT) ? s_p[lane] : 0.0;
      const double sp = seg_sum<64>(p);
      const double sq = seg_sum<64>(p * p);
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
        a.final_state[(j * a.n + x) * 2 + 0] = static_cast<double>(amp<NP, T>(S, t, 0, x));
        a.final_state[(j * a.n + x) * 2 + 1] = static_cast<double>(amp<NP, T>(S, t, 1, x));
      }
    }
  }
  if (a.jump_totals && tid < 3 && s_kind[tid])
    atomicAdd(reinterpret_cast<unsigned long long*>(&a.jump_totals[tid]),
              static_cast<unsigned long long>(s_kind[tid]));
  __syncthreads();   // the shared tile state may be reused by the caller
#undef q0
#undef frag_index
}

// Wavefronts per SIMD the register allocation must leave room for: the small-level
// FP32/BF16 kernels are latency-bound (jump handling), and three or four resident
// wavefronts per SIMD hide more of it than the registers the compiler would
// otherwise keep; the large-level and FP64 kernels keep the compiler's choice.
template <int NP, class Mode>
constexpr int min_waves_per_simd() {
  return (sizeof(typename Mode::T) == 8 || NP > 64) ? 1 : (NP <= 16 ? 4 : 3);
}

template <int NP, int TQ, class Mode>
__global__ __launch_bounds__((waves_for<NP, Mode>() * 64))
__attribute__((amdgpu_waves_per_eu(min_waves_per_simd<NP, Mode>()))) void k_trajectories(StepArgs a) {
  constexpr int WV = waves_for<NP, Mode>();
  __shared__ TileShared<NP, TQ, Mode, WV> sh;
  run_tile<NP, TQ, Mode, WV>(a, blockIdx.x, sh);
}

// Compensated (Neumaier) running sum: s + c carries the rounding error of every addition.
struct CompSum {
  double s = 0.0, c = 0.0;
  __device__ void add(double x) {
    const double t = s + x;
    c += (fabs(s) >= fabs(x)) ? (s - t) + x : (x - t) + s;
    s = t;
  }
  __device__ double value() const { return s + c; }
};

__global__ void k_reduce_partials(const double* __restrict__ partial, int64_t tiles, int M, double K,
                                  double* __restrict__ sum, double* __restrict__ sumsq) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= M) return;
  double s = 0.0, q = 0.0;
  if (g == 0) {
    s = K;   // every trajectory starts in the ground state of H(0)
    q = K;
  } else {
    CompSum cs, cq;
    for (int64_t t = 0; t < tiles; ++t) {
      cs.add(partial[(t * M + g) * 2]);
      cq.add(partial[(t * M + g) * 2 + 1]);
    }
    s = cs.value();
    q = cq.value();
  }
  if (sum) sum[g] = s;
  if (sumsq) sumsq[g] = q;
}

// Column-tile counts instantiated per level count and precision.
constexpr int kTQ[] = {1, 2, 4, 5, 8};

__host__ __device__ constexpr bool tq_allowed(int NP, int TQ, bool f64) {
  return (NP <= 64) ? (TQ != 5 && !(f64 && NP == 64 && TQ == 8))
                    : (TQ <= 5 && !(f64 && TQ > 2));
}

// ------------------------------------------------------------- batched ----
// Many instances in few persistent launches.  Items (instance, tile) are grouped by
// padded level count and tile width; one launch per group (largest levels first)
// has its workgroups pull the group's items from an atomic queue (longest first)
// and run each with the trajectory kernel's tile body, wavefront count and
// occupancy floor.
struct BatchItem {
  int inst;
  int tile;
};

constexpr int kLevelClasses[] = {256, 128, 64, 32, 16};   // launch order
constexpr int kTileClasses[] = {1, 2, 4, 8};              // column tiles
constexpr int kNumClasses = 20;                           // (levels, tile) groups

__global__ void k_batch_reset(int* counter, int n) {
  if (blockIdx.x == 0 && static_cast<int>(threadIdx.x) < n) counter[threadIdx.x] = 0;
}

// BF16 runs of 16-level instances use the K = 16 MFMA, as in the single-instance launch
template <int NP, class Mode>
using BatchMode = typename std::conditional<NP == 16 && Mode::KC == 32, ModeBF16K16, Mode>::type;

// column tiles a batch may use: 1, 2, 4, 8 up to 64 levels, 1, 2 above
__host__ __device__ constexpr bool batch_tq(int NP, int TQ, bool f64) {
  return tq_allowed(NP, TQ, f64) && ((NP <= 64) ? (TQ == 1 || TQ == 2 || TQ == 4 || TQ == 8) : (TQ == 1 || TQ == 2));
}

template <int NP, int TQ, class Mode>
__global__ __launch_bounds__((waves_for<NP, BatchMode<NP, Mode>>() * 64))
__attribute__((amdgpu_waves_per_eu(min_waves_per_simd<NP, BatchMode<NP, Mode>>()))) void k_batch(
    const StepArgs* __restrict__ args, const BatchItem* __restrict__ items, int n_items, int* counter) {
  using M = BatchMode<NP, Mode>;
  constexpr int WV = waves_for<NP, M>();
  __shared__ TileShared<NP, TQ, M, WV> sh;
  __shared__ int s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (it >= n_items) break;
    const int inst = __builtin_amdgcn_readfirstlane(items[it].inst);
    const int tile = __builtin_amdgcn_readfirstlane(items[it].tile);
    run_tile<NP, TQ, M, WV>(args[inst], tile, sh);
  }
}

__global__ void k_reduce_batch(const StepArgs* __restrict__ args) {
  const StepArgs& a = args[blockIdx.y];
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= a.M) return;
  double s = 0.0, q = 0.0;
  if (g == 0) {
    s = static_cast<double>(a.K);
    q = s;
  } else {
    CompSum cs, cq;
    for (int64_t t = 0; t < a.tiles; ++t) {
      cs.add(a.partial[(t * a.M + g) * 2]);
      cq.add(a.partial[(t * a.M + g) * 2 + 1]);
    }
    s = cs.value();
    q = cq.value();
  }
  if (a.pgs_sum) a.pgs_sum[g] = s;
  if (a.pgs_sumsq) a.pgs_sumsq[g] = q;
}

template <class Mode, int NP>
hipError_t launch_tq(int TQ, const StepArgs& a, int64_t blocks, hipStream_t st) {
  constexpr bool f64 = sizeof(typename Mode::T) == 8;
#define AQT_CASE(tq)                                                                          \
  if constexpr (tq_allowed(NP, tq, f64)) {                                                    \
    if (TQ == tq) {                                                                           \
      hipLaunchKernelGGL((k_trajectories<NP, tq, Mode>), dim3(static_cast<unsigned>(blocks)), \
                         dim3(waves_for<NP, Mode>() * 64), 0, st, a);                         \
      return hipGetLastError();                                                               \
    }                                                                                         \
  }
  AQT_CASE(1) AQT_CASE(2) AQT_CASE(4) AQT_CASE(5) AQT_CASE(8)
#undef AQT_CASE
  return hipErrorInvalidValue;
}

template <class Mode>
hipError_t launch_mode(int NP, int TQ, const StepArgs& a, int64_t blocks, hipStream_t st) {
  switch (NP) {
    case 16:
      if constexpr (Mode::KC == 4) return launch_tq<Mode, 16>(TQ, a, blocks, st);
      else return launch_tq<ModeBF16K16, 16>(TQ, a, blocks, st);
    case 32: return launch_tq<Mode, 32>(TQ, a, blocks, st);
    case 64: return launch_tq<Mode, 64>(TQ, a, blocks, st);
    case 128: return launch_tq<Mode, 128>(TQ, a, blocks, st);
    case 256: return launch_tq<Mode, 256>(TQ, a, blocks, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

// Column tiles per workgroup: minimise the largest per-CU load
// ceil(workgroups / CUs) * TQ (every workgroup does the same work per
// trajectory-step), preferring larger tiles on ties (fewer overlap re-reads).
// Trajectories per workgroup (TQ column tiles of 8).  >= 128 levels: one workgroup per
// CU, so the launch takes ceil(workgroups / CUs) rounds, each costing the measured
// time of one tile of that width (relative units, n = 256 on MI355X; wider tiles
// amortise the overlap operand over more trajectories).  Smaller level counts fit
// several workgroups per CU: the widest tile that still gives every CU a workgroup.
int choose_tq(int NP, int precision, int64_t K, int cus) {
  const int64_t tiles8 = (K + 7) / 8;
  const bool f64 = precision == AQT_FP64;
  if (NP <= 64) {
    int best = 1;
    for (int tq : kTQ)
      if (tq_allowed(NP, tq, f64) && (tiles8 + tq - 1) / tq >= cus) best = tq > best ? tq : best;
    return best;
  }
  auto round_cost = [&](int tq) -> int64_t {
    if (f64) return tq == 1 ? 24 : 43;
    switch (tq) {   // ms per CU-full round at 256 levels, measured on a 2000-point anneal
      case 1: return 30;
      case 2: return 63;
      case 4: return 41;
      default: return 50;
    }
  };
  int best = 1;
  int64_t best_cost = INT64_MAX;
  for (int tq : kTQ) {
    if (!tq_allowed(NP, tq, f64)) continue;
    const int64_t wgs = (tiles8 + tq - 1) / tq;
    const int64_t cost = ((wgs + cus - 1) / cus) * round_cost(tq);
    if (cost < best_cost || (cost == best_cost && tq > best)) {
      best = tq;
      best_cost = cost;
    }
  }
  return best;
}

namespace {

// Column tiles per workgroup of a run (explicit or chosen); 0 for an unsupported tile.
int run_tq(const aqt_ctx* ctx, const aqt_run_params* p) {
  const int prec = p->precision;
  const int cus = ctx->cus > 0 ? ctx->cus : 256;
  const int tq = p->tile ? p->tile / 8 : choose_tq(ctx->NP, prec, p->n_traj, cus);
  if (p->tile && (p->tile % 8 || !(tq == 1 || tq == 2 || tq == 4 || tq == 5 || tq == 8) ||
                  !tq_allowed(ctx->NP, tq, prec == AQT_FP64)))
    return 0;
  return tq;
}

// Enqueues the trajectory kernel and the observable reduction with the per-tile sums
// in `partial` ([tiles][M][2] doubles; every entry g >= 1 is written before it is read).
aqt_status enqueue_run(aqt_ctx* ctx, const aqt_run_params* p, const aqt_outputs* o, int tq, double* partial) {
  const int prec = p->precision;
  const int64_t TT = 8 * tq;
  const int64_t tiles = (p->n_traj + TT - 1) / TT;
  StepArgs a{};
  a.M = ctx->M;
  a.M_run = ctx->M;
  a.NP = ctx->NP;
  a.TQ = tq;
  a.tiles = tiles;
  a.pgs_sum = o->pgs_sum;
  a.pgs_sumsq = o->pgs_sumsq;
  a.n = ctx->n;
  a.nq = ctx->tab_nch;   // jump channels
  a.tbeg = ctx->tbeg.as<double>();
  a.tlen = ctx->tlen.as<double>();
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
  a.Rcol = ctx->Rcol.as<double>();
  a.ehalf = ctx->ehalf.as<double>();
  a.zdiag = ctx->zdiag.as<double>();
  a.chf = (prec == AQT_FP32) ? ctx->pk_ch.as<float4>() : nullptr;
  a.E = ctx->E.as<double>();
  a.gs = ctx->gs.as<int>();
  a.partial = partial;
  a.jump_totals = o->jump_totals;
  a.jump_count = o->jump_count;
  a.jumps = o->jumps;
  a.net_gs = o->net_gs;
  a.net_hist = o->net_hist;
  a.hist_lo = o->hist_lo;
  a.hist_hi = o->hist_hi;
  a.final_state = o->final_state;
  a.flags = ctx->run_flags.as<int>();

  hipError_t e;
  if (prec == AQT_FP64) e = launch_mode<ModeF64>(ctx->NP, tq, a, tiles, ctx->stream);
  else if (prec == AQT_FP32) e = launch_mode<ModeF32>(ctx->NP, tq, a, tiles, ctx->stream);
  else e = launch_mode<ModeBF16>(ctx->NP, tq, a, tiles, ctx->stream);
  if (e != hipSuccess) return ctx->fail(AQT_EHIP, std::string("trajectory kernel launch: ") + hipGetErrorString(e));
  if (o->pgs_sum || o->pgs_sumsq) {
    hipLaunchKernelGGL(k_reduce_partials, dim3((ctx->M + 255) / 256), dim3(256), 0, ctx->stream,
                       partial, tiles, ctx->M, static_cast<double>(p->n_traj), o->pgs_sum, o->pgs_sumsq);
    e = hipGetLastError();
    if (e != hipSuccess) return ctx->fail(AQT_EHIP, std::string("reduction launch: ") + hipGetErrorString(e));
  }
  return AQT_OK;
}

// ---------------------------------------------------------- no allocation ----
// Per-tile observable sums of aqt_run_noalloc: a fixed buffer in device memory, one
// copy per device (held until the process ends).  Host code never passes `scratch`
// itself to a kernel: its device address comes from hipGetSymbolAddress, taken once
// per device with that device current, and only that address is used.
constexpr size_t kScratchBytes = static_cast<size_t>(AQT_NOALLOC_SCRATCH_BYTES);
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};

}  // namespace

aqt_status launch_run(aqt_ctx* ctx, const aqt_run_params* p, const aqt_outputs* o) {
  const int prec = p->precision;
  aqt_status s = check_step_decay(ctx, prec);
  if (s != AQT_OK) return s;
  s = pack_for_precision(ctx, prec);
  if (s != AQT_OK) return s;
  const int tq = run_tq(ctx, p);
  if (!tq) return ctx->fail(AQT_EINVAL, "unsupported tile size for this level count and precision");
  const int64_t tiles = (p->n_traj + 8 * tq - 1) / (8 * tq);
  const size_t need = static_cast<size_t>(tiles) * ctx->M * 2 * sizeof(double);
  if (ctx->partial.reserve(need) != hipSuccess) return ctx->fail(AQT_ENOMEM, "workspace allocation failed");
  return enqueue_run(ctx, p, o, tq, ctx->partial.as<double>());
}

aqt_status setup_noalloc_scratch(aqt_ctx* ctx) {
  const int dev = ctx->device;
  if (dev < 0 || dev >= kMaxDevices) return ctx->fail(AQT_EINVAL, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_done[dev]) {
    void* ptr = nullptr;
    g_scratch_err[dev] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));   // the device is current
    g_scratch_ptr[dev] = (g_scratch_err[dev] == hipSuccess) ? ptr : nullptr;
    g_scratch_done[dev] = true;
  }
  if (g_scratch_err[dev] != hipSuccess)
    return ctx->fail(AQT_EHIP, std::string("scratch address: ") + hipGetErrorString(g_scratch_err[dev]));
  return AQT_OK;
}

aqt_status launch_run_noalloc(aqt_ctx* ctx, const aqt_run_params* p, const aqt_outputs* o) {
  const int prec = p->precision;
  aqt_status s = check_step_decay(ctx, prec);
  if (s != AQT_OK) return s;
  if (ctx->packed_for != prec)
    return ctx->fail(AQT_ESTATE, "the step operands of this precision are not resident; one aqt_run in this "
                                 "precision after the tables were loaded packs them");
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (ctx->device >= 0 && ctx->device < kMaxDevices) base = g_scratch_ptr[ctx->device];
  }
  if (!base) return ctx->fail(AQT_ESTATE, "the device scratch buffer has no address (aqt_create did not set it up)");
  const int tq = run_tq(ctx, p);
  if (!tq) return ctx->fail(AQT_EINVAL, "unsupported tile size for this level count and precision");
  const int64_t tiles = (p->n_traj + 8 * tq - 1) / (8 * tq);
  const double need = static_cast<double>(tiles) * ctx->M * 2 * sizeof(double);
  if (need > static_cast<double>(kScratchBytes))
    return ctx->fail(AQT_EINVAL, "the run needs " + std::to_string(static_cast<long long>(need)) +
                                     " bytes of per-tile sums (tiles x n_grid x 16), more than the " +
                                     std::to_string(kScratchBytes) + "-byte no-allocation buffer");
  return enqueue_run(ctx, p, o, tq, static_cast<double*>(base));
}

}  // namespace aqt

// ================================================================ batches ===
struct aqt_batch {
  int device = 0;
  hipStream_t capture_stream = nullptr;   // private stream used only for graph capture
  hipStream_t stream = nullptr;           // launch stream (the first context's)
  std::string err;
  int precision = AQT_FP32;
  int n = 0;
  std::vector<aqt_ctx*> ctxs;
  std::vector<aqt::StepArgs> hargs;
  std::vector<int> tiles_per_inst;        // trajectories per workgroup tile chosen per instance
  aqt::DevBuf dargs, ditems, dcounter;
  int n_items = 0;
  int class_off[20] = {};                 // items of each (levels, tile) group
  int class_cnt[20] = {};
  int class_grid[20] = {};                // persistent workgroups per group launch
  // groups after the first run on side streams forked from and joined back into the
  // launch stream, so that one group's tail overlaps the next group's work
  hipStream_t side[3] = {nullptr, nullptr, nullptr};
  hipEvent_t fork = nullptr;
  hipEvent_t join[3] = {nullptr, nullptr, nullptr};
  bool use_graph = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  aqt_status fail(aqt_status s, const std::string& m) {
    err = m;
    return s;
  }
};

namespace aqt {
namespace {

// Items of a launch per (levels, tile) group: [off, off + cnt) of the item array.
struct ClassSpans {
  int off[kNumClasses] = {};
  int cnt[kNumClasses] = {};
};

int batch_class(int NP, int TQ) {
  int l = -1, t = -1;
  for (int c = 0; c < 5; ++c)
    if (kLevelClasses[c] == NP) l = c;
  for (int c = 0; c < 4; ++c)
    if (kTileClasses[c] == TQ) t = c;
  return (l < 0 || t < 0) ? -1 : 4 * l + t;
}

// Calls f.template operator()<NP, TQ>() for the (levels, tile) group c, if the batch allows it.
template <class Mode, class F>
hipError_t with_class(int c, const F& f) {
  constexpr bool f64 = sizeof(typename Mode::T) == 8;
  hipError_t e = hipErrorInvalidValue;
  auto tq = [&](auto np_tag) {
    constexpr int NP = decltype(np_tag)::value;
    switch (kTileClasses[c % 4]) {
      case 1: if constexpr (batch_tq(NP, 1, f64)) e = f.template operator()<NP, 1>(); break;
      case 2: if constexpr (batch_tq(NP, 2, f64)) e = f.template operator()<NP, 2>(); break;
      case 4: if constexpr (batch_tq(NP, 4, f64)) e = f.template operator()<NP, 4>(); break;
      default: if constexpr (batch_tq(NP, 8, f64)) e = f.template operator()<NP, 8>(); break;
    }
  };
  switch (kLevelClasses[c / 4]) {
    case 256: tq(std::integral_constant<int, 256>{}); break;
    case 128: tq(std::integral_constant<int, 128>{}); break;
    case 64: tq(std::integral_constant<int, 64>{}); break;
    case 32: tq(std::integral_constant<int, 32>{}); break;
    default: tq(std::integral_constant<int, 16>{}); break;
  }
  return e;
}

template <class Mode>
struct LaunchGroup {
  const StepArgs* dargs;
  const BatchItem* items;
  int n;
  int* counter;
  int grid;
  hipStream_t st;
  template <int NP, int TQ>
  hipError_t operator()() const {
    hipLaunchKernelGGL((k_batch<NP, TQ, Mode>), dim3(grid), dim3(waves_for<NP, BatchMode<NP, Mode>>() * 64), 0, st,
                       dargs, items, n, counter);
    return hipGetLastError();
  }
};

template <class Mode>
struct GroupOccupancy {
  int* blocks;
  template <int NP, int TQ>
  hipError_t operator()() const {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_batch<NP, TQ, Mode>,
                                                        waves_for<NP, BatchMode<NP, Mode>>() * 64, 0);
  }
};

// One reset of the group counters, then one persistent launch per non-empty group:
// the first on st, the others on the side streams (forked after the reset, joined
// back into st), so the groups run concurrently.
template <class Mode>
hipError_t enqueue_mode(const aqt_batch* b, const StepArgs* dargs, const BatchItem* items, const ClassSpans& sp,
                        int* counter, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, st, counter, kNumClasses);
  hipError_t e = hipGetLastError();
  bool forked = false, used[3] = {false, false, false};
  int k = 0;   // non-empty groups so far
  for (int c = 0; c < kNumClasses && e == hipSuccess; ++c) {
    if (!sp.cnt[c]) continue;
    hipStream_t s = st;
    if (k > 0 && b->side[0]) {
      if (!forked) {
        e = hipEventRecord(b->fork, st);
        forked = true;
      }
      const int j = (k - 1) % 3;
      if (e == hipSuccess && !used[j]) {
        e = hipStreamWaitEvent(b->side[j], b->fork, 0);
        used[j] = true;
      }
      s = b->side[j];
    }
    ++k;
    if (e != hipSuccess) break;
    e = with_class<Mode>(c, LaunchGroup<Mode>{dargs, items + sp.off[c], sp.cnt[c], counter + c, b->class_grid[c], s});
  }
  for (int j = 0; j < 3 && e == hipSuccess; ++j)
    if (used[j]) {
      e = hipEventRecord(b->join[j], b->side[j]);
      if (e == hipSuccess) e = hipStreamWaitEvent(st, b->join[j], 0);
    }
  return e;
}

hipError_t enqueue_batch(const aqt_batch* b, const StepArgs* dargs, const BatchItem* items, const ClassSpans& sp,
                         int* counter, hipStream_t st) {
  if (b->precision == AQT_FP64) return enqueue_mode<ModeF64>(b, dargs, items, sp, counter, st);
  if (b->precision == AQT_FP32) return enqueue_mode<ModeF32>(b, dargs, items, sp, counter, st);
  return enqueue_mode<ModeBF16>(b, dargs, items, sp, counter, st);
}

// Resident workgroups per CU of group c's kernel (0 if the group is not allowed).
template <class Mode>
int class_occupancy(int c) {
  int blocks = 0;
  const hipError_t e = with_class<Mode>(c, GroupOccupancy<Mode>{&blocks});
  return e == hipSuccess ? (blocks > 0 ? blocks : 1) : 0;
}

int class_occupancy_for(int c, int precision) {
  if (precision == AQT_FP64) return class_occupancy<ModeF64>(c);
  if (precision == AQT_FP32) return class_occupancy<ModeF32>(c);
  return class_occupancy<ModeBF16>(c);
}

bool batch_tq_ok(int NP, int tq, int precision) {
  return batch_class(NP, tq) >= 0 && batch_tq(NP, tq, precision == AQT_FP64);
}

// Items of all instances grouped by (levels, tile), largest levels first, longest first
// within a group (work per item ~ TQ * (M-1) * NP^2).
std::vector<BatchItem> build_items(const std::vector<StepArgs>& args, ClassSpans* sp) {
  std::vector<std::pair<double, BatchItem>> v[kNumClasses];
  for (int i = 0; i < static_cast<int>(args.size()); ++i) {
    const StepArgs& a = args[i];
    const double w = static_cast<double>(a.TQ) * (a.M_run - 1) * (64.0 + static_cast<double>(a.NP) * a.NP);
    const int c = batch_class(a.NP, a.TQ);
    for (int64_t t = 0; t < a.tiles; ++t) v[c].push_back({w, BatchItem{i, static_cast<int>(t)}});
  }
  std::vector<BatchItem> out;
  for (int c = 0; c < kNumClasses; ++c) {
    std::stable_sort(v[c].begin(), v[c].end(), [](const auto& x, const auto& y) { return x.first > y.first; });
    sp->off[c] = static_cast<int>(out.size());
    sp->cnt[c] = static_cast<int>(v[c].size());
    for (auto& p : v[c]) out.push_back(p.second);
  }
  return out;
}

// Time each allowed tile size per level count on a shortened anneal (outputs
// discarded) and keep the fastest per trajectory-step.
aqt_status autotune(aqt_batch* b) {
  const int tune_steps = 24;
  std::vector<int> nps;
  for (auto& a : b->hargs)
    if (std::find(nps.begin(), nps.end(), a.NP) == nps.end()) nps.push_back(a.NP);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return b->fail(AQT_EHIP, "event creation failed");
  aqt_status st = AQT_OK;
  DevBuf dargs, ditems, dctr, scratch;
  if (dctr.reserve(kNumClasses * sizeof(int)) != hipSuccess) st = b->fail(AQT_ENOMEM, "tuning allocation failed");
  for (int np : nps) {
    if (st != AQT_OK) break;
    double best_t = 1e300;
    int best_tq = 1;
    for (int tq : kTQ) {
      if (!batch_tq_ok(np, tq, b->precision)) continue;
      std::vector<StepArgs> ta;
      size_t scratch_need = 0;
      double traj_steps = 0.0;
      for (size_t i = 0; i < b->hargs.size(); ++i) {
        StepArgs a = b->hargs[i];
        if (a.NP != np) continue;
        a.TQ = tq;
        a.M_run = std::min(a.M, tune_steps + 1);
        a.tiles = (a.K + 8 * tq - 1) / (8 * tq);
        a.jump_totals = nullptr;
        a.jump_count = nullptr;
        a.jumps = nullptr;
        a.cap = 0;
        a.net_gs = nullptr;
        a.net_hist = nullptr;
        a.final_state = nullptr;
        a.pgs_sum = a.pgs_sumsq = nullptr;
        scratch_need = std::max(scratch_need, static_cast<size_t>(a.tiles) * a.M * 2 * sizeof(double));
        traj_steps += static_cast<double>(a.K) * (a.M_run - 1);
        ta.push_back(a);
      }
      if (scratch.reserve(scratch_need) != hipSuccess) {
        st = b->fail(AQT_ENOMEM, "tuning allocation failed");
        break;
      }
      for (auto& a : ta) a.partial = scratch.as<double>();   // shared scratch, contents discarded
      ClassSpans sp;
      std::vector<BatchItem> items = build_items(ta, &sp);
      if (dargs.reserve(ta.size() * sizeof(StepArgs)) != hipSuccess ||
          ditems.reserve(items.size() * sizeof(BatchItem)) != hipSuccess) {
        st = b->fail(AQT_ENOMEM, "tuning allocation failed");
        break;
      }
      (void)hipMemcpyAsync(dargs.p, ta.data(), ta.size() * sizeof(StepArgs), hipMemcpyHostToDevice, b->stream);
      (void)hipMemcpyAsync(ditems.p, items.data(), items.size() * sizeof(BatchItem), hipMemcpyHostToDevice, b->stream);
      double t_ms = 1e300;
      for (int rep = 0; rep < 2; ++rep) {
        (void)hipEventRecord(e0, b->stream);
        if (enqueue_batch(b, dargs.as<StepArgs>(), ditems.as<BatchItem>(), sp, dctr.as<int>(), b->stream) !=
            hipSuccess) {
          st = b->fail(AQT_EHIP, "tuning launch failed");
          break;
        }
        (void)hipEventRecord(e1, b->stream);
        if (hipEventSynchronize(e1) != hipSuccess) {
          st = b->fail(AQT_EHIP, "tuning run failed");
          break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (rep) t_ms = std::min(t_ms, static_cast<double>(ms));   // first repetition warms up
      }
      if (st != AQT_OK) break;
      const double per = t_ms / traj_steps;
      if (per < best_t) {
        best_t = per;
        best_tq = tq;
      }
    }
    for (size_t i = 0; i < b->hargs.size(); ++i)
      if (b->hargs[i].NP == np && b->tiles_per_inst[i] == 0) b->tiles_per_inst[i] = 8 * best_tq;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

}  // namespace
}  // namespace aqt

extern "C" {

aqt_status aqt_batch_create(aqt_batch** out, aqt_ctx* const* ctxs, int n, const aqt_run_params* params,
                            const aqt_outputs* outs, int flags) {
  using namespace aqt;
  if (!out) return AQT_EINVAL;
  *out = nullptr;
  if (!ctxs || !params || !outs || n < 1) return AQT_EINVAL;
  aqt_batch* b = new (std::nothrow) aqt_batch();
  if (!b) return AQT_ENOMEM;
  auto bail = [&](aqt_status s) {
    if (s != AQT_OK) {
      // keep the object so the caller can read the message, then destroy it
      *out = b;
      return s;
    }
    return s;
  };
  b->n = n;
  b->ctxs.assign(ctxs, ctxs + n);
  b->device = ctxs[0] ? ctxs[0]->device : 0;
  b->stream = ctxs[0] ? ctxs[0]->stream : nullptr;
  b->precision = params[0].precision;
  b->use_graph = (flags & 1) != 0;
  const bool tune = (flags & 2) != 0;
  if (hipSetDevice(b->device) != hipSuccess) return bail(b->fail(AQT_EHIP, "hipSetDevice failed"));
  if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess)
    return bail(b->fail(AQT_EHIP, "event creation failed"));
  for (int j = 0; j < 3; ++j)
    if (hipStreamCreateWithFlags(&b->side[j], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->join[j], hipEventDisableTiming) != hipSuccess)
      return bail(b->fail(AQT_EHIP, "stream creation failed"));
  for (int i = 0; i < n; ++i) {
    aqt_ctx* c = ctxs[i];
    if (!c) return bail(b->fail(AQT_EINVAL, "null context in batch"));
    if (!c->have_tables) return bail(b->fail(AQT_ESTATE, "every context needs tables before batching"));
    if (c->device != b->device) return bail(b->fail(AQT_EINVAL, "all contexts must be on one device"));
    if (params[i].precision != b->precision) return bail(b->fail(AQT_EINVAL, "one precision per batch"));
    if (params[i].n_traj < 1) return bail(b->fail(AQT_EINVAL, "n_traj must be >= 1"));
    if (params[i].record_capacity > 0 && !outs[i].jumps)
      return bail(b->fail(AQT_EINVAL, "record_capacity > 0 needs a jumps buffer"));
    if (outs[i].net_hist && outs[i].hist_hi < outs[i].hist_lo) return bail(b->fail(AQT_EINVAL, "hist_hi < hist_lo"));
    if (params[i].tile && (params[i].tile % 8 || !batch_tq_ok(c->NP, params[i].tile / 8, b->precision)))
      return bail(b->fail(AQT_EINVAL, "unsupported tile size in batch"));
    if (batch_class(c->NP, 1) < 0) return bail(b->fail(AQT_EINVAL, "unsupported level count in batch"));
    aqt_status s = check_step_decay(c, b->precision);
    if (s == AQT_OK) s = pack_for_precision(c, b->precision);
    if (s != AQT_OK) return bail(b->fail(s, c->err));
  }
  if (hipStreamSynchronize(b->stream) != hipSuccess) return bail(b->fail(AQT_EHIP, "packing failed"));
  b->tiles_per_inst.assign(n, 0);
  for (int i = 0; i < n; ++i) b->tiles_per_inst[i] = params[i].tile;
  // provisional args (TQ fixed below)
  b->hargs.resize(n);
  for (int i = 0; i < n; ++i) {
    aqt_ctx* c = ctxs[i];
    StepArgs a{};
    a.M = c->M;
    a.M_run = c->M;
    a.n = c->n;
    a.nq = c->tab_nch;   // jump channels
    a.NP = c->NP;
    a.tbeg = c->tbeg.as<double>();
    a.tlen = c->tlen.as<double>();
    a.K = params[i].n_traj;
    a.seed = params[i].seed;
    a.iid = params[i].instance_id;
    a.traj0 = params[i].traj_offset;
    a.cap = params[i].record_capacity;
    a.dlt_a = c->pk_a.p;
    a.dlt_b = c->pk_b.p;
    a.dre = c->pk_dre.p;
    a.dim = c->pk_dim.p;
    a.cinit = c->cinit.as<double>();
    a.Gamma = c->Gamma.as<double>();
    a.d64re = c->dre.as<double>();
    a.d64im = c->dim.as<double>();
    a.R = c->R.as<double>();
    a.Rcol = c->Rcol.as<double>();
    a.ehalf = c->ehalf.as<double>();
    a.zdiag = c->zdiag.as<double>();
    a.E = c->E.as<double>();
    a.gs = c->gs.as<int>();
    a.jump_totals = outs[i].jump_totals;
    a.jump_count = outs[i].jump_count;
    a.jumps = outs[i].jumps;
    a.net_gs = outs[i].net_gs;
    a.net_hist = outs[i].net_hist;
    a.hist_lo = outs[i].hist_lo;
    a.hist_hi = outs[i].hist_hi;
    a.final_state = outs[i].final_state;
    a.pgs_sum = outs[i].pgs_sum;
    a.pgs_sumsq = outs[i].pgs_sumsq;
    a.flags = c->run_flags.as<int>();
    a.TQ = 1;
    a.tiles = (a.K + 7) / 8;
    b->hargs[i] = a;
  }
  const int cus = ctxs[0]->cus > 0 ? ctxs[0]->cus : 256;
  for (int c = 0; c < kNumClasses; ++c) b->class_grid[c] = cus * class_occupancy_for(c, b->precision);
  if (tune) {
    aqt_status s = autotune(b);
    if (s != AQT_OK) return bail(s);
  }
  for (int i = 0; i < n; ++i) {
    if (b->tiles_per_inst[i] == 0) {
      // heuristic: the largest allowed tile that still gives every CU several items
      int best = 1;
      for (int tq : kTQ)
        if (batch_tq_ok(b->hargs[i].NP, tq, b->precision)) best = tq;
      b->tiles_per_inst[i] = 8 * std::min(best, 4);
    }
    StepArgs& a = b->hargs[i];
    a.TQ = b->tiles_per_inst[i] / 8;
    a.tiles = (a.K + 8 * a.TQ - 1) / (8 * a.TQ);
    aqt_ctx* c = ctxs[i];
    const size_t need = static_cast<size_t>(a.tiles) * a.M * 2 * sizeof(double);
    if (c->partial.reserve(need) != hipSuccess) return bail(b->fail(AQT_ENOMEM, "workspace allocation failed"));
    a.partial = c->partial.as<double>();
  }
  ClassSpans sp;
  std::vector<BatchItem> items = build_items(b->hargs, &sp);
  b->n_items = static_cast<int>(items.size());
  for (int c = 0; c < kNumClasses; ++c) {
    b->class_off[c] = sp.off[c];
    b->class_cnt[c] = sp.cnt[c];
  }
  if (b->dargs.reserve(n * sizeof(StepArgs)) != hipSuccess ||
      b->ditems.reserve(items.size() * sizeof(BatchItem)) != hipSuccess ||
      b->dcounter.reserve(kNumClasses * sizeof(int)) != hipSuccess)
    return bail(b->fail(AQT_ENOMEM, "batch allocation failed"));
  if (hipMemcpy(b->dargs.p, b->hargs.data(), n * sizeof(StepArgs), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->ditems.p, items.data(), items.size() * sizeof(BatchItem), hipMemcpyHostToDevice) != hipSuccess)
    return bail(b->fail(AQT_EHIP, "batch upload failed"));
  if (b->use_graph) {
    if (hipStreamCreate(&b->capture_stream) != hipSuccess) return bail(b->fail(AQT_EHIP, "stream creation failed"));
    if (hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return bail(b->fail(AQT_EHIP, "graph capture failed to start"));
    hipError_t e = enqueue_batch(b, b->dargs.as<StepArgs>(), b->ditems.as<BatchItem>(), sp, b->dcounter.as<int>(),
                                 b->capture_stream);
    int maxM = 0;
    for (auto& a : b->hargs) maxM = std::max(maxM, a.M);
    hipLaunchKernelGGL(k_reduce_batch, dim3((maxM + 255) / 256, n), dim3(256), 0, b->capture_stream,
                       b->dargs.as<StepArgs>());
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->capture_stream, &g);
    if (e != hipSuccess || e2 != hipSuccess || !g) return bail(b->fail(AQT_EHIP, "graph capture failed"));
    b->graph = g;
    if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess)
      return bail(b->fail(AQT_EHIP, "graph instantiation failed"));
  }
  *out = b;
  return AQT_OK;
}

aqt_status aqt_batch_launch(aqt_batch* b) {
  using namespace aqt;
  if (!b) return AQT_EINVAL;
  if (!b->dargs.p) return b->fail(AQT_ESTATE, "batch was not created successfully");
  if (hipSetDevice(b->device) != hipSuccess) return b->fail(AQT_EHIP, "hipSetDevice failed");
  if (b->use_graph) {
    if (hipGraphLaunch(b->exec, b->stream) != hipSuccess) return b->fail(AQT_EHIP, "graph launch failed");
    return AQT_OK;
  }
  ClassSpans sp;
  for (int c = 0; c < kNumClasses; ++c) {
    sp.off[c] = b->class_off[c];
    sp.cnt[c] = b->class_cnt[c];
  }
  if (enqueue_batch(b, b->dargs.as<StepArgs>(), b->ditems.as<BatchItem>(), sp, b->dcounter.as<int>(), b->stream) !=
      hipSuccess)
    return b->fail(AQT_EHIP, "batch launch failed");
  int maxM = 0;
  for (auto& a : b->hargs) maxM = std::max(maxM, a.M);
  hipLaunchKernelGGL(k_reduce_batch, dim3((maxM + 255) / 256, b->n), dim3(256), 0, b->stream, b->dargs.as<StepArgs>());
  if (hipGetLastError() != hipSuccess) return b->fail(AQT_EHIP, "batch reduction launch failed");
  return AQT_OK;
}

aqt_status aqt_batch_tiles(const aqt_batch* b, int32_t* tile_per_instance) {
  if (!b || !tile_per_instance) return AQT_EINVAL;
  for (int i = 0; i < b->n; ++i) tile_per_instance[i] = b->tiles_per_inst.empty() ? 0 : b->tiles_per_inst[i];
  return AQT_OK;
}

const char* aqt_batch_last_error(const aqt_batch* b) { return b ? b->err.c_str() : "null batch"; }

void aqt_batch_destroy(aqt_batch* b) {
  if (!b) return;
  (void)hipSetDevice(b->device);
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  else (void)hipDeviceSynchronize();
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
  for (int j = 0; j < 3; ++j) {
    if (b->side[j]) (void)hipStreamSynchronize(b->side[j]);
    if (b->side[j]) (void)hipStreamDestroy(b->side[j]);
    if (b->join[j]) (void)hipEventDestroy(b->join[j]);
  }
  if (b->fork) (void)hipEventDestroy(b->fork);
  delete b;
}

}  // extern "C"
