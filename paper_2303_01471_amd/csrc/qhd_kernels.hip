// HIP kernels of the QHD split-operator engine (gfx950 / CDNA4).
//
// One symmetric step of the product formula (App. C.2.1, eqs. prod_qhd and
// prod_qhd_fft; App. E.1, Algorithm 1, taken in its symmetric form with
// midpoint coefficients) is
//
//     psi <- V_j^{1/2} F^{-1} K_j F V_j^{1/2} psi,
//     V_j^{1/2} = exp(-i (dt/2) b_j f(x)),   K_j = exp(-i dt a_j |k|^2 / 2),
//
// with a_j = a(t_{j+1/2}), b_j = b(t_{j+1/2}).  In 2-D, F = F_y F_x and the
// state between steps is kept in (k_x, y) space, so one step costs two HBM
// passes over the state:
//
//   row pass    (lines along x):  F_x . V_{j-1}^{1/2} V_j^{1/2} . F_x^{-1}
//               (the trailing half step of step j-1 merged with the leading half
//               of step j; on the first step of a clean state only V_j^{1/2} F_x)
//   column pass (lines along y):  F_y^{-1} . K_j . F_y
//
// and the observe kernel closes the pending V_{k-1}^{1/2} F_x^{-1} on a copy.
// In 1-D a single pass does V . F^{-1} K F.
//
// Memory layout in HBM (2-D): 8x8 tiles of 64 consecutive complex64 values,
// tile rows of the mesh stored one after another, so that a tile row (8 mesh
// rows) and a tile column (8 mesh columns) are both made of 512-byte contiguous
// chunks.  f is stored as FP64 in the same layout: carrying f at FP64 precision
// matters because the potential phase accumulates f * integral(b dt) (up to
// ~8e4 f at T = 20), far beyond FP32's 2^-24 relative precision.
//
// Phases: every phase argument is formed in FP64 and reduced to [-1/2, 1/2]
// turns, then evaluated in FP32 and given one Newton magnitude correction
// (w <- w (3 - |w|^2) / 2) so that phase factors do not bias the norm.  The
// kinetic factor is separable, K = E_x(k_x) E_y(k_y); E_y is computed once per
// lane, instance and step (FP64 Newton step, with the 1/(nx ny) of the inverse
// transforms folded in exactly) and E_x once per column.
#include <climits>

#include "line_fft.h"
#include "pass_common.h"
#include "qhd_internal.h"

namespace qhd {

// Line transforms of a model: the DFT for QHD (kinetic term diagonal in Fourier
// space), the Walsh-Hadamard transform for QAA (transverse field diagonal in the
// Hadamard basis; its own inverse up to 1/N).
//
// Working precision in registers.  A near-uniform state (QHD starts uniform; the QAA
// state stays close to the ground state of the transverse field) is concentrated in
// the transformed basis, and every FP32 rounding of its few large coefficients moves
// the norm by up to ~1e-7, a random walk over the steps.  The column pass is where the
// whole mesh concentrates into one coefficient: there the last stage of the forward
// transform, the diagonal factor and the first stage of the inverse run in FP64
// (line_fft_io), so those coefficients are not rounded between them.  The row pass
// concentrates each row separately (one coefficient per row) and stays FP32, which
// measured the same drift.  QAA lines need no LDS and run in FP64 throughout
// (additions and xor shuffles).

// ------------------------------------------------------------------------------------
// 2-D row pass: lines along x, one line per TPL lanes.

// 512-point QHD rows with 16 points per lane (R4): four blocks per CU, four waves per
// SIMD.  Their LDS fits four blocks (39 KB each) with one pad slot per 16 line entries
// (the radix-16 scatter of the first stage then puts a group of 16 lanes on 16 distinct
// bank pairs) and a table of first twiddle powers (the powers formed in FP64); the slot
// loads and stores go through buffer views, so 112 registers hold the line.  Measured
// against the three-wave form (eight-entry padding, full twiddle table, 64-bit slot
// addresses): 208 vs 213 us per launch on 160 x 512^2.  Other shapes keep three waves
// (512 points with 16 per lane, QAA) or the compiler's choice.
template <int NX, int P, int MODEL>
struct RowCfg {
  static constexpr bool R4 = MODEL == kModelQHD && NX == 512 && P == 16;
  static constexpr int SLOTS = R4 ? NX + NX / 16 : LineLds<NX>::kSlots;
  static constexpr int WAVES = R4 ? 4 : ((P == 16 && NX == 512) ? 3 : 1);
};
struct Slot16Ix {
  __device__ static constexpr int at(int i) { return i + (i >> 4); }
};
template <>
struct IxShift<Slot16Ix> {
  static constexpr int value = 4;
};
// a row's psi and f slots at the lane's offset (the instance is wave-uniform)
template <int NX, int TPL>
struct RowView {
  LaneView<float2> ps;
  LaneView<double> fs;
  __device__ __forceinline__ RowView(float2* psi_i, const double* f_i, int t, int y)
      : ps(psi_i, (int)row_slot<NX, TPL>(t, 0, y)), fs(f_i, (int)row_slot<NX, TPL>(t, 0, y)) {}
};

template <int NX, int P, int MODEL = kModelQHD, bool Y4 = true>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(RowCfg<NX, P, MODEL>::WAVES)))
k_row_pass_2d(const InstDev* __restrict__ inst, const int* __restrict__ nact_p,
                                                     int ny_log2, float2* __restrict__ psi,
                                                     const double* __restrict__ f,
                                                     const double2* __restrict__ twtab, int s,
                                                     long long max_steps) {
  const int ninst = *nact_p;  // members active in this sub-step (device, set per chunk)
  constexpr int TPL = NX / P;
  constexpr int LPW = 256 / TPL;
  using RC = RowCfg<NX, P, MODEL>;
  constexpr int SLOTS = RC::SLOTS;
  __shared__ float2 lds[LPW * SLOTS];
  const int ll = threadIdx.x / TPL, t = threadIdx.x % TPL;
  float2* my = lds + ll * SLOTS;
  using TW = typename std::conditional<RC::R4, TwiddlesLds<NX, P, true>, TwiddlesFor<NX, P>>::type;
  __shared__ double2 twl[RC::R4 ? TwiddlesLds<NX, P, true>::kEntries : TwLdsSize<NX, P>::value];
  TW tw;
  load_twiddles(tw, twtab, twl, t);
  const long long total = (long long)ninst << ny_log2;
  long long begin, end;
  block_share(total, LPW, begin, end);
  for (long long l0 = begin; l0 < end; l0 += LPW) {
    const long long L = l0 + ll;
    const bool valid = L < end;
    const long long Lc = valid ? L : end - 1;
    int i = (int)(Lc >> ny_log2);
    const int y = (int)(Lc & ((1 << ny_log2) - 1));
    // a wavefront's rows (64 P / NX of them, aligned) lie in one instance when they are
    // at most 8, the smallest mesh size: the index is then wave-uniform and the instance
    // record is read with scalar loads instead of a chain of waited vector loads
    if constexpr (64 * P <= 8 * NX) i = __builtin_amdgcn_readfirstlane(i);
    const InstDev& I = inst[i];
    const bool active = valid && s < step_limit(I, max_steps);
    const long long j = I.steps_done + s;
    const bool entry = (s == 0 && I.mode == kModeClean);
    const double cpot = potential_turns<Y4>(I, j, entry);
    float2* __restrict__ pl = psi + I.psi_off;
    const double* __restrict__ fl = f + I.psi_off;
    if constexpr (MODEL == kModelQAA) {
      double2 reg[P];
#pragma unroll
      for (int q = 0; q < P; ++q) assign(reg[q], pl[row_slot<NX, TPL>(t, q, y)]);
      if (!entry) line_wht<NX, P>(reg, t);
#pragma unroll
      for (int q = 0; q < P; ++q) reg[q] = cmul_fd(reg[q], phase_turns_d(cpot * fl[row_slot<NX, TPL>(t, q, y)]));
      line_wht<NX, P>(reg, t);
      if (active) {
#pragma unroll
        for (int q = 0; q < P; ++q) assign(pl[row_slot<NX, TPL>(t, q, y)], reg[q]);
      }
    } else if constexpr (NX == 128) {
      // 128-point rows: FP64 at the four ends of the two transforms and in the potential
      // factor, so that neither a state concentrated in k_x (near uniform, early) nor one
      // localised in x (late) is rounded where it is concentrated; the stages between
      // and their exchanges stay FP32.  Over the 128^2 members of the 768-instance batch
      // this cut the largest norm drift from 9.8e-6 to 5.5e-6 per 1e4 steps (median
      // 1.8e-6 to 1.3e-6) for 4 % more time in this pass.
      double2 xd[P];
      {
        double2 in[P];
#pragma unroll
        for (int q = 0; q < P; ++q) assign(in[q], pl[row_slot<NX, TPL>(t, q, y)]);
        if (!entry) {
          line_fft_io<NX, P, +1>(in, xd, t, tw, my);
        } else {
#pragma unroll
          for (int q = 0; q < P; ++q) xd[q] = in[q];
        }
      }
#pragma unroll
      for (int q = 0; q < P; ++q) xd[q] = cmul_fd(xd[q], phase_turns_d(cpot * fl[row_slot<NX, TPL>(t, q, y)]));
      double2 out[P];
      line_fft_io<NX, P, -1>(xd, out, t, tw, my);
      if (active) {
#pragma unroll
        for (int q = 0; q < P; ++q) assign(pl[row_slot<NX, TPL>(t, q, y)], out[q]);
      }
    } else if constexpr (RC::R4) {
      static_assert(64 * P <= 8 * NX && TPL % 8 == 0, "wave-uniform instance, whole-tile slot stride");
      const RowView<NX, TPL> row(pl, fl, t, y);
      float2 reg[P];
#pragma unroll
      for (int q = 0; q < P; ++q) reg[q] = row.ps.load(q * TPL * 8);
      if (!entry) line_fft<NX, P, +1, false, Slot16Ix>(reg, t, tw, my);
#pragma unroll
      for (int q = 0; q < P; ++q) reg[q] = cmul_fd(reg[q], phase_turns_d(cpot * row.fs.load(q * TPL * 8)));
      line_fft<NX, P, -1, false, Slot16Ix>(reg, t, tw, my);
      if (active) {
#pragma unroll
        for (int q = 0; q < P; ++q) row.ps.store(q * TPL * 8, reg[q]);
      }
    } else {
      float2 reg[P];
#pragma unroll
      for (int q = 0; q < P; ++q) reg[q] = pl[row_slot<NX, TPL>(t, q, y)];
      if (!entry) line_fft<NX, P, +1>(reg, t, tw, my);
#pragma unroll
      for (int q = 0; q < P; ++q) reg[q] = cmul_fd(reg[q], phase_turns_d(cpot * fl[row_slot<NX, TPL>(t, q, y)]));
      line_fft<NX, P, -1>(reg, t, tw, my);
      if (active) {
#pragma unroll
        for (int q = 0; q < P; ++q) pl[row_slot<NX, TPL>(t, q, y)] = reg[q];
      }
    }
  }
}

// ------------------------------------------------------------------------------------
// 2-D column pass: a tile column (8 mesh columns) is staged through LDS with
// 512-byte tile loads; each column is then one line of TPL lanes.

template <int NY, int P, bool WIDE = false>  // WIDE: the staged pass's one-line-per-wave form
struct ColCfg {
  static constexpr int TPL = NY / P;
  static constexpr bool EY_LDS = WIDE && NY == 512 && P == 8;           // one line per wave, E_y in LDS
  static constexpr int NT = EY_LDS ? 512 : 256;                           // threads per block
  static constexpr int ITEMS = (8 * TPL >= NT) ? 1 : NT / (8 * TPL);     // tile columns per block
  // waves per SIMD the register budget must allow: the LDS of a block (line buffers,
  // twiddle table) lets three blocks share a CU when 8 points per lane; at 512 points a
  // block of 8 waves takes one line each and keeps E_y in LDS (100 VGPRs instead of 168;
  // 128 with the next tile column held in registers), two blocks per CU: four waves per
  // SIMD (measured 9 % faster than three blocks of 4)
  static constexpr int MIN_WAVES = EY_LDS ? 4 : (P == 8 ? 3 : 1);
  static constexpr int LINES = ITEMS * 8;                                 // columns per block
  static constexpr int SUBS = (LINES * TPL) / NT;                         // column rounds per item
  // line stride in LDS slots, = 2 (mod 16) so the tile scatter hits distinct banks
  static constexpr int STRIDE = ((LineLds<NY>::kSlots + 13) / 16) * 16 + 2;
};

template <int NY, int P, int MODEL = kModelQHD, bool Y4 = true>
__global__ void __launch_bounds__((ColCfg<NY, P, true>::NT)) __attribute__((amdgpu_waves_per_eu(ColCfg<NY, P, true>::MIN_WAVES))) k_col_pass_2d(
    const InstDev* __restrict__ inst, const int* __restrict__ nact_p, int nx_log2, float2* __restrict__ psi,
    const double2* __restrict__ twtab, int s, long long max_steps) {
  const int ninst = *nact_p;  // members active in this sub-step (device, set per chunk)
  using C = ColCfg<NY, P, true>;
  constexpr int TPL = C::TPL, ITEMS = C::ITEMS, NT = C::NT, STRIDE = C::STRIDE, SUBS = C::SUBS;
  constexpr int TILES = NY / 8;
  __shared__ float2 lds[C::LINES * STRIDE];
  __shared__ double2 eyl[C::EY_LDS ? NY : 1];
  const int tid = threadIdx.x;
  const int line0 = tid / TPL, t = tid % TPL;  // first column of this lane group
  __shared__ double2 twl[TwLdsSize<NY, P>::value];
  TwiddlesFor<NY, P> tw;
  load_twiddles(tw, twtab, twl, t);
  const int nx = 1 << nx_log2, tc_log2 = nx_log2 - 3, tcols = nx >> 3;
  const long long total = (long long)ninst << tc_log2;
  const double inv_n = 1.0 / ((double)nx * (double)NY);
  long long begin, end;
  block_share(total, ITEMS, begin, end);
  double cached = -1.0;  // E_y depends on the instance only through a_j * pi dt / L_y^2
  double2 ey[P];
  // 512-point form (one item per block): the next item's tile column is loaded into
  // registers while the current one is transformed, so its HBM latency overlaps the
  // line transforms instead of standing between the block's barriers
  constexpr int PF = C::EY_LDS ? (TILES * 32) / NT : 1;  // float4 per thread and item
  float4 pf[PF];
  bool pf_live = false;
  double a_item = 0.0;  // a_j of the block's current item
  auto fetch = [&](long long g) -> bool {
    const int i = (int)(g >> tc_log2), tc = (int)(g & (tcols - 1));
    const InstDev& I = inst[i];
    if (!(s < step_limit(I, max_steps))) return false;
    const float4* __restrict__ src = reinterpret_cast<const float4*>(psi + I.psi_off) + tc * 32;
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      const int e = tid + k * NT, ty = e >> 5, w = e & 31;
      pf[k] = src[(long long)ty * tcols * 32 + w];
    }
    return true;
  };
  if constexpr (C::EY_LDS) {
    static_assert(ITEMS == 1 && (TILES * 32) % NT == 0, "one item per block, whole float4 rounds");
    if (begin < end) pf_live = fetch(begin);
  }
  for (long long g0 = begin; g0 < end; g0 += ITEMS) {
    if constexpr (C::EY_LDS) {
      // the block's item is one tile column of one instance: E_y / (nx ny) for it, read
      // after the staging barrier
      const InstDev& I = inst[(int)(g0 >> tc_log2)];
      double a, b;
      sched_ab<Y4>(I, I.steps_done + s, a, b);
      a_item = a;
      const double cy = a * (MODEL == kModelQAA ? I.dt : I.kin_turns[1]);
      if (cy != cached) {
        for (int k = tid; k < NY; k += NT) {
          double arg;
          if constexpr (MODEL == kModelQAA) {
            arg = a * axis_turns<MODEL>(I, 1, k, NY);
          } else {
            const int nyf = freq(k, NY);
            arg = cy * (double)(nyf * nyf);
          }
          const double2 e = phase_turns_d(arg);
          eyl[k] = make_double2(e.x * inv_n, e.y * inv_n);
        }
        cached = cy;
      }
    }
    if constexpr (C::EY_LDS) {
      if (pf_live) {
#pragma unroll
        for (int k = 0; k < PF; ++k) {
          const int e = tid + k * NT, ty = e >> 5, w = e & 31;
          const int y = ty * 8 + (w >> 2), xx = (w & 3) << 1;
          lds[xx * STRIDE + lds_slot(y)] = make_float2(pf[k].x, pf[k].y);
          lds[(xx + 1) * STRIDE + lds_slot(y)] = make_float2(pf[k].z, pf[k].w);
        }
      }
    } else {
      // stage the tile columns: each thread moves float4 = two complex values; the
      // item decode is wave-uniform
#pragma unroll
      for (int it = 0; it < ITEMS; ++it) {
        const long long g = g0 + it;
        if (g < end) {
          const int i = (int)(g >> tc_log2), tc = (int)(g & (tcols - 1));
          const InstDev& I = inst[i];
          if (s < step_limit(I, max_steps)) {
            const float4* __restrict__ src = reinterpret_cast<const float4*>(psi + I.psi_off) + tc * 32;
            float2* __restrict__ dst = lds + it * 8 * STRIDE;
#pragma unroll
            for (int e = tid; e < TILES * 32; e += NT) {
              const int ty = e >> 5, w = e & 31;
              const float4 v = src[(long long)ty * tcols * 32 + w];
              const int y = ty * 8 + (w >> 2), xx = (w & 3) << 1;
              dst[xx * STRIDE + lds_slot(y)] = make_float2(v.x, v.y);
              dst[(xx + 1) * STRIDE + lds_slot(y)] = make_float2(v.z, v.w);
            }
          }
        }
      }
    }
    __syncthreads();
    if constexpr (C::EY_LDS) pf_live = g0 + 1 < end && fetch(g0 + 1);
#pragma unroll
    for (int sub = 0; sub < SUBS; ++sub) {
      const int line = line0 + sub * (NT / TPL);
      float2* my = lds + line * STRIDE;
      // one item per block: a block-uniform index keeps the instance reads on the scalar
      // unit, whose waits do not wait for the prefetched tile column.  Otherwise, with at
      // least 8 lanes per line a wavefront's lines (aligned) lie in one 8-line item: the
      // item index is wave-uniform and goes through readfirstlane for the same reason.
      const int item_of_line = TPL >= 8 ? __builtin_amdgcn_readfirstlane(line / 8) : line / 8;
      const long long g = C::EY_LDS ? g0 : g0 + item_of_line;
      const long long gc = g < end ? g : end - 1;
      const int i = (int)(gc >> tc_log2), tc = (int)(gc & (tcols - 1));
      const InstDev& I = inst[i];
      const int x = tc * 8 + (line & 7);
      double a, b = 0.0;
      // a_j of the item, evaluated before the prefetch: a schedule-table read here would
      // be a vector load whose wait also waits for the prefetched loads
      if constexpr (C::EY_LDS) a = a_item;
      else sched_ab<Y4>(I, I.steps_done + s, a, b);
      const double cy = a * (MODEL == kModelQAA ? I.dt : I.kin_turns[1]);
      if (!C::EY_LDS && cy != cached) {
        // E_y / (nx ny) for this lane's slots: computed once per distinct coefficient
#pragma unroll
        for (int q = 0; q < P; ++q) {
          double arg;
          if constexpr (MODEL == kModelQAA) {
            arg = a * axis_turns<MODEL>(I, 1, t + q * TPL, NY);
          } else {
            const int nyf = freq(t + q * TPL, NY);
            arg = cy * (double)(nyf * nyf);
          }
          const double2 e = phase_turns_d(arg);
          ey[q] = make_double2(e.x * inv_n, e.y * inv_n);
        }
        cached = cy;
      }
      double xarg;
      if constexpr (MODEL == kModelQAA) {
        xarg = a * axis_turns<MODEL>(I, 0, x, nx);
      } else {
        const int nxf = freq(x, nx);
        xarg = a * I.kin_turns[0] * (double)(nxf * nxf);
      }
      const double2 ex = phase_turns_d(xarg);
      float2 reg[P];
#pragma unroll
      for (int q = 0; q < P; ++q) reg[q] = my[lds_slot(t + q * TPL)];
      wave_lds_sync();
      double2 kd[P];
      if constexpr (MODEL == kModelQAA) {
#pragma unroll
        for (int q = 0; q < P; ++q) assign(kd[q], reg[q]);
        line_wht<NY, P>(kd, t);
      } else {
        line_fft_io<NY, P, -1>(reg, kd, t, tw, my);
      }
#pragma unroll
      for (int q = 0; q < P; ++q) {
        // E_x E_y and its product with psi in FP64: a factor rounded to FP32 has a
        // one-sided magnitude error where the phase is tiny (cos rounds to 1, sin does
        // not), and that error repeats every step
        const double2 eq = C::EY_LDS ? eyl[t + q * TPL] : ey[q];
        const double2 k = make_double2(fma(ex.x, eq.x, -ex.y * eq.y), fma(ex.x, eq.y, ex.y * eq.x));
        kd[q] = cmul_fd(kd[q], k);
      }
      if constexpr (MODEL == kModelQAA) {
        line_wht<NY, P>(kd, t);
#pragma unroll
        for (int q = 0; q < P; ++q) assign(reg[q], kd[q]);
        wave_lds_sync();  // the transforms did not touch LDS
      } else {
        line_fft_io<NY, P, +1>(kd, reg, t, tw, my);
      }
#pragma unroll
      for (int q = 0; q < P; ++q) my[lds_slot(t + q * TPL)] = reg[q];
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
      const long long g = g0 + it;
      if (g < end) {
        const int i = (int)(g >> tc_log2), tc = (int)(g & (tcols - 1));
        const InstDev& I = inst[i];
        if (s < step_limit(I, max_steps)) {
          float4* __restrict__ dstg = reinterpret_cast<float4*>(psi + I.psi_off) + tc * 32;
          const float2* __restrict__ srcl = lds + it * 8 * STRIDE;
#pragma unroll
          for (int e = tid; e < TILES * 32; e += NT) {
            const int ty = e >> 5, w = e & 31;
            const int y = ty * 8 + (w >> 2), xx = (w & 3) << 1;
            const float2 p0 = srcl[xx * STRIDE + lds_slot(y)];
            const float2 p1 = srcl[(xx + 1) * STRIDE + lds_slot(y)];
            dstg[(long long)ty * tcols * 32 + w] = make_float4(p0.x, p0.y, p1.x, p1.y);
          }
        }
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------------------------
// 2-D column pass, split form (512-point columns, QHD).  A block of 8 wavefronts takes
// one tile column (8 columns x 512 rows) per item, in two lane layouts:
//   tile view   lane l of wavefront w holds column l & 7, rows t + 64 q with
//               t = (l >> 3) + 8 w: slot q of a wavefront is one whole 8x8 tile, loaded
//               from (and stored to) HBM straight into registers;
//   line view   wavefront w holds column w as one line, lane t = l with rows t + 64 q.
// The tile view runs the first forward stage and writes its outputs to the columns'
// LDS lines; after a block barrier each wavefront transforms its line (forward stages
// 1-2, the last in FP64, K = E_x E_y / (nx ny) in FP64, inverse stage 0 in FP64 and
// stage 1) with wavefront-local exchanges and writes the last stage's inputs back; after
// a second barrier the tile view runs the last inverse stage and stores.  The staged
// form's tile scatter, line read, line write and tile gather (four LDS round trips per
// point) become two.  The next item's tiles are loaded into registers while the current
// item's lines are transformed.

template <int NY>
struct ColSplitCfg {
  static constexpr int P = 8, TPL = NY / P, NT = 512;
  static constexpr int STRIDE = ColCfg<NY, P, true>::STRIDE;  // line stride in LDS slots
};

template <int NY, bool Y4>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) k_col_pass_split(
    const InstDev* __restrict__ inst, const int* __restrict__ nact_p, int nx_log2, float2* __restrict__ psi,
    const double2* __restrict__ twtab, int s, long long max_steps) {
  const int ninst = *nact_p;  // members active in this sub-step (device, set per chunk)
  using C = ColSplitCfg<NY>;
  constexpr int P = C::P, TPL = C::TPL, NT = C::NT, STRIDE = C::STRIDE;
  static_assert(TPL == 64 && StagePlan<NY, P>::count() == 3, "split form: 512-point lines, radices 8, 8, 8");
  __shared__ float2 lds[8 * STRIDE];
  __shared__ double2 eyl[NY];
  __shared__ double2 twl[TwLdsSize<NY, P>::value];
  // the wavefront index is uniform: tile offsets are then scalar and not held per lane
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int c_tv = lane & 7, t_tv = (lane >> 3) + 8 * wave;  // tile view: column, line position
  float2* my = lds + wave * STRIDE;                           // line view: this wavefront's column
  float2* mc = lds + c_tv * STRIDE;                           // tile view: this lane's column
  TwiddlesFor<NY, P> tw;
  load_twiddles(tw, twtab, twl, lane);
  TwiddlesFor<NY, P> twt = tw;  // the same table seen from the tile view's line positions
  twt.tab = twl + t_tv;
  const int nx = 1 << nx_log2, tc_log2 = nx_log2 - 3, tcols = nx >> 3;
  const long long total = (long long)ninst << tc_log2;
  const double inv_n = 1.0 / ((double)nx * (double)NY);
  long long begin, end;
  block_share(total, 1, begin, end);
  double cached = -1.0;  // E_y depends on the instance only through a_j * pi dt / L_y^2
  // tile view: slot q of the item is tile row wave + 8 q of its tile column, lane = the
  // position inside the tile
  float2 pf[P];
  auto fetch = [&](long long g) -> bool {
    const int i = (int)(g >> tc_log2), tc = (int)(g & (tcols - 1));
    const InstDev& I = inst[i];
    if (!(s < step_limit(I, max_steps))) return false;
    const LaneView<float2> src(psi + I.psi_off + tc * 64, lane);
#pragma unroll
    for (int q = 0; q < P; ++q) pf[q] = src.load((wave + 8 * q) * tcols * 64);
    return true;
  };
  bool pf_live = begin < end && fetch(begin);
  for (long long g0 = begin; g0 < end; ++g0) {
    const int i = (int)(g0 >> tc_log2), tc = (int)(g0 & (tcols - 1));
    const InstDev& I = inst[i];
    const bool active = pf_live;  // the item's instance takes this sub-step
    double a, b;
    sched_ab<Y4>(I, I.steps_done + s, a, b);
    const double cy = a * I.kin_turns[1];
    if (cy != cached) {
      // E_y / (nx ny) for the item's instance; the previous item's readers passed its
      // second barrier
      for (int k = tid; k < NY; k += NT) {
        const int nyf = freq(k, NY);
        const double2 e = phase_turns_d(cy * (double)(nyf * nyf));
        eyl[k] = make_double2(e.x * inv_n, e.y * inv_n);
      }
      cached = cy;
    }
    // tile view: forward stage 0 into the lines
    stage_outputs_to_lds<NY, P, -1, 0, float2, SlotIx>(pf, t_tv, twt, mc);
    __syncthreads();
    pf_live = g0 + 1 < end && fetch(g0 + 1);
    // line view: forward stages 1 and 2 (FP64), K, inverse stages 0 (FP64) and 1
    {
      float2 reg[P];
      stage_inputs<NY, P, SlotIx>(reg, lane, my);
      wave_lds_sync();
      fft_stage_io<NY, P, -1, 1, false, float2, SlotIx>(reg, reg, lane, tw, my);
      double2 kd[P];
      fft_stage_io<NY, P, -1, 2, false, double2, SlotIx>(reg, kd, lane, tw, my);
      const int nxf = freq(tc * 8 + wave, nx);
      const double2 ex = phase_turns_d(a * I.kin_turns[0] * (double)(nxf * nxf));
#pragma unroll
      for (int q = 0; q < P; ++q) {
        // E_x E_y and its product with psi in FP64 (a factor rounded to FP32 has a
        // one-sided magnitude error where its phase is tiny)
        const double2 eq = eyl[lane + q * TPL];
        const double2 k = make_double2(fma(ex.x, eq.x, -ex.y * eq.y), fma(ex.x, eq.y, ex.y * eq.x));
        kd[q] = cmul_fd(kd[q], k);
      }
      fft_stage_io<NY, P, +1, 0, false, double2, SlotIx>(kd, reg, lane, tw, my);
      stage_outputs_to_lds<NY, P, +1, 1, float2, SlotIx>(reg, lane, tw, my);
    }
    __syncthreads();
    // tile view: inverse stage 2, to HBM
    {
      float2 x[P];
      stage_inputs<NY, P, SlotIx>(x, t_tv, mc);
      fft_stage_io<NY, P, +1, 2, false, float2, SlotIx>(x, x, t_tv, twt, mc);
      if (active) {
        const LaneView<float2> dst(psi + I.psi_off + tc * 64, lane);
#pragma unroll
        for (int q = 0; q < P; ++q) dst.store((wave + 8 * q) * tcols * 64, x[q]);
      }
    }
    __syncthreads();  // the next item's first stage rewrites the lines
  }
}

// ------------------------------------------------------------------------------------
// 2-D column pass, tile-wave form (NY >= 64).  Lane l of wavefront w of an item
// owns column c = l & 7 of a tile column and row group t = (l >> 3) + 8 w, and
// holds the rows t + q*TPL (q = 0..P-1).  Slot q of a wavefront is then exactly
// one 8x8 tile (64 consecutive complex values, 512 bytes): loads and stores are
// fully coalesced and go straight to registers.  A column spans W = TPL/8
// wavefronts; with W > 1 the FFT exchanges use workgroup barriers.  256-point columns
// take 16 points per lane (radices 16 and 16: one exchange per transform over two
// wavefronts, instead of two exchanges over four), with E_y in an LDS table per item
// instead of 16 FP64 pairs per lane.  128-point columns take 16 points per lane too
// (radices 16 and 8, one wavefront per column): with 8 (radices 8, 8, 2) the FP32
// exchange before the FP64 last stage rounds values that each carry half of a
// concentrated column's mass, with 16 a sixteenth before it and an eighth after the
// FP64 first inverse stage, which roughly halves the norm's rounding walk while the
// state is near uniform (and no block barrier is needed).  Columns of 64 points or fewer
// keep 8 points per lane, the arithmetic of the resident steps.

template <int NY, int P>
struct ColTwCfg {
  static constexpr int TPL = NY / P;
  static constexpr int W = TPL / 8;                       // wavefronts per tile column
  static constexpr int ITEMS = W >= 4 ? 1 : 4 / W;        // tile columns per block
  static constexpr int NT = ITEMS * W * 64;
  static constexpr int STRIDE = ((LineLds<NY>::kSlots + 13) / 16) * 16 + 2;
  static constexpr bool EY_LDS = P >= 16;                 // E_y / (nx ny) per item in LDS
  // 16 points per lane: three waves per SIMD (168 VGPRs; the LDS of a block admits three)
  static constexpr int MIN_WAVES = (NT == 512) ? 2 : (P >= 16 ? 3 : 1);
  static_assert(TPL % 8 == 0, "tile-wave column pass needs TPL multiple of 8");
};

template <int NY, int P, bool Y4 = true>
__global__ void __launch_bounds__((ColTwCfg<NY, P>::NT)) __attribute__((amdgpu_waves_per_eu(ColTwCfg<NY, P>::MIN_WAVES))) k_col_pass_tw(
    const InstDev* __restrict__ inst, const int* __restrict__ nact_p, int nx_log2, float2* __restrict__ psi,
    const double2* __restrict__ twtab, int s, long long max_steps) {
  const int ninst = *nact_p;  // members active in this sub-step (device, set per chunk)
  using C = ColTwCfg<NY, P>;
  constexpr int TPL = C::TPL, W = C::W, ITEMS = C::ITEMS, STRIDE = C::STRIDE;
  __shared__ float2 lds[ITEMS * 8 * STRIDE];
  __shared__ double2 eyl[C::EY_LDS ? ITEMS * NY : 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // item within the block and wave within the item; wave-uniform, so the instance
  // record is read with scalar loads
  const int item = __builtin_amdgcn_readfirstlane(wave / W), wv = wave - item * W;
  const int c = lane & 7;
  const int t = (lane >> 3) + 8 * wv;
  float2* my = lds + (item * 8 + c) * STRIDE;
  __shared__ double2 twl[TwLdsSize<NY, P>::value];
  TwiddlesFor<NY, P> tw;
  load_twiddles(tw, twtab, twl, t);
  const int nx = 1 << nx_log2, tc_log2 = nx_log2 - 3, tcols = nx >> 3;
  const long long total = (long long)ninst << tc_log2;
  const double inv_n = 1.0 / ((double)nx * (double)NY);
  long long begin, end;
  block_share(total, ITEMS, begin, end);
  double cached = -1.0;  // E_y depends on the instance only through a_j * pi dt / L_y^2
  double2 ey[C::EY_LDS ? 1 : P];
  double cached_items[ITEMS];
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) cached_items[it] = -1.0;
  for (long long g0 = begin; g0 < end; g0 += ITEMS) {
    const long long g = g0 + item;
    const bool valid = g < end;
    const long long gc = valid ? g : end - 1;
    const int i = (int)(gc >> tc_log2), tc = (int)(gc & (tcols - 1));
    const InstDev& I = inst[i];
    const bool active = valid && s < step_limit(I, max_steps);
    double a, b;
    sched_ab<Y4>(I, I.steps_done + s, a, b);
    const double cy = a * I.kin_turns[1];
    if constexpr (C::EY_LDS) {
      // every thread evaluates the coefficient of every item of the block, so the
      // refresh decision (and its barriers) is block-uniform
      double cys[ITEMS];
      bool refresh = false;
#pragma unroll
      for (int it = 0; it < ITEMS; ++it) {
        const long long gi = g0 + it < end ? g0 + it : end - 1;
        const InstDev& Ii = inst[(int)(gi >> tc_log2)];
        double ai, bi;
        sched_ab<Y4>(Ii, Ii.steps_done + s, ai, bi);
        cys[it] = ai * Ii.kin_turns[1];
        refresh |= cys[it] != cached_items[it];
      }
      if (refresh) {
        __syncthreads();  // the previous items' readers are done
        for (int e = threadIdx.x; e < ITEMS * NY; e += C::NT) {
          const int it = e / NY, k = e - it * NY;
          double cyi = cys[0];
#pragma unroll
          for (int u = 1; u < ITEMS; ++u) cyi = it == u ? cys[u] : cyi;
          const int nyf = freq(k, NY);
          const double2 ph = phase_turns_d(cyi * (double)(nyf * nyf));
          eyl[e] = make_double2(ph.x * inv_n, ph.y * inv_n);
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) cached_items[it] = cys[it];
      }
    } else if (cy != cached) {
#pragma unroll
      for (int q = 0; q < P; ++q) {
        const int nyf = freq(t + q * TPL, NY);
        const double2 e = phase_turns_d(cy * (double)(nyf * nyf));
        ey[q] = make_double2(e.x * inv_n, e.y * inv_n);
      }
      cached = cy;
    }
    const int nxf = freq(tc * 8 + c, nx);
    const double2 ex = phase_turns_d(a * I.kin_turns[0] * (double)(nxf * nxf));
    // the item's tile column: scalar base, the lane's offset in one register, slot
    // offsets scalar (tile rows t + q TPL, W tile rows apart)
    const LaneView<float2> col(psi + I.psi_off + ((long long)tc << 6), lane + wv * tcols * 64);
    float2 reg[P];
#pragma unroll
    for (int q = 0; q < P; ++q) reg[q] = col.load(q * W * tcols * 64);
    double2 kd[P];
    line_fft_io<NY, P, -1, (W > 1)>(reg, kd, t, tw, my);
#pragma unroll
    for (int q = 0; q < P; ++q) {
      const double2 e = C::EY_LDS ? eyl[item * NY + t + q * TPL] : ey[C::EY_LDS ? 0 : q];
      const double2 k = make_double2(fma(ex.x, e.x, -ex.y * e.y), fma(ex.x, e.y, ex.y * e.x));
      kd[q] = cmul_fd(kd[q], k);
    }
    line_fft_io<NY, P, +1, (W > 1)>(kd, reg, t, tw, my);
    if (active) {
#pragma unroll
      for (int q = 0; q < P; ++q) col.store(q * W * tcols * 64, reg[q]);
    }
  }
}

// ------------------------------------------------------------------------------------
// Leapfrog stages of the QAA model (the paper's integrator for its baseline QAA).  The
// state stays in position space, R = psi.x, I = psi.y.  A stage applies
//     H v = a W^{-1} D0 W v + b f v,   D0 = d_x(u) + d_y(v), d(u) = 2 popcount(u) - bits,
// to its source component v and adds c H v to its target component, in two passes that
// use the separability of D0: the row pass stores u = a W_x^{-1} d_x W_x v + b f v into
// the class scratch buffer (same tiled layout as psi); the column pass adds
// a W_y^{-1} d_y W_y v and updates the target.  Lines in FP64.

template <int NX, int P>
__global__ void __launch_bounds__(256) k_lf_row_2d(const InstDev* __restrict__ inst, const int* __restrict__ nact_p, int ny_log2,
                                                   const float2* __restrict__ psi, const double* __restrict__ f,
                                                   float* __restrict__ scratch, int s, long long max_steps) {
  const int ninst = *nact_p;  // members active in this sub-step (device, set per chunk)
  constexpr int TPL = NX / P;
  constexpr int LPW = 256 / TPL;
  constexpr int BITS = ilog2_c(NX);
  const int ll = threadIdx.x / TPL, t = threadIdx.x % TPL;
  const long long total = (long long)ninst << ny_log2;
  long long begin, end;
  block_share(total, LPW, begin, end);
  for (long long l0 = begin; l0 < end; l0 += LPW) {
    const long long L = l0 + ll;
    const bool valid = L < end;
    const long long Lc = valid ? L : end - 1;
    int i = (int)(Lc >> ny_log2);
    const int y = (int)(Lc & ((1 << ny_log2) - 1));
    if constexpr (64 * P <= 8 * NX) i = __builtin_amdgcn_readfirstlane(i);  // as in the row pass
    const InstDev& I = inst[i];
    const bool active = valid && s < step_limit(I, max_steps);
    double a, b, c;
    bool kick;
    leapfrog_stage(I, I.steps_done + s, a, b, c, kick);
    const float2* __restrict__ pl = psi + I.psi_off;
    double v[P], h[P];
#pragma unroll
    for (int q = 0; q < P; ++q) {
      const float2 z = pl[row_slot<NX, TPL>(t, q, y)];
      v[q] = kick ? z.x : z.y;
      h[q] = v[q];
    }
    line_wht<NX, P>(h, t);
#pragma unroll
    for (int q = 0; q < P; ++q) h[q] *= (double)(2 * __builtin_popcount(t + q * TPL) - BITS);
    line_wht<NX, P>(h, t);
    if (active) {
      const double* __restrict__ fl = f + I.psi_off;
      float* __restrict__ ul = scratch + I.psi_off;
      constexpr double kInvN = 1.0 / NX;
#pragma unroll
      for (int q = 0; q < P; ++q) {
        const long long o = row_slot<NX, TPL>(t, q, y);
        ul[o] = (float)fma(a * kInvN, h[q], b * fl[o] * v[q]);
      }
    }
  }
}

template <int NY, int P>
__global__ void __launch_bounds__(256) k_lf_col_2d(const InstDev* __restrict__ inst, const int* __restrict__ nact_p, int nx_log2,
                                                   float2* __restrict__ psi, const float* __restrict__ scratch, int s,
                                                   long long max_steps) {
  const int ninst = *nact_p;  // members active in this sub-step (device, set per chunk)
  using C = ColCfg<NY, P>;
  constexpr int TPL = C::TPL, ITEMS = C::ITEMS, NT = C::NT, STRIDE = C::STRIDE, SUBS = C::SUBS;
  constexpr int TILES = NY / 8;
  constexpr int BITS = ilog2_c(NY);
  __shared__ float2 lds[C::LINES * STRIDE];
  __shared__ float ulds[C::LINES * STRIDE];
  const int tid = threadIdx.x;
  const int line0 = tid / TPL, t = tid % TPL;
  const int nx = 1 << nx_log2, tc_log2 = nx_log2 - 3, tcols = nx >> 3;
  const long long total = (long long)ninst << tc_log2;
  long long begin, end;
  block_share(total, ITEMS, begin, end);
  for (long long g0 = begin; g0 < end; g0 += ITEMS) {
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
      const long long g = g0 + it;
      if (g < end) {
        const int i = (int)(g >> tc_log2), tc = (int)(g & (tcols - 1));
        const InstDev& I = inst[i];
        if (s < step_limit(I, max_steps)) {
          const float4* __restrict__ src = reinterpret_cast<const float4*>(psi + I.psi_off) + tc * 32;
          const float4* __restrict__ srcu = reinterpret_cast<const float4*>(scratch + I.psi_off) + tc * 16;
          float2* __restrict__ dst = lds + it * 8 * STRIDE;
          float* __restrict__ dstu = ulds + it * 8 * STRIDE;
#pragma unroll
          for (int e = tid; e < TILES * 32; e += NT) {
            const int ty = e >> 5, w = e & 31;
            const float4 v = src[(long long)ty * tcols * 32 + w];
            const int y = ty * 8 + (w >> 2), xx = (w & 3) << 1;
            dst[xx * STRIDE + lds_slot(y)] = make_float2(v.x, v.y);
            dst[(xx + 1) * STRIDE + lds_slot(y)] = make_float2(v.z, v.w);
          }
#pragma unroll
          for (int e = tid; e < TILES * 16; e += NT) {
            const int ty = e >> 4, w = e & 15;
            const float4 v = srcu[(long long)ty * tcols * 16 + w];
            const int y = ty * 8 + (w >> 1), xx = (w & 1) << 2;
            dstu[xx * STRIDE + lds_slot(y)] = v.x;
            dstu[(xx + 1) * STRIDE + lds_slot(y)] = v.y;
            dstu[(xx + 2) * STRIDE + lds_slot(y)] = v.z;
            dstu[(xx + 3) * STRIDE + lds_slot(y)] = v.w;
          }
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int sub = 0; sub < SUBS; ++sub) {
      const int line = line0 + sub * (NT / TPL);
      float2* my = lds + line * STRIDE;
      const float* myu = ulds + line * STRIDE;
      // wave-uniform with at least 8 lanes per line, as in the staged column pass
      const long long g = g0 + (TPL >= 8 ? __builtin_amdgcn_readfirstlane(line / 8) : line / 8);
      const long long gc = g < end ? g : end - 1;
      const InstDev& I = inst[(int)(gc >> tc_log2)];
      double a, b, c;
      bool kick;
      leapfrog_stage(I, I.steps_done + s, a, b, c, kick);
      double h[P];
#pragma unroll
      for (int q = 0; q < P; ++q) {
        const float2 z = my[lds_slot(t + q * TPL)];
        h[q] = kick ? z.x : z.y;
      }
      line_wht<NY, P>(h, t);
#pragma unroll
      for (int q = 0; q < P; ++q) h[q] *= (double)(2 * __builtin_popcount(t + q * TPL) - BITS);
      line_wht<NY, P>(h, t);
      constexpr double kInvN = 1.0 / NY;
#pragma unroll
      for (int q = 0; q < P; ++q) {
        const int slot = lds_slot(t + q * TPL);
        const double w = fma(a * kInvN, h[q], (double)myu[slot]);
        float2 z = my[slot];
        if (kick) z.y = (float)fma(c, w, (double)z.y);
        else z.x = (float)fma(c, w, (double)z.x);
        my[slot] = z;
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
      const long long g = g0 + it;
      if (g < end) {
        const int i = (int)(g >> tc_log2), tc = (int)(g & (tcols - 1));
        const InstDev& I = inst[i];
        if (s < step_limit(I, max_steps)) {
          float4* __restrict__ dstg = reinterpret_cast<float4*>(psi + I.psi_off) + tc * 32;
          const float2* __restrict__ srcl = lds + it * 8 * STRIDE;
#pragma unroll
          for (int e = tid; e < TILES * 32; e += NT) {
            const int ty = e >> 5, w = e & 31;
            const int y = ty * 8 + (w >> 2), xx = (w & 3) << 1;
            const float2 p0 = srcl[xx * STRIDE + lds_slot(y)];
            const float2 p1 = srcl[(xx + 1) * STRIDE + lds_slot(y)];
            dstg[(long long)ty * tcols * 32 + w] = make_float4(p0.x, p0.y, p1.x, p1.y);
          }
        }
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------------------------
// 1-D pass: V (merged halves) . F . K . F^{-1}, the state stays in position space
// with the trailing half step of the last step pending.

template <int N, int P>
__global__ void __launch_bounds__(256) k_line_pass_1d(const InstDev* __restrict__ inst, const int* __restrict__ nact_p,
                                                      float2* __restrict__ psi,
                                                      const double* __restrict__ f,
                                                      const double2* __restrict__ twtab, int s,
                                                      long long max_steps) {
  const int ninst = *nact_p;  // members active in this sub-step (device, set per chunk)
  constexpr int TPL = N / P;
  constexpr int LPW = (256 / TPL) > 0 ? 256 / TPL : 1;
  constexpr int SLOTS = LineLds<N>::kSlots;
  __shared__ float2 lds[LPW * SLOTS];
  const int ll = threadIdx.x / TPL, t = threadIdx.x % TPL;
  float2* my = lds + ll * SLOTS;
  Twiddles<N, P> tw;
  tw.load(twtab, t);
  for (long long l0 = (long long)blockIdx.x * LPW; l0 < ninst; l0 += (long long)gridDim.x * LPW) {
    const long long L = l0 + ll;
    const bool valid = L < ninst;
    const int i = (int)(valid ? L : ninst - 1);
    const InstDev& I = inst[i];
    const bool active = valid && s < step_limit(I, max_steps);
    const long long j = I.steps_done + s;
    const bool entry = (s == 0 && I.mode == kModeClean);
    double a, b;
    sched_ab(I, j, a, b);
    const double cpot = potential_turns(I, j, entry);
    const double ck = a * I.kin_turns[0];
    const double inv_n = 1.0 / (double)N;
    const long long base = I.psi_off;
    float2 reg[P];
#pragma unroll
    for (int q = 0; q < P; ++q) {
      const long long p = base + t + q * TPL;
      reg[q] = cmul_fd(psi[p], phase_turns_d(cpot * f[p]));
    }
    double2 kd[P];
    line_fft_io<N, P, -1>(reg, kd, t, tw, my);
#pragma unroll
    for (int q = 0; q < P; ++q) {
      const int nf = freq(t + q * TPL, N);
      const double2 w = phase_turns_d(ck * (double)(nf * nf));
      kd[q] = cmul_fd(kd[q], make_double2(w.x * inv_n, w.y * inv_n));
    }
    line_fft_io<N, P, +1>(kd, reg, t, tw, my);
    if (active) {
#pragma unroll
      for (int q = 0; q < P; ++q) psi[base + t + q * TPL] = reg[q];
    }
  }
}

__global__ void k_chunk_plan(const InstDev* __restrict__ inst, int ninst, long long max_steps, int S,
                             int* __restrict__ nact) {
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < S; s += gridDim.x * blockDim.x) {
    int n = 0;
    for (int k = ninst - 1; k >= 0; --k) {
      if (s < step_limit(inst[k], max_steps)) {
        n = k + 1;
        break;
      }
    }
    nact[s] = n;
  }
}

__global__ void k_reset_inst(InstDev* __restrict__ inst, int ninst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ninst) return;
  inst[i].steps_done = 0;
  inst[i].mode = kModeClean;
}

__global__ void k_commit(InstDev* __restrict__ inst, int ninst, long long max_steps) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ninst) return;
  const long long lim = step_limit(inst[i], max_steps);
  if (lim > 0) {
    inst[i].steps_done += lim;
    inst[i].mode = kModePending;
  }
}

// ------------------------------------------------------------------------------------
// Observe (readouts of App. B / Algorithm 1 / main-text fig. 2)

// deterministic sum over the TPL lanes of one line (lanes are contiguous)
template <int TPL>
__device__ __forceinline__ double line_sum(double v) {
#pragma unroll
  for (int o = TPL / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ bool in_ball(int dxi, int dyi, int dzi, const InstDev& I) {
  // same FP64 operations, in the same order and without contraction, as the oracle
  const double dx = __dmul_rn((double)dxi, I.h[0]);
  const double dy = __dmul_rn((double)dyi, I.h[1]);
  const double dz = __dmul_rn((double)dzi, I.h[2]);
  return __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz)) < I.r2;
}

template <int NX, int P, int MODEL = kModelQHD>
__global__ void __launch_bounds__(256) k_observe_2d(const InstDev* __restrict__ inst, int ninst,
                                                    int ny_log2, int slab_log2,
                                                    const float2* __restrict__ psi,
                                                    const double* __restrict__ f,
                                                    const double2* __restrict__ twtab,
                                                    float2* __restrict__ out_psi,
                                                    float* __restrict__ out_rho,
                                                    double* __restrict__ partials) {
  constexpr int TPL = NX / P;
  constexpr int LPW = 256 / TPL;
  constexpr int SLOTS = LineLds<NX>::kSlots;
  __shared__ float2 lds[LPW * SLOTS];
  const int ll = threadIdx.x / TPL, t = threadIdx.x % TPL;
  float2* my = lds + ll * SLOTS;
  Twiddles<NX, P> tw;
  tw.load(twtab, t);
  const long long total = (long long)ninst << ny_log2;
  for (long long l0 = (long long)blockIdx.x * LPW; l0 < total; l0 += (long long)gridDim.x * LPW) {
    const long long L = l0 + ll;
    const bool valid = L < total;
    const long long Lc = valid ? L : total - 1;
    const int i = (int)(Lc >> ny_log2), y = (int)(Lc & ((1 << ny_log2) - 1));
    const InstDev& I = inst[i];
    // leapfrog keeps the state in position space, in step with the clock
    const bool pending = (I.mode == kModePending) && I.scheme != kSchemeLeapfrog;
    const long long base = I.psi_off;
    float2 reg[P];
#pragma unroll
    for (int q = 0; q < P; ++q) reg[q] = psi[base + tile_index(t + q * TPL, y, NX)];
    double fv[P];
#pragma unroll
    for (int q = 0; q < P; ++q) fv[q] = f[base + tile_index(t + q * TPL, y, NX)];
    if (pending) {
      // back to position space; the symmetric scheme also owes the trailing half step
      double2 in[P];
#pragma unroll
      for (int q = 0; q < P; ++q) assign(in[q], reg[q]);
      if constexpr (MODEL == kModelQAA) {
        line_wht<NX, P>(in, t);
#pragma unroll
        for (int q = 0; q < P; ++q) assign(reg[q], in[q]);
      } else {
        line_fft_io<NX, P, +1>(in, reg, t, tw, my);
      }
      if (I.scheme != kSchemeLie) {
        const double cpot = closing_turns(I);
#pragma unroll
        for (int q = 0; q < P; ++q) reg[q] = cmul_fd(reg[q], phase_turns_d(cpot * fv[q]));
      }
    }
    const long long rs = I.argmin / NX;
    const int xs = (int)(I.argmin % NX);
    const int ys = (int)(rs & ((1 << slab_log2) - 1)), zs = (int)(rs >> slab_log2);
    const int yy = y & ((1 << slab_log2) - 1), zz = y >> slab_log2;
    double sr = 0.0, sf = 0.0, sm = 0.0;
#pragma unroll
    for (int q = 0; q < P; ++q) {
      const int x = t + q * TPL;
      const float2 v = reg[q];
      const double rho = (double)v.x * v.x + (double)v.y * v.y;
      sr += rho;
      sf += fv[q] * rho;
      if (in_ball(x - xs, yy - ys, zz - zs, I)) sm += rho;
      if (valid) {
        const long long o = I.out_off + (long long)y * NX + x;
        if (out_psi) out_psi[o] = v;
        if (out_rho) out_rho[o] = (float)rho;
      }
    }
    sr = line_sum<TPL>(sr);
    sf = line_sum<TPL>(sf);
    sm = line_sum<TPL>(sm);
    if (valid && t == 0) {
      partials[3 * L + 0] = sr;
      partials[3 * L + 1] = sf;
      partials[3 * L + 2] = sm;
    }
  }
}

template <int N, int P>
__global__ void __launch_bounds__(256) k_observe_1d(const InstDev* __restrict__ inst, int ninst,
                                                    const float2* __restrict__ psi,
                                                    const double* __restrict__ f,
                                                    float2* __restrict__ out_psi,
                                                    float* __restrict__ out_rho,
                                                    double* __restrict__ partials) {
  constexpr int TPL = N / P;
  constexpr int LPW = (256 / TPL) > 0 ? 256 / TPL : 1;
  const int ll = threadIdx.x / TPL, t = threadIdx.x % TPL;
  for (long long l0 = (long long)blockIdx.x * LPW; l0 < ninst; l0 += (long long)gridDim.x * LPW) {
    const long long L = l0 + ll;
    const bool valid = L < ninst;
    const int i = (int)(valid ? L : ninst - 1);
    const InstDev& I = inst[i];
    // the symmetric scheme leaves its trailing half step pending; the first-order
    // product leaves nothing
    const bool close = I.mode == kModePending && I.scheme != kSchemeLie;
    const double cpot = close ? closing_turns(I) : 0.0;
    const int xs = (int)I.argmin;
    double sr = 0.0, sf = 0.0, sm = 0.0;
#pragma unroll
    for (int q = 0; q < P; ++q) {
      const int x = t + q * TPL;
      const long long p = I.psi_off + x;
      const double fv = f[p];
      float2 v = psi[p];
      if (close) v = cmul_fd(v, phase_turns_d(cpot * fv));
      const double rho = (double)v.x * v.x + (double)v.y * v.y;
      sr += rho;
      sf += fv * rho;
      const double dx = __dmul_rn((double)(x - xs), I.h[0]);
      if (__dmul_rn(dx, dx) < I.r2) sm += rho;
      if (valid) {
        const long long o = I.out_off + x;
        if (out_psi) out_psi[o] = v;
        if (out_rho) out_rho[o] = (float)rho;
      }
    }
    sr = line_sum<TPL>(sr);
    sf = line_sum<TPL>(sf);
    sm = line_sum<TPL>(sm);
    if (valid && t == 0) {
      partials[3 * L + 0] = sr;
      partials[3 * L + 1] = sf;
      partials[3 * L + 2] = sm;
    }
  }
}

// Fixed-order compensated sum of each instance's line partials, one block per instance:
// every thread sums a contiguous run of lines (Neumaier), then the 256 runs are combined
// pairwise in a fixed tree (sums and compensations separately), so the result does not
// depend on timing.
__device__ __forceinline__ void neumaier_add(double& s, double& comp, double v) {
  const double t = s + v;
  comp += (fabs(s) >= fabs(v)) ? ((s - t) + v) : ((v - t) + s);
  s = t;
}

__global__ void __launch_bounds__(256) k_finalize(const double* __restrict__ partials, int lines, int ninst,
                                                  double* __restrict__ results) {
  __shared__ double ss[3][256], sc[3][256];
  const int i = blockIdx.x;
  const int per = (lines + 255) / 256;
  const int l0 = threadIdx.x * per, l1 = l0 + per < lines ? l0 + per : lines;
  double s[3] = {0.0, 0.0, 0.0}, comp[3] = {0.0, 0.0, 0.0};
  for (int l = l0; l < l1; ++l) {
    const double* pl = partials + 3 * ((long long)i * lines + l);
#pragma unroll
    for (int c = 0; c < 3; ++c) neumaier_add(s[c], comp[c], pl[c]);
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    ss[c][threadIdx.x] = s[c];
    sc[c][threadIdx.x] = comp[c];
  }
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double a = ss[c][threadIdx.x], ca = sc[c][threadIdx.x] + sc[c][threadIdx.x + o];
        neumaier_add(a, ca, ss[c][threadIdx.x + o]);
        ss[c][threadIdx.x] = a;
        sc[c][threadIdx.x] = ca;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 3) results[3 * i + threadIdx.x] = ss[threadIdx.x][0] + sc[threadIdx.x][0];
}

// ------------------------------------------------------------------------------------
// uploads

__global__ void k_import_f_2d(const double* __restrict__ user, double* __restrict__ dst, int nx,
                              int ny) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (long long)nx * ny) return;
  const int x = (int)(p % nx), y = (int)(p / nx);
  dst[tile_index(x, y, nx)] = user[p];
}

__global__ void k_import_psi_2d(const float2* __restrict__ user, float2* __restrict__ dst, int nx,
                                int ny) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (long long)nx * ny) return;
  const int x = (int)(p % nx), y = (int)(p / nx);
  dst[tile_index(x, y, nx)] = user[p];
}

__global__ void k_copy_f(const double* __restrict__ src, double* __restrict__ dst, long long n) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) dst[p] = src[p];
}

__global__ void k_copy_psi(const float2* __restrict__ src, float2* __restrict__ dst, long long n) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) dst[p] = src[p];
}

__global__ void k_fill(float2* __restrict__ dst, long long n, float v) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) dst[p] = make_float2(v, 0.0f);
}

// lowest-index minimiser; also counts non-finite entries.  Stage 1: every block reduces a
// contiguous share of f to (value, index, non-finite count); stage 2: one block reduces
// the blocks' partials.  Ties go to the lower index in both stages, so the result is the
// lowest-index minimiser whatever the block count.
__device__ __forceinline__ void argmin_merge(double& v, long long& i, double v2, long long i2) {
  if (v2 < v || (v2 == v && i2 < i)) {
    v = v2;
    i = i2;
  }
}

template <int NT>
__device__ __forceinline__ void argmin_block(double bv, long long bi, long long bad, double* sv, long long* si,
                                             long long* sbad) {
  sv[threadIdx.x] = bv;
  si[threadIdx.x] = bi;
  sbad[threadIdx.x] = bad;
  __syncthreads();
  for (int o = NT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      double v = sv[threadIdx.x];
      long long id = si[threadIdx.x];
      argmin_merge(v, id, sv[threadIdx.x + o], si[threadIdx.x + o]);
      sv[threadIdx.x] = v;
      si[threadIdx.x] = id;
      sbad[threadIdx.x] += sbad[threadIdx.x + o];
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) k_argmin_partial(const double* __restrict__ f, long long n,
                                                        double* __restrict__ part_val,
                                                        long long* __restrict__ part_idx,
                                                        long long* __restrict__ part_bad) {
  __shared__ double sv[256];
  __shared__ long long si[256], sbad[256];
  const long long per = (n + gridDim.x - 1) / gridDim.x;
  const long long b0 = (long long)blockIdx.x * per, b1 = b0 + per < n ? b0 + per : n;
  double bv = INFINITY;
  long long bi = LLONG_MAX, bad = 0;
  for (long long p = b0 + threadIdx.x; p < b1; p += 256) {
    const double v = f[p];
    if (!isfinite(v)) {
      ++bad;
      continue;
    }
    argmin_merge(bv, bi, v, p);
  }
  argmin_block<256>(bv, bi, bad, sv, si, sbad);
  if (threadIdx.x == 0) {
    part_val[blockIdx.x] = sv[0];
    part_idx[blockIdx.x] = si[0];
    part_bad[blockIdx.x] = sbad[0];
  }
}

__global__ void __launch_bounds__(kArgminBlocks) k_argmin_final(const double* __restrict__ part_val,
                                                                const long long* __restrict__ part_idx,
                                                                const long long* __restrict__ part_bad,
                                                                double* __restrict__ out_val,
                                                                long long* __restrict__ out_idx) {
  __shared__ double sv[kArgminBlocks];
  __shared__ long long si[kArgminBlocks], sbad[kArgminBlocks];
  argmin_block<kArgminBlocks>(part_val[threadIdx.x], part_idx[threadIdx.x], part_bad[threadIdx.x], sv, si, sbad);
  if (threadIdx.x == 0) {
    out_val[0] = sv[0];
    out_idx[0] = si[0];
    out_idx[1] = sbad[0];
  }
}

// ------------------------------------------------------------------------------------
// launchers

namespace {

template <int N>
constexpr int pts_per_lane() { return N >= 1024 ? 16 : 8; }

inline int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

inline int blocks_for(long long items, int per_block, int cap) {
  long long b = (items + per_block - 1) / per_block;
  if (cap > 0 && b > cap) b = cap;
  return (int)(b < 1 ? 1 : b);
}

#define QHD_SWITCH_N(n, BODY)                 \
  switch (n) {                                \
    case 8: { constexpr int N_ = 8; BODY; }     \
    case 16: { constexpr int N_ = 16; BODY; }   \
    case 32: { constexpr int N_ = 32; BODY; }   \
    case 64: { constexpr int N_ = 64; BODY; }   \
    case 128: { constexpr int N_ = 128; BODY; } \
    case 256: { constexpr int N_ = 256; BODY; } \
    case 512: { constexpr int N_ = 512; BODY; } \
    case 1024: { constexpr int N_ = 1024; BODY; } \
    default: return hipErrorInvalidValue;     \
  }

}  // namespace

int row_points_resolve(int nx, int points_per_lane) {
  if (nx >= 1024) return 16;
  if (points_per_lane == 16 && (nx == 256 || nx == 512)) return 16;
  return 8;
}

int pass_blocks_row_2d(int nx, int ny, int ninst, int grid_cap, int points_per_lane) {
  const int P = row_points_resolve(nx, points_per_lane);
  const int lpw = 256 / (nx / P);
  return blocks_for((long long)ninst * ny, lpw, grid_cap);
}

template <int N>
constexpr int col_tw_p() { return (N >= 1024 || N == 256 || N == 128) ? 16 : 8; }

template <int N, bool Y4>
hipError_t launch_col_tw(int blocks, int nx, const InstDev* inst, int ninst, const int* nact, float2* psi,
                         const double2* tw, int s, long long max_steps, hipStream_t stream) {
  if constexpr (N >= 64 && N <= 1024) {
    constexpr int P_ = col_tw_p<N>();
    QHD_LAUNCH((k_col_pass_tw<N, P_, Y4>), dim3(blocks), dim3(ColTwCfg<N, P_>::NT), 0, stream,
                       inst, nact, ilog2(nx), psi, tw, s, max_steps);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

int col_variant_resolve(int ny, int variant) {
  const bool tw_ok = ny >= 64 && ny <= 1024;
  if (variant == kColTileWave && tw_ok) return kColTileWave;
  if (variant == kColStaged16 && (ny == 256 || ny == 512)) return kColStaged16;
  if (variant == kColSplit && ny == 512) return kColSplit;
  if (variant == kColStaged) return kColStaged;
  // measured defaults (the split form: 62 vs 66-72 us for the staged one on 48 x 512^2)
  return (ny >= 64 && ny <= 256) ? kColTileWave : (ny == 512 ? kColSplit : kColStaged);
}

int pass_blocks_col_2d(int nx, int ny, int ninst, int grid_cap, int variant) {
  int items;
  const int v = col_variant_resolve(ny, variant);
  if (v == kColTileWave) {
    const int P = (ny >= 1024 || ny == 256 || ny == 128) ? 16 : 8;  // col_tw_p<N>() for every tile-wave size
    const int w = ny / P / 8;
    items = w >= 4 ? 1 : 4 / w;
  } else if (v == kColStaged16) {
    const int tpl = ny / 16;
    items = (8 * tpl >= 256) ? 1 : 256 / (8 * tpl);
  } else if (v == kColSplit) {
    items = 1;
  } else {
    const int tpl = ny / 8;
    items = (8 * tpl >= 256) ? 1 : 256 / (8 * tpl);
  }
  return blocks_for((long long)ninst * (nx / 8), items, grid_cap);
}

template <bool Y4>
hipError_t row_pass_qhd(int nx, int ny, const InstDev* inst, int ninst, const int* nact, float2* psi, const double* f,
                        const double2* tw, int s, long long max_steps, int grid_cap, int points_per_lane,
                        hipStream_t stream) {
  const int blocks = pass_blocks_row_2d(nx, ny, ninst, grid_cap, points_per_lane);
  if (row_points_resolve(nx, points_per_lane) == 16 && nx < 1024) {
    if (nx == 256)
      QHD_LAUNCH((k_row_pass_2d<256, 16, kModelQHD, Y4>), dim3(blocks), dim3(256), 0, stream, inst, nact,
                         ilog2(ny), psi, f, tw, s, max_steps);
    else
      QHD_LAUNCH((k_row_pass_2d<512, 16, kModelQHD, Y4>), dim3(blocks), dim3(256), 0, stream, inst, nact,
                         ilog2(ny), psi, f, tw, s, max_steps);
    return hipGetLastError();
  }
  QHD_SWITCH_N(nx, {
    constexpr int P_ = pts_per_lane<N_>();
    QHD_LAUNCH((k_row_pass_2d<N_, P_, kModelQHD, Y4>), dim3(blocks), dim3(256), 0, stream, inst, nact,
                       ilog2(ny), psi, f, tw, s, max_steps);
    return hipGetLastError();
  });
}

hipError_t launch_row_pass_2d(int nx, int ny, const InstDev* inst, int ninst, const int* nact, float2* psi,
                              const double* f, const double2* tw, int s, long long max_steps,
                              int grid_cap, int points_per_lane, hipStream_t stream, int model, bool y4) {
  if (model == kModelQAA) {  // the QAA model runs the symmetric scheme or leapfrog
    const int blocks = pass_blocks_row_2d(nx, ny, ninst, grid_cap, 8);
    QHD_SWITCH_N(nx, {
      constexpr int P_ = pts_per_lane<N_>();
      QHD_LAUNCH((k_row_pass_2d<N_, P_, kModelQAA, false>), dim3(blocks), dim3(256), 0, stream, inst, nact,
                         ilog2(ny), psi, f, tw, s, max_steps);
      return hipGetLastError();
    });
  }
  return y4 ? row_pass_qhd<true>(nx, ny, inst, ninst, nact, psi, f, tw, s, max_steps, grid_cap, points_per_lane, stream)
            : row_pass_qhd<false>(nx, ny, inst, ninst, nact, psi, f, tw, s, max_steps, grid_cap, points_per_lane, stream);
}

template <bool Y4>
hipError_t col_pass_qhd(int nx, int ny, const InstDev* inst, int ninst, const int* nact, float2* psi, const double2* tw, int s,
                        long long max_steps, int grid_cap, int variant, hipStream_t stream) {
  const int blocks = pass_blocks_col_2d(nx, ny, ninst, grid_cap, variant);
  const int v = col_variant_resolve(ny, variant);
  if (v == kColTileWave) {
    QHD_SWITCH_N(ny, { return (launch_col_tw<N_, Y4>)(blocks, nx, inst, ninst, nact, psi, tw, s, max_steps, stream); });
  }
  if (v == kColSplit) {
    QHD_LAUNCH((k_col_pass_split<512, Y4>), dim3(blocks), dim3(ColSplitCfg<512>::NT), 0, stream, inst, nact,
                       ilog2(nx), psi, tw, s, max_steps);
    return hipGetLastError();
  }
  if (v == kColStaged16) {
    if (ny == 256)
      QHD_LAUNCH((k_col_pass_2d<256, 16, kModelQHD, Y4>), dim3(blocks), dim3(ColCfg<256, 16, true>::NT), 0, stream,
                         inst, nact, ilog2(nx), psi, tw, s, max_steps);
    else
      QHD_LAUNCH((k_col_pass_2d<512, 16, kModelQHD, Y4>), dim3(blocks), dim3(ColCfg<512, 16, true>::NT), 0, stream,
                         inst, nact, ilog2(nx), psi, tw, s, max_steps);
    return hipGetLastError();
  }
  QHD_SWITCH_N(ny, {
    constexpr int P_ = pts_per_lane<N_>();
    QHD_LAUNCH((k_col_pass_2d<N_, P_, kModelQHD, Y4>), dim3(blocks), dim3(ColCfg<N_, P_, true>::NT), 0, stream,
                       inst, nact, ilog2(nx), psi, tw, s, max_steps);
    return hipGetLastError();
  });
}

hipError_t launch_col_pass_2d(int nx, int ny, const InstDev* inst, int ninst, const int* nact, float2* psi,
                              const double2* tw, int s, long long max_steps, int grid_cap,
                              int variant, hipStream_t stream, int model, bool y4) {
  if (model == kModelQAA) {  // staged form only: the Walsh-Hadamard lines use in-wave shuffles
    const int blocks = pass_blocks_col_2d(nx, ny, ninst, grid_cap, kColStaged);
    QHD_SWITCH_N(ny, {
      constexpr int P_ = pts_per_lane<N_>();
      QHD_LAUNCH((k_col_pass_2d<N_, P_, kModelQAA, false>), dim3(blocks), dim3(ColCfg<N_, P_, true>::NT), 0,
                         stream, inst, nact, ilog2(nx), psi, tw, s, max_steps);
      return hipGetLastError();
    });
  }
  return y4 ? col_pass_qhd<true>(nx, ny, inst, ninst, nact, psi, tw, s, max_steps, grid_cap, variant, stream)
            : col_pass_qhd<false>(nx, ny, inst, ninst, nact, psi, tw, s, max_steps, grid_cap, variant, stream);
}

hipError_t launch_lf_row_2d(int nx, int ny, const InstDev* inst, int ninst, const int* nact, const float2* psi, const double* f,
                            float* scratch, int s, long long max_steps, int grid_cap, hipStream_t stream) {
  const int blocks = pass_blocks_row_2d(nx, ny, ninst, grid_cap, 8);
  QHD_SWITCH_N(nx, {
    constexpr int P_ = pts_per_lane<N_>();
    QHD_LAUNCH((k_lf_row_2d<N_, P_>), dim3(blocks), dim3(256), 0, stream, inst, nact, ilog2(ny), psi, f,
                       scratch, s, max_steps);
    return hipGetLastError();
  });
}

hipError_t launch_lf_col_2d(int nx, int ny, const InstDev* inst, int ninst, const int* nact, float2* psi, const float* scratch, int s,
                            long long max_steps, int grid_cap, hipStream_t stream) {
  const int blocks = pass_blocks_col_2d(nx, ny, ninst, grid_cap, kColStaged);
  QHD_SWITCH_N(ny, {
    constexpr int P_ = pts_per_lane<N_>();
    QHD_LAUNCH((k_lf_col_2d<N_, P_>), dim3(blocks), dim3(ColCfg<N_, P_>::NT), 0, stream, inst, nact,
                       ilog2(nx), psi, scratch, s, max_steps);
    return hipGetLastError();
  });
}

hipError_t launch_line_pass_1d(int n, const InstDev* inst, int ninst, const int* nact, float2* psi, const double* f,
                               const double2* tw, int s, long long max_steps, int grid_cap,
                               hipStream_t stream) {
  QHD_SWITCH_N(n, {
    constexpr int P_ = pts_per_lane<N_>();
    constexpr int TPL_ = N_ / P_;
    constexpr int LPW_ = (256 / TPL_) > 0 ? 256 / TPL_ : 1;
    const int blocks = blocks_for(ninst, LPW_, grid_cap);
    QHD_LAUNCH((k_line_pass_1d<N_, P_>), dim3(blocks), dim3(256), 0, stream, inst, nact,
                       psi, f, tw, s, max_steps);
    return hipGetLastError();
  });
}

hipError_t launch_commit(InstDev* inst, int ninst, long long max_steps, hipStream_t stream) {
  QHD_LAUNCH(k_commit, dim3((ninst + 255) / 256), dim3(256), 0, stream, inst, ninst,
                     max_steps);
  return hipGetLastError();
}

hipError_t launch_chunk_plan(const InstDev* inst, int ninst, long long max_steps, int S, int* nact,
                             hipStream_t stream) {
  if (S <= 0) return hipSuccess;
  QHD_LAUNCH(k_chunk_plan, dim3((S + 255) / 256), dim3(256), 0, stream, inst, ninst, max_steps, S, nact);
  return hipGetLastError();
}

hipError_t launch_reset_inst(InstDev* inst, int ninst, hipStream_t stream) {
  QHD_LAUNCH(k_reset_inst, dim3((ninst + 255) / 256), dim3(256), 0, stream, inst, ninst);
  return hipGetLastError();
}

hipError_t launch_observe_2d(int nx, int rows, int ny, const InstDev* inst, int ninst,
                             const float2* psi, const double* f, const double2* tw,
                             float2* out_psi, float* out_rho, double* partials,
                             hipStream_t stream, int model) {
  QHD_SWITCH_N(nx, {
    constexpr int P_ = pts_per_lane<N_>();
    constexpr int LPW_ = 256 / (N_ / P_);
    const int blocks = blocks_for((long long)ninst * rows, LPW_, 4096);
    if (model == kModelQAA)
      QHD_LAUNCH((k_observe_2d<N_, P_, kModelQAA>), dim3(blocks), dim3(256), 0, stream, inst, ninst,
                         ilog2(rows), ilog2(ny), psi, f, tw, out_psi, out_rho, partials);
    else
      QHD_LAUNCH((k_observe_2d<N_, P_>), dim3(blocks), dim3(256), 0, stream, inst, ninst,
                         ilog2(rows), ilog2(ny), psi, f, tw, out_psi, out_rho, partials);
    return hipGetLastError();
  });
}

hipError_t launch_observe_1d(int n, const InstDev* inst, int ninst, const float2* psi,
                             const double* f, float2* out_psi, float* out_rho, double* partials,
                             hipStream_t stream) {
  QHD_SWITCH_N(n, {
    constexpr int P_ = pts_per_lane<N_>();
    constexpr int TPL_ = N_ / P_;
    constexpr int LPW_ = (256 / TPL_) > 0 ? 256 / TPL_ : 1;
    const int blocks = blocks_for(ninst, LPW_, 4096);
    QHD_LAUNCH((k_observe_1d<N_, P_>), dim3(blocks), dim3(256), 0, stream, inst, ninst,
                       psi, f, out_psi, out_rho, partials);
    return hipGetLastError();
  });
}

hipError_t launch_finalize(const double* partials, int lines_per_inst, int ninst, double* results,
                           hipStream_t stream) {
  QHD_LAUNCH(k_finalize, dim3(ninst), dim3(256), 0, stream, partials, lines_per_inst, ninst, results);
  return hipGetLastError();
}

hipError_t launch_import_f(int ndim, int nx, int ny, const double* user, double* dst,
                           hipStream_t stream) {
  const long long n = (long long)nx * ny;
  const int blocks = (int)((n + 255) / 256);
  if (ndim == 2)
    QHD_LAUNCH(k_import_f_2d, dim3(blocks), dim3(256), 0, stream, user, dst, nx, ny);
  else
    QHD_LAUNCH(k_copy_f, dim3(blocks), dim3(256), 0, stream, user, dst, n);
  return hipGetLastError();
}

hipError_t launch_import_psi(int ndim, int nx, int ny, const float2* user, float2* dst,
                             hipStream_t stream) {
  const long long n = (long long)nx * ny;
  const int blocks = (int)((n + 255) / 256);
  if (ndim == 2)
    QHD_LAUNCH(k_import_psi_2d, dim3(blocks), dim3(256), 0, stream, user, dst, nx, ny);
  else
    QHD_LAUNCH(k_copy_psi, dim3(blocks), dim3(256), 0, stream, user, dst, n);
  return hipGetLastError();
}

hipError_t launch_fill_psi(float2* dst, long long count, float value, hipStream_t stream) {
  const int blocks = (int)((count + 255) / 256);
  QHD_LAUNCH(k_fill, dim3(blocks), dim3(256), 0, stream, dst, count, value);
  return hipGetLastError();
}

hipError_t launch_argmin(const double* f, long long count, double* out_val, long long* out_idx, double* part_val,
                         long long* part_idx, long long* part_bad, hipStream_t stream) {
  QHD_LAUNCH(k_argmin_partial, dim3(kArgminBlocks), dim3(256), 0, stream, f, count, part_val, part_idx,
                     part_bad);
  QHD_LAUNCH(k_argmin_final, dim3(1), dim3(kArgminBlocks), 0, stream, part_val, part_idx, part_bad, out_val,
                     out_idx);
  return hipGetLastError();
}

}  // namespace qhd
