// Line FFTs for the QHD split-operator passes (gfx950).
//
// The kinetic factor of the product formula is diagonal in the Fourier basis
// (App. C.2.1, eq. prod_qhd_fft; App. E.1): every pass transforms whole mesh
// lines, multiplies by a diagonal phase and transforms back.  This header holds
// the per-line transform used by every pass kernel and the phase helpers.
//
// Design (CDNA4):
//   * A line of N points is owned by TPL = N / P lanes of ONE wavefront; lane t
//     holds the P points t + q*TPL (q = 0..P-1) in registers.  Input and output
//     of a full transform are in that same layout, so a pass loads a line
//     straight from HBM, transforms, applies its phase and transforms back
//     without any reordering.
//   * Stockham auto-sort stages of radix R = min(P, N/Ns).  Data and butterfly
//     additions are FP32.  Every product by an irrational constant is formed so
//     that the constant carries more than FP32 precision: inter-stage twiddles
//     are FP64 (the FP32 value is widened, multiplied in FP64 and rounded once),
//     and the radix-8/16 internal constants are FP32 hi+lo pairs.  A twiddle
//     rounded to FP32 has |w| != 1 by a fixed amount; used on every transform it
//     drains the norm by ~5e-8 per transform, which 10^4 steps cannot afford.
//   * Between stages the line is exchanged through LDS in FP32 with one pad slot
//     every 8 entries (the radix-8 scatter then hits distinct banks).  A line
//     never spans two wavefronts, so the exchange needs no workgroup barrier.
//   * Twiddles W_N^j = exp(-2 pi i j / N) come from an FP64 table computed on
//     the host; each lane keeps the few it needs in registers.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace qhd {

// ---------------------------------------------------------------------------------
// complex FP32 helpers

__device__ __forceinline__ float2 fadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 fsub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 fadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 fsub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

// z * w with z in FP32 and w in FP64: one rounding per component
__device__ __forceinline__ float2 cmul_fd(float2 z, double2 w) {
  const double zr = (double)z.x, zi = (double)z.y;
  return make_float2((float)fma(zr, w.x, -zi * w.y), (float)fma(zr, w.y, zi * w.x));
}
// both in FP64
__device__ __forceinline__ double2 cmul_fd(double2 z, double2 w) {
  return make_double2(fma(z.x, w.x, -z.y * w.y), fma(z.x, w.y, z.y * w.x));
}
__device__ __forceinline__ float2 cmul_fd_conj(float2 z, double2 w) {
  const double zr = (double)z.x, zi = (double)z.y;
  return make_float2((float)fma(zr, w.x, zi * w.y), (float)fma(zi, w.x, -zr * w.y));
}
__device__ __forceinline__ double2 cmul_fd_conj(double2 z, double2 w) {
  return make_double2(fma(z.x, w.x, z.y * w.y), fma(z.y, w.x, -z.x * w.y));
}

// conversions between the FP32 storage type and a line's working type
__device__ __forceinline__ void assign(float2& d, float2 v) { d = v; }
__device__ __forceinline__ void assign(double2& d, float2 v) { d = make_double2(v.x, v.y); }
__device__ __forceinline__ void assign(float2& d, double2 v) { d = make_float2((float)v.x, (float)v.y); }
__device__ __forceinline__ void assign(double2& d, double2 v) { d = v; }

// multiply by S*i (S = -1: -i z, S = +1: +i z), exact
template <int S, typename W>
__device__ __forceinline__ W mul_si(W z) {
  W r;
  if constexpr (S < 0) {
    r.x = z.y;
    r.y = -z.x;
  } else {
    r.x = -z.y;
    r.y = z.x;
  }
  return r;
}

// cos, sin of k pi / 8 as FP64, and their FP32 hi+lo splits
__host__ __device__ constexpr double c16d(int k) {
  return k == 0 ? 1.0 : k == 1 ? 0.92387953251128675613 : k == 2 ? 0.70710678118654752440
       : k == 3 ? 0.38268343236508977173 : k == 4 ? 0.0 : k == 5 ? -0.38268343236508977173
       : k == 6 ? -0.70710678118654752440 : -0.92387953251128675613;
}
__host__ __device__ constexpr double s16d(int k) {
  return k == 0 ? 0.0 : k == 1 ? 0.38268343236508977173 : k == 2 ? 0.70710678118654752440
       : k == 3 ? 0.92387953251128675613 : k == 4 ? 1.0 : k == 5 ? 0.92387953251128675613
       : k == 6 ? 0.70710678118654752440 : 0.38268343236508977173;
}
__host__ __device__ constexpr float hi32(double v) { return (float)v; }
__host__ __device__ constexpr float lo32(double v) { return (float)(v - (double)(float)v); }

// z * e^{S 2 pi i K / 16}: exact for multiples of pi/2; otherwise an FP32 product
// with a hi+lo constant (the small cross terms first, the large ones last)
template <int S, int K, typename W>
__device__ __forceinline__ W rot16(W z) {
  if constexpr (K == 0) {
    return z;
  } else if constexpr (K == 4) {
    return mul_si<S>(z);
  } else if constexpr (std::is_same<W, double2>::value) {
    // FP64 working type: the constant itself carries enough precision
    constexpr double c = c16d(K), sn = S * s16d(K);
    return make_double2(fma(z.x, c, -z.y * sn), fma(z.x, sn, z.y * c));
  } else if constexpr (K == 2 || K == 6) {
    // (1/sqrt2) (z.x - S z.y, S z.x + z.y) for K=2 ; (1/sqrt2)(-z.x - S z.y, S z.x - z.y) for K=6
    constexpr float ch = hi32(0.70710678118654752440), cl = lo32(0.70710678118654752440);
    const float u = (K == 2) ? (S < 0 ? z.x + z.y : z.x - z.y) : (S < 0 ? z.y - z.x : -z.x - z.y);
    const float v = (K == 2) ? (S < 0 ? z.y - z.x : z.x + z.y) : (S < 0 ? -z.x - z.y : z.x - z.y);
    return make_float2(fmaf(u, ch, u * cl), fmaf(v, ch, v * cl));
  } else {
    constexpr float crh = hi32(c16d(K)), crl = lo32(c16d(K));
    constexpr float cih = hi32(S * s16d(K)), cil = lo32(S * s16d(K));
    const float re = fmaf(z.x, crh, fmaf(-z.y, cih, fmaf(z.x, crl, -z.y * cil)));
    const float im = fmaf(z.x, cih, fmaf(z.y, crh, fmaf(z.x, cil, z.y * crl)));
    return make_float2(re, im);
  }
}

// ---------------------------------------------------------------------------------
// small DFTs on registers: X_k = sum_m x_m e^{S 2 pi i m k / R}, in place, natural order

template <int S, typename W>
__device__ __forceinline__ void dft2(W (&u)[2]) {
  const W a = u[0], b = u[1];
  u[0] = fadd(a, b);
  u[1] = fsub(a, b);
}

template <int S, typename W>
__device__ __forceinline__ void dft4(W (&u)[4]) {
  const W s02 = fadd(u[0], u[2]), d02 = fsub(u[0], u[2]);
  const W s13 = fadd(u[1], u[3]), d13 = mul_si<S>(fsub(u[1], u[3]));
  u[0] = fadd(s02, s13);
  u[2] = fsub(s02, s13);
  u[1] = fadd(d02, d13);
  u[3] = fsub(d02, d13);
}

template <int S, typename W>
__device__ __forceinline__ void dft8(W (&u)[8]) {
  W e[4] = {u[0], u[2], u[4], u[6]};
  W o[4] = {u[1], u[3], u[5], u[7]};
  dft4<S>(e);
  dft4<S>(o);
  o[1] = rot16<S, 2>(o[1]);
  o[2] = rot16<S, 4>(o[2]);
  o[3] = rot16<S, 6>(o[3]);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    u[k] = fadd(e[k], o[k]);
    u[k + 4] = fsub(e[k], o[k]);
  }
}

template <int S, typename W>
__device__ __forceinline__ void dft16(W (&u)[16]) {
  W e[8], o[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    e[k] = u[2 * k];
    o[k] = u[2 * k + 1];
  }
  dft8<S>(e);
  dft8<S>(o);
  o[1] = rot16<S, 1>(o[1]);
  o[2] = rot16<S, 2>(o[2]);
  o[3] = rot16<S, 3>(o[3]);
  o[4] = rot16<S, 4>(o[4]);
  o[5] = rot16<S, 5>(o[5]);
  o[6] = rot16<S, 6>(o[6]);
  o[7] = rot16<S, 7>(o[7]);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    u[k] = fadd(e[k], o[k]);
    u[k + 8] = fsub(e[k], o[k]);
  }
}

template <int R, int S, typename W>
__device__ __forceinline__ void dft(W (&u)[R]) {
  if constexpr (R == 2) dft2<S>(u);
  else if constexpr (R == 4) dft4<S>(u);
  else if constexpr (R == 8) dft8<S>(u);
  else if constexpr (R == 16) dft16<S>(u);
  else static_assert(R == 2, "unsupported radix");
}

// ---------------------------------------------------------------------------------
// stage plan: stage s has radix R_s = min(P, N / Ns_s), Ns_0 = 1, Ns_{s+1} = Ns_s R_s

__host__ __device__ constexpr int cmin(int a, int b) { return a < b ? a : b; }

template <int N, int P>
struct StagePlan {
  static constexpr int count() {
    int c = 0;
    for (int ns = 1; ns < N; ns *= cmin(P, N / ns)) ++c;
    return c;
  }
  static constexpr int ns(int s) {
    int v = 1;
    for (int i = 0; i < s; ++i) v *= cmin(P, N / v);
    return v;
  }
  static constexpr int radix(int s) { return cmin(P, N / ns(s)); }
};

// LDS slot of line position i: one pad entry after every 8
__host__ __device__ constexpr int lds_slot(int i) { return i + (i >> 3); }

// Where a line keeps position i of its LDS exchange buffer, relative to the line's base
// pointer: the padded contiguous layout (default), or a fixed stride (a column of a
// row-major array in LDS, exchanged in place).
struct SlotIx {
  __device__ static constexpr int at(int i) { return lds_slot(i); }
};
template <int STRIDE>
struct StrideIx {
  __device__ static constexpr int at(int i) { return i * STRIDE; }
};
// Placements of the form at(i) = i + (i >> S) (one pad slot per 2^S entries) or
// linear (S = 0) split over a sum, at(a + b) = at(a) + at(b), whenever b is a multiple
// of 2^S (no carry out of the low S bits).  An exchange access t + q TPL (or base +
// r NS) is then one per-lane address plus a compile-time offset instead of an address
// register per slot.
template <typename IX>
struct IxShift {
  static constexpr int value = -1;  // no such split
};
template <>
struct IxShift<SlotIx> {
  static constexpr int value = 3;
};
template <int STRIDE>
struct IxShift<StrideIx<STRIDE>> {
  static constexpr int value = 0;
};
template <typename IX, int K>
__host__ __device__ constexpr bool ix_splits() {
  return IxShift<IX>::value >= 0 && K % (1 << (IxShift<IX>::value < 0 ? 0 : IxShift<IX>::value)) == 0;
}
// the P slots t + q TPL of a lane
template <int N, int P, typename IX, typename T, typename V>
__device__ __forceinline__ void lds_read_slots(V (&dst)[P], int t, const T* __restrict__ lds) {
  constexpr int TPL = N / P;
  if constexpr (ix_splits<IX, TPL>()) {
    const T* __restrict__ b = lds + IX::at(t);
#pragma unroll
    for (int q = 0; q < P; ++q) assign(dst[q], b[IX::at(q * TPL)]);
  } else {
#pragma unroll
    for (int q = 0; q < P; ++q) assign(dst[q], lds[IX::at(t + q * TPL)]);
  }
}
// the R Stockham outputs base + r NS of one butterfly (base = a multiple of R when NS = 1)
template <int R, int NS, typename IX, typename T, typename V>
__device__ __forceinline__ void lds_write_outputs(T* __restrict__ lds, int base, const V (&u)[R]) {
  if constexpr (ix_splits<IX, NS>() || (NS == 1 && ix_splits<IX, R>())) {
    T* __restrict__ b = lds + IX::at(base);
#pragma unroll
    for (int r = 0; r < R; ++r) assign(b[IX::at(r * NS)], u[r]);
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r) assign(lds[IX::at(base + r * NS)], u[r]);
  }
}

template <int N>
struct LineLds {
  static constexpr int kSlots = N + N / 8;
};

// wavefront-local ordering of LDS accesses (a line never spans two waves)
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------------
// per-lane twiddle cache: for each stage s >= 1 and butterfly m of the lane,
// w^r = W_{Ns R}^{(v mod Ns) r}, r = 1..R-1, stored (FP64) for the forward sign.

template <int N, int P>
struct Twiddles {
  using SP = StagePlan<N, P>;
  static constexpr int kStages = SP::count();
  static constexpr int kTPL = N / P;
  double2 w[kStages > 1 ? kStages - 1 : 1][P];

  template <int STAGE>
  __device__ __forceinline__ void load_stage(const double2* __restrict__ tab, int t) {
    if constexpr (STAGE < kStages) {
      constexpr int NS = SP::ns(STAGE), R = SP::radix(STAGE);
      constexpr int NB = P / R, STEP = N / (NS * R);
#pragma unroll
      for (int m = 0; m < NB; ++m) {
        const int k = (t + m * kTPL) % NS;
#pragma unroll
        for (int r = 1; r < R; ++r) w[STAGE - 1][m * (R - 1) + (r - 1)] = tab[(k * r * STEP) & (N - 1)];
      }
      load_stage<STAGE + 1>(tab, t);
    }
  }

  __device__ __forceinline__ void load(const double2* __restrict__ tab, int t) { load_stage<1>(tab, t); }

  template <int STAGE>
  __device__ __forceinline__ double2 get(int j) const { return w[STAGE - 1][j]; }
};

// The same twiddles read from LDS, laid out in lane order: for every stage s >= 1 and
// butterfly m there are rows of TPL entries, entry t holding lane t's twiddle.  A lane
// keeps only its base address; each read is one ds_read_b128 with an immediate offset,
// and consecutive lanes read consecutive entries (no bank conflicts).
//   POW = false: one row per power r = 1..R-1, the values of Twiddles (bitwise equal
//                results);
//   POW = true:  one row of first powers w^1 = W_{Ns R}^{(v mod Ns)}; the powers r >= 2
//                are formed by FP64 products (w^r = w^{r-1} w^1, relative error below
//                1e-14 for r <= 15, far below the FP32 rounding of the product with the
//                data).  Fewer LDS reads for more FP64 arithmetic and registers: measured
//                faster for 128-, 512- (8 points per lane) and 1024-point lines, slower
//                for 256-point lines and where the register budget is tight (512 points
//                with 16 per lane spill the chain of powers).
template <int N, int P, bool POW>
struct TwiddlesLds {
  using SP = StagePlan<N, P>;
  static constexpr int kStages = SP::count();
  static constexpr int kTPL = N / P;
  static constexpr bool kPow = POW;
  // rows of stage s: NB first powers, or NB (R - 1) powers
  static constexpr int rows_of(int st) { return (P / SP::radix(st)) * (POW ? 1 : SP::radix(st) - 1); }
  static constexpr int rows_before(int st) {
    int c = 0;
    for (int q = 1; q < st; ++q) c += rows_of(q);
    return c;
  }
  static constexpr int kRows = rows_before(kStages);
  static constexpr int kEntries = kRows > 0 ? kRows * kTPL : 1;
  const double2* tab;  // this lane's column of the table

  // rows of stage ST: row (m, r) holds lane tt's W^{k r STEP}, k = (tt + m TPL) mod NS
  // (r = 1 only when POW)
  template <int ST>
  __device__ __forceinline__ static void fill_stage(const double2* __restrict__ g, double2* lds_tab) {
    if constexpr (ST < kStages) {
      constexpr int NS = SP::ns(ST), R = SP::radix(ST), STEP = N / (NS * R);
      constexpr int RPM = POW ? 1 : R - 1;  // rows per butterfly
      constexpr int BASE = rows_before(ST);
      for (int e = threadIdx.x; e < rows_of(ST) * kTPL; e += blockDim.x) {
        const int j = e / kTPL, tt = e % kTPL;  // powers of two: shifts and masks
        const int m = j / RPM, r = j - m * RPM + 1;
        const int k = (tt + m * kTPL) % NS;
        lds_tab[BASE * kTPL + e] = g[(k * r * STEP) & (N - 1)];
      }
      fill_stage<ST + 1>(g, lds_tab);
    }
  }

  // lds_tab: kEntries entries of LDS, filled from the global table W_N^j by the whole
  // block (ends with a block barrier: call it where every thread of the block arrives)
  __device__ __forceinline__ void load(const double2* __restrict__ global_tab, double2* lds_tab, int t) {
    fill_stage<1>(global_tab, lds_tab);
    __syncthreads();
    tab = lds_tab + t;
  }

  // row j of stage STAGE: power (j mod RPM) + 1 of butterfly j / RPM
  template <int STAGE>
  __device__ __forceinline__ double2 get(int j) const { return tab[(rows_before(STAGE) + j) * kTPL]; }
};

// w * v with both in FP64 (twiddle powers)
__device__ __forceinline__ double2 cmul_dd(double2 w, double2 v) {
  return make_double2(fma(w.x, v.x, -w.y * v.y), fma(w.x, v.y, w.y * v.x));
}

// Twiddles w^r = W^{k r STEP}, r = 1..R-1, of one butterfly group from its first power
// (TwiddlesLds with POW): applied to u[1..R-1] while the next power is formed.
template <typename TW>
struct TwPowers : std::false_type {};
template <int N, int P>
struct TwPowers<TwiddlesLds<N, P, true>> : std::true_type {};

template <int S, int STAGE, int R, typename W, typename TW>
__device__ __forceinline__ void apply_twiddle_powers(W (&u)[R], const TW& tw, int m) {
  const double2 w1 = tw.template get<STAGE>(m);
  double2 wr = w1;
#pragma unroll
  for (int r = 1; r < R; ++r) {
    u[r] = S < 0 ? cmul_fd(u[r], wr) : cmul_fd_conj(u[r], wr);
    if (r + 1 < R) wr = cmul_dd(wr, w1);
  }
}

// One Stockham stage on the lane's registers.  If LAST, results stay in the
// lane's own layout; otherwise they are scattered to LDS for the next stage.
// BLOCK_SYNC: the lanes of one line span several wavefronts of the block, so the
// exchange needs a workgroup barrier instead of a wavefront-local one.
template <bool BLOCK_SYNC>
__device__ __forceinline__ void line_lds_sync() {
  if constexpr (BLOCK_SYNC) __syncthreads();
  else wave_lds_sync();
}

template <int N, int P, int S, int STAGE, bool BLOCK_SYNC = false, typename IX = SlotIx, typename TW>
__device__ __forceinline__ void fft_stage(float2 (&reg)[P], int t, const TW& tw, float2* __restrict__ lds) {
  using SP = StagePlan<N, P>;
  constexpr int NS = SP::ns(STAGE);
  constexpr int R = SP::radix(STAGE);
  constexpr int NB = P / R;
  constexpr int TPL = N / P;
  constexpr bool LAST = (STAGE == SP::count() - 1);
#pragma unroll
  for (int m = 0; m < NB; ++m) {
    float2 u[R];
#pragma unroll
    for (int r = 0; r < R; ++r) u[r] = reg[m + r * NB];
    if constexpr (STAGE > 0) {
      if constexpr (TwPowers<TW>::value) {
        apply_twiddle_powers<S, STAGE>(u, tw, m);
      } else {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const double2 w = tw.template get<STAGE>(m * (R - 1) + (r - 1));
          u[r] = S < 0 ? cmul_fd(u[r], w) : cmul_fd_conj(u[r], w);
        }
      }
    }
    dft<R, S>(u);
    if constexpr (LAST) {
#pragma unroll
      for (int r = 0; r < R; ++r) reg[m + r * NB] = u[r];
    } else {
      const int v = t + m * TPL;
      const int base = (v / NS) * NS * R + (v % NS);
      lds_write_outputs<R, NS, IX>(lds, base, u);
    }
  }
  if constexpr (!LAST) {
    line_lds_sync<BLOCK_SYNC>();
    lds_read_slots<N, P, IX>(reg, t, lds);
    line_lds_sync<BLOCK_SYNC>();
  }
}

template <int N, int P, int S, bool BLOCK_SYNC, int STAGE = 0, typename IX = SlotIx, typename TW>
__device__ __forceinline__ void line_fft_from(float2 (&reg)[P], int t, const TW& tw, float2* __restrict__ lds) {
  if constexpr (STAGE < StagePlan<N, P>::count()) {
    fft_stage<N, P, S, STAGE, BLOCK_SYNC, IX>(reg, t, tw, lds);
    line_fft_from<N, P, S, BLOCK_SYNC, STAGE + 1, IX>(reg, t, tw, lds);
  }
}

// Full unnormalised transform of one line, X_k = sum_m x_m e^{S 2 pi i m k / N};
// TW is Twiddles<N, P> or TwiddlesLds<N, P>; IX places the exchange buffer's positions.
template <int N, int P, int S, bool BLOCK_SYNC = false, typename IX = SlotIx, typename TW>
__device__ __forceinline__ void line_fft(float2 (&reg)[P], int t, const TW& tw, float2* __restrict__ lds) {
  line_fft_from<N, P, S, BLOCK_SYNC, 0, IX>(reg, t, tw, lds);
}

// ---------------------------------------------------------------------------------
// Mixed-precision form: the first stage computes in the type of the input array and
// the last stage in the type of the output array; the stages between, and every LDS
// exchange, are FP32.  A transform of a near-uniform line concentrates its mass into
// a few coefficients in the last stage (and an inverse transform starts from them in
// the first), where every FP32 rounding moves the norm by up to ~1e-7 of the whole
// line; with those two stages in FP64 (and the diagonal factor between two transforms
// applied in FP64 too) the concentrated values are rounded once, when they are
// stored.  The FP64 stages need no widening around their twiddle products.  (On
// gfx950 FP64 arithmetic and FP32<->FP64 conversions issue at half the unpacked FP32
// rate, measured 37 vs 74 T lane-operations/s; the passes are not issue-bound, and
// twiddle products moved to FP32 hi+lo pairs were measured to gain nothing at 512^2
// and 1-2 % at 128^2 / 256^2.)

template <int N, int P, int S, int STAGE, bool BLOCK_SYNC, typename W, typename IX, typename A, typename B,
          typename TW>
__device__ __forceinline__ void fft_stage_io(const A (&src)[P], B (&dst)[P], int t, const TW& tw,
                                             float2* __restrict__ lds) {
  using SP = StagePlan<N, P>;
  constexpr int NS = SP::ns(STAGE);
  constexpr int R = SP::radix(STAGE);
  constexpr int NB = P / R;
  constexpr int TPL = N / P;
  constexpr bool LAST = (STAGE == SP::count() - 1);
  static_assert(LAST || std::is_same<B, float2>::value, "an exchanged stage writes FP32");
#pragma unroll
  for (int m = 0; m < NB; ++m) {
    W u[R];
#pragma unroll
    for (int r = 0; r < R; ++r) assign(u[r], src[m + r * NB]);
    if constexpr (STAGE > 0) {
      if constexpr (TwPowers<TW>::value) {
        apply_twiddle_powers<S, STAGE>(u, tw, m);
      } else {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const double2 w = tw.template get<STAGE>(m * (R - 1) + (r - 1));
          u[r] = S < 0 ? cmul_fd(u[r], w) : cmul_fd_conj(u[r], w);
        }
      }
    }
    dft<R, S>(u);
    if constexpr (LAST) {
#pragma unroll
      for (int r = 0; r < R; ++r) assign(dst[m + r * NB], u[r]);
    } else {
      const int v = t + m * TPL;
      const int base = (v / NS) * NS * R + (v % NS);
      lds_write_outputs<R, NS, IX>(lds, base, u);
    }
  }
  if constexpr (!LAST) {
    line_lds_sync<BLOCK_SYNC>();
    lds_read_slots<N, P, IX>(dst, t, lds);
    line_lds_sync<BLOCK_SYNC>();
  }
}

// The compute-and-write half of an exchanged stage: stage STAGE of the lane's values
// (working type W) written to its LDS line at the Stockham output positions, with no
// synchronisation and no read-back.  The caller synchronises (a workgroup barrier when
// other lanes read the line next) and reads the next stage's inputs with
// stage_inputs(); fft_stage_io is these two halves with wavefront-local syncs.
template <int N, int P, int S, int STAGE, typename W, typename IX, typename A, typename TW>
__device__ __forceinline__ void stage_outputs_to_lds(const A (&src)[P], int t, const TW& tw, float2* __restrict__ lds) {
  using SP = StagePlan<N, P>;
  constexpr int NS = SP::ns(STAGE);
  constexpr int R = SP::radix(STAGE);
  constexpr int NB = P / R;
  constexpr int TPL = N / P;
  static_assert(STAGE < SP::count() - 1, "the last stage keeps its results in registers");
#pragma unroll
  for (int m = 0; m < NB; ++m) {
    W u[R];
#pragma unroll
    for (int r = 0; r < R; ++r) assign(u[r], src[m + r * NB]);
    if constexpr (STAGE > 0) {
      if constexpr (TwPowers<TW>::value) {
        apply_twiddle_powers<S, STAGE>(u, tw, m);
      } else {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const double2 w = tw.template get<STAGE>(m * (R - 1) + (r - 1));
          u[r] = S < 0 ? cmul_fd(u[r], w) : cmul_fd_conj(u[r], w);
        }
      }
    }
    dft<R, S>(u);
    const int v = t + m * TPL;
    const int base = (v / NS) * NS * R + (v % NS);
    lds_write_outputs<R, NS, IX>(lds, base, u);
  }
}

// the inputs of the next stage, positions t + q TPL of the LDS line
template <int N, int P, typename IX>
__device__ __forceinline__ void stage_inputs(float2 (&dst)[P], int t, const float2* __restrict__ lds) {
  lds_read_slots<N, P, IX>(dst, t, lds);
}

template <int N, int P, int S, bool BLOCK_SYNC, int STAGE, typename IX, typename TW>
__device__ __forceinline__ void fft_mid_stages(float2 (&reg)[P], int t, const TW& tw, float2* __restrict__ lds) {
  if constexpr (STAGE < StagePlan<N, P>::count() - 1) {
    fft_stage_io<N, P, S, STAGE, BLOCK_SYNC, float2, IX>(reg, reg, t, tw, lds);
    fft_mid_stages<N, P, S, BLOCK_SYNC, STAGE + 1, IX>(reg, t, tw, lds);
  }
}

// Full unnormalised transform of one line from `in` (float2 or double2) to `out`
// (float2 or double2), same layout as line_fft.
template <int N, int P, int S, bool BLOCK_SYNC = false, typename IX = SlotIx, typename TIN, typename TOUT,
          typename TW>
__device__ __forceinline__ void line_fft_io(TIN (&in)[P], TOUT (&out)[P], int t, const TW& tw,
                                            float2* __restrict__ lds) {
  constexpr int C = StagePlan<N, P>::count();
  if constexpr (C == 1) {
    using W = typename std::conditional<std::is_same<TIN, double2>::value || std::is_same<TOUT, double2>::value,
                                        double2, float2>::type;
    fft_stage_io<N, P, S, 0, BLOCK_SYNC, W, IX>(in, out, t, tw, lds);
  } else {
    float2 mid[P];
    fft_stage_io<N, P, S, 0, BLOCK_SYNC, TIN, IX>(in, mid, t, tw, lds);
    fft_mid_stages<N, P, S, BLOCK_SYNC, 1, IX>(mid, t, tw, lds);
    fft_stage_io<N, P, S, C - 1, BLOCK_SYNC, TOUT, IX>(mid, out, t, tw, lds);
  }
}

// Twiddle storage per line length: an LDS table for the long lines (register
// pressure), per-lane registers for the short ones.
template <int N, int P>
struct TwPow {
  static constexpr bool value = N != 256 && !(N == 512 && P == 16);
};
template <int N, int P>
using TwiddlesFor =
    typename std::conditional<(N >= 128), TwiddlesLds<N, P, TwPow<N, P>::value>, Twiddles<N, P>>::type;

template <int N, int P>
struct TwLdsSize {
  static constexpr int value = N >= 128 ? TwiddlesLds<N, P, TwPow<N, P>::value>::kEntries : 1;
};

// load either kind (the LDS kind needs its table slot and a block-uniform call site)
template <int N, int P>
__device__ __forceinline__ void load_twiddles(Twiddles<N, P>& tw, const double2* __restrict__ g, double2*, int t) {
  tw.load(g, t);
}
template <int N, int P, bool POW>
__device__ __forceinline__ void load_twiddles(TwiddlesLds<N, P, POW>& tw, const double2* __restrict__ g, double2* l,
                                              int t) {
  tw.load(g, l, t);
}

// ---------------------------------------------------------------------------------
// Walsh-Hadamard transform of one line (unnormalised, natural order):
// X_u = sum_i (-1)^{popcount(u & i)} x_i.  Point i = t + q TPL: the bits of q are
// combined in registers, the bits of t across the line's TPL consecutive lanes (a line
// never spans two wavefronts, and its first lane is a multiple of TPL).  Additions
// only: exact up to one rounding per butterfly.
//
// Lane exchanges (partner lane ^ H) without LDS where the pattern allows: H = 1, 2 are
// DPP quad permutations, H = 8 a DPP rotation by 8 within a row of 16 lanes, H = 4 and
// 16 ds_swizzle in bitmask mode (no LDS memory access); H = 32 a permute through LDS.
template <int H>
__device__ __forceinline__ int lane_xor(int v) {
  if constexpr (H == 1) return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true);   // quad_perm [1,0,3,2]
  else if constexpr (H == 2) return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true);  // quad_perm [2,3,0,1]
  else if constexpr (H == 8) return __builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, true);  // row_ror:8
  else if constexpr (H == 4 || H == 16) return __builtin_amdgcn_ds_swizzle(v, 0x1F | (H << 10));
  else return __shfl_xor(v, H);
}

template <int H>
__device__ __forceinline__ double lane_xor(double v) {
  const long long u = __double_as_longlong(v);
  const int lo = lane_xor<H>((int)(u & 0xffffffffLL)), hi = lane_xor<H>((int)(u >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int H>
__device__ __forceinline__ double2 lane_xor(double2 v) {
  return make_double2(lane_xor<H>(v.x), lane_xor<H>(v.y));
}

template <int H>
__device__ __forceinline__ float2 lane_xor(float2 v) {
  return make_float2(__int_as_float(lane_xor<H>(__float_as_int(v.x))), __int_as_float(lane_xor<H>(__float_as_int(v.y))));
}

__device__ __forceinline__ double wadd(double a, double b) { return a + b; }
__device__ __forceinline__ double wsub(double a, double b) { return a - b; }
template <typename T>
__device__ __forceinline__ T wadd(T a, T b) { return fadd(a, b); }
template <typename T>
__device__ __forceinline__ T wsub(T a, T b) { return fsub(a, b); }

// butterflies over the lane bits H, 2H, ... < TPL
template <int H, int TPL, int P, typename T>
__device__ __forceinline__ void wht_lanes(T (&reg)[P], int t) {
  if constexpr (H < TPL) {
    const bool upper = (t & H) != 0;
#pragma unroll
    for (int q = 0; q < P; ++q) {
      const T o = lane_xor<H>(reg[q]);
      reg[q] = upper ? wsub(o, reg[q]) : wadd(reg[q], o);
    }
    wht_lanes<2 * H, TPL, P>(reg, t);
  }
}

// T: double (a real line), float2 or double2 (a complex line)
template <int N, int P, typename T>
__device__ __forceinline__ void line_wht(T (&reg)[P], int t) {
#pragma unroll
  for (int h = 1; h < P; h <<= 1) {
#pragma unroll
    for (int q = 0; q < P; ++q) {
      if (!(q & h)) {
        const T a = reg[q], b = reg[q | h];
        reg[q] = wadd(a, b);
        reg[q | h] = wsub(a, b);
      }
    }
  }
  wht_lanes<1, N / P, P>(reg, t);
}

// ---------------------------------------------------------------------------------
// unit phase factors

// sin(2 pi r), cos(2 pi r) for |r| <= 1/2 (turns).
//   kHwSinCos: the CDNA transcendental unit (v_sin_f32 / v_cos_f32 take turns;
//   measured max error 1.2e-7 on [-1/2, 1/2]).
//   otherwise: exact reduction to the octant |y| <= 1/8 (r - q/4 is exact by
//   Sterbenz), then polynomials in y fitted (weighted least squares, Chebyshev
//   nodes) to sin(2 pi y) and cos(2 pi y); max error ~1.5 ulp of 1.
#ifndef QHD_HW_SINCOS
#define QHD_HW_SINCOS 1
#endif
__device__ __forceinline__ void sincos_turns(float r, float& s, float& c) {
#if QHD_HW_SINCOS
  s = __builtin_amdgcn_sinf(r);
  c = __builtin_amdgcn_cosf(r);
#else
  const float q = rintf(4.0f * r);
  const float y = fmaf(-0.25f, q, r);
  const float y2 = y * y;
  float ps = fmaf(y2, -75.240064049398f, 81.58812463672584f);
  ps = fmaf(ps, y2, -41.34162804267381f);
  ps = fmaf(ps, y2, 6.283185220341756f);
  const float sn = ps * y;
  float pc = fmaf(y2, 59.220407261791806f, -85.44285212009325f);
  pc = fmaf(pc, y2, 64.93931620843469f);
  pc = fmaf(pc, y2, -19.73920865035785f);
  const float cn = fmaf(pc, y2, 0.9999999999526002f);
  const int qi = (int)q;
  const bool swap = qi & 1;
  float so = swap ? cn : sn, co = swap ? sn : cn;
  so = (qi & 2) ? -so : so;
  co = ((qi + 1) & 2) ? -co : co;
  s = so;
  c = co;
#endif
}

// exp(-2 pi i tau), tau in turns (FP64), with one Newton magnitude step
// w <- w (3 - |w|^2) / 2 taken in FP64, so |w| = 1 to ~1e-14.  (In FP32 the
// step is one-sided: 1 + 2^-25 is not representable, so magnitudes just below
// 1 would never be corrected and the norm would shrink step after step.)
__device__ __forceinline__ double2 phase_turns_d(double tau) {
  const float r = (float)(tau - rint(tau));
  float s, c;
  sincos_turns(r, s, c);
  const double cd = (double)c, sd = (double)s;
  const double m = fma(cd, cd, sd * sd);
  const double g = fma(-0.5, m, 1.5);
  return make_double2(cd * g, -sd * g);
}

}  // namespace qhd
