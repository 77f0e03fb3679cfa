// Line FFTs for the QHD split-operator passes (gfx950).
//
// The kinetic factor of the product formula is diagonal in the Fourier basis
// (App. C.2.1, eq. prod_qhd_fft; App. E.1): every pass transforms whole mesh
// lines, multiplies by a diagonal phase and transforms back.  This header holds
// the per-line transform used by every pass kernel.
//
// Design (CDNA4):
//   * A line of N points is owned by TPL = N / P lanes of ONE wavefront; lane t
//     holds the P points t + q*TPL (q = 0..P-1) in registers.  Input and output
//     of a full transform are in that same layout, so a pass loads a line
//     straight from HBM, transforms, applies its phase and transforms back
//     without any reordering.
//   * Stockham auto-sort stages of radix R = min(P, N/Ns); the butterflies and
//     all twiddle products run in FP64 registers (FP64 FMA issues at the same
//     rate as unpacked FP32 on this chip), so each twiddle product is rounded
//     once, in FP64.  Rounding FP32-stored twiddles instead biases |w| and drains
//     the norm by ~5e-8 per transform, which 10^4 steps cannot afford.
//   * Between stages the line is exchanged through LDS as FP32 complex (one
//     unbiased rounding of the data per stage), with one pad slot every 8
//     entries so that the radix-8 scatter is bank-conflict free.  A line never
//     spans two wavefronts, so the exchange needs no workgroup barrier.
//   * Twiddles are W_N^j = exp(-2 pi i j / N) from an FP64 table computed on the
//     host; each lane keeps the few it needs in registers for its whole life.
#pragma once

#include <hip/hip_runtime.h>

namespace qhd {

// ---------------------------------------------------------------------------------
// complex FP64 helpers

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 w) {
  return make_double2(fma(a.x, w.x, -a.y * w.y), fma(a.x, w.y, a.y * w.x));
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 to_d2(float2 v) { return make_double2((double)v.x, (double)v.y); }
__device__ __forceinline__ float2 to_f2(double2 v) { return make_float2((float)v.x, (float)v.y); }

// multiply by S*i (S = -1: -i z, S = +1: +i z)
template <int S>
__device__ __forceinline__ double2 mul_si(double2 z) {
  if constexpr (S < 0) return make_double2(z.y, -z.x);
  else return make_double2(-z.y, z.x);
}

// e^{S 2 pi i k / 16} for k = 0..7 (cos, sin of multiples of pi/8)
__device__ __forceinline__ constexpr double c16(int k) {
  return k == 0 ? 1.0 : k == 1 ? 0.92387953251128675613 : k == 2 ? 0.70710678118654752440
       : k == 3 ? 0.38268343236508977173 : k == 4 ? 0.0 : k == 5 ? -0.38268343236508977173
       : k == 6 ? -0.70710678118654752440 : -0.92387953251128675613;
}
__device__ __forceinline__ constexpr double s16(int k) {
  return k == 0 ? 0.0 : k == 1 ? 0.38268343236508977173 : k == 2 ? 0.70710678118654752440
       : k == 3 ? 0.92387953251128675613 : k == 4 ? 1.0 : k == 5 ? 0.92387953251128675613
       : k == 6 ? 0.70710678118654752440 : 0.38268343236508977173;
}

// z * e^{S 2 pi i k / 16}, exact for multiples of pi/2
template <int S, int K>
__device__ __forceinline__ double2 rot16(double2 z) {
  if constexpr (K == 0) return z;
  else if constexpr (K == 4) return mul_si<S>(z);
  else if constexpr (K == 2 || K == 6) {
    // c * (z.x - S z.y, S z.x + z.y) for K=2 ; c * (-z.x - S z.y, S z.x - z.y) for K=6
    constexpr double c = 0.70710678118654752440;
    if constexpr (K == 2) return make_double2(c * (z.x - S * z.y), c * (S * z.x + z.y));
    else return make_double2(c * (-z.x - S * z.y), c * (S * z.x - z.y));
  } else {
    return cmul(z, make_double2(c16(K), S * s16(K)));
  }
}

// ---------------------------------------------------------------------------------
// small DFTs on registers: X_k = sum_m x_m e^{S 2 pi i m k / R}, in place, natural order

template <int S>
__device__ __forceinline__ void dft2(double2 (&u)[2]) {
  const double2 a = u[0], b = u[1];
  u[0] = cadd(a, b);
  u[1] = csub(a, b);
}

template <int S>
__device__ __forceinline__ void dft4(double2 (&u)[4]) {
  const double2 s02 = cadd(u[0], u[2]), d02 = csub(u[0], u[2]);
  const double2 s13 = cadd(u[1], u[3]), d13 = mul_si<S>(csub(u[1], u[3]));
  u[0] = cadd(s02, s13);
  u[2] = csub(s02, s13);
  u[1] = cadd(d02, d13);
  u[3] = csub(d02, d13);
}

template <int S>
__device__ __forceinline__ void dft8(double2 (&u)[8]) {
  double2 e[4] = {u[0], u[2], u[4], u[6]};
  double2 o[4] = {u[1], u[3], u[5], u[7]};
  dft4<S>(e);
  dft4<S>(o);
  o[1] = rot16<S, 2>(o[1]);
  o[2] = rot16<S, 4>(o[2]);
  o[3] = rot16<S, 6>(o[3]);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    u[k] = cadd(e[k], o[k]);
    u[k + 4] = csub(e[k], o[k]);
  }
}

template <int S>
__device__ __forceinline__ void dft16(double2 (&u)[16]) {
  double2 e[8], o[8];
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
    u[k] = cadd(e[k], o[k]);
    u[k + 8] = csub(e[k], o[k]);
  }
}

template <int R, int S>
__device__ __forceinline__ void dft(double2 (&u)[R]) {
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
__device__ __forceinline__ constexpr int lds_slot(int i) { return i + (i >> 3); }
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
// w^r = W_{Ns R}^{(v mod Ns) r}, r = 1..R-1, stored for the forward sign.

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
};

// One Stockham stage on the lane's registers.  If LAST, results stay in the
// lane's own layout; otherwise they are scattered to LDS for the next stage.
template <int N, int P, int S, int STAGE>
__device__ __forceinline__ void fft_stage(double2 (&reg)[P], int t, const Twiddles<N, P>& tw,
                                          float2* __restrict__ lds) {
  using SP = StagePlan<N, P>;
  constexpr int NS = SP::ns(STAGE);
  constexpr int R = SP::radix(STAGE);
  constexpr int NB = P / R;
  constexpr int TPL = N / P;
  constexpr bool LAST = (STAGE == SP::count() - 1);
#pragma unroll
  for (int m = 0; m < NB; ++m) {
    double2 u[R];
#pragma unroll
    for (int r = 0; r < R; ++r) u[r] = reg[m + r * NB];
    if constexpr (STAGE > 0) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const double2 w = tw.w[STAGE - 1][m * (R - 1) + (r - 1)];
        u[r] = cmul(u[r], S < 0 ? w : cconj(w));
      }
    }
    dft<R, S>(u);
    if constexpr (LAST) {
#pragma unroll
      for (int r = 0; r < R; ++r) reg[m + r * NB] = u[r];
    } else {
      const int v = t + m * TPL;
      const int base = (v / NS) * NS * R + (v % NS);
#pragma unroll
      for (int r = 0; r < R; ++r) lds[lds_slot(base + r * NS)] = to_f2(u[r]);
    }
  }
  if constexpr (!LAST) {
    wave_lds_sync();
#pragma unroll
    for (int q = 0; q < P; ++q) reg[q] = to_d2(lds[lds_slot(t + q * TPL)]);
    wave_lds_sync();
  }
}

template <int N, int P, int S, int STAGE = 0>
__device__ __forceinline__ void line_fft_from(double2 (&reg)[P], int t, const Twiddles<N, P>& tw,
                                              float2* __restrict__ lds) {
  if constexpr (STAGE < StagePlan<N, P>::count()) {
    fft_stage<N, P, S, STAGE>(reg, t, tw, lds);
    line_fft_from<N, P, S, STAGE + 1>(reg, t, tw, lds);
  }
}

// Full unnormalised transform of one line, X_k = sum_m x_m e^{S 2 pi i m k / N}.
template <int N, int P, int S>
__device__ __forceinline__ void line_fft(double2 (&reg)[P], int t, const Twiddles<N, P>& tw,
                                         float2* __restrict__ lds) {
  line_fft_from<N, P, S, 0>(reg, t, tw, lds);
}

}  // namespace qhd
