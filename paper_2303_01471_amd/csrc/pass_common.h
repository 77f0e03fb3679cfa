// Device helpers shared by the pass kernels (2-D/1-D in qhd_kernels.hip, 3-D in
// qhd_kernels_3d.hip): tiled indexing, the schedule, step limits, work shares.
#pragma once

#include <hip/hip_runtime.h>

#include "qhd_internal.h"

namespace qhd {

constexpr double kInv2Pi = 0.15915494309189533577;

__host__ __device__ constexpr int ilog2_c(int n) { return n <= 1 ? 0 : 1 + ilog2_c(n >> 1); }

// 8x8-tiled index of mesh point (x, y) on an nx-wide slab (rows y may run over
// several z slabs: row = y + ny z)
__device__ __forceinline__ long long tile_index(int x, int y, int nx) {
  return ((long long)((y >> 3) * (nx >> 3) + (x >> 3)) << 6) + ((y & 7) << 3) + (x & 7);
}

// integer frequency of FFT output index m on an axis of n points
__device__ __forceinline__ int freq(int m, int n) { return m < (n >> 1) ? m : m - n; }

// Fourth-order triple jump (Yoshida 1990): a step of length dt is three symmetric
// stages of lengths w1 dt, w0 dt, w1 dt, with w1 = 1 / (2 - 2^{1/3}) and
// w0 = 1 - 2 w1 = -2^{1/3} / (2 - 2^{1/3}).
constexpr double kYoshidaW1 = 1.3512071919596576340;
constexpr double kYoshidaW0 = -1.7024143839193152681;

// a(t), b(t) of the closed-form schedules (not kSchedTable; App. C.2.1, eq.
// nonconvex_QHD_h, constants, or the adiabatic interpolation)
__device__ __forceinline__ void sched_at_time(const InstDev& I, double t, double& a, double& b) {
  if (I.sched == kSchedConst) {
    a = I.sched_p0;
    b = I.sched_p1;
  } else if (I.sched == kSchedLinear) {
    const double g = t / I.sched_p0;
    a = 1.0 - g;
    b = g;
  } else {
    const double t3 = t * t * t;
    a = 2.0 / (I.sched_p0 + t3);
    b = 2.0 * t3;
  }
}

// Coefficients of stage j, multiplied by the stage's length in units of dt: every
// phase of a stage is then (coefficient) x dt.  Strang and the fourth-order
// composition take a and b at the stage midpoint; the printed first-order product at
// the left end of the step; TABLE schedules give them per step.  One stage per step
// except for the fourth-order scheme (stage j is stage j mod 3 of step j / 3).
// Y4 = false compiles the stage arithmetic of the fourth-order scheme out (kernels of
// shape classes without such members: fewer live registers in the hot passes).
template <bool Y4 = true>
__device__ __forceinline__ void sched_ab(const InstDev& I, long long j, double& a, double& b) {
  if (I.sched == kSchedTable) {
    // lines of finished instances still evaluate (and discard) their step: never
    // read outside the table
    const bool in = (j >= 0 && j < I.nsteps);
    a = in ? I.table[2 * j] : 0.0;
    b = in ? I.table[2 * j + 1] : 0.0;
    return;
  }
  double t, w = 1.0;
  if (Y4 && I.scheme == kSchemeYoshida4) {
    // stage counts stay below 2^31 (checked at plan creation): 32-bit division
    const int step = (int)j / 3;
    const int k = (int)j - 3 * step;
    w = k == 1 ? kYoshidaW0 : kYoshidaW1;
    const double start = k == 0 ? 0.0 : (k == 1 ? kYoshidaW1 : kYoshidaW1 + kYoshidaW0);
    t = ((double)step + start + 0.5 * w) * I.dt;
  } else {
    // symmetric scheme: step midpoint; printed first-order product: left end
    t = ((double)j + (I.scheme == kSchemeLie ? 0.0 : 0.5)) * I.dt;
  }
  sched_at_time(I, t, a, b);
  a *= w;
  b *= w;
}

// Phase of the transformed-basis factor along one axis, in turns per unit of the
// coefficient a: QHD, the kinetic term (pi dt / L^2) n^2 of frequency n (App. C.2.1);
// QAA, the transverse field -sum sigma_x of the axis' qubits, whose eigenvalue in the
// Walsh-Hadamard basis is 2 popcount(u) - bits, times dt / (2 pi).
template <int MODEL>
__device__ __forceinline__ double axis_turns(const InstDev& I, int axis, int idx, int n) {
  if constexpr (MODEL == kModelQAA) {
    const int bits = 31 - __builtin_clz(n);
    return I.dt * kInv2Pi * (double)(2 * __builtin_popcount(idx) - bits);
  } else {
    const int m = freq(idx, n);
    return I.kin_turns[axis] * (double)(m * m);
  }
}

// Potential phase of the pass that applies V in step j, in turns per unit f.
// Symmetric scheme: the leading half step of j merged with the trailing half step of
// j-1 (only the leading half on the entry step, where nothing is pending).
// First-order product: the full step dt b_j.
template <bool Y4 = true>
__device__ __forceinline__ double potential_turns(const InstDev& I, long long j, bool entry) {
  double a, b;
  sched_ab<Y4>(I, j, a, b);
  if (I.scheme == kSchemeLie) return I.dt * b * kInv2Pi;
  double beta = 0.5 * I.dt * b;
  if (!entry && j > 0) {
    double ap, bp;
    sched_ab<Y4>(I, j - 1, ap, bp);
    beta += 0.5 * I.dt * bp;
  }
  return beta * kInv2Pi;
}

// Coefficient of the half step that closes a pending state at a readout (symmetric
// scheme only: the first-order product leaves no potential factor pending).
__device__ __forceinline__ double closing_turns(const InstDev& I) {
  if (I.scheme == kSchemeLie) return 0.0;
  double a, b;
  sched_ab(I, I.steps_done - 1, a, b);
  return 0.5 * I.dt * b * kInv2Pi;
}

// Leapfrog stage j of the QAA model (the paper's integrator for its baseline QAA):
// with psi = R + i I, stage 0 of step n kicks I by -dt/2 H(t_n) R, stage 1 drifts R by
// +dt H(t_{n+1/2}) I, stage 2 kicks I by -dt/2 H(t_{n+1}) R.  Returns a, b of H at
// that time, the coefficient c and whether the stage is a kick (source R, target I).
__device__ __forceinline__ void leapfrog_stage(const InstDev& I, long long j, double& a, double& b, double& c,
                                               bool& kick) {
  const int step = (int)j / 3;
  const int k = (int)j - 3 * step;
  kick = k != 1;
  c = kick ? -0.5 * I.dt : I.dt;
  sched_at_time(I, ((double)step + 0.5 * k) * I.dt, a, b);
}

// stages instance I takes in an evolve call capped at max_steps steps (< 0: no cap)
__device__ __forceinline__ long long step_limit(const InstDev& I, long long max_steps) {
  const long long rem = I.nsteps - I.steps_done;
  const long long cap = max_steps * I.stages;
  return (max_steps < 0 || cap > rem) ? rem : cap;
}


// offset of slot q of lane t on tiled row y (x = t + q*TPL); compile-time stride
// between slots once a slot spans whole tiles
template <int NX, int TPL>
__device__ __forceinline__ long long row_slot(int t, int q, int y) {
  if constexpr (TPL % 8 == 0) {
    return ((long long)((y >> 3) * (NX >> 3) + (t >> 3)) << 6) + ((y & 7) << 3) + (t & 7) +
           (long long)q * (TPL * 8);
  } else {
    return tile_index(t + q * TPL, y, NX);
  }
}

// 8-byte values (complex FP32 or FP64) of one instance reached through a raw buffer
// resource: a wave-uniform base in scalar registers, the lane's element offset in one
// vector register and each access's wave-uniform element offset as the scalar soffset.
// A slot loop over 64-bit vector addresses holds two registers per slot from the loads
// to the stores (a 16-slot line: 32 registers); here it holds one.  Every mesh fits the
// 32-bit byte offsets (at most 2^21 points per instance).
template <typename T>
struct LaneView {
  static_assert(sizeof(T) == 8, "8-byte elements");
  __amdgpu_buffer_rsrc_t r;
  int vo;  // the lane's byte offset
  __device__ __forceinline__ LaneView(const T* base, int lane_elem)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(base), 0, 0x7fffffff, 0x00020000)), vo(lane_elem * 8) {}
  __device__ __forceinline__ T load(int elem) const {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, vo, elem * 8, 0);
    T out;
    __builtin_memcpy(&out, &v, 8);
    return out;
  }
  __device__ __forceinline__ void store(int elem, T z) const {
    __attribute__((ext_vector_type(2))) unsigned v;
    __builtin_memcpy(&v, &z, 8);
    __builtin_amdgcn_raw_buffer_store_b64(v, r, vo, elem * 8, 0);
  }
};

// contiguous share [begin, end) of `total` work items for this block, in units of `step`
__device__ __forceinline__ void block_share(long long total, int step, long long& begin, long long& end) {
  const long long units = (total + step - 1) / step;
  const long long per = (units + gridDim.x - 1) / gridDim.x;
  begin = (long long)blockIdx.x * per * step;
  end = begin + per * step;
  if (end > total) end = total;
}

}  // namespace qhd
