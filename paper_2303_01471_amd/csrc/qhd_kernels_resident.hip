// Resident 2-D QHD steps (gfx950): one workgroup owns an instance of at most 128 x 128
// points for a whole evolve call.
//
// The product formula's step (App. C.2.1, eq. prod_qhd_fft; App. E.1, Algorithm 1 in its
// symmetric form with midpoint coefficients) is the same as in the streaming passes:
// a row phase F_x . V_{j-1}^{1/2} V_j^{1/2} . F_x^{-1} and a column phase
// F_y^{-1} . K_j . F_y, with the state kept in (k_x, y) space between steps.  Here the
// state stays in LDS across all the steps of the call: it is read from HBM once at
// the start (8x8-tiled layout), every step runs out of LDS, and it is written back
// once at the end, so a step moves no HBM bytes for psi (f, FP64, is re-read every
// step and stays in L2 / the last-level cache).  Small instances, whose streaming
// passes are bound by launch latency, run at the speed of one CU.
//
// LDS layout: row-major, point (x, y) at y * RS + slot(x), slot(x) = x + x / 8 (one pad
// entry per 8, as the line transforms' exchange buffers use), RS odd, so both a row
// (contiguous, padded) and a column (stride RS) are exchanged in place: a line loads
// its points into registers, and its own storage then serves as the exchange buffer
// of its transforms.  Every arithmetic step (line transforms, twiddles, phases, the
// FP64 kinetic factor and the FP64 ends of the column transforms) is the one of the
// streaming passes with 8 points per lane, so both paths give the same values.  The
// QAA model (App. E.2's baseline) runs the same two phases with FP64 Walsh-Hadamard
// lines, which need no LDS exchange.
#include "line_fft.h"
#include "pass_common.h"
#include "qhd_internal.h"

namespace qhd {

template <int NX, int NY, int MODEL = kModelQHD>
struct ResCfg {
  static constexpr int P = 8;
  static constexpr int TX = NX / P, TY = NY / P;               // lanes per row / column line
  // 1024 threads (four waves per SIMD) where the registers fit in 128 per lane
  static constexpr int MAXT = ((NX == 128 && NY == 64) || (MODEL == kModelQAA && NX * NY == 16384)) ? 512 : 1024;
  static constexpr int NT = (NX * NY / P) < MAXT ? (NX * NY / P) : MAXT;
  static constexpr int RS = ((NX + NX / 8) | 1);               // row stride in slots (odd)
  static constexpr int ROWS_PER_IT = NT / TX, COLS_PER_IT = NT / TY;
  static_assert(NX >= 32 && NY >= 32 && NX <= 128 && NY <= 128, "resident sizes: 32..128 per axis");
  static_assert(NY % ROWS_PER_IT == 0 && NX % COLS_PER_IT == 0, "whole line rounds");
};

template <int NX, int NY, int MODEL, bool Y4>
__global__ void __launch_bounds__((ResCfg<NX, NY, MODEL>::NT)) k_resident_2d(const InstDev* __restrict__ inst, const int* __restrict__ nact_p,
                                                                     float2* __restrict__ psi,
                                                                     const double* __restrict__ f,
                                                                     const double2* __restrict__ twx,
                                                                     const double2* __restrict__ twy,
                                                                     long long max_steps) {
  const int ninst = *nact_p;  // members active in this sub-step (device, set per chunk)
  using C = ResCfg<NX, NY, MODEL>;
  constexpr int P = C::P, TX = C::TX, TY = C::TY, NT = C::NT, RS = C::RS;
  __shared__ float2 st[NY * RS];
  __shared__ double2 twlx[TwLdsSize<NX, P>::value];
  __shared__ double2 twly[NX == NY ? 1 : TwLdsSize<NY, P>::value];
  __shared__ double2 eyl[NY];  // E_y(k_y) / (nx ny) of the current step
  const int tid = threadIdx.x;
  const int rl = tid / TX, rt = tid % TX;  // row phase: line of this lane group, lane in the line
  const int cl = tid / TY, ct = tid % TY;  // column phase
  TwiddlesFor<NX, P> tx;
  load_twiddles(tx, twx, twlx, rt);
  TwiddlesFor<NY, P> ty;
  load_twiddles(ty, twy, NX == NY ? twlx : twly, ct);  // equal sizes share one table
  const double inv_n = 1.0 / ((double)NX * (double)NY);
  for (int i = blockIdx.x; i < ninst; i += gridDim.x) {
    const InstDev& I = inst[i];
    const long long lim = step_limit(I, max_steps);
    if (lim <= 0) continue;  // block-uniform
    float2* __restrict__ pg = psi + I.psi_off;
    const double* __restrict__ fg = f + I.psi_off;
    // tiled HBM -> row-major LDS: element 2e and 2e+1 are (x, y) and (x + 1, y), x even
    for (int e = tid; e < NX * NY / 2; e += NT) {
      const float4 v = reinterpret_cast<const float4*>(pg)[e];
      const int idx = 2 * e, tile = idx >> 6, w = idx & 63;
      const int y = ((tile / (NX / 8)) << 3) + (w >> 3), x = ((tile % (NX / 8)) << 3) + (w & 7);
      st[y * RS + lds_slot(x)] = make_float2(v.x, v.y);
      st[y * RS + lds_slot(x) + 1] = make_float2(v.z, v.w);
    }
    __syncthreads();
    for (long long s = 0; s < lim; ++s) {
      const long long j = I.steps_done + s;
      const bool entry = (s == 0 && I.mode == kModeClean);
      double a, b;
      sched_ab<Y4>(I, j, a, b);
      const double cx = a * I.kin_turns[0];
      if (tid < NY) {
        // read in the column phase, after the barrier that ends the row phase
        double arg;
        if constexpr (MODEL == kModelQAA) {
          arg = a * axis_turns<MODEL>(I, 1, tid, NY);
        } else {
          const int nyf = freq(tid, NY);
          arg = a * I.kin_turns[1] * (double)(nyf * nyf);
        }
        const double2 e = phase_turns_d(arg);
        eyl[tid] = make_double2(e.x * inv_n, e.y * inv_n);
      }
      // row phase: [F_x^{-1}] . merged potential half steps . F_x
      const double cpot = potential_turns<Y4>(I, j, entry);
#pragma unroll 1
      for (int y = rl; y < NY; y += C::ROWS_PER_IT) {
        float2* my = st + y * RS;
        if constexpr (MODEL == kModelQAA) {
          double2 reg[P];
#pragma unroll
          for (int q = 0; q < P; ++q) assign(reg[q], my[lds_slot(rt + q * TX)]);
          if (!entry) line_wht<NX, P>(reg, rt);
#pragma unroll
          for (int q = 0; q < P; ++q)
            reg[q] = cmul_fd(reg[q], phase_turns_d(cpot * fg[tile_index(rt + q * TX, y, NX)]));
          line_wht<NX, P>(reg, rt);
#pragma unroll
          for (int q = 0; q < P; ++q) assign(my[lds_slot(rt + q * TX)], reg[q]);
        } else {
          float2 reg[P];
#pragma unroll
          for (int q = 0; q < P; ++q) reg[q] = my[lds_slot(rt + q * TX)];
          wave_lds_sync();
          if (!entry) line_fft<NX, P, +1>(reg, rt, tx, my);
#pragma unroll
          for (int q = 0; q < P; ++q)
            reg[q] = cmul_fd(reg[q], phase_turns_d(cpot * fg[tile_index(rt + q * TX, y, NX)]));
          line_fft<NX, P, -1>(reg, rt, tx, my);
#pragma unroll
          for (int q = 0; q < P; ++q) my[lds_slot(rt + q * TX)] = reg[q];
        }
      }
      __syncthreads();
      // column phase: F_y . K . F_y^{-1} with K = E_x E_y / (nx ny) in FP64
#pragma unroll 1
      for (int x = cl; x < NX; x += C::COLS_PER_IT) {
        float2* my = st + lds_slot(x);
        float2 reg[P];
#pragma unroll
        for (int q = 0; q < P; ++q) reg[q] = my[(ct + q * TY) * RS];
        double2 kd[P];
        double xarg;
        if constexpr (MODEL == kModelQAA) {
#pragma unroll
          for (int q = 0; q < P; ++q) assign(kd[q], reg[q]);
          line_wht<NY, P>(kd, ct);
          xarg = a * axis_turns<MODEL>(I, 0, x, NX);
        } else {
          wave_lds_sync();
          line_fft_io<NY, P, -1, false, StrideIx<RS>>(reg, kd, ct, ty, my);
          const int nxf = freq(x, NX);
          xarg = cx * (double)(nxf * nxf);
        }
        const double2 ex = phase_turns_d(xarg);
#pragma unroll
        for (int q = 0; q < P; ++q) {
          const double2 ey = eyl[ct + q * TY];
          const double2 k = make_double2(fma(ex.x, ey.x, -ex.y * ey.y), fma(ex.x, ey.y, ex.y * ey.x));
          kd[q] = cmul_fd(kd[q], k);
        }
        if constexpr (MODEL == kModelQAA) {
          line_wht<NY, P>(kd, ct);
#pragma unroll
          for (int q = 0; q < P; ++q) assign(reg[q], kd[q]);
        } else {
          line_fft_io<NY, P, +1, false, StrideIx<RS>>(kd, reg, ct, ty, my);
        }
#pragma unroll
        for (int q = 0; q < P; ++q) my[(ct + q * TY) * RS] = reg[q];
      }
      __syncthreads();
    }
    // row-major LDS -> tiled HBM
    for (int e = tid; e < NX * NY / 2; e += NT) {
      const int idx = 2 * e, tile = idx >> 6, w = idx & 63;
      const int y = ((tile / (NX / 8)) << 3) + (w >> 3), x = ((tile % (NX / 8)) << 3) + (w & 7);
      const float2 p0 = st[y * RS + lds_slot(x)], p1 = st[y * RS + lds_slot(x) + 1];
      reinterpret_cast<float4*>(pg)[e] = make_float4(p0.x, p0.y, p1.x, p1.y);
    }
    __syncthreads();  // the next instance's load reuses the LDS
  }
}

bool resident_supported(int nx, int ny) {
  auto ok = [](int n) { return n == 32 || n == 64 || n == 128; };
  return ok(nx) && ok(ny);
}

hipError_t launch_resident_2d(int nx, int ny, const InstDev* inst, int ninst, const int* nact, float2* psi,
                              const double* f,
                              const double2* tw_nx, const double2* tw_ny, long long max_steps, int model,
                              bool y4, hipStream_t stream) {
  if (ninst <= 0) return hipSuccess;
  if (!resident_supported(nx, ny)) return hipErrorInvalidValue;
#define QHD_RES_LAUNCH(NX_, NY_)                                                                              \
  if (nx == NX_ && ny == NY_) {                                                                               \
    constexpr int NT_ = ResCfg<NX_, NY_>::NT, NTQ_ = ResCfg<NX_, NY_, kModelQAA>::NT;                         \
    if (model == kModelQAA)                                                                                   \
      QHD_LAUNCH((k_resident_2d<NX_, NY_, kModelQAA, false>), dim3(ninst), dim3(NTQ_), 0, stream,     \
                         inst, nact, psi, f, tw_nx, tw_ny, max_steps);                                       \
    else if (y4)                                                                                              \
      QHD_LAUNCH((k_resident_2d<NX_, NY_, kModelQHD, true>), dim3(ninst), dim3(NT_), 0, stream,       \
                         inst, nact, psi, f, tw_nx, tw_ny, max_steps);                                       \
    else                                                                                                      \
      QHD_LAUNCH((k_resident_2d<NX_, NY_, kModelQHD, false>), dim3(ninst), dim3(NT_), 0, stream,      \
                         inst, nact, psi, f, tw_nx, tw_ny, max_steps);                                       \
    return hipGetLastError();                                                                                 \
  }
  QHD_RES_LAUNCH(32, 32)
  QHD_RES_LAUNCH(32, 64)
  QHD_RES_LAUNCH(32, 128)
  QHD_RES_LAUNCH(64, 32)
  QHD_RES_LAUNCH(64, 64)
  QHD_RES_LAUNCH(64, 128)
  QHD_RES_LAUNCH(128, 32)
  QHD_RES_LAUNCH(128, 64)
  QHD_RES_LAUNCH(128, 128)
#undef QHD_RES_LAUNCH
  return hipErrorInvalidValue;
}

}  // namespace qhd
