// 3-D passes of the QHD split-operator engine (gfx950): an x-pass and a (y, z)-plane
// pass, two HBM passes per step.
//
// In three dimensions the symmetric step reads
//     ... V^{1/2} F_x^{-1} F_y^{-1} F_z^{-1} K F_z F_y F_x V^{1/2} ...
// (App. C.2.1 eq. prod_qhd_fft / App. E.1 with F = F_z F_y F_x, the kinetic factor K
// diagonal in (k_x, k_y, k_z)).  With the state kept in (k_x, y, z) space between steps
// the step is two passes over it:
//   x-pass      F_x . V_{j-1}^{1/2} V_j^{1/2} . F_x^{-1}   (lines along x, f read)
//   plane pass  F_y^{-1} F_z^{-1} . K_j . F_z F_y          (one (y, z) plane per k_x,
//                                                          held in LDS)
// so a step moves 24 + 16 = 40 bytes per grid point (psi read and written twice, f read
// once in FP64).
//
// Layout in HBM ("plane layout"): x is the slowest axis; the (y, z) plane of every x is
// contiguous and stored in 8 x 8 tiles of (y, z) (64 complex values, 512 bytes; y
// fastest inside a tile), tile rows along y one after another:
//     offset(x, y, z) = x * ny * nz + tile_index(y, z, ny).
// f (FP64) uses the same layout.  The x-pass gives the 64 lanes of a wavefront the 64
// (y, z) points of one tile and its wavefronts the x positions, so every slot load or
// store of a wavefront is one whole tile; the plane pass reads and writes a plane as one
// contiguous block.
#include "line_fft.h"
#include "pass_common.h"
#include "qhd_internal.h"

namespace qhd {

// position of (y, z) inside a plane
__device__ __forceinline__ long long plane_index(int y, int z, int ny) { return tile_index(y, z, ny); }

// ------------------------------------------------------------------------------------
// x-pass: lane l of wavefront w owns point l of a (y, z) tile and the x positions
// w + q*W (q = 0..P-1).  A line spans W wavefronts, so each exchange of its transform is
// a block barrier; 128-point lines take 16 points per lane (radices 16 and 8: one
// exchange per transform, eight wavefronts).

template <int NX>
struct XCfg {
  static constexpr int P = NX >= 128 ? 16 : 8;
  static constexpr int W = NX / P;  // wavefronts per block = lanes per line
  static constexpr int NT = W * 64;
  // line stride = 1 (mod 16) float2 slots: the 64 lines of a wavefront spread over the banks
  static constexpr int STRIDE = ((LineLds<NX>::kSlots + 14) / 16) * 16 + 1;
};

template <int NX, bool Y4>
__global__ void __launch_bounds__((XCfg<NX>::NT)) k_xpass_3d(const InstDev* __restrict__ inst,
                                                             const int* __restrict__ nact_p, int ny_log2,
                                                             int nz_log2, float2* __restrict__ psi,
                                                             const double* __restrict__ f,
                                                             const double2* __restrict__ twtab, int s,
                                                             long long max_steps) {
  const int ninst = *nact_p;  // members active in this sub-step (device, set per chunk)
  using C = XCfg<NX>;
  constexpr int P = C::P, W = C::W, STRIDE = C::STRIDE;
  __shared__ float2 lds[64 * STRIDE];
  __shared__ double2 twl[TwLdsSize<NX, P>::value];
  const int lane = threadIdx.x & 63, t = threadIdx.x >> 6;
  float2* my = lds + lane * STRIDE;
  // twiddles from an LDS table (a wavefront's lanes share t, so each read is a
  // broadcast): with the register cache (16 FP64 pairs per lane at 128 points) the pass
  // took 1.48x as long on 16 x 128^3
  TwiddlesFor<NX, P> tw;
  load_twiddles(tw, twtab, twl, t);
  const int tiles_log2 = ny_log2 + nz_log2 - 6;  // 8 x 8 tiles per plane
  const long long plane = 1LL << (ny_log2 + nz_log2);
  const long long total = (long long)ninst << tiles_log2;
  long long begin, end;
  block_share(total, 1, begin, end);
  for (long long g = begin; g < end; ++g) {
    // the block's item is one tile of one instance: block-uniform instance reads
    const int i = (int)(g >> tiles_log2);
    const int tile = (int)(g & ((1LL << tiles_log2) - 1));
    const InstDev& I = inst[i];
    const bool active = s < step_limit(I, max_steps);
    const long long j = I.steps_done + s;
    const bool entry = (s == 0 && I.mode == kModeClean);
    const double cpot = potential_turns<Y4>(I, j, entry);
    // scalar base (the item's tile), the lane's offset (its point and plane t) in one
    // register, the slot offsets (planes t + q W) scalar
    const long long off = I.psi_off + ((long long)tile << 6);
    const int lane_off = lane + t * (int)plane;
    const LaneView<float2> pv(psi + off, lane_off);
    const LaneView<double> fv(f + off, lane_off);
    float2 reg[P];
#pragma unroll
    for (int q = 0; q < P; ++q) reg[q] = pv.load(q * W * (int)plane);
    if (!entry) line_fft<NX, P, +1, (W > 1)>(reg, t, tw, my);
#pragma unroll
    for (int q = 0; q < P; ++q) reg[q] = cmul_fd(reg[q], phase_turns_d(cpot * fv.load(q * W * (int)plane)));
    line_fft<NX, P, -1, (W > 1)>(reg, t, tw, my);
    if (active) {
#pragma unroll
      for (int q = 0; q < P; ++q) pv.store(q * W * (int)plane, reg[q]);
    }
    if constexpr (W > 1) __syncthreads();  // the next item's first exchange reuses the LDS
  }
}

// ------------------------------------------------------------------------------------
// plane pass: one workgroup per (instance, k_x) plane.  The plane is copied into LDS
// row-major, point (y, z) at z * RS + slot(y), slot(y) = y + y / 8, RS odd: a y-line
// (a row) is contiguous and padded, a z-line (a column) has stride RS, and each line runs
// its transforms' exchanges in its own storage.  Row phase F_y; column phase F_z, K,
// F_z^{-1} with the last forward stage, K and the first inverse stage in FP64 (there the
// uniform start concentrates into one coefficient); row phase F_y^{-1}.  A 128 x 128
// plane takes 148.5 KB of LDS: one workgroup per CU.

template <int NY, int NZ>
struct PlaneCfg {
  static constexpr int P = 8;
  static constexpr int TY = NY / P, TZ = NZ / P;  // lanes per row / column line
  static constexpr int WORK = NY * NZ / P;
  static constexpr int NT = WORK < 64 ? 64 : (WORK > 1024 ? 1024 : WORK);
  static constexpr int RS = ((NY + NY / 8) | 1);  // row stride in slots (odd)
  static constexpr int ROWS_PER_IT = NT / TY, COLS_PER_IT = NT / TZ;
};

template <int NY, int NZ, bool Y4>
__global__ void __launch_bounds__((PlaneCfg<NY, NZ>::NT)) k_plane_3d(const InstDev* __restrict__ inst,
                                                                     const int* __restrict__ nact_p, int nx,
                                                                     float2* __restrict__ psi,
                                                                     const double2* __restrict__ twy,
                                                                     const double2* __restrict__ twz, int s,
                                                                     long long max_steps) {
  const int ninst = *nact_p;  // members active in this sub-step (device, set per chunk)
  using C = PlaneCfg<NY, NZ>;
  constexpr int P = C::P, TY = C::TY, TZ = C::TZ, NT = C::NT, RS = C::RS;
  constexpr int PLANE = NY * NZ;
  __shared__ float2 st[NZ * RS];
  __shared__ double2 twly[TwLdsSize<NY, P>::value];
  __shared__ double2 twlz[NY == NZ ? 1 : TwLdsSize<NZ, P>::value];
  __shared__ double2 ezl[NZ];  // E_z(k_z) / (nx ny nz) of the plane's instance and step
  const int tid = threadIdx.x;
  const int rl = tid / TY, rt = tid % TY;  // row phase: line of this lane group, lane in the line
  const int cl = tid / TZ, ct = tid % TZ;  // column phase
  TwiddlesFor<NY, P> ty;
  load_twiddles(ty, twy, twly, rt);
  TwiddlesFor<NZ, P> tz;
  load_twiddles(tz, twz, NY == NZ ? twly : twlz, ct);  // equal sizes share one table
  const double inv_n = 1.0 / ((double)nx * (double)NY * (double)NZ);
  const long long total = (long long)ninst * nx;
  double cached = -1.0;  // E_z depends on the instance and step only through a_j pi dt / L_z^2
  for (long long g = blockIdx.x; g < total; g += gridDim.x) {
    const int i = (int)(g / nx), x = (int)(g - (long long)i * nx);
    const InstDev& I = inst[i];
    if (!(s < step_limit(I, max_steps))) continue;  // block-uniform
    double a, b;
    sched_ab<Y4>(I, I.steps_done + s, a, b);
    const double cz = a * I.kin_turns[2];
    if (cz != cached) {
      // the previous plane's readers of the table passed the barrier after its column phase
      for (int k = tid; k < NZ; k += NT) {
        const int nzf = freq(k, NZ);
        const double2 e = phase_turns_d(cz * (double)(nzf * nzf));
        ezl[k] = make_double2(e.x * inv_n, e.y * inv_n);
      }
      cached = cz;
    }
    float2* __restrict__ pg = psi + I.psi_off + (long long)x * PLANE;
    // tiled HBM -> row-major LDS: elements 2e and 2e+1 are (y, z) and (y + 1, z), y even
    for (int e = tid; e < PLANE / 2; e += NT) {
      const float4 v = reinterpret_cast<const float4*>(pg)[e];
      const int idx = 2 * e, tile = idx >> 6, w = idx & 63;
      const int z = ((tile / (NY / 8)) << 3) + (w >> 3), y = ((tile % (NY / 8)) << 3) + (w & 7);
      st[z * RS + lds_slot(y)] = make_float2(v.x, v.y);
      st[z * RS + lds_slot(y) + 1] = make_float2(v.z, v.w);
    }
    __syncthreads();
    // row phase: F_y on every z-row
#pragma unroll 1
    for (int z = rl; z < NZ; z += C::ROWS_PER_IT) {
      float2* my = st + z * RS;
      float2 reg[P];
#pragma unroll
      for (int q = 0; q < P; ++q) reg[q] = my[lds_slot(rt + q * TY)];
      wave_lds_sync();
      line_fft<NY, P, -1>(reg, rt, ty, my);
#pragma unroll
      for (int q = 0; q < P; ++q) my[lds_slot(rt + q * TY)] = reg[q];
    }
    __syncthreads();
    // column phase: F_z . K . F_z^{-1}, K = E_x E_y E_z / (nx ny nz) in FP64
    const int nxf = freq(x, nx);
    const double cx = a * I.kin_turns[0] * (double)(nxf * nxf);
#pragma unroll 1
    for (int y = cl; y < NY; y += C::COLS_PER_IT) {
      float2* my = st + lds_slot(y);
      float2 reg[P];
#pragma unroll
      for (int q = 0; q < P; ++q) reg[q] = my[(ct + q * TZ) * RS];
      double2 kd[P];
      wave_lds_sync();
      line_fft_io<NZ, P, -1, false, StrideIx<RS>>(reg, kd, ct, tz, my);
      const int nyf = freq(y, NY);
      const double2 exy = phase_turns_d(fma(a * I.kin_turns[1], (double)(nyf * nyf), cx));
#pragma unroll
      for (int q = 0; q < P; ++q) {
        const double2 ez = ezl[ct + q * TZ];
        kd[q] = cmul_fd(kd[q], make_double2(fma(exy.x, ez.x, -exy.y * ez.y), fma(exy.x, ez.y, exy.y * ez.x)));
      }
      line_fft_io<NZ, P, +1, false, StrideIx<RS>>(kd, reg, ct, tz, my);
#pragma unroll
      for (int q = 0; q < P; ++q) my[(ct + q * TZ) * RS] = reg[q];
    }
    __syncthreads();
    // row phase: F_y^{-1}
#pragma unroll 1
    for (int z = rl; z < NZ; z += C::ROWS_PER_IT) {
      float2* my = st + z * RS;
      float2 reg[P];
#pragma unroll
      for (int q = 0; q < P; ++q) reg[q] = my[lds_slot(rt + q * TY)];
      wave_lds_sync();
      line_fft<NY, P, +1>(reg, rt, ty, my);
#pragma unroll
      for (int q = 0; q < P; ++q) my[lds_slot(rt + q * TY)] = reg[q];
    }
    __syncthreads();
    // row-major LDS -> tiled HBM
    for (int e = tid; e < PLANE / 2; e += NT) {
      const int idx = 2 * e, tile = idx >> 6, w = idx & 63;
      const int z = ((tile / (NY / 8)) << 3) + (w >> 3), y = ((tile % (NY / 8)) << 3) + (w & 7);
      const float2 p0 = st[z * RS + lds_slot(y)], p1 = st[z * RS + lds_slot(y) + 1];
      reinterpret_cast<float4*>(pg)[e] = make_float4(p0.x, p0.y, p1.x, p1.y);
    }
    __syncthreads();  // the next plane's load reuses the LDS
  }
}

// ------------------------------------------------------------------------------------
// plane pass, direct form (64- and 128-point y-lines): a row line of NY points takes 8
// lanes (NY / 8 points each, lane t holding y = t + 8 q), so a wavefront's 8 row lines
// are the 8 z-rows of one tile row and every slot of theirs is one whole 8 x 8 tile of
// the HBM plane: the first row phase loads from HBM straight into registers and the
// second stores from registers, and only the column phase reads the plane from LDS.
// The row lines exchange inside their own rows of the plane buffer (wavefront-local,
// no block barrier), then write their results there for the column phase.  Lines of
// 128 points take 16 points per lane (radices 16 and 8: one exchange per transform).
//
// LDS placement (the LDS serves an 8-byte access 16 lanes per clock over 32 four-byte
// banks, so each group of 16 lanes should touch 16 distinct bank pairs): point (y, z) at
// z RS + y with RS = 2 (mod 16).  The 16 lanes of a group hold two row lines z and
// z + 4 (4 RS = 8 mod 16), whose accesses are 8 consecutive bank pairs each (row
// exchange slot i + i/16), or two column lines y and y + 1, whose accesses are 8
// distinct even bank pairs each (column exchange slot: z = i with its low four bits
// rotated by i/16, so the radix-16 scatter does not put a line's 8 lanes on one bank).
struct PlaneRowIx {
  __device__ static constexpr int at(int i) { return i + (i >> 4); }
};
template <int RS>
struct PlaneColIx {
  __device__ static constexpr int at(int i) { return ((i & ~15) | ((i + (i >> 4)) & 15)) * RS; }
};

template <int NY, int NZ>
struct PlaneDCfg {
  static constexpr int TY = 8, PY = NY / 8;       // lanes per row line, points per lane
  static constexpr int PZ = NZ >= 128 ? 16 : 8;   // points per lane of a column line
  static constexpr int TZ = NZ / PZ;
  // row lines per 8 lanes (two, in blocks of 512 threads without spills, measured 4 %
  // slower at 128 x 128 than one in blocks of 1024)
  static constexpr int ROW_ITS = 1;
  static constexpr int NT = NZ * TY / ROW_ITS;
  static constexpr int RS = ((NY + NY / 16 + 13) / 16) * 16 + 2;  // row stride, = 2 (mod 16)
  static constexpr int COLS_PER_IT = NT / TZ;
  static constexpr bool SHARE_TW = NY == NZ && PY == PZ;
};

template <int NY, int NZ, bool Y4>
__global__ void __launch_bounds__((PlaneDCfg<NY, NZ>::NT)) k_plane_direct_3d(const InstDev* __restrict__ inst,
                                                                             const int* __restrict__ nact_p, int nx,
                                                                             float2* __restrict__ psi,
                                                                             const double2* __restrict__ twy,
                                                                             const double2* __restrict__ twz, int s,
                                                                             long long max_steps, double inv_n) {
  const int ninst = *nact_p;  // members active in this sub-step (device, set per chunk)
  using C = PlaneDCfg<NY, NZ>;
  constexpr int TY = C::TY, PY = C::PY, PZ = C::PZ, TZ = C::TZ, NT = C::NT, RS = C::RS;
  constexpr int PLANE = NY * NZ;
  static_assert(NY == 64 || NY == 128, "direct plane pass: 64- or 128-point y-lines");
  __shared__ float2 st[NZ * RS];
  __shared__ double2 twly[TwLdsSize<NY, PY>::value];
  __shared__ double2 twlz[C::SHARE_TW ? 1 : TwLdsSize<NZ, PZ>::value];
  __shared__ double2 ezl[NZ];  // E_z(k_z) / (nx ny nz) of the plane's instance and step
  const int tid = threadIdx.x;
  // row phase: line li of a wavefront's 8 takes z-row 8 w + 4 (li & 1) + li / 2, so the
  // two lines of each group of 16 lanes are 4 rows apart; lane rt of the line
  const int li = (tid >> 3) & 7;
  const int rz0 = ((tid >> 6) << 3) + ((li & 1) << 2) + (li >> 1), rt = tid % TY;
  constexpr int ROW_ITS = C::ROW_ITS, RSTEP = NT / TY;  // row lines of a lane: rz0 + it RSTEP
  const int cl = tid / TZ, ct = tid % TZ;  // column phase
  TwiddlesFor<NY, PY> ty;
  load_twiddles(ty, twy, twly, rt);
  TwiddlesFor<NZ, PZ> tz;
  load_twiddles(tz, twz, C::SHARE_TW ? twly : twlz, ct);
  const long long total = (long long)ninst * nx;
  // this lane's first element of its first row line in a plane: y = rt, z = rz0
  const int row_off = (rz0 >> 3) * (NY / 8) * 64 + (rz0 & 7) * 8 + rt;
  double cached = -1.0;  // E_z depends on the instance and step only through a_j pi dt / L_z^2
  for (long long g = blockIdx.x; g < total; g += gridDim.x) {
    const int i = (int)(g / nx), x = (int)(g - (long long)i * nx);
    const InstDev& I = inst[i];
    if (!(s < step_limit(I, max_steps))) continue;  // block-uniform
    double a, b;
    sched_ab<Y4>(I, I.steps_done + s, a, b);
    const double cz = a * I.kin_turns[2];
    if (cz != cached) {
      // the previous plane's readers of the table passed the barrier after its column phase
      for (int k = tid; k < NZ; k += NT) {
        const int nzf = freq(k, NZ);
        const double2 e = phase_turns_d(cz * (double)(nzf * nzf));
        ezl[k] = make_double2(e.x * inv_n, e.y * inv_n);
      }
      cached = cz;
    }
    float2* __restrict__ rowg = psi + I.psi_off + (long long)x * PLANE + row_off;
    // row phase: F_y on every z-row, from HBM (slot q of a wavefront is one tile)
#pragma unroll 1
    for (int it = 0; it < ROW_ITS; ++it) {
      float2* my = st + (rz0 + it * RSTEP) * RS;
      const float2* rg = rowg + it * (RSTEP / 8) * (NY / 8) * 64;
      float2 reg[PY];
#pragma unroll
      for (int q = 0; q < PY; ++q) reg[q] = rg[q * 64];
      line_fft<NY, PY, -1, false, PlaneRowIx>(reg, rt, ty, my);
#pragma unroll
      for (int q = 0; q < PY; ++q) my[rt + q * TY] = reg[q];
    }
    __syncthreads();
    // column phase: F_z . K . F_z^{-1}, K = E_x E_y E_z / (nx ny nz) in FP64
    const int nxf = freq(x, nx);
    const double cx = a * I.kin_turns[0] * (double)(nxf * nxf);
#pragma unroll 1
    for (int y = cl; y < NY; y += C::COLS_PER_IT) {
      float2* mc = st + y;
      float2 reg[PZ];
#pragma unroll
      for (int q = 0; q < PZ; ++q) reg[q] = mc[(ct + q * TZ) * RS];
      double2 kd[PZ];
      wave_lds_sync();
      line_fft_io<NZ, PZ, -1, false, PlaneColIx<RS>>(reg, kd, ct, tz, mc);
      const int nyf = freq(y, NY);
      const double2 exy = phase_turns_d(fma(a * I.kin_turns[1], (double)(nyf * nyf), cx));
#pragma unroll
      for (int q = 0; q < PZ; ++q) {
        const double2 ez = ezl[ct + q * TZ];
        kd[q] = cmul_fd(kd[q], make_double2(fma(exy.x, ez.x, -exy.y * ez.y), fma(exy.x, ez.y, exy.y * ez.x)));
      }
      line_fft_io<NZ, PZ, +1, false, PlaneColIx<RS>>(kd, reg, ct, tz, mc);
#pragma unroll
      for (int q = 0; q < PZ; ++q) mc[(ct + q * TZ) * RS] = reg[q];
    }
    __syncthreads();
    // row phase: F_y^{-1}, to HBM
#pragma unroll 1
    for (int it = 0; it < ROW_ITS; ++it) {
      float2* my = st + (rz0 + it * RSTEP) * RS;
      float2* rg = rowg + it * (RSTEP / 8) * (NY / 8) * 64;
      float2 reg[PY];
#pragma unroll
      for (int q = 0; q < PY; ++q) reg[q] = my[rt + q * TY];
      wave_lds_sync();
      line_fft<NY, PY, +1, false, PlaneRowIx>(reg, rt, ty, my);
#pragma unroll
      for (int q = 0; q < PY; ++q) rg[q * 64] = reg[q];
      wave_lds_sync();  // the next row line (or plane) reuses this wavefront's rows
    }
  }
}

// ------------------------------------------------------------------------------------
// observe in the plane layout: the x-pass's item and lane layout; closes the pending
// F_x^{-1} and trailing half step, writes the user-layout psi / rho (optional), and one
// FP64 partial triple per x-line (sum rho, sum f rho, sum of rho inside the success
// ball), line (y, z) of instance i at 3 * (i * ny * nz + z * ny + y).

__device__ __forceinline__ bool in_ball_3d(int dxi, int dyi, int dzi, const InstDev& I) {
  // same FP64 operations, in the same order and without contraction, as the oracle
  const double dx = __dmul_rn((double)dxi, I.h[0]);
  const double dy = __dmul_rn((double)dyi, I.h[1]);
  const double dz = __dmul_rn((double)dzi, I.h[2]);
  return __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz)) < I.r2;
}

template <int NX>
__global__ void __launch_bounds__((XCfg<NX>::NT)) k_observe_plane(const InstDev* __restrict__ inst, int ninst,
                                                                  int ny_log2, int nz_log2,
                                                                  const float2* __restrict__ psi,
                                                                  const double* __restrict__ f,
                                                                  const double2* __restrict__ twtab,
                                                                  float2* __restrict__ out_psi,
                                                                  float* __restrict__ out_rho,
                                                                  double* __restrict__ partials) {
  using C = XCfg<NX>;
  constexpr int P = C::P, W = C::W, STRIDE = C::STRIDE;
  __shared__ float2 lds[64 * STRIDE];
  __shared__ double red[3][W][64];
  const int lane = threadIdx.x & 63, t = threadIdx.x >> 6;
  float2* my = lds + lane * STRIDE;
  Twiddles<NX, P> tw;
  tw.load(twtab, t);
  const int ny = 1 << ny_log2;
  const int tiles_log2 = ny_log2 + nz_log2 - 6;
  const long long plane = 1LL << (ny_log2 + nz_log2);
  const long long total = (long long)ninst << tiles_log2;
  for (long long g = blockIdx.x; g < total; g += gridDim.x) {
    const int i = (int)(g >> tiles_log2);
    const int tile = (int)(g & ((1LL << tiles_log2) - 1));
    const InstDev& I = inst[i];
    const bool pending = I.mode == kModePending;
    const long long off = I.psi_off + ((long long)tile << 6) + lane + (long long)t * plane;
    float2 reg[P];
    double fv[P];
#pragma unroll
    for (int q = 0; q < P; ++q) {
      reg[q] = psi[off + (long long)q * W * plane];
      fv[q] = f[off + (long long)q * W * plane];
    }
    if (pending) {  // block-uniform
      double2 in[P];
#pragma unroll
      for (int q = 0; q < P; ++q) assign(in[q], reg[q]);
      line_fft_io<NX, P, +1, (W > 1)>(in, reg, t, tw, my);
      if (I.scheme != kSchemeLie) {
        const double cpot = closing_turns(I);
#pragma unroll
        for (int q = 0; q < P; ++q) reg[q] = cmul_fd(reg[q], phase_turns_d(cpot * fv[q]));
      }
    }
    // (y, z) of this lane's line, x* from the user-layout flat index
    const int tiles_y = ny >> 3;
    const int y = ((tile % tiles_y) << 3) + (lane & 7), z = ((tile / tiles_y) << 3) + (lane >> 3);
    const long long am = I.argmin;
    const int xs = (int)(am % NX);
    const long long rs = am / NX;
    const int ys = (int)(rs & (ny - 1)), zs = (int)(rs >> ny_log2);
    double sr = 0.0, sf = 0.0, sm = 0.0;
#pragma unroll
    for (int q = 0; q < P; ++q) {
      const int x = t + q * W;
      const float2 v = reg[q];
      const double rho = (double)v.x * v.x + (double)v.y * v.y;
      sr += rho;
      sf += fv[q] * rho;
      if (in_ball_3d(x - xs, y - ys, z - zs, I)) sm += rho;
      const long long o = I.out_off + ((long long)z * ny + y) * NX + x;
      if (out_psi) out_psi[o] = v;
      if (out_rho) out_rho[o] = (float)rho;
    }
    // the W lanes of a line sit in W wavefronts: reduce through LDS in a fixed order
    red[0][t][lane] = sr;
    red[1][t][lane] = sf;
    red[2][t][lane] = sm;
    __syncthreads();
    if (t == 0) {
      double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        a0 += red[0][w][lane];
        a1 += red[1][w][lane];
        a2 += red[2][w][lane];
      }
      const long long L = (long long)i * plane + (long long)z * ny + y;
      partials[3 * L + 0] = a0;
      partials[3 * L + 1] = a1;
      partials[3 * L + 2] = a2;
    }
    __syncthreads();
  }
}

// user row-major (x fastest) -> plane layout
template <typename T>
__global__ void k_import_plane(const T* __restrict__ user, T* __restrict__ dst, int nx, int ny, int nz) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (long long)nx * ny * nz) return;
  const int x = (int)(p % nx);
  const long long r = p / nx;
  const int y = (int)(r % ny), z = (int)(r / ny);
  dst[(long long)x * ny * nz + plane_index(y, z, ny)] = user[p];
}

// ------------------------------------------------------------------------------------
// launchers

namespace {

inline int ilog2_3d(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

inline int blocks3d(long long items, int cap) {
  long long b = items;
  if (cap > 0 && b > cap) b = cap;
  return (int)(b < 1 ? 1 : b);
}

template <int NX>
hipError_t launch_x(int ny, int nz, const InstDev* inst, int ninst, const int* nact, float2* psi, const double* f,
                    const double2* tw, int s, long long max_steps, int cap, bool y4, hipStream_t stream) {
  using C = XCfg<NX>;
  const int blocks = blocks3d((long long)ninst * (ny / 8) * (nz / 8), cap);
  if (y4)
    QHD_LAUNCH((k_xpass_3d<NX, true>), dim3(blocks), dim3(C::NT), 0, stream, inst, nact, ilog2_3d(ny),
                       ilog2_3d(nz), psi, f, tw, s, max_steps);
  else
    QHD_LAUNCH((k_xpass_3d<NX, false>), dim3(blocks), dim3(C::NT), 0, stream, inst, nact, ilog2_3d(ny),
                       ilog2_3d(nz), psi, f, tw, s, max_steps);
  return hipGetLastError();
}

template <int NY, int NZ>
hipError_t launch_plane(int nx, const InstDev* inst, int ninst, const int* nact, float2* psi, const double2* twy,
                        const double2* twz, int s, long long max_steps, int cap, bool y4, hipStream_t stream) {
  const int blocks = blocks3d((long long)ninst * nx, cap);
  if constexpr (NY >= 64) {
    using C = PlaneDCfg<NY, NZ>;
    const double inv_n = 1.0 / ((double)nx * (double)NY * (double)NZ);
    if (y4)
      QHD_LAUNCH((k_plane_direct_3d<NY, NZ, true>), dim3(blocks), dim3(C::NT), 0, stream, inst, nact, nx, psi,
                         twy, twz, s, max_steps, inv_n);
    else
      QHD_LAUNCH((k_plane_direct_3d<NY, NZ, false>), dim3(blocks), dim3(C::NT), 0, stream, inst, nact, nx,
                         psi, twy, twz, s, max_steps, inv_n);
    return hipGetLastError();
  }
  using C = PlaneCfg<NY, NZ>;
  if (y4)
    QHD_LAUNCH((k_plane_3d<NY, NZ, true>), dim3(blocks), dim3(C::NT), 0, stream, inst, nact, nx, psi, twy, twz,
                       s, max_steps);
  else
    QHD_LAUNCH((k_plane_3d<NY, NZ, false>), dim3(blocks), dim3(C::NT), 0, stream, inst, nact, nx, psi, twy,
                       twz, s, max_steps);
  return hipGetLastError();
}

template <int NY>
hipError_t launch_plane_nz(int nz, int nx, const InstDev* inst, int ninst, const int* nact, float2* psi,
                           const double2* twy, const double2* twz, int s, long long max_steps, int cap, bool y4,
                           hipStream_t stream) {
  switch (nz) {
    case 16: return launch_plane<NY, 16>(nx, inst, ninst, nact, psi, twy, twz, s, max_steps, cap, y4, stream);
    case 32: return launch_plane<NY, 32>(nx, inst, ninst, nact, psi, twy, twz, s, max_steps, cap, y4, stream);
    case 64: return launch_plane<NY, 64>(nx, inst, ninst, nact, psi, twy, twz, s, max_steps, cap, y4, stream);
    case 128: return launch_plane<NY, 128>(nx, inst, ninst, nact, psi, twy, twz, s, max_steps, cap, y4, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_xpass_3d(int nx, int ny, int nz, const InstDev* inst, int ninst, const int* nact, float2* psi,
                           const double* f, const double2* tw_x, int s, long long max_steps, int grid_cap, bool y4,
                           hipStream_t stream) {
  switch (nx) {
    case 16: return launch_x<16>(ny, nz, inst, ninst, nact, psi, f, tw_x, s, max_steps, grid_cap, y4, stream);
    case 32: return launch_x<32>(ny, nz, inst, ninst, nact, psi, f, tw_x, s, max_steps, grid_cap, y4, stream);
    case 64: return launch_x<64>(ny, nz, inst, ninst, nact, psi, f, tw_x, s, max_steps, grid_cap, y4, stream);
    case 128: return launch_x<128>(ny, nz, inst, ninst, nact, psi, f, tw_x, s, max_steps, grid_cap, y4, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_plane_3d(int nx, int ny, int nz, const InstDev* inst, int ninst, const int* nact, float2* psi,
                           const double2* tw_y, const double2* tw_z, int s, long long max_steps, int grid_cap,
                           bool y4, hipStream_t stream) {
  switch (ny) {
    case 16: return launch_plane_nz<16>(nz, nx, inst, ninst, nact, psi, tw_y, tw_z, s, max_steps, grid_cap, y4, stream);
    case 32: return launch_plane_nz<32>(nz, nx, inst, ninst, nact, psi, tw_y, tw_z, s, max_steps, grid_cap, y4, stream);
    case 64: return launch_plane_nz<64>(nz, nx, inst, ninst, nact, psi, tw_y, tw_z, s, max_steps, grid_cap, y4, stream);
    case 128:
      return launch_plane_nz<128>(nz, nx, inst, ninst, nact, psi, tw_y, tw_z, s, max_steps, grid_cap, y4, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_observe_plane(int nx, int ny, int nz, const InstDev* inst, int ninst, const float2* psi,
                                const double* f, const double2* tw_x, float2* out_psi, float* out_rho,
                                double* partials, hipStream_t stream) {
  const int blocks = blocks3d((long long)ninst * (ny / 8) * (nz / 8), 4096);
#define QHD_OBS_PLANE(NXV)                                                                                      \
  case NXV:                                                                                                     \
    QHD_LAUNCH((k_observe_plane<NXV>), dim3(blocks), dim3(XCfg<NXV>::NT), 0, stream, inst, ninst,       \
                       ilog2_3d(ny), ilog2_3d(nz), psi, f, tw_x, out_psi, out_rho, partials);                   \
    return hipGetLastError();
  switch (nx) {
    QHD_OBS_PLANE(16)
    QHD_OBS_PLANE(32)
    QHD_OBS_PLANE(64)
    QHD_OBS_PLANE(128)
    default:
      return hipErrorInvalidValue;
  }
#undef QHD_OBS_PLANE
}

hipError_t launch_import_f_plane(int nx, int ny, int nz, const double* user, double* dst, hipStream_t stream) {
  const long long n = (long long)nx * ny * nz;
  QHD_LAUNCH(k_import_plane<double>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, user, dst, nx,
                     ny, nz);
  return hipGetLastError();
}

hipError_t launch_import_psi_plane(int nx, int ny, int nz, const float2* user, float2* dst, hipStream_t stream) {
  const long long n = (long long)nx * ny * nz;
  QHD_LAUNCH(k_import_plane<float2>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, user, dst, nx,
                     ny, nz);
  return hipGetLastError();
}

}  // namespace qhd
