// 3-D passes of the QHD split-operator engine (gfx950).
//
// In three dimensions the symmetric step reads, per axis,
//     ... V^{1/2} F_x^{-1} F_y^{-1} F_z^{-1} K F_z F_y F_x V^{1/2} ...
// (App. C.2.1 eq. prod_qhd_fft / App. E.1 with F = F_z F_y F_x).  Grouping the
// line transforms into single-axis streaming passes gives four passes per step:
//   x-pass  F_x . V_{j-1}^{1/2} V_j^{1/2} . F_x^{-1}   (the 2-D row pass, rows = ny*nz)
//   y-pass  F_y                                        (forward)
//   z-pass  F_z^{-1} . K_j . F_z                       (K = E_x E_y E_z / (nx ny nz))
//   y-pass  F_y^{-1}                                   (inverse)
// The state between steps stays in (k_x, y, z) space exactly as in 2-D.  Each
// z-slab is stored like a 2-D instance (8x8 tiles), slab after slab.
//
// Both kernels are "tile-wave": a slot load or store of one wavefront is one
// whole 8x8 tile (64 consecutive complex values).
#include "line_fft.h"
#include "pass_common.h"
#include "qhd_internal.h"

namespace qhd {

// ------------------------------------------------------------------------------------
// y-pass: lanes l of wavefront w own column c = l & 7 of a tile column of one slab
// and row group t = (l >> 3) + 8 w; slot q holds row t + q*TPL.

template <int NY>
struct YCfg {
  static constexpr int P = NY >= 64 ? 8 : NY / 8;
  static constexpr int TPL = NY / P;
  static constexpr int W = TPL / 8;
  static constexpr int ITEMS = W >= 4 ? 1 : 4 / W;
  static constexpr int NT = ITEMS * W * 64;
  static constexpr int STRIDE = ((LineLds<NY>::kSlots + 13) / 16) * 16 + 2;
};

template <int NY, int DIR>
__global__ void __launch_bounds__((YCfg<NY>::NT)) k_ypass_3d(
    const InstDev* __restrict__ inst, int ninst, int nx_log2, int nz_log2, float2* __restrict__ psi,
    const double2* __restrict__ twtab, int s, long long max_steps) {
  using C = YCfg<NY>;
  constexpr int P = C::P, TPL = C::TPL, W = C::W, ITEMS = C::ITEMS, STRIDE = C::STRIDE;
  __shared__ float2 lds[ITEMS * 8 * STRIDE];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // wave-uniform: the instance record is read with scalar loads
  const int item = __builtin_amdgcn_readfirstlane(wave / W), wv = wave - item * W;
  const int c = lane & 7;
  const int t = (lane >> 3) + 8 * wv;
  float2* my = lds + (item * 8 + c) * STRIDE;
  Twiddles<NY, P> tw;
  tw.load(twtab, t);
  const int nx = 1 << nx_log2, tc_log2 = nx_log2 - 3, tcols = nx >> 3;
  const long long slab = (long long)nx * NY;
  const int per_inst_log2 = tc_log2 + nz_log2;  // items per instance: tcols * nz
  const long long total = (long long)ninst << per_inst_log2;
  long long begin, end;
  block_share(total, ITEMS, begin, end);
  for (long long g0 = begin; g0 < end; g0 += ITEMS) {
    const long long g = g0 + item;
    const bool valid = g < end;
    const long long gc = valid ? g : end - 1;
    const int i = (int)(gc >> per_inst_log2);
    const int rem = (int)(gc & ((1LL << per_inst_log2) - 1));
    const int z = rem >> tc_log2, tc = rem & (tcols - 1);
    const InstDev& I = inst[i];
    const bool active = valid && s < step_limit(I, max_steps);
    float2* __restrict__ base = psi + I.psi_off + (long long)z * slab + ((long long)(wv * tcols + tc) << 6) + lane;
    // first and last stages in FP64 (a forward transform ends, an inverse one starts,
    // in the concentrated coefficients)
    double2 in[P], out[P];
#pragma unroll
    for (int q = 0; q < P; ++q) assign(in[q], base[(long long)q * W * tcols * 64]);
    line_fft_io<NY, P, DIR, (W > 1)>(in, out, t, tw, my);
    if (active) {
#pragma unroll
      for (int q = 0; q < P; ++q) assign(base[(long long)q * W * tcols * 64], out[q]);
    }
    if constexpr (W == 1) wave_lds_sync();
  }
}

// ------------------------------------------------------------------------------------
// z-pass: the 64 lanes of a wavefront own the 64 (x, y) points of one 8x8 tile,
// wavefront w is row group t = w of every z-line, slot q holds z = w + q*W.  A line
// spans W wavefronts, so every exchange of its transform is a block barrier: 128-point
// lines take 16 points per lane (radices 16 and 8, one exchange per transform, eight
// wavefronts) instead of 8 (radices 8, 8, 2, two exchanges, sixteen wavefronts), which
// cuts the pass time by a quarter at the price of two waves per SIMD.

template <int NZ>
struct ZCfg {
  static constexpr int P = NZ >= 128 ? 16 : 8;
  static constexpr int W = NZ / P;  // wavefronts per block = lanes per line
  static constexpr int NT = W * 64;
  // line stride = 1 (mod 16) float2 slots: the 64 lines of a wavefront spread over the banks
  static constexpr int STRIDE = ((LineLds<NZ>::kSlots + 14) / 16) * 16 + 1;
};

template <int NZ>
__global__ void __launch_bounds__((ZCfg<NZ>::NT)) k_zpass_3d(
    const InstDev* __restrict__ inst, int ninst, int nx_log2, int ny_log2, float2* __restrict__ psi,
    const double2* __restrict__ twtab, int s, long long max_steps) {
  using C = ZCfg<NZ>;
  constexpr int P = C::P, W = C::W, STRIDE = C::STRIDE;
  __shared__ float2 lds[64 * STRIDE];
  __shared__ double2 ezl[NZ];  // E_z(k_z) / (nx ny nz) of the current instance and step
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int t = wave;
  float2* my = lds + lane * STRIDE;
  Twiddles<NZ, P> tw;
  tw.load(twtab, t);
  const int nx = 1 << nx_log2, ny = 1 << ny_log2;
  const int tx_log2 = nx_log2 - 3;
  const int tiles_log2 = tx_log2 + ny_log2 - 3;  // 8x8 tiles per slab
  const long long slab = (long long)nx * ny;
  const long long total = (long long)ninst << tiles_log2;
  const double inv_n = 1.0 / ((double)nx * (double)ny * (double)NZ);
  long long begin, end;
  block_share(total, 1, begin, end);
  double cached = -1.0;  // the block's item is one tile of one instance: cz is block-uniform
  for (long long g = begin; g < end; ++g) {
    const int i = (int)(g >> tiles_log2);
    const int tile = (int)(g & ((1LL << tiles_log2) - 1));
    const int tx = tile & ((1 << tx_log2) - 1), ty = tile >> tx_log2;
    const InstDev& I = inst[i];
    const bool active = s < step_limit(I, max_steps);
    double a, b;
    sched_ab(I, I.steps_done + s, a, b);
    const int x = tx * 8 + (lane & 7), y = ty * 8 + (lane >> 3);
    const int nxf = freq(x, nx), nyf = freq(y, ny);
    // kinetic phase in turns: a (pi dt / L_x^2 n_x^2 + pi dt / L_y^2 n_y^2 + pi dt / L_z^2 n_z^2)
    const double cxy = a * fma(I.kin_turns[0], (double)(nxf * nxf), I.kin_turns[1] * (double)(nyf * nyf));
    const double cz = a * I.kin_turns[2];
    if (cz != cached) {
      // K = E_xy E_z, separable: E_z once per coefficient into LDS, E_xy once per lane
      __syncthreads();  // the previous item's readers are done
      for (int k = threadIdx.x; k < NZ; k += C::NT) {
        const int nzf = freq(k, NZ);
        const double2 e = phase_turns_d(cz * (double)(nzf * nzf));
        ezl[k] = make_double2(e.x * inv_n, e.y * inv_n);
      }
      __syncthreads();
      cached = cz;
    }
    const double2 exy = phase_turns_d(cxy);
    float2* __restrict__ base = psi + I.psi_off + ((long long)tile << 6) + lane + (long long)t * slab;
    float2 reg[P];
#pragma unroll
    for (int q = 0; q < P; ++q) reg[q] = base[(long long)q * W * slab];
    double2 kd[P];
    line_fft_io<NZ, P, -1, (W > 1)>(reg, kd, t, tw, my);
#pragma unroll
    for (int q = 0; q < P; ++q) {
      const double2 ez = ezl[t + q * W];
      kd[q] = cmul_fd(kd[q], make_double2(fma(exy.x, ez.x, -exy.y * ez.y), fma(exy.x, ez.y, exy.y * ez.x)));
    }
    line_fft_io<NZ, P, +1, (W > 1)>(kd, reg, t, tw, my);
    if (active) {
#pragma unroll
      for (int q = 0; q < P; ++q) base[(long long)q * W * slab] = reg[q];
    }
    if constexpr (W > 1) __syncthreads();
  }
}

// ------------------------------------------------------------------------------------
// launchers

namespace {

inline int ilog2_3d(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

inline int blocks3d(long long items, int per_block, int cap) {
  long long b = (items + per_block - 1) / per_block;
  if (cap > 0 && b > cap) b = cap;
  return (int)(b < 1 ? 1 : b);
}

template <int NY, int DIR>
hipError_t launch_y(int nx, int nz, const InstDev* inst, int ninst, float2* psi, const double2* tw,
                    int s, long long max_steps, int cap, hipStream_t stream) {
  using C = YCfg<NY>;
  const int blocks = blocks3d((long long)ninst * (nx / 8) * nz, C::ITEMS, cap);
  hipLaunchKernelGGL((k_ypass_3d<NY, DIR>), dim3(blocks), dim3(C::NT), 0, stream, inst, ninst,
                     ilog2_3d(nx), ilog2_3d(nz), psi, tw, s, max_steps);
  return hipGetLastError();
}

template <int NZ>
hipError_t launch_z(int nx, int ny, const InstDev* inst, int ninst, float2* psi, const double2* tw,
                    int s, long long max_steps, int cap, hipStream_t stream) {
  using C = ZCfg<NZ>;
  const int blocks = blocks3d((long long)ninst * (nx / 8) * (ny / 8), 1, cap);
  hipLaunchKernelGGL((k_zpass_3d<NZ>), dim3(blocks), dim3(C::NT), 0, stream, inst, ninst,
                     ilog2_3d(nx), ilog2_3d(ny), psi, tw, s, max_steps);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_ypass_3d(int nx, int ny, int nz, int dir, const InstDev* inst, int ninst,
                           float2* psi, const double2* tw_y, int s, long long max_steps,
                           int grid_cap, hipStream_t stream) {
#define QHD_Y(NYV)                                                                              \
  case NYV:                                                                                     \
    return dir < 0 ? launch_y<NYV, -1>(nx, nz, inst, ninst, psi, tw_y, s, max_steps, grid_cap, stream) \
                   : launch_y<NYV, +1>(nx, nz, inst, ninst, psi, tw_y, s, max_steps, grid_cap, stream);
  switch (ny) {
    QHD_Y(16)
    QHD_Y(32)
    QHD_Y(64)
    QHD_Y(128)
    default:
      return hipErrorInvalidValue;
  }
#undef QHD_Y
}

hipError_t launch_zpass_3d(int nx, int ny, int nz, const InstDev* inst, int ninst, float2* psi,
                           const double2* tw_z, int s, long long max_steps, int grid_cap,
                           hipStream_t stream) {
  switch (nz) {
    case 16: return launch_z<16>(nx, ny, inst, ninst, psi, tw_z, s, max_steps, grid_cap, stream);
    case 32: return launch_z<32>(nx, ny, inst, ninst, psi, tw_z, s, max_steps, grid_cap, stream);
    case 64: return launch_z<64>(nx, ny, inst, ninst, psi, tw_z, s, max_steps, grid_cap, stream);
    case 128: return launch_z<128>(nx, ny, inst, ninst, psi, tw_z, s, max_steps, grid_cap, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace qhd
