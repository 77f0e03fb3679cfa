// 3-D passes with the line transforms as dense DFT products on the CDNA4 matrix
// cores (128^3 meshes), an alternative to the FP32 Stockham passes of
// qhd_kernels_3d.hip with the same four-pass step and the same state convention
// (App. C.2.1 eq. prod_qhd_fft / App. E.1 with F = F_z F_y F_x):
//   x-pass  F_x . V . F_x^{-1}      y-pass  F_y       z-pass  F_z^{-1} . K . F_z      y-pass  F_y^{-1}
//
// A work item is a group of 32 lines of one axis.  The group is staged in LDS as
// split FP16 operands: each line is scaled by a power of two 2^e (its largest
// component then lies in [1/2, 1)) and every component v is stored as two terms,
// x0 = fp16(v 2^-e) and x1 = fp16((v 2^-e - x0) 2^12) (the second term scaled up so that
// it stays in FP16's normal range).  The DFT matrix W_jk = e^{-+2 pi i jk / 128} has only
// 128 distinct entries, w(m) with m = jk mod 128; each is written as three terms
// w = w0 + 2^-12 w1 + 2^-24 w2 (each FP16, normal range), a table of 4 KB that every
// workgroup keeps in LDS and from which a lane gathers its MFMA operand entries.  The
// products run on v_mfma_f32_32x32x16_f16 with FP32 accumulation in three accumulators
// by scale:
//     a0 = w0 x0,   a1 = w0 x1 + w1 x0,   a2 = w2 x0,    W X = a0 + 2^-12 a1 + 2^-24 a2.
// The terms left out (w1 x1, w2 x1 and beyond) are at most ~2^-24 of the result and
// carry the rounding residual x1 of the data, whose sign varies from point to point;
// every term that carries W's own residual is kept, since that one repeats identically
// on every transform: with W represented to 2^-22 only (two terms), its error drained the
// norm systematically, ~2e-8 per step on 128^3.
//
#include "line_fft.h"
#include "pass_common.h"
#include "qhd_internal.h"

namespace qhd {

namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kN = 128;                    // points per line (every axis)
constexpr int kLines = 32;                 // lines per work item
constexpr int kGroups = kN * kN / kLines;  // work items per instance and axis
constexpr int kPitch = kN + 8;             // FP16 row pitch in LDS (272 bytes)
constexpr int kYPitch = kN + 1;            // float2 row pitch of the output staging
constexpr long long kSlab = (long long)kN * kN;
constexpr float kLoScale = 4096.0f;        // 2^12: scale of the second operand term

// element offset (instance-relative) of point k of line n in group g
template <int AXIS>
__device__ __forceinline__ long long line_off(int g, int n, int k) {
  if constexpr (AXIS == 0) {  // x-lines: g = (z/4, y/8); n = (z&3, y&7); 8x8-tiled slabs
    const int ty = g & 15, zq = g >> 4;
    const int z = zq * 4 + (n >> 3);
    return z * kSlab + (long long)ty * (16 * 64) + (n & 7) * 8 + (k >> 3) * 64 + (k & 7);
  } else if constexpr (AXIS == 1) {  // y-lines: g = (z, x/32); n = x & 31
    const int xq = g & 3, z = g >> 2;
    const int x = xq * 32 + n;
    return z * kSlab + (x >> 3) * 64 + (x & 7) + (long long)(k >> 3) * (16 * 64) + (k & 7) * 8;
  } else {  // z-lines: g = (tile, half); n = position - 32 half within the 8x8 tile
    const int half = g & 1, tile = g >> 1;
    return (long long)k * kSlab + tile * 64 + half * 32 + n;
  }
}

// load mapping: thread -> (line, first point); each thread moves 16 points of one line
template <int AXIS>
__device__ __forceinline__ void load_map(int tid, int& n, int& k0) {
  if constexpr (AXIS == 0) {  // 8 threads per line: 64-byte runs along x
    n = tid >> 3;
    k0 = (tid & 7) * 16;
  } else {  // consecutive threads take consecutive lines (adjacent in memory)
    n = tid & 31;
    k0 = (tid >> 5) * 16;
  }
}

__device__ __forceinline__ int scale_exp(unsigned bits) {
  const float m = __uint_as_float(bits);
  int e = 0;
  if (m > 0.0f) (void)frexpf(m, &e);  // m = f 2^e, f in [1/2, 1)
  return e;
}

// operand planes in LDS: [re x0, re x1, im x0, im x1][line][k]
__device__ __forceinline__ void split_store(_Float16* xs, int n, int k, float2 v, int e) {
  const float vr = ldexpf(v.x, -e), vi = ldexpf(v.y, -e);
  const _Float16 rh = (_Float16)vr, ih = (_Float16)vi;
  xs[(0 * kLines + n) * kPitch + k] = rh;
  xs[(1 * kLines + n) * kPitch + k] = (_Float16)((vr - (float)rh) * kLoScale);
  xs[(2 * kLines + n) * kPitch + k] = ih;
  xs[(3 * kLines + n) * kPitch + k] = (_Float16)((vi - (float)ih) * kLoScale);
}

__device__ __forceinline__ half8 neg8(half8 v) {
  // flip the sign bits (exact)
  uint4 u = __builtin_bit_cast(uint4, v);
  u.x ^= 0x80008000u;
  u.y ^= 0x80008000u;
  u.z ^= 0x80008000u;
  u.w ^= 0x80008000u;
  return __builtin_bit_cast(half8, u);
}

// W table entry m of one sign: (re w0, re w1, re w2, im w0, im w1, im w2, 0, 0)
struct WEntry {
  _Float16 v[8];
};

// (real, imaginary) of W X for this wavefront's 32 rows as the three scaled
// accumulators; wt = the 128-entry table of W's sign (LDS)
__device__ __forceinline__ void dft_gemm(const WEntry* wt, const _Float16* xs, int wave, int lane, f32x16 (&ar)[3],
                                         f32x16 (&ai)[3]) {
  const int row = 32 * wave + (lane & 31), h = lane >> 5, n = lane & 31;
  const _Float16* xrow = xs + n * kPitch + 8 * h;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    ar[c] = f32x16{};
    ai[c] = f32x16{};
  }
#pragma unroll 2
  for (int kk = 0; kk < kN / 16; ++kk) {
    // this lane's A operand: row `row`, k = 16 kk + 8 h + i, entries w((row k) mod 128)
    half8 w0r, w1r, w2r, w0i, w1i, w2i;
    const int kb = 16 * kk + 8 * h;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const WEntry e = wt[(row * (kb + i)) & (kN - 1)];
      w0r[i] = e.v[0];
      w1r[i] = e.v[1];
      w2r[i] = e.v[2];
      w0i[i] = e.v[3];
      w1i[i] = e.v[4];
      w2i[i] = e.v[5];
    }
    const half8 xr0 = *reinterpret_cast<const half8*>(xrow + 0 * kLines * kPitch + 16 * kk);
    const half8 xr1 = *reinterpret_cast<const half8*>(xrow + 1 * kLines * kPitch + 16 * kk);
    const half8 xi0 = *reinterpret_cast<const half8*>(xrow + 2 * kLines * kPitch + 16 * kk);
    const half8 xi1 = *reinterpret_cast<const half8*>(xrow + 3 * kLines * kPitch + 16 * kk);
    const half8 nxi0 = neg8(xi0), nxi1 = neg8(xi1);
    // Re: Wr Xr - Wi Xi ; Im: Wr Xi + Wi Xr
    ar[0] = __builtin_amdgcn_mfma_f32_32x32x16_f16(w0r, xr0, ar[0], 0, 0, 0);
    ar[0] = __builtin_amdgcn_mfma_f32_32x32x16_f16(w0i, nxi0, ar[0], 0, 0, 0);
    ar[1] = __builtin_amdgcn_mfma_f32_32x32x16_f16(w0r, xr1, ar[1], 0, 0, 0);
    ar[1] = __builtin_amdgcn_mfma_f32_32x32x16_f16(w0i, nxi1, ar[1], 0, 0, 0);
    ar[1] = __builtin_amdgcn_mfma_f32_32x32x16_f16(w1r, xr0, ar[1], 0, 0, 0);
    ar[1] = __builtin_amdgcn_mfma_f32_32x32x16_f16(w1i, nxi0, ar[1], 0, 0, 0);
    ar[2] = __builtin_amdgcn_mfma_f32_32x32x16_f16(w2r, xr0, ar[2], 0, 0, 0);
    ar[2] = __builtin_amdgcn_mfma_f32_32x32x16_f16(w2i, nxi0, ar[2], 0, 0, 0);
    ai[0] = __builtin_amdgcn_mfma_f32_32x32x16_f16(w0r, xi0, ai[0], 0, 0, 0);
    ai[0] = __builtin_amdgcn_mfma_f32_32x32x16_f16(w0i, xr0, ai[0], 0, 0, 0);
    ai[1] = __builtin_amdgcn_mfma_f32_32x32x16_f16(w0r, xi1, ai[1], 0, 0, 0);
    ai[1] = __builtin_amdgcn_mfma_f32_32x32x16_f16(w0i, xr1, ai[1], 0, 0, 0);
    ai[1] = __builtin_amdgcn_mfma_f32_32x32x16_f16(w1r, xi0, ai[1], 0, 0, 0);
    ai[1] = __builtin_amdgcn_mfma_f32_32x32x16_f16(w1i, xr0, ai[1], 0, 0, 0);
    ai[2] = __builtin_amdgcn_mfma_f32_32x32x16_f16(w2r, xi0, ai[2], 0, 0, 0);
    ai[2] = __builtin_amdgcn_mfma_f32_32x32x16_f16(w2i, xr0, ai[2], 0, 0, 0);
  }
}

// register r of the combined product a0 + 2^-12 a1 + 2^-24 a2 (FP32)
__device__ __forceinline__ float combine(const f32x16 (&a)[3], int r) {
  return fmaf(a[2][r], 0x1p-24f, fmaf(a[1][r], 0x1p-12f, a[0][r]));
}

// output row of accumulator register r
__device__ __forceinline__ int acc_row(int wave, int lane, int r) {
  return 32 * wave + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
}

// MODE 0: Y = W_dir X (y-pass).  MODE 1: x-pass F_x V F_x^{-1} (the first product
// is skipped on the entry step, where the state is in position space).  MODE 2:
// z-pass F_z^{-1} K F_z.  tables: [sign][128] W entries, sign 0 = e^{-i..}.
template <int AXIS, int MODE>
__global__ void __launch_bounds__(256) k_mfma_pass_3d(const InstDev* __restrict__ inst, const int* __restrict__ nact_p,
                                                      const WEntry* __restrict__ tables,
                                                      float2* __restrict__ psi, const double* __restrict__ f,
                                                      int dir, int s, long long max_steps) {
  const int ninst = *nact_p;  // members active in this sub-step (device, set per chunk)
  __shared__ __attribute__((aligned(16))) _Float16 xs[4 * kLines * kPitch];
  __shared__ unsigned smax[2][kLines];
  float2* ys = reinterpret_cast<float2*>(xs);  // output staging, aliases the operands
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ WEntry wl[2 * kN];  // both signs of the W table
  for (int e = threadIdx.x; e < 2 * kN; e += blockDim.x) wl[e] = tables[e];
  __syncthreads();
  const WEntry* wfwd = wl;
  const WEntry* winv = wl + kN;
  const long long total = (long long)ninst * kGroups;
  long long begin, end;
  block_share(total, 1, begin, end);
  int n_ld, k0;
  load_map<AXIS>(tid, n_ld, k0);
  const int n_acc = lane & 31;
  for (long long gi = begin; gi < end; ++gi) {
    const int i = (int)(gi / kGroups), g = (int)(gi - (long long)i * kGroups);
    const InstDev& I = inst[i];
    if (!(s < step_limit(I, max_steps))) continue;  // block-uniform
    const long long j = I.steps_done + s;
    double a, b;
    sched_ab(I, j, a, b);
    const bool entry = MODE == 1 && s == 0 && I.mode == kModeClean;
    const double cpot = MODE == 1 ? potential_turns(I, j, entry) : 0.0;
    float2* __restrict__ pl = psi + I.psi_off;
    const double* __restrict__ fl = f + I.psi_off;
    if (tid < 2 * kLines) smax[tid >> 5][tid & 31] = 0u;
    __syncthreads();
    // ---- load 16 points of one line, per-line scale, split into FP16 hi/lo
    float2 v[16];
    float m = 0.0f;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const long long off = line_off<AXIS>(g, n_ld, k0 + q);
      v[q] = pl[off];
      if constexpr (MODE == 1) {
        if (entry) v[q] = cmul_fd(v[q], phase_turns_d(cpot * fl[off]));
      }
      m = fmaxf(m, fmaxf(fabsf(v[q].x), fabsf(v[q].y)));
    }
    atomicMax(&smax[0][n_ld], __float_as_uint(m));
    __syncthreads();
    {
      const int e = scale_exp(smax[0][n_ld]);
#pragma unroll
      for (int q = 0; q < 16; ++q) split_store(xs, n_ld, k0 + q, v[q], e);
    }
    __syncthreads();
    f32x16 ar[3], ai[3];
    float pr[16], pi[16];
    int e_acc = scale_exp(smax[0][n_acc]);
    if (MODE == 2 || (MODE == 1 && !entry)) {
      // ---- first product, phase, re-split
      dft_gemm(MODE == 1 ? winv : wfwd, xs, wave, lane, ar, ai);
      float mm = 0.0f;
      if constexpr (MODE == 1) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int k = acc_row(wave, lane, r);
          const float2 y = make_float2(ldexpf(combine(ar, r), e_acc), ldexpf(combine(ai, r), e_acc));
          const float2 z = cmul_fd(y, phase_turns_d(cpot * fl[line_off<AXIS>(g, n_acc, k)]));
          pr[r] = z.x;
          pi[r] = z.y;
          mm = fmaxf(mm, fmaxf(fabsf(z.x), fabsf(z.y)));
        }
      } else {
        // kinetic factor E_x E_y E_z / (nx ny nz) at (k_x, k_y) of the line and k_z = row
        const int p = ((g & 1) << 5) + n_acc, tile = g >> 1;
        const int x = (tile & 15) * 8 + (p & 7), y = (tile >> 4) * 8 + (p >> 3);
        const int nxf = freq(x, kN), nyf = freq(y, kN);
        const double cxy = a * fma(I.kin_turns[0], (double)(nxf * nxf), I.kin_turns[1] * (double)(nyf * nyf));
        const double cz = a * I.kin_turns[2];
        const double inv_n = 1.0 / ((double)kN * kN * kN);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int nzf = freq(acc_row(wave, lane, r), kN);
          const double2 kf = phase_turns_d(fma(cz, (double)(nzf * nzf), cxy));
          const float2 y2 = make_float2(ldexpf(combine(ar, r), e_acc), ldexpf(combine(ai, r), e_acc));
          const float2 z = cmul_fd(y2, make_double2(kf.x * inv_n, kf.y * inv_n));
          pr[r] = z.x;
          pi[r] = z.y;
          mm = fmaxf(mm, fmaxf(fabsf(z.x), fabsf(z.y)));
        }
      }
      atomicMax(&smax[1][n_acc], __float_as_uint(mm));
      __syncthreads();  // every wavefront has finished reading the operands
      e_acc = scale_exp(smax[1][n_acc]);
#pragma unroll
      for (int r = 0; r < 16; ++r)
        split_store(xs, n_acc, acc_row(wave, lane, r), make_float2(pr[r], pi[r]), e_acc);
      __syncthreads();
    }
    // ---- final product
    const WEntry* wlast = MODE == 0 ? (dir < 0 ? wfwd : winv) : (MODE == 1 ? wfwd : winv);
    dft_gemm(wlast, xs, wave, lane, ar, ai);
    __syncthreads();  // operands no longer needed: stage the output in the same LDS
#pragma unroll
    for (int r = 0; r < 16; ++r)
      ys[n_acc * kYPitch + acc_row(wave, lane, r)] =
          make_float2(ldexpf(combine(ar, r), e_acc), ldexpf(combine(ai, r), e_acc));
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) pl[line_off<AXIS>(g, n_ld, k0 + q)] = ys[n_ld * kYPitch + k0 + q];
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_mfma_pass_3d(int axis, int dir, const InstDev* inst, int ninst, const int* nact, const void* tables,
                               float2* psi, const double* f, int s, long long max_steps, int grid_cap,
                               hipStream_t stream) {
  long long items = (long long)ninst * kGroups;
  if (grid_cap > 0 && items > grid_cap) items = grid_cap;
  const dim3 grid((unsigned)items), block(256);
  const WEntry* t = static_cast<const WEntry*>(tables);
  if (axis == 0)
    QHD_LAUNCH((k_mfma_pass_3d<0, 1>), grid, block, 0, stream, inst, nact, t, psi, f, dir, s, max_steps);
  else if (axis == 1)
    QHD_LAUNCH((k_mfma_pass_3d<1, 0>), grid, block, 0, stream, inst, nact, t, psi, f, dir, s, max_steps);
  else if (axis == 2)
    QHD_LAUNCH((k_mfma_pass_3d<2, 2>), grid, block, 0, stream, inst, nact, t, psi, f, dir, s, max_steps);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace qhd
