// Kernels of the spectrum entry point: the matrix-vector product
//     H(t) v = a(t) F^{-1} diag(|k|^2/2) F v + b(t) f v
// (the Fourier-diagonal kinetic operator of the split-operator scheme, App. C.2.1
// eq. prod_qhd_fft) on a plain row-major (x fastest) complex64 vector of one 2-D
// instance, and the Krylov vector operations of the Lanczos iteration.
#include <hip/hip_runtime.h>

#include "line_fft.h"
#include "pass_common.h"
#include "qhd_internal.h"

namespace qhd {

namespace {

template <int N>
constexpr int spec_p() { return N >= 1024 ? 16 : (N >= 8 ? 8 : N); }

// lines along x: line y is v[y*N .. y*N+N); one line per TPL lanes
template <int N, int S>
__global__ void __launch_bounds__(256) k_spec_rows(float2* __restrict__ v, int nlines, const double2* __restrict__ twtab) {
  constexpr int P = spec_p<N>(), TPL = N / P;
  constexpr int LPW = 256 / TPL;
  constexpr int SLOTS = LineLds<N>::kSlots;
  __shared__ float2 lds[LPW * SLOTS];
  const int ll = threadIdx.x / TPL, t = threadIdx.x % TPL;
  float2* my = lds + ll * SLOTS;
  Twiddles<N, P> tw;
  tw.load(twtab, t);
  for (long long l0 = (long long)blockIdx.x * LPW; l0 < nlines; l0 += (long long)gridDim.x * LPW) {
    const long long L = l0 + ll;
    const bool valid = L < nlines;
    float2* __restrict__ line = v + (valid ? L : 0) * N;
    float2 reg[P];
#pragma unroll
    for (int q = 0; q < P; ++q) reg[q] = line[t + q * TPL];
    line_fft<N, P, S>(reg, t, tw, my);
    if (valid) {
#pragma unroll
      for (int q = 0; q < P; ++q) line[t + q * TPL] = reg[q];
    }
  }
}

// lines along y (stride nx): LPW adjacent columns per block, lane order (t, column) so
// that a slot access of consecutive threads touches consecutive columns; a line spans
// several wavefronts, so the exchanges take block barriers
template <int N, int S>
__global__ void __launch_bounds__(256) k_spec_cols(float2* __restrict__ v, int nx, const double2* __restrict__ twtab) {
  constexpr int P = spec_p<N>(), TPL = N / P;
  constexpr int LPW = 256 / TPL;
  constexpr int SLOTS = LineLds<N>::kSlots;
  __shared__ float2 lds[LPW * SLOTS];
  const int ll = threadIdx.x % LPW, t = threadIdx.x / LPW;
  float2* my = lds + ll * SLOTS;
  Twiddles<N, P> tw;
  tw.load(twtab, t);
  for (long long c0 = (long long)blockIdx.x * LPW; c0 < nx; c0 += (long long)gridDim.x * LPW) {
    const long long x = c0 + ll;
    const bool valid = x < nx;
    float2* __restrict__ col = v + (valid ? x : 0);
    float2 reg[P];
#pragma unroll
    for (int q = 0; q < P; ++q) reg[q] = col[(long long)(t + q * TPL) * nx];
    line_fft<N, P, S, true>(reg, t, tw, my);
    if (valid) {
#pragma unroll
      for (int q = 0; q < P; ++q) col[(long long)(t + q * TPL) * nx] = reg[q];
    }
    __syncthreads();
  }
}

// v <- v * a (|k|^2 / 2) / (nx ny), |k|^2 = (2 pi n_x / L_x)^2 + (2 pi n_y / L_y)^2
__global__ void k_spec_kinetic(float2* __restrict__ v, int nx, int ny, double cx, double cy, double s) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)nx * ny) return;
  const int x = (int)(e % nx), y = (int)(e / nx);
  const int fx = freq(x, nx), fy = freq(y, ny);
  const double m = s * fma(cx, (double)fx * fx, cy * (double)fy * fy);
  const float2 w = v[e];
  v[e] = make_float2((float)(m * w.x), (float)(m * w.y));
}

// out = w + b f v, f read from the plan's 8x8-tiled FP64 copy
__global__ void k_spec_finish(float2* __restrict__ out, const float2* __restrict__ w, const float2* __restrict__ v,
                              const double* __restrict__ f, double b, int nx, int ny) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)nx * ny) return;
  const int x = (int)(e % nx), y = (int)(e / nx);
  const double bf = b * f[tile_index(x, y, nx)];
  const float2 a = w[e], c = v[e];
  out[e] = make_float2((float)(a.x + bf * c.x), (float)(a.y + bf * c.y));
}

// partials[(i * nblk + block) * 2 + {0,1}] = block's share of <V_i, w> (conj on V_i), FP64
__global__ void __launch_bounds__(256) k_spec_multidot(const float2* __restrict__ V, long long n, int count,
                                                       const float2* __restrict__ w, double* __restrict__ partials) {
  __shared__ double sr[256], si[256];
  const int i = blockIdx.y;
  const float2* __restrict__ vi = V + (long long)i * n;
  double ar = 0.0, ai = 0.0;
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
    const float2 a = vi[e], c = w[e];
    ar += (double)a.x * c.x + (double)a.y * c.y;
    ai += (double)a.x * c.y - (double)a.y * c.x;
  }
  sr[threadIdx.x] = ar;
  si[threadIdx.x] = ai;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      sr[threadIdx.x] += sr[threadIdx.x + o];
      si[threadIdx.x] += si[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partials[((long long)i * gridDim.x + blockIdx.x) * 2 + 0] = sr[0];
    partials[((long long)i * gridDim.x + blockIdx.x) * 2 + 1] = si[0];
  }
}

// coef[2 i + {0,1}] = sum over the nblk block partials of <V_i, w>, in block order (the
// same FP64 additions in the same order as a host-side sum); when `keep` is set,
// keep[0] = coef[2 (count - 1)] (the Lanczos diagonal entry of the newest vector)
__global__ void k_spec_coef(const double* __restrict__ partials, int count, int nblk, double* __restrict__ coef,
                            double* __restrict__ keep) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 2 * count) return;
  const int i = k >> 1, c = k & 1;
  double acc = 0.0;
  for (int b = 0; b < nblk; ++b) acc += partials[((long long)i * nblk + b) * 2 + c];
  coef[k] = acc;
  if (keep && k == 2 * (count - 1)) keep[0] = acc;
}

// norm of one vector from its <y, y> partials: keep[0] = sqrt(max(sum, 0)), and
// scale[0] = 1 / that (the factor of the normalising multiaxpy)
__global__ void k_spec_norm(const double* __restrict__ partials, int nblk, double* __restrict__ keep,
                            double* __restrict__ scale) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double acc = 0.0;
  for (int b = 0; b < nblk; ++b) acc += partials[2 * b];
  const double nrm = sqrt(acc > 0.0 ? acc : 0.0);
  keep[0] = nrm;
  scale[0] = 1.0 / nrm;
}

// w <- scale (w - sum_i c_i V_i), c_i complex (FP64, device copy); the scale from
// device memory when scale_dev is given
__global__ void k_spec_multiaxpy(float2* __restrict__ w, const float2* __restrict__ V, long long n, int count,
                                 const double* __restrict__ c, double scale_host, const double* __restrict__ scale_dev) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const double scale = scale_dev ? scale_dev[0] : scale_host;
  double xr = w[e].x, xi = w[e].y;
  for (int i = 0; i < count; ++i) {
    const float2 a = V[(long long)i * n + e];
    const double cr = c[2 * i], ci = c[2 * i + 1];
    xr -= cr * a.x - ci * a.y;
    xi -= cr * a.y + ci * a.x;
  }
  w[e] = make_float2((float)(scale * xr), (float)(scale * xi));
}

// Grouped form of the same update for long bases: group g of the grid's y dimension
// sums c_i V_i over its share of i into part[g] (FP64), then k_spec_axpy_fin subtracts
// the groups' sums in group order.  One thread per element and group instead of one per
// element gives the loads of a 16 K-point vector enough waves to be in flight.
__global__ void k_spec_axpy_part(const float2* __restrict__ V, long long n, int count, const double* __restrict__ c,
                                 double2* __restrict__ part) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int g = blockIdx.y, groups = gridDim.y;
  const int per = (count + groups - 1) / groups;
  const int i0 = g * per, i1 = min(count, i0 + per);
  double xr = 0.0, xi = 0.0;
  for (int i = i0; i < i1; ++i) {
    const float2 a = V[(long long)i * n + e];
    const double cr = c[2 * i], ci = c[2 * i + 1];
    xr += cr * a.x - ci * a.y;
    xi += cr * a.y + ci * a.x;
  }
  part[(long long)g * n + e] = make_double2(xr, xi);
}

__global__ void k_spec_axpy_fin(float2* __restrict__ w, long long n, const double2* __restrict__ part, int groups,
                                double scale) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double xr = w[e].x, xi = w[e].y;
  for (int g = 0; g < groups; ++g) {
    const double2 p = part[(long long)g * n + e];
    xr -= p.x;
    xi -= p.y;
  }
  w[e] = make_float2((float)(scale * xr), (float)(scale * xi));
}

// deterministic start vector from a counter-based hash (splitmix64 of the index)
__global__ void k_spec_random(float2* __restrict__ v, long long n, unsigned long long seed) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  unsigned long long z = seed + 0x9E3779B97F4A7C15ull * (unsigned long long)(e + 1);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  const float r = (float)((z >> 40) * (1.0 / 16777216.0)) - 0.5f;
  const float i = (float)((z & 0xFFFFFF) * (1.0 / 16777216.0)) - 0.5f;
  v[e] = make_float2(r, i);
}

inline unsigned grid1(long long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t spec_lines(int axis, int sign, float2* v, int nx, int ny, const double2* tw, hipStream_t st) {
  const int n = axis == 0 ? nx : ny;
#define QHD_SPEC(N_)                                                                                         \
  case N_: {                                                                                                 \
    constexpr int TPL = N_ / spec_p<N_>(), LPW = 256 / TPL;                                                  \
    if (axis == 0) {                                                                                         \
      const unsigned blocks = (unsigned)((ny + LPW - 1) / LPW);                                              \
      if (sign < 0) hipLaunchKernelGGL((k_spec_rows<N_, -1>), dim3(blocks), dim3(256), 0, st, v, ny, tw);    \
      else hipLaunchKernelGGL((k_spec_rows<N_, +1>), dim3(blocks), dim3(256), 0, st, v, ny, tw);             \
    } else {                                                                                                 \
      const unsigned blocks = (unsigned)((nx + LPW - 1) / LPW);                                              \
      if (sign < 0) hipLaunchKernelGGL((k_spec_cols<N_, -1>), dim3(blocks), dim3(256), 0, st, v, nx, tw);    \
      else hipLaunchKernelGGL((k_spec_cols<N_, +1>), dim3(blocks), dim3(256), 0, st, v, nx, tw);             \
    }                                                                                                        \
    return hipGetLastError();                                                                                \
  }
  switch (n) {
    QHD_SPEC(8)
    QHD_SPEC(16)
    QHD_SPEC(32)
    QHD_SPEC(64)
    QHD_SPEC(128)
    QHD_SPEC(256)
    QHD_SPEC(512)
    QHD_SPEC(1024)
    default:
      return hipErrorInvalidValue;
  }
#undef QHD_SPEC
}

hipError_t spec_kinetic(float2* v, int nx, int ny, double cx, double cy, double s, hipStream_t st) {
  hipLaunchKernelGGL(k_spec_kinetic, dim3(grid1((long long)nx * ny)), dim3(256), 0, st, v, nx, ny, cx, cy, s);
  return hipGetLastError();
}

hipError_t spec_finish(float2* out, const float2* w, const float2* v, const double* f, double b, int nx, int ny,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_spec_finish, dim3(grid1((long long)nx * ny)), dim3(256), 0, st, out, w, v, f, b, nx, ny);
  return hipGetLastError();
}

hipError_t spec_multidot(const float2* V, long long n, int count, const float2* w, double* partials, int nblk,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_spec_multidot, dim3(nblk, count), dim3(256), 0, st, V, n, count, w, partials);
  return hipGetLastError();
}

hipError_t spec_multiaxpy(float2* w, const float2* V, long long n, int count, const double* c, double scale,
                          hipStream_t st, const double* scale_dev, double2* part, int groups) {
  if (part && groups > 1 && count >= 2 * groups && !scale_dev) {
    hipLaunchKernelGGL(k_spec_axpy_part, dim3(grid1(n), groups), dim3(256), 0, st, V, n, count, c, part);
    hipLaunchKernelGGL(k_spec_axpy_fin, dim3(grid1(n)), dim3(256), 0, st, w, n, part, groups, scale);
  } else {
    hipLaunchKernelGGL(k_spec_multiaxpy, dim3(grid1(n)), dim3(256), 0, st, w, V, n, count, c, scale, scale_dev);
  }
  return hipGetLastError();
}

hipError_t spec_coef(const double* partials, int count, int nblk, double* coef, double* keep, hipStream_t st) {
  hipLaunchKernelGGL(k_spec_coef, dim3((unsigned)((2 * count + 255) / 256)), dim3(256), 0, st, partials, count, nblk,
                     coef, keep);
  return hipGetLastError();
}

hipError_t spec_norm(const double* partials, int nblk, double* keep, double* scale, hipStream_t st) {
  hipLaunchKernelGGL(k_spec_norm, dim3(1), dim3(64), 0, st, partials, nblk, keep, scale);
  return hipGetLastError();
}

hipError_t spec_random(float2* v, long long n, unsigned long long seed, hipStream_t st) {
  hipLaunchKernelGGL(k_spec_random, dim3(grid1(n)), dim3(256), 0, st, v, n, seed);
  return hipGetLastError();
}

}  // namespace qhd
