// Kernels of the relaxed QHD for box-constrained QP (App. F.2, eq.
// relaxed-qhd-discrete; Algorithm 2): the state lives on the (r+1)^d lattice
// (NP = r + 1 points per axis, axis 1 fastest), one FP32 complex value per point.
//
// A step of the symmetric product is d axis passes.  Pass k multiplies every line
// along axis k by the same NP x NP complex matrix
//     M = U diag(e^{i theta lambda_m}) U^T,   theta = dt a r^2 / 2,
// the exact kinetic factor exp(+i theta A') of one axis (A' = U diag(lambda) U^T);
// the factors of different axes commute, so their product is the kinetic factor of
// A'_d.  The first pass also applies the potential factor exp(-i beta f) (the merged
// half steps) to each point before its line is transformed.  M is formed in FP64 once
// per step by a one-block kernel into a small global buffer; the passes read it with
// wave-uniform (scalar) loads, so the matrix costs no LDS or VGPR bandwidth, and lines
// accumulate in FP64 and round once on store.
//
// Lines of stride s < 64 (axes 1, 2 and, for small NP, a few more) are staged through
// LDS so that global accesses are contiguous; lines of stride >= 64 are read directly
// (consecutive threads own consecutive lines, i.e. consecutive addresses).
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>

#include "line_fft.h"
#include "rqp_internal.h"

namespace qhd {

namespace {

constexpr int kThreads = 256;

// M[m][n] = sum_k U[m][k] e^{i theta lam_k} U[n][k] into global memory (one block)
template <int NP>
__global__ void __launch_bounds__(kThreads) k_rqp_matrix(const double* __restrict__ U, const double* __restrict__ lam,
                                                        double theta, double2* __restrict__ M) {
  __shared__ double2 ph[NP];
  if (threadIdx.x < NP) {
    double s, c;
    sincos(theta * lam[threadIdx.x], &s, &c);
    ph[threadIdx.x] = make_double2(c, s);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < NP * NP; e += blockDim.x) {
    const int m = e / NP, n = e - m * NP;
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      const double w = U[m * NP + k] * U[n * NP + k];
      re = fma(w, ph[k].x, re);
      im = fma(w, ph[k].y, im);
    }
    M[e] = make_double2(re, im);
  }
}

// A wave-uniform zero the compiler cannot see through (no memory access).  Offsetting
// the matrix by it once per line keeps the matrix reads (scalar loads, the same entry for
// every lane) inside the line loops: hoisted out of them, the NP^2 FP64 complex entries
// would sit in vector registers (~400 VGPRs and 140 AGPRs at NP = 9, one wave per SIMD).
__device__ __forceinline__ int opaque_zero() {
  int z;
  asm volatile("s_mov_b32 %0, 0" : "=s"(z));
  return z;
}

// y = M x for one line, FP64; M in global memory, read wave-uniformly
template <int NP>
__device__ __forceinline__ void line_apply(const double2* __restrict__ Mg, const double2 (&x)[NP], double2 (&y)[NP]) {
  const double2* __restrict__ M = Mg + opaque_zero();
#pragma unroll
  for (int m = 0; m < NP; ++m) {
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int n = 0; n < NP; ++n) {
      const double2 w = M[m * NP + n];
      re = fma(w.x, x[n].x, fma(-w.y, x[n].y, re));
      im = fma(w.x, x[n].y, fma(w.y, x[n].x, im));
    }
    y[m] = make_double2(re, im);
  }
}

// Staged pass: the block owns lines [blockIdx * LB, ...) of stride s (LB a multiple of
// s), i.e. the contiguous points [blockIdx * LB * NP, ...).
template <int NP, bool FUSE_V>
__global__ void __launch_bounds__(kThreads) k_rqp_axis_staged(float2* __restrict__ psi, const double* __restrict__ f,
                                                             long long total_points, int s, int LB,
                                                             const double2* __restrict__ Ml, double beta_turns) {
  __shared__ float2 seg[kThreads * NP];
  const long long p0 = (long long)blockIdx.x * LB * NP;
  const int npts = (int)((total_points - p0 < (long long)LB * NP) ? total_points - p0 : (long long)LB * NP);
  for (int e = threadIdx.x; e < npts; e += kThreads) {
    float2 v = psi[p0 + e];
    if constexpr (FUSE_V) v = cmul_fd(v, phase_turns_d(beta_turns * f[p0 + e]));
    seg[e] = v;
  }
  __syncthreads();
  const int line = threadIdx.x;
  if (line < LB && line * NP < npts) {
    // line -> (outer chunk, inner offset) within the segment
    const int outer = line / s, inner = line - outer * s;
    const int base = outer * s * NP + inner;
    double2 x[NP], y[NP];
#pragma unroll
    for (int m = 0; m < NP; ++m) assign(x[m], seg[base + m * s]);
    line_apply<NP>(Ml, x, y);
#pragma unroll
    for (int m = 0; m < NP; ++m) assign(seg[base + m * s], y[m]);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < npts; e += kThreads) psi[p0 + e] = seg[e];
}

// Fused pass: axes 1..K at once.  A chunk is the NP^K contiguous points that share the
// indices of axes K+1..d; a block holds a run of whole chunks in LDS (at most
// kFusedPoints points), applies the potential factor on load, then the matrix along
// axis 1, 2, ..., K with a barrier between axes, and stores once.  Each axis rounds to
// FP32 on its LDS store exactly as a separate pass rounds on its HBM store, so the
// values are those of K separate passes, for 16 B of HBM traffic per point instead of
// 16 K.  (9^4 points: 52.5 KB, three blocks per CU.)
template <int NP>
__global__ void __launch_bounds__(kThreads) k_rqp_fused(float2* __restrict__ psi, const double* __restrict__ f,
                                                       long long total_points, int K, int run,
                                                       const double2* __restrict__ Ml, double beta_turns) {
  __shared__ float2 seg[kFusedPoints];
  for (long long p0 = (long long)blockIdx.x * run; p0 < total_points; p0 += (long long)gridDim.x * run) {
    // total_points and run are whole numbers of chunks, so every run holds whole lines
    const int npts = (int)((total_points - p0 < (long long)run) ? total_points - p0 : (long long)run);
    for (int e = threadIdx.x; e < npts; e += kThreads)
      seg[e] = cmul_fd(psi[p0 + e], phase_turns_d(beta_turns * f[p0 + e]));
    __syncthreads();
    const int lines = npts / NP;
    int s = 1;
    for (int k = 0; k < K; ++k) {
      for (int line = threadIdx.x; line < lines; line += kThreads) {
        const int outer = line / s, inner = line - outer * s;
        const int base = outer * s * NP + inner;
        double2 x[NP], y[NP];
#pragma unroll
        for (int m = 0; m < NP; ++m) assign(x[m], seg[base + m * s]);
        line_apply<NP>(Ml, x, y);
#pragma unroll
        for (int m = 0; m < NP; ++m) assign(seg[base + m * s], y[m]);
      }
      __syncthreads();
      s *= NP;
    }
    for (int e = threadIdx.x; e < npts; e += kThreads) psi[p0 + e] = seg[e];
    __syncthreads();  // the next run reuses the LDS
  }
}

// Direct pass for strides >= 64: thread = line.
template <int NP>
__global__ void __launch_bounds__(kThreads) k_rqp_axis_direct(float2* __restrict__ psi, long long total_lines, int s,
                                                             const double2* __restrict__ Ml) {
  for (long long L = (long long)blockIdx.x * kThreads + threadIdx.x; L < total_lines;
       L += (long long)gridDim.x * kThreads) {
    const long long outer = L / s, inner = L - outer * s;
    float2* __restrict__ line = psi + outer * s * NP + inner;
    double2 x[NP], y[NP];
#pragma unroll
    for (int m = 0; m < NP; ++m) assign(x[m], line[(long long)m * s]);
    line_apply<NP>(Ml, x, y);
#pragma unroll
    for (int m = 0; m < NP; ++m) assign(line[(long long)m * s], y[m]);
  }
}

// f on the lattice: f = 1/2 x^T Q x + b^T x, x_k = j_k / r (FP64); Qb = [Q (d x d), b (d)]
// per instance
__global__ void k_rqp_objective(double* __restrict__ f, const double* __restrict__ Qb, int d, int NP,
                                long long N, long long total) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const long long inst = g / N;
  long long p = g - inst * N;
  const double* Q = Qb + inst * (long long)(d * d + d);
  const double* b = Q + d * d;
  const double inv_r = 1.0 / (double)(NP - 1);
  double x[kRqpMaxDim];
  for (int k = 0; k < d; ++k) {
    x[k] = (double)(p % NP) * inv_r;
    p /= NP;
  }
  double v = 0.0;
  for (int k = 0; k < d; ++k) {
    double qx = 0.0;
    for (int l = 0; l < d; ++l) qx = fma(Q[k * d + l], x[l], qx);
    v = fma(x[k], fma(0.5, qx, b[k]), v);
  }
  f[g] = v;
}

// one block per instance: lowest-index minimiser of f
__global__ void __launch_bounds__(kThreads) k_rqp_argmin(const double* __restrict__ f, long long N,
                                                        double* __restrict__ fmin, long long* __restrict__ amin) {
  __shared__ double sv[kThreads];
  __shared__ long long si[kThreads];
  const double* fi = f + (long long)blockIdx.x * N;
  double bv = INFINITY;
  long long bi = LLONG_MAX;
  for (long long p = threadIdx.x; p < N; p += kThreads) {
    const double v = fi[p];
    if (v < bv) {
      bv = v;
      bi = p;
    }
  }
  sv[threadIdx.x] = bv;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int o = kThreads / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      const double v = sv[threadIdx.x + o];
      const long long id = si[threadIdx.x + o];
      if (v < sv[threadIdx.x] || (v == sv[threadIdx.x] && id < si[threadIdx.x])) {
        sv[threadIdx.x] = v;
        si[threadIdx.x] = id;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    fmin[blockIdx.x] = sv[0];
    amin[blockIdx.x] = si[0];
  }
}

// psi <- discrete Gaussian prod_k amp[j_k]
__global__ void k_rqp_init(float2* __restrict__ psi, const double* __restrict__ amp, int d, int NP, long long N,
                           long long total) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  long long p = g % N;
  double v = 1.0;
  for (int k = 0; k < d; ++k) {
    v *= amp[p % NP];
    p /= NP;
  }
  psi[g] = make_float2((float)v, 0.0f);
}

// one block per instance: sums of rho, f rho, rho over the minimisers (FP64, fixed
// order: per-thread strided partial sums, then a tree), optional rho output
__global__ void __launch_bounds__(kThreads) k_rqp_observe(const float2* __restrict__ psi, const double* __restrict__ f,
                                                         long long N, const double* __restrict__ fmin, double tol,
                                                         double* __restrict__ out, float* __restrict__ prob,
                                                         float2* __restrict__ psi_out, double close_turns) {
  __shared__ double s0[kThreads], s1[kThreads], s2[kThreads];
  const long long off = (long long)blockIdx.x * N;
  const double thr = fmin[blockIdx.x] + tol;
  double a = 0.0, b = 0.0, c = 0.0;
  for (long long p = threadIdx.x; p < N; p += kThreads) {
    const float2 v = psi[off + p];
    const double rho = (double)v.x * v.x + (double)v.y * v.y;
    const double fv = f[off + p];
    a += rho;
    b = fma(fv, rho, b);
    if (fv <= thr) c += rho;
    if (prob) prob[off + p] = (float)rho;
    if (psi_out) psi_out[off + p] = close_turns != 0.0 ? cmul_fd(v, phase_turns_d(close_turns * fv)) : v;
  }
  s0[threadIdx.x] = a;
  s1[threadIdx.x] = b;
  s2[threadIdx.x] = c;
  __syncthreads();
  for (int o = kThreads / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      s0[threadIdx.x] += s0[threadIdx.x + o];
      s1[threadIdx.x] += s1[threadIdx.x + o];
      s2[threadIdx.x] += s2[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[3 * blockIdx.x + 0] = s0[0];
    out[3 * blockIdx.x + 1] = s1[0];
    out[3 * blockIdx.x + 2] = s2[0];
  }
}

// block (instance, axis k): marginal distribution over j_k, per-thread bins in LDS
template <int NP>
__global__ void __launch_bounds__(kThreads) k_rqp_marginals(const float2* __restrict__ psi, long long N, int d,
                                                           float* __restrict__ marg) {
  __shared__ double bins[kThreads * NP];
  const int inst = blockIdx.x / d, k = blockIdx.x - inst * d;
  long long stride = 1;
  for (int q = 0; q < k; ++q) stride *= NP;
  double* my = bins + threadIdx.x * NP;
#pragma unroll
  for (int j = 0; j < NP; ++j) my[j] = 0.0;
  const long long off = (long long)inst * N;
  for (long long p = threadIdx.x; p < N; p += kThreads) {
    const float2 v = psi[off + p];
    const int j = (int)((p / stride) % NP);
    my[j] += (double)v.x * v.x + (double)v.y * v.y;
  }
  __syncthreads();
  for (int o = kThreads / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
#pragma unroll
      for (int j = 0; j < NP; ++j) my[j] += bins[(threadIdx.x + o) * NP + j];
    }
    __syncthreads();
  }
  if ((int)threadIdx.x < NP) marg[((long long)inst * d + k) * NP + threadIdx.x] = (float)bins[threadIdx.x];
}

template <int NP>
hipError_t axis_pass_np(float2* psi, const double* f, long long total_points, int s, const double2* M, bool fuse_v,
                        double beta_turns, hipStream_t st) {
  if (s < 64) {
    const int LB = (kThreads / s) * s;
    const long long lines = total_points / NP;
    const unsigned blocks = (unsigned)((lines + LB - 1) / LB);
    if (fuse_v)
      hipLaunchKernelGGL((k_rqp_axis_staged<NP, true>), dim3(blocks), dim3(kThreads), 0, st, psi, f, total_points, s,
                         LB, M, beta_turns);
    else
      hipLaunchKernelGGL((k_rqp_axis_staged<NP, false>), dim3(blocks), dim3(kThreads), 0, st, psi, f, total_points,
                         s, LB, M, beta_turns);
  } else {
    if (fuse_v) return hipErrorInvalidValue;  // the potential is fused into the axis-1 pass only
    const long long lines = total_points / NP;
    long long b = (lines + kThreads - 1) / kThreads;
    if (b > 65536) b = 65536;
    hipLaunchKernelGGL((k_rqp_axis_direct<NP>), dim3((unsigned)b), dim3(kThreads), 0, st, psi, lines, s, M);
  }
  return hipGetLastError();
}

template <int NP>
hipError_t fused_np(float2* psi, const double* f, long long total_points, int K, const double2* M, double beta_turns,
                    hipStream_t st) {
  long long chunk = 1;
  for (int k = 0; k < K; ++k) chunk *= NP;
  if (K < 1 || chunk > kFusedPoints || total_points % chunk != 0) return hipErrorInvalidValue;
  const int run = (int)((kFusedPoints / chunk) * chunk);
  long long blocks = (total_points + run - 1) / run;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL((k_rqp_fused<NP>), dim3((unsigned)blocks), dim3(kThreads), 0, st, psi, f, total_points, K, run,
                     M, beta_turns);
  return hipGetLastError();
}

template <int NP>
hipError_t marginals_np(const float2* psi, long long N, int d, int batch, float* marg, hipStream_t st) {
  hipLaunchKernelGGL((k_rqp_marginals<NP>), dim3((unsigned)(batch * d)), dim3(kThreads), 0, st, psi, N, d, marg);
  return hipGetLastError();
}

}  // namespace

#define QHD_RQP_NP_CASES(X) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

hipError_t rqp_matrix(int NP, const double* U, const double* lam, double theta, double2* M, hipStream_t st) {
  switch (NP) {
#define QHD_RQP_CASE(n)                                                                        \
  case n:                                                                                      \
    hipLaunchKernelGGL((k_rqp_matrix<n>), dim3(1), dim3(kThreads), 0, st, U, lam, theta, M); \
    return hipGetLastError();
    QHD_RQP_NP_CASES(QHD_RQP_CASE)
#undef QHD_RQP_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t rqp_axis_pass(int NP, float2* psi, const double* f, long long total_points, int stride, const double2* M,
                         bool fuse_v, double beta_turns, hipStream_t st) {
  switch (NP) {
#define QHD_RQP_CASE(n) \
  case n:               \
    return axis_pass_np<n>(psi, f, total_points, stride, M, fuse_v, beta_turns, st);
    QHD_RQP_NP_CASES(QHD_RQP_CASE)
#undef QHD_RQP_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t rqp_fused_pass(int NP, float2* psi, const double* f, long long total_points, int K, const double2* M,
                          double beta_turns, hipStream_t st) {
  switch (NP) {
#define QHD_RQP_CASE(n) \
  case n:               \
    return fused_np<n>(psi, f, total_points, K, M, beta_turns, st);
    QHD_RQP_NP_CASES(QHD_RQP_CASE)
#undef QHD_RQP_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t rqp_marginals(int NP, const float2* psi, long long N, int d, int batch, float* marg, hipStream_t st) {
  switch (NP) {
#define QHD_RQP_CASE(n) \
  case n:               \
    return marginals_np<n>(psi, N, d, batch, marg, st);
    QHD_RQP_NP_CASES(QHD_RQP_CASE)
#undef QHD_RQP_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t rqp_objective(double* f, const double* Qb, int d, int NP, long long N, int batch, hipStream_t st) {
  const long long total = N * batch;
  hipLaunchKernelGGL(k_rqp_objective, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, f, Qb, d, NP, N, total);
  return hipGetLastError();
}

hipError_t rqp_argmin(const double* f, long long N, int batch, double* fmin, long long* amin, hipStream_t st) {
  hipLaunchKernelGGL(k_rqp_argmin, dim3((unsigned)batch), dim3(kThreads), 0, st, f, N, fmin, amin);
  return hipGetLastError();
}

hipError_t rqp_init(float2* psi, const double* amp, int d, int NP, long long N, int batch, hipStream_t st) {
  const long long total = N * batch;
  hipLaunchKernelGGL(k_rqp_init, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, psi, amp, d, NP, N, total);
  return hipGetLastError();
}

hipError_t rqp_observe(const float2* psi, const double* f, long long N, int batch, const double* fmin, double tol,
                       double* out, float* prob, float2* psi_out, double close_turns, hipStream_t st) {
  hipLaunchKernelGGL(k_rqp_observe, dim3((unsigned)batch), dim3(kThreads), 0, st, psi, f, N, fmin, tol, out, prob,
                     psi_out, close_turns);
  return hipGetLastError();
}

}  // namespace qhd
