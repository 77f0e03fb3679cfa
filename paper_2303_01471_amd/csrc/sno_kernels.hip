// Elementwise and reduction kernels of the spectral neural-operator surrogate.
// Activation storage is BF16 (training / inference) or FP32 (gradient checks);
// every reduction accumulates in FP32 within a thread and FP64 across threads.
#include <hip/hip_runtime.h>

#include <cmath>

#include "sno_internal.h"

namespace qhd {

namespace {

template <typename T>
__device__ __forceinline__ float ld(const T* p, long long i) { return (float)p[i]; }

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * __expf(-0.5f * z * z);
}

// block-wide FP64 sum over 256 threads
__device__ __forceinline__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ float block_max(float v, float* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  const float r = sh[0];
  __syncthreads();
  return r;
}

// features per pixel: standardised f, x / S, y / S
template <typename T>
__global__ void __launch_bounds__(256) k_prep(const double* __restrict__ f, int S, T* __restrict__ in) {
  __shared__ double sh[256];
  const int b = blockIdx.x, npix = S * S;
  const double* fb = f + (long long)b * npix;
  double s1 = 0.0, s2 = 0.0;
  for (int p = threadIdx.x; p < npix; p += 256) {
    s1 += fb[p];
    s2 += fb[p] * fb[p];
  }
  const double mean = block_sum(s1, sh) / npix;
  const double var = block_sum(s2, sh) / npix - mean * mean;
  const double inv = 1.0 / sqrt(var > 1e-24 ? var : 1e-24);
  T* ib = in + (long long)b * npix * 3;
  for (int p = threadIdx.x; p < npix; p += 256) {
    ib[3 * p + 0] = (T)(float)((fb[p] - mean) * inv);
    ib[3 * p + 1] = (T)((float)(p % S) / (float)S);
    ib[3 * p + 2] = (T)((float)(p / S) / (float)S);
  }
}

// z += bias (kept for the backward pass when keep_z); h = act(z), act = identity (0)
// or GELU (1)
template <typename T>
__global__ void k_bias_act(float* __restrict__ z, const float* __restrict__ bias, long long n, int C,
                           T* __restrict__ h, int act, int keep_z) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float v = z[e] + bias[e % C];
  if (keep_z) z[e] = v;
  h[e] = (T)(act ? gelu(v) : v);
}

// the same with 4 consecutive elements per thread, for C a multiple of 4 dividing 1024
// (a block's 1024 elements then start on a row boundary: the channel of element 4 t + i
// is (4 t + i) mod C, no 64-bit division); n a multiple of 4
template <typename T>
__global__ void __launch_bounds__(256) k_bias_act4(float* __restrict__ z, const float* __restrict__ bias,
                                                   long long n4, int C, T* __restrict__ h, int act, int keep_z) {
  const long long e4 = (long long)blockIdx.x * 256 + threadIdx.x;
  if (e4 >= n4) return;
  const int c0 = (4 * (int)threadIdx.x) & (C - 1);
  const float4 zv = reinterpret_cast<const float4*>(z)[e4];
  float v[4] = {zv.x + bias[c0], zv.y + bias[c0 + 1], zv.z + bias[c0 + 2], zv.w + bias[c0 + 3]};
  if (keep_z) reinterpret_cast<float4*>(z)[e4] = make_float4(v[0], v[1], v[2], v[3]);
  T o[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) o[i] = (T)(act ? gelu(v[i]) : v[i]);
#pragma unroll
  for (int i = 0; i < 4; ++i) h[4 * e4 + i] = o[i];
}

// Inference form of a layer's closing 1x1 map for width 32: out[p][n] = act(z[p][n] +
// sum_k h[p][k] W[n][k] + b[n]) in BF16, z the layer's spectral part (FP32).  One
// wavefront per 32 pixels on v_mfma_f32_32x32x16_bf16 (two k steps): the A operand is
// the pixels' rows of h straight from HBM (lane l: pixel l mod 32, k 8 (l / 32) + i), the
// B operand the weights, loaded once per wavefront (lane l: n = l mod 32, same k), and
// the 32 x 32 result (register r: pixel 8 (r / 4) + 4 (l / 32) + r mod 4, channel
// l mod 32) gets z, the bias and the activation before its one store.  The pre-activation
// is not written back (the backward pass of training keeps the GEMM + bias_act form).
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

// LDS writes of a wavefront visible to its own later LDS reads (no block barrier)
__device__ __forceinline__ void sno_wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
typedef float f32x16_t __attribute__((ext_vector_type(16)));

template <int ACT>
__global__ void __launch_bounds__(256) k_pointwise32(const __bf16* __restrict__ h, const __bf16* __restrict__ W,
                                                     const float* __restrict__ z, const float* __restrict__ bias,
                                                     long long npix, __bf16* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const long long p0 = (((long long)blockIdx.x * 256 + threadIdx.x) >> 6) * 32;
  if (p0 >= npix) return;  // wavefront-uniform
  const int n = lane & 31, kh = 8 * (lane >> 5);
  const bf16x8_t b0 = *reinterpret_cast<const bf16x8_t*>(W + n * 32 + kh);
  const bf16x8_t b1 = *reinterpret_cast<const bf16x8_t*>(W + n * 32 + 16 + kh);
  const long long pa = p0 + n;
  bf16x8_t a0 = {}, a1 = {};
  if (pa < npix) {
    a0 = *reinterpret_cast<const bf16x8_t*>(h + pa * 32 + kh);
    a1 = *reinterpret_cast<const bf16x8_t*>(h + pa * 32 + 16 + kh);
  }
  f32x16_t acc = {};
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, acc, 0, 0, 0);
  const float bn = bias[n];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const long long p = p0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    if (p < npix) {
      const float v = acc[r] + z[p * 32 + n] + bn;
      out[p * 32 + n] = (__bf16)(ACT ? gelu(v) : v);
    }
  }
}

// one block per sample: logits q = h . wp + bp, then softmax over the grid
template <typename T>
__global__ void __launch_bounds__(256) k_project_softmax(const T* __restrict__ h, const float* __restrict__ wp,
                                                         const float* __restrict__ bp, int npix, int C,
                                                         float* __restrict__ rho) {
  __shared__ double sh[256];
  __shared__ float shf[256];
  const int b = blockIdx.x;
  const T* hb = h + (long long)b * npix * C;
  float* rb = rho + (long long)b * npix;
  float mx = -INFINITY;
  if (sizeof(T) == 2 && C == 32) {
    // width 32 in BF16: a pixel's 64-byte row in four 16-byte loads, the same FMA order
    typedef T t8 __attribute__((ext_vector_type(8)));
    for (int p = threadIdx.x; p < npix; p += 256) {
      const t8* row = reinterpret_cast<const t8*>(hb + (long long)p * 32);
      float q = bp[0];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const t8 x = row[v];
#pragma unroll
        for (int i = 0; i < 8; ++i) q = fmaf((float)x[i], wp[8 * v + i], q);
      }
      rb[p] = q;
      mx = fmaxf(mx, q);
    }
  } else {
    for (int p = threadIdx.x; p < npix; p += 256) {
      float q = bp[0];
      for (int c = 0; c < C; ++c) q = fmaf(ld(hb, (long long)p * C + c), wp[c], q);
      rb[p] = q;
      mx = fmaxf(mx, q);
    }
  }
  mx = block_max(mx, shf);
  double s = 0.0;
  for (int p = threadIdx.x; p < npix; p += 256) {
    const float e = __expf(rb[p] - mx);
    rb[p] = e;
    s += e;
  }
  const double tot = block_sum(s, sh);
  const float inv = (float)(1.0 / tot);
  for (int p = threadIdx.x; p < npix; p += 256) rb[p] *= inv;
}

// one block per sample: loss_b = sum |rho_hat - rho|; dq = rho_hat (g - <rho_hat, g>), g = sign / B
__global__ void __launch_bounds__(256) k_loss_grad(const float* __restrict__ rh, const float* __restrict__ r,
                                                   int batch, int npix, float* __restrict__ dq,
                                                   double* __restrict__ loss) {
  __shared__ double sh[256];
  const int b = blockIdx.x;
  const float* a = rh + (long long)b * npix;
  const float* t = r + (long long)b * npix;
  float* d = dq + (long long)b * npix;
  const float invb = 1.0f / (float)batch;
  double l = 0.0, s = 0.0;
  for (int p = threadIdx.x; p < npix; p += 256) {
    const float diff = a[p] - t[p];
    const float g = diff > 0.0f ? invb : (diff < 0.0f ? -invb : 0.0f);
    l += fabs((double)diff);
    s += (double)a[p] * g;
    d[p] = g;
  }
  const double lt = block_sum(l, sh);
  const float st = (float)block_sum(s, sh);
  for (int p = threadIdx.x; p < npix; p += 256) d[p] = a[p] * (d[p] - st);
  if (threadIdx.x == 0) loss[b] = lt;
}

// dh = dq wp (outer product), and per-block partial sums of dWp = sum dq h, dbp = sum dq
template <typename T>
__global__ void __launch_bounds__(256) k_project_backward(const float* __restrict__ dq, const T* __restrict__ h,
                                                          const float* __restrict__ wp, long long rows, int C,
                                                          float* __restrict__ dh, float* __restrict__ partials) {
  __shared__ double sh[256];
  const int c = threadIdx.x % C, r0 = threadIdx.x / C, rstep = 256 / C;
  const long long per = (rows + gridDim.x - 1) / gridDim.x;
  const long long beg = (long long)blockIdx.x * per;
  const long long end = beg + per < rows ? beg + per : rows;
  float accw = 0.0f, accb = 0.0f;
  for (long long r = beg + r0; r < end; r += rstep) {
    const float g = dq[r];
    accw = fmaf(g, ld(h, r * C + c), accw);
    if (c == 0) accb += g;
    dh[r * C + c] = g * wp[c];
  }
  // reduce over the row groups of equal c
  sh[threadIdx.x] = accw;
  __syncthreads();
  if ((int)threadIdx.x < C) {
    double s = 0.0;
    for (int k = 0; k < rstep; ++k) s += sh[threadIdx.x + k * C];
    partials[(long long)blockIdx.x * (C + 1) + threadIdx.x] = (float)s;
  }
  __syncthreads();
  sh[threadIdx.x] = accb;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int k = 0; k < rstep; ++k) s += sh[k * C];
    partials[(long long)blockIdx.x * (C + 1) + C] = (float)s;
  }
}

// dz = dh * GELU'(z), stored as T, and per-block partial column sums of dz taken
// from the FP32 products before rounding (the bias gradient: its terms cancel
// heavily, since the softmax gradient sums to zero over each sample)
template <typename T>
__global__ void __launch_bounds__(256) k_gelu_backward(const float* __restrict__ dh, const float* __restrict__ z,
                                                       long long rows, int C, T* __restrict__ dz,
                                                       float* __restrict__ partials) {
  __shared__ double sh[256];
  const int c = threadIdx.x % C, r0 = threadIdx.x / C, rstep = 256 / C;
  const long long per = (rows + gridDim.x - 1) / gridDim.x;
  const long long beg = (long long)blockIdx.x * per;
  const long long end = beg + per < rows ? beg + per : rows;
  float acc = 0.0f;
  for (long long r = beg + r0; r < end; r += rstep) {
    const long long e = r * C + c;
    const float v = dh[e] * gelu_grad(z[e]);
    dz[e] = (T)v;
    acc += v;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  if ((int)threadIdx.x < C) {
    double s = 0.0;
    for (int k = 0; k < rstep; ++k) s += sh[threadIdx.x + k * C];
    partials[(long long)blockIdx.x * C + threadIdx.x] = (float)s;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_colsum(const T* __restrict__ x, long long rows, int C,
                                                float* __restrict__ partials) {
  __shared__ double sh[256];
  const int c = threadIdx.x % C, r0 = threadIdx.x / C, rstep = 256 / C;
  const long long per = (rows + gridDim.x - 1) / gridDim.x;
  const long long beg = (long long)blockIdx.x * per;
  const long long end = beg + per < rows ? beg + per : rows;
  float acc = 0.0f;
  for (long long r = beg + r0; r < end; r += rstep) acc += ld(x, r * C + c);
  sh[threadIdx.x] = acc;
  __syncthreads();
  if ((int)threadIdx.x < C) {
    double s = 0.0;
    for (int k = 0; k < rstep; ++k) s += sh[threadIdx.x + k * C];
    partials[(long long)blockIdx.x * C + threadIdx.x] = (float)s;
  }
}

// out[j] (+)= sum over k of partials[k][j] in FP64, in a fixed order: 16 interleaved partial
// sums per output (k = q, q + 16, ...), then those 16 in order q = 0..15. A block takes 16
// outputs with 16 threads each.
__global__ void __launch_bounds__(256) k_reduce_partials(const float* __restrict__ partials, int nparts, int len,
                                                         float* __restrict__ out, int accumulate) {
  __shared__ double sh[16][17];
  const int jl = threadIdx.x & 15, q = threadIdx.x >> 4;
  const int j = blockIdx.x * 16 + jl;
  double s = 0.0;
  if (j < len)
    for (int k = q; k < nparts; k += 16) s += partials[(long long)k * len + j];
  sh[q][jl] = s;
  __syncthreads();
  if (q == 0 && j < len) {
    double t = 0.0;
    for (int r = 0; r < 16; ++r) t += sh[r][jl];
    out[j] = accumulate ? out[j] + (float)t : (float)t;
  }
}

template <typename T>
__global__ void k_cast(const float* __restrict__ src, T* __restrict__ dst, long long n) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) dst[e] = (T)src[e];
}

template <typename T>
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, long long n, float lr, float b1, float b2, float eps,
                       float c1, float c2, T* __restrict__ copy) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float gi = g[e];
  const float mi = b1 * m[e] + (1.0f - b1) * gi;
  const float vi = b2 * v[e] + (1.0f - b2) * gi * gi;
  m[e] = mi;
  v[e] = vi;
  const float pi = p[e] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[e] = pi;
  if (copy) copy[e] = (T)pi;
}

__global__ void k_fill(float* __restrict__ p, long long n, float v) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) p[e] = v;
}

inline dim3 grid1(long long n) { return dim3((unsigned)((n + 255) / 256)); }

}  // namespace

hipError_t sno_prep_input(const double* f, int batch, int S, void* in, bool bf16, hipStream_t st) {
  if (bf16) hipLaunchKernelGGL(k_prep<__bf16>, dim3(batch), dim3(256), 0, st, f, S, (__bf16*)in);
  else hipLaunchKernelGGL(k_prep<float>, dim3(batch), dim3(256), 0, st, f, S, (float*)in);
  return hipGetLastError();
}

hipError_t sno_bias_act(float* z, const float* bias, long long rows, int C, void* h, bool bf16, int act,
                        hipStream_t st, bool keep_z) {
  const long long n = rows * C;
  const bool pow2 = C >= 4 && (C & (C - 1)) == 0 && 1024 % C == 0;
  if (pow2 && (reinterpret_cast<uintptr_t>(z) & 15) == 0) {
    const long long n4 = n / 4;
    if (bf16)
      hipLaunchKernelGGL(k_bias_act4<__bf16>, grid1(n4), dim3(256), 0, st, z, bias, n4, C, (__bf16*)h, act,
                         keep_z ? 1 : 0);
    else
      hipLaunchKernelGGL(k_bias_act4<float>, grid1(n4), dim3(256), 0, st, z, bias, n4, C, (float*)h, act,
                         keep_z ? 1 : 0);
    return hipGetLastError();
  }
  if (bf16)
    hipLaunchKernelGGL(k_bias_act<__bf16>, grid1(n), dim3(256), 0, st, z, bias, n, C, (__bf16*)h, act, keep_z ? 1 : 0);
  else
    hipLaunchKernelGGL(k_bias_act<float>, grid1(n), dim3(256), 0, st, z, bias, n, C, (float*)h, act, keep_z ? 1 : 0);
  return hipGetLastError();
}

// inference form at width 32 in BF16: one sample's features, formed as k_prep forms them and
// rounded to BF16 like the lift's operands, and the lift h0 = x0 Wl^T + bl in one pass; the
// features are not stored. Thread t writes channels 8(t%4) .. 8(t%4)+7 of its pixels.
__global__ void __launch_bounds__(256) k_prep_lift32(const double* __restrict__ f, int S,
                                                     const __bf16* __restrict__ Wl, const float* __restrict__ bl,
                                                     __bf16* __restrict__ h) {
  __shared__ double sh[256];
  const int b = blockIdx.x, npix = S * S;
  const double* fb = f + (long long)b * npix;
  double s1 = 0.0, s2 = 0.0;
  for (int p = threadIdx.x; p < npix; p += 256) {
    s1 += fb[p];
    s2 += fb[p] * fb[p];
  }
  const double mean = block_sum(s1, sh) / npix;
  const double var = block_sum(s2, sh) / npix - mean * mean;
  const double inv = 1.0 / sqrt(var > 1e-24 ? var : 1e-24);
  const int c = threadIdx.x & 3;
  float w0[8], w1[8], w2[8], bb[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int n = 8 * c + i;
    w0[i] = (float)Wl[3 * n];
    w1[i] = (float)Wl[3 * n + 1];
    w2[i] = (float)Wl[3 * n + 2];
    bb[i] = bl[n];
  }
  bf16x8_t* hb = reinterpret_cast<bf16x8_t*>(h + (long long)b * npix * 32);
  // S is a power of two: coordinates by mask and shift, scaled exactly by 1/S
  const int sl = 31 - __clz(S);
  const float rs = 1.0f / (float)S;
  for (int e = threadIdx.x; e < npix * 4; e += 256) {
    const int p = e >> 2;
    const float x0 = (float)(__bf16)(float)((fb[p] - mean) * inv);
    const float x1 = (float)(__bf16)((float)(p & (S - 1)) * rs);
    const float x2 = (float)(__bf16)((float)(p >> sl) * rs);
    bf16x8_t o;
#pragma unroll
    for (int i = 0; i < 8; ++i) o[i] = (__bf16)(fmaf(x2, w2[i], fmaf(x1, w1[i], x0 * w0[i])) + bb[i]);
    hb[e] = o;
  }
}

hipError_t sno_prep_lift32(const double* f, int batch, int S, const void* Wl, const float* bl, void* h,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_prep_lift32, dim3(batch), dim3(256), 0, st, f, S, (const __bf16*)Wl, bl, (__bf16*)h);
  return hipGetLastError();
}

// inference at width 32 with 16 modes per axis, BF16: the x-contraction of the truncated inverse
// transform, the 1x1 map, bias and activation in one pass. For the row (b, y) of S pixels:
// out (S x 32) = act(gx U_row + h_row W^T + b), gx (S x 32), U_row (32 x 32, [k][channel]), W
// ([out][in]); all four products accumulate in one FP32 tile. One wave per row, 32 pixels per step.
// With NEXT the next layer's forward x-contraction T_row = fx out_row (fx 32 x S) is formed from
// the rounded outputs while they are in registers and written over U_row (each wave reads its
// U_row before it writes T_row, so U and T may be the same buffer).
// With PROJ (the last layer) the rounded outputs are not stored: each is projected to its
// pixel's logit q = bp + sum_c out[c] wp[c] (FP32, channels in order, as k_project_softmax
// forms it) from the LDS tile, and q goes to qout.
template <int ACT, bool NEXT, bool PROJ>
__global__ void __launch_bounds__(256) k_spectral_pointwise32(const __bf16* __restrict__ gx, const __bf16* U,
                                                              const __bf16* __restrict__ h,
                                                              const __bf16* __restrict__ W,
                                                              const float* __restrict__ bias, int S, long long nrows,
                                                              __bf16* __restrict__ out, const __bf16* __restrict__ fx,
                                                              __bf16* T, const float* __restrict__ wp,
                                                              const float* __restrict__ bp, float* __restrict__ qout) {
  typedef __bf16 bf16x4_t __attribute__((ext_vector_type(4)));
  const int lane = threadIdx.x & 63;
  const long long row = ((long long)blockIdx.x * 256 + threadIdx.x) >> 6;
  if (row >= nrows) return;  // wavefront-uniform
  const int n = lane & 31, j = lane >> 5, kh = 8 * j;
  const bf16x8_t w0 = *reinterpret_cast<const bf16x8_t*>(W + n * 32 + kh);
  const bf16x8_t w1 = *reinterpret_cast<const bf16x8_t*>(W + n * 32 + 16 + kh);
  const __bf16* Ur = U + row * 1024;
  bf16x8_t u0, u1;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    u0[i] = Ur[(kh + i) * 32 + n];
    u1[i] = Ur[(16 + kh + i) * 32 + n];
  }
  const float bn = bias[n];
  const long long pbase = row * S;
  // the 32 x 32 output tile goes through LDS (row stride 40: the two lane halves' rows, 4
  // apart, fall on disjoint banks) so that it leaves as two 16-byte stores per lane
  __shared__ __attribute__((aligned(16))) __bf16 stage[4][32 * 40];
  __bf16* sw = stage[threadIdx.x >> 6];
  bf16x8_t* const ob = reinterpret_cast<bf16x8_t*>(out + pbase * 32);
  f32x16_t tacc = {};
  // operands of the step at x0 are loaded during the step before it
  bf16x8_t g0 = *reinterpret_cast<const bf16x8_t*>(gx + n * 32 + kh);
  bf16x8_t g1 = *reinterpret_cast<const bf16x8_t*>(gx + n * 32 + 16 + kh);
  bf16x8_t a0 = *reinterpret_cast<const bf16x8_t*>(h + (pbase + n) * 32 + kh);
  bf16x8_t a1 = *reinterpret_cast<const bf16x8_t*>(h + (pbase + n) * 32 + 16 + kh);
  for (int x0 = 0; x0 < S; x0 += 32) {
    f32x16_t acc = {};
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(g0, u0, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(g1, u1, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, w0, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, w1, acc, 0, 0, 0);
    if (x0 + 32 < S) {
      const int x = x0 + 32 + n;
      const long long pa = pbase + x;
      g0 = *reinterpret_cast<const bf16x8_t*>(gx + x * 32 + kh);
      g1 = *reinterpret_cast<const bf16x8_t*>(gx + x * 32 + 16 + kh);
      a0 = *reinterpret_cast<const bf16x8_t*>(h + pa * 32 + kh);
      a1 = *reinterpret_cast<const bf16x8_t*>(h + pa * 32 + 16 + kh);
    }
    bf16x8_t o0, o1;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float v = acc[r] + bn;
      const __bf16 o = (__bf16)(ACT ? gelu(v) : v);
      sw[(8 * (r >> 2) + 4 * j + (r & 3)) * 40 + n] = o;
      if (r < 8) o0[r] = o;
      else o1[r - 8] = o;
    }
    sno_wave_lds_sync();
    if constexpr (PROJ) {
      if (lane < 32) {  // pixel x0 + lane: its row of the tile
        float q = bp[0];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const bf16x8_t xv = *reinterpret_cast<const bf16x8_t*>(sw + lane * 40 + 8 * v);
#pragma unroll
          for (int i = 0; i < 8; ++i) q = fmaf((float)xv[i], wp[8 * v + i], q);
        }
        qout[pbase + x0 + lane] = q;
      }
    } else {
      const bf16x8_t s0 = *reinterpret_cast<const bf16x8_t*>(sw + (lane >> 2) * 40 + 8 * (lane & 3));
      const bf16x8_t s1 = *reinterpret_cast<const bf16x8_t*>(sw + (16 + (lane >> 2)) * 40 + 8 * (lane & 3));
      ob[x0 * 4 + lane] = s0;  // pixel x0 + lane / 4, channels 8 (lane % 4) ..
      ob[x0 * 4 + 64 + lane] = s1;
    }
    sno_wave_lds_sync();  // the next step rewrites the tile
    if constexpr (NEXT) {
      // k slot i of lane half j holds pixel x0 + 4j + i (i < 4) or x0 + 8 + 4j + (i - 4) of the
      // output layout (o0), 16 more for o1: fx's operand takes the same pixels
      const __bf16* fr = fx + n * S + x0 + 4 * j;
      const bf16x4_t f0 = *reinterpret_cast<const bf16x4_t*>(fr);
      const bf16x4_t f1 = *reinterpret_cast<const bf16x4_t*>(fr + 8);
      const bf16x4_t f2 = *reinterpret_cast<const bf16x4_t*>(fr + 16);
      const bf16x4_t f3 = *reinterpret_cast<const bf16x4_t*>(fr + 24);
      const bf16x8_t fa = {f0[0], f0[1], f0[2], f0[3], f1[0], f1[1], f1[2], f1[3]};
      const bf16x8_t fb = {f2[0], f2[1], f2[2], f2[3], f3[0], f3[1], f3[2], f3[3]};
      tacc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa, o0, tacc, 0, 0, 0);
      tacc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fb, o1, tacc, 0, 0, 0);
    }
  }
  if constexpr (NEXT) {
    // T_row (32 x 32, [k][channel]) through the same LDS tile
#pragma unroll
    for (int r = 0; r < 16; ++r) sw[(8 * (r >> 2) + 4 * j + (r & 3)) * 40 + n] = (__bf16)tacc[r];
    sno_wave_lds_sync();
    bf16x8_t* const tb = reinterpret_cast<bf16x8_t*>(T + row * 1024);
    tb[lane] = *reinterpret_cast<const bf16x8_t*>(sw + (lane >> 2) * 40 + 8 * (lane & 3));
    tb[64 + lane] = *reinterpret_cast<const bf16x8_t*>(sw + (16 + (lane >> 2)) * 40 + 8 * (lane & 3));
  }
}

hipError_t sno_spectral_pointwise32(const void* gx, const void* U, const void* h, const void* W, const float* bias,
                                    int S, long long nrows, void* out, int act, const void* fx, void* T,
                                    const float* wp, const float* bp, float* q, hipStream_t st) {
  const unsigned blocks = (unsigned)((nrows + 3) / 4);
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), 0, st, (const __bf16*)gx, (const __bf16*)U, (const __bf16*)h,
                       (const __bf16*)W, bias, S, nrows, (__bf16*)out, (const __bf16*)fx, (__bf16*)T, wp, bp, q);
  };
  if (fx) {
    if (act) go(k_spectral_pointwise32<1, true, false>);
    else go(k_spectral_pointwise32<0, true, false>);
  } else if (q) {
    if (act) go(k_spectral_pointwise32<1, false, true>);
    else go(k_spectral_pointwise32<0, false, true>);
  } else {
    if (act) go(k_spectral_pointwise32<1, false, false>);
    else go(k_spectral_pointwise32<0, false, false>);
  }
  return hipGetLastError();
}

// per sample, rho = softmax of its logits in place: the max, the FP64 sum of exp(q - max)
// and the scaling exactly as k_project_softmax takes them (same threads, same order)
__global__ void __launch_bounds__(256) k_softmax_rows(float* __restrict__ rho, int npix) {
  __shared__ double sh[256];
  __shared__ float shf[256];
  float* rb = rho + (long long)blockIdx.x * npix;
  float mx = -INFINITY;
  for (int p = threadIdx.x; p < npix; p += 256) mx = fmaxf(mx, rb[p]);
  mx = block_max(mx, shf);
  double s = 0.0;
  for (int p = threadIdx.x; p < npix; p += 256) {
    const float e = __expf(rb[p] - mx);
    rb[p] = e;
    s += e;
  }
  const double tot = block_sum(s, sh);
  const float inv = (float)(1.0 / tot);
  for (int p = threadIdx.x; p < npix; p += 256) rb[p] *= inv;
}

hipError_t sno_softmax_rows(float* rho, int batch, int npix, hipStream_t st) {
  hipLaunchKernelGGL(k_softmax_rows, dim3(batch), dim3(256), 0, st, rho, npix);
  return hipGetLastError();
}

// x-contraction of the truncated forward transform at width 32 with 16 modes, BF16: for the row
// (b, y) of S pixels, T_row (32 x 32, [k][channel]) = fx (32 x S) X_row (S x 32), FP32 accumulation,
// BF16 result. One wave per row; lane = channel, so each pixel's channels are gathered as the
// k-operand of the matrix cores.
__global__ void __launch_bounds__(256) k_dft_x32(const __bf16* __restrict__ fx, const __bf16* __restrict__ X,
                                                 int S, long long nrows, __bf16* __restrict__ T) {
  const int lane = threadIdx.x & 63;
  const long long row = ((long long)blockIdx.x * 256 + threadIdx.x) >> 6;
  if (row >= nrows) return;  // wavefront-uniform
  const int c = lane & 31, kh = 8 * (lane >> 5);
  const __bf16* Xr = X + row * S * 32;
  f32x16_t acc = {};
#pragma unroll 4
  for (int x0 = 0; x0 < S; x0 += 16) {
    const bf16x8_t a = *reinterpret_cast<const bf16x8_t*>(fx + c * S + x0 + kh);
    bf16x8_t b;
#pragma unroll
    for (int i = 0; i < 8; ++i) b[i] = Xr[(x0 + kh + i) * 32 + c];
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
  }
  __bf16* Tr = T + row * 1024;
#pragma unroll
  for (int r = 0; r < 16; ++r) Tr[(8 * (r >> 2) + 4 * (lane >> 5) + (r & 3)) * 32 + c] = (__bf16)acc[r];
}

hipError_t sno_dft_x32(const void* fx, const void* X, int S, long long nrows, void* T, hipStream_t st) {
  hipLaunchKernelGGL(k_dft_x32, dim3((unsigned)((nrows + 3) / 4)), dim3(256), 0, st, (const __bf16*)fx,
                     (const __bf16*)X, S, nrows, (__bf16*)T);
  return hipGetLastError();
}

// inverse transform's y-contraction at width 32 with 16 modes, BF16, one sample per
// workgroup: U (2S x 512) = Gy (2S x 64) G_b (64 x 512), Gy's rows 2y, 2y+1 the cosine and
// sine rows of y. G_b is staged in LDS transposed ([column][k], row stride 72: each lane's
// 16-byte k operand is contiguous and aligned); each wavefront keeps the Gy operands of its
// 32-row tiles in registers and runs over the 16 column tiles.
__global__ void __launch_bounds__(256) k_inv_y32(const __bf16* __restrict__ Gy, const __bf16* __restrict__ G,
                                                 long long gstride, int S, __bf16* __restrict__ U) {
  __shared__ __attribute__((aligned(16))) __bf16 gt[512 * 72];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c = lane & 31, h = lane >> 5;
  const __bf16* Gb = G + (long long)blockIdx.x * gstride;
  for (int e = tid; e < 64 * 64; e += 256) {  // 16-byte pieces: row k = e % 64, columns 8 (e / 64) ..
    // (a wavefront's lanes take the 64 rows of one column group, so each of its transposed
    // 2-byte writes covers 64 consecutive entries of one LDS row)
    const int k = e & 63, c0 = (e >> 6) * 8;
    const bf16x8_t v = *reinterpret_cast<const bf16x8_t*>(Gb + k * 512 + c0);
#pragma unroll
    for (int i = 0; i < 8; ++i) gt[(c0 + i) * 72 + k] = v[i];
  }
  __syncthreads();
  __bf16* Ub = U + (long long)blockIdx.x * S * 1024;
  for (int rt = wave; rt < S / 16; rt += 4) {  // 2S rows in tiles of 32
    bf16x8_t a[4];
#pragma unroll
    for (int st = 0; st < 4; ++st) a[st] = *reinterpret_cast<const bf16x8_t*>(Gy + (32 * rt + c) * 64 + 16 * st + 8 * h);
    for (int ct = 0; ct < 16; ++ct) {
      f32x16_t acc = {};
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const bf16x8_t b = *reinterpret_cast<const bf16x8_t*>(gt + (32 * ct + c) * 72 + 16 * st + 8 * h);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[st], b, acc, 0, 0, 0);
      }
      __bf16* Ut = Ub + (long long)(32 * rt) * 512 + 32 * ct + c;
#pragma unroll
      for (int r = 0; r < 16; ++r) Ut[(8 * (r >> 2) + 4 * h + (r & 3)) * 512] = (__bf16)acc[r];
    }
  }
}

hipError_t sno_inv_y32(const void* Gy, const void* G, long long gstride, int batch, int S, void* U, hipStream_t st) {
  hipLaunchKernelGGL(k_inv_y32, dim3(batch), dim3(256), 0, st, (const __bf16*)Gy, (const __bf16*)G, gstride, S,
                     (__bf16*)U);
  return hipGetLastError();
}

// forward transform's y-contraction at width 32 with 16 modes, BF16, one sample per
// workgroup: [Hr; Hi] (64 x 512) = Fy1 (64 x S) Tr + Fy2 (64 x S) Ti, with Tr and Ti the two
// halves of each row of T_b (S x 1024). Fy1 and Fy2 are staged in LDS (row stride S + 8);
// T's k operand (8 rows of one column per lane half) is gathered from HBM, each element
// once; wavefront w takes the column tiles w, w + 4, ..., both 32-row tiles of each.
__global__ void __launch_bounds__(256) k_fwd_y32(const __bf16* __restrict__ Fy1, const __bf16* __restrict__ Fy2,
                                                 const __bf16* __restrict__ T, int S, __bf16* __restrict__ H,
                                                 long long hstride) {
  extern __shared__ __attribute__((aligned(16))) __bf16 fy[];  // 2 x 64 x (S + 8), sized at launch
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c = lane & 31, h = lane >> 5, ld = S + 8;
  for (int e = tid; e < 64 * S / 8; e += 256) {  // 16-byte pieces of both matrices
    const int r = e / (S / 8), k0 = (e - r * (S / 8)) * 8;
    *reinterpret_cast<bf16x8_t*>(fy + r * ld + k0) = *reinterpret_cast<const bf16x8_t*>(Fy1 + r * S + k0);
    *reinterpret_cast<bf16x8_t*>(fy + 64 * ld + r * ld + k0) =
        *reinterpret_cast<const bf16x8_t*>(Fy2 + r * S + k0);
  }
  __syncthreads();
  const __bf16* Tb = T + (long long)blockIdx.x * S * 1024;
  __bf16* Hb = H + (long long)blockIdx.x * hstride;
  for (int ct = wave; ct < 16; ct += 4) {
    f32x16_t acc0 = {}, acc1 = {};
    const __bf16* tc = Tb + 32 * ct + c;
    for (int k0 = 0; k0 < S; k0 += 16) {
      bf16x8_t br, bi;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        br[i] = tc[(k0 + 8 * h + i) * 1024];
        bi[i] = tc[(k0 + 8 * h + i) * 1024 + 512];
      }
      const __bf16* f1 = fy + c * ld + k0 + 8 * h;
      const __bf16* f2 = f1 + 64 * ld;
      acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(*reinterpret_cast<const bf16x8_t*>(f1), br, acc0, 0, 0, 0);
      acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(*reinterpret_cast<const bf16x8_t*>(f2), bi, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(*reinterpret_cast<const bf16x8_t*>(f1 + 32 * ld), br, acc1, 0,
                                                     0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(*reinterpret_cast<const bf16x8_t*>(f2 + 32 * ld), bi, acc1, 0,
                                                     0, 0);
    }
    __bf16* ho = Hb + 32 * ct + c;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = 8 * (r >> 2) + 4 * h + (r & 3);
      ho[row * 512] = (__bf16)acc0[r];
      ho[(32 + row) * 512] = (__bf16)acc1[r];
    }
  }
}

hipError_t sno_fwd_y32(const void* Fy1, const void* Fy2, const void* T, int batch, int S, void* H, long long hstride,
                       hipStream_t st) {
  const size_t lds = (size_t)2 * 64 * (S + 8) * sizeof(__bf16);
  if (lds > 65536) {  // above the default dynamic LDS limit (S = 256: 66 KB)
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fwd_y32),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_fwd_y32, dim3(batch), dim3(256), lds, st, (const __bf16*)Fy1, (const __bf16*)Fy2,
                     (const __bf16*)T, S, (__bf16*)H, hstride);
  return hipGetLastError();
}

// per-mode complex mixing at width 32, BF16: for mode m and 32 samples, Gr = Hr Rr[m]^T -
// Hi Ri[m]^T and Gi = Hr Ri[m]^T + Hi Rr[m]^T (R[m] is [out][in]); spectra are [b][re | im]
// [mode][channel], half = nmodes x 32 apart. One wavefront per (mode, 32 samples), modes
// fastest; the sine products' weights are negated in BF16 (exact).
__global__ void __launch_bounds__(256) k_mix32(const __bf16* __restrict__ H, const __bf16* __restrict__ Rr,
                                               const __bf16* __restrict__ Ri, int nmodes, long long spec, int B,
                                               __bf16* __restrict__ G) {
  const int lane = threadIdx.x & 63;
  const long long wid = ((long long)blockIdx.x * 256 + threadIdx.x) >> 6;
  const int mode = (int)(wid % nmodes);
  const int b0 = (int)(wid / nmodes) * 32;
  if (b0 >= B) return;  // wavefront-uniform
  const int r = lane & 31, h = lane >> 5, kh = 8 * h;
  const long long half = (long long)nmodes * 32;
  bf16x8_t hr0 = {}, hr1 = {}, hi0 = {}, hi1 = {};
  if (b0 + r < B) {
    const __bf16* hb = H + (long long)(b0 + r) * spec + mode * 32 + kh;
    hr0 = *reinterpret_cast<const bf16x8_t*>(hb);
    hr1 = *reinterpret_cast<const bf16x8_t*>(hb + 16);
    hi0 = *reinterpret_cast<const bf16x8_t*>(hb + half);
    hi1 = *reinterpret_cast<const bf16x8_t*>(hb + half + 16);
  }
  const __bf16* rr = Rr + (long long)mode * 1024 + r * 32 + kh;
  const __bf16* ri = Ri + (long long)mode * 1024 + r * 32 + kh;
  const bf16x8_t rr0 = *reinterpret_cast<const bf16x8_t*>(rr), rr1 = *reinterpret_cast<const bf16x8_t*>(rr + 16);
  const bf16x8_t ri0 = *reinterpret_cast<const bf16x8_t*>(ri), ri1 = *reinterpret_cast<const bf16x8_t*>(ri + 16);
  bf16x8_t ni0, ni1;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    ni0[i] = -ri0[i];
    ni1[i] = -ri1[i];
  }
  f32x16_t gr = {}, gi = {};
  gr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(hr0, rr0, gr, 0, 0, 0);
  gr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(hr1, rr1, gr, 0, 0, 0);
  gr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(hi0, ni0, gr, 0, 0, 0);
  gr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(hi1, ni1, gr, 0, 0, 0);
  gi = __builtin_amdgcn_mfma_f32_32x32x16_bf16(hr0, ri0, gi, 0, 0, 0);
  gi = __builtin_amdgcn_mfma_f32_32x32x16_bf16(hr1, ri1, gi, 0, 0, 0);
  gi = __builtin_amdgcn_mfma_f32_32x32x16_bf16(hi0, rr0, gi, 0, 0, 0);
  gi = __builtin_amdgcn_mfma_f32_32x32x16_bf16(hi1, rr1, gi, 0, 0, 0);
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int b = b0 + 8 * (q >> 2) + 4 * h + (q & 3);
    if (b < B) {
      __bf16* g = G + (long long)b * spec + mode * 32 + r;
      g[0] = (__bf16)gr[q];
      g[half] = (__bf16)gi[q];
    }
  }
}

hipError_t sno_mix32(const void* H, const void* Rr, const void* Ri, int nmodes, long long spec, int batch, void* G,
                     hipStream_t st) {
  const long long waves = (long long)nmodes * ((batch + 31) / 32);
  hipLaunchKernelGGL(k_mix32, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st, (const __bf16*)H,
                     (const __bf16*)Rr, (const __bf16*)Ri, nmodes, spec, batch, (__bf16*)G);
  return hipGetLastError();
}

hipError_t sno_pointwise32(const void* h, const void* W, const float* z, const float* bias, long long npix,
                           void* out, int act, hipStream_t st) {
  const long long waves = (npix + 31) / 32;
  const unsigned blocks = (unsigned)((waves + 3) / 4);
  if (act)
    hipLaunchKernelGGL(k_pointwise32<1>, dim3(blocks), dim3(256), 0, st, (const __bf16*)h, (const __bf16*)W, z, bias,
                       npix, (__bf16*)out);
  else
    hipLaunchKernelGGL(k_pointwise32<0>, dim3(blocks), dim3(256), 0, st, (const __bf16*)h, (const __bf16*)W, z, bias,
                       npix, (__bf16*)out);
  return hipGetLastError();
}

hipError_t sno_project_softmax(const void* h, const float* wp, const float* bp, int batch, int npix,
                               int C, bool bf16, float* rho, hipStream_t st) {
  if (bf16)
    hipLaunchKernelGGL(k_project_softmax<__bf16>, dim3(batch), dim3(256), 0, st, (const __bf16*)h, wp, bp,
                       npix, C, rho);
  else
    hipLaunchKernelGGL(k_project_softmax<float>, dim3(batch), dim3(256), 0, st, (const float*)h, wp, bp,
                       npix, C, rho);
  return hipGetLastError();
}

hipError_t sno_loss_grad(const float* rho_hat, const float* rho, int batch, int npix, float* dq,
                         double* loss_per_sample, hipStream_t st) {
  hipLaunchKernelGGL(k_loss_grad, dim3(batch), dim3(256), 0, st, rho_hat, rho, batch, npix, dq,
                     loss_per_sample);
  return hipGetLastError();
}

hipError_t sno_project_backward(const float* dq, const void* h, const float* wp, int batch, int npix,
                                int C, bool bf16, float* dh, float* partials, int nparts,
                                hipStream_t st) {
  const long long rows = (long long)batch * npix;
  if (bf16)
    hipLaunchKernelGGL(k_project_backward<__bf16>, dim3(nparts), dim3(256), 0, st, dq, (const __bf16*)h,
                       wp, rows, C, dh, partials);
  else
    hipLaunchKernelGGL(k_project_backward<float>, dim3(nparts), dim3(256), 0, st, dq, (const float*)h, wp,
                       rows, C, dh, partials);
  return hipGetLastError();
}

hipError_t sno_gelu_backward(const float* dh, const float* z, long long rows, int C, void* dz, bool bf16,
                             float* partials, int nparts, hipStream_t st) {
  if (bf16)
    hipLaunchKernelGGL(k_gelu_backward<__bf16>, dim3(nparts), dim3(256), 0, st, dh, z, rows, C, (__bf16*)dz,
                       partials);
  else
    hipLaunchKernelGGL(k_gelu_backward<float>, dim3(nparts), dim3(256), 0, st, dh, z, rows, C, (float*)dz,
                       partials);
  return hipGetLastError();
}

hipError_t sno_colsum(const void* x, bool bf16, long long rows, int C, float* partials, int nparts,
                      hipStream_t st) {
  if (bf16)
    hipLaunchKernelGGL(k_colsum<__bf16>, dim3(nparts), dim3(256), 0, st, (const __bf16*)x, rows, C, partials);
  else
    hipLaunchKernelGGL(k_colsum<float>, dim3(nparts), dim3(256), 0, st, (const float*)x, rows, C, partials);
  return hipGetLastError();
}

hipError_t sno_reduce_partials(const float* partials, int nparts, int len, float* out, bool accumulate,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_partials, dim3((unsigned)((len + 15) / 16)), dim3(256), 0, st, partials, nparts, len,
                     out, accumulate ? 1 : 0);
  return hipGetLastError();
}

hipError_t sno_cast(const float* src, void* dst, long long n, bool bf16, hipStream_t st) {
  if (bf16) hipLaunchKernelGGL(k_cast<__bf16>, grid1(n), dim3(256), 0, st, src, (__bf16*)dst, n);
  else hipLaunchKernelGGL(k_cast<float>, grid1(n), dim3(256), 0, st, src, (float*)dst, n);
  return hipGetLastError();
}

hipError_t sno_adam(float* p, const float* g, float* m, float* v, long long n, float lr, float b1,
                    float b2, float eps, float c1, float c2, void* copy, bool bf16, hipStream_t st) {
  if (bf16)
    hipLaunchKernelGGL(k_adam<__bf16>, grid1(n), dim3(256), 0, st, p, g, m, v, n, lr, b1, b2, eps, c1, c2,
                       (__bf16*)copy);
  else
    hipLaunchKernelGGL(k_adam<float>, grid1(n), dim3(256), 0, st, p, g, m, v, n, lr, b1, b2, eps, c1, c2,
                       (float*)copy);
  return hipGetLastError();
}

hipError_t sno_fill(float* p, long long n, float v, hipStream_t st) {
  hipLaunchKernelGGL(k_fill, grid1(n), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

}  // namespace qhd
