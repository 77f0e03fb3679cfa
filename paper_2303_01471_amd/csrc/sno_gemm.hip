// Batched GEMM on the CDNA4 matrix cores for the spectral neural-operator
// surrogate: C = alpha * op(A) op(B) + beta * C, op(X) = X or X^T.
//
//   T = __bf16 : v_mfma_f32_32x32x16_bf16 (BF16 operands, FP32 accumulation)
//   T = float  : v_mfma_f32_32x32x2_f32   (FP32 operands; used to check gradients)
//
// An optional second product op(A2) op(B2) (same shapes and layouts, scaled by
// +1 or -1) is accumulated in the same registers, so complex products such as
// Re(W X) = Wr Xr - Wi Xi need no intermediate rounding.
//
// Block tile 64 x 64 (four wavefronts, 32 x 32 each), K tile 32, operands staged
// through LDS as [row][k] so every lane reads its 8 (BF16) or 1 (FP32) consecutive
// k values of one row/column, whatever the storage order in memory.  Operand
// lane layouts (verified on gfx950): A lane l -> row l%32, k = 8(l/32)+i;
// B lane l -> column l%32, same k; D register r -> row 8(r/4)+4(l/32)+r%4,
// column l%32.  Out-of-range rows, columns and k are zero-filled.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sno_internal.h"

namespace qhd {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

namespace {

constexpr int BM = 64, BN = 64, BK = 32;

template <typename T>
struct Lds {
  // row pitch in elements: 32 k values + padding; rows stay 16-byte aligned for the
  // vector stores of the staging
  static constexpr int PITCH = sizeof(T) == 2 ? BK + 8 : BK + 4;
};

template <typename T, bool TRANS>
__device__ __forceinline__ void stage(T* __restrict__ s, const T* __restrict__ g, int ld, int rows,
                                      int K, int r0, int k0, bool negate, bool vec) {
  // stage rows [r0, r0+64) x k [k0, k0+32) of op(X) into s[row][k]; with `vec` (16-byte
  // aligned rows, ld a multiple of the vector length) whole 16-byte vectors are moved
  constexpr int P = Lds<T>::PITCH;
  constexpr int V = 16 / sizeof(T);  // elements per 16-byte vector
  typedef T vecT __attribute__((ext_vector_type(V)));
  if (vec) {
    if (!TRANS) {  // X stored [row][k]: vectors along k
      for (int e = threadIdx.x; e < 64 * (32 / V); e += 256) {
        const int r = e / (32 / V), kv = (e % (32 / V)) * V;
        const int gr = r0 + r, gk = k0 + kv;
        vecT v;
        if (gr < rows && gk + V <= K) {
          v = *reinterpret_cast<const vecT*>(g + (long long)gr * ld + gk);
        } else {
#pragma unroll
          for (int i = 0; i < V; ++i) v[i] = (gr < rows && gk + i < K) ? g[(long long)gr * ld + gk + i] : (T)0.0f;
        }
        if (negate) {
#pragma unroll
          for (int i = 0; i < V; ++i) v[i] = (T)(-(float)v[i]);
        }
        *reinterpret_cast<vecT*>(s + r * P + kv) = v;
      }
    } else {  // X stored [k][row]: vectors along rows, scattered into [row][k]
      for (int e = threadIdx.x; e < 32 * (64 / V); e += 256) {
        const int k = e / (64 / V), rv = (e % (64 / V)) * V;
        const int gr = r0 + rv, gk = k0 + k;
        vecT v;
        if (gk < K && gr + V <= rows) {
          v = *reinterpret_cast<const vecT*>(g + (long long)gk * ld + gr);
        } else {
#pragma unroll
          for (int i = 0; i < V; ++i) v[i] = (gk < K && gr + i < rows) ? g[(long long)gk * ld + gr + i] : (T)0.0f;
        }
#pragma unroll
        for (int i = 0; i < V; ++i) s[(rv + i) * P + k] = negate ? (T)(-(float)v[i]) : v[i];
      }
    }
    return;
  }
  for (int e = threadIdx.x; e < 64 * 32; e += 256) {
    int r, k;
    if (!TRANS) {  // X stored [row][k]: consecutive threads walk k
      r = e >> 5;
      k = e & 31;
    } else {  // X stored [k][row]: consecutive threads walk rows
      k = e >> 6;
      r = e & 63;
    }
    const int gr = r0 + r, gk = k0 + k;
    T v = (T)0.0f;
    if (gr < rows && gk < K) v = TRANS ? g[(long long)gk * ld + gr] : g[(long long)gr * ld + gk];
    s[r * P + k] = negate ? (T)(-(float)v) : v;
  }
}

template <typename T, bool TA, bool TB, typename TO>
__global__ void __launch_bounds__(256) k_gemm(int M, int N, int K, const T* __restrict__ A, int lda,
                                              long long sA, const T* __restrict__ B, int ldb,
                                              long long sB, TO* __restrict__ C, int ldc, long long sC,
                                              float alpha, float beta, const T* __restrict__ A2,
                                              const T* __restrict__ B2, int neg2, int batch, int vecA,
                                              int vecB) {
  constexpr int P = Lds<T>::PITCH;
  __shared__ __attribute__((aligned(16))) T As[BM * P];
  __shared__ __attribute__((aligned(16))) T Bs[BN * P];
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  for (long long bz = blockIdx.z; bz < batch; bz += gridDim.z) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  f32x16 acc = {};
  const int npairs = A2 ? 2 : 1;
  for (int pair = 0; pair < npairs; ++pair) {
    const T* Ap = (pair == 0 ? A : A2) + bz * sA;
    const T* Bp = (pair == 0 ? B : B2) + bz * sB;
    const bool neg = pair == 1 && neg2;
    for (int k0 = 0; k0 < K; k0 += BK) {
      // op(A) is M x K ; op(B) is K x N, staged as [n][k]
      stage<T, TA>(As, Ap, lda, M, K, m0, k0, neg, vecA != 0);
      stage<T, !TB>(Bs, Bp, ldb, N, K, n0, k0, false, vecB != 0);
      __syncthreads();
      if constexpr (sizeof(T) == 2) {
#pragma unroll
        for (int kk = 0; kk < BK; kk += 16) {
          const bf16x8 a = *reinterpret_cast<const bf16x8*>(&As[(wm + (lane & 31)) * P + kk + 8 * (lane >> 5)]);
          const bf16x8 b = *reinterpret_cast<const bf16x8*>(&Bs[(wn + (lane & 31)) * P + kk + 8 * (lane >> 5)]);
          acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        }
      } else {
#pragma unroll
        for (int kk = 0; kk < BK; kk += 2) {
          const float a = As[(wm + (lane & 31)) * P + kk + (lane >> 5)];
          const float b = Bs[(wn + (lane & 31)) * P + kk + (lane >> 5)];
          acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
        }
      }
      __syncthreads();
    }
  }
  TO* Cb = C + bz * sC;
  const int col = n0 + wn + (lane & 31);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = m0 + wm + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    if (row < M && col < N) {
      TO* dst = Cb + (long long)row * ldc + col;
      float v = alpha * acc[r];
      if (beta != 0.0f) v += beta * (float)(*dst);
      *dst = (TO)v;
    }
  }
  }
}

template <typename T, typename TO>
hipError_t dispatch(bool ta, bool tb, const GemmArgs& g, hipStream_t stream) {
  const dim3 grid((g.N + BN - 1) / BN, (g.M + BM - 1) / BM, g.batch < 65535 ? g.batch : 65535);
  const T* A = static_cast<const T*>(g.A);
  const T* B = static_cast<const T*>(g.B);
  TO* C = static_cast<TO*>(g.C);
  const T* A2 = static_cast<const T*>(g.A2);
  const T* B2 = static_cast<const T*>(g.B2);
  const int neg2 = g.scale2 < 0.0f ? 1 : 0;
  if ((A2 == nullptr) != (B2 == nullptr)) return hipErrorInvalidValue;
  // 16-byte vector staging when every row start of every batch entry is 16-byte aligned
  constexpr int V = 16 / sizeof(T);
  auto aligned = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  const int vecA = (g.lda % V == 0 && g.sA % V == 0 && aligned(A) && (!A2 || aligned(A2))) ? 1 : 0;
  const int vecB = (g.ldb % V == 0 && g.sB % V == 0 && aligned(B) && (!B2 || aligned(B2))) ? 1 : 0;
#define QHD_GEMM(TA_, TB_)                                                                    \
  hipLaunchKernelGGL((k_gemm<T, TA_, TB_, TO>), grid, dim3(256), 0, stream, g.M, g.N, g.K, A, \
                     g.lda, g.sA, B, g.ldb, g.sB, C, g.ldc, g.sC, g.alpha, g.beta, A2, B2, neg2, g.batch, \
                     vecA, vecB)
  if (!ta && !tb) QHD_GEMM(false, false);
  else if (!ta && tb) QHD_GEMM(false, true);
  else if (ta && !tb) QHD_GEMM(true, false);
  else QHD_GEMM(true, true);
#undef QHD_GEMM
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm(const GemmArgs& g, hipStream_t stream) {
  if (g.M <= 0 || g.N <= 0 || g.K <= 0 || g.batch <= 0) return hipSuccess;
  if (g.in_bf16) {
    if (g.out_bf16) return dispatch<__bf16, __bf16>(g.transA, g.transB, g, stream);
    return dispatch<__bf16, float>(g.transA, g.transB, g, stream);
  }
  return dispatch<float, float>(g.transA, g.transB, g, stream);
}

}  // namespace qhd
