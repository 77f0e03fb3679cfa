// Internal interfaces of the spectral neural-operator surrogate (sno.cpp,
// sno_gemm.hip, sno_kernels.hip).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>

namespace qhd {

// C[b] = alpha * op(A[b]) op(B[b]) + beta * C[b], b = 0..batch-1, row-major
// storage with leading dimensions; op(X) = X^T when trans is set.
struct GemmArgs {
  int M = 0, N = 0, K = 0, batch = 1;
  const void* A = nullptr;
  int lda = 0;
  long long sA = 0;
  bool transA = false;
  const void* B = nullptr;
  int ldb = 0;
  long long sB = 0;
  bool transB = false;
  void* C = nullptr;
  int ldc = 0;
  long long sC = 0;
  float alpha = 1.0f, beta = 0.0f;
  // optional second product accumulated in the same registers:
  // C = alpha (op(A) op(B) + scale2 op(A2) op(B2)) + beta C, with A2/B2 sharing
  // the leading dimensions, strides and transposition of A/B; scale2 is +1 or -1
  const void* A2 = nullptr;
  const void* B2 = nullptr;
  float scale2 = 1.0f;
  bool in_bf16 = true;   // operands BF16 (else FP32)
  bool out_bf16 = false; // C BF16 (only with BF16 operands), else FP32
};

hipError_t launch_gemm(const GemmArgs& g, hipStream_t stream);

// Elementwise / reduction kernels (sno_kernels.hip).  `bf16` selects the
// activation storage type (BF16 or FP32).
hipError_t sno_prep_input(const double* f, int batch, int S, void* in, bool bf16, hipStream_t st);
// z += bias; h = z (act 0) or GELU(z) (act 1)
hipError_t sno_bias_act(float* z, const float* bias, long long rows, int C, void* h, bool bf16, int act,
                        hipStream_t st, bool keep_z = true);
// inference at width 32 in BF16: features and lift (h0 = x0 Wl^T + bl, Wl is C x 3) in one pass
hipError_t sno_prep_lift32(const double* f, int batch, int S, const void* Wl, const float* bl, void* h,
                           hipStream_t st);
// inference at width 32, 16 modes, BF16: per row of S pixels (nrows = batch x S rows),
// out = act(gx U_row + h W^T + bias); gx is S x 32, U holds a 32 x 32 block per row, S % 32 == 0.
// With fx (32 x S) non-null, also T_row = fx out_row (the next layer's forward x-contraction) into
// T, which may be U.
// With q non-null (and fx null) the outputs are not stored: per pixel the logit
// q = bp + sum_c out[c] wp[c] goes to q (nrows x S floats) instead.
hipError_t sno_spectral_pointwise32(const void* gx, const void* U, const void* h, const void* W, const float* bias,
                                    int S, long long nrows, void* out, int act, const void* fx, void* T,
                                    const float* wp, const float* bp, float* q, hipStream_t st);
// per sample, softmax of npix logits in place (as sno_project_softmax forms it)
hipError_t sno_softmax_rows(float* rho, int batch, int npix, hipStream_t st);
// width 32, 16 modes, BF16: per row of S pixels (nrows = batch x S), T_row (32 x 32) = fx (32 x S) X_row;
// S % 16 == 0
hipError_t sno_dft_x32(const void* fx, const void* X, int S, long long nrows, void* T, hipStream_t st);
// width 32, 16 modes, BF16: per sample U (2S x 512, row stride 512, sample stride 1024 S) =
// Gy (2S x 64) G_b (64 x 512, sample stride gstride); S % 16 == 0
hipError_t sno_inv_y32(const void* Gy, const void* G, long long gstride, int batch, int S, void* U, hipStream_t st);
// width 32, 16 modes, BF16, S % 16 == 0 and S <= 256: per sample [Hr; Hi] (64 x 512, row stride
// 512, sample stride hstride) = Fy1 (64 x S) T_r + Fy2 (64 x S) T_i, T_b (S x 1024, halves r | i)
hipError_t sno_fwd_y32(const void* Fy1, const void* Fy2, const void* T, int batch, int S, void* H, long long hstride,
                       hipStream_t st);
// width 32, BF16: per mode m and sample b, G = R[m] H (complex; R [mode][out][in] as Rr, Ri;
// spectra [b][re | im][mode][channel] with sample stride spec)
hipError_t sno_mix32(const void* H, const void* Rr, const void* Ri, int nmodes, long long spec, int batch, void* G,
                     hipStream_t st);
// inference: out = act(z + h W^T + b) in BF16 for width 32 (h, W, out BF16; z, b FP32)
hipError_t sno_pointwise32(const void* h, const void* W, const float* z, const float* bias, long long npix,
                           void* out, int act, hipStream_t st);
hipError_t sno_project_softmax(const void* h, const float* wp, const float* bp, int batch, int npix,
                               int C, bool bf16, float* rho, hipStream_t st);
hipError_t sno_loss_grad(const float* rho_hat, const float* rho, int batch, int npix, float* dq,
                         double* loss_per_sample, hipStream_t st);
hipError_t sno_project_backward(const float* dq, const void* h, const float* wp, int batch, int npix,
                                int C, bool bf16, float* dh, float* partials, int nparts,
                                hipStream_t st);
// dz = dh * GELU'(z) (stored as T) and nparts x C partial column sums of dz (FP32, before rounding)
hipError_t sno_gelu_backward(const float* dh, const float* z, long long rows, int C, void* dz, bool bf16,
                             float* partials, int nparts, hipStream_t st);
hipError_t sno_colsum(const void* x, bool bf16, long long rows, int C, float* partials, int nparts,
                      hipStream_t st);
hipError_t sno_reduce_partials(const float* partials, int nparts, int len, float* out, bool accumulate,
                               hipStream_t st);
hipError_t sno_cast(const float* src, void* dst, long long n, bool bf16, hipStream_t st);
hipError_t sno_adam(float* p, const float* g, float* m, float* v, long long n, float lr, float b1,
                    float b2, float eps, float c1, float c2, void* copy, bool bf16, hipStream_t st);
hipError_t sno_fill(float* p, long long n, float v, hipStream_t st);

}  // namespace qhd
