// Declarations shared by the relaxed-QP host code (rqp.cpp) and its kernels
// (rqp_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace qhd {

constexpr int kRqpMaxDim = 8;
constexpr int kRqpMaxPoints = 16;  // r + 1 <= 16

// M = U diag(e^{i theta lam}) U^T (NP x NP, FP64 complex, row-major) into device memory.
hipError_t rqp_matrix(int NP, const double* U, const double* lam, double theta, double2* M, hipStream_t st);
// One axis pass over every instance: lines of `stride` (points of one axis are
// `stride` apart) times M; with fuse_v the potential factor exp(-2 pi i beta_turns f)
// first (stride 1 only).  total_points = batch * N.
hipError_t rqp_axis_pass(int NP, float2* psi, const double* f, long long total_points, int stride, const double2* M,
                         bool fuse_v, double beta_turns, hipStream_t st);
// Axes 1..K in one pass (with the potential factor first), K >= 1 and NP^K <= kFusedPoints:
// the same values as K axis passes.
constexpr int kFusedPoints = 6561;  // 9^4: 52.5 KB of FP32 complex values in LDS per block
hipError_t rqp_fused_pass(int NP, float2* psi, const double* f, long long total_points, int K, const double2* M,
                          double beta_turns, hipStream_t st);
hipError_t rqp_marginals(int NP, const float2* psi, long long N, int d, int batch, float* marg, hipStream_t st);
hipError_t rqp_objective(double* f, const double* Qb, int d, int NP, long long N, int batch, hipStream_t st);
hipError_t rqp_argmin(const double* f, long long N, int batch, double* fmin, long long* amin, hipStream_t st);
hipError_t rqp_init(float2* psi, const double* amp, int d, int NP, long long N, int batch, hipStream_t st);
// Sums per instance (rho, f rho, rho over the minimisers), optional rho output and, with
// psi_out, the state times exp(-2 pi i close_turns f) (the owed potential half step)
hipError_t rqp_observe(const float2* psi, const double* f, long long N, int batch, const double* fmin, double tol,
                       double* out, float* prob, float2* psi_out, double close_turns, hipStream_t st);

}  // namespace qhd
