// qhd_spectrum: lowest eigenpairs of the discrete QHD Hamiltonian
//     H(t) = a(t) K + b(t) diag(f),   K = F^{-1} diag(|k|^2/2) F
// of one 2-D instance (the operator whose exponentials the split-operator step
// multiplies, App. C.2.1 eq. prod_qhd_fft; its low-lying spectrum along the path is
// what App. D studies), by the Lanczos iteration with full reorthogonalisation.
// The matrix-vector products and the Krylov vector operations run on the GPU
// (qhd_spectrum_kernels.hip); the tridiagonal eigenproblem (at most 400 x 400) is
// solved on the host by cyclic Jacobi rotations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <numeric>
#include <vector>

#include "../../include/qhd.h"
#include "qhd_internal.h"

namespace qhd {
void set_error_message(const char* msg);
qhd_status plan_instance_view(qhd_plan p, int i, InstanceView* v);
}  // namespace qhd

using namespace qhd;

namespace {

qhd_status sfail(qhd_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  set_error_message(buf);
  return st;
}

#define SP_TRY(expr)                                                                           \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      return sfail(e_ == hipErrorOutOfMemory ? QHD_ENOMEM : QHD_EDEVICE, "%s: %s", #expr,        \
                   hipGetErrorString(e_));                                                     \
  } while (0)

constexpr int kMaxKrylov = 400;
constexpr int kDotBlocks = 128;

// a(t), b(t) of the instance's schedule at time t
qhd_status schedule_at(const InstanceView& v, double t, double& a, double& b) {
  const InstDev& I = v.host;
  if (I.sched == kSchedConst) {
    a = I.sched_p0;
    b = I.sched_p1;
  } else if (I.sched == kSchedTable) {
    if (I.nsteps <= 0) return sfail(QHD_EINVAL, "TABLE schedule with no steps");
    long long j = (long long)std::floor(t / I.dt);
    j = std::min(std::max(j, 0LL), I.nsteps - 1);
    double ab[2];
    hipError_t e = hipMemcpy(ab, I.table + 2 * j, sizeof ab, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return sfail(QHD_EDEVICE, "schedule table read: %s", hipGetErrorString(e));
    a = ab[0];
    b = ab[1];
  } else {
    const double t3 = t * t * t;
    a = 2.0 / (I.sched_p0 + t3);
    b = 2.0 * t3;
  }
  return QHD_OK;
}

// Eigen-decomposition of a real symmetric m x m matrix (row-major) by cyclic Jacobi
// rotations; eigenvalues in w, eigenvectors in the columns of z.
void jacobi_eigen(std::vector<double> A, int m, std::vector<double>& w, std::vector<double>& z) {
  z.assign((size_t)m * m, 0.0);
  for (int k = 0; k < m; ++k) z[(size_t)k * m + k] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int p = 0; p < m; ++p)
      for (int q = 0; q < m; ++q) {
        const double v2 = A[(size_t)p * m + q] * A[(size_t)p * m + q];
        tot += v2;
        if (p != q) off += v2;
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int p = 0; p < m - 1; ++p)
      for (int q = p + 1; q < m; ++q) {
        const double apq = A[(size_t)p * m + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double app = A[(size_t)p * m + p], aqq = A[(size_t)q * m + q];
        // rotation angle that zeroes A[p][q]: tan(2 phi) = 2 apq / (aqq - app)
        const double theta = (aqq - app) / (2.0 * apq);
        const double tt = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(tt * tt + 1.0), s = tt * c;
        for (int k = 0; k < m; ++k) {  // columns p, q
          const double akp = A[(size_t)k * m + p], akq = A[(size_t)k * m + q];
          A[(size_t)k * m + p] = c * akp - s * akq;
          A[(size_t)k * m + q] = s * akp + c * akq;
        }
        for (int k = 0; k < m; ++k) {  // rows p, q
          const double apk = A[(size_t)p * m + k], aqk = A[(size_t)q * m + k];
          A[(size_t)p * m + k] = c * apk - s * aqk;
          A[(size_t)q * m + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < m; ++k) {
          const double zkp = z[(size_t)k * m + p], zkq = z[(size_t)k * m + q];
          z[(size_t)k * m + p] = c * zkp - s * zkq;
          z[(size_t)k * m + q] = s * zkp + c * zkq;
        }
      }
  }
  w.resize(m);
  for (int k = 0; k < m; ++k) w[k] = A[(size_t)k * m + k];
}

struct Work {
  float2* V = nullptr;   // (m + 1) Krylov vectors
  float2* u = nullptr;   // matvec scratch
  float2* x = nullptr;   // Ritz vector
  float2* r = nullptr;   // residual
  double* partials = nullptr;
  double* coef = nullptr;
  ~Work() {
    (void)hipFree(V);
    (void)hipFree(u);
    (void)hipFree(x);
    (void)hipFree(r);
    (void)hipFree(partials);
    (void)hipFree(coef);
  }
};

struct Ctx {
  const InstanceView& v;
  Work& w;
  long long n;
  double a, b;
  hipStream_t st;
  std::vector<double> hp;  // host partials

  // out = H in (in and out distinct)
  qhd_status matvec(const float2* in, float2* out) {
    const double L0 = v.length[0], L1 = v.length[1];
    const double cx = 0.5 * std::pow(2.0 * M_PI / L0, 2) * a, cy = 0.5 * std::pow(2.0 * M_PI / L1, 2) * a;
    SP_TRY(hipMemcpyAsync(w.u, in, sizeof(float2) * n, hipMemcpyDeviceToDevice, st));
    SP_TRY(spec_lines(0, -1, w.u, v.nx, v.ny, v.tw_x, st));
    SP_TRY(spec_lines(1, -1, w.u, v.nx, v.ny, v.tw_y, st));
    SP_TRY(spec_kinetic(w.u, v.nx, v.ny, cx, cy, 1.0 / (double)n, st));
    SP_TRY(spec_lines(1, +1, w.u, v.nx, v.ny, v.tw_y, st));
    SP_TRY(spec_lines(0, +1, w.u, v.nx, v.ny, v.tw_x, st));
    SP_TRY(spec_finish(out, w.u, in, v.f, b, v.nx, v.ny, st));
    return QHD_OK;
  }

  // c[i] = <V_i, y> for i < count (complex, FP64), synchronous
  qhd_status dots(const float2* Vb, int count, const float2* y, std::vector<double>& c) {
    SP_TRY(spec_multidot(Vb, n, count, y, w.partials, kDotBlocks, st));
    hp.resize((size_t)count * kDotBlocks * 2);
    SP_TRY(hipMemcpyAsync(hp.data(), w.partials, sizeof(double) * hp.size(), hipMemcpyDeviceToHost, st));
    SP_TRY(hipStreamSynchronize(st));
    c.assign((size_t)2 * count, 0.0);
    for (int i = 0; i < count; ++i)
      for (int k = 0; k < kDotBlocks; ++k) {
        c[2 * i] += hp[((size_t)i * kDotBlocks + k) * 2];
        c[2 * i + 1] += hp[((size_t)i * kDotBlocks + k) * 2 + 1];
      }
    return QHD_OK;
  }

  // y <- scale (y - sum_i c_i V_i)
  qhd_status axpy(float2* y, const float2* Vb, int count, const std::vector<double>& c, double scale) {
    if (count > 0) {
      // the host vector is reused by the caller: finish the upload before returning
      SP_TRY(hipMemcpyAsync(w.coef, c.data(), sizeof(double) * 2 * count, hipMemcpyHostToDevice, st));
      SP_TRY(hipStreamSynchronize(st));
    }
    SP_TRY(spec_multiaxpy(y, Vb, n, count, w.coef, scale, st));
    return QHD_OK;
  }

  qhd_status norm(const float2* y, double& out) {
    std::vector<double> c;
    qhd_status s = dots(y, 1, y, c);
    if (s != QHD_OK) return s;
    out = std::sqrt(std::max(c[0], 0.0));
    return QHD_OK;
  }
};

}  // namespace

extern "C" qhd_status qhd_spectrum(qhd_plan plan, int32_t i, double t, int32_t nev, int32_t krylov,
                                   const float* psi_dev, double* energies, double* overlaps, double* residuals,
                                   void* stream) {
  set_error_message("");
  if (!plan || !energies) return sfail(QHD_EINVAL, "plan and energies must not be NULL");
  InstanceView v;
  qhd_status s = plan_instance_view(plan, i, &v);
  if (s != QHD_OK) return s;
  if (v.ndim != 2) return sfail(QHD_EUNSUPPORTED, "qhd_spectrum supports 2-D instances (instance %d is %d-D)", i, v.ndim);
  if (v.host.model != kModelQHD) return sfail(QHD_EUNSUPPORTED, "qhd_spectrum is built for the QHD Hamiltonian");
  if (!v.potential_set) return sfail(QHD_ESTATE, "instance %d: qhd_set_potential was not called", i);
  const long long n = (long long)v.nx * v.ny;
  if (nev < 1) return sfail(QHD_EINVAL, "nev must be >= 1");
  if (krylov <= nev || krylov > kMaxKrylov || krylov > n)
    return sfail(QHD_EINVAL, "krylov %d must be in (nev, min(%d, points)]", krylov, kMaxKrylov);
  if (!std::isfinite(t) || t < 0.0) return sfail(QHD_EINVAL, "t must be finite and >= 0");
  if (overlaps && !psi_dev) return sfail(QHD_EINVAL, "overlaps need psi_dev");
  hipStream_t st = (hipStream_t)stream;
  SP_TRY(hipSetDevice(v.device));
  SP_TRY(hipStreamSynchronize(v.internal));  // potentials uploaded on the plan's stream
  Work work;  // device buffers, freed on every return
  Ctx c{v, work, n, 0.0, 0.0, st, {}};
  s = schedule_at(v, t, c.a, c.b);
  if (s != QHD_OK) return s;
  const int m = krylov;
  SP_TRY(hipMalloc(&c.w.V, sizeof(float2) * n * (m + 1)));
  SP_TRY(hipMalloc(&c.w.u, sizeof(float2) * n));
  SP_TRY(hipMalloc(&c.w.x, sizeof(float2) * n));
  SP_TRY(hipMalloc(&c.w.r, sizeof(float2) * n));
  SP_TRY(hipMalloc(&c.w.partials, sizeof(double) * 2 * kDotBlocks * (m + 1)));
  SP_TRY(hipMalloc(&c.w.coef, sizeof(double) * 2 * (m + 1)));
  float2* V = c.w.V;
  std::vector<double> alpha, beta, co;
  // deterministic start vector, normalised
  SP_TRY(spec_random(V, n, 0x51ED5EEDull + (unsigned long long)i, st));
  double nrm = 0.0;
  if ((s = c.norm(V, nrm)) != QHD_OK) return s;
  if ((s = c.axpy(V, V, 0, co, 1.0 / nrm)) != QHD_OK) return s;
  int mm = 0;
  for (int j = 0; j < m; ++j) {
    float2* w = V + (long long)(j + 1) * n;
    if ((s = c.matvec(V + (long long)j * n, w)) != QHD_OK) return s;
    double a_j = 0.0;
    for (int pass = 0; pass < 2; ++pass) {  // classical Gram-Schmidt, twice
      if ((s = c.dots(V, j + 1, w, co)) != QHD_OK) return s;
      if (pass == 0) a_j = co[2 * j];
      if ((s = c.axpy(w, V, j + 1, co, 1.0)) != QHD_OK) return s;
    }
    double b_j = 0.0;
    if ((s = c.norm(w, b_j)) != QHD_OK) return s;
    alpha.push_back(a_j);
    mm = j + 1;
    if (!(b_j > 1e-10 * std::max(1.0, std::fabs(a_j)))) break;  // invariant subspace
    beta.push_back(b_j);
    if ((s = c.axpy(w, V, 0, co, 1.0 / b_j)) != QHD_OK) return s;
  }
  if (mm < nev) return sfail(QHD_ENUMERIC, "Krylov space exhausted after %d steps (< nev = %d)", mm, nev);
  std::vector<double> T((size_t)mm * mm, 0.0), evals, evecs;
  for (int k = 0; k < mm; ++k) {
    T[(size_t)k * mm + k] = alpha[k];
    if (k + 1 < mm) T[(size_t)k * mm + k + 1] = T[(size_t)(k + 1) * mm + k] = beta[k];
  }
  jacobi_eigen(T, mm, evals, evecs);
  std::vector<int> order(mm);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int p, int q) { return evals[p] < evals[q]; });
  double psi_norm2 = 0.0;
  if (psi_dev) {
    std::vector<double> pc;
    if ((s = c.dots((const float2*)psi_dev, 1, (const float2*)psi_dev, pc)) != QHD_OK) return s;
    psi_norm2 = pc[0];
  }
  for (int k = 0; k < nev; ++k) {
    const int col = order[k];
    energies[k] = evals[col];
    if (!residuals && !overlaps) continue;
    // Ritz vector x = sum_j y_j V_j
    std::vector<double> y(2 * (size_t)mm, 0.0);
    for (int j = 0; j < mm; ++j) y[2 * j] = -evecs[(size_t)j * mm + col];
    SP_TRY(hipMemsetAsync(c.w.x, 0, sizeof(float2) * n, st));
    if ((s = c.axpy(c.w.x, V, mm, y, 1.0)) != QHD_OK) return s;
    double xn = 0.0;
    if ((s = c.norm(c.w.x, xn)) != QHD_OK) return s;
    if ((s = c.axpy(c.w.x, V, 0, co, 1.0 / xn)) != QHD_OK) return s;
    if (residuals) {
      if ((s = c.matvec(c.w.x, c.w.r)) != QHD_OK) return s;
      std::vector<double> th = {evals[col], 0.0};
      if ((s = c.axpy(c.w.r, c.w.x, 1, th, 1.0)) != QHD_OK) return s;
      if ((s = c.norm(c.w.r, residuals[k])) != QHD_OK) return s;
    }
    if (overlaps) {
      std::vector<double> ov;
      if ((s = c.dots(c.w.x, 1, (const float2*)psi_dev, ov)) != QHD_OK) return s;
      overlaps[k] = (ov[0] * ov[0] + ov[1] * ov[1]) / std::max(psi_norm2, 1e-300);
    }
  }
  SP_TRY(hipStreamSynchronize(st));
  return QHD_OK;
}
