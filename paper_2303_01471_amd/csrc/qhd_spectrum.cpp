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
constexpr int kDotBlocks = 16;  // blocks per vector of a multidot (partials summed in order)
constexpr int kAxpyGroups = 8;  // groups of the grouped multiaxpy

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

// Lowest eigenpairs of the Lanczos matrix: the symmetric tridiagonal T with diagonal
// d[0..m) and off-diagonal e[0..m-1) (e[i] couples i and i+1).

// number of eigenvalues of T below x (Sylvester's law of inertia on the LDL^T pivots)
int sturm_count(const std::vector<double>& d, const std::vector<double>& e, double x, double tiny) {
  int neg = 0;
  double q = 1.0;
  for (size_t i = 0; i < d.size(); ++i) {
    const double e2 = i > 0 ? e[i - 1] * e[i - 1] : 0.0;
    q = (d[i] - x) - (i > 0 ? e2 / q : 0.0);
    if (q == 0.0) q = -tiny;
    if (q < 0.0) ++neg;
  }
  return neg;
}

// the k-th smallest eigenvalue (k from 0) by bisection on the Sturm count inside the
// Gershgorin interval [lo, hi]
double kth_eigenvalue(const std::vector<double>& d, const std::vector<double>& e, int k, double lo, double hi,
                      double tiny) {
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (!(mid > lo && mid < hi)) break;  // the interval is one ulp wide
    if (sturm_count(d, e, mid, tiny) > k) hi = mid;
    else lo = mid;
  }
  return 0.5 * (lo + hi);
}

// eigenvector of T for the eigenvalue lam by inverse iteration: (T - lam I) x = b solved
// by Gaussian elimination with row interchanges (the band of U grows to two
// super-diagonals), x orthogonalised against the vectors of eigenvalues closer than
// `gap` (earlier members of a cluster) and normalised, three times from a fixed start
void inverse_iteration(const std::vector<double>& d, const std::vector<double>& e, double lam, double tiny,
                       const std::vector<std::vector<double>>& close, std::vector<double>& x) {
  const int m = (int)d.size();
  std::vector<double> dd(m), du(m, 0.0), du2(m, 0.0), dl(m, 0.0);
  std::vector<char> swp(m, 0);
  for (int i = 0; i < m; ++i) dd[i] = d[i] - lam;
  for (int i = 0; i + 1 < m; ++i) du[i] = dl[i] = e[i];
  for (int i = 0; i + 1 < m; ++i) {
    if (std::fabs(dd[i]) >= std::fabs(dl[i])) {
      if (dd[i] == 0.0) dd[i] = tiny;
      const double f = dl[i] / dd[i];
      dl[i] = f;
      dd[i + 1] -= f * du[i];
    } else {  // interchange rows i and i + 1
      const double f = dd[i] / dl[i];
      dd[i] = dl[i];
      dl[i] = f;
      const double t = du[i];
      du[i] = dd[i + 1];
      dd[i + 1] = t - f * dd[i + 1];
      if (i + 2 < m) {
        du2[i] = du[i + 1];
        du[i + 1] = -f * du[i + 1];
      }
      swp[i] = 1;
    }
  }
  if (dd[m - 1] == 0.0) dd[m - 1] = tiny;
  x.assign(m, 0.0);
  std::vector<double> b(m);
  for (int i = 0; i < m; ++i) b[i] = 1.0 + 0.1 * std::sin(1.0 + 2.3 * i);  // fixed, no special structure
  for (int it = 0; it < 3; ++it) {
    for (int i = 0; i + 1 < m; ++i) {  // L
      if (swp[i]) std::swap(b[i], b[i + 1]);
      b[i + 1] -= dl[i] * b[i];
    }
    for (int i = m - 1; i >= 0; --i) {  // U
      double v = b[i];
      if (i + 1 < m) v -= du[i] * x[i + 1];
      if (i + 2 < m) v -= du2[i] * x[i + 2];
      x[i] = v / dd[i];
    }
    for (const auto& u : close) {
      double p = 0.0;
      for (int i = 0; i < m; ++i) p += u[i] * x[i];
      for (int i = 0; i < m; ++i) x[i] -= p * u[i];
    }
    double nn = 0.0;
    for (int i = 0; i < m; ++i) nn += x[i] * x[i];
    nn = std::sqrt(nn);
    for (int i = 0; i < m; ++i) b[i] = x[i] /= nn;
  }
}

// the nev lowest eigenvalues of T (ascending) and their unit eigenvectors
void tridiag_lowest(const std::vector<double>& d, const std::vector<double>& e, int nev, std::vector<double>& w,
                    std::vector<std::vector<double>>& z) {
  const int m = (int)d.size();
  double lo = d[0], hi = d[0], big = 0.0;
  for (int i = 0; i < m; ++i) {
    const double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(e[i]) : 0.0);
    lo = std::min(lo, d[i] - r);
    hi = std::max(hi, d[i] + r);
    big = std::max(big, std::fabs(d[i]) + r);
  }
  const double tiny = 1e-300 + 1e-16 * big;
  w.resize(nev);
  z.assign(nev, {});
  for (int k = 0; k < nev; ++k) w[k] = kth_eigenvalue(d, e, k, lo, hi, tiny);
  for (int k = 0; k < nev; ++k) {
    std::vector<std::vector<double>> close;
    for (int j = 0; j < k; ++j)
      if (std::fabs(w[k] - w[j]) < 1e-8 * big) close.push_back(z[j]);
    inverse_iteration(d, e, w[k], tiny, close, z[k]);
  }
}

struct Work {
  float2* V = nullptr;   // (m + 1) Krylov vectors
  float2* u = nullptr;   // matvec scratch
  float2* x = nullptr;   // Ritz vector
  float2* r = nullptr;   // residual
  double* partials = nullptr;
  double* coef = nullptr;
  double* hist = nullptr;  // Lanczos diagonal and off-diagonal entries, norm and scale
  double2* part = nullptr;  // grouped multiaxpy sums
  ~Work() {
    (void)hipFree(hist);
    (void)hipFree(part);
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
    SP_TRY(spec_multiaxpy(y, Vb, n, count, w.coef, scale, st, nullptr, w.part, kAxpyGroups));
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
  SP_TRY(hipMalloc(&c.w.hist, sizeof(double) * (2 * m + 2)));
  SP_TRY(hipMalloc(&c.w.part, sizeof(double2) * n * kAxpyGroups));
  float2* V = c.w.V;
  std::vector<double> alpha, beta, co;
  // The Lanczos recurrence runs on the stream without host round trips: the
  // Gram-Schmidt coefficients and norms are reduced on the device (block partials summed
  // in block order in FP64, the sums a host loop would form) and used there; the
  // diagonal and off-diagonal entries are kept in device memory and read once at the
  // end.  A breakdown (an invariant subspace) is found there too: the recurrence keeps
  // going on meaningless vectors and the tridiagonal matrix is cut at the first
  // vanishing off-diagonal entry.
  double* d_alpha = c.w.hist;
  double* d_beta = c.w.hist + m;
  double* d_nrm = c.w.hist + 2 * m;
  double* d_scale = c.w.hist + 2 * m + 1;
  // deterministic start vector, normalised
  SP_TRY(spec_random(V, n, 0x51ED5EEDull + (unsigned long long)i, st));
  SP_TRY(spec_multidot(V, n, 1, V, c.w.partials, kDotBlocks, st));
  SP_TRY(spec_norm(c.w.partials, kDotBlocks, d_nrm, d_scale, st));
  SP_TRY(spec_multiaxpy(V, V, n, 0, c.w.coef, 0.0, st, d_scale));
  for (int j = 0; j < m; ++j) {
    float2* w = V + (long long)(j + 1) * n;
    if ((s = c.matvec(V + (long long)j * n, w)) != QHD_OK) return s;
    for (int pass = 0; pass < 2; ++pass) {  // classical Gram-Schmidt, twice
      SP_TRY(spec_multidot(V, n, j + 1, w, c.w.partials, kDotBlocks, st));
      SP_TRY(spec_coef(c.w.partials, j + 1, kDotBlocks, c.w.coef, pass == 0 ? d_alpha + j : nullptr, st));
      SP_TRY(spec_multiaxpy(w, V, n, j + 1, c.w.coef, 1.0, st, nullptr, c.w.part, kAxpyGroups));
    }
    SP_TRY(spec_multidot(w, n, 1, w, c.w.partials, kDotBlocks, st));
    SP_TRY(spec_norm(c.w.partials, kDotBlocks, d_beta + j, d_scale, st));
    SP_TRY(spec_multiaxpy(w, V, n, 0, c.w.coef, 0.0, st, d_scale));
  }
  {
    std::vector<double> hab((size_t)2 * m);
    SP_TRY(hipMemcpyAsync(hab.data(), c.w.hist, sizeof(double) * 2 * m, hipMemcpyDeviceToHost, st));
    SP_TRY(hipStreamSynchronize(st));
    for (int j = 0; j < m; ++j) {
      const double a_j = hab[j], b_j = hab[m + j];
      alpha.push_back(a_j);
      if (!(b_j > 1e-10 * std::max(1.0, std::fabs(a_j)))) break;  // invariant subspace
      beta.push_back(b_j);
    }
  }
  const int mm = (int)alpha.size();
  if (mm < nev) return sfail(QHD_ENUMERIC, "Krylov space exhausted after %d steps (< nev = %d)", mm, nev);
  std::vector<double> evals;
  std::vector<std::vector<double>> evecs;
  beta.resize(mm > 0 ? mm - 1 : 0);
  tridiag_lowest(alpha, beta, nev, evals, evecs);
  double psi_norm2 = 0.0;
  if (psi_dev) {
    std::vector<double> pc;
    if ((s = c.dots((const float2*)psi_dev, 1, (const float2*)psi_dev, pc)) != QHD_OK) return s;
    psi_norm2 = pc[0];
  }
  for (int k = 0; k < nev; ++k) {
    energies[k] = evals[k];
    if (!residuals && !overlaps) continue;
    // Ritz vector x = sum_j y_j V_j
    std::vector<double> y(2 * (size_t)mm, 0.0);
    for (int j = 0; j < mm; ++j) y[2 * j] = -evecs[k][j];
    SP_TRY(hipMemsetAsync(c.w.x, 0, sizeof(float2) * n, st));
    if ((s = c.axpy(c.w.x, V, mm, y, 1.0)) != QHD_OK) return s;
    double xn = 0.0;
    if ((s = c.norm(c.w.x, xn)) != QHD_OK) return s;
    if ((s = c.axpy(c.w.x, V, 0, co, 1.0 / xn)) != QHD_OK) return s;
    if (residuals) {
      if ((s = c.matvec(c.w.x, c.w.r)) != QHD_OK) return s;
      std::vector<double> th = {evals[k], 0.0};
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
