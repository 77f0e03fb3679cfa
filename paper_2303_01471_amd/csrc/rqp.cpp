// Relaxed QHD for box-constrained QP: the C ABI of include/qhd_rqp.h.
//
// Host side: validation, the eigen-decomposition of the relaxed chain adjacency A'
// (FP64 cyclic Jacobi, once per handle), the schedule per step, and the launch
// sequence of one symmetric step (d axis passes, the merged potential half steps
// fused into the first).  Kernels in rqp_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../../include/qhd_rqp.h"
#include "rqp_internal.h"

namespace qhd {
void set_error_message(const char* msg);
}

using namespace qhd;

struct qhd_rqp_s {
  qhd_rqp_desc desc{};
  std::vector<double> table;  // TABLE schedule (host copy)
  int batch = 0, NP = 0, device = 0;
  long long N = 0;
  float2* psi = nullptr;
  double* f = nullptr;
  double* Qb = nullptr;     // per instance [Q (d x d), b (d)]
  double* U = nullptr;      // eigenvectors of A' (columns), row-major NP x NP
  double* lam = nullptr;    // eigenvalues of A'
  double2* M = nullptr;     // kinetic factor of one axis for the current step (NP x NP)
  double* amp = nullptr;    // discrete Gaussian amplitudes of one axis
  double* fmin = nullptr;
  long long* amin = nullptr;
  double* sums = nullptr;   // [batch][3]
  double* host_sums = nullptr;  // pinned
  std::vector<double> fmin_h;
  std::vector<long long> amin_h;
  std::vector<char> has_obj;
  long long steps_done = 0;
  bool pending = false;     // the trailing potential half step of the last step is owed
  int fused_axes = 0;       // axes 1..K run as one LDS pass (0: every axis its own pass)
};

namespace {

qhd_status rfail(qhd_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  set_error_message(buf);
  return st;
}

#define RQP_TRY(expr)                                                                                 \
  do {                                                                                                \
    hipError_t e_ = (expr);                                                                           \
    if (e_ != hipSuccess)                                                                             \
      return rfail(e_ == hipErrorOutOfMemory ? QHD_ENOMEM : QHD_EDEVICE, "%s: %s", #expr,             \
                   hipGetErrorString(e_));                                                            \
  } while (0)

// symmetric tridiagonal A' of one axis: off-diagonal sqrt((j+1)(r-j)/r), j = 0..r-1
std::vector<double> relaxed_adjacency(int r) {
  const int n = r + 1;
  std::vector<double> A((size_t)n * n, 0.0);
  for (int j = 0; j < r; ++j) {
    const double v = std::sqrt((double)(j + 1) * (double)(r - j) / (double)r);
    A[(size_t)(j + 1) * n + j] = A[(size_t)j * n + j + 1] = v;
  }
  return A;
}

// cyclic Jacobi: A = Z diag(w) Z^T for a real symmetric n x n matrix (row-major)
void jacobi(std::vector<double> A, int n, std::vector<double>& w, std::vector<double>& Z) {
  Z.assign((size_t)n * n, 0.0);
  for (int k = 0; k < n; ++k) Z[(size_t)k * n + k] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += A[(size_t)p * n + q] * A[(size_t)p * n + q];
    if (off < 1e-32) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[(size_t)p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
        const double th = 0.5 * (aqq - app) / apq;
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // A <- A J
          const double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
          A[(size_t)k * n + p] = c * akp - s * akq;
          A[(size_t)k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // A <- J^T A
          const double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
          A[(size_t)p * n + k] = c * apk - s * aqk;
          A[(size_t)q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {  // Z <- Z J
          const double zkp = Z[(size_t)k * n + p], zkq = Z[(size_t)k * n + q];
          Z[(size_t)k * n + p] = c * zkp - s * zkq;
          Z[(size_t)k * n + q] = s * zkp + c * zkq;
        }
      }
  }
  w.resize(n);
  for (int k = 0; k < n; ++k) w[k] = A[(size_t)k * n + k];
}

// a, b of step j at the step midpoint (TABLE: the j-th pair)
void schedule(const qhd_rqp_s* h, long long j, double& a, double& b) {
  const qhd_rqp_desc& d = h->desc;
  if (d.sched_kind == QHD_SCHED_TABLE) {
    a = h->table[2 * j];
    b = h->table[2 * j + 1];
    return;
  }
  if (d.sched_kind == QHD_SCHED_CONST) {
    a = d.sched_p[0];
    b = d.sched_p[1];
    return;
  }
  const double t = ((double)j + 0.5) * d.dt;
  if (d.sched_kind == QHD_SCHED_LINEAR) {
    const double g = t / d.sched_p[0];
    a = 1.0 - g;
    b = g;
  } else {
    const double t3 = t * t * t;
    a = 2.0 / (d.sched_p[0] + t3);
    b = 2.0 * t3;
  }
}

void release(qhd_rqp h) {
  if (!h) return;
  (void)hipSetDevice(h->device);
  for (void* p : {(void*)h->psi, (void*)h->f, (void*)h->Qb, (void*)h->U, (void*)h->lam, (void*)h->M, (void*)h->amp,
                  (void*)h->fmin, (void*)h->amin, (void*)h->sums})
    if (p) (void)hipFree(p);
  if (h->host_sums) (void)hipHostFree(h->host_sums);
  delete h;
}

qhd_status validate(const qhd_rqp_desc* d, int batch) {
  if (!d) return rfail(QHD_EINVAL, "desc is NULL");
  if (batch < 1) return rfail(QHD_EINVAL, "batch must be >= 1");
  if (d->dim < 1 || d->dim > kRqpMaxDim) return rfail(QHD_EINVAL, "dim must be in [1, %d]", kRqpMaxDim);
  if (d->r < 1 || d->r + 1 > kRqpMaxPoints) return rfail(QHD_EINVAL, "r must be in [1, %d]", kRqpMaxPoints - 1);
  if (!std::isfinite(d->dt) || !(d->dt > 0.0)) return rfail(QHD_EINVAL, "dt must be finite and > 0");
  if (d->nsteps < 0) return rfail(QHD_EINVAL, "nsteps must be >= 0");
  if (!std::isfinite(d->min_tol) || d->min_tol < 0.0) return rfail(QHD_EINVAL, "min_tol must be finite and >= 0");
  switch (d->sched_kind) {
    case QHD_SCHED_NESTEROV:
    case QHD_SCHED_LINEAR:
      if (!std::isfinite(d->sched_p[0]) || !(d->sched_p[0] > 0.0))
        return rfail(QHD_EINVAL, "schedule parameter sched_p[0] must be > 0");
      break;
    case QHD_SCHED_CONST:
      if (!std::isfinite(d->sched_p[0]) || !std::isfinite(d->sched_p[1]))
        return rfail(QHD_EINVAL, "CONST schedule needs finite a0, b0");
      break;
    case QHD_SCHED_TABLE:
      if (d->nsteps > 0 && !d->sched_table) return rfail(QHD_EINVAL, "TABLE schedule needs sched_table");
      for (long long j = 0; j < 2 * d->nsteps; ++j)
        if (!std::isfinite(d->sched_table[j])) return rfail(QHD_EINVAL, "sched_table[%lld] is not finite", j);
      break;
    default:
      return rfail(QHD_EINVAL, "unknown sched_kind %d", d->sched_kind);
  }
  double pts = 1.0;
  for (int k = 0; k < d->dim; ++k) pts *= (double)(d->r + 1);
  if (pts > (double)(1 << 24)) return rfail(QHD_EUNSUPPORTED, "(r + 1)^d = %.0f lattice points exceeds 2^24", pts);
  if (pts * batch > 4.0e9) return rfail(QHD_EUNSUPPORTED, "batch x (r + 1)^d exceeds 4e9 points");
  return QHD_OK;
}

}  // namespace

extern "C" {

qhd_status qhd_rqp_create(const qhd_rqp_desc* desc, int32_t batch, qhd_rqp* out) {
  set_error_message("");
  if (!out) return rfail(QHD_EINVAL, "out is NULL");
  *out = nullptr;
  qhd_status st = validate(desc, batch);
  if (st != QHD_OK) return st;
  qhd_rqp h = new qhd_rqp_s;
  h->desc = *desc;
  if (desc->sched_kind == QHD_SCHED_TABLE)
    h->table.assign(desc->sched_table, desc->sched_table + 2 * desc->nsteps);
  h->desc.sched_table = nullptr;
  h->batch = batch;
  h->NP = desc->r + 1;
  h->N = 1;
  for (int k = 0; k < desc->dim; ++k) h->N *= h->NP;
  // the most leading axes whose chunk fits the fused pass's LDS run (QHD_RQP_UNFUSED=1:
  // one pass per axis, the reference form of the same arithmetic)
  const char* unfused = std::getenv("QHD_RQP_UNFUSED");
  if (!(unfused && std::strcmp(unfused, "1") == 0)) {
    long long chunk = h->NP;
    for (int k = 1; k <= desc->dim && chunk <= kFusedPoints; ++k, chunk *= h->NP) h->fused_axes = k;
  }
  h->fmin_h.assign(batch, 0.0);
  h->amin_h.assign(batch, 0);
  h->has_obj.assign(batch, 0);
  hipError_t e = hipGetDevice(&h->device);
  const size_t pts = (size_t)h->N * batch;
  const int d = desc->dim, NP = h->NP;
  if (e == hipSuccess) e = hipMalloc(&h->psi, sizeof(float2) * pts);
  if (e == hipSuccess) e = hipMalloc(&h->f, sizeof(double) * pts);
  if (e == hipSuccess) e = hipMalloc(&h->Qb, sizeof(double) * (size_t)batch * (d * d + d));
  if (e == hipSuccess) e = hipMalloc(&h->U, sizeof(double) * NP * NP);
  if (e == hipSuccess) e = hipMalloc(&h->lam, sizeof(double) * NP);
  if (e == hipSuccess) e = hipMalloc(&h->M, sizeof(double2) * NP * NP);
  if (e == hipSuccess) e = hipMalloc(&h->amp, sizeof(double) * NP);
  if (e == hipSuccess) e = hipMalloc(&h->fmin, sizeof(double) * batch);
  if (e == hipSuccess) e = hipMalloc(&h->amin, sizeof(long long) * batch);
  if (e == hipSuccess) e = hipMalloc(&h->sums, sizeof(double) * 3 * batch);
  if (e == hipSuccess) e = hipHostMalloc((void**)&h->host_sums, sizeof(double) * 3 * batch);
  if (e == hipSuccess) {
    std::vector<double> w, Z, amp(NP);
    jacobi(relaxed_adjacency(desc->r), NP, w, Z);
    double c = std::ldexp(1.0, -desc->r);  // C(r, j) / 2^r, built up multiplicatively
    for (int j = 0; j <= desc->r; ++j) {
      amp[j] = std::sqrt(c);
      c = c * (double)(desc->r - j) / (double)(j + 1);
    }
    e = hipMemcpy(h->U, Z.data(), sizeof(double) * NP * NP, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(h->lam, w.data(), sizeof(double) * NP, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(h->amp, amp.data(), sizeof(double) * NP, hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = hipMemset(h->f, 0, sizeof(double) * pts);
  if (e == hipSuccess) e = rqp_init(h->psi, h->amp, d, NP, h->N, batch, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    st = rfail(e == hipErrorOutOfMemory ? QHD_ENOMEM : QHD_EDEVICE, "relaxed-QP allocation: %s", hipGetErrorString(e));
    release(h);
    return st;
  }
  *out = h;
  return QHD_OK;
}

qhd_status qhd_rqp_set_objective(qhd_rqp h, int32_t i, const double* Q, const double* b) {
  set_error_message("");
  if (!h || !Q || !b) return rfail(QHD_EINVAL, "NULL argument");
  if (i < 0 || i >= h->batch) return rfail(QHD_EINVAL, "instance index %d out of range", i);
  const int d = h->desc.dim;
  std::vector<double> qb((size_t)d * d + d);
  for (int k = 0; k < d; ++k)
    for (int l = 0; l < d; ++l) {
      const double v = 0.5 * (Q[k * d + l] + Q[l * d + k]);
      if (!std::isfinite(v)) return rfail(QHD_EINVAL, "Q[%d][%d] is not finite", k, l);
      qb[(size_t)k * d + l] = v;
    }
  for (int k = 0; k < d; ++k) {
    if (!std::isfinite(b[k])) return rfail(QHD_EINVAL, "b[%d] is not finite", k);
    qb[(size_t)d * d + k] = b[k];
  }
  RQP_TRY(hipSetDevice(h->device));
  double* dst = h->Qb + (size_t)i * qb.size();
  RQP_TRY(hipMemcpy(dst, qb.data(), sizeof(double) * qb.size(), hipMemcpyHostToDevice));
  RQP_TRY(rqp_objective(h->f + (size_t)i * h->N, dst, d, h->NP, h->N, 1, nullptr));
  RQP_TRY(rqp_argmin(h->f + (size_t)i * h->N, h->N, 1, h->fmin + i, h->amin + i, nullptr));
  RQP_TRY(hipMemcpy(&h->fmin_h[i], h->fmin + i, sizeof(double), hipMemcpyDeviceToHost));
  RQP_TRY(hipMemcpy(&h->amin_h[i], h->amin + i, sizeof(long long), hipMemcpyDeviceToHost));
  h->has_obj[i] = 1;
  return QHD_OK;
}

qhd_status qhd_rqp_evolve(qhd_rqp h, int64_t max_steps, void* stream_v) {
  set_error_message("");
  if (!h) return rfail(QHD_EINVAL, "handle is NULL");
  for (int i = 0; i < h->batch; ++i)
    if (!h->has_obj[i]) return rfail(QHD_ESTATE, "instance %d: qhd_rqp_set_objective was not called", i);
  hipStream_t st = (hipStream_t)stream_v;
  RQP_TRY(hipSetDevice(h->device));
  const qhd_rqp_desc& d = h->desc;
  const long long rem = d.nsteps - h->steps_done;
  const long long n = (max_steps < 0 || max_steps > rem) ? rem : max_steps;
  const long long total = h->N * h->batch;
  const double r2 = (double)d.r * (double)d.r;
  for (long long s = 0; s < n; ++s) {
    const long long j = h->steps_done + s;
    double a, b;
    schedule(h, j, a, b);
    // merged potential half steps: the trailing half of step j-1 and the leading half of j
    double beta = 0.5 * d.dt * b;
    if (h->pending || s > 0) {
      double ap, bp;
      schedule(h, j - 1, ap, bp);
      beta += 0.5 * d.dt * bp;
    }
    const double theta = 0.5 * d.dt * a * r2;
    long long stride = 1;
    int k = 0;
    RQP_TRY(rqp_matrix(h->NP, h->U, h->lam, theta, h->M, st));
    if (h->fused_axes > 0) {
      // axes 1..K in one pass through LDS, the rest one pass each
      RQP_TRY(rqp_fused_pass(h->NP, h->psi, h->f, total, h->fused_axes, h->M, beta * 0.15915494309189533577, st));
      for (; k < h->fused_axes; ++k) stride *= h->NP;
    }
    for (; k < d.dim; ++k) {
      RQP_TRY(rqp_axis_pass(h->NP, h->psi, h->f, total, (int)stride, h->M, k == 0, beta * 0.15915494309189533577,
                            st));
      stride *= h->NP;
    }
  }
  if (n > 0) {
    h->steps_done += n;
    h->pending = true;
  }
  return QHD_OK;
}

qhd_status qhd_rqp_observe(qhd_rqp h, void* stream_v, qhd_rqp_obs* out, float* marginals_dev, float* prob_dev,
                           float* psi_dev) {
  set_error_message("");
  if (!h || !out) return rfail(QHD_EINVAL, "NULL argument");
  hipStream_t st = (hipStream_t)stream_v;
  RQP_TRY(hipSetDevice(h->device));
  // the owed potential half step is a phase: |phi|^2, and every readout, is unchanged; the
  // state output gets it (exp(-i (dt/2) b_{j-1} f) of the last step j-1, in turns)
  double close_turns = 0.0;
  if (psi_dev && h->pending && h->steps_done > 0) {
    double a, b;
    schedule(h, h->steps_done - 1, a, b);
    close_turns = 0.5 * h->desc.dt * b * 0.15915494309189533577;
  }
  RQP_TRY(rqp_observe(h->psi, h->f, h->N, h->batch, h->fmin, h->desc.min_tol, h->sums, prob_dev,
                      reinterpret_cast<float2*>(psi_dev), close_turns, st));
  if (marginals_dev) RQP_TRY(rqp_marginals(h->NP, h->psi, h->N, h->desc.dim, h->batch, marginals_dev, st));
  RQP_TRY(hipMemcpyAsync(h->host_sums, h->sums, sizeof(double) * 3 * h->batch, hipMemcpyDeviceToHost, st));
  RQP_TRY(hipStreamSynchronize(st));
  qhd_status status = QHD_OK;
  for (int i = 0; i < h->batch; ++i) {
    const double* s = h->host_sums + 3 * i;
    qhd_rqp_obs& o = out[i];
    o.norm = s[0];
    o.e_f = s[1] / s[0];
    o.p_min = s[2] / s[0];
    o.f_min = h->fmin_h[i];
    o.argmin_index = h->amin_h[i];
    o.steps_done = h->steps_done;
    o.t = (double)h->steps_done * h->desc.dt;
    if (!std::isfinite(o.norm) || !std::isfinite(o.e_f) || !std::isfinite(o.p_min))
      if (status == QHD_OK) status = rfail(QHD_ENUMERIC, "instance %d: non-finite readout", i);
  }
  return status;
}

qhd_status qhd_rqp_reset(qhd_rqp h, void* stream_v) {
  set_error_message("");
  if (!h) return rfail(QHD_EINVAL, "handle is NULL");
  RQP_TRY(hipSetDevice(h->device));
  RQP_TRY(rqp_init(h->psi, h->amp, h->desc.dim, h->NP, h->N, h->batch, (hipStream_t)stream_v));
  h->steps_done = 0;
  h->pending = false;
  return QHD_OK;
}

qhd_status qhd_rqp_points(qhd_rqp h, int64_t* points) {
  set_error_message("");
  if (!h || !points) return rfail(QHD_EINVAL, "NULL argument");
  *points = h->N;
  return QHD_OK;
}

qhd_status qhd_rqp_destroy(qhd_rqp h) {
  set_error_message("");
  if (!h) return QHD_OK;
  (void)hipDeviceSynchronize();
  release(h);
  return QHD_OK;
}

}  // extern "C"
