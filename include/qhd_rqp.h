/*
 * qhd_rqp.h - C ABI of the relaxed QHD for box-constrained quadratic programming.
 *
 * What it computes (paper: App. F.2, eqs. relaxed-qhd-discrete, d_relaxed_adjacency,
 * relaxed_adjacency, and Algorithm 2; simulated on a classical machine as the paper's
 * Sim-QHD of App. G):
 *   minimise f(x) = 1/2 x^T Q x + b^T x  over the box [0, 1]^d  (eq. qp-analog)
 *   lattice    x_k = j_k / r, j_k = 0..r on every axis (r cells, r + 1 points, not
 *              periodic); state phi over (j_1, ..., j_d), j_1 fastest
 *   H(t)     = -(a(t) / 2) r^2 A'_d + b(t) F_d,   A'_d = sum_k (A' on axis k),
 *              F_d = diag f on the lattice, A' the symmetric tridiagonal (r+1)x(r+1)
 *              matrix with off-diagonal entries sqrt((j+1)(r-j)/r), j = 0..r-1
 *              (Hamming encoding: S_x / sqrt(r) on the symmetric subspace of r qubits,
 *              App. F.3; r^2 = 1/h^2 is the finite-difference scale of the Laplacian)
 *   phi_0    = prod_k sqrt(C(r, j_k) / 2^r), the discrete Gaussian image of the uniform
 *              superposition of the d r qubits (App. F.3, prop. multi-gaussian)
 *   stepping   symmetric split step with a, b at the step midpoint; the kinetic factor
 *              exp(+i dt a r^2 / 2 A') acts along every axis as one (r+1)x(r+1) complex
 *              matrix, formed in FP64 from the eigen-decomposition of A' (computed once
 *              on the host); the state is FP32 complex, every product accumulates in FP64
 *   readouts   norm, E[f], the probability of the lattice minimisers, per-axis
 *              marginal distributions (the measurement of Algorithm 2)
 * The paper's Sim-QHD uses the D-Wave annealing curves A(s), B(s) (App. G), which are
 * not reproduced here: pass them as a QHD_SCHED_TABLE of per-step (a_j, b_j) values,
 * or use NESTEROV / CONST / LINEAR.
 *
 * Conventions as in qhd.h: qhd_status codes, qhd_last_error(), device pointers on the
 * device current at creation, "stream" = hipStream_t (NULL: the default stream).  A
 * handle is not thread-safe.  Every instance of a handle shares d, r, dt, nsteps and
 * the schedule; each has its own (Q, b).
 */
#ifndef QHD_RQP_H
#define QHD_RQP_H

#include <stdint.h>

#include "qhd.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qhd_rqp_s *qhd_rqp;

typedef struct {
  int32_t dim;        /* d, 1 <= d <= 8                                                */
  int32_t r;          /* cells per axis, 1 <= r <= 15 (r + 1 lattice points per axis);
                         (r + 1)^d <= 2^24 points per instance                           */
  double dt;          /* step > 0                                                      */
  int64_t nsteps;     /* steps to the end time T = nsteps dt, >= 0                     */
  int32_t sched_kind; /* qhd_sched_kind: NESTEROV, CONST, LINEAR or TABLE              */
  double sched_p[2];  /* schedule parameters as in qhd.h                               */
  const double *sched_table; /* TABLE: host array of 2 nsteps doubles, copied           */
  double min_tol;     /* lattice points with f <= min f + min_tol count as minimisers
                         (>= 0)                                                         */
} qhd_rqp_desc;

/* Per-instance readouts (FP64). */
typedef struct {
  double norm;        /* sum |phi|^2                                                   */
  double e_f;         /* sum f |phi|^2 / norm                                          */
  double p_min;       /* sum over the lattice minimisers of |phi|^2 / norm             */
  double f_min;       /* min of f over the lattice                                     */
  int64_t argmin_index; /* flat lattice index of the first minimiser (j_1 fastest)     */
  int64_t steps_done;
  double t;           /* steps_done * dt                                               */
} qhd_rqp_obs;

/* Validate the descriptor, allocate every device buffer for `batch` instances (state,
 * objective values, partial sums) and set each state to phi_0.  On failure nothing is
 * left allocated.  QHD_EINVAL for out-of-range fields or batch < 1; QHD_EUNSUPPORTED if
 * (r + 1)^d exceeds 2^24. */
qhd_status qhd_rqp_create(const qhd_rqp_desc *desc, int32_t batch, qhd_rqp *out);

/* Objective of instance i: Q (d x d, row-major, symmetrised as (Q + Q^T)/2) and b (d),
 * host FP64 arrays, copied.  f is evaluated on the lattice in FP64 on the device. */
qhd_status qhd_rqp_set_objective(qhd_rqp h, int32_t i, const double *Q, const double *b);

/* Advance every instance by min(max_steps, remaining) steps (max_steps < 0: to the
 * end).  Asynchronous on `stream`; allocates nothing.  QHD_ESTATE if an objective is
 * missing.  The leading axes whose (r+1)^K points fit 6561 run as one pass through
 * LDS (the 9^5 lattice: axes 1-4 fused, axis 5 alone), with the values of K separate
 * passes; the environment variable QHD_RQP_UNFUSED=1, read at creation, keeps one pass
 * per axis. */
qhd_status qhd_rqp_evolve(qhd_rqp h, int64_t max_steps, void *stream);

/* Readouts of every instance into host `out` (batch entries); optional device outputs:
 * marginals_dev (FP32, [batch][d][r+1], axis k = 1..d), prob_dev (FP32,
 * [batch][(r+1)^d], |phi|^2) and psi_dev (interleaved complex FP32, [batch][(r+1)^d],
 * j_1 fastest: the state phi at the current step, the trailing potential half step of
 * the last step applied to this copy; the handle's own state keeps it owed).
 * Synchronises `stream`.  QHD_ENUMERIC on a non-finite readout. */
qhd_status qhd_rqp_observe(qhd_rqp h, void *stream, qhd_rqp_obs *out, float *marginals_dev, float *prob_dev,
                           float *psi_dev);

/* Back to phi_0 at step 0 (objectives kept). */
qhd_status qhd_rqp_reset(qhd_rqp h, void *stream);

/* Lattice points per instance, (r + 1)^d. */
qhd_status qhd_rqp_points(qhd_rqp h, int64_t *points);

/* Release everything; NULL is accepted. */
qhd_status qhd_rqp_destroy(qhd_rqp h);

#ifdef __cplusplus
}
#endif

#endif /* QHD_RQP_H */
