/*
 * qhd_sno.h - C ABI of the spectral neural-operator surrogate of the QHD engine.
 *
 * The surrogate is not part of the paper's method.  It learns the map from a
 * potential f on an S x S mesh to the final position density |psi_T|^2 of the
 * QHD evolution (the measurement distribution of Algorithm 1, App. E.1), from
 * pairs produced by the solver of qhd.h, so that many landscapes can be screened
 * quickly while the solver stays the reference and the fallback.
 *
 * Model (all sizes from qhd_sno_desc; S = grid, C = width, M = modes, L = layers):
 *   features   x0 = ((f - mean f) / std f, x / S, y / S)             per mesh point
 *   lift       h0 = Wl x0 + bl                                       (1x1, 3 -> C)
 *   L layers   h  <- GELU(W h + b + Spec(h))                          (GELU with erf)
 *   Spec(h)    = (1/S^2) sum_{ky in [-M, M), kx in [0, M)} w(kx) Re( R(ky,kx) H(ky,kx) e^{+i theta} )
 *              with H(ky,kx) = sum_{y,x} h(y,x) e^{-i theta}, theta = 2 pi (ky y + kx x) / S,
 *              w(0) = 1, w(kx > 0) = 2, R(ky,kx) a complex C x C matrix per mode
 *   project    q = Wp h + bp ;  rho_hat = softmax over the S^2 mesh points
 *   loss       (1/B) sum_b sum_p |rho_hat - rho|                     (mean L1 of densities)
 * Parameters, in the order of the flat FP32 vector used by get/set_params:
 *   Wl[C][3], bl[C], then per layer Rr[2M][M][C][C], Ri[2M][M][C][C], W[C][C], b[C],
 *   then Wp[C], bp[1].  (W matrices are [out][in].)
 * All contractions run as batched GEMMs on the matrix cores (BF16 operands with
 * FP32 accumulation, or FP32 operands for gradient checks); Adam keeps FP32
 * master weights.
 *
 * Conventions as in qhd.h: status codes, qhd_last_error(), device pointers on
 * the device current at creation, "stream" = hipStream_t.  A handle is not
 * thread-safe.  f is FP64 [batch][S*S] row-major (x fastest); densities FP32.
 */
#ifndef QHD_SNO_H
#define QHD_SNO_H

#include <stdint.h>

#include "qhd.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qhd_sno_s *qhd_sno;

#define QHD_SNO_BF16 0 /* BF16 weights/activations, FP32 accumulation (training, inference) */
#define QHD_SNO_FP32 1 /* FP32 throughout (gradient checks) */

typedef struct {
  int32_t grid;      /* S: power of two, 32 <= S <= 256                              */
  int32_t width;     /* C: 8, 16, 32 or 64                                           */
  int32_t modes;     /* M: 1 <= M <= S/2                                             */
  int32_t layers;    /* L: 1 <= L <= 8                                               */
  int32_t max_batch; /* largest batch any call will pass, >= 1                       */
  int32_t precision; /* QHD_SNO_BF16 or QHD_SNO_FP32                                 */
  int32_t train;     /* nonzero: keep per-layer activations so backward can run      */
  uint64_t seed;     /* parameter initialisation (deterministic)                      */
} qhd_sno_desc;

/* Validate, allocate every buffer the surrogate will use, initialise parameters
 * (uniform +-1/sqrt(fan_in) for 1x1 maps, (1/C^2) U[0,1) for spectral weights). */
qhd_status qhd_sno_create(const qhd_sno_desc *desc, qhd_sno *out);

/* Number of FP32 parameters (length of the flat vector). */
qhd_status qhd_sno_param_count(qhd_sno sno, int64_t *count);

/* Copy the FP32 master parameters to / from a host vector of param_count floats
 * (set also resets the Adam state).  Synchronous. */
qhd_status qhd_sno_get_params(qhd_sno sno, float *host_params);
qhd_status qhd_sno_set_params(qhd_sno sno, const float *host_params);

/* Densities for `batch` potentials: f_dev FP64 [batch][S*S] -> rho_dev FP32
 * [batch][S*S] (each row sums to 1).  Asynchronous on stream.  On a handle created
 * with train == 0 in BF16 at width 32 the layers run as fused matrix-core passes
 * (with 16 modes: each layer's inverse x-contraction, 1x1 map, bias and GELU in one
 * pass that also forms the next layer's forward x-contraction, or the logits in the
 * last layer); the result equals the training form's to BF16 rounding. */
qhd_status qhd_sno_forward(qhd_sno sno, const double *f_dev, int32_t batch, float *rho_dev,
                           void *stream);

/* Forward, loss against rho_target_dev (FP32 [batch][S*S]) and backward; the
 * gradient is kept for qhd_sno_step.  Writes the loss to *loss (host) and, if
 * grad_host is not NULL, the flat FP32 gradient.  Synchronises the stream.
 * Needs a handle created with train != 0. */
qhd_status qhd_sno_backward(qhd_sno sno, const double *f_dev, const float *rho_target_dev,
                            int32_t batch, double *loss, float *grad_host, void *stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with the last gradient. */
qhd_status qhd_sno_step(qhd_sno sno, float lr, void *stream);

qhd_status qhd_sno_destroy(qhd_sno sno);

#ifdef __cplusplus
}
#endif

#endif /* QHD_SNO_H */
