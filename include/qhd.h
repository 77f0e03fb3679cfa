/*
 * qhd.h - C ABI of the MI355X (gfx950) engine for the classical simulation of
 * Quantum Hamiltonian Descent (Leng, Hickman, Li, Wu, arXiv 2303.01471).
 *
 * The library evolves batches of discretised wave functions under
 *
 *     i dpsi/dt = [ a(t) (-1/2 Lap) + b(t) f(x) ] psi
 *
 * (the QHD Hamiltonian: main text eq. main1, App. A eq. qhd_operator, with
 * a = e^{phi_t}, b = e^{chi_t}) on the periodic mesh of App. E.1, by the
 * pseudo-spectral product formula of App. C.2.1 (eqs. prod_qhd, prod_qhd_fft)
 * taken in its symmetric (Strang) form with the coefficients at the step
 * midpoint.  The statement of the problem follows Algorithm 1 of App. E.1:
 * a box, 2^q points per axis, an initial state, the schedule, a step and an
 * iteration count, then a position measurement.
 *
 * Conventions shared by every entry point:
 *   - All functions return a qhd_status; none aborts or exits.  On failure,
 *     qhd_last_error() returns a message for the calling thread.
 *   - A plan is not thread-safe; distinct plans are independent.
 *   - Device pointers are HIP device addresses on the device that was current
 *     when the plan was created.  "stream" arguments are hipStream_t values
 *     (NULL = the default stream).
 *   - Grid arrays are row-major with axis 0 (x) fastest: flat index
 *     i0 + n0 * (i1 + n1 * i2).  Complex values are interleaved (re, im) FP32.
 */
#ifndef QHD_H
#define QHD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QHD_OK = 0,
  QHD_EINVAL = 1,       /* invalid argument (descriptor, index, pointer, size)      */
  QHD_EUNSUPPORTED = 2, /* valid but not supported by this build                    */
  QHD_ENOMEM = 3,       /* device or host allocation failed                         */
  QHD_EDEVICE = 4,      /* a HIP runtime call failed                                */
  QHD_ESTATE = 5,       /* call out of order (e.g. evolve before set_potential)     */
  QHD_ENUMERIC = 6      /* NaN/Inf in an observable, or |norm - 1| above tolerance */
} qhd_status;

/* Schedule of the damping coefficients a(t) = e^{phi_t}, b(t) = e^{chi_t}. */
typedef enum {
  /* App. C.2.1, eq. nonconvex_QHD_h: a = 2/(eps + t^3), b = 2 t^3, eps = sched_p[0] */
  QHD_SCHED_NESTEROV = 0,
  /* a = sched_p[0], b = sched_p[1] */
  QHD_SCHED_CONST = 1,
  /* per-step values: a_j = sched_table[2j], b_j = sched_table[2j+1], j = 0..nsteps-1,
   * each applied over step j as given, whatever the scheme */
  QHD_SCHED_TABLE = 2,
  /* adiabatic interpolation g(t) = t / T, T = sched_p[0]: a = 1 - g, b = g (the
   * baseline QAA's linear schedule, App. C.2 "Quantum Adiabatic Algorithm") */
  QHD_SCHED_LINEAR = 3
} qhd_sched_kind;

/* Which Hamiltonian the instance evolves under: H = a(t) H_0 + b(t) diag(f). */
typedef enum {
  /* QHD: H_0 = -1/2 Laplacian on the periodic mesh (main text, App. C.2.1) */
  QHD_MODEL_QHD = 0,
  /* the baseline quantum adiabatic algorithm the paper compares with (App. C.2): each
   * axis index written in radix 2 (log2 n qubits), H_0 = -sum_j sigma_x^(j) over all
   * qubits, diagonal in the Walsh-Hadamard basis.  2-D only; use QHD_SCHED_LINEAR with
   * T = nsteps * dt for the paper's setting.  The box only labels the mesh points. */
  QHD_MODEL_QAA = 1
} qhd_model;

typedef enum {
  QHD_INIT_UNIFORM = 0, /* psi0 = N^{-1/2} at every mesh point (App. C.2.1 experiment) */
  QHD_INIT_USER = 1     /* qhd_set_state must be called before the first evolve       */
} qhd_init_kind;

/* Product formula of one step. */
typedef enum {
  /* symmetric: e^{-i dt/2 b V} F^{-1} e^{-i dt a L} F e^{-i dt/2 b V}, a and b at the step
   * midpoint t_{j+1/2} = (j + 1/2) dt (second order) */
  QHD_SCHEME_STRANG = 0,
  /* the printed first-order product of App. C.2.1 eq. prod_qhd_fft / Algorithm 1:
   * F^{-1} e^{-i dt a L} F e^{-i dt b V}, a and b at the left end t_j = j dt */
  QHD_SCHEME_LIE = 1,
  /* fourth order: the symmetric step composed as a triple jump (Yoshida 1990), three
   * symmetric stages of lengths w1 dt, w0 dt, w1 dt with w1 = 1/(2 - 2^{1/3}),
   * w0 = 1 - 2 w1, each with a and b at its own midpoint; three times the passes of
   * QHD_SCHEME_STRANG per step.  Not with QHD_SCHED_TABLE (QHD_EUNSUPPORTED). */
  QHD_SCHEME_YOSHIDA4 = 2,
  /* QHD_MODEL_QAA only: the leapfrog integrator the paper uses for its baseline QAA
   * (App. C.2): with psi = R + i I, kick I -= dt/2 H(t_j) R, drift R += dt H(t_{j+1/2}) I,
   * kick I -= dt/2 H(t_{j+1}) R (second order, time-reversible, stable for dt |H| < 2;
   * the norm is not exactly conserved).  Not with QHD_SCHED_TABLE. */
  QHD_SCHEME_LEAPFROG = 3
} qhd_scheme;

/* One problem instance (Algorithm 1 of App. E.1). */
typedef struct {
  int32_t ndim;         /* 1, 2 or 3                                                   */
  int32_t n[3];         /* points per axis, powers of two, 8 <= n <= 1024 (3-D: 16 <= n
                           <= 128, else QHD_EUNSUPPORTED); unused axes are ignored     */
  double lo[3], hi[3];  /* periodic box [lo, hi) per axis, hi > lo (App. E.1 mesh)     */
  double dt;            /* time step s > 0                                             */
  int64_t nsteps;       /* number of steps, >= 0; the end time is T = nsteps * dt      */
  int32_t sched_kind;   /* qhd_sched_kind                                              */
  double sched_p[2];    /* schedule parameters (see qhd_sched_kind)                    */
  const double *sched_table; /* QHD_SCHED_TABLE: host array of 2*nsteps doubles, copied
                                at plan creation; ignored otherwise                      */
  int32_t init_kind;    /* qhd_init_kind                                               */
  double success_radius;/* r > 0 of the success test |x - x*| < r (main text, fig. 2)  */
  int32_t scheme;       /* qhd_scheme (0, the zero-initialised default: symmetric)     */
  int32_t model;        /* qhd_model (0, the zero-initialised default: QHD)            */
} qhd_instance;

/* Plan options.  Zero-initialise and set what you need. */
typedef struct {
  uint32_t flags;          /* QHD_OPT_* bits                                          */
  double norm_tolerance;   /* qhd_observe returns QHD_ENUMERIC if |norm-1| exceeds
                              this; <= 0 selects 1e-3                                  */
  int32_t timing_stride;   /* with QHD_OPT_TIME_PASSES: time every pass of one evolve
                              chunk in this many (<= 0 selects 16)                     */
  const char *tune_cache;  /* path of a text tuning cache, or NULL.  Entries found for
                              a shape class are used; with QHD_OPT_AUTOTUNE, classes
                              without an entry are tuned and appended.  A missing or
                              unreadable file is treated as empty                      */
} qhd_plan_opts;

#define QHD_OPT_TIME_PASSES 0x1u /* record HIP events around sampled pass launches   */
#define QHD_OPT_AUTOTUNE 0x2u    /* at plan creation, time the row- and column-pass
                                    variants (points per lane, staged / tile-wave) and
                                    the grid sizes of every 2-D shape class on its own
                                    batch and keep the fastest (a few ms per class)     */
#define QHD_OPT_NO_GRAPH 0x4u    /* never replay captured step chunks (see qhd_evolve)  */
#define QHD_OPT_MFMA_DFT 0x8u    /* 3-D instances with n = 128 on every axis: the line
                                    transforms run as dense 128 x 128 DFT products on
                                    the matrix cores (FP16 operands, FP32 accumulation):
                                    the data in two scaled FP16 terms, the DFT matrix in
                                    three (to ~2^-36, so that no error of its own repeats
                                    on every transform), relative error ~2^-23 per
                                    transform; four streaming passes per step (72 bytes
                                    per grid point) in the slab layout; other instances
                                    are unaffected                                      */
#define QHD_OPT_RESIDENT 0x10u   /* 2-D instances with n_x, n_y in {32, 64, 128} (QHD
                                    with any scheme, or QAA integrated by the split step):
                                    all the steps of an evolve call run in
                                    one launch, one workgroup per instance holding psi
                                    in LDS (n_y (9 n_x / 8 + 1) 8 bytes, ~148 KB and one
                                    instance per CU at 128^2), so psi crosses HBM only
                                    at the start and the end of the call (the scope's
                                    resident mode of the two-pass step, App. C.2.1).
                                    Same arithmetic as the streaming passes with 8
                                    points per lane.  With QHD_OPT_AUTOTUNE as well,
                                    each such class keeps resident steps only if 16 of
                                    them beat 16 streaming steps on its own batch (one
                                    CU per 128^2 instance loses against the whole GPU
                                    for a lone instance); the choice is kept in the
                                    tuning cache.  Leapfrog QAA and other shapes
                                    unaffected                                          */

typedef struct qhd_plan_s *qhd_plan;

/* Per-instance readouts (App. B: E[f] = <f>; Algorithm 1: position measurement;
 * main text fig. 2: success criterion |x - x*| < r). */
typedef struct {
  double norm;          /* sum |psi|^2 (FP64 accumulation)                              */
  double e_f;           /* sum f |psi|^2 / norm                                          */
  double success_mass;  /* sum over |x - x*| < r of |psi|^2 / norm (unwrapped distance)  */
  double f_min;         /* f(x*)                                                         */
  int64_t argmin_index; /* flat index of x*, the lowest-index minimiser of f on the mesh */
  int64_t steps_done;   /* steps completed                                               */
  double t;             /* steps_done * dt                                               */
} qhd_observables;

/* Per-kernel timing gathered with QHD_OPT_TIME_PASSES. */
typedef struct {
  char name[48];        /* kernel family, e.g. "row_pass_2d/n512"                        */
  int64_t launches;     /* launches that were timed                                      */
  double total_ms;      /* summed HIP-event durations of the timed launches              */
  double points;        /* grid points processed by the timed launches                   */
  double bytes_per_point; /* algorithmic HBM bytes moved per grid point by this kernel   */
} qhd_kernel_timing;

/* Launch configuration of one shape class of a plan (instances with equal ndim
 * and n), as chosen at plan creation. */
typedef struct {
  int32_t ndim, n[3];
  int32_t members;       /* instances in the class                                      */
  int32_t col_variant;   /* 2-D column pass: 1 staged through LDS (8 points per lane),
                            2 tile-wave, 3 staged with 16 points per lane               */
  int32_t grid_cap_row;  /* workgroup caps of the row (x) and column passes             */
  int32_t grid_cap_col;
  int32_t tuned;         /* 1 if the autotuner chose them while creating this plan      */
  int32_t mfma_dft;      /* 1 if the class runs the matrix-core DFT passes              */
  int32_t row_points_per_lane; /* 2-D row pass: 8 or 16 points of a line per lane       */
  int32_t resident;      /* 1 if the class runs resident steps (QHD_OPT_RESIDENT)       */
} qhd_class_info;

/* Create a plan for `batch` instances.  Validates every descriptor first (no
 * device work happens for an invalid batch), then allocates all device memory
 * the plan will ever use; later calls allocate nothing.  The uniform initial
 * state is written here.  *out receives the plan, or NULL on failure. */
qhd_status qhd_plan_create(const qhd_instance *inst, int32_t batch, const qhd_plan_opts *opts,
                           qhd_plan *out);

/* Upload f (FP64, n0*n1*n2 values, row-major) for instance i.  on_device != 0
 * means `f` is a device pointer.  The call also finds x* and f(x*).  It is
 * ordered on the plan's internal stream and synchronises before returning;
 * the caller keeps ownership of `f`.  Must precede the first evolve. */
qhd_status qhd_set_potential(qhd_plan plan, int32_t i, const double *f, int32_t on_device);

/* Replace the state of instance i by psi (interleaved complex FP32, row-major),
 * e.g. a user initial state or a checkpoint.  The state is taken as exact
 * (no pending half step).  Synchronous, like qhd_set_potential. */
qhd_status qhd_set_state(qhd_plan plan, int32_t i, const float *psi_c64, int32_t on_device);

/* Set the global step index of instance i (0 <= j <= nsteps) so that a resumed
 * run continues the schedule at t_{j+1/2}.  Use after qhd_set_state. */
qhd_status qhd_set_steps_done(qhd_plan plan, int32_t i, int64_t j);

/* Advance every instance by min(max_steps, remaining) steps (max_steps < 0:
 * to the end).  Asynchronous on `stream`; allocates nothing.  Between evolve
 * calls the state may carry a pending half step; the result does not depend on
 * how the steps are split into calls.
 * The steps run in chunks of at most K steps (K = 64 / the most stages per step of
 * any instance; qhd_plan_info reports it).  Inside a chunk every shape class runs
 * on a stream of its own, forked from `stream` and joined back before the chunk's
 * step commit, so classes overlap on the GPU; the members a pass visits are
 * counted on the device at the start of the chunk.  A full chunk of every class is
 * captured as a HIP graph at plan creation and replayed for every chunk in which
 * each class still has a member with K steps to go, uneven batches included; the
 * rest runs as direct launches.  The arithmetic is the same, so the results are
 * bitwise identical to direct launches.  Not with QHD_OPT_NO_GRAPH, and not while
 * `stream` is itself being captured (the passes are then launched directly into
 * the caller's capture).  With QHD_OPT_TIME_PASSES one chunk in timing_stride is
 * launched directly with its classes serialised and every pass timed. */
qhd_status qhd_evolve(qhd_plan plan, int64_t max_steps, void *stream);

/* Lowest eigenpairs of the discrete Hamiltonian of 2-D instance i at time t,
 *     H(t) = a(t) F^{-1} diag(|k|^2/2) F + b(t) diag(f)
 * (the operator the split-operator step exponentiates, App. C.2.1 eq.
 * prod_qhd_fft; its low-lying spectrum along the path is the subject of App. D),
 * by the Lanczos iteration with full reorthogonalisation over `krylov` steps
 * (nev < krylov <= min(400, points)), from a fixed pseudo-random start vector.
 * a(t), b(t) follow the instance's schedule (TABLE: the entry of step floor(t/dt)).
 * Writes the nev lowest Ritz values to energies[] (ascending); if residuals is not
 * NULL, ||H phi - E phi|| of each unit Ritz vector; if overlaps is not NULL,
 * |<phi_n|psi>|^2 / <psi|psi> for psi_dev, a device complex64 state of the instance
 * in row-major order (x fastest; e.g. the instance's slice of qhd_observe's psi
 * output).  Degenerate eigenvalues are found once (single-vector Krylov space).
 * Matrix-vector products in FP32 on the GPU, scalars in FP64.  Allocates and frees
 * (krylov + 4) vectors of the instance's size; synchronous on `stream`.  Not for
 * stream capture.  QHD_EUNSUPPORTED for 1-D/3-D instances. */
qhd_status qhd_spectrum(qhd_plan plan, int32_t i, double t, int32_t nev, int32_t krylov,
                        const float *psi_dev, double *energies, double *overlaps, double *residuals,
                        void *stream);

/* Launch configuration: up to `cap` classes into out[], their number into
 * *n_classes, and the steps per captured graph chunk into *graph_steps (0: no
 * graph).  Host-only. */
qhd_status qhd_plan_info(qhd_plan plan, qhd_class_info *out, int32_t cap, int32_t *n_classes,
                         int32_t *graph_steps);

/* Return every instance to step 0: UNIFORM instances get psi0 = N^{-1/2} again,
 * USER instances need a new qhd_set_state before the next evolve.  Potentials
 * are kept.  Asynchronous on `stream`; allocates nothing. */
qhd_status qhd_reset(qhd_plan plan, void *stream);

/* Readouts for every instance.  Closes any pending half step on a copy (the
 * plan state is untouched, evolution can continue).  host_out: `batch` entries.
 * rho_dev / psi_dev: optional caller-owned device buffers receiving |psi|^2
 * (FP32) and psi (interleaved FP32), instances concatenated in order; NULL to
 * skip.  Synchronises `stream` before returning.  Returns QHD_ENUMERIC (with
 * host_out filled) if an observable is not finite or |norm - 1| exceeds the
 * plan's tolerance. */
qhd_status qhd_observe(qhd_plan plan, void *stream, qhd_observables *host_out, float *rho_dev,
                       float *psi_dev);

/* One instance's readouts as qhd_readouts_static writes them (device memory). */
typedef struct {
  double norm;          /* sum |psi|^2                                                   */
  double e_f;           /* sum f |psi|^2 / norm                                          */
  double success_mass;  /* sum over |x - x*| < r of |psi|^2 / norm (unwrapped distance)  */
  double f_min;         /* f(x*)                                                         */
  int64_t argmin_index; /* flat index of x*, lowest-index minimiser of the finite f values;
                           -1 (and success_mass 0) if f has no finite value              */
} qhd_readout;

/* Mesh lines (count * n[1] * n[2]) one qhd_readouts_static call may cover. */
#define QHD_STATIC_MAX_LINES 65536

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the readouts of qhd_observe for
 * states the caller holds, without a plan and without any allocation.
 *   psi_dev  count states, interleaved complex FP32, row-major (x fastest), instance
 *            after instance, each taken as it is (no pending half step is closed);
 *   f_dev    count potentials, FP64, same layout;
 *   n, lo, hi  host arrays of ndim entries (axis 0 = x): the mesh and periodic box of
 *            every instance (App. E.1), powers of two 8 <= n <= 1024;
 *   success_radius  r of |x - x*| < r;
 *   out_dev  count qhd_readout entries in device memory, written on `stream`.
 * Asynchronous on `stream` (four kernel launches, no host synchronisation, capturable).
 * The per-line partial results live in a static device array of the library (about
 * 3.5 MB on every GPU it runs on, held until the process ends), which bounds a call to
 * count * n[1] * n[2] <= QHD_STATIC_MAX_LINES mesh lines (QHD_EINVAL beyond).  Calls
 * whose work overlaps on one GPU share that array and race: order them on one stream.
 * Non-finite f values are skipped by the x* search and make the sums non-finite. */
qhd_status qhd_readouts_static(int32_t ndim, const int32_t *n, const double *lo, const double *hi,
                               double success_radius, int32_t count, const float *psi_dev,
                               const double *f_dev, qhd_readout *out_dev, void *stream);

/* Total mesh points of the plan (sum over instances), for sizing rho/psi buffers. */
qhd_status qhd_plan_points(qhd_plan plan, int64_t *total_points);

/* With QHD_OPT_TIME_PASSES: copy up to `cap` entries of per-kernel timing into
 * `out`, set *count, and reset the counters.  Synchronises the plan's streams. */
qhd_status qhd_kernel_timings(qhd_plan plan, qhd_kernel_timing *out, int32_t cap, int32_t *count);

/* Release every resource of the plan.  NULL is accepted. */
qhd_status qhd_plan_destroy(qhd_plan plan);

/* Message describing the last failure on the calling thread ("" if none). */
const char *qhd_last_error(void);

/* Library version string. */
const char *qhd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* QHD_H */
