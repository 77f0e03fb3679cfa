/*
 * FP64 CPU oracle for the Quantum Hamiltonian Descent split-operator evolution.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path links, loads or calls
 * this file: only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark use it.  It shares no code, header, table or helper with the HIP
 * library; the two meet only through the seeded input arrays.
 *
 * What it computes (paper: Leng, Hickman, Li, Wu, "Quantum Hamiltonian Descent",
 * arXiv 2303.01471):
 *   * the QHD Schroedinger equation  i dpsi/dt = [a(t)(-1/2 Lap) + b(t) f(x)] psi
 *     (main text, eq. main1; App. A, eq. qhd_operator), with the damping functions
 *     a = e^{phi_t}, b = e^{chi_t};
 *   * on the regular periodic mesh of App. E.1 ({a, a+dx, ..., b-dx} per axis,
 *     dx = (b-a)/N, N = 2^q), with the discrete normalisation sum |c|^2 = 1
 *     (eq. wave-rep);
 *   * advanced by the pseudo-spectral product formula of App. C.2.1
 *     (eqs. prod_qhd, prod_qhd_fft) and App. E.1 (eq.
 *     trotterized_qhd_evolution_operator, Algorithm 1): the potential factor is
 *     diagonal on the mesh, the kinetic factor is diagonal in the Fourier basis
 *     with eigenvalue |k|^2/2, k = 2 pi n / L;
 *   * the schedule of App. C.2.1 (eq. nonconvex_QHD_h): a(t) = 2/(eps + t^3),
 *     b(t) = 2 t^3;
 *   * readouts: the loss E[f] = <f> (App. B, eq. expect_O and the definition
 *     after it), position-measurement density |psi|^2 (Algorithm 1, last step),
 *     and the success mass within |x - x*| < r of the grid minimiser (main text,
 *     caption of fig. 2).
 *
 * Readings where the paper leaves a choice (each also listed in the design notes):
 *   * SCHEME_STRANG (default): symmetric splitting
 *       V(dt/2) . F^{-1} K(dt) F . V(dt/2)
 *     with a, b evaluated at the step midpoint t_{j+1/2} = (j + 1/2) dt, t computed
 *     from the integer j.  SCHEME_LIE is the paper's printed first-order formula:
 *     V(dt) first, then the kinetic factor, coefficients at the left end t_j = j dt.
 *     SCHEME_YOSHIDA4 composes the symmetric step as a fourth-order triple jump
 *     (Yoshida, Phys. Lett. A 150, 262 (1990)): three symmetric steps of lengths
 *     w1 dt, w0 dt, w1 dt with w1 = 1 / (2 - 2^{1/3}) and w0 = 1 - 2 w1, each with
 *     a, b at its own midpoint (time advances with the stages).
 *   * The shifted Fourier transform only re-orders frequencies; |k|^2 is what
 *     enters, so a plain DFT with n in {0..N/2-1, -N/2..-1} is used.
 *   * x* = argmin of f on the mesh, ties to the lowest flat index; the success
 *     test uses the unwrapped Euclidean distance (no periodic image).
 *   * E[f] is divided by sum |psi|^2; the norm is reported separately.
 *
 * Layout: psi is interleaved (re, im) doubles; f is doubles; the flat index is
 * i0 + n0 * (i1 + n1 * i2), i.e. axis 0 (x) fastest.
 *
 * "mutation" plants a deliberate mistake so that the tests can show the pins
 * catch it; 0 is the correct oracle.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_SCHED_NESTEROV 0 /* a = 2/(p0 + t^3), b = 2 t^3          */
#define ORACLE_SCHED_CONST 1    /* a = p0, b = p1                         */
#define ORACLE_SCHED_TABLE 2    /* a_j = table[2j], b_j = table[2j+1]      */

#define ORACLE_SCHEME_STRANG 0
#define ORACLE_SCHEME_LIE 1
#define ORACLE_SCHEME_YOSHIDA4 2

/* planted mistakes, test use only */
#define MUT_NONE 0
#define MUT_DROP_HALF_IN_LAMBDA 1   /* kinetic eigenvalue |k|^2 instead of |k|^2/2 */
#define MUT_KINETIC_SIGN 2          /* e^{+i dt a Lambda}                          */
#define MUT_FREQ_NO_WRAP 3          /* n = m instead of n in {-N/2..N/2-1}         */
#define MUT_SWAP_AXIS_LENGTH 4      /* axis 0 uses the length of axis 1            */
#define MUT_LEFT_END_COEFF 5        /* Strang with t_j instead of t_{j+1/2}        */
#define MUT_NO_IFFT_SCALE 6         /* inverse transform without the 1/N           */
#define MUT_POTENTIAL_SIGN 7        /* e^{+i (dt/2) b f}                            */
#define MUT_ONE_HALF_STEP 8         /* only the leading potential half step        */
#define MUT_EF_UNNORMALISED 9       /* readout: sum f rho without / norm           */
#define MUT_SUCCESS_WRAP 10         /* readout: periodic distance to x*            */
#define MUT_TWIDDLE_CONJ 11         /* FFT butterflies use the conjugate twiddle   */

typedef struct {
  int32_t ndim;     /* 1, 2 or 3 */
  int32_t n[3];     /* points per axis, powers of two */
  double lo[3];     /* box [lo, hi) per axis */
  double hi[3];
  double dt;        /* step (may be negative: time reversal) */
  int32_t sched;    /* ORACLE_SCHED_* */
  int32_t scheme;   /* ORACLE_SCHEME_* */
  double p[2];      /* schedule parameters */
  const double *table; /* ORACLE_SCHED_TABLE: (a_j, b_j) per global step j */
  int64_t table_len;   /* number of steps the table covers */
  double radius;    /* success radius */
  int32_t mutation; /* MUT_* (tests only) */
  int32_t threads;  /* OpenMP threads, <= 0 means the runtime default */
} oracle_desc;

typedef struct {
  double norm;        /* sum |psi|^2 */
  double e_f;         /* sum f |psi|^2 / norm */
  double success;     /* sum_{|x - x*| < r} |psi|^2 / norm */
  double f_min;       /* f(x*) */
  int64_t argmin;     /* flat index of x* */
} oracle_obs;

static int64_t npoints(const oracle_desc *d) {
  int64_t p = 1;
  for (int a = 0; a < d->ndim; ++a) p *= d->n[a];
  return p;
}

static int is_pow2(int32_t v) { return v > 0 && (v & (v - 1)) == 0; }

static int check_desc(const oracle_desc *d) {
  if (!d || d->ndim < 1 || d->ndim > 3) return -1;
  for (int a = 0; a < d->ndim; ++a) {
    if (!is_pow2(d->n[a]) || d->n[a] < 2) return -1;
    if (!(d->hi[a] > d->lo[a])) return -1;
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Discrete Fourier transform of one line: X_k = sum_m x_m e^{sign 2 pi i m k / N}
 * (unnormalised), computed by the textbook iterative radix-2 Cooley-Tukey
 * algorithm: bit-reversal permutation, then log2 N butterfly stages.  Each
 * twiddle is evaluated directly with cos/sin of its exact angle. */
static void fft_line(double *re, double *im, int n, int sign, int mutation) {
  /* bit reversal */
  for (int i = 1, j = 0; i < n; ++i) {
    int bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) {
      double t = re[i]; re[i] = re[j]; re[j] = t;
      t = im[i]; im[i] = im[j]; im[j] = t;
    }
  }
  const int wsign = (mutation == MUT_TWIDDLE_CONJ) ? -sign : sign;
  for (int len = 2; len <= n; len <<= 1) {
    const int half = len >> 1;
    for (int k = 0; k < half; ++k) {
      const double ang = 2.0 * M_PI * (double)k / (double)len;
      const double wr = cos(ang), wi = (double)wsign * sin(ang);
      for (int s = 0; s < n; s += len) {
        const int p = s + k, q = s + k + half;
        const double tr = re[q] * wr - im[q] * wi;
        const double ti = re[q] * wi + im[q] * wr;
        re[q] = re[p] - tr; im[q] = im[p] - ti;
        re[p] += tr;        im[p] += ti;
      }
    }
  }
}

/* Transform along every axis of the d-dimensional array (interleaved complex). */
static void fft_nd(const oracle_desc *d, double *psi, int sign) {
  int64_t total = npoints(d);
  for (int a = 0; a < d->ndim; ++a) {
    const int n = d->n[a];
    int64_t stride = 1;
    for (int b = 0; b < a; ++b) stride *= d->n[b];
    const int64_t nlines = total / n;
#pragma omp parallel
    {
      double *re = (double *)malloc(sizeof(double) * (size_t)n);
      double *im = (double *)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(static)
      for (int64_t l = 0; l < nlines; ++l) {
        /* line l: the index with the axis-a coordinate removed */
        const int64_t lo_part = l % stride, hi_part = l / stride;
        const int64_t base = lo_part + hi_part * stride * n;
        for (int m = 0; m < n; ++m) {
          re[m] = psi[2 * (base + m * stride)];
          im[m] = psi[2 * (base + m * stride) + 1];
        }
        fft_line(re, im, n, sign, d->mutation);
        for (int m = 0; m < n; ++m) {
          psi[2 * (base + m * stride)] = re[m];
          psi[2 * (base + m * stride) + 1] = im[m];
        }
      }
      free(re);
      free(im);
    }
  }
}

/* ------------------------------------------------------------------------ */
/* a(t), b(t) of eq. nonconvex_QHD_h (or the constants) at time t. */
static void coefficients_at(const oracle_desc *d, double t, double *a, double *b) {
  if (d->sched == ORACLE_SCHED_CONST) {
    *a = d->p[0];
    *b = d->p[1];
    return;
  }
  const double t3 = t * t * t;
  *a = 2.0 / (d->p[0] + t3);
  *b = 2.0 * t3;
}

/* Schedule: a(t), b(t) of the Hamiltonian for global step j. */
static void coefficients(const oracle_desc *d, int64_t j, double *a, double *b) {
  if (d->sched == ORACLE_SCHED_TABLE) {
    *a = d->table[2 * j];
    *b = d->table[2 * j + 1];
    return;
  }
  if (d->sched == ORACLE_SCHED_CONST) {
    *a = d->p[0];
    *b = d->p[1];
    return;
  }
  /* eq. nonconvex_QHD_h: a = 2/(eps + t^3), b = 2 t^3.  Strang evaluates at the
   * midpoint (j + 1/2) dt; the printed first-order formula at the left end j dt. */
  double t;
  if (d->scheme == ORACLE_SCHEME_LIE || d->mutation == MUT_LEFT_END_COEFF)
    t = (double)j * d->dt;
  else
    t = ((double)j + 0.5) * d->dt;
  const double t3 = t * t * t;
  *a = 2.0 / (d->p[0] + t3);
  *b = 2.0 * t3;
}

/* Integer frequency of FFT output index m on an axis of N points. */
static int freq_of(int m, int n, int mutation) {
  if (mutation == MUT_FREQ_NO_WRAP) return m;
  return (m < n / 2) ? m : m - n;
}

static double axis_length(const oracle_desc *d, int a) {
  if (d->mutation == MUT_SWAP_AXIS_LENGTH && a == 0 && d->ndim > 1)
    return d->hi[1] - d->lo[1];
  return d->hi[a] - d->lo[a];
}

/* psi <- exp(-i * coef * f) psi, elementwise. */
static void potential_phase(const oracle_desc *d, double *psi, const double *f, double coef) {
  const int64_t total = npoints(d);
  const double sgn = (d->mutation == MUT_POTENTIAL_SIGN) ? 1.0 : -1.0;
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < total; ++p) {
    const double th = sgn * coef * f[p];
    const double c = cos(th), s = sin(th);
    const double re = psi[2 * p], im = psi[2 * p + 1];
    psi[2 * p] = re * c - im * s;
    psi[2 * p + 1] = re * s + im * c;
  }
}

/* psi_hat <- exp(-i * coef * Lambda(k)) psi_hat with Lambda = |k|^2 / 2. */
static void kinetic_phase(const oracle_desc *d, double *psi, double coef) {
  const int64_t total = npoints(d);
  const double sgn = (d->mutation == MUT_KINETIC_SIGN) ? 1.0 : -1.0;
  const double half = (d->mutation == MUT_DROP_HALF_IN_LAMBDA) ? 1.0 : 0.5;
  double two_pi_over_l[3] = {0, 0, 0};
  for (int a = 0; a < d->ndim; ++a) two_pi_over_l[a] = 2.0 * M_PI / axis_length(d, a);
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < total; ++p) {
    int64_t rem = p;
    double k2 = 0.0;
    for (int a = 0; a < d->ndim; ++a) {
      const int m = (int)(rem % d->n[a]);
      rem /= d->n[a];
      const double k = two_pi_over_l[a] * (double)freq_of(m, d->n[a], d->mutation);
      k2 += k * k;
    }
    const double th = sgn * coef * half * k2;
    const double c = cos(th), s = sin(th);
    const double re = psi[2 * p], im = psi[2 * p + 1];
    psi[2 * p] = re * c - im * s;
    psi[2 * p + 1] = re * s + im * c;
  }
}

static void inverse_scale(const oracle_desc *d, double *psi) {
  if (d->mutation == MUT_NO_IFFT_SCALE) return;
  const int64_t total = npoints(d);
  const double s = 1.0 / (double)total;
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < 2 * total; ++p) psi[p] *= s;
}

/* ------------------------------------------------------------------------ */
/* Public entry points (called through ctypes by the tests). */

int oracle_fft(const oracle_desc *d, double *psi, int sign) {
  if (check_desc(d) || !psi || (sign != 1 && sign != -1)) return -1;
#ifdef _OPENMP
  if (d->threads > 0) omp_set_num_threads(d->threads);
#endif
  fft_nd(d, psi, sign);
  return 0;
}

/* Advance psi (interleaved complex, in place) through global steps
 * j = j0 .. j0 + nsteps - 1. */
int oracle_evolve(const oracle_desc *d, const double *f, double *psi, int64_t j0, int64_t nsteps) {
  if (check_desc(d) || !f || !psi || nsteps < 0 || j0 < 0) return -1;
  if (d->sched == ORACLE_SCHED_TABLE && (!d->table || j0 + nsteps > d->table_len)) return -1;
  if (d->scheme == ORACLE_SCHEME_YOSHIDA4 && d->sched == ORACLE_SCHED_TABLE) return -1;
#ifdef _OPENMP
  if (d->threads > 0) omp_set_num_threads(d->threads);
#endif
  const double dt = d->dt;
  for (int64_t j = j0; j < j0 + nsteps; ++j) {
    double a, b;
    if (d->scheme == ORACLE_SCHEME_YOSHIDA4) {
      /* three symmetric steps; stage k starts at j dt + c_k dt, lasts w_k dt */
      const double w1 = 1.0 / (2.0 - cbrt(2.0)), w0 = 1.0 - 2.0 * w1;
      const double w[3] = {w1, w0, w1};
      double start = (double)j * dt;
      for (int k = 0; k < 3; ++k) {
        const double h = w[k] * dt;
        coefficients_at(d, start + 0.5 * h, &a, &b);
        potential_phase(d, psi, f, 0.5 * h * b);
        fft_nd(d, psi, -1);
        kinetic_phase(d, psi, h * a);
        fft_nd(d, psi, +1);
        inverse_scale(d, psi);
        potential_phase(d, psi, f, 0.5 * h * b);
        start += h;
      }
      continue;
    }
    coefficients(d, j, &a, &b);
    if (d->scheme == ORACLE_SCHEME_LIE) {
      /* eq. prod_qhd_fft: psi_{j+1} = F^{-1} e^{-i s a_j L} F e^{-i s b_j f} psi_j
       * (F denotes our forward DFT; the paper's F_s / F_s^{-1} pair acts the same
       * way on the kinetic factor). */
      potential_phase(d, psi, f, dt * b);
      fft_nd(d, psi, -1);
      kinetic_phase(d, psi, dt * a);
      fft_nd(d, psi, +1);
      inverse_scale(d, psi);
    } else {
      /* symmetric splitting: half potential, kinetic, half potential */
      potential_phase(d, psi, f, 0.5 * dt * b);
      fft_nd(d, psi, -1);
      kinetic_phase(d, psi, dt * a);
      fft_nd(d, psi, +1);
      inverse_scale(d, psi);
      if (d->mutation != MUT_ONE_HALF_STEP) potential_phase(d, psi, f, 0.5 * dt * b);
    }
  }
  return 0;
}

/* Neumaier-compensated running sum. */
typedef struct { double s, c; } ksum;
static void kadd(ksum *k, double v) {
  const double t = k->s + v;
  if (fabs(k->s) >= fabs(v)) k->c += (k->s - t) + v;
  else k->c += (v - t) + k->s;
  k->s = t;
}
static double kval(const ksum *k) { return k->s + k->c; }

int oracle_readout(const oracle_desc *d, const double *f, const double *psi, oracle_obs *out,
                   double *rho_out) {
  if (check_desc(d) || !f || !psi || !out) return -1;
  const int64_t total = npoints(d);
  /* grid minimiser: lowest flat index among equal minima */
  int64_t amin = 0;
  for (int64_t p = 1; p < total; ++p)
    if (f[p] < f[amin]) amin = p;
  int64_t ci[3] = {0, 0, 0};
  {
    int64_t rem = amin;
    for (int a = 0; a < d->ndim; ++a) { ci[a] = rem % d->n[a]; rem /= d->n[a]; }
  }
  double h[3] = {0, 0, 0};
  for (int a = 0; a < d->ndim; ++a) h[a] = (d->hi[a] - d->lo[a]) / (double)d->n[a];
  const double r2 = d->radius * d->radius;

  ksum norm = {0, 0}, ef = {0, 0}, succ = {0, 0};
  for (int64_t p = 0; p < total; ++p) {
    const double re = psi[2 * p], im = psi[2 * p + 1];
    const double rho = re * re + im * im;
    if (rho_out) rho_out[p] = rho;
    kadd(&norm, rho);
    kadd(&ef, f[p] * rho);
    int64_t rem = p;
    double dist2 = 0.0;
    for (int a = 0; a < d->ndim; ++a) {
      int64_t di = rem % d->n[a] - ci[a];
      rem /= d->n[a];
      if (d->mutation == MUT_SUCCESS_WRAP) {
        if (di > d->n[a] / 2) di -= d->n[a];
        if (di < -d->n[a] / 2) di += d->n[a];
      }
      const double dx = (double)di * h[a];
      dist2 += dx * dx;
    }
    if (dist2 < r2) kadd(&succ, rho);
  }
  out->norm = kval(&norm);
  out->e_f = (d->mutation == MUT_EF_UNNORMALISED) ? kval(&ef) : kval(&ef) / out->norm;
  out->success = kval(&succ) / out->norm;
  out->f_min = f[amin];
  out->argmin = amin;
  return 0;
}

/* Uniform initial state of eq. nonconvex_QHD_h's experiment: every mesh point has
 * amplitude N^{-1/2} (N = total points), so sum |psi|^2 = 1 (eq. wave-rep). */
int oracle_uniform_state(const oracle_desc *d, double *psi) {
  if (check_desc(d) || !psi) return -1;
  const int64_t total = npoints(d);
  const double v = 1.0 / sqrt((double)total);
  for (int64_t p = 0; p < total; ++p) {
    psi[2 * p] = v;
    psi[2 * p + 1] = 0.0;
  }
  return 0;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
