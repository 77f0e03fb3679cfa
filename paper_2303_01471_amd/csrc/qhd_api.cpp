// C ABI of the QHD engine: argument validation, plan (instances grouped into
// shape classes, device arenas, twiddle tables), the evolve driver and the
// readouts.  The statement of the problem follows Algorithm 1 of App. E.1 of
// the paper; the kernels are in qhd_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <tuple>
#include <string>
#include <vector>

#include "../../include/qhd.h"
#include "qhd_internal.h"

using namespace qhd;

namespace {

thread_local std::string g_err;

qhd_status fail(qhd_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(e_ == hipErrorOutOfMemory ? QHD_ENOMEM : QHD_EDEVICE, "%s: %s (%s:%d)", \
                  #expr, hipGetErrorString(e_), __FILE__, __LINE__);                    \
  } while (0)

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// Host-only validation of one descriptor (no device work).
// stages of one step: the fourth-order composition runs three symmetric stages, the
// leapfrog step kick, drift and kick
int stages_per_step(const qhd_instance& d) {
  return (d.scheme == QHD_SCHEME_YOSHIDA4 || d.scheme == QHD_SCHEME_LEAPFROG) ? 3 : 1;
}

qhd_status validate(const qhd_instance& d, int idx) {
  if (d.ndim < 1 || d.ndim > 3) return fail(QHD_EINVAL, "instance %d: ndim must be 1, 2 or 3 (got %d)", idx, d.ndim);
  for (int a = 0; a < d.ndim; ++a) {
    if (!is_pow2(d.n[a]) || d.n[a] < 8 || d.n[a] > 1024)
      return fail(QHD_EINVAL, "instance %d: n[%d]=%d must be a power of two in [8, 1024]", idx, a, d.n[a]);
    if (d.ndim == 3 && (d.n[a] < 16 || d.n[a] > 128))
      return fail(QHD_EUNSUPPORTED, "instance %d: 3-D axes need 16 <= n <= 128 (n[%d]=%d)", idx, a, d.n[a]);
    if (!std::isfinite(d.lo[a]) || !std::isfinite(d.hi[a]) || !(d.hi[a] > d.lo[a]))
      return fail(QHD_EINVAL, "instance %d: box axis %d needs finite lo < hi", idx, a);
  }
  if (!std::isfinite(d.dt) || !(d.dt > 0.0)) return fail(QHD_EINVAL, "instance %d: dt must be finite and > 0", idx);
  if (d.nsteps < 0) return fail(QHD_EINVAL, "instance %d: nsteps must be >= 0", idx);
  if (d.nsteps > (int64_t)600000000) return fail(QHD_EINVAL, "instance %d: nsteps must be <= 6e8", idx);
  if (!(d.success_radius > 0.0) || !std::isfinite(d.success_radius))
    return fail(QHD_EINVAL, "instance %d: success_radius must be finite and > 0", idx);
  switch (d.sched_kind) {
    case QHD_SCHED_NESTEROV:
      if (!std::isfinite(d.sched_p[0]) || !(d.sched_p[0] > 0.0))
        return fail(QHD_EINVAL, "instance %d: NESTEROV schedule needs eps = sched_p[0] > 0", idx);
      break;
    case QHD_SCHED_CONST:
      if (!std::isfinite(d.sched_p[0]) || !std::isfinite(d.sched_p[1]))
        return fail(QHD_EINVAL, "instance %d: CONST schedule needs finite a0, b0", idx);
      break;
    case QHD_SCHED_LINEAR:
      if (!std::isfinite(d.sched_p[0]) || !(d.sched_p[0] > 0.0))
        return fail(QHD_EINVAL, "instance %d: LINEAR schedule needs T = sched_p[0] > 0", idx);
      break;
    case QHD_SCHED_TABLE:
      if (d.nsteps > 0 && !d.sched_table) return fail(QHD_EINVAL, "instance %d: TABLE schedule needs sched_table", idx);
      for (int64_t j = 0; j < 2 * d.nsteps; ++j)
        if (!std::isfinite(d.sched_table[j])) return fail(QHD_EINVAL, "instance %d: sched_table[%lld] is not finite", idx, (long long)j);
      break;
    default:
      return fail(QHD_EINVAL, "instance %d: unknown sched_kind %d", idx, d.sched_kind);
  }
  if (d.scheme != QHD_SCHEME_STRANG && d.scheme != QHD_SCHEME_LIE && d.scheme != QHD_SCHEME_YOSHIDA4 &&
      d.scheme != QHD_SCHEME_LEAPFROG)
    return fail(QHD_EINVAL, "instance %d: unknown scheme %d", idx, d.scheme);
  if (d.scheme == QHD_SCHEME_YOSHIDA4 && d.sched_kind == QHD_SCHED_TABLE)
    return fail(QHD_EUNSUPPORTED, "instance %d: the fourth-order scheme evaluates the schedule between table "
                                  "points; use NESTEROV, CONST or LINEAR", idx);
  if (d.model != QHD_MODEL_QHD && d.model != QHD_MODEL_QAA)
    return fail(QHD_EINVAL, "instance %d: unknown model %d", idx, d.model);
  if (d.model == QHD_MODEL_QAA && d.ndim != 2)
    return fail(QHD_EUNSUPPORTED, "instance %d: the QAA model is built for 2-D meshes", idx);
  if (d.scheme == QHD_SCHEME_LEAPFROG && d.model != QHD_MODEL_QAA)
    return fail(QHD_EUNSUPPORTED, "instance %d: the leapfrog integrator is built for the QAA model", idx);
  if (d.model == QHD_MODEL_QAA && d.scheme != QHD_SCHEME_STRANG && d.scheme != QHD_SCHEME_LEAPFROG)
    return fail(QHD_EUNSUPPORTED, "instance %d: the QAA model runs the symmetric scheme or leapfrog", idx);
  if (d.scheme == QHD_SCHEME_LEAPFROG && d.sched_kind == QHD_SCHED_TABLE)
    return fail(QHD_EUNSUPPORTED, "instance %d: leapfrog evaluates the schedule between table points", idx);
  if (d.init_kind != QHD_INIT_UNIFORM && d.init_kind != QHD_INIT_USER)
    return fail(QHD_EINVAL, "instance %d: unknown init_kind %d", idx, d.init_kind);
  return QHD_OK;
}

struct Pending {
  hipEvent_t start, stop;
  int family;
  double points;
};

struct Family {
  std::string name;
  int64_t launches = 0;
  double total_ms = 0.0, points = 0.0, bytes_per_point = 0.0;
};

}  // namespace

struct ShapeClass {
  int ndim = 0, nx = 1, ny = 1, nz = 1;
  long long points = 0;            // per instance
  std::vector<int> members;        // plan indices, sorted by nsteps (descending)
  std::vector<InstDev> host;       // mirror of the device array
  InstDev* dev = nullptr;
  float2* psi = nullptr;
  double* f = nullptr;
  double* partials = nullptr;      // 3 per line
  double* results = nullptr;       // 3 per member
  int lines = 0;                   // lines per instance for the readout partials
  const double2* tw_x = nullptr;
  const double2* tw_y = nullptr;
  const double2* tw_z = nullptr;
  int fam_row = -1, fam_col = -1, fam_line = -1, fam_y = -1, fam_z = -1;
  // launch configuration (defaults, a tuning-cache entry, or the autotuner's choice)
  int col_variant = kColAuto;
  int row_points = 8;  // points per lane of the row pass
  int cap_row = 2048, cap_col = 2048;
  bool tuned = false;
  bool mfma = false;  // 3-D 128^3 with QHD_OPT_MFMA_DFT
  bool plane = false; // 3-D in the plane layout (x slowest, (y, z) planes in 8x8 tiles)
  int model = kModelQHD;
  bool leapfrog = false;           // QAA members integrated by leapfrog stages
  bool y4 = false;                 // some member runs the fourth-order scheme
  float* scratch = nullptr;        // leapfrog: partial H v between the row and column passes
  bool resident = false;           // QHD_OPT_RESIDENT: all steps of a chunk in one launch, psi in LDS
  int fam_res = -1;
  int sps = 1;                     // stages per step of the class (the most of its members)
  // device counts: [0, kMaxSub) members visited per sub-step of the current chunk (written
  // by the chunk-plan kernel), [kMaxSub] every member (launches outside evolve)
  int* nact = nullptr;
  hipStream_t stream = nullptr;    // the class's own stream inside a chunk (default priority)
  hipEvent_t join = nullptr;
};

struct qhd_plan_s {
  int device = 0;
  hipStream_t internal = nullptr;
  hipStream_t last_stream = nullptr;
  bool last_stream_valid = false;
  qhd_plan_opts opts{};
  std::vector<qhd_instance> inst;
  std::vector<int> cls_of, pos_of;
  std::vector<ShapeClass> classes;
  std::vector<double*> dev_tables;
  std::vector<char> potential_set, state_ready;
  double2* twiddles = nullptr;
  std::map<int, size_t> tw_off;
  double* staging_f = nullptr;
  float2* staging_psi = nullptr;
  double* amin_val = nullptr;
  long long* amin_idx = nullptr;
  double* host_results = nullptr;   // pinned, 3 per member of the largest class
  long long total_points = 0;
  int grid_cap = 2048;
  std::string tune_cache;
  void* dft_tables = nullptr;  // FP16 split DFT matrices for the matrix-core 3-D passes
  // evolve runs in chunks of at most chunk_k steps; a full chunk of every class (chunk
  // plan, passes, commit) is captured once as a graph and replayed (see qhd_evolve)
  int chunk_k = 64;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  // timing
  std::vector<Family> families;
  std::vector<Pending> pending;
  std::vector<hipEvent_t> free_events;
  // inside a chunk the classes run concurrently, each on its own stream, forked from
  // the caller's stream and joined back before the step commit
  hipEvent_t fork = nullptr;
};

namespace {

void free_plan(qhd_plan p) {
  if (!p) return;
  (void)hipSetDevice(p->device);
  if (p->internal) (void)hipStreamSynchronize(p->internal);
  if (p->last_stream_valid) (void)hipStreamSynchronize(p->last_stream);
  for (auto& c : p->classes)
    if (c.stream) (void)hipStreamSynchronize(c.stream);
  if (p->fork) (void)hipEventDestroy(p->fork);
  for (auto& c : p->classes) {
    if (c.join) (void)hipEventDestroy(c.join);
    if (c.stream) (void)hipStreamDestroy(c.stream);
    (void)hipFree(c.nact);
    (void)hipFree(c.dev);
    (void)hipFree(c.psi);
    (void)hipFree(c.f);
    (void)hipFree(c.scratch);
    (void)hipFree(c.partials);
    (void)hipFree(c.results);
  }
  for (double* t : p->dev_tables) (void)hipFree(t);
  (void)hipFree(p->twiddles);
  (void)hipFree(p->dft_tables);
  (void)hipFree(p->staging_f);
  (void)hipFree(p->staging_psi);
  (void)hipFree(p->amin_val);
  (void)hipFree(p->amin_idx);
  if (p->host_results) (void)hipHostFree(p->host_results);
  for (auto& pe : p->pending) {
    (void)hipEventDestroy(pe.start);
    (void)hipEventDestroy(pe.stop);
  }
  for (auto e : p->free_events) (void)hipEventDestroy(e);
  if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->internal) (void)hipStreamDestroy(p->internal);
  delete p;
}

int family_index(qhd_plan p, const std::string& name, double bpp) {
  for (size_t k = 0; k < p->families.size(); ++k)
    if (p->families[k].name == name) return (int)k;
  Family f;
  f.name = name;
  f.bytes_per_point = bpp;
  p->families.push_back(f);
  return (int)p->families.size() - 1;
}

hipEvent_t take_event(qhd_plan p) {
  if (!p->free_events.empty()) {
    hipEvent_t e = p->free_events.back();
    p->free_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

qhd_status sync_user_stream(qhd_plan p) {
  if (p->last_stream_valid) HIP_TRY(hipStreamSynchronize(p->last_stream));
  return QHD_OK;
}

qhd_status push_inst(qhd_plan p, int i) {
  ShapeClass& c = p->classes[p->cls_of[i]];
  const int pos = p->pos_of[i];
  HIP_TRY(hipMemcpyAsync(c.dev + pos, &c.host[pos], sizeof(InstDev), hipMemcpyHostToDevice, p->internal));
  HIP_TRY(hipStreamSynchronize(p->internal));
  return QHD_OK;
}

constexpr int kMaxSub = 64;  // sub-steps of one class in one chunk (chunk_k * stages <= 64)

// stages member I takes in a chunk capped at ks steps (host mirror of step_limit)
long long host_limit(const InstDev& I, long long ks) {
  const long long rem = I.nsteps - I.steps_done;
  const long long cap = ks * I.stages;
  return cap > rem ? rem : cap;
}

// members visited in sub-step s of such a chunk (host mirror of the chunk-plan kernel)
int host_nact(const ShapeClass& c, long long ks, long long s) {
  for (int k = (int)c.members.size() - 1; k >= 0; --k)
    if (s < host_limit(c.host[k], ks)) return k + 1;
  return 0;
}

// Launch one chunk of at most ks steps of every class: per class the chunk plan (the
// members each sub-step visits, from the device step counters), then its sub-steps;
// then the commit that advances every member by min(ks, remaining) steps.  full: every
// class issues ks * sps sub-steps (the captured form, valid whatever the counters say);
// otherwise each class issues the sub-steps its members need (from the host mirror).
// concurrent: each class on its own stream, forked from and joined back to `stream`.
// timing: every pass launch is bracketed by HIP events (serialised on `stream`).
qhd_status enqueue_chunk(qhd_plan p, long long ks, hipStream_t stream, bool timing, bool concurrent, bool full) {
  auto timed_on = [&](hipStream_t st, int fam, double points, auto&& fn) -> hipError_t {
    (void)st;
    hipEvent_t a = nullptr, b = nullptr;
    if (timing) {
      a = take_event(p);
      b = take_event(p);
      if (a && b) launch_timing() = LaunchTiming{a, b};  // the pass launch records them
    }
    hipError_t r = fn();
    if (timing && a && b) {
      if (launch_timing().start) {
        // no launch took them (an error before the launch): back to the pool
        launch_timing() = LaunchTiming{};
        p->free_events.push_back(a);
        p->free_events.push_back(b);
      } else {
        p->pending.push_back({a, b, fam, points});
      }
    }
    return r;
  };
  concurrent = concurrent && !timing && p->classes.size() > 1;
  if (concurrent) HIP_TRY(hipEventRecord(p->fork, stream));
  std::vector<int> joined;
  for (size_t ci = 0; ci < p->classes.size(); ++ci) {
    ShapeClass& c = p->classes[ci];
    const int m = (int)c.members.size();
    long long S = 0;
    if (full) {
      S = ks * c.sps;
    } else {
      for (int k = 0; k < m; ++k) S = std::max(S, host_limit(c.host[k], ks));
    }
    if (S <= 0) continue;
    if (S > kMaxSub) return fail(QHD_EINVAL, "internal: %lld sub-steps in one chunk", S);
    hipStream_t st = concurrent ? c.stream : stream;
    if (concurrent) HIP_TRY(hipStreamWaitEvent(st, p->fork, 0));
    HIP_TRY(launch_chunk_plan(c.dev, m, ks, (int)S, c.nact, st));
    if (c.resident) {
      // every sub-step of the chunk in one launch, psi in LDS (timed as a whole: points =
      // the chunk's grid-point stages)
      double gps = 0.0;
      if (timing)
        for (int k = 0; k < m; ++k) gps += (double)host_limit(c.host[k], ks) * (double)c.points;
      HIP_TRY(timed_on(st, c.fam_res, gps, [&] {
        return launch_resident_2d(c.nx, c.ny, c.dev, m, c.nact, c.psi, c.f, c.tw_x, c.tw_y, ks, c.model, c.y4, st);
      }));
    } else {
      for (long long sub = 0; sub < S; ++sub) {
        const int s = (int)sub;
        const int* na = c.nact + s;
        const double pts = timing ? (double)host_nact(c, ks, s) * (double)c.points : 0.0;
        if (c.ndim == 3 && c.mfma) {
          HIP_TRY(timed_on(st, c.fam_row, pts, [&] {
            return launch_mfma_pass_3d(0, 0, c.dev, m, na, p->dft_tables, c.psi, c.f, s, ks, p->grid_cap, st);
          }));
          HIP_TRY(timed_on(st, c.fam_y, pts, [&] {
            return launch_mfma_pass_3d(1, -1, c.dev, m, na, p->dft_tables, c.psi, c.f, s, ks, p->grid_cap, st);
          }));
          HIP_TRY(timed_on(st, c.fam_z, pts, [&] {
            return launch_mfma_pass_3d(2, 0, c.dev, m, na, p->dft_tables, c.psi, c.f, s, ks, p->grid_cap, st);
          }));
          HIP_TRY(timed_on(st, c.fam_y, pts, [&] {
            return launch_mfma_pass_3d(1, +1, c.dev, m, na, p->dft_tables, c.psi, c.f, s, ks, p->grid_cap, st);
          }));
        } else if (c.ndim == 3) {
          HIP_TRY(timed_on(st, c.fam_row, pts, [&] {
            return launch_xpass_3d(c.nx, c.ny, c.nz, c.dev, m, na, c.psi, c.f, c.tw_x, s, ks, p->grid_cap, c.y4, st);
          }));
          HIP_TRY(timed_on(st, c.fam_y, pts, [&] {
            return launch_plane_3d(c.nx, c.ny, c.nz, c.dev, m, na, c.psi, c.tw_y, c.tw_z, s, ks, p->grid_cap, c.y4,
                                   st);
          }));
        } else if (c.ndim == 2 && c.leapfrog) {
          HIP_TRY(timed_on(st, c.fam_row, pts, [&] {
            return launch_lf_row_2d(c.nx, c.ny, c.dev, m, na, c.psi, c.f, c.scratch, s, ks, c.cap_row, st);
          }));
          HIP_TRY(timed_on(st, c.fam_col, pts, [&] {
            return launch_lf_col_2d(c.nx, c.ny, c.dev, m, na, c.psi, c.scratch, s, ks, c.cap_col, st);
          }));
        } else if (c.ndim == 2) {
          HIP_TRY(timed_on(st, c.fam_row, pts, [&] {
            return launch_row_pass_2d(c.nx, c.ny, c.dev, m, na, c.psi, c.f, c.tw_x, s, ks, c.cap_row, c.row_points,
                                      st, c.model, c.y4);
          }));
          HIP_TRY(timed_on(st, c.fam_col, pts, [&] {
            return launch_col_pass_2d(c.nx, c.ny, c.dev, m, na, c.psi, c.tw_y, s, ks, c.cap_col, c.col_variant, st,
                                      c.model, c.y4);
          }));
        } else {
          HIP_TRY(timed_on(st, c.fam_line, pts, [&] {
            return launch_line_pass_1d(c.nx, c.dev, m, na, c.psi, c.f, c.tw_x, s, ks, p->grid_cap, st);
          }));
        }
      }
    }
    if (concurrent) {
      HIP_TRY(hipEventRecord(c.join, st));
      joined.push_back((int)ci);
    }
  }
  for (int ci : joined) HIP_TRY(hipStreamWaitEvent(stream, p->classes[ci].join, 0));
  for (auto& c : p->classes) HIP_TRY(launch_commit(c.dev, (int)c.members.size(), ks, stream));
  return QHD_OK;
}

// advance the host mirror as a chunk of ks steps does on the device
void mirror_chunk(qhd_plan p, long long ks) {
  for (auto& c : p->classes)
    for (auto& I : c.host) {
      const long long l = host_limit(I, ks);
      if (l > 0) {
        I.steps_done += l;
        I.mode = kModePending;
      }
    }
}

// ---- launch tuning ----------------------------------------------------------------

// Tuning-cache lines: "qhd-tune 1 <arch> <nx> <ny> <members_pow2> <col_variant> <cap_row> <cap_col>
// [<row points per lane>]" (the last field is optional, 8 when absent)
std::string tune_key(const std::string& arch, const ShapeClass& c) {
  int m = 1;
  while (m < (int)c.members.size()) m <<= 1;
  char buf[160];
  snprintf(buf, sizeof buf, "qhd-tune 1 %s %d %d %d", arch.c_str(), c.nx, c.ny, m);
  return buf;
}

bool tune_lookup(const std::string& path, const std::string& key, ShapeClass& c) {
  FILE* fh = fopen(path.c_str(), "r");
  if (!fh) return false;
  char line[256];
  bool found = false;
  while (fgets(line, sizeof line, fh)) {
    const size_t k = key.size();
    if (strncmp(line, key.c_str(), k) != 0 || line[k] != ' ') continue;
    int v = 0, cr = 0, cc = 0, rp = 8;
    const int got = sscanf(line + k, "%d %d %d %d", &v, &cr, &cc, &rp);
    if (got >= 3 && v >= kColAuto && v <= kColSplit && cr >= 0 && cc >= 0 && (rp == 8 || rp == 16)) {
      c.col_variant = v;  // the last matching line wins
      c.cap_row = cr;
      c.cap_col = cc;
      c.row_points = got == 4 ? rp : 8;
      found = true;
    }
  }
  fclose(fh);
  return found;
}

void tune_append(const std::string& path, const std::string& key, const ShapeClass& c, double us_row,
                 double us_col) {
  FILE* fh = fopen(path.c_str(), "a");
  if (!fh) return;
  fprintf(fh, "%s %d %d %d %d  # row %.2f us, col %.2f us\n", key.c_str(), c.col_variant, c.cap_row, c.cap_col,
          c.row_points, us_row, us_col);
  fclose(fh);
}

// mean duration (us) of `reps` launches after two untimed ones; negative on error
template <typename F>
double time_launches(hipStream_t st, hipEvent_t a, hipEvent_t b, int reps, F&& fn) {
  for (int k = 0; k < 2; ++k)
    if (fn() != hipSuccess) return -1.0;
  if (hipEventRecord(a, st) != hipSuccess) return -1.0;
  for (int k = 0; k < reps; ++k)
    if (fn() != hipSuccess) return -1.0;
  if (hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess) return -1.0;
  float ms = 0.0f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return -1.0;
  return 1e3 * ms / reps;
}

// Time the row pass over grid caps and the column pass over variants x grid caps on
// the class's own buffers (one sub-step with every member active), keep the
// fastest.  The state is overwritten; the caller restores it.
qhd_status autotune_class(qhd_plan p, ShapeClass& c, double& us_row, double& us_col) {
  const int m = (int)c.members.size();
  static const int caps[] = {512, 1024, 2048, 4096, 8192};
  hipEvent_t a = nullptr, b = nullptr;
  HIP_TRY(hipEventCreate(&a));
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return fail(QHD_EDEVICE, "hipEventCreate failed");
  }
  const int reps = 4;
  us_row = 1e30;
  us_col = 1e30;
  int best_row = c.cap_row, best_col = c.cap_col, best_var = c.col_variant, best_pts = c.row_points;
  bool ok = true;
  std::vector<int> row_pts = {8};
  if (row_points_resolve(c.nx, 16) == 16 && c.nx < 1024) row_pts.push_back(16);
  for (int rp : row_pts)
    for (int cap : caps) {
      const double t = time_launches(p->internal, a, b, reps, [&] {
        return launch_row_pass_2d(c.nx, c.ny, c.dev, m, c.nact + kMaxSub, c.psi, c.f, c.tw_x, 0, 1, cap, rp,
                                  p->internal, c.model,
                                  c.y4);
      });
      if (t < 0) ok = false;
      else if (t < us_row) us_row = t, best_row = cap, best_pts = rp;
    }
  std::vector<int> variants = {kColStaged};
  if (col_variant_resolve(c.ny, kColTileWave) == kColTileWave) variants.push_back(kColTileWave);
  if (col_variant_resolve(c.ny, kColStaged16) == kColStaged16) variants.push_back(kColStaged16);
  if (c.model == kModelQHD && col_variant_resolve(c.ny, kColSplit) == kColSplit) variants.push_back(kColSplit);
  for (int v : variants)
    for (int cap : caps) {
      const double t = time_launches(p->internal, a, b, reps, [&] {
        return launch_col_pass_2d(c.nx, c.ny, c.dev, m, c.nact + kMaxSub, c.psi, c.tw_y, 0, 1, cap, v, p->internal,
                                  c.model, c.y4);
      });
      if (t < 0) ok = false;
      else if (t < us_col) us_col = t, best_col = cap, best_var = v;
    }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (!ok) return fail(QHD_EDEVICE, "autotune launch failed: %s", hipGetErrorString(hipGetLastError()));
  c.cap_row = best_row;
  c.cap_col = best_col;
  c.col_variant = best_var;
  c.row_points = best_pts;
  c.tuned = true;
  return QHD_OK;
}

// Tuning-cache lines of the resident-or-streaming choice: "qhd-resident 1 <arch> <nx> <ny>
// <members_pow2> <model> <1 resident | 0 streaming>"
std::string resident_key(const std::string& arch, const ShapeClass& c) {
  int m = 1;
  while (m < (int)c.members.size()) m <<= 1;
  char buf[160];
  snprintf(buf, sizeof buf, "qhd-resident 1 %s %d %d %d %d", arch.c_str(), c.nx, c.ny, m, c.model);
  return buf;
}

int resident_lookup(const std::string& path, const std::string& key) {
  FILE* fh = fopen(path.c_str(), "r");
  if (!fh) return -1;
  char line[256];
  int dec = -1;
  while (fgets(line, sizeof line, fh)) {
    const size_t k = key.size();
    if (strncmp(line, key.c_str(), k) != 0 || line[k] != ' ') continue;
    int v = -1;
    if (sscanf(line + k, "%d", &v) == 1 && (v == 0 || v == 1)) dec = v;  // the last matching line wins
  }
  fclose(fh);
  return dec;
}

void resident_append(const std::string& path, const std::string& key, int dec, double us_res, double us_str) {
  FILE* fh = fopen(path.c_str(), "a");
  if (!fh) return;
  fprintf(fh, "%s %d  # 16 steps: resident %.2f us, streaming %.2f us\n", key.c_str(), dec, us_res, us_str);
  fclose(fh);
}

// Time 16 steps of the class (every member) as one resident launch and as streaming
// passes with the class's launch configuration.  The state is overwritten; the caller
// restores it.
qhd_status compare_resident(qhd_plan p, ShapeClass& c, double& us_res, double& us_str) {
  const int m = (int)c.members.size();
  const int k = 16;
  hipEvent_t a = nullptr, b = nullptr;
  HIP_TRY(hipEventCreate(&a));
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return fail(QHD_EDEVICE, "hipEventCreate failed");
  }
  us_res = time_launches(p->internal, a, b, 2, [&] {
    return launch_resident_2d(c.nx, c.ny, c.dev, m, c.nact + kMaxSub, c.psi, c.f, c.tw_x, c.tw_y, k, c.model, c.y4,
                              p->internal);
  });
  us_str = time_launches(p->internal, a, b, 2, [&] {
    hipError_t r = hipSuccess;
    for (int s = 0; s < k && r == hipSuccess; ++s) {
      r = launch_row_pass_2d(c.nx, c.ny, c.dev, m, c.nact + kMaxSub, c.psi, c.f, c.tw_x, s, k, c.cap_row, c.row_points,
                             p->internal,
                             c.model, c.y4);
      if (r == hipSuccess)
        r = launch_col_pass_2d(c.nx, c.ny, c.dev, m, c.nact + kMaxSub, c.psi, c.tw_y, s, k, c.cap_col, c.col_variant, p->internal,
                               c.model, c.y4);
    }
    return r;
  });
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (us_res < 0 || us_str < 0)
    return fail(QHD_EDEVICE, "resident comparison launch failed: %s", hipGetErrorString(hipGetLastError()));
  return QHD_OK;
}

// Capture one full chunk of chunk_k steps of every class (classes concurrent) on the
// plan's internal stream; replayed by qhd_evolve for every chunk in which every class
// still has a member with at least chunk_k steps to go.
qhd_status build_chunk_graph(qhd_plan p) {
  HIP_TRY(hipStreamBeginCapture(p->internal, hipStreamCaptureModeThreadLocal));
  qhd_status st = enqueue_chunk(p, p->chunk_k, p->internal, false, true, true);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(p->internal, &g);
  if (st != QHD_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return fail(QHD_EDEVICE, "graph capture: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(&p->graph_exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(QHD_EDEVICE, "graph instantiate: %s", hipGetErrorString(e));
  }
  p->graph = g;
  return QHD_OK;
}

}  // namespace

namespace qhd {
LaunchTiming& launch_timing() {
  thread_local LaunchTiming t;
  return t;
}

// shared with the surrogate's entry points, which report through qhd_last_error()
void set_error_message(const char* msg) { g_err = msg ? msg : ""; }

// read-only view of one instance for the spectrum entry point
qhd_status plan_instance_view(qhd_plan p, int i, InstanceView* v) {
  if (!p || !v) return fail(QHD_EINVAL, "NULL argument");
  if (i < 0 || i >= (int)p->inst.size()) return fail(QHD_EINVAL, "instance index %d out of range", i);
  const ShapeClass& c = p->classes[p->cls_of[i]];
  const int pos = p->pos_of[i];
  const qhd_instance& d = p->inst[i];
  v->ndim = c.ndim;
  v->nx = c.nx;
  v->ny = c.ny;
  v->nz = c.nz;
  v->f = c.f + c.host[pos].psi_off;
  v->tw_x = c.tw_x;
  v->tw_y = c.tw_y;
  v->host = c.host[pos];
  v->device = p->device;
  v->potential_set = p->potential_set[i] != 0;
  for (int a = 0; a < 3; ++a) v->length[a] = d.hi[a] - d.lo[a];
  v->internal = p->internal;
  return QHD_OK;
}
}  // namespace qhd

extern "C" {

const char* qhd_last_error(void) { return g_err.c_str(); }

const char* qhd_version(void) { return "qhd-mi355x 0.1 (gfx950)"; }

qhd_status qhd_plan_create(const qhd_instance* inst, int32_t batch, const qhd_plan_opts* opts,
                           qhd_plan* out) {
  g_err.clear();
  if (!out) return fail(QHD_EINVAL, "out must not be NULL");
  *out = nullptr;
  if (batch <= 0) return fail(QHD_EINVAL, "batch must be > 0 (got %d)", batch);
  if (!inst) return fail(QHD_EINVAL, "inst must not be NULL");
  for (int i = 0; i < batch; ++i) {
    qhd_status st = validate(inst[i], i);
    if (st != QHD_OK) return st;
  }
  qhd_plan p = new qhd_plan_s();
  if (opts) p->opts = *opts;
  if (!(p->opts.norm_tolerance > 0.0)) p->opts.norm_tolerance = 1e-3;
  if (p->opts.timing_stride <= 0) p->opts.timing_stride = 16;
  if (const char* gc = std::getenv("QHD_GRID_CAP")) p->grid_cap = std::max(0, std::atoi(gc));
  p->inst.assign(inst, inst + batch);
  p->cls_of.assign(batch, -1);
  p->pos_of.assign(batch, -1);
  p->potential_set.assign(batch, 0);
  p->state_ready.assign(batch, 0);

  auto bail = [&](qhd_status st) {
    std::string keep = g_err;
    free_plan(p);
    g_err = keep;
    return st;
  };
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) {
    fail(QHD_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    return bail(QHD_EDEVICE);
  }
  e = hipStreamCreateWithFlags(&p->internal, hipStreamNonBlocking);
  if (e != hipSuccess) {
    fail(QHD_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
    return bail(QHD_EDEVICE);
  }

  // group into shape classes
  std::map<std::tuple<int, int, int, int, int, int>, int> key2cls;
  for (int i = 0; i < batch; ++i) {
    const qhd_instance& d = inst[i];
    const int nx = d.n[0], ny = d.ndim >= 2 ? d.n[1] : 1, nz = d.ndim >= 3 ? d.n[2] : 1;
    const bool lf = d.scheme == QHD_SCHEME_LEAPFROG;
    auto key = std::make_tuple(d.ndim, nx, ny, nz, d.model, (int)lf);
    auto it = key2cls.find(key);
    int c;
    if (it == key2cls.end()) {
      c = (int)p->classes.size();
      key2cls[key] = c;
      ShapeClass sc;
      sc.ndim = d.ndim;
      sc.nx = nx;
      sc.ny = ny;
      sc.nz = nz;
      sc.points = (long long)nx * ny * nz;
      sc.model = d.model;
      sc.leapfrog = lf;
      p->classes.push_back(sc);
    } else {
      c = it->second;
    }
    p->classes[c].members.push_back(i);
    p->classes[c].y4 = p->classes[c].y4 || d.scheme == QHD_SCHEME_YOSHIDA4;
    p->classes[c].sps = std::max(p->classes[c].sps, stages_per_step(d));
    p->cls_of[i] = c;
  }
  // twiddle tables W_N^j = exp(-2 pi i j / N) for every line length in use
  std::vector<int> lengths;
  for (auto& c : p->classes) {
    lengths.push_back(c.nx);
    if (c.ndim >= 2) lengths.push_back(c.ny);
    if (c.ndim >= 3) lengths.push_back(c.nz);
  }
  std::sort(lengths.begin(), lengths.end());
  lengths.erase(std::unique(lengths.begin(), lengths.end()), lengths.end());
  size_t tw_total = 0;
  for (int n : lengths) {
    p->tw_off[n] = tw_total;
    tw_total += (size_t)n;
  }
  {
    std::vector<double2> tw(tw_total);
    for (int n : lengths) {
      for (int j = 0; j < n; ++j) {
        const long double ang = 2.0L * 3.141592653589793238462643383279502884L * (long double)j / (long double)n;
        tw[p->tw_off[n] + j] = make_double2((double)cosl(ang), -(double)sinl(ang));
      }
    }
    e = hipMalloc(&p->twiddles, tw_total * sizeof(double2));
    if (e == hipSuccess)
      e = hipMemcpy(p->twiddles, tw.data(), tw_total * sizeof(double2), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      fail(e == hipErrorOutOfMemory ? QHD_ENOMEM : QHD_EDEVICE, "twiddle upload: %s", hipGetErrorString(e));
      return bail(g_err.find("out of memory") != std::string::npos ? QHD_ENOMEM : QHD_EDEVICE);
    }
  }

  long long max_pts = 0;
  size_t max_members = 0;
  long long out_off = 0;
  std::vector<long long> out_off_of(batch);
  for (int i = 0; i < batch; ++i) {
    const qhd_instance& d = inst[i];
    out_off_of[i] = out_off;
    out_off += (long long)d.n[0] * (d.ndim >= 2 ? d.n[1] : 1) * (d.ndim >= 3 ? d.n[2] : 1);
  }
  p->total_points = out_off;

  for (size_t ci = 0; ci < p->classes.size(); ++ci) {
    ShapeClass& c = p->classes[ci];
    std::stable_sort(c.members.begin(), c.members.end(),
                     [&](int a, int b) { return inst[a].nsteps * stages_per_step(inst[a]) >
                                                inst[b].nsteps * stages_per_step(inst[b]); });
    const int m = (int)c.members.size();
    max_pts = std::max(max_pts, c.points);
    max_members = std::max(max_members, (size_t)m);
    c.lines = c.ndim >= 2 ? c.ny * c.nz : 1;
    c.tw_x = p->twiddles + p->tw_off[c.nx];
    c.tw_y = c.ndim >= 2 ? p->twiddles + p->tw_off[c.ny] : nullptr;
    c.tw_z = c.ndim >= 3 ? p->twiddles + p->tw_off[c.nz] : nullptr;
    c.host.resize(m);
    for (int pos = 0; pos < m; ++pos) {
      const int i = c.members[pos];
      const qhd_instance& d = inst[i];
      p->pos_of[i] = pos;
      InstDev& I = c.host[pos];
      std::memset(&I, 0, sizeof I);
      I.dt = d.dt;
      for (int a = 0; a < 3; ++a) {
        if (a < d.ndim) {
          const double L = d.hi[a] - d.lo[a];
          I.kin_turns[a] = 3.141592653589793 * d.dt / (L * L);
          I.h[a] = L / (double)d.n[a];
        }
      }
      I.sched = d.sched_kind;
      I.scheme = d.scheme;
      I.model = d.model;
      I.sched_p0 = d.sched_p[0];
      I.sched_p1 = d.sched_p[1];
      I.r2 = d.success_radius * d.success_radius;
      I.stages = stages_per_step(d);
      I.nsteps = d.nsteps * I.stages;
      I.steps_done = 0;
      I.mode = kModeClean;
      I.plan_index = i;
      I.psi_off = (long long)pos * c.points;
      I.out_off = out_off_of[i];
      if (d.sched_kind == QHD_SCHED_TABLE && d.nsteps > 0) {
        double* t = nullptr;
        e = hipMalloc(&t, sizeof(double) * 2 * d.nsteps);
        if (e == hipSuccess) {
          p->dev_tables.push_back(t);
          e = hipMemcpy(t, d.sched_table, sizeof(double) * 2 * d.nsteps, hipMemcpyHostToDevice);
        }
        if (e != hipSuccess) {
          fail(e == hipErrorOutOfMemory ? QHD_ENOMEM : QHD_EDEVICE, "schedule table upload: %s", hipGetErrorString(e));
          return bail(e == hipErrorOutOfMemory ? QHD_ENOMEM : QHD_EDEVICE);
        }
        I.table = t;
        p->inst[i].sched_table = nullptr;  // the caller's pointer is not kept
      }
    }
    const size_t pts = (size_t)m * (size_t)c.points;
    e = hipMalloc(&c.dev, sizeof(InstDev) * m);
    if (e == hipSuccess) e = hipMalloc(&c.psi, sizeof(float2) * pts);
    if (e == hipSuccess && c.leapfrog) e = hipMalloc(&c.scratch, sizeof(float) * pts);
    if (e == hipSuccess) e = hipMalloc(&c.f, sizeof(double) * pts);
    if (e == hipSuccess) e = hipMalloc(&c.partials, sizeof(double) * 3 * (size_t)m * c.lines);
    if (e == hipSuccess) e = hipMalloc(&c.results, sizeof(double) * 3 * (size_t)m);
    if (e == hipSuccess) e = hipMalloc(&c.nact, sizeof(int) * (kMaxSub + 1));
    if (e == hipSuccess) {
      std::vector<int> counts(kMaxSub + 1, m);
      e = hipMemcpy(c.nact, counts.data(), sizeof(int) * counts.size(), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipMemcpy(c.dev, c.host.data(), sizeof(InstDev) * m, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
      // uniform initial state N^{-1/2} (App. C.2.1 experiment); USER states are
      // overwritten by qhd_set_state
      e = launch_fill_psi(c.psi, (long long)pts, (float)(1.0 / std::sqrt((double)c.points)), p->internal);
    }
    if (e == hipSuccess) e = hipMemsetAsync(c.f, 0, sizeof(double) * pts, p->internal);
    if (e != hipSuccess) {
      fail(e == hipErrorOutOfMemory ? QHD_ENOMEM : QHD_EDEVICE, "class allocation: %s", hipGetErrorString(e));
      return bail(e == hipErrorOutOfMemory ? QHD_ENOMEM : QHD_EDEVICE);
    }
    char name[48];
    c.mfma = (p->opts.flags & QHD_OPT_MFMA_DFT) && c.ndim == 3 && c.nx == 128 && c.ny == 128 && c.nz == 128;
    if (c.mfma) {
      c.fam_row = family_index(p, "xpass_3d_mfma/n128", 24.0);
      c.fam_y = family_index(p, "ypass_3d_mfma/n128", 16.0);
      c.fam_z = family_index(p, "zpass_3d_mfma/n128", 16.0);
    } else if (c.ndim == 3) {
      // plane layout: an x-pass (psi read + write, f read) and a (y, z)-plane pass
      c.plane = true;
      snprintf(name, sizeof name, "xpass_3d/n%d", c.nx);
      c.fam_row = family_index(p, name, 24.0);
      snprintf(name, sizeof name, "plane_3d/n%dx%d", c.ny, c.nz);
      c.fam_y = family_index(p, name, 16.0);
    } else if (c.ndim == 2) {
      if ((p->opts.flags & QHD_OPT_RESIDENT) && !c.leapfrog && resident_supported(c.nx, c.ny)) {
        // psi stays in LDS; per grid-point step only f (8 B, FP64) is read, from the caches.
        // The streaming families below are kept too: the autotuner may choose them.
        c.resident = true;
        snprintf(name, sizeof name, "resident_2d%s/n%d", c.model == kModelQAA ? "_qaa" : "", c.nx);
        c.fam_res = family_index(p, name, 8.0);
      }
      // leapfrog stages: the row pass reads psi and f and writes the partial H v (4 B),
      // the column pass reads psi and it and writes psi
      const char* tag = c.leapfrog ? "_qaa_lf" : (c.model == kModelQAA ? "_qaa" : "");
      snprintf(name, sizeof name, "row_pass_2d%s/n%d", tag, c.nx);
      c.fam_row = family_index(p, name, c.leapfrog ? 20.0 : 24.0);
      snprintf(name, sizeof name, "col_pass_2d%s/n%d", tag, c.ny);
      c.fam_col = family_index(p, name, c.leapfrog ? 20.0 : 16.0);
    } else {
      snprintf(name, sizeof name, "line_pass_1d/n%d", c.nx);
      c.fam_line = family_index(p, name, 24.0);
    }
  }
  for (int i = 0; i < batch; ++i) p->state_ready[i] = inst[i].init_kind == QHD_INIT_UNIFORM;
  if (std::any_of(p->classes.begin(), p->classes.end(), [](const ShapeClass& c) { return c.mfma; })) {
    // the 128 distinct entries w(m) = e^{-+2 pi i m / 128} of W_jk = w(jk mod 128), each
    // part written as w0 + 2^-12 w1 + 2^-24 w2 with FP16 terms: [sign][m][re w0, re w1,
    // re w2, im w0, im w1, im w2, 0, 0]
    const int n = 128;
    std::vector<_Float16> tab((size_t)2 * n * 8, (_Float16)0.0f);
    auto split3 = [](long double v, _Float16* out) {
      const _Float16 a = (_Float16)(float)v;
      const long double r1 = (v - (long double)(float)a) * 4096.0L;
      const _Float16 b = (_Float16)(float)r1;
      const long double r2 = (r1 - (long double)(float)b) * 4096.0L;
      out[0] = a;
      out[1] = b;
      out[2] = (_Float16)(float)r2;
    };
    for (int sg = 0; sg < 2; ++sg)
      for (int m = 0; m < n; ++m) {
        const long double ang = 2.0L * 3.141592653589793238462643383279502884L * (long double)m / n;
        _Float16* e = &tab[((size_t)sg * n + m) * 8];
        split3(cosl(ang), e);
        split3((sg == 0 ? -1.0L : 1.0L) * sinl(ang), e + 3);
      }
    e = hipMalloc(&p->dft_tables, tab.size() * sizeof(_Float16));
    if (e == hipSuccess) e = hipMemcpy(p->dft_tables, tab.data(), tab.size() * sizeof(_Float16), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      fail(e == hipErrorOutOfMemory ? QHD_ENOMEM : QHD_EDEVICE, "DFT table upload: %s", hipGetErrorString(e));
      return bail(e == hipErrorOutOfMemory ? QHD_ENOMEM : QHD_EDEVICE);
    }
  }
  // launch configuration per class: tuning cache, else autotune (QHD_OPT_AUTOTUNE), else defaults
  if (p->opts.tune_cache) p->tune_cache = p->opts.tune_cache;
  p->opts.tune_cache = nullptr;  // the caller's string is not kept
  {
    std::string arch = "gfx";
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) arch = prop.gcnArchName;
    for (auto& c : arch) if (c == ' ' || c == ':') c = '_';
    bool refill = false;
    const bool env_cap = std::getenv("QHD_GRID_CAP") != nullptr;
    const bool autotune = (p->opts.flags & QHD_OPT_AUTOTUNE) != 0;
    for (auto& c : p->classes) {
      c.cap_row = c.cap_col = p->grid_cap;
      if (c.ndim != 2) continue;
      if (c.model != kModelQAA) {  // QAA passes have one fixed launch form
        if (!env_cap) {
          // measured defaults (uniform batches of 256 instances per size on MI355X)
          c.cap_row = c.nx >= 512 ? 8192 : (c.nx >= 256 ? 4096 : 1024);
          c.cap_col = c.ny >= 512 ? 4096 : (c.ny >= 256 ? 2048 : 1024);
        }
        // 1024-point columns of one or two members: the tile-wave form runs 8 waves per
        // tile column where the staged one runs 4 (one 1024^2 instance: column pass 21.5
        // -> 15.7 us); larger classes keep the staged default (4 members: 28.9 vs 31.2 us)
        if (c.ny == 1024 && c.members.size() <= 2) c.col_variant = kColTileWave;
        const std::string key = tune_key(arch, c);
        const bool cached = !p->tune_cache.empty() && tune_lookup(p->tune_cache, key, c);
        if (!cached && autotune) {
          double us_row = 0.0, us_col = 0.0;
          qhd_status st = autotune_class(p, c, us_row, us_col);
          if (st != QHD_OK) return bail(st);
          refill = true;
          if (!p->tune_cache.empty()) tune_append(p->tune_cache, key, c, us_row, us_col);
        }
      }
      if (c.resident && autotune) {
        // resident or streaming, whichever runs this class faster (or the cached choice)
        const std::string rkey = resident_key(arch, c);
        int dec = p->tune_cache.empty() ? -1 : resident_lookup(p->tune_cache, rkey);
        if (dec < 0) {
          double us_res = 0.0, us_str = 0.0;
          qhd_status st = compare_resident(p, c, us_res, us_str);
          if (st != QHD_OK) return bail(st);
          refill = true;
          dec = us_res <= us_str ? 1 : 0;
          if (!p->tune_cache.empty()) resident_append(p->tune_cache, rkey, dec, us_res, us_str);
        }
        c.resident = dec == 1;
      }
    }
    if (refill) {
      for (auto& c : p->classes) {
        e = launch_fill_psi(c.psi, (long long)c.members.size() * c.points,
                            (float)(1.0 / std::sqrt((double)c.points)), p->internal);
        if (e != hipSuccess) {
          fail(QHD_EDEVICE, "state fill after tuning: %s", hipGetErrorString(e));
          return bail(QHD_EDEVICE);
        }
      }
    }
  }
  // a stream and a join event per class, one fork event: the classes of a chunk run
  // concurrently (default stream priority)
  if (p->classes.size() > 1) {
    e = hipEventCreateWithFlags(&p->fork, hipEventDisableTiming);
    for (auto& c : p->classes) {
      if (e == hipSuccess) e = hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&c.join, hipEventDisableTiming);
    }
    if (e != hipSuccess) {
      fail(QHD_EDEVICE, "class streams: %s", hipGetErrorString(e));
      return bail(QHD_EDEVICE);
    }
  }
  // chunk length: 64 sub-steps of the class with the most stages per step; one full chunk
  // of every class captured as a graph
  {
    int sps = 1;
    for (auto& c : p->classes) sps = std::max(sps, c.sps);
    p->chunk_k = std::max(1, kMaxSub / sps);
    long long most = 0;
    for (int i = 0; i < batch; ++i) most = std::max(most, (long long)inst[i].nsteps);
    if (most >= p->chunk_k && !(p->opts.flags & QHD_OPT_NO_GRAPH)) {
      qhd_status st = build_chunk_graph(p);
      if (st != QHD_OK) return bail(st);
    }
  }
  e = hipMalloc(&p->staging_f, sizeof(double) * max_pts);
  if (e == hipSuccess) e = hipMalloc(&p->staging_psi, sizeof(float2) * max_pts);
  if (e == hipSuccess) e = hipMalloc(&p->amin_val, sizeof(double) * (1 + kArgminBlocks));
  if (e == hipSuccess) e = hipMalloc(&p->amin_idx, sizeof(long long) * (2 + 2 * kArgminBlocks));
  if (e == hipSuccess) e = hipHostMalloc((void**)&p->host_results, sizeof(double) * 3 * max_members);
  if (e == hipSuccess) e = hipStreamSynchronize(p->internal);
  if (e != hipSuccess) {
    fail(e == hipErrorOutOfMemory ? QHD_ENOMEM : QHD_EDEVICE, "plan allocation: %s", hipGetErrorString(e));
    return bail(e == hipErrorOutOfMemory ? QHD_ENOMEM : QHD_EDEVICE);
  }
  *out = p;
  return QHD_OK;
}

qhd_status qhd_plan_destroy(qhd_plan plan) {
  g_err.clear();
  free_plan(plan);
  return QHD_OK;
}

qhd_status qhd_plan_points(qhd_plan plan, int64_t* total_points) {
  g_err.clear();
  if (!plan || !total_points) return fail(QHD_EINVAL, "plan and total_points must not be NULL");
  *total_points = plan->total_points;
  return QHD_OK;
}

qhd_status qhd_set_potential(qhd_plan p, int32_t i, const double* f, int32_t on_device) {
  g_err.clear();
  if (!p) return fail(QHD_EINVAL, "plan is NULL");
  if (i < 0 || i >= (int)p->inst.size()) return fail(QHD_EINVAL, "instance index %d out of range", i);
  if (!f) return fail(QHD_EINVAL, "f is NULL");
  HIP_TRY(hipSetDevice(p->device));
  qhd_status st = sync_user_stream(p);
  if (st != QHD_OK) return st;
  ShapeClass& c = p->classes[p->cls_of[i]];
  const int pos = p->pos_of[i];
  HIP_TRY(hipMemcpyAsync(p->staging_f, f, sizeof(double) * c.points,
                         on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, p->internal));
  HIP_TRY(launch_argmin(p->staging_f, c.points, p->amin_val, p->amin_idx, p->amin_val + 1, p->amin_idx + 2,
                        p->amin_idx + 2 + kArgminBlocks, p->internal));
  if (c.plane)
    HIP_TRY(launch_import_f_plane(c.nx, c.ny, c.nz, p->staging_f, c.f + c.host[pos].psi_off, p->internal));
  else
    HIP_TRY(launch_import_f(c.ndim >= 2 ? 2 : 1, c.nx, c.ny * c.nz, p->staging_f, c.f + c.host[pos].psi_off,
                            p->internal));
  double v = 0.0;
  long long idx[2] = {0, 0};
  HIP_TRY(hipMemcpyAsync(&v, p->amin_val, sizeof v, hipMemcpyDeviceToHost, p->internal));
  HIP_TRY(hipMemcpyAsync(idx, p->amin_idx, sizeof idx, hipMemcpyDeviceToHost, p->internal));
  HIP_TRY(hipStreamSynchronize(p->internal));
  if (idx[1] != 0) return fail(QHD_EINVAL, "instance %d: f has %lld non-finite values", i, idx[1]);
  c.host[pos].f_min = v;
  c.host[pos].argmin = idx[0];
  p->potential_set[i] = 1;
  return push_inst(p, i);
}

qhd_status qhd_set_state(qhd_plan p, int32_t i, const float* psi, int32_t on_device) {
  g_err.clear();
  if (!p) return fail(QHD_EINVAL, "plan is NULL");
  if (i < 0 || i >= (int)p->inst.size()) return fail(QHD_EINVAL, "instance index %d out of range", i);
  if (!psi) return fail(QHD_EINVAL, "psi is NULL");
  HIP_TRY(hipSetDevice(p->device));
  qhd_status st = sync_user_stream(p);
  if (st != QHD_OK) return st;
  ShapeClass& c = p->classes[p->cls_of[i]];
  const int pos = p->pos_of[i];
  HIP_TRY(hipMemcpyAsync(p->staging_psi, psi, sizeof(float2) * c.points,
                         on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, p->internal));
  if (c.plane)
    HIP_TRY(launch_import_psi_plane(c.nx, c.ny, c.nz, p->staging_psi, c.psi + c.host[pos].psi_off, p->internal));
  else
    HIP_TRY(launch_import_psi(c.ndim >= 2 ? 2 : 1, c.nx, c.ny * c.nz, p->staging_psi, c.psi + c.host[pos].psi_off,
                              p->internal));
  c.host[pos].mode = kModeClean;
  p->state_ready[i] = 1;
  return push_inst(p, i);
}

qhd_status qhd_set_steps_done(qhd_plan p, int32_t i, int64_t j) {
  g_err.clear();
  if (!p) return fail(QHD_EINVAL, "plan is NULL");
  if (i < 0 || i >= (int)p->inst.size()) return fail(QHD_EINVAL, "instance index %d out of range", i);
  if (j < 0 || j > p->inst[i].nsteps) return fail(QHD_EINVAL, "steps_done %lld outside [0, nsteps]", (long long)j);
  HIP_TRY(hipSetDevice(p->device));
  qhd_status st = sync_user_stream(p);
  if (st != QHD_OK) return st;
  ShapeClass& c = p->classes[p->cls_of[i]];
  InstDev& I = c.host[p->pos_of[i]];
  if (I.mode != kModeClean)
    return fail(QHD_ESTATE, "instance %d: set_steps_done needs a clean state (call qhd_set_state first)", i);
  I.steps_done = j * I.stages;
  return push_inst(p, i);
}

qhd_status qhd_evolve(qhd_plan p, int64_t max_steps, void* stream_v) {
  g_err.clear();
  if (!p) return fail(QHD_EINVAL, "plan is NULL");
  const char* inj = std::getenv("QHD_FAULT_INJECT");
  if (inj && std::strcmp(inj, "evolve") == 0) return fail(QHD_EDEVICE, "fault injected in qhd_evolve");
  for (size_t i = 0; i < p->inst.size(); ++i) {
    if (!p->potential_set[i]) return fail(QHD_ESTATE, "instance %zu: qhd_set_potential was not called", i);
    if (!p->state_ready[i]) return fail(QHD_ESTATE, "instance %zu: INIT_USER needs qhd_set_state before evolve", i);
  }
  hipStream_t stream = (hipStream_t)stream_v;
  HIP_TRY(hipSetDevice(p->device));
  // steps every class still has to take in this call (host mirror of the device counters)
  long long S = 0, rmin = -1;
  for (auto& c : p->classes) {
    long long rc = 0;
    for (auto& I : c.host) {
      long long r = (I.nsteps - I.steps_done) / I.stages;
      if (max_steps >= 0 && r > max_steps) r = max_steps;
      rc = std::max(rc, r);
    }
    S = std::max(S, rc);
    rmin = rmin < 0 ? rc : std::min(rmin, rc);
  }
  const bool timing = (p->opts.flags & QHD_OPT_TIME_PASSES) != 0;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  HIP_TRY(hipStreamIsCapturing(stream, &cap));
  const long long K = p->chunk_k;
  // full chunks, in which every class has a member to advance by all K steps: replays of
  // the captured chunk (with pass timing, one in timing_stride of them is launched directly
  // with every pass timed instead); then the rest in direct chunks of at most K steps,
  // each issuing only the sub-steps its members need
  const bool replay = p->graph_exec && cap == hipStreamCaptureStatusNone && !(p->opts.flags & QHD_OPT_NO_GRAPH);
  const long long full = replay ? rmin / K : 0;
  long long done = 0;
  for (long long ch = 0; ch < full; ++ch, done += K) {
    if (timing && ch % p->opts.timing_stride == 0) {
      qhd_status st = enqueue_chunk(p, K, stream, true, false, true);
      if (st != QHD_OK) return st;
    } else {
      HIP_TRY(hipGraphLaunch(p->graph_exec, stream));
    }
    mirror_chunk(p, K);
  }
  for (long long ch = 0; done < S; ++ch) {
    const long long ks = std::min(K, S - done);
    qhd_status st = enqueue_chunk(p, ks, stream, timing && ch % p->opts.timing_stride == 0, true, false);
    if (st != QHD_OK) return st;
    mirror_chunk(p, ks);
    done += ks;
  }
  p->last_stream = stream;
  p->last_stream_valid = true;
  return QHD_OK;
}

qhd_status qhd_plan_info(qhd_plan p, qhd_class_info* out, int32_t cap, int32_t* n_classes,
                         int32_t* graph_steps) {
  g_err.clear();
  if (!p || !n_classes || !graph_steps || (cap > 0 && !out)) return fail(QHD_EINVAL, "NULL argument");
  *n_classes = (int32_t)p->classes.size();
  *graph_steps = p->graph_exec ? p->chunk_k : 0;
  for (int k = 0; k < cap && k < (int)p->classes.size(); ++k) {
    const ShapeClass& c = p->classes[k];
    qhd_class_info& o = out[k];
    o.ndim = c.ndim;
    o.n[0] = c.nx;
    o.n[1] = c.ny;
    o.n[2] = c.nz;
    o.members = (int32_t)c.members.size();
    o.col_variant = c.ndim == 2 && !c.resident ? col_variant_resolve(c.ny, c.col_variant) : 0;
    o.grid_cap_row = c.cap_row;
    o.grid_cap_col = c.cap_col;
    o.tuned = c.tuned ? 1 : 0;
    o.mfma_dft = c.mfma ? 1 : 0;
    o.row_points_per_lane = c.ndim == 2 && !c.resident ? row_points_resolve(c.nx, c.row_points) : 0;
    o.resident = c.resident ? 1 : 0;
  }
  return QHD_OK;
}

qhd_status qhd_reset(qhd_plan p, void* stream_v) {
  g_err.clear();
  if (!p) return fail(QHD_EINVAL, "plan is NULL");
  hipStream_t stream = (hipStream_t)stream_v;
  HIP_TRY(hipSetDevice(p->device));
  for (auto& c : p->classes) {
    const int m = (int)c.members.size();
    HIP_TRY(launch_fill_psi(c.psi, (long long)m * c.points, (float)(1.0 / std::sqrt((double)c.points)), stream));
    HIP_TRY(launch_reset_inst(c.dev, m, stream));
    for (int k = 0; k < m; ++k) {
      c.host[k].steps_done = 0;
      c.host[k].mode = kModeClean;
      const int i = c.host[k].plan_index;
      p->state_ready[i] = p->inst[i].init_kind == QHD_INIT_UNIFORM;
    }
  }
  p->last_stream = stream;
  p->last_stream_valid = true;
  return QHD_OK;
}

qhd_status qhd_observe(qhd_plan p, void* stream_v, qhd_observables* out, float* rho_dev,
                       float* psi_dev) {
  g_err.clear();
  if (!p) return fail(QHD_EINVAL, "plan is NULL");
  if (!out) return fail(QHD_EINVAL, "host_out is NULL");
  for (size_t i = 0; i < p->inst.size(); ++i)
    if (!p->potential_set[i]) return fail(QHD_ESTATE, "instance %zu: qhd_set_potential was not called", i);
  hipStream_t stream = (hipStream_t)stream_v;
  HIP_TRY(hipSetDevice(p->device));
  qhd_status status = QHD_OK;
  for (auto& c : p->classes) {
    const int m = (int)c.members.size();
    if (c.plane)
      HIP_TRY(launch_observe_plane(c.nx, c.ny, c.nz, c.dev, m, c.psi, c.f, c.tw_x, reinterpret_cast<float2*>(psi_dev),
                                   rho_dev, c.partials, stream));
    else if (c.ndim >= 2)
      HIP_TRY(launch_observe_2d(c.nx, c.ny * c.nz, c.ny, c.dev, m, c.psi, c.f, c.tw_x,
                                reinterpret_cast<float2*>(psi_dev), rho_dev, c.partials, stream, c.model));
    else
      HIP_TRY(launch_observe_1d(c.nx, c.dev, m, c.psi, c.f, reinterpret_cast<float2*>(psi_dev),
                                rho_dev, c.partials, stream));
    HIP_TRY(launch_finalize(c.partials, c.lines, m, c.results, stream));
    HIP_TRY(hipMemcpyAsync(p->host_results, c.results, sizeof(double) * 3 * m, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    for (int k = 0; k < m; ++k) {
      const InstDev& I = c.host[k];
      qhd_observables& o = out[I.plan_index];
      const double* r = p->host_results + 3 * k;
      o.norm = r[0];
      o.e_f = r[1] / r[0];
      o.success_mass = r[2] / r[0];
      o.f_min = I.f_min;
      o.argmin_index = I.argmin;
      o.steps_done = I.steps_done / I.stages;
      o.t = (double)o.steps_done * I.dt;
      if (!std::isfinite(o.norm) || !std::isfinite(o.e_f) || !std::isfinite(o.success_mass)) {
        if (status == QHD_OK) status = fail(QHD_ENUMERIC, "instance %d: non-finite observable", I.plan_index);
      } else if (std::fabs(o.norm - 1.0) > p->opts.norm_tolerance) {
        if (status == QHD_OK)
          status = fail(QHD_ENUMERIC, "instance %d: |norm - 1| = %.3e exceeds %.3e", I.plan_index,
                        std::fabs(o.norm - 1.0), p->opts.norm_tolerance);
      }
    }
  }
  p->last_stream = stream;
  p->last_stream_valid = true;
  return status;
}

qhd_status qhd_kernel_timings(qhd_plan p, qhd_kernel_timing* out, int32_t cap, int32_t* count) {
  g_err.clear();
  if (!p || !count) return fail(QHD_EINVAL, "plan and count must not be NULL");
  HIP_TRY(hipSetDevice(p->device));
  qhd_status st = sync_user_stream(p);
  if (st != QHD_OK) return st;
  for (auto& pe : p->pending) {
    float ms = 0.0f;
    HIP_TRY(hipEventSynchronize(pe.stop));
    HIP_TRY(hipEventElapsedTime(&ms, pe.start, pe.stop));
    Family& f = p->families[pe.family];
    f.launches += 1;
    f.total_ms += ms;
    f.points += pe.points;
    p->free_events.push_back(pe.start);
    p->free_events.push_back(pe.stop);
  }
  p->pending.clear();
  int n = 0;
  for (auto& f : p->families) {
    if (out && n < cap) {
      qhd_kernel_timing& o = out[n];
      std::memset(&o, 0, sizeof o);
      std::snprintf(o.name, sizeof o.name, "%s", f.name.c_str());
      o.launches = f.launches;
      o.total_ms = f.total_ms;
      o.points = f.points;
      o.bytes_per_point = f.bytes_per_point;
    }
    ++n;
    f.launches = 0;
    f.total_ms = 0.0;
    f.points = 0.0;
  }
  *count = n;
  return QHD_OK;
}

}  // extern "C"
