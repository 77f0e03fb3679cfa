// Internal types shared by the C-ABI layer (qhd_api.cpp) and the kernels
// (qhd_kernels.hip).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stdint.h>

namespace qhd {

enum : int { kModeClean = 0, kModePending = 1 };
enum : int { kSchemeStrang = 0, kSchemeLie = 1, kSchemeYoshida4 = 2, kSchemeLeapfrog = 3 };
enum : int { kModelQHD = 0, kModelQAA = 1 };
enum : int { kSchedNesterov = 0, kSchedConst = 1, kSchedTable = 2, kSchedLinear = 3 };

// Per-instance parameters as the kernels see them.  One array per shape class.
struct InstDev {
  double dt;
  double kin_turns[3];   // pi * dt / L_a^2: kinetic phase in turns per (a * n_a^2)
  double h[3];           // mesh spacing per axis
  double sched_p0, sched_p1;
  const double* table;   // device copy of (a_j, b_j) pairs, kSchedTable only
  double r2;             // success radius squared
  double f_min;          // f(x*)
  long long nsteps;      // in stages (steps x stages)
  long long steps_done;  // in stages; authoritative device copy (updated by the commit kernel)
  long long psi_off;     // element offset of the instance in its class buffers
  long long out_off;     // element offset in plan-wide concatenated outputs
  long long argmin;      // flat index of x*
  int sched;
  int mode;              // kModeClean / kModePending
  int plan_index;        // position in the user's batch
  int scheme;            // kSchemeStrang / kSchemeLie / kSchemeYoshida4
  int model;             // kModelQHD / kModelQAA
  int stages;            // stages per step: 3 for kSchemeYoshida4, else 1
};

// What the spectrum entry point (qhd_spectrum.cpp) reads of one plan instance.
struct InstanceView {
  int ndim, nx, ny, nz;
  const double* f;        // the instance's tiled FP64 potential
  const double2* tw_x;    // twiddle tables W_N^j of the x and y line lengths
  const double2* tw_y;
  InstDev host;           // host mirror of the instance parameters
  int device;
  bool potential_set;
  double length[3];       // box lengths per axis
  hipStream_t internal;   // the plan's own stream
};

// Sampled HIP-event timing of pass launches.
struct TimingSink {
  hipEvent_t* ev;        // pairs (start, stop); nullptr when timing is off
  int* used;             // host counter of pairs in use for this launch family
};

// Launchers (qhd_kernels.hip).  All are asynchronous on `stream` and return
// hipSuccess or the launch error.  `nx`, `ny` are the class's mesh sizes.
// Pass launchers take two member counts: `ninst` sizes the grid (the class's members),
// `nact` is the device address of the number of members the kernel visits in this
// sub-step (a prefix of the class, written by launch_chunk_plan or set once at plan
// creation), so that a captured launch stays valid while members finish.
hipError_t launch_row_pass_2d(int nx, int ny, const InstDev* inst, int ninst, const int* nact, float2* psi,
                              const double* f, const double2* tw_nx, int s, long long max_steps,
                              int grid_cap, int points_per_lane, hipStream_t stream, int model = kModelQHD,
                              bool y4 = true);
// Sampled pass timing.  When armed, the next pass launch of this host thread records
// the two events itself: hipExtLaunchKernelGGL stamps them with the dispatch's own start
// and end (what a kernel trace reports), where events recorded around a launch would
// add the marker packets and the wait between them to every sampled duration.
struct LaunchTiming {
  hipEvent_t start = nullptr, stop = nullptr;
};
LaunchTiming& launch_timing();
#define QHD_LAUNCH(kernel, grid, block, shmem, stream, ...)                                                    \
  do {                                                                                                        \
    ::qhd::LaunchTiming& qhd_lt_ = ::qhd::launch_timing();                                                    \
    if (qhd_lt_.start) {                                                                                      \
      hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, qhd_lt_.start, qhd_lt_.stop, 0, __VA_ARGS__); \
      qhd_lt_ = ::qhd::LaunchTiming{};                                                                        \
    } else {                                                                                                  \
      hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);                                    \
    }                                                                                                         \
  } while (0)

// column-pass variants: staged (tile column through LDS, one wavefront per line, 8
// or 16 points per lane), tile-wave (8x8 tiles straight to registers, a line spread
// over TPL/8 wavefronts) or split (512 points: the first forward and the last inverse
// stage in the tile-wave layout, straight from and to HBM, the stages between one
// wavefront per line); kColAuto takes the measured default for the size
enum { kColAuto = 0, kColStaged = 1, kColTileWave = 2, kColStaged16 = 3, kColSplit = 4 };
int col_variant_resolve(int ny, int variant);
// points per lane of the row pass: 8, or 16 (chosen for 256 and 512; always at 1024)
int row_points_resolve(int nx, int points_per_lane);
// leapfrog stages of the QAA model: the row pass writes the partial H v into scratch
// (float per point, psi's layout), the column pass completes H v and updates psi
hipError_t launch_lf_row_2d(int nx, int ny, const InstDev* inst, int ninst, const int* nact, const float2* psi,
                            const double* f,
                            float* scratch, int s, long long max_steps, int grid_cap, hipStream_t stream);
hipError_t launch_lf_col_2d(int nx, int ny, const InstDev* inst, int ninst, const int* nact, float2* psi,
                            const float* scratch, int s,
                            long long max_steps, int grid_cap, hipStream_t stream);
hipError_t launch_col_pass_2d(int nx, int ny, const InstDev* inst, int ninst, const int* nact, float2* psi,
                              const double2* tw_ny, int s, long long max_steps, int grid_cap,
                              int variant, hipStream_t stream, int model = kModelQHD, bool y4 = true);
hipError_t launch_line_pass_1d(int n, const InstDev* inst, int ninst, const int* nact, float2* psi, const double* f,
                               const double2* tw, int s, long long max_steps, int grid_cap,
                               hipStream_t stream);
hipError_t launch_commit(InstDev* inst, int ninst, long long max_steps, hipStream_t stream);
// Active-member counts of the sub-steps s = 0..S-1 of an evolve chunk capped at
// max_steps steps: nact[s] = 1 + the last member k with step_limit(inst[k]) > s (0 if
// none).  Members are sorted by step count, so the prefix is tight for batches evolved
// together; a finished member inside it is computed and its result discarded.
hipError_t launch_chunk_plan(const InstDev* inst, int ninst, long long max_steps, int S, int* nact,
                             hipStream_t stream);

// Resident 2-D steps (qhd_kernels_resident.hip): one workgroup per instance holds psi in
// LDS for every step of the call (max_steps as for the passes), reading and writing the
// tiled HBM state once.  nx, ny in {32, 64, 128}.
bool resident_supported(int nx, int ny);
hipError_t launch_resident_2d(int nx, int ny, const InstDev* inst, int ninst, const int* nact, float2* psi,
                              const double* f,
                              const double2* tw_nx, const double2* tw_ny, long long max_steps, int model,
                              bool y4, hipStream_t stream);

// 3-D (qhd_kernels_3d.hip), plane layout: x slowest, every (y, z) plane contiguous in 8x8
// tiles of (y, z).  The x-pass does F_x . V . F_x^{-1} (lines along x, f read), the plane
// pass F_y^{-1} F_z^{-1} K F_z F_y on one (y, z) plane per k_x held in LDS.
hipError_t launch_xpass_3d(int nx, int ny, int nz, const InstDev* inst, int ninst, const int* nact, float2* psi,
                           const double* f, const double2* tw_x, int s, long long max_steps, int grid_cap, bool y4,
                           hipStream_t stream);
hipError_t launch_plane_3d(int nx, int ny, int nz, const InstDev* inst, int ninst, const int* nact, float2* psi,
                           const double2* tw_y, const double2* tw_z, int s, long long max_steps, int grid_cap,
                           bool y4, hipStream_t stream);
// readouts of plane-layout instances: partials as launch_observe_2d (one triple per x-line,
// line (y, z) of instance i at i * ny * nz + z * ny + y)
hipError_t launch_observe_plane(int nx, int ny, int nz, const InstDev* inst, int ninst, const float2* psi,
                                const double* f, const double2* tw_x, float2* out_psi, float* out_rho,
                                double* partials, hipStream_t stream);
// user row-major (x fastest) -> plane layout
hipError_t launch_import_f_plane(int nx, int ny, int nz, const double* user, double* dst, hipStream_t stream);
hipError_t launch_import_psi_plane(int nx, int ny, int nz, const float2* user, float2* dst, hipStream_t stream);

// Observe: closes the pending half step, writes the user-layout psi / rho
// (optional, plan-wide concatenated buffers) and per-line FP64 partial sums
// (3 per line: sum rho, sum f rho, sum of rho inside the success ball).
// `rows` = ny (2-D) or ny*nz (3-D); `ny` is the slab height used to recover
// (y, z) from a row for the success test.
hipError_t launch_observe_2d(int nx, int rows, int ny, const InstDev* inst, int ninst,
                             const float2* psi, const double* f, const double2* tw_nx,
                             float2* out_psi, float* out_rho, double* partials,
                             hipStream_t stream, int model = kModelQHD);
hipError_t launch_observe_1d(int n, const InstDev* inst, int ninst, const float2* psi,
                             const double* f, float2* out_psi, float* out_rho, double* partials,
                             hipStream_t stream);
// Sum the per-line partials of each instance in a fixed order -> results[3*i + c].
hipError_t launch_finalize(const double* partials, int lines_per_inst, int ninst, double* results,
                           hipStream_t stream);

// Potential / state upload helpers (user row-major <-> internal layout).
hipError_t launch_import_f(int ndim, int nx, int ny, const double* user, double* dst,
                           hipStream_t stream);
hipError_t launch_import_psi(int ndim, int nx, int ny, const float2* user, float2* dst,
                             hipStream_t stream);
hipError_t launch_fill_psi(float2* dst, long long count, float value, hipStream_t stream);
// steps_done = 0, mode = clean for every instance of a class
hipError_t launch_reset_inst(InstDev* inst, int ninst, hipStream_t stream);
// Lowest-index minimiser of f (user row-major layout) and the count of non-finite values:
// out_val[0], out_idx[0], out_idx[1].  Two launches: per-block partials into
// part_val / part_idx / part_bad (kArgminBlocks entries each), then their reduction.
constexpr int kArgminBlocks = 512;
hipError_t launch_argmin(const double* f, long long count, double* out_val, long long* out_idx, double* part_val,
                         long long* part_idx, long long* part_bad, hipStream_t stream);

// Size the launch of the pass kernels (blocks actually used for a class).
// 3-D pass with the line transforms as split-FP16 DFT products on the matrix cores
// (128^3 only): axis 0 = x-pass (F_x V F_x^{-1}), 1 = y-pass (dir -1 forward, +1
// inverse), 2 = z-pass (F_z^{-1} K F_z).  tables: FP16 [sign][re hi, re lo, im hi,
// im lo][128][128], sign 0 = e^{-2 pi i jk/128}, 1 = e^{+2 pi i jk/128}.
hipError_t launch_mfma_pass_3d(int axis, int dir, const InstDev* inst, int ninst, const int* nact, const void* tables,
                               float2* psi, const double* f, int s, long long max_steps, int grid_cap,
                               hipStream_t stream);

int pass_blocks_row_2d(int nx, int ny, int ninst, int grid_cap, int points_per_lane);
int pass_blocks_col_2d(int nx, int ny, int ninst, int grid_cap, int variant);

// spectrum kernels (qhd_spectrum_kernels.hip); v is a plain row-major (x fastest)
// complex64 vector of one nx x ny instance
hipError_t spec_lines(int axis, int sign, float2* v, int nx, int ny, const double2* tw, hipStream_t st);
hipError_t spec_kinetic(float2* v, int nx, int ny, double cx, double cy, double s, hipStream_t st);
hipError_t spec_finish(float2* out, const float2* w, const float2* v, const double* f, double b, int nx, int ny,
                       hipStream_t st);
hipError_t spec_multidot(const float2* V, long long n, int count, const float2* w, double* partials, int nblk,
                         hipStream_t st);
// (with `part`, groups x n FP64 pairs of scratch, long bases take the grouped two-kernel
// form; scale_dev: the scale read from device memory)
hipError_t spec_multiaxpy(float2* w, const float2* V, long long n, int count, const double* c, double scale,
                          hipStream_t st, const double* scale_dev = nullptr, double2* part = nullptr,
                          int groups = 1);
// device-side reductions of the multidot partials (block order, FP64): coefficients
// (optionally keeping the newest one), and a vector's norm with its reciprocal
hipError_t spec_coef(const double* partials, int count, int nblk, double* coef, double* keep, hipStream_t st);
hipError_t spec_norm(const double* partials, int nblk, double* keep, double* scale, hipStream_t st);
hipError_t spec_random(float2* v, long long n, unsigned long long seed, hipStream_t st);

}  // namespace qhd
