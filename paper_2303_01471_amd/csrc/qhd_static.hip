// Readouts of caller-owned states without any allocation (qhd_readouts_static).
//
// The readouts are those of qhd_observe: the norm sum |psi|^2, E[f] = sum f |psi|^2 /
// norm (App. B, the loss <f>), the success mass of the ball |x - x*| < r around the
// lowest-index grid minimiser x* of f (main text, fig. 2; Algorithm 1's position
// measurement), and x*, f(x*).  Here the states and potentials are the caller's
// (row-major, x fastest, instances one after another) and no plan is involved: the
// per-line partial results live in a file-scope device array, so the entry point never
// calls the allocator and can run inside a stream capture or a serving loop.
//
// Four launches, all on the caller's stream:
//   k_st_linemin   per mesh line: lowest-index minimum of f (finite values only)
//   k_st_argmin    per instance: x*, f(x*) from its lines' minima
//   k_st_sums      per mesh line: sum rho, sum f rho, sum of rho inside the ball (FP64)
//   k_st_finalize  per instance: fixed-order compensated sum of its lines' partials
// Every scratch entry a launch reads was written by an earlier launch of the same call,
// so nothing needs clearing between calls; calls that overlap on one GPU share the
// array and race.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdio>
#include <mutex>

#include "../../include/qhd.h"
#include "qhd_internal.h"

namespace qhd {
void set_error_message(const char* msg);
}

namespace {

constexpr long long kMaxLines = QHD_STATIC_MAX_LINES;
// line minima (value, index), line partial sums (3 per line), per instance x* and f(x*)
constexpr size_t kOffMinVal = 0;
constexpr size_t kOffMinIdx = kOffMinVal + sizeof(double) * kMaxLines;
constexpr size_t kOffSums = kOffMinIdx + sizeof(long long) * kMaxLines;
constexpr size_t kOffArg = kOffSums + sizeof(double) * 3 * kMaxLines;
constexpr size_t kOffFmin = kOffArg + sizeof(long long) * kMaxLines;
constexpr size_t kScratchBytes = kOffFmin + sizeof(double) * kMaxLines;

// The library's scratch memory for this entry point: one copy per GPU, held until the
// process ends.  Host code never passes `scratch` itself to a kernel (in host code the
// name is a stand-in, not a device address); it uses the per-device address obtained
// with hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char* g_scratch_dev[kMaxDevices] = {};

struct Geo {
  int nx, lines_per_inst;  // points per line (x), lines per instance (ny nz)
  int ny;                  // for (y, z) of a line
  long long points;        // per instance
  double h[3];             // mesh spacing per axis (0 for absent axes)
  double r2;               // success radius squared
};

__device__ __forceinline__ void min_pair(double& v, long long& i, double v2, long long i2) {
  if (v2 < v || (v2 == v && i2 < i)) {
    v = v2;
    i = i2;
  }
}

// one wavefront per mesh line, four per block, grid-stride
__global__ void __launch_bounds__(256) k_st_linemin(const double* __restrict__ f, long long nlines, Geo g,
                                                     double* __restrict__ minv, long long* __restrict__ mini) {
  const int lane = threadIdx.x & 63;
  for (long long L = (long long)blockIdx.x * 4 + (threadIdx.x >> 6); L < nlines; L += (long long)gridDim.x * 4) {
    const long long i = L / g.lines_per_inst, r = L - i * g.lines_per_inst;
    const double* __restrict__ line = f + i * g.points + r * g.nx;
    double bv = INFINITY;
    long long bi = LLONG_MAX;
    for (int x = lane; x < g.nx; x += 64) {
      const double v = line[x];
      if (isfinite(v)) min_pair(bv, bi, v, r * g.nx + x);
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double v2 = __shfl_xor(bv, o, 64);
      const long long i2 = __shfl_xor(bi, o, 64);
      min_pair(bv, bi, v2, i2);
    }
    if (lane == 0) {
      minv[L] = bv;
      mini[L] = bi;
    }
  }
}

// one block per instance
__global__ void __launch_bounds__(256) k_st_argmin(const double* __restrict__ minv, const long long* __restrict__ mini,
                                                    int lines_per_inst, long long* __restrict__ arg,
                                                    double* __restrict__ fmin) {
  __shared__ double sv[256];
  __shared__ long long si[256];
  const int i = blockIdx.x;
  double bv = INFINITY;
  long long bi = LLONG_MAX;
  for (int l = threadIdx.x; l < lines_per_inst; l += 256) {
    const long long L = (long long)i * lines_per_inst + l;
    min_pair(bv, bi, minv[L], mini[L]);
  }
  sv[threadIdx.x] = bv;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      double v = sv[threadIdx.x];
      long long id = si[threadIdx.x];
      min_pair(v, id, sv[threadIdx.x + o], si[threadIdx.x + o]);
      sv[threadIdx.x] = v;
      si[threadIdx.x] = id;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    arg[i] = si[0] == LLONG_MAX ? -1 : si[0];
    fmin[i] = sv[0];
  }
}

__device__ __forceinline__ bool st_in_ball(long long dxi, long long dyi, long long dzi, const Geo& g) {
  // the success test of the readouts, FP64 operations in a fixed order without contraction
  const double dx = __dmul_rn((double)dxi, g.h[0]);
  const double dy = __dmul_rn((double)dyi, g.h[1]);
  const double dz = __dmul_rn((double)dzi, g.h[2]);
  return __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz)) < g.r2;
}

__global__ void __launch_bounds__(256) k_st_sums(const float2* __restrict__ psi, const double* __restrict__ f,
                                                  long long nlines, Geo g, const long long* __restrict__ arg,
                                                  double* __restrict__ sums) {
  const int lane = threadIdx.x & 63;
  for (long long L = (long long)blockIdx.x * 4 + (threadIdx.x >> 6); L < nlines; L += (long long)gridDim.x * 4) {
    const long long i = L / g.lines_per_inst, r = L - i * g.lines_per_inst;
    const long long off = i * g.points + r * g.nx;
    const long long a = arg[i];
    // x* as (x, y, z); an instance without a finite f value has no success ball
    const long long as = a < 0 ? 0 : a;
    const long long xs = as % g.nx, rs = as / g.nx;
    const long long ys = rs % g.ny, zs = rs / g.ny;
    const long long yy = r % g.ny, zz = r / g.ny;
    double sr = 0.0, sf = 0.0, sm = 0.0;
    for (int x = lane; x < g.nx; x += 64) {
      const float2 v = psi[off + x];
      const double rho = (double)v.x * v.x + (double)v.y * v.y;
      sr += rho;
      sf += f[off + x] * rho;
      if (a >= 0 && st_in_ball(x - xs, yy - ys, zz - zs, g)) sm += rho;
    }
    for (int o = 32; o > 0; o >>= 1) {
      sr += __shfl_xor(sr, o, 64);
      sf += __shfl_xor(sf, o, 64);
      sm += __shfl_xor(sm, o, 64);
    }
    if (lane == 0) {
      sums[3 * L + 0] = sr;
      sums[3 * L + 1] = sf;
      sums[3 * L + 2] = sm;
    }
  }
}

__global__ void k_st_finalize(const double* __restrict__ sums, int lines_per_inst, int count,
                              const long long* __restrict__ arg, const double* __restrict__ fmin,
                              qhd_readout* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  double tot[3];
  for (int c = 0; c < 3; ++c) {
    double s = 0.0, comp = 0.0;
    for (int l = 0; l < lines_per_inst; ++l) {
      const double v = sums[3 * ((long long)i * lines_per_inst + l) + c];
      const double t = s + v;
      comp += (fabs(s) >= fabs(v)) ? ((s - t) + v) : ((v - t) + s);
      s = t;
    }
    tot[c] = s + comp;
  }
  qhd_readout o;
  o.norm = tot[0];
  o.e_f = tot[1] / tot[0];
  o.success_mass = tot[2] / tot[0];
  o.f_min = fmin[i];
  o.argmin_index = arg[i];
  out[i] = o;
}

qhd_status st_fail(qhd_status st, const char* msg) {
  qhd::set_error_message(msg);
  return st;
}

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

}  // namespace

extern "C" qhd_status qhd_readouts_static(int32_t ndim, const int32_t* n, const double* lo, const double* hi,
                                          double success_radius, int32_t count, const float* psi_dev,
                                          const double* f_dev, qhd_readout* out_dev, void* stream_v) {
  qhd::set_error_message("");
  char msg[256];
  if (ndim < 1 || ndim > 3) return st_fail(QHD_EINVAL, "qhd_readouts_static: ndim must be 1, 2 or 3");
  if (!n || !lo || !hi) return st_fail(QHD_EINVAL, "qhd_readouts_static: n, lo and hi must not be NULL");
  if (!psi_dev || !f_dev || !out_dev)
    return st_fail(QHD_EINVAL, "qhd_readouts_static: psi_dev, f_dev and out_dev must not be NULL");
  if (count < 1) return st_fail(QHD_EINVAL, "qhd_readouts_static: count must be >= 1");
  if (!(success_radius > 0.0) || !std::isfinite(success_radius))
    return st_fail(QHD_EINVAL, "qhd_readouts_static: success_radius must be finite and > 0");
  Geo g{};
  long long lines_per_inst = 1;
  for (int a = 0; a < ndim; ++a) {
    if (!pow2(n[a]) || n[a] < 8 || n[a] > 1024) {
      snprintf(msg, sizeof msg, "qhd_readouts_static: n[%d]=%d must be a power of two in [8, 1024]", a, n[a]);
      return st_fail(QHD_EINVAL, msg);
    }
    if (!std::isfinite(lo[a]) || !std::isfinite(hi[a]) || !(hi[a] > lo[a])) {
      snprintf(msg, sizeof msg, "qhd_readouts_static: box axis %d needs finite lo < hi", a);
      return st_fail(QHD_EINVAL, msg);
    }
    g.h[a] = (hi[a] - lo[a]) / (double)n[a];
    if (a > 0) lines_per_inst *= n[a];
  }
  const long long nlines = lines_per_inst * (long long)count;
  if (nlines > kMaxLines) {
    snprintf(msg, sizeof msg,
             "qhd_readouts_static: %lld mesh lines (count x points / n[0]) exceed the static scratch of %lld lines",
             nlines, kMaxLines);
    return st_fail(QHD_EINVAL, msg);
  }
  g.nx = n[0];
  g.ny = ndim >= 2 ? n[1] : 1;
  g.lines_per_inst = (int)lines_per_inst;
  g.points = lines_per_inst * n[0];
  g.r2 = success_radius * success_radius;

  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    snprintf(msg, sizeof msg, "qhd_readouts_static: hipGetDevice: %s", hipGetErrorString(e));
    return st_fail(QHD_EDEVICE, msg);
  }
  unsigned char* base = nullptr;
  {
    // the array's address on this device, looked up once per device with it current
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch_dev[dev]) {
      void* p = nullptr;
      e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p) {
        snprintf(msg, sizeof msg, "qhd_readouts_static: hipGetSymbolAddress: %s", hipGetErrorString(e));
        return st_fail(QHD_EDEVICE, msg);
      }
      g_scratch_dev[dev] = static_cast<unsigned char*>(p);
    }
    base = g_scratch_dev[dev];
  }
  double* minv = reinterpret_cast<double*>(base + kOffMinVal);
  long long* mini = reinterpret_cast<long long*>(base + kOffMinIdx);
  double* sums = reinterpret_cast<double*>(base + kOffSums);
  long long* arg = reinterpret_cast<long long*>(base + kOffArg);
  double* fmin = reinterpret_cast<double*>(base + kOffFmin);
  hipStream_t st = (hipStream_t)stream_v;
  const int blocks = (int)std::min<long long>((nlines + 3) / 4, 4096);
  const float2* psi = reinterpret_cast<const float2*>(psi_dev);
  hipLaunchKernelGGL(k_st_linemin, dim3(blocks), dim3(256), 0, st, f_dev, nlines, g, minv, mini);
  hipLaunchKernelGGL(k_st_argmin, dim3(count), dim3(256), 0, st, minv, mini, g.lines_per_inst, arg, fmin);
  hipLaunchKernelGGL(k_st_sums, dim3(blocks), dim3(256), 0, st, psi, f_dev, nlines, g, arg, sums);
  hipLaunchKernelGGL(k_st_finalize, dim3((count + 63) / 64), dim3(64), 0, st, sums, g.lines_per_inst, count, arg,
                     fmin, out_dev);
  e = hipGetLastError();
  if (e != hipSuccess) {
    snprintf(msg, sizeof msg, "qhd_readouts_static: launch: %s", hipGetErrorString(e));
    return st_fail(QHD_EDEVICE, msg);
  }
  return QHD_OK;
}
