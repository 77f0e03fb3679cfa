// Spectral neural-operator surrogate: parameters, buffers, forward, backward,
// Adam, and the C ABI of include/qhd_sno.h.  The model is defined in that
// header; every contraction below is a batched GEMM (sno_gemm.hip).
//
// Activation layouts (element type T = BF16 or FP32):
//   h      [b][y][x][c]            channel-last, c fastest
//   T1/U   [b][y][ri][kx][c]       after the x-contraction (ri: 0 real, 1 imaginary)
//   H/G    [b][ri][j][kx][c]       truncated spectrum, j indexes ky in [0,M) U [-M,0)
// so that each stage of the separable truncated DFT, the per-mode mixing and the
// 1x1 maps are plain strided batched GEMMs.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <string>
#include <vector>

#include "../../include/qhd_sno.h"
#include "sno_internal.h"

namespace qhd {
void set_error_message(const char* msg);
}

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

#define SNO_TRY(expr)                                                                             \
  do {                                                                                            \
    hipError_t e_ = (expr);                                                                       \
    if (e_ != hipSuccess)                                                                         \
      return sfail(e_ == hipErrorOutOfMemory ? QHD_ENOMEM : QHD_EDEVICE, "%s: %s", #expr,           \
                   hipGetErrorString(e_));                                                        \
  } while (0)

uint64_t splitmix(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
double uniform01(uint64_t& s) { return (double)(splitmix(s) >> 11) * (1.0 / 9007199254740992.0); }

}  // namespace

struct qhd_sno_s {
  int S = 0, C = 0, M = 0, L = 0, Bmax = 0;
  bool bf16 = true, train = false;
  int device = 0;
  long long npix = 0;
  int nmodes = 0;  // 2M * M
  size_t es = 2;   // bytes per activation element
  long long nparams = 0;
  long long o_wl = 0, o_bl = 0, o_wp = 0, o_bp = 0;
  std::vector<long long> o_rr, o_ri, o_w, o_b;
  float *params = nullptr, *grad = nullptr, *am = nullptr, *av = nullptr;
  void* pt = nullptr;  // T copy of the parameters (GEMM operands)
  int adam_t = 0;
  bool have_grad = false;
  void *Fx = nullptr, *Fxw = nullptr, *Fy1 = nullptr, *Fy2 = nullptr;
  void *Gy = nullptr, *Gxw = nullptr, *Gx = nullptr;  // Gy: rows 2y, 2y+1 = GyR, GyI rows y
  void* in = nullptr;
  std::vector<void*> h;
  std::vector<float*> z;
  std::vector<void*> Hs;
  void *T1 = nullptr, *G = nullptr, *dH = nullptr, *dz = nullptr;
  float *rho_hat = nullptr, *dq = nullptr, *dh = nullptr, *partials = nullptr;
  double* loss_dev = nullptr;
  std::vector<void*> allocs;
  std::vector<std::pair<const char*, size_t>> spans;  // every buffer the library owns
  bool dry = false;  // shape validation only: no device memory, no launches
  std::vector<float> dry_params;
  unsigned long long fake_next = 1ull << 44;
  int nsplit = 256;
  long long spec = 0;  // elements of one sample's truncated spectrum: 4M * M * C

  void* T(const void* base, long long elems) const { return (char*)base + elems * (long long)es; }
};

namespace {

hipError_t alloc(qhd_sno_s* m, void** p, size_t bytes) {
  bytes = bytes < 16 ? 16 : bytes;
  if (m->dry) {
    // distinct, never dereferenced addresses with a gap after each buffer, so
    // that the bounds checks below see overruns as they would on the device
    *p = (void*)m->fake_next;
    m->fake_next += ((bytes + 255) & ~255ull) + 65536;
  } else {
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) return e;
    m->allocs.push_back(*p);
  }
  m->spans.push_back({(const char*)*p, bytes});
  return hipSuccess;
}

void release(qhd_sno_s* m) {
  if (!m) return;
  if (!m->dry) {
    (void)hipSetDevice(m->device);
    (void)hipDeviceSynchronize();
    for (void* p : m->allocs) (void)hipFree(p);
  }
  delete m;
}

// a device call, skipped when only validating shapes
#define DEV(m, expr) ((m)->dry ? hipSuccess : (expr))

#define ST_TRY(expr)               \
  do {                             \
    qhd_status s_ = (expr);        \
    if (s_ != QHD_OK) return s_;   \
  } while (0)

// every byte in [p, p + bytes) lies inside one buffer of the library
bool inside(const qhd_sno_s* m, const void* p, long long bytes) {
  const char* c = (const char*)p;
  for (const auto& sp : m->spans)
    if (c >= sp.first && c + bytes <= sp.first + sp.second) return true;
  return false;
}

qhd_status check(const qhd_sno_s* m, const void* p, long long bytes, const char* what) {
  if (bytes <= 0 || inside(m, p, bytes)) return QHD_OK;
  return sfail(QHD_EDEVICE, "internal bounds check failed: %s (%lld bytes)", what, bytes);
}

qhd_status launch(const qhd_sno_s* m, hipError_t e, const char* what) {
  (void)m;
  if (e != hipSuccess) return sfail(QHD_EDEVICE, "%s: %s", what, hipGetErrorString(e));
  return QHD_OK;
}

// C[b] = alpha op(A[b]) op(B[b]) (+ scale2 op(A2[b]) op(B2[b])) + beta C[b]; every operand
// is a buffer of the library and is checked against it before the launch
qhd_status gemm(const qhd_sno_s* m, int M, int N, int K, int batch, const void* A, int lda, long long sA,
                bool tA, const void* B, int ldb, long long sB, bool tB, void* C, int ldc, long long sC,
                bool c_is_t, float alpha, float beta, hipStream_t st, const void* A2 = nullptr,
                const void* B2 = nullptr, float scale2 = 1.0f) {
  if (M <= 0 || N <= 0 || K <= 0 || batch <= 0) return QHD_OK;
  const long long es = (long long)m->es, ces = (m->bf16 && c_is_t) ? 2 : 4;
  // one past the largest element index each operand touches
  const long long ea = (long long)(batch - 1) * sA + (tA ? (long long)(K - 1) * lda + M : (long long)(M - 1) * lda + K);
  const long long eb = (long long)(batch - 1) * sB + (tB ? (long long)(N - 1) * ldb + K : (long long)(K - 1) * ldb + N);
  const long long ec = (long long)(batch - 1) * sC + (long long)(M - 1) * ldc + N;
  ST_TRY(check(m, A, ea * es, "gemm A"));
  ST_TRY(check(m, B, eb * es, "gemm B"));
  ST_TRY(check(m, C, ec * ces, "gemm C"));
  if (A2) ST_TRY(check(m, A2, ea * es, "gemm A2"));
  if (B2) ST_TRY(check(m, B2, eb * es, "gemm B2"));
  GemmArgs g;
  g.M = M;
  g.N = N;
  g.K = K;
  g.batch = batch;
  g.A = A;
  g.lda = lda;
  g.sA = sA;
  g.transA = tA;
  g.B = B;
  g.ldb = ldb;
  g.sB = sB;
  g.transB = tB;
  g.C = C;
  g.ldc = ldc;
  g.sC = sC;
  g.alpha = alpha;
  g.beta = beta;
  g.A2 = A2;
  g.B2 = B2;
  g.scale2 = scale2;
  g.in_bf16 = m->bf16;
  g.out_bf16 = m->bf16 && c_is_t;
  return launch(m, DEV(m, launch_gemm(g, st)), "gemm launch");
}

// truncated forward DFT of X [B][S][S][C] (T) into H [B][4M][M][C] (T); fx = Fx or Fxw
// (x_done: T1 already holds the x-contraction of X)
qhd_status fwd_dft(qhd_sno_s* m, const void* X, const void* fx, void* H, int B, hipStream_t st,
                   bool x_done = false) {
  const int S = m->S, C = m->C, M = m->M;
  // x-contraction, per (b, y): T1 (2M x C) = fx (2M x S) . X_by (S x C)
  if (x_done) {
  } else if (m->bf16 && C == 32 && M == 16 && S % 16 == 0) {
    ST_TRY(check(m, X, (long long)B * S * S * C * m->es, "transform input"));
    ST_TRY(check(m, m->T1, (long long)B * S * 2 * M * C * m->es, "x-contraction"));
    ST_TRY(launch(m, DEV(m, sno_dft_x32(fx, X, S, (long long)B * S, m->T1, st)), "x-contraction"));
  } else {
    ST_TRY(gemm(m, 2 * M, C, S, B * S, fx, S, 0, false, X, C, (long long)S * C, false, m->T1, C, 2LL * M * C,
                true, 1.0f, 0.0f, st));
  }
  // y-contraction, per b: [Hr; Hi] (4M x MC) = Fy1 (4M x S) . Tr_b + Fy2 (4M x S) . Ti_b
  if (m->bf16 && C == 32 && M == 16 && S % 16 == 0 && S <= 256) {
    ST_TRY(check(m, H, (long long)B * m->spec * m->es, "spectrum"));
    return launch(m, DEV(m, sno_fwd_y32(m->Fy1, m->Fy2, m->T1, B, S, H, m->spec, st)), "y-contraction");
  }
  return gemm(m, 4 * M, M * C, S, B, m->Fy1, S, 0, false, m->T1, 2 * M * C, (long long)S * 2 * M * C,
              false, H, M * C, m->spec, true, 1.0f, 0.0f, st, m->Fy2, m->T(m->T1, (long long)M * C), 1.0f);
}

// truncated inverse (c2r) of G [B][4M][M][C] into out FP32 [B][S][S][C]; gx = Gxw or Gx
// y-contraction of the truncated inverse, per b: Ur (S x MC) = GyR (S x 4M) . G_b ; Ui = GyI . G_b
// -> U in the T1 buffer, [B][S][2M][C]. One product: with the rows of GyR and GyI interleaved
// (Gy, 2S x 4M), output row 2y is Ur's row y and row 2y+1 is Ui's, which is U's layout at a
// row stride of MC
qhd_status inv_dft_y(qhd_sno_s* m, const void* Gsp, int B, hipStream_t st) {
  const int S = m->S, C = m->C, M = m->M;
  if (m->bf16 && C == 32 && M == 16 && S % 16 == 0) {
    ST_TRY(check(m, Gsp, (long long)B * m->spec * m->es, "inverse input"));
    ST_TRY(check(m, m->T1, (long long)B * S * 2 * M * C * m->es, "inverse y-contraction"));
    return launch(m, DEV(m, sno_inv_y32(m->Gy, Gsp, m->spec, B, S, m->T1, st)), "inverse y-contraction");
  }
  return gemm(m, 2 * S, M * C, 4 * M, B, m->Gy, 4 * M, 0, false, Gsp, M * C, m->spec, false, m->T1, M * C,
              (long long)S * 2 * M * C, true, 1.0f, 0.0f, st);
}

qhd_status inv_dft(qhd_sno_s* m, const void* Gsp, const void* gx, float* out, int B, float beta,
                   hipStream_t st) {
  const int S = m->S, C = m->C, M = m->M;
  ST_TRY(inv_dft_y(m, Gsp, B, st));
  // x-contraction, per (b, y): out_by (S x C) = gx (S x 2M) . U_by (2M x C)
  return gemm(m, S, C, 2 * M, B * S, gx, 2 * M, 0, false, m->T1, C, 2LL * M * C, false, out, C,
              (long long)S * C, false, 1.0f, beta, st);
}

// per-mode complex mixing G = R H, R = Rr + i Ri ([mode][out][in])
qhd_status mix(qhd_sno_s* m, const void* H, void* Gout, int l, int B, hipStream_t st) {
  const int C = m->C, nm = m->nmodes;
  const long long half = (long long)nm * C;  // offset of the imaginary block in a sample
  const void* Rr = m->T(m->pt, m->o_rr[l]);
  const void* Ri = m->T(m->pt, m->o_ri[l]);
  const int ld = (int)m->spec;
  if (m->bf16 && C == 32) {
    ST_TRY(check(m, H, (long long)B * m->spec * m->es, "mixing input"));
    ST_TRY(check(m, Gout, (long long)B * m->spec * m->es, "mixing output"));
    return launch(m, DEV(m, sno_mix32(H, Rr, Ri, nm, m->spec, B, Gout, st)), "mixing");
  }
  // Gr = Hr Rr^T - Hi Ri^T
  ST_TRY(gemm(m, B, C, C, nm, H, ld, C, false, Rr, C, (long long)C * C, true, Gout, ld, C, true, 1.0f, 0.0f,
              st, m->T(H, half), Ri, -1.0f));
  // Gi = Hr Ri^T + Hi Rr^T
  return gemm(m, B, C, C, nm, H, ld, C, false, Ri, C, (long long)C * C, true, m->T(Gout, half), ld, C, true,
              1.0f, 0.0f, st, m->T(H, half), Rr, 1.0f);
}

// DFT matrices (FP64 on the host, stored as T)
qhd_status build_dft(qhd_sno_s* m) {
  const int S = m->S, M = m->M;
  const double tp = 2.0 * M_PI / S;
  auto ky = [&](int j) { return j < M ? j : j - 2 * M; };
  auto wk = [&](int kx) { return kx == 0 ? 1.0 : 2.0; };
  std::vector<float> fx(2 * M * S), fxw(2 * M * S), fy1(4 * M * S), fy2(4 * M * S);
  std::vector<float> gy(2 * S * 4 * M), gxw(S * 2 * M), gx(S * 2 * M);
  for (int kx = 0; kx < M; ++kx)
    for (int x = 0; x < S; ++x) {
      const double a = tp * kx * x;
      const double sc = wk(kx) / ((double)S * S);
      fx[kx * S + x] = (float)cos(a);
      fx[(M + kx) * S + x] = (float)-sin(a);
      fxw[kx * S + x] = (float)(sc * cos(a));
      fxw[(M + kx) * S + x] = (float)(-sc * sin(a));
      gx[x * 2 * M + kx] = (float)cos(a);
      gx[x * 2 * M + M + kx] = (float)-sin(a);
      gxw[x * 2 * M + kx] = (float)(sc * cos(a));
      gxw[x * 2 * M + M + kx] = (float)(-sc * sin(a));
    }
  for (int j = 0; j < 2 * M; ++j)
    for (int y = 0; y < S; ++y) {
      const double a = tp * ky(j) * y;
      const double c = cos(a), s = sin(a);  // Fy = e^{-ia} = c - i s ; Gy = e^{+ia} = c + i s
      // [Hr; Hi] = [Fyr; Fyi] Tr + [-Fyi; Fyr] Ti with Fyr = c, Fyi = -s
      fy1[j * S + y] = (float)c;
      fy1[(2 * M + j) * S + y] = (float)-s;
      fy2[j * S + y] = (float)s;
      fy2[(2 * M + j) * S + y] = (float)c;
      // Ur = [Gyr | -Gyi] [Gr; Gi], Ui = [Gyi | Gyr] [Gr; Gi] with Gyr = c, Gyi = s
      gy[2 * y * 4 * M + j] = (float)c;
      gy[2 * y * 4 * M + 2 * M + j] = (float)-s;
      gy[(2 * y + 1) * 4 * M + j] = (float)s;
      gy[(2 * y + 1) * 4 * M + 2 * M + j] = (float)c;
    }
  struct Item {
    std::vector<float>* v;
    void** dst;
  } items[] = {{&fx, &m->Fx}, {&fxw, &m->Fxw}, {&fy1, &m->Fy1}, {&fy2, &m->Fy2},
               {&gy, &m->Gy}, {&gxw, &m->Gxw}, {&gx, &m->Gx}};
  for (auto& it : items)
    if (alloc(m, it.dst, it.v->size() * m->es) != hipSuccess) return sfail(QHD_ENOMEM, "DFT matrix allocation");
  if (m->dry) return QHD_OK;
  float* tmp = nullptr;
  SNO_TRY(hipMalloc(&tmp, (size_t)2 * S * 4 * M * sizeof(float)));
  qhd_status st = QHD_OK;
  for (auto& it : items) {
    hipError_t e = hipMemcpy(tmp, it.v->data(), it.v->size() * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = sno_cast(tmp, *it.dst, (long long)it.v->size(), m->bf16, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
      st = sfail(QHD_EDEVICE, "DFT matrix upload: %s", hipGetErrorString(e));
      break;
    }
  }
  (void)hipFree(tmp);
  return st;
}

qhd_status forward(qhd_sno_s* m, const double* f, int B, hipStream_t st) {
  const int C = m->C;
  const long long npix = m->npix, rows = (long long)B * npix;
  const long long es = (long long)m->es;
  ST_TRY(check(m, m->h[0], rows * C * es, "h0"));
  if (!m->train && m->bf16 && C == 32) {
    // inference: features and lift in one pass (the features are kept only for the lift's gradient)
    ST_TRY(launch(m, DEV(m, sno_prep_lift32(f, B, m->S, m->T(m->pt, m->o_wl), m->params + m->o_bl, m->h[0], st)),
                  "features+lift"));
  } else {
    ST_TRY(check(m, m->in, rows * 3 * es, "features"));
    ST_TRY(launch(m, DEV(m, sno_prep_input(f, B, m->S, m->in, m->bf16, st)), "features launch"));
    // lift: z = x0 Wl^T (per sample: npix x C), then h0 = z + bl
    float* z0 = m->z[0];
    ST_TRY(gemm(m, (int)npix, C, 3, B, m->in, 3, npix * 3, false, m->T(m->pt, m->o_wl), 3, 0, true, z0, C,
                npix * C, false, 1.0f, 0.0f, st));
    // (the biased pre-activations are kept only for the backward pass of training)
    ST_TRY(launch(m, DEV(m, sno_bias_act(z0, m->params + m->o_bl, rows, C, m->h[0], m->bf16, 0, st, m->train)),
                  "lift bias"));
  }
  // inference at width 32 with 16 modes: a layer's inverse x-contraction, 1x1 map, bias and GELU
  // are one pass, which also forms the next layer's forward x-contraction
  const bool fused = !m->train && m->bf16 && C == 32 && m->M == 16 && m->S % 32 == 0;
  for (int l = 0; l < m->L; ++l) {
    void* hin = m->train ? m->h[l] : m->h[l % 2];
    void* hout = m->train ? m->h[l + 1] : m->h[(l + 1) % 2];
    float* zl = m->train ? m->z[l] : m->z[0];
    void* Hl = m->train ? m->Hs[l] : m->Hs[0];
    ST_TRY(fwd_dft(m, hin, m->Fx, Hl, B, st, fused && l > 0));
    ST_TRY(mix(m, Hl, m->G, l, B, st));
    ST_TRY(check(m, hout, rows * C * es, "layer output"));
    if (fused) {
      ST_TRY(inv_dft_y(m, m->G, B, st));
      ST_TRY(check(m, m->T1, (long long)B * m->S * 2 * m->M * C * es, "inverse y-contraction"));
      const bool next = l + 1 < m->L;
      // the last layer projects its outputs to the logits (in the density buffer) in the same pass
      ST_TRY(check(m, m->rho_hat, rows * 4, "logits"));
      ST_TRY(launch(m, DEV(m, sno_spectral_pointwise32(m->Gxw, m->T1, hin, m->T(m->pt, m->o_w[l]),
                                                       m->params + m->o_b[l], m->S, (long long)B * m->S, hout, 1,
                                                       next ? m->Fx : nullptr, m->T1, m->params + m->o_wp,
                                                       m->params + m->o_bp, next ? nullptr : m->rho_hat, st)),
                    "inverse+1x1 map+GELU"));
      continue;
    }
    ST_TRY(inv_dft(m, m->G, m->Gxw, zl, B, 0.0f, st));
    ST_TRY(check(m, zl, rows * C * 4, "layer pre-activation"));
    if (!m->train && m->bf16 && C == 32) {
      // inference: the 1x1 map, bias and GELU in one pass (the pre-activation is not kept)
      ST_TRY(launch(m, DEV(m, sno_pointwise32(hin, m->T(m->pt, m->o_w[l]), zl, m->params + m->o_b[l], rows, hout,
                                              1, st)), "1x1 map+GELU"));
    } else {
      // z += h W^T
      ST_TRY(gemm(m, (int)npix, C, C, B, hin, C, npix * C, false, m->T(m->pt, m->o_w[l]), C, 0, true, zl, C,
                  npix * C, false, 1.0f, 1.0f, st));
      ST_TRY(launch(m, DEV(m, sno_bias_act(zl, m->params + m->o_b[l], rows, C, hout, m->bf16, 1, st, m->train)),
                    "bias+GELU"));
    }
  }
  ST_TRY(check(m, m->rho_hat, rows * 4, "density"));
  if (fused) return launch(m, DEV(m, sno_softmax_rows(m->rho_hat, B, (int)npix, st)), "softmax");
  void* hL = m->train ? m->h[m->L] : m->h[m->L % 2];
  ST_TRY(launch(m, DEV(m, sno_project_softmax(hL, m->params + m->o_wp, m->params + m->o_bp, B, (int)npix, C,
                                              m->bf16, m->rho_hat, st)), "projection"));
  return QHD_OK;
}

// gradient of a 1x1 map: out (a x b) = sum over rows of dzp^T (rows x a) x (rows x b), split over
// nsplit row chunks into partials, then reduced in FP64
qhd_status splitk(qhd_sno_s* m, const void* dzp, int a, const void* x, int b, long long rows, float* out,
                  hipStream_t st) {
  const int ns = m->nsplit;
  const long long chunk = rows / ns;
  ST_TRY(gemm(m, a, b, (int)chunk, ns, dzp, a, chunk * a, true, x, b, chunk * b, false, m->partials, b,
              (long long)a * b, false, 1.0f, 0.0f, st));
  ST_TRY(check(m, out, (long long)a * b * 4, "split-K output"));
  return launch(m, DEV(m, sno_reduce_partials(m->partials, ns, a * b, out, false, st)), "split-K reduce");
}

qhd_status backward(qhd_sno_s* m, const float* target, int B, hipStream_t st) {
  const int C = m->C, nm = m->nmodes;
  const long long npix = m->npix, rows = (long long)B * npix;
  const long long half = (long long)nm * C;
  const int ld = (int)m->spec;
  const int nparts = 512;
  const long long es = (long long)m->es;
  ST_TRY(check(m, m->dq, rows * 4, "dq"));
  ST_TRY(launch(m, DEV(m, sno_loss_grad(m->rho_hat, target, B, (int)npix, m->dq, m->loss_dev, st)), "loss"));
  ST_TRY(check(m, m->dh, rows * C * 4, "dh"));
  ST_TRY(check(m, m->partials, (long long)nparts * (C + 1) * 4, "partials"));
  ST_TRY(launch(m, DEV(m, sno_project_backward(m->dq, m->h[m->L], m->params + m->o_wp, B, (int)npix, C, m->bf16,
                                               m->dh, m->partials, nparts, st)), "projection backward"));
  ST_TRY(launch(m, DEV(m, sno_reduce_partials(m->partials, nparts, C + 1, m->grad + m->o_wp, false, st)),
                "projection reduce"));
  for (int l = m->L - 1; l >= 0; --l) {
    ST_TRY(check(m, m->dz, rows * C * es, "dz"));
    ST_TRY(launch(m, DEV(m, sno_gelu_backward(m->dh, m->z[l], rows, C, m->dz, m->bf16, m->partials, nparts, st)),
                  "GELU backward"));
    ST_TRY(launch(m, DEV(m, sno_reduce_partials(m->partials, nparts, C, m->grad + m->o_b[l], false, st)),
                  "bias reduce"));
    ST_TRY(splitk(m, m->dz, C, m->h[l], C, rows, m->grad + m->o_w[l], st));
    // dG = (w / S^2) F dz  (the adjoint of the weighted inverse)
    ST_TRY(fwd_dft(m, m->dz, m->Fxw, m->G, B, st));
    const void* Hl = m->Hs[l];
    // dRr = dGr^T Hr + dGi^T Hi ; dRi = dGi^T Hr - dGr^T Hi   (summed over the batch)
    ST_TRY(gemm(m, C, C, B, nm, m->G, ld, C, true, Hl, ld, C, false, m->grad + m->o_rr[l], C, (long long)C * C,
                false, 1.0f, 0.0f, st, m->T(m->G, half), m->T(Hl, half), 1.0f));
    ST_TRY(gemm(m, C, C, B, nm, m->T(m->G, half), ld, C, true, Hl, ld, C, false, m->grad + m->o_ri[l], C,
                (long long)C * C, false, 1.0f, 0.0f, st, m->G, m->T(Hl, half), -1.0f));
    // dH = R^H dG:  dHr = dGr Rr + dGi Ri ; dHi = dGi Rr - dGr Ri
    const void* Rr = m->T(m->pt, m->o_rr[l]);
    const void* Ri = m->T(m->pt, m->o_ri[l]);
    ST_TRY(gemm(m, B, C, C, nm, m->G, ld, C, false, Rr, C, (long long)C * C, false, m->dH, ld, C, true, 1.0f,
                0.0f, st, m->T(m->G, half), Ri, 1.0f));
    ST_TRY(gemm(m, B, C, C, nm, m->T(m->G, half), ld, C, false, Rr, C, (long long)C * C, false,
                m->T(m->dH, half), ld, C, true, 1.0f, 0.0f, st, m->G, Ri, -1.0f));
    // dh = Re(F^H dH) + dz W
    ST_TRY(inv_dft(m, m->dH, m->Gx, m->dh, B, 0.0f, st));
    ST_TRY(gemm(m, (int)npix, C, C, B, m->dz, C, npix * C, false, m->T(m->pt, m->o_w[l]), C, 0, false, m->dh, C,
                npix * C, false, 1.0f, 1.0f, st));
  }
  // lift: dbl = sum dh ; dWl = dh^T x0
  ST_TRY(launch(m, DEV(m, sno_colsum(m->dh, false, rows, C, m->partials, nparts, st)), "lift bias gradient"));
  ST_TRY(launch(m, DEV(m, sno_reduce_partials(m->partials, nparts, C, m->grad + m->o_bl, false, st)),
                "lift bias reduce"));
  ST_TRY(launch(m, DEV(m, sno_cast(m->dh, m->dz, rows * C, m->bf16, st)), "cast"));
  return splitk(m, m->dz, C, m->in, 3, rows, m->grad + m->o_wl, st);
}

}  // namespace

extern "C" {

qhd_status qhd_sno_create(const qhd_sno_desc* d, qhd_sno* out) {
  set_error_message("");
  if (!out || !d) return sfail(QHD_EINVAL, "desc and out must not be NULL");
  *out = nullptr;
  const int S = d->grid, C = d->width, M = d->modes, L = d->layers;
  if (S < 32 || S > 256 || (S & (S - 1))) return sfail(QHD_EINVAL, "grid %d must be a power of two in [32, 256]", S);
  if (C != 8 && C != 16 && C != 32 && C != 64) return sfail(QHD_EINVAL, "width %d must be 8, 16, 32 or 64", C);
  if (M < 1 || M > S / 2) return sfail(QHD_EINVAL, "modes %d must be in [1, grid/2]", M);
  if (L < 1 || L > 8) return sfail(QHD_EINVAL, "layers %d must be in [1, 8]", L);
  if (d->max_batch < 1) return sfail(QHD_EINVAL, "max_batch must be >= 1");
  if (d->precision != QHD_SNO_BF16 && d->precision != QHD_SNO_FP32)
    return sfail(QHD_EINVAL, "unknown precision %d", d->precision);
  qhd_sno_s* m = new qhd_sno_s();
  m->S = S;
  m->C = C;
  m->M = M;
  m->L = L;
  m->Bmax = d->max_batch;
  m->bf16 = d->precision == QHD_SNO_BF16;
  m->train = d->train != 0;
  m->es = m->bf16 ? 2 : 4;
  m->npix = (long long)S * S;
  m->nmodes = 2 * M * M;
  m->spec = 4LL * M * M * C;
  {
    // host-only validation of every launch's extents against the buffers, with no
    // device: QHD_SNO_VALIDATE_ONLY=1 (used by the CPU tests)
    const char* v = getenv("QHD_SNO_VALIDATE_ONLY");
    m->dry = v && v[0] == '1';
  }
  if (!m->dry && hipGetDevice(&m->device) != hipSuccess) {
    delete m;
    return sfail(QHD_EDEVICE, "hipGetDevice failed");
  }
  // parameter layout
  long long o = 0;
  m->o_wl = o;
  o += (long long)C * 3;
  m->o_bl = o;
  o += C;
  for (int l = 0; l < L; ++l) {
    m->o_rr.push_back(o);
    o += (long long)m->nmodes * C * C;
    m->o_ri.push_back(o);
    o += (long long)m->nmodes * C * C;
    m->o_w.push_back(o);
    o += (long long)C * C;
    m->o_b.push_back(o);
    o += C;
  }
  m->o_wp = o;
  o += C;
  m->o_bp = o;
  o += 1;
  m->nparams = o;
  // deterministic initialisation
  std::vector<float> p(o);
  uint64_t s = d->seed ^ 0x5DEECE66Dull;
  auto fill_u = [&](long long off, long long n, double bound) {
    for (long long k = 0; k < n; ++k) p[off + k] = (float)((2.0 * uniform01(s) - 1.0) * bound);
  };
  fill_u(m->o_wl, (long long)C * 3, 1.0 / sqrt(3.0));
  fill_u(m->o_bl, C, 1.0 / sqrt(3.0));
  for (int l = 0; l < L; ++l) {
    for (long long k = 0; k < 2LL * m->nmodes * C * C; ++k) p[m->o_rr[l] + k] = (float)(uniform01(s) / (C * C));
    fill_u(m->o_w[l], (long long)C * C, 1.0 / sqrt((double)C));
    fill_u(m->o_b[l], C, 1.0 / sqrt((double)C));
  }
  fill_u(m->o_wp, C, 1.0 / sqrt((double)C));
  fill_u(m->o_bp, 1, 1.0 / sqrt((double)C));

  const long long Bm = m->Bmax, rows = Bm * m->npix;
  const size_t es = m->es;
  hipError_t e = hipSuccess;
  auto A = [&](void** ptr, size_t bytes) {
    if (e == hipSuccess) e = alloc(m, ptr, bytes);
  };
  A((void**)&m->params, o * sizeof(float));
  A((void**)&m->grad, o * sizeof(float));
  A((void**)&m->am, o * sizeof(float));
  A((void**)&m->av, o * sizeof(float));
  A(&m->pt, o * es);
  A(&m->in, (size_t)rows * 3 * es);
  const int nh = m->train ? L + 1 : 2, nz = m->train ? L : 1, nH = m->train ? L : 1;
  m->h.assign(nh, nullptr);
  m->z.assign(nz, nullptr);
  m->Hs.assign(nH, nullptr);
  for (auto& x : m->h) A(&x, (size_t)rows * C * es);
  for (auto& x : m->z) A((void**)&x, (size_t)rows * C * sizeof(float));
  for (auto& x : m->Hs) A(&x, (size_t)Bm * m->spec * es);
  A(&m->T1, (size_t)Bm * S * 2 * M * C * es);
  A(&m->G, (size_t)Bm * m->spec * es);
  A((void**)&m->rho_hat, (size_t)Bm * m->npix * sizeof(float));
  A((void**)&m->loss_dev, (size_t)Bm * sizeof(double));
  if (m->train) {
    A(&m->dH, (size_t)Bm * m->spec * es);
    A(&m->dz, (size_t)rows * C * es);
    A((void**)&m->dq, (size_t)Bm * m->npix * sizeof(float));
    A((void**)&m->dh, (size_t)rows * C * sizeof(float));
    const size_t part = std::max<size_t>((size_t)m->nsplit * C * C, (size_t)512 * (C + 1));
    A((void**)&m->partials, part * sizeof(float));
  }
  if (m->dry) m->dry_params = p;
  if (e == hipSuccess) e = DEV(m, hipMemcpy(m->params, p.data(), o * sizeof(float), hipMemcpyHostToDevice));
  if (e == hipSuccess) e = DEV(m, hipMemset(m->am, 0, o * sizeof(float)));
  if (e == hipSuccess) e = DEV(m, hipMemset(m->av, 0, o * sizeof(float)));
  if (e == hipSuccess) e = DEV(m, sno_cast(m->params, m->pt, o, m->bf16, nullptr));
  if (e == hipSuccess) e = DEV(m, hipDeviceSynchronize());
  if (e != hipSuccess) {
    qhd_status st = sfail(e == hipErrorOutOfMemory ? QHD_ENOMEM : QHD_EDEVICE, "surrogate allocation: %s",
                          hipGetErrorString(e));
    release(m);
    return st;
  }
  qhd_status st = build_dft(m);
  if (st != QHD_OK) {
    release(m);
    return st;
  }
  *out = m;
  return QHD_OK;
}

qhd_status qhd_sno_param_count(qhd_sno m, int64_t* count) {
  if (!m || !count) return sfail(QHD_EINVAL, "NULL argument");
  *count = m->nparams;
  return QHD_OK;
}

qhd_status qhd_sno_get_params(qhd_sno m, float* host) {
  if (!m || !host) return sfail(QHD_EINVAL, "NULL argument");
  if (m->dry) {
    std::copy(m->dry_params.begin(), m->dry_params.end(), host);
    return QHD_OK;
  }
  SNO_TRY(hipSetDevice(m->device));
  SNO_TRY(hipDeviceSynchronize());
  SNO_TRY(hipMemcpy(host, m->params, m->nparams * sizeof(float), hipMemcpyDeviceToHost));
  return QHD_OK;
}

qhd_status qhd_sno_set_params(qhd_sno m, const float* host) {
  if (!m || !host) return sfail(QHD_EINVAL, "NULL argument");
  m->adam_t = 0;
  m->have_grad = false;
  if (m->dry) {
    std::copy(host, host + m->nparams, m->dry_params.begin());
    return QHD_OK;
  }
  SNO_TRY(hipSetDevice(m->device));
  SNO_TRY(hipDeviceSynchronize());
  SNO_TRY(hipMemcpy(m->params, host, m->nparams * sizeof(float), hipMemcpyHostToDevice));
  SNO_TRY(hipMemset(m->am, 0, m->nparams * sizeof(float)));
  SNO_TRY(hipMemset(m->av, 0, m->nparams * sizeof(float)));
  SNO_TRY(sno_cast(m->params, m->pt, m->nparams, m->bf16, nullptr));
  SNO_TRY(hipDeviceSynchronize());
  return QHD_OK;
}

qhd_status qhd_sno_forward(qhd_sno m, const double* f, int32_t batch, float* rho, void* stream) {
  if (!m || !f || !rho) return sfail(QHD_EINVAL, "NULL argument");
  if (batch < 1 || batch > m->Bmax) return sfail(QHD_EINVAL, "batch %d outside [1, %d]", batch, m->Bmax);
  hipStream_t st = (hipStream_t)stream;
  SNO_TRY(DEV(m, hipSetDevice(m->device)));
  ST_TRY(forward(m, f, batch, st));
  SNO_TRY(DEV(m, hipMemcpyAsync(rho, m->rho_hat, (size_t)batch * m->npix * sizeof(float),
                                hipMemcpyDeviceToDevice, st)));
  return QHD_OK;
}

qhd_status qhd_sno_backward(qhd_sno m, const double* f, const float* target, int32_t batch, double* loss,
                            float* grad_host, void* stream) {
  if (!m || !f || !target || !loss) return sfail(QHD_EINVAL, "NULL argument");
  if (!m->train) return sfail(QHD_ESTATE, "backward needs a surrogate created with train != 0");
  if (batch < 1 || batch > m->Bmax) return sfail(QHD_EINVAL, "batch %d outside [1, %d]", batch, m->Bmax);
  if (m->npix % m->nsplit || ((long long)batch * m->npix) % m->nsplit)
    return sfail(QHD_EUNSUPPORTED, "grid too small for the split-K reductions");
  hipStream_t st = (hipStream_t)stream;
  SNO_TRY(DEV(m, hipSetDevice(m->device)));
  ST_TRY(forward(m, f, batch, st));
  ST_TRY(backward(m, target, batch, st));
  if (m->dry) {
    *loss = 0.0;
    if (grad_host) std::fill(grad_host, grad_host + m->nparams, 0.0f);
    m->have_grad = true;
    return QHD_OK;
  }
  std::vector<double> l(batch);
  SNO_TRY(hipMemcpyAsync(l.data(), m->loss_dev, batch * sizeof(double), hipMemcpyDeviceToHost, st));
  if (grad_host)
    SNO_TRY(hipMemcpyAsync(grad_host, m->grad, m->nparams * sizeof(float), hipMemcpyDeviceToHost, st));
  SNO_TRY(hipStreamSynchronize(st));
  double tot = 0.0;
  for (double v : l) tot += v;
  *loss = tot / batch;
  m->have_grad = true;
  if (!std::isfinite(*loss)) return sfail(QHD_ENUMERIC, "non-finite loss");
  return QHD_OK;
}

qhd_status qhd_sno_step(qhd_sno m, float lr, void* stream) {
  if (!m) return sfail(QHD_EINVAL, "NULL argument");
  if (!m->have_grad) return sfail(QHD_ESTATE, "qhd_sno_step needs a gradient from qhd_sno_backward");
  if (!(lr > 0.0f) || !std::isfinite(lr)) return sfail(QHD_EINVAL, "lr must be finite and > 0");
  m->adam_t += 1;
  if (m->dry) return QHD_OK;
  SNO_TRY(hipSetDevice(m->device));
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.0f - powf(b1, (float)m->adam_t), c2 = 1.0f - powf(b2, (float)m->adam_t);
  SNO_TRY(sno_adam(m->params, m->grad, m->am, m->av, m->nparams, lr, b1, b2, 1e-8f, c1, c2, m->pt, m->bf16,
                   (hipStream_t)stream));
  return QHD_OK;
}

qhd_status qhd_sno_destroy(qhd_sno m) {
  release(m);
  return QHD_OK;
}

}  // extern "C"
