// Host runtime of the EPI solver library: problem handle, workspace, DCT tables, solver
// drivers and the C ABI declared in include/epi.h.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <string>
#include <vector>

#include "epi.h"
#include "epi_common.hpp"
#include "epi_launch.hpp"
#include "epi_internal.hpp"

using namespace epi;

#define EPI_API extern "C" __attribute__((visibility("default")))

// ------------------------------------------------------------------------------------
// errors
// ------------------------------------------------------------------------------------
static thread_local std::string g_err;

epi_status epi::fail(epi_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIPCHK(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(e_ == hipErrorOutOfMemory ? EPI_ENOMEM : EPI_EHIP, "%s: %s (%s:%d)", \
                  #call, hipGetErrorString(e_), __FILE__, __LINE__);                  \
  } while (0)

#define CHKLAUNCH()                                                                   \
  do {                                                                                \
    hipError_t e_ = hipGetLastError();                                                \
    if (e_ != hipSuccess)                                                             \
      return fail(EPI_EHIP, "kernel launch: %s (%s:%d)", hipGetErrorString(e_),        \
                  __FILE__, __LINE__);                                                \
  } while (0)

// ------------------------------------------------------------------------------------
// the handle
// ------------------------------------------------------------------------------------
struct epi_problem {
  epi_grid grid;
  int M, m2, m3, L, P;
  long long n, N;
  double v;
  const float* Ip;
  const float* Im;
  float *wp = nullptr, *wm = nullptr;   // spline coefficients of Ip, Im (image_model 1)
  hipStream_t user = nullptr;
  hipStream_t exec = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  LineArgs la;
  // workspace (n floats each)
  float *w = nullptr, *t1 = nullptr, *t2 = nullptr;
  float *g = nullptr, *hd = nullptr, *ho = nullptr, *x = nullptr, *r = nullptr, *zz = nullptr,
        *p = nullptr;
  double* partial = nullptr;     // general partial sums
  double* partial_e = nullptr;   // ADMM z/u epilogue
  size_t partial_cap = 0;
  DevState* st = nullptr;
  DevState* st_h = nullptr;      // pinned mirror
  int* hard_list = nullptr;
  int hard_blocks = 0;
  // DCT tables (packed MFMA fragments), eigenvalues
  DctTables tab;
  // per-slice j-axis operators for one fixed rho (split-bfloat16, inside the t2 allocation;
  // zop_rho 0: not built)
  void* zop = nullptr;   // per-slice j-axis operators in the precision's fragments
  double zop_rho = 0.0;
  bool use_zop = false;
  double* hist = nullptr;
  int hist_cap = 0;
  // captured ADMM chunk
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  // GN-PCG: four PCG iterations per graph, the first four of a solve ([0]) and any later
  // four ([1]), per line-local preconditioner (BLOCK, JACOBI, NONE)
  hipGraphExec_t pcg_exec[2][3] = {};
  int g_chunk = 0, g_sqp = 0, g_lagr = 0;
  float *g_b = nullptr, *g_z = nullptr, *g_u = nullptr;
  bool g_zop = false;
  // per-kernel event timing (epi_profile_admm)
  bool prof_on = false;
  std::vector<hipEvent_t> prof_ev;
  std::vector<int> prof_kind;
  int prof_used = 0;
  double prof_ms[8] = {0};
  long long prof_cnt[8] = {0};
};

static void prof_begin(epi_problem* p, int kind) {
  if (!p->prof_on) return;
  const size_t need = 2 * (size_t)(p->prof_used + 1);
  while (p->prof_ev.size() < need) {
    hipEvent_t e;
    (void)hipEventCreate(&e);
    p->prof_ev.push_back(e);
  }
  if (p->prof_kind.size() < (size_t)(p->prof_used + 1)) p->prof_kind.resize(p->prof_used + 1);
  p->prof_kind[p->prof_used] = kind;
  (void)hipEventRecord(p->prof_ev[2 * p->prof_used], p->exec);
}
static void prof_end(epi_problem* p) {
  if (!p->prof_on) return;
  (void)hipEventRecord(p->prof_ev[2 * p->prof_used + 1], p->exec);
  p->prof_used += 1;
}
// after a stream synchronisation: fold the recorded pairs into the totals
static void prof_collect(epi_problem* p) {
  for (int i = 0; i < p->prof_used; ++i) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, p->prof_ev[2 * i], p->prof_ev[2 * i + 1]) == hipSuccess) {
      p->prof_ms[p->prof_kind[i]] += ms;
      p->prof_cnt[p->prof_kind[i]] += 1;
    }
  }
  p->prof_used = 0;
}

static void enter(epi_problem* p) {
  (void)hipEventRecord(p->ev_in, p->user);
  (void)hipStreamWaitEvent(p->exec, p->ev_in, 0);
}
static void leave(epi_problem* p) {
  (void)hipEventRecord(p->ev_out, p->exec);
  (void)hipStreamWaitEvent(p->user, p->ev_out, 0);
}

EPI_API int32_t epi_abi_version(void) { return EPI_ABI_VERSION; }

EPI_API const char* epi_last_error(void) { return g_err.c_str(); }

EPI_API void epi_gn_default_opts(epi_gn_opts* o) {
  if (!o) return;
  o->max_iter = 10;
  o->pcg_max = 30;
  o->precond = EPI_PRECOND_BLOCK;
  o->ls_max = 10;
  o->use_stopping = 1;
  o->eta = 0.1;
  o->eps_obj = 1e-3;
  o->eps_iter = 1e-2;
  o->eps_grad = 1e-2;
  o->ls_c1 = 1e-4;
  o->rel_grad_tol = 0.0;
}

EPI_API void epi_admm_default_opts(epi_admm_opts* o) {
  if (!o) return;
  o->max_iter = 100;
  o->sqp_iters = 1;
  o->check_every = 8;
  o->rho = 1e3;
  o->rho_mode = EPI_RHO_FIXED;
  o->tau = 1.3;
  o->mu = 10.0;
  o->rho_min = 1e2;
  o->eps_abs = 0.2;
  o->eps_rel = 0.2;
  o->qp_max_iter = 0;
  o->with_lagrangian = 0;
}

// ------------------------------------------------------------------------------------
// DCT tables: orthonormal DCT-II C[j'][j] = s_j' cos(pi j' (2j+1) / (2m)) (eq. dctdiag),
// eigenvalues of D~(m,h)'D~(m,h): (2 - 2 cos(pi j / m)) / h^2.
// ------------------------------------------------------------------------------------
static void dct_host(int m, std::vector<double>& C) {
  C.assign((size_t)m * m, 0.0);
  for (int a = 0; a < m; ++a) {
    const double s = (a == 0) ? sqrt(1.0 / m) : sqrt(2.0 / m);
    for (int j = 0; j < m; ++j) C[(size_t)a * m + j] = s * cos(M_PI * a * (2.0 * j + 1.0) / (2.0 * m));
  }
}

static uint16_t bf16_rn(float x) {
  uint32_t u;
  memcpy(&u, &x, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
static float bf16_to_f(uint16_t h) {
  uint32_t u = ((uint32_t)h) << 16;
  float x;
  memcpy(&x, &u, 4);
  return x;
}

// Even/odd split of the DCT for the split-bfloat16 kernels (c = ceil(m/2), f = floor(m/2)):
// the even half holds rows k = 2r (forward: C[2r][q], q < c; inverse: C[2q][n], n, q < c),
// the odd half rows k = 2r + 1 (forward: C[2r+1][q]; inverse: C[2q+1][n]; n, r, q < f), in
// row tiles [0, RTh) and [RTh, 2 RTh) with KS steps of 32 over the half's own contraction.
// Fragment (rt, ks) of v_mfma_f32_16x16x32_bf16: lane l holds the half's
// A[16 (rt % RTh) + l % 16][32 ks + 8 (l / 16) + e], e < 8; the hi block, then the lo block
// (a = hi + lo).
static std::vector<uint16_t> pack_bf16_split(const std::vector<double>& C, int m, bool inverse,
                                             int& RT, int& KS) {
  const int ce = (m + 1) / 2, fo = m / 2;
  const int RTh = (ce + 15) / 16;
  RT = 2 * RTh;
  KS = (ce + 31) / 32;
  const size_t nfr = (size_t)RT * KS * 64 * 8;
  std::vector<uint16_t> out(2 * nfr, 0);
  for (int rt = 0; rt < RT; ++rt)
    for (int ks = 0; ks < KS; ++ks)
      for (int l = 0; l < 64; ++l)
        for (int e = 0; e < 8; ++e) {
          const int half = rt / RTh, row = 16 * (rt % RTh) + (l & 15);
          const int q = 32 * ks + 8 * (l >> 4) + e;
          const int cnt = half ? fo : ce;
          double val = 0.0;
          if (row < cnt && q < cnt)
            val = inverse ? C[(size_t)(2 * q + half) * m + row] : C[(size_t)(2 * row + half) * m + q];
          const uint16_t hi = bf16_rn((float)val);
          const uint16_t lo = bf16_rn((float)(val - (double)bf16_to_f(hi)));
          const size_t idx = (((size_t)rt * KS + ks) * 64 + l) * 8 + e;
          out[idx] = hi;
          out[nfr + idx] = lo;
        }
  return out;
}

// The same split for the float32 kernels: fragment (rt, ks) lane l holds the half's
// A[16 (rt % RTh) + l % 16][4 ks + l / 16]; KS = 4 RTh steps of 4 (the half's contraction
// padded to whole 16-row tiles).
static std::vector<float> pack_f32_split(const std::vector<double>& C, int m, bool inverse,
                                         int& RT, int& KS) {
  const int ce = (m + 1) / 2, fo = m / 2;
  const int RTh = (ce + 15) / 16;
  RT = 2 * RTh;
  KS = 4 * RTh;
  std::vector<float> out((size_t)RT * KS * 64, 0.0f);
  for (int rt = 0; rt < RT; ++rt)
    for (int ks = 0; ks < KS; ++ks)
      for (int l = 0; l < 64; ++l) {
        const int half = rt / RTh, row = 16 * (rt % RTh) + (l & 15), q = 4 * ks + (l >> 4);
        const int cnt = half ? fo : ce;
        double val = 0.0;
        if (row < cnt && q < cnt)
          val = inverse ? C[(size_t)(2 * q + half) * m + row] : C[(size_t)(2 * row + half) * m + q];
        out[((size_t)rt * KS + ks) * 64 + l] = (float)val;
      }
  return out;
}

epi_status epi::build_dct_tables(int m2, int m3, double h2, double h3, int precision,
                                 DctTables* t) {
  std::vector<double> C;
  for (int axis = 2; axis <= 3; ++axis) {
    const int m = axis == 2 ? m2 : m3;
    const double h = axis == 2 ? h2 : h3;
    dct_host(m, C);
    void** fw = axis == 2 ? &t->A2f : &t->A3f;
    void** iv = axis == 2 ? &t->A2i : &t->A3i;
    int& RTa = axis == 2 ? t->RT2 : t->RT3;
    int& KSa = axis == 2 ? t->KS2 : t->KS3;
    // even/odd split in both precisions; spectral data in half order (even k first, then
    // odd k)
    for (int inv = 0; inv < 2; ++inv) {
      void** dst = inv ? iv : fw;
      if (precision == EPI_PREC_MIXED) {
        auto v = pack_bf16_split(C, m, inv == 1, RTa, KSa);
        HIPCHK(hipMalloc(dst, v.size() * sizeof(uint16_t)));
        HIPCHK(hipMemcpy(*dst, v.data(), v.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
      } else {
        auto v = pack_f32_split(C, m, inv == 1, RTa, KSa);
        HIPCHK(hipMalloc(dst, v.size() * sizeof(float)));
        HIPCHK(hipMemcpy(*dst, v.data(), v.size() * sizeof(float), hipMemcpyHostToDevice));
      }
    }
    std::vector<float> lam(m);
    const int ce = (m + 1) / 2;
    for (int j = 0; j < m; ++j) {
      // eigenvalue of spectral row j in half order
      const int k = j < ce ? 2 * j : 2 * (j - ce) + 1;
      lam[j] = (float)((2.0 - 2.0 * cos(M_PI * k / m)) / (h * h));
    }
    float** dl = axis == 2 ? &t->lam2 : &t->lam3;
    HIPCHK(hipMalloc(dl, m * sizeof(float)));
    HIPCHK(hipMemcpy(*dl, lam.data(), m * sizeof(float), hipMemcpyHostToDevice));
  }
  return EPI_OK;
}

void epi::free_dct_tables(DctTables* t) {
  void* bufs[] = {t->A2f, t->A2i, t->A3f, t->A3i, t->lam2, t->lam3};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  *t = DctTables();
}

static void free_graph(epi_problem* p) {
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->gexec = nullptr;
  p->graph = nullptr;
  p->g_chunk = 0;
  for (auto& row : p->pcg_exec)
    for (auto& g : row) {
      if (g) (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
}

EPI_API void epi_destroy(epi_problem* p) {
  if (!p) return;
  if (p->exec) (void)hipStreamSynchronize(p->exec);
  free_graph(p);
  void* bufs[] = {p->w, p->t1, p->t2, p->g, p->hd, p->ho, p->x, p->r, p->zz, p->p,
                  p->partial, p->partial_e, p->st, p->hard_list, p->hist, p->wp, p->wm};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  free_dct_tables(&p->tab);
  if (p->st_h) (void)hipHostFree(p->st_h);
  for (hipEvent_t e : p->prof_ev) (void)hipEventDestroy(e);
  if (p->ev_in) (void)hipEventDestroy(p->ev_in);
  if (p->ev_out) (void)hipEventDestroy(p->ev_out);
  if (p->exec) (void)hipStreamDestroy(p->exec);
  delete p;
}

int epi::tiles_axis3(int M, int m2) {
  const long long Q = (long long)m2 * (M + 1);
  return (int)((Q + 63) / 64);
}
int epi::tiles_axis2(int M, int m3) { return m3 * ((M + 1 + 63) / 64); }
static int dct_tiles_axis3(const epi_problem* p) { return tiles_axis3(p->M, p->m2); }
static int dct_tiles_axis2(const epi_problem* p) { return tiles_axis2(p->M, p->m3); }

epi_status epi::validate_grid(const epi_grid* grid) {
  if (grid->ndim != 2 && grid->ndim != 3) return fail(EPI_EINVAL, "ndim must be 2 or 3");
  const int M = grid->m[0], m2 = grid->m[1], m3 = grid->m[2];
  if (M < 2 || m2 < 1 || m3 < 1) return fail(EPI_EINVAL, "cell counts must be M >= 2, m2, m3 >= 1");
  if (grid->ndim == 2 && m3 != 1) return fail(EPI_EINVAL, "2D problems need m[2] = 1");
  if (M + 1 > 64 * EPI_PMAX) return fail(EPI_EINVAL, "M + 1 = %d exceeds %d faces per PE line", M + 1, 64 * EPI_PMAX);
  if (m2 > 256 || m3 > 256) return fail(EPI_EINVAL, "m2, m3 must be <= 256 (DCT axes)");
  for (int a = 0; a < 3; ++a)
    if (!(grid->h[a] > 0.0)) return fail(EPI_EINVAL, "h[%d] must be > 0", a);
  if (!(grid->alpha >= 0.0) || !(grid->beta >= 0.0) || !(grid->gamma >= 0.0))
    return fail(EPI_EINVAL, "alpha, beta, gamma must be >= 0");
  if (grid->precision != EPI_PREC_FP32 && grid->precision != EPI_PREC_MIXED)
    return fail(EPI_EINVAL, "unknown precision %d", grid->precision);
  if (grid->image_model != EPI_IMAGE_LINEAR && grid->image_model != EPI_IMAGE_SPLINE)
    return fail(EPI_EINVAL, "unknown image model %d", grid->image_model);
  if (!(grid->theta >= 0.0)) return fail(EPI_EINVAL, "theta must be >= 0");
  return EPI_OK;
}

// The line system of the cubic B-spline coefficients, factored as L D L' in float64 (band
// half-width 3). theta = 0: the collocation matrix B itself, B[c][k] = beta3(c - k) with
// beta3(0) = 2/3, beta3(+-1) = 1/6 (interpolation). theta > 0: B'B + theta G, with
// (B'B)[k][k] = 1/2 (17/36 at the two end coefficients, which miss a neighbouring sample),
// (B'B)[k][k+1] = 2/9, (B'B)[k][k+2] = 1/36, and G the Gram matrix of the second
// derivatives, integral beta3''(s - k) beta3''(s - l) ds = 8/3, -3/2, 0, 1/6 for |k - l| =
// 0..3 (beta3'' is linear between integers, so these are exact). Lf[3k + j - 1] = L[k][k-j].
static void spline_factor(int M, double theta, std::vector<double>& Lf, std::vector<double>& Dinv) {
  auto A = [&](int k, int l) -> double {
    const int d = k > l ? k - l : l - k;
    if (d > 3) return 0.0;
    if (theta == 0.0) return d == 0 ? 2.0 / 3.0 : (d == 1 ? 1.0 / 6.0 : 0.0);
    double btb = 0.0;
    if (d == 0) btb = (k == 0 || k == M - 1) ? (M == 1 ? 4.0 / 9.0 : 17.0 / 36.0) : 0.5;
    else if (d == 1) btb = 2.0 / 9.0;
    else if (d == 2) btb = 1.0 / 36.0;
    const double g[4] = {8.0 / 3.0, -1.5, 0.0, 1.0 / 6.0};
    return btb + theta * g[d];
  };
  Lf.assign((size_t)3 * M, 0.0);
  Dinv.assign(M, 0.0);
  std::vector<double> D(M, 0.0);
  auto Lget = [&](int i, int k) { return (i > k && i - k <= 3) ? Lf[3 * i + (i - k) - 1] : (i == k ? 1.0 : 0.0); };
  for (int k = 0; k < M; ++k) {
    double d = A(k, k);
    for (int j = 1; j <= 3 && k - j >= 0; ++j) d -= Lget(k, k - j) * Lget(k, k - j) * D[k - j];
    D[k] = d;
    Dinv[k] = 1.0 / d;
    for (int i = k + 1; i <= k + 3 && i < M; ++i) {
      double v = A(i, k);
      for (int m = 1; m <= 3 && k - m >= 0; ++m) v -= Lget(i, k - m) * Lget(k, k - m) * D[k - m];
      Lf[3 * i + (i - k) - 1] = v / d;
    }
  }
}

LineArgs epi::make_line_args(const epi_grid* grid, const float* Ip, const float* Im) {
  LineArgs a{};
  a.Ip = Ip;
  a.Im = Im;
  a.M = grid->m[0];
  a.m2 = grid->m[1];
  a.m3 = grid->m[2];
  a.L = a.m2 * a.m3;
  a.hp = (float)grid->h[0];
  a.inv_hp = (float)(1.0 / grid->h[0]);
  a.inv_h2sq = (float)(1.0 / (grid->h[1] * grid->h[1]));
  a.inv_h3sq = (float)(1.0 / (grid->h[2] * grid->h[2]));
  a.v = (float)(grid->h[0] * grid->h[1] * grid->h[2]);
  a.alpha = (float)grid->alpha;
  a.beta = (float)grid->beta;
  a.gamma = (float)grid->gamma;
  a.nblk = line_blocks(a);
  a.model = grid->image_model;
  return a;
}

static epi_status setup_impl(const epi_grid* grid, const float* Ip, const float* Im, void* stream,
                             epi_problem** out) {
  if (!grid || !Ip || !Im || !out) return fail(EPI_EINVAL, "null argument");
  *out = nullptr;
  epi_status vs = validate_grid(grid);
  if (vs != EPI_OK) return vs;
  const int M = grid->m[0], m2 = grid->m[1], m3 = grid->m[2];
  epi_problem* p = new epi_problem();
  p->grid = *grid;
  p->M = M;
  p->m2 = m2;
  p->m3 = m3;
  p->L = m2 * m3;
  p->P = (M + 1 + 63) / 64;
  p->n = (long long)(M + 1) * p->L;
  p->N = (long long)M * p->L;
  p->v = grid->h[0] * grid->h[1] * grid->h[2];
  p->Ip = Ip;
  p->Im = Im;
  p->user = (hipStream_t)stream;
  p->la = make_line_args(grid, Ip, Im);
  LineArgs& a = p->la;
  *out = p;

  static bool lds_set = false;
  if (!lds_set) {
    // a failure here only matters for tiles above 64 KB, whose launches then report it
    (void)dct_set_lds_limits();
    lds_set = true;
  }
  (void)hipGetLastError();
  HIPCHK(hipStreamCreateWithFlags(&p->exec, hipStreamNonBlocking));
  HIPCHK(hipEventCreateWithFlags(&p->ev_in, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&p->ev_out, hipEventDisableTiming));
  const size_t nb = (size_t)p->n * sizeof(float);
  // the per-slice operators of the j-axis pass (fixed rho) sit behind t2
  const size_t nb_al = (nb + 255) & ~(size_t)255;
  const size_t zb = zop_bytes(grid->precision, p->m2, p->m3);
  float** bufs[] = {&p->w, &p->t1, &p->t2, &p->g, &p->hd, &p->ho, &p->x, &p->r, &p->zz, &p->p};
  for (float** b : bufs) HIPCHK(hipMalloc(b, b == &p->t2 ? nb_al + zb : nb));
  if (zb) p->zop = reinterpret_cast<char*>(p->t2) + nb_al;
  const int lb = line_blocks(a);
  p->hard_blocks = p->L < 128 ? p->L : 128;
  size_t cap = (size_t)lb * NQ_EVAL;
  cap = std::max(cap, (size_t)2048 * 2);
  // the augmented-Lagrangian monitor: two objective evaluations and one dot product
  cap = std::max(cap, (size_t)2 * lb * NQ_EVAL + (size_t)flat_blocks(p->n));
  cap = std::max(cap, (size_t)std::max(dct_tiles_axis2(p), dct_tiles_axis3(p)) * 4);
  p->partial_cap = cap;
  HIPCHK(hipMalloc(&p->partial, cap * sizeof(double)));
  HIPCHK(hipMalloc(&p->partial_e, (size_t)std::max(dct_tiles_axis2(p), dct_tiles_axis3(p)) * NQ_ADMM_E * sizeof(double)));
  HIPCHK(hipMalloc(&p->st, sizeof(DevState)));
  HIPCHK(hipHostMalloc((void**)&p->st_h, sizeof(DevState), hipHostMallocDefault));
  memset(p->st_h, 0, sizeof(DevState));
  HIPCHK(hipMemcpy(p->st, p->st_h, sizeof(DevState), hipMemcpyHostToDevice));
  HIPCHK(hipMalloc(&p->hard_list, (size_t)p->L * sizeof(int)));
  epi_status s = build_dct_tables(m2, m3, grid->h[1], grid->h[2], grid->precision, &p->tab);
  if (s != EPI_OK) return s;

  // the images must be finite
  enter(p);
  launch_count_nonfinite(p->exec, p->N, Ip, p->partial);
  launch_count_nonfinite(p->exec, p->N, Im, p->partial + flat_blocks(p->N));
  CHKLAUNCH();
  FinArgs f{};
  f.kind = FIN_DOT;
  f.partial = p->partial;
  f.nb1 = 2 * flat_blocks(p->N);
  launch_finalize(p->exec, f, p->st);
  CHKLAUNCH();
  HIPCHK(hipMemcpyAsync(p->st_h, p->st, sizeof(DevState), hipMemcpyDeviceToHost, p->exec));
  HIPCHK(hipStreamSynchronize(p->exec));
  if (p->st_h->gTd != 0.0) {
    leave(p);
    return fail(EPI_ENUMERIC, "images contain %.0f non-finite values", p->st_h->gTd);
  }
  if (grid->image_model == EPI_IMAGE_SPLINE) {
    // the kernels read the spline coefficients of both images where the linear model reads
    // the samples
    std::vector<double> Lf, Dinv;
    spline_factor(M, grid->theta, Lf, Dinv);
    double *dL = nullptr, *dD = nullptr, *Y = nullptr;
    const size_t nbc = (size_t)p->N * sizeof(float);
    HIPCHK(hipMalloc(&p->wp, nbc));
    HIPCHK(hipMalloc(&p->wm, nbc));
    HIPCHK(hipMalloc(&dL, Lf.size() * sizeof(double)));
    HIPCHK(hipMalloc(&dD, Dinv.size() * sizeof(double)));
    HIPCHK(hipMalloc(&Y, (size_t)p->N * sizeof(double)));
    HIPCHK(hipMemcpy(dL, Lf.data(), Lf.size() * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dD, Dinv.data(), Dinv.size() * sizeof(double), hipMemcpyHostToDevice));
    const int normal = grid->theta > 0.0 ? 1 : 0;
    launch_spline_coef(p->exec, Ip, p->wp, Y, M, p->L, normal, dL, dD);
    launch_spline_coef(p->exec, Im, p->wm, Y, M, p->L, normal, dL, dD);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(p->exec);
    (void)hipFree(dL);
    (void)hipFree(dD);
    (void)hipFree(Y);
    if (e != hipSuccess) return fail(EPI_EHIP, "spline coefficients: %s", hipGetErrorString(e));
    p->la.Ip = p->wp;
    p->la.Im = p->wm;
  }
  leave(p);
  return EPI_OK;
}

EPI_API epi_status epi_setup(const epi_grid* grid, const float* d_Iplus, const float* d_Iminus,
                                void* stream, epi_problem** out) {
  epi_status s = setup_impl(grid, d_Iplus, d_Iminus, stream, out);
  if (s != EPI_OK && out && *out) {
    epi_destroy(*out);
    *out = nullptr;
  }
  return s;
}

// ------------------------------------------------------------------------------------
// objective (eq. D, eq. S, eq. P and their gradients)
// ------------------------------------------------------------------------------------
static epi_status eval_terms(epi_problem* p, const float* b, int mode, int with_pen, float* grad) {
  launch_eval(p->exec, p->P, mode, p->la, b, nullptr, 0, with_pen, grad, p->hd, p->ho,
              p->partial, p->st);
  CHKLAUNCH();
  FinArgs f{};
  f.kind = FIN_EVAL;
  f.partial = p->partial;
  f.nb1 = line_blocks(p->la);
  f.v = p->v;
  launch_finalize(p->exec, f, p->st);
  CHKLAUNCH();
  return EPI_OK;
}

static void terms_from_state(const epi_problem* p, const DevState* s, int with_pen, epi_terms* t) {
  t->D = s->evalD;
  t->S = 0.5 * p->v * (s->evalS1 + s->evalSx);
  t->feasible = s->eval_infeasible == 0;
  if (with_pen)
    t->P = t->feasible ? p->grid.beta * p->v * s->evalP : INFINITY;
  else
    t->P = 0.0;
  t->J = t->D + p->grid.alpha * t->S + t->P;
}

EPI_API epi_status epi_corrected_images(epi_problem* p, const float* d_b, float* d_Iplus_corr,
                                        float* d_Iminus_corr, epi_quality* out) {
  if (!p || !d_b || !out) return fail(EPI_EINVAL, "null argument");
  if ((d_Iplus_corr == nullptr) != (d_Iminus_corr == nullptr))
    return fail(EPI_EINVAL, "give both corrected-image buffers or neither");
  enter(p);
  launch_correct(p->exec, p->P, p->la, d_b, d_Iplus_corr, d_Iminus_corr, p->partial);
  CHKLAUNCH();
  FinArgs f{};
  f.kind = FIN_QUALITY;
  f.partial = p->partial;
  f.nb1 = line_blocks(p->la);
  launch_finalize(p->exec, f, p->st);
  CHKLAUNCH();
  HIPCHK(hipMemcpyAsync(p->st_h, p->st, sizeof(DevState), hipMemcpyDeviceToHost, p->exec));
  HIPCHK(hipStreamSynchronize(p->exec));
  leave(p);
  const double* q = p->st_h->quality;
  const double n = (double)p->N;
  const double mp = q[0] / n, mm = q[1] / n;
  const double vp = q[2] - n * mp * mp, vm = q[3] - n * mm * mm, cov = q[4] - n * mp * mm;
  out->D = 0.5 * p->v * q[5];
  out->ncc = (vp > 0.0 && vm > 0.0) ? cov / sqrt(vp * vm) : 0.0;
  out->mean_plus = mp;
  out->mean_minus = mm;
  if (!(out->D == out->D)) return fail(EPI_ENUMERIC, "corrected images are not finite");
  return EPI_OK;
}

EPI_API epi_status epi_objective(epi_problem* p, const float* d_b, int32_t with_penalty,
                                    epi_terms* out, float* d_grad) {
  if (!p || !d_b || !out) return fail(EPI_EINVAL, "null argument");
  enter(p);
  epi_status s = eval_terms(p, d_b, d_grad ? 1 : 0, with_penalty ? 1 : 0, d_grad);
  if (s != EPI_OK) return s;
  HIPCHK(hipMemcpyAsync(p->st_h, p->st, sizeof(DevState), hipMemcpyDeviceToHost, p->exec));
  HIPCHK(hipStreamSynchronize(p->exec));
  leave(p);
  terms_from_state(p, p->st_h, with_penalty, out);
  if (!(out->D == out->D) || !(out->S == out->S)) return fail(EPI_ENUMERIC, "objective is NaN");
  return EPI_OK;
}

// ------------------------------------------------------------------------------------
// z-step passes
// ------------------------------------------------------------------------------------
GemmArgs epi::make_gemm_axis3(int M, int m2, int m3, float alpha, const DctTables& t,
                              const float* in, float* out, bool inverse, const DevState* st) {
  GemmArgs g{};
  g.in = in;
  g.out = out;
  g.rows = m3;
  g.ncol = m2 * (M + 1);
  g.ld = (long long)m2 * (M + 1);
  g.bstride = 0;
  g.nbatch = 1;
  g.col_tiles = (g.ncol + 63) / 64;
  g.RT = t.RT3;
  g.KS = t.KS3;
  g.dir = inverse ? 1 : 0;
  g.A1 = inverse ? t.A3i : t.A3f;
  g.A2 = nullptr;
  g.alpha = alpha;
  g.st = st;
  return g;
}

GemmArgs epi::make_gemm_axis2(int M, int m2, int m3, float alpha, const DctTables& t,
                              const float* in, float* out, const DevState* st) {
  GemmArgs g{};
  g.in = in;
  g.out = out;
  g.rows = m2;
  g.ncol = M + 1;
  g.ld = M + 1;
  g.bstride = (long long)m2 * (M + 1);
  g.nbatch = m3;
  g.col_tiles = (g.ncol + 63) / 64;
  g.RT = t.RT2;
  g.KS = t.KS2;
  g.A1 = t.A2f;
  g.A2 = t.A2i;
  g.lam_row = t.lam2;
  g.lam_batch = t.lam3;
  g.alpha = alpha;
  g.st = st;
  return g;
}

static GemmArgs gemm_axis3(const epi_problem* p, const float* in, float* out, bool inverse) {
  return make_gemm_axis3(p->M, p->m2, p->m3, (float)p->grid.alpha, p->tab, in, out, inverse, p->st);
}
static GemmArgs gemm_axis2(const epi_problem* p, const float* in, float* out) {
  GemmArgs g = make_gemm_axis2(p->M, p->m2, p->m3, (float)p->grid.alpha, p->tab, in, out, p->st);
  if (p->use_zop) {
    g.dir = 2;
    g.A1 = p->zop;
    g.A2 = nullptr;
    // per slice: hi and lo blocks of 16-byte fragments (bfloat16), or floats (float32)
    g.a_bstride = (p->grid.precision == EPI_PREC_MIXED ? 2LL : 1LL) * p->tab.RT2 * p->tab.KS2 * 64;
  }
  return g;
}
static void launch_axis2(const epi_problem* p, int prec, const GemmArgs& g) {
  if (p->use_zop) launch_dct_axis2_op(p->exec, prec, g);
  else launch_dct_axis2_fused(p->exec, prec, g);
}

// With a fixed rho the split-bfloat16 z-step takes the j-axis forward, spectral scale and
// inverse of each k-slice as one product with the slice's operator C_h^T S_h C_h (built
// once per rho); with an adaptive rho, or in float32, the fused pass applies the three.
static epi_status prepare_zop(epi_problem* p, double rho, bool fixed_rho) {
  p->use_zop = false;
  if (!p->zop || !fixed_rho) return EPI_OK;
  if (p->zop_rho == 0.0)   // padding entries of the fragments stay zero
    HIPCHK(hipMemsetAsync(p->zop, 0, zop_bytes(p->grid.precision, p->m2, p->m3), p->exec));
  if (p->zop_rho != rho) {
    if (launch_build_zop(p->exec, p->grid.precision, p->m2, p->m3, p->grid.h[1], p->grid.h[2],
                         p->grid.alpha, rho, p->tab.RT2, p->tab.KS2, p->zop))
      return fail(EPI_EINVAL, "transform length %d not supported", p->m2);
    CHKLAUNCH();
    p->zop_rho = rho;
  }
  p->use_zop = true;
  return EPI_OK;
}

// z = smoothness solve of w; with admm != 0 the last pass performs the u-step epilogue
// (reads b, u, z; writes z, u; partial sums into partial_e).
static epi_status launch_zstep(epi_problem* p, const float* w, float* z, int admm, const float* b,
                               float* u) {
  const int prec = p->grid.precision;
  const int* done = admm ? &p->st->admm_done : nullptr;
  if (p->m3 == 1) {
    GemmArgs g2 = gemm_axis2(p, w, z);
    g2.done = done;
    if (admm) {
      g2.epi = 1;
      g2.b = b;
      g2.z = z;
      g2.u = u;
      g2.partial = p->partial_e;
    }
    prof_begin(p, EPI_K_DCT_LAST);
    launch_axis2(p, prec, g2);
    prof_end(p);
    CHKLAUNCH();
    return EPI_OK;
  }
  GemmArgs g1 = gemm_axis3(p, w, p->t1, false);
  g1.done = done;
  prof_begin(p, EPI_K_DCT_AXIS3);
  launch_dct_axis3(p->exec, prec, g1);
  prof_end(p);
  CHKLAUNCH();
  GemmArgs g2 = gemm_axis2(p, p->t1, p->t2);
  g2.done = done;
  prof_begin(p, EPI_K_DCT_AXIS2);
  launch_axis2(p, prec, g2);
  prof_end(p);
  CHKLAUNCH();
  GemmArgs g3 = gemm_axis3(p, p->t2, z, true);
  g3.done = done;
  if (admm) {
    g3.epi = 1;
    g3.b = b;
    g3.z = z;
    g3.u = u;
    g3.partial = p->partial_e;
  }
  prof_begin(p, EPI_K_DCT_LAST);
  launch_dct_axis3(p->exec, prec, g3);
  prof_end(p);
  CHKLAUNCH();
  return EPI_OK;
}

static int zstep_epi_blocks(const epi_problem* p) {
  return p->m3 == 1 ? dct_tiles_axis2(p) : dct_tiles_axis3(p);
}

EPI_API epi_status epi_smooth_solve(epi_problem* p, const float* d_w, double rho, float* d_z) {
  if (!p || !d_w || !d_z) return fail(EPI_EINVAL, "null argument");
  if (!(rho > 0.0)) return fail(EPI_EINVAL, "rho must be > 0");
  enter(p);
  HIPCHK(hipStreamSynchronize(p->exec));   // the pinned mirror is reused below
  p->st_h->rho = rho;
  HIPCHK(hipMemcpyAsync(&p->st->rho, &p->st_h->rho, sizeof(double), hipMemcpyHostToDevice, p->exec));
  epi_status s = prepare_zop(p, rho, true);
  if (s != EPI_OK) return s;
  s = launch_zstep(p, d_w, d_z, 0, nullptr, nullptr);
  if (s != EPI_OK) return s;
  HIPCHK(hipStreamSynchronize(p->exec));
  leave(p);
  return EPI_OK;
}

// ------------------------------------------------------------------------------------
// ADMM (Section 4.2)
// ------------------------------------------------------------------------------------
// The augmented Lagrangian (eq. Lp) at the iterate just finished: D and |D1 b|^2 from an
// objective evaluation of b, |D2 z|^2 + |D3 z|^2 from one of z, u'(b - z) from a dot
// product; the finalisation adds the rho terms from the history row of that iteration.
static epi_status admm_lagrangian(epi_problem* p, const float* b, const float* z, const float* u) {
  const int lb = line_blocks(p->la);
  double* p1 = p->partial;
  double* p2 = p1 + (size_t)lb * NQ_EVAL;
  double* p3 = p2 + (size_t)lb * NQ_EVAL;
  launch_eval(p->exec, p->P, 0, p->la, b, nullptr, 0, 0, nullptr, nullptr, nullptr, p1, p->st);
  launch_eval(p->exec, p->P, 0, p->la, z, nullptr, 0, 0, nullptr, nullptr, nullptr, p2, p->st);
  launch_udot(p->exec, p->n, u, b, z, p3);
  CHKLAUNCH();
  FinArgs f{};
  f.kind = FIN_LAGRANGIAN;
  f.partial = p1;
  f.nb1 = lb;
  f.partial2 = p2;
  f.nb2 = lb;
  f.partial3 = p3;
  f.nb3 = flat_blocks(p->n);
  f.v = p->v;
  f.alpha = p->grid.alpha;
  f.hist = p->hist;
  f.hist_len = p->hist_cap;
  launch_finalize(p->exec, f, p->st);
  CHKLAUNCH();
  return EPI_OK;
}

static epi_status admm_iteration(epi_problem* p, float* b, float* z, float* u, int sqp,
                                 int lagr) {
  const int lb = line_blocks(p->la);
  for (int s = 0; s < sqp; ++s) {
    if (s > 0) {
      FinArgs f{};
      f.kind = FIN_HARD_RESET;
      launch_finalize(p->exec, f, p->st);
    }
    launch_admm_bstep(p->exec, p->P, p->la, b, z, u, p->w, p->hard_list, p->st, p->hard_blocks,
                      [&](int k) { prof_begin(p, k); }, [&]() { prof_end(p); });
    CHKLAUNCH();
  }
  epi_status st = launch_zstep(p, p->w, z, 1, b, u);
  if (st != EPI_OK) return st;
  FinArgs f{};
  f.kind = FIN_ADMM;
  f.partial = p->partial_e;
  f.nb1 = zstep_epi_blocks(p);
  f.hist = p->hist;
  f.hist_len = p->hist_cap;
  prof_begin(p, EPI_K_FINALIZE);
  launch_finalize(p->exec, f, p->st);
  prof_end(p);
  CHKLAUNCH();
  if (lagr) return admm_lagrangian(p, b, z, u);
  return EPI_OK;
}

static epi_status count_violations(epi_problem* p, const float* b, float thr, double* count) {
  launch_count_violations(p->exec, p->la, b, thr, p->partial);
  CHKLAUNCH();
  FinArgs f{};
  f.kind = FIN_DOT;
  f.partial = p->partial;
  f.nb1 = flat_blocks(p->N);
  launch_finalize(p->exec, f, p->st);
  CHKLAUNCH();
  HIPCHK(hipMemcpyAsync(p->st_h, p->st, sizeof(DevState), hipMemcpyDeviceToHost, p->exec));
  HIPCHK(hipStreamSynchronize(p->exec));
  *count = p->st_h->gTd;
  return EPI_OK;
}

epi_status epi::validate_rho_opts(const epi_admm_opts* o) {
  if (o->rho_mode < EPI_RHO_FIXED || o->rho_mode > EPI_RHO_ADAPT_FLOOR)
    return fail(EPI_EINVAL, "unknown rho_mode %d", o->rho_mode);
  if (o->rho_mode != EPI_RHO_FIXED && !(o->tau > 1.0 && o->mu >= 1.0 && o->rho_min > 0.0))
    return fail(EPI_EINVAL, "adaptive rho needs tau > 1, mu >= 1, rho_min > 0");
  return EPI_OK;
}

void epi::init_rho_state(DevState* h, const epi_admm_opts* o) {
  h->u_scale = 1.0;
  h->rho_mode = o->rho_mode;
  h->tau = o->tau;
  h->mu = o->mu;
  h->rho_min = o->rho_min;
}

static epi_status solve_admm_impl(epi_problem* p, float* d_b, float* d_z, float* d_u,
                                  const epi_admm_opts* opts, epi_admm_report* rep) {
  if (!p || !d_b || !d_z || !d_u || !opts) return fail(EPI_EINVAL, "null argument");
  if (!(opts->rho > 0.0)) return fail(EPI_EINVAL, "rho must be > 0");
  if (opts->max_iter < 0 || opts->sqp_iters < 1 || opts->check_every < 1 || opts->qp_max_iter < 0)
    return fail(EPI_EINVAL, "max_iter >= 0, sqp_iters >= 1, check_every >= 1, qp_max_iter >= 0 required");
  const int lagr = opts->with_lagrangian ? 1 : 0;
  epi_status vo = validate_rho_opts(opts);
  if (vo != EPI_OK) return vo;
  enter(p);
  double viol = 0.0;
  epi_status s = count_violations(p, d_b, 1.0f + 1e-5f, &viol);
  if (s != EPI_OK) return s;
  if (viol > 0.0) {
    leave(p);
    return fail(EPI_EINFEASIBLE, "starting field has %.0f cells with |D1 b| > 1", viol);
  }
  const int cap = opts->max_iter > 0 ? opts->max_iter : 1;
  if (cap > p->hist_cap) {
    if (p->hist) HIPCHK(hipFree(p->hist));
    p->hist = nullptr;
    HIPCHK(hipMalloc(&p->hist, (size_t)EPI_HIST_ROWS * cap * sizeof(double)));
    p->hist_cap = cap;
    free_graph(p);   // the finalize node holds the history pointer
  }
  DevState* h = p->st_h;
  memset(h, 0, sizeof(DevState));
  h->rho = opts->rho;
  h->eps_abs = opts->eps_abs;
  h->eps_rel = opts->eps_rel;
  h->sqrt_n = sqrt((double)p->n);
  h->v = p->v;
  h->admm_max = opts->max_iter;
  h->admm_done = opts->max_iter == 0 ? 2 : 0;
  h->qp_max_iter = opts->qp_max_iter;
  init_rho_state(h, opts);
  HIPCHK(hipMemcpyAsync(p->st, h, sizeof(DevState), hipMemcpyHostToDevice, p->exec));
  s = prepare_zop(p, opts->rho, opts->rho_mode == EPI_RHO_FIXED);
  if (s != EPI_OK) return s;

  const int chunk = opts->check_every;
  const bool use_graph = !p->prof_on;
  if (use_graph && (p->g_chunk != chunk || p->g_sqp != opts->sqp_iters || p->g_b != d_b ||
                    p->g_z != d_z || p->g_u != d_u || p->g_zop != p->use_zop ||
                    p->g_lagr != lagr)) {
    free_graph(p);
    HIPCHK(hipStreamBeginCapture(p->exec, hipStreamCaptureModeThreadLocal));
    for (int i = 0; i < chunk; ++i) {
      s = admm_iteration(p, d_b, d_z, d_u, opts->sqp_iters, lagr);
      if (s != EPI_OK) {
        hipGraph_t tmp = nullptr;
        (void)hipStreamEndCapture(p->exec, &tmp);
        if (tmp) (void)hipGraphDestroy(tmp);
        return s;
      }
    }
    HIPCHK(hipStreamEndCapture(p->exec, &p->graph));
    HIPCHK(hipGraphInstantiate(&p->gexec, p->graph, nullptr, nullptr, 0));
    p->g_chunk = chunk;
    p->g_sqp = opts->sqp_iters;
    p->g_b = d_b;
    p->g_z = d_z;
    p->g_u = d_u;
    p->g_zop = p->use_zop;
    p->g_lagr = lagr;
  }
  int done = opts->max_iter == 0;
  int launched = 0;
  while (!done) {
    if (use_graph) {
      HIPCHK(hipGraphLaunch(p->gexec, p->exec));
    } else {
      for (int i = 0; i < chunk; ++i) {
        s = admm_iteration(p, d_b, d_z, d_u, opts->sqp_iters, lagr);
        if (s != EPI_OK) return s;
      }
    }
    launched += chunk;
    HIPCHK(hipMemcpyAsync(h, p->st, sizeof(DevState), hipMemcpyDeviceToHost, p->exec));
    HIPCHK(hipStreamSynchronize(p->exec));
    prof_collect(p);
    done = h->admm_done != 0 || launched >= opts->max_iter;
  }
  HIPCHK(hipMemcpyAsync(h, p->st, sizeof(DevState), hipMemcpyDeviceToHost, p->exec));
  HIPCHK(hipStreamSynchronize(p->exec));
  const int iters = h->admm_iter;
  if (rep) {
    rep->iters = iters;
    rep->converged = h->admm_done == 1 && h->numeric_bad == 0;
    rep->max_active = h->max_active;
    rep->hard_lines = h->hard_total;
    rep->status = h->numeric_bad ? EPI_ENUMERIC : EPI_OK;
    double* outs[EPI_HIST_ROWS] = {rep->r_pri, rep->r_dual, rep->eps_pri, rep->eps_dual,
                                   rep->rho, lagr ? rep->lagrangian : nullptr};
    for (int k = 0; k < EPI_HIST_ROWS; ++k)
      if (outs[k] && iters > 0)
        HIPCHK(hipMemcpy(outs[k], p->hist + (size_t)k * p->hist_cap, iters * sizeof(double),
                         hipMemcpyDeviceToHost));
  }
  leave(p);
  if (h->numeric_bad) return fail(EPI_ENUMERIC, "non-finite value during ADMM");
  return EPI_OK;
}

EPI_API epi_status epi_solve_admm(epi_problem* p, float* d_b, float* d_z, float* d_u,
                                  const epi_admm_opts* opts, epi_admm_report* rep) {
  if (!p) return fail(EPI_EINVAL, "null argument");
  p->prof_on = false;
  return solve_admm_impl(p, d_b, d_z, d_u, opts, rep);
}

// Back-to-back launch times of each kernel family of an ADMM iteration: the final state
// of the profiled solve is copied into the GN work vectors (x <- b, r <- z, zz <- u), the
// device state is set so that no kernel stops early (stopping test off, no cap, history
// writes past the end of the history), and every family runs `reps` times in a row
// between one pair of events.
static epi_status profile_isolated(epi_problem* p, const float* d_b, const float* d_z,
                                   const float* d_u, int reps, epi_kernel_profile* prof) {
  const size_t nb = (size_t)p->n * sizeof(float);
  float *b = p->x, *z = p->r, *u = p->zz;
  HIPCHK(hipMemcpyAsync(b, d_b, nb, hipMemcpyDeviceToDevice, p->exec));
  HIPCHK(hipMemcpyAsync(z, d_z, nb, hipMemcpyDeviceToDevice, p->exec));
  HIPCHK(hipMemcpyAsync(u, d_u, nb, hipMemcpyDeviceToDevice, p->exec));
  HIPCHK(hipMemcpyAsync(p->st_h, p->st, sizeof(DevState), hipMemcpyDeviceToHost, p->exec));
  HIPCHK(hipStreamSynchronize(p->exec));
  DevState* h = p->st_h;
  h->admm_done = 0;
  h->admm_max = 0x7fffffff;
  h->admm_iter = p->hist_cap;     // admm_finalize writes history rows below hist_cap only
  h->eps_abs = 0.0;
  h->eps_rel = 0.0;
  h->numeric_bad = 0;
  h->rho_mode = 0;
  h->u_scale = 1.0;
  HIPCHK(hipMemcpyAsync(p->st, h, sizeof(DevState), hipMemcpyHostToDevice, p->exec));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  const int prec = p->grid.precision;
  auto run = [&](int fam) {
    for (int r = 0; r < reps; ++r) {
      switch (fam) {
        case EPI_K_BSTEP:
        case EPI_K_BSTEP_HARD:
          launch_admm_bstep_part(p->exec, fam == EPI_K_BSTEP ? 0 : 1, p->P, p->la, b, z, u,
                                 p->w, p->hard_list, p->st, p->hard_blocks);
          break;
        case EPI_K_DCT_AXIS3: {
          GemmArgs g = gemm_axis3(p, p->w, p->t1, false);
          g.done = &p->st->admm_done;
          launch_dct_axis3(p->exec, prec, g);
        } break;
        case EPI_K_DCT_AXIS2: {
          GemmArgs g = gemm_axis2(p, p->t1, p->t2);
          g.done = &p->st->admm_done;
          launch_axis2(p, prec, g);
        } break;
        case EPI_K_DCT_LAST: {
          GemmArgs g = p->m3 == 1 ? gemm_axis2(p, p->w, z) : gemm_axis3(p, p->t2, z, true);
          g.done = &p->st->admm_done;
          g.epi = 1;
          g.b = b;
          g.z = z;
          g.u = u;
          g.partial = p->partial_e;
          if (p->m3 == 1) launch_axis2(p, prec, g);
          else launch_dct_axis3(p->exec, prec, g);
        } break;
        default: {
          FinArgs f{};
          f.kind = FIN_ADMM;
          f.partial = p->partial_e;
          f.nb1 = zstep_epi_blocks(p);
          f.hist = p->hist;
          f.hist_len = p->hist_cap;
          launch_finalize(p->exec, f, p->st);
        } break;
      }
    }
  };
  epi_status out = EPI_OK;
  for (int fam = 0; fam < EPI_K_COUNT && out == EPI_OK; ++fam) {
    prof->us_isolated[fam] = 0.0;
    if (p->m3 == 1 && (fam == EPI_K_DCT_AXIS3 || fam == EPI_K_DCT_AXIS2)) continue;
    run(fam);   // warm-up of the family (code object, caches)
    (void)hipEventRecord(e0, p->exec);
    run(fam);
    (void)hipEventRecord(e1, p->exec);
    if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
      out = fail(EPI_EHIP, "isolated kernel timing");
      break;
    }
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess) prof->us_isolated[fam] = 1e3 * ms / reps;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return out;
}

EPI_API epi_status epi_profile_admm(epi_problem* p, float* d_b, float* d_z, float* d_u,
                                    const epi_admm_opts* opts, epi_admm_report* rep,
                                    epi_kernel_profile* prof) {
  if (!p || !prof) return fail(EPI_EINVAL, "null argument");
  p->prof_on = true;
  p->prof_used = 0;
  for (int k = 0; k < 8; ++k) {
    p->prof_ms[k] = 0.0;
    p->prof_cnt[k] = 0;
  }
  const int reps = prof->isolated_reps;
  epi_status s = solve_admm_impl(p, d_b, d_z, d_u, opts, rep);
  p->prof_on = false;
  for (int k = 0; k < 8; ++k) {
    prof->ms[k] = p->prof_ms[k];
    prof->launches[k] = p->prof_cnt[k];
    prof->us_isolated[k] = 0.0;
  }
  if (s == EPI_OK && reps > 0) {
    enter(p);
    s = profile_isolated(p, d_b, d_z, d_u, reps, prof);
    leave(p);
  }
  return s;
}

// ------------------------------------------------------------------------------------
// GN-PCG (Section 4.1)
// ------------------------------------------------------------------------------------
// One PCG iteration (Section 4.1, the inner solve of eq. GNstep): matvec with the direction
// update, step length, update of x and r with the preconditioner (SGS: unpreconditioned
// update, then the two sweeps), next beta. f carries the finalisation's constants.
static void pcg_iteration(epi_problem* p, int it, int precond, bool sgs, FinArgs f) {
  const int lb = line_blocks(p->la);
  const long long n = p->n;
  float* pbuf[2] = {p->p, p->t1};
  float* pcur = pbuf[it & 1];
  if (it == 0)
    launch_matvec(p->exec, p->P, p->la, nullptr, pcur, nullptr, p->hd, p->ho, p->partial, p->st);
  else
    launch_matvec(p->exec, p->P, p->la, p->zz, pbuf[(it - 1) & 1], pcur, p->hd, p->ho,
                  p->partial, p->st);
  f.kind = FIN_PCG_ALPHA;
  f.nb1 = lb;
  launch_finalize(p->exec, f, p->st);
  launch_pcg_update(p->exec, p->P, p->la, sgs ? EPI_PRECOND_NONE : precond, p->hd, p->ho, p->x,
                    p->r, p->zz, pcur, p->partial, p->st);
  if (sgs) {
    launch_sgs(p->exec, p->P, p->la, p->hd, p->ho, p->r, p->zz, p->st, 1);
    launch_sgs_finish(p->exec, n, p->r, p->zz, nullptr, p->partial, 0, p->st);
  }
  f.kind = FIN_PCG_UPDATE;
  f.nb1 = sgs ? flat_blocks(n) : lb;
  launch_finalize(p->exec, f, p->st);
}

EPI_API epi_status epi_precond_apply(epi_problem* p, const float* d_b, int32_t precond,
                                     const float* d_r, float* d_z) {
  if (!p || !d_b || !d_r || !d_z) return fail(EPI_EINVAL, "null argument");
  if (precond < EPI_PRECOND_BLOCK || precond > EPI_PRECOND_SGS)
    return fail(EPI_EINVAL, "unknown preconditioner %d", precond);
  const auto overlap = [&](const float* x) { return x < d_z + p->n && d_z < x + p->n; };
  if (overlap(d_r) || overlap(d_b)) return fail(EPI_EINVAL, "d_z must not overlap d_r or d_b");
  enter(p);
  epi_status s = eval_terms(p, d_b, 2, 1, p->g);
  if (s != EPI_OK) return s;
  HIPCHK(hipMemcpyAsync(p->st_h, p->st, sizeof(DevState), hipMemcpyDeviceToHost, p->exec));
  HIPCHK(hipStreamSynchronize(p->exec));
  if (p->st_h->eval_infeasible) {
    leave(p);
    return fail(EPI_EINFEASIBLE, "field has %d cells with |D1 b| >= 1", p->st_h->eval_infeasible);
  }
  if (precond == EPI_PRECOND_SGS)
    launch_sgs(p->exec, p->P, p->la, p->hd, p->ho, d_r, d_z, p->st, 0);
  else
    launch_precond(p->exec, p->P, p->la, precond, p->hd, p->ho, d_r, d_z);
  CHKLAUNCH();
  HIPCHK(hipStreamSynchronize(p->exec));
  leave(p);
  return EPI_OK;
}

EPI_API epi_status epi_solve_gnpcg(epi_problem* p, float* d_b, const epi_gn_opts* opts,
                                      epi_gn_report* rep) {
  if (!p || !d_b || !opts) return fail(EPI_EINVAL, "null argument");
  if (opts->max_iter < 0 || opts->pcg_max < 0 || opts->ls_max < 1 || opts->precond < 0 ||
      opts->precond > EPI_PRECOND_SGS || !(opts->eta > 0.0))
    return fail(EPI_EINVAL, "invalid GN options");
  enter(p);
  const long long n = p->n;
  const int lb = line_blocks(p->la);
  const bool sgs = opts->precond == EPI_PRECOND_SGS;
  DevState* h = p->st_h;
  HIPCHK(hipStreamSynchronize(p->exec));
  memset(h, 0, sizeof(DevState));
  h->eta2 = opts->eta * opts->eta;
  h->c1 = opts->ls_c1;
  HIPCHK(hipMemcpyAsync(p->st, h, sizeof(DevState), hipMemcpyHostToDevice, p->exec));
  epi_status s = eval_terms(p, d_b, 2, 1, p->g);
  if (s != EPI_OK) return s;
  HIPCHK(hipMemcpyAsync(h, p->st, sizeof(DevState), hipMemcpyDeviceToHost, p->exec));
  HIPCHK(hipStreamSynchronize(p->exec));
  epi_terms t;
  terms_from_state(p, h, 1, &t);
  if (!t.feasible) {
    leave(p);
    return fail(EPI_EINFEASIBLE, "starting field has %d cells with |D1 b| >= 1", h->eval_infeasible);
  }
  if (!(t.J == t.J)) return fail(EPI_ENUMERIC, "objective is NaN at the starting field");
  double J = t.J, J0 = t.J;
  double gn = sqrt(h->evalG2), g0 = gn;
  if (rep) {
    rep->iters = 0;
    rep->converged = 0;
    rep->ls_failed = 0;
    rep->status = EPI_OK;
    if (rep->J) rep->J[0] = J;
    if (rep->grad_norm) rep->grad_norm[0] = gn;
  }
  double Jprev = 0.0, dstep = 0.0, bprev = 0.0;
  bool converged = false, ls_failed = false;
  int k = 0;
  for (;; ++k) {
    if (k > 0 && opts->use_stopping) {
      const bool c1 = fabs(J - Jprev) <= opts->eps_obj * (1.0 + fabs(J0));
      const bool c2 = dstep <= opts->eps_iter * (1.0 + bprev);
      const bool c3 = gn <= opts->eps_grad * (1.0 + fabs(J0));
      if (c1 && c2 && c3) {
        converged = true;
        break;
      }
    }
    if (opts->rel_grad_tol > 0.0 && gn <= opts->rel_grad_tol * g0) {
      converged = true;
      break;
    }
    if (k >= opts->max_iter) break;
    // PCG on H d = -g, the hessian blocks are in hd/ho from the last evaluation. With SGS
    // the line kernels run unpreconditioned and the two sweeps then replace z (and p at the
    // start) and the partial sums.
    launch_pcg_init(p->exec, p->P, p->la, sgs ? EPI_PRECOND_NONE : opts->precond, p->g, p->hd,
                    p->ho, p->x, p->r, p->zz, p->p, p->partial);
    if (sgs) {
      launch_sgs(p->exec, p->P, p->la, p->hd, p->ho, p->r, p->zz, p->st, 0);
      launch_sgs_finish(p->exec, n, p->r, p->zz, p->p, p->partial, 1, p->st);
    }
    CHKLAUNCH();
    FinArgs f{};
    f.partial = p->partial;
    f.v = p->v;
    f.alpha = p->grid.alpha;
    f.beta = p->grid.beta;
    f.kind = FIN_PCG_INIT;
    f.nb1 = sgs ? flat_blocks(n) : lb;
    launch_finalize(p->exec, f, p->st);
    // the direction p alternates between two buffers: from the second PCG iteration on, the
    // matvec forms p = z + beta p_old itself and writes it to the other buffer. Four
    // iterations at a time, then a host check of the PCG stop; with a line-local
    // preconditioner every full group of four is one graph launch (the kernels of an
    // iteration after the stop return at once).
    for (int it = 0; it < opts->pcg_max;) {
      const int cnt = std::min(4, opts->pcg_max - it);
      if (!sgs && cnt == 4) {
        hipGraphExec_t& ge = p->pcg_exec[it == 0 ? 0 : 1][opts->precond];
        if (!ge) {
          hipGraph_t gr = nullptr;
          HIPCHK(hipStreamBeginCapture(p->exec, hipStreamCaptureModeThreadLocal));
          for (int k = 0; k < 4; ++k) pcg_iteration(p, it + k, opts->precond, false, f);
          hipError_t e = hipGetLastError();
          const hipError_t e2 = hipStreamEndCapture(p->exec, &gr);
          if (e == hipSuccess) e = e2;
          if (e == hipSuccess) e = hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0);
          if (gr) (void)hipGraphDestroy(gr);
          if (e != hipSuccess) {
            ge = nullptr;
            return fail(EPI_EHIP, "PCG graph: %s", hipGetErrorString(e));
          }
        }
        HIPCHK(hipGraphLaunch(ge, p->exec));
      } else {
        for (int k = 0; k < cnt; ++k) pcg_iteration(p, it + k, opts->precond, sgs, f);
        CHKLAUNCH();
      }
      it += cnt;
      if (it < opts->pcg_max) {
        HIPCHK(hipMemcpyAsync(h, p->st, sizeof(DevState), hipMemcpyDeviceToHost, p->exec));
        HIPCHK(hipStreamSynchronize(p->exec));
        if (h->pcg_done) break;
      }
    }
    // Armijo line search on J_GN along d = x
    launch_dot(p->exec, n, p->g, p->x, p->partial);
    f.kind = FIN_DOT;
    f.nb1 = flat_blocks(n);
    launch_finalize(p->exec, f, p->st);
    f.kind = FIN_LS_INIT;
    f.value = J;
    launch_finalize(p->exec, f, p->st);
    for (int t2 = 0; t2 < opts->ls_max; ++t2) {
      launch_eval(p->exec, p->P, 0, p->la, d_b, p->x, t2, 1, nullptr, nullptr, nullptr,
                  p->partial, p->st);
      f.kind = FIN_LS;
      f.nb1 = lb;
      f.trial = t2;
      launch_finalize(p->exec, f, p->st);
    }
    launch_gn_step(p->exec, n, d_b, p->x, p->partial, p->st);
    f.kind = FIN_STEP;
    f.nb1 = flat_blocks(n);
    launch_finalize(p->exec, f, p->st);
    CHKLAUNCH();
    s = eval_terms(p, d_b, 2, 1, p->g);
    if (s != EPI_OK) return s;
    HIPCHK(hipMemcpyAsync(h, p->st, sizeof(DevState), hipMemcpyDeviceToHost, p->exec));
    HIPCHK(hipStreamSynchronize(p->exec));
    const double lam = h->lam_acc;
    if (rep) {
      if (rep->pcg_iters) rep->pcg_iters[k] = h->pcg_iters;
      if (rep->pcg_relres) rep->pcg_relres[k] = h->relres;
      if (rep->step) rep->step[k] = lam;
      rep->iters = k + 1;
    }
    if (!(lam > 0.0)) {
      ls_failed = true;
      break;
    }
    Jprev = J;
    terms_from_state(p, h, 1, &t);
    J = t.J;
    gn = sqrt(h->evalG2);
    dstep = sqrt(h->step2);
    bprev = sqrt(h->bold2);
    if (rep) {
      if (rep->J) rep->J[k + 1] = J;
      if (rep->grad_norm) rep->grad_norm[k + 1] = gn;
    }
    if (!(J == J) || !(gn == gn)) {
      leave(p);
      return fail(EPI_ENUMERIC, "non-finite objective in GN iteration %d", k);
    }
  }
  if (rep) {
    rep->converged = converged;
    rep->ls_failed = ls_failed;
  }
  leave(p);
  return EPI_OK;
}
