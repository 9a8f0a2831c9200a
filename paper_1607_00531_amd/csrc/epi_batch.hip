// Continuous-batching ADMM engine (the served form of the Section 4.2 solver).
//
// Up to EPI_BATCH_MAX volumes of different sizes are resident at once. One ADMM iteration
// of all of them is one persistent launch per kernel class: the b-step walks the PE lines
// of every running volume with P faces per lane, the z-step kernels walk the 64-column DCT
// tiles of every running volume of a tile class, and one finalisation launch evaluates
// every volume's float64 stopping test. The work lists live in device memory, so the
// captured graph of an iteration stays valid while volumes come and go; it is captured
// again only when the set of kernel classes changes. Each volume keeps its own stopping
// flag; a finished volume's work items return at once and its slot is reused by the next
// admitted request. Per-volume arithmetic (and its reduction order) does not depend on
// the other volumes in the batch.
#include <hip/hip_runtime.h>

#include <string.h>

#include <algorithm>
#include <vector>

#include "epi.h"
#include "epi_common.hpp"
#include "epi_dct_body.hpp"
#include "epi_device.hpp"
#include "epi_internal.hpp"
#include "epi_launch.hpp"
#include "epi_line_body.hpp"

#define EPI_API extern "C" __attribute__((visibility("default")))

namespace epi {

#define BATCH_HARD_GRID 128

// index k of the range holding item i: first[k] <= i < first[k+1]
__device__ __forceinline__ int range_find(const RangeTable& T, int i) {
  int lo = 0, hi = T.n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (T.first[mid] <= i) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <int P>
__global__ __launch_bounds__(256) void k_batch_bstep(BatchDev* bd, int cls) {
  const RangeTable& T = bd->bt[cls];
  const int nr = T.n;
  if (nr == 0) return;
  const int total = T.first[nr];
  __shared__ float sbuf[EPI_LINE_WAVES][LinePad + 5 * LineBuf<P>::SIZE];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int unit = xcd_remap(blockIdx.x, gridDim.x);
  const int gl = unit * EPI_LINE_WAVES + wave;
  if (gl >= total) return;
  const int k = range_find(T, gl);
  const int slot = T.slot[k];
  const BatchSlotDev& S = bd->slots[slot];
  DevState* st = S.st;
  if (st->admm_done) return;
  const int line = gl - T.first[k];
  const bool hard = bstep_line_body<P>(S.la, (float)st->rho, (float)st->u_scale, S.b, S.z, S.u, S.w, line, true,
                                       &sbuf[wave][LinePad], lane, &st->numeric_bad);
  if (hard && lane == 0) {
    const int idx = atomicAdd(&bd->hard_count[cls], 1);
    if (idx < total) bd->hard_list[cls][idx] = HardItem{slot, line};   // total entries
    atomicAdd(&st->hard_count, 1);
  }
}

template <int P>
__global__ __launch_bounds__(64) void k_batch_hard(BatchDev* bd, int cls) {
  const RangeTable& T = bd->bt[cls];
  const int nh = T.n ? min(bd->hard_count[cls], T.first[T.n]) : 0;
  if ((int)blockIdx.x >= nh) return;
  __shared__ HardLds<P> L;
  for (int h = blockIdx.x; h < nh; h += gridDim.x) {
    const HardItem it = bd->hard_list[cls][h];
    const BatchSlotDev& S = bd->slots[it.slot];
    hard_line_body<P>(S.la, (float)S.st->rho, (float)S.st->u_scale, S.b, S.z, S.u, S.w, it.line, L, threadIdx.x,
                      &S.st->max_active, S.st->qp_max_iter);
  }
}

template <int PREC, bool FUSED, int EPI, int KSM, int SLOTS>
__global__ __launch_bounds__(PREC == 1 ? 64 * EPI_DCT_NW : 256) void k_batch_dct(BatchDev* bd,
                                                                                 int cls, int pass) {
  const RangeTable& T = bd->dt[cls];
  const int nr = T.n;
  if (nr == 0) return;
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  if (t >= T.first[nr]) return;
  const int k = range_find(T, t);
  const BatchSlotDev& S = bd->slots[T.slot[k]];
  if (S.st->admm_done) return;
  // a copy: the body reads its fields between global stores
  const GemmArgs g = pass == 1 ? S.g1 : (pass == 2 ? S.g2 : S.g3);
  const int local = t - T.first[k];
  const int batch = local / g.col_tiles;
  const int c0 = (local % g.col_tiles) * DCT_NT;
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  if (PREC == 1) {
    // a fixed-rho slot's j-axis pass goes through its per-slice operators (dir 2, the
    // unfused body): a separate inlined body, so each keeps its own register budget
    if (FUSED && g.dir == 2)
      dct_bf16_body<false, EPI, KSM, EPI_DCT_NW>(g, batch, c0, local,
                                                 reinterpret_cast<unsigned short*>(lds_raw));
    else
      dct_bf16_body<FUSED, EPI, KSM, EPI_DCT_NW>(g, batch, c0, local,
                                                 reinterpret_cast<unsigned short*>(lds_raw));
  } else if (FUSED && g.dir == 2) {
    dct_f32_body<false, EPI, KSM * 4, SLOTS>(g, batch, c0, local,
                                             reinterpret_cast<float*>(lds_raw));
  } else {
    dct_f32_body<FUSED, EPI, KSM * 4, SLOTS>(g, batch, c0, local,
                                             reinterpret_cast<float*>(lds_raw));
  }
}

// one workgroup per slot: float64 reduction of the last pass's sums and the stopping test
__global__ __launch_bounds__(256) void k_batch_finalize(BatchDev* bd) {
  if (blockIdx.x == 0 && threadIdx.x <= EPI_PMAX) bd->hard_count[threadIdx.x] = 0;
  const BatchSlotDev& S = bd->slots[blockIdx.x];
  if (!S.active || S.st->admm_done) return;
  __shared__ double sums[NQ_ADMM_E];
  reduce_partials<NQ_ADMM_E>(S.last_partial, S.last_ntiles, sums);
  if (threadIdx.x == 0) admm_finalize(S.st, sums, S.hist, S.hist_len);
}

// ------------------------------------------------------------------------------------
// host runtime
// ------------------------------------------------------------------------------------
static size_t dct_class_lds(int prec, bool small) {
  GemmArgs g{};
  g.KS = small ? (prec == 1 ? 2 : 16) : (prec == 1 ? 4 : 32);   // steps of one half
  g.RT = small ? 8 : 16;
  return dct_lds_bytes(prec, g);
}

template <bool FUSED, int EPI>
static void launch_batch_dct(hipStream_t s, int prec, BatchDev* bd, int cls, int pass, bool small,
                             int grid) {
  const size_t lds = dct_class_lds(prec, small);
  const dim3 g(grid), blk(prec == 1 ? 64 * EPI_DCT_NW : 256);
  if (prec == 1) {
    if (small) hipLaunchKernelGGL((k_batch_dct<1, FUSED, EPI, 4, 2>), g, blk, lds, s, bd, cls, pass);
    else hipLaunchKernelGGL((k_batch_dct<1, FUSED, EPI, 8, 4>), g, blk, lds, s, bd, cls, pass);
  } else {
    if (small) hipLaunchKernelGGL((k_batch_dct<0, FUSED, EPI, 4, 2>), g, blk, lds, s, bd, cls, pass);
    else hipLaunchKernelGGL((k_batch_dct<0, FUSED, EPI, 8, 4>), g, blk, lds, s, bd, cls, pass);
  }
}

// Launch width for n work units: n rounded up to 8..15 times a power of two, so that the
// captured graph (whose launch widths are fixed) is captured again only when the work
// of a class moves to another bucket; the spare workgroups return at once (< 1/8).
static int bucket_grid(long long n) {
  if (n <= 16) return (int)(n < 1 ? 1 : n);
  int e = 0;
  while ((n >> e) >= 16) ++e;
  const long long step = 1LL << e;
  return (int)(((n + step - 1) / step) * step);
}

template <bool FUSED, int EPI>
static hipError_t set_batch_lds(int big) {
  hipError_t e = hipFuncSetAttribute((const void*)k_batch_dct<1, FUSED, EPI, 8, 4>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, big);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_batch_dct<0, FUSED, EPI, 8, 4>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, big);
}

}  // namespace epi

using namespace epi;

#define BHIPCHK(call)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(e_ == hipErrorOutOfMemory ? EPI_ENOMEM : EPI_EHIP, "%s: %s (%s:%d)",  \
                  #call, hipGetErrorString(e_), __FILE__, __LINE__);                   \
  } while (0)

namespace {

// Device workspace of one resident volume. Released slots hand theirs to the engine's
// cache, and admission takes a cached workspace whose buffers are large enough, so a
// stream of requests of recurring sizes is admitted without device allocation: the DCT
// tables are kept when the transverse grid matches, the per-slice operators when the
// grid, alpha and rho match.
struct Workspace {
  float *w = nullptr, *t1 = nullptr, *t2 = nullptr;
  double *partial = nullptr, *hist = nullptr;
  size_t nb_cap = 0;      // bytes of w and t1 each
  size_t t2_data = 0;     // bytes of t2 before the operator region
  size_t zop_cap = 0;     // bytes of the operator region after t2_data
  size_t part_cap = 0;    // doubles of partial
  size_t hist_cap = 0;    // doubles of hist
  DctTables tab;          // valid when tab_m2 > 0
  int tab_m2 = 0, tab_m3 = 0, tab_prec = -1;
  double tab_h2 = 0.0, tab_h3 = 0.0;
  // operators in the region after t2_data, built for this grid and (alpha, rho)
  int zop_m2 = 0, zop_m3 = 0;
  double zop_h2 = 0.0, zop_h3 = 0.0, zop_alpha = 0.0, zop_rho = 0.0;
  size_t bytes() const { return 2 * nb_cap + t2_data + zop_cap + 8 * (part_cap + hist_cap); }
};

static void free_workspace(Workspace& ws) {
  void* bufs[] = {ws.w, ws.t1, ws.t2, ws.partial, ws.hist};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  free_dct_tables(&ws.tab);
  ws = Workspace();
}

struct SlotHost {
  bool used = false, finished = false;
  epi_grid grid{};
  int M = 0, m2 = 0, m3 = 0, L = 0, P = 0;
  long long n = 0, N = 0;
  const float *Ip = nullptr, *Im = nullptr;
  float *b = nullptr, *z = nullptr, *u = nullptr;
  Workspace ws;
  float *w = nullptr, *t1 = nullptr, *t2 = nullptr;
  double* partial = nullptr;
  double* hist = nullptr;
  int hist_len = 0;
  DctTables tab;
  void* zop = nullptr;   // per-slice j-axis operators (fixed rho; inside the t2 allocation)
  int64_t footprint = 0;
  epi_admm_opts opts{};
};

int64_t workspace_bytes(const epi_grid* g, int max_iter) {
  const long long M = g->m[0], m2 = g->m[1], m3 = g->m[2];
  const long long n = (M + 1) * m2 * m3;
  const long long tiles = std::max<long long>(tiles_axis3((int)M, (int)m2), tiles_axis2((int)M, (int)m3));
  const long long part = std::max<long long>(tiles * NQ_ADMM_E, 4096);
  // the packed DCT matrices (forward and inverse per axis, the larger of the two
  // precisions' fragment layouts) and the eigenvalues
  const auto mat = [](long long m) {
    const long long ce = (m + 1) / 2, RTh = (ce + 15) / 16;
    const long long bf = 2 * (2 * RTh) * ((ce + 31) / 32) * 64 * 8 * 2;   // hi and lo blocks
    const long long f32 = (2 * RTh) * (4 * RTh) * 64 * 4;
    return bf > f32 ? bf : f32;
  };
  const long long tables = 2 * (mat(m2) + mat(m3)) + 4 * (m2 + m3);
  // the per-slice operators of a fixed-rho volume (counted for every volume, at the size of
  // the split-bfloat16 fragments, which is at least that of the float32 ones)
  const long long zop = (long long)zop_bytes(EPI_PREC_MIXED, (int)m2, (int)m3);
  return 3 * n * 4 + part * 8 + (long long)EPI_HIST_ROWS * std::max(max_iter, 1) * 8 + tables + zop;
}

}  // namespace

// Launch widths of every kernel class of one captured iteration (0: class absent).
struct BatchKey {
  int bstep[EPI_PMAX + 1] = {0};
  int dct[8] = {0};
  bool operator==(const BatchKey& o) const {
    return memcmp(bstep, o.bstep, sizeof(bstep)) == 0 && memcmp(dct, o.dct, sizeof(dct)) == 0;
  }
  bool operator!=(const BatchKey& o) const { return !(*this == o); }
};

struct epi_batch {
  int max_slots = 0, precision = 1, iters_per_step = 8;
  std::vector<Workspace> cache;   // workspaces of released slots (at most max_slots)
  long long admissions = 0, admissions_allocating = 0, captures = 0;
  int64_t budget = 0, used_bytes = 0;
  hipStream_t user = nullptr, exec = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  BatchDev* d_bd = nullptr;
  BatchDev* h_bd = nullptr;
  DevState* d_st = nullptr;
  DevState* h_st = nullptr;
  HardItem* hard[EPI_PMAX + 1] = {nullptr};
  int hard_cap[EPI_PMAX + 1] = {0};
  std::vector<SlotHost> slots;
  bool dirty = true;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  BatchKey graph_key;
  int running = 0;
};

// j-axis pass of a slot with per-slice operators: one product per tile (dir 2)
static void use_zop(const SlotHost& s, GemmArgs& g) {
  if (!s.zop) return;
  g.dir = 2;
  g.A1 = s.zop;
  g.A2 = nullptr;
  // per slice: hi and lo blocks of 16-byte fragments (bfloat16), or floats (float32)
  g.a_bstride = (s.grid.precision == EPI_PREC_MIXED ? 2LL : 1LL) * s.tab.RT2 * s.tab.KS2 * 64;
}

// Release a slot: its workspace goes to the cache (the least recently cached one is
// freed when the cache is full), or is freed when `keep` is false.
static void batch_free_slot(epi_batch* bt, SlotHost& s, bool keep = true) {
  if (keep && s.ws.w) {
    if ((int)bt->cache.size() >= bt->max_slots) {
      free_workspace(bt->cache.front());
      bt->cache.erase(bt->cache.begin());
    }
    bt->cache.push_back(s.ws);
  } else {
    free_workspace(s.ws);
  }
  s = SlotHost();
}

// A workspace for slot s (sizes from s and the request): the smallest cached one that is
// large enough, else a new allocation. Tables and operators are (re)built only when the
// cached ones were made for another grid or another (alpha, rho).
static epi_status take_workspace(epi_batch* bt, SlotHost& s, const epi_grid* grid,
                                 const epi_admm_opts* opts) {
  const size_t nb = (size_t)s.n * sizeof(float);
  const size_t nb_al = (nb + 255) & ~(size_t)255;
  const size_t zb = opts->rho_mode == EPI_RHO_FIXED ? zop_bytes(bt->precision, s.m2, s.m3) : 0;
  const long long tiles = std::max(tiles_axis3(s.M, s.m2), tiles_axis2(s.M, s.m3));
  const size_t part = (size_t)std::max<long long>(tiles * NQ_ADMM_E, 4096);
  const size_t hist = (size_t)EPI_HIST_ROWS * s.hist_len;
  int best = -1;
  for (int i = 0; i < (int)bt->cache.size(); ++i) {
    const Workspace& c = bt->cache[i];
    if (c.nb_cap >= nb && c.t2_data >= nb_al && c.zop_cap >= zb && c.part_cap >= part &&
        c.hist_cap >= hist && (best < 0 || c.bytes() < bt->cache[best].bytes()))
      best = i;
  }
  bt->admissions += 1;
  Workspace& ws = s.ws;
  if (best >= 0) {
    ws = bt->cache[best];
    bt->cache.erase(bt->cache.begin() + best);
  } else {
    bt->admissions_allocating += 1;
    ws.nb_cap = nb;
    ws.t2_data = nb_al;
    ws.zop_cap = zb;
    ws.part_cap = part;
    ws.hist_cap = hist;
    if (hipMalloc(&ws.w, nb) != hipSuccess || hipMalloc(&ws.t1, nb) != hipSuccess ||
        hipMalloc(&ws.t2, nb_al + zb) != hipSuccess ||
        hipMalloc(&ws.partial, part * sizeof(double)) != hipSuccess ||
        hipMalloc(&ws.hist, hist * sizeof(double)) != hipSuccess)
      return fail(EPI_ENOMEM, "slot workspace");
  }
  const double h2 = grid->h[1], h3 = grid->h[2];
  if (ws.tab_m2 != s.m2 || ws.tab_m3 != s.m3 || ws.tab_h2 != h2 || ws.tab_h3 != h3 ||
      ws.tab_prec != bt->precision) {
    free_dct_tables(&ws.tab);
    ws.tab_m2 = 0;
    epi_status ts = build_dct_tables(s.m2, s.m3, h2, h3, bt->precision, &ws.tab);
    if (ts != EPI_OK) return ts;
    ws.tab_m2 = s.m2;
    ws.tab_m3 = s.m3;
    ws.tab_h2 = h2;
    ws.tab_h3 = h3;
    ws.tab_prec = bt->precision;
  }
  s.w = ws.w;
  s.t1 = ws.t1;
  s.t2 = ws.t2;
  s.partial = ws.partial;
  s.hist = ws.hist;
  s.tab = ws.tab;
  s.zop = nullptr;
  if (zb) {
    s.zop = reinterpret_cast<char*>(ws.t2) + ws.t2_data;
    if (ws.zop_m2 != s.m2 || ws.zop_m3 != s.m3 || ws.zop_h2 != h2 || ws.zop_h3 != h3 ||
        ws.zop_alpha != grid->alpha || ws.zop_rho != opts->rho) {
      ws.zop_m2 = 0;
      if (hipMemsetAsync(s.zop, 0, zb, bt->exec) != hipSuccess ||
          launch_build_zop(bt->exec, bt->precision, s.m2, s.m3, h2, h3, grid->alpha, opts->rho,
                           s.tab.RT2, s.tab.KS2, s.zop) != 0 ||
          hipGetLastError() != hipSuccess)
        return fail(EPI_EHIP, "slot operator build");
      ws.zop_m2 = s.m2;
      ws.zop_m3 = s.m3;
      ws.zop_h2 = h2;
      ws.zop_h3 = h3;
      ws.zop_alpha = grid->alpha;
      ws.zop_rho = opts->rho;
    }
  }
  return EPI_OK;
}

EPI_API int64_t epi_batch_footprint(const epi_grid* grid, int32_t max_iter) {
  if (!grid) return -1;
  const long long M = grid->m[0], m2 = grid->m[1], m3 = grid->m[2];
  const long long n = (M + 1) * m2 * m3, N = M * m2 * m3;
  return 4 * (2 * N + 3 * n) + workspace_bytes(grid, max_iter);
}

EPI_API void epi_batch_destroy(epi_batch* bt) {
  if (!bt) return;
  if (bt->exec) (void)hipStreamSynchronize(bt->exec);
  if (bt->gexec) (void)hipGraphExecDestroy(bt->gexec);
  if (bt->graph) (void)hipGraphDestroy(bt->graph);
  for (auto& s : bt->slots)
    if (s.used) batch_free_slot(bt, s, false);
  for (auto& ws : bt->cache) free_workspace(ws);
  for (int c = 0; c <= EPI_PMAX; ++c)
    if (bt->hard[c]) (void)hipFree(bt->hard[c]);
  if (bt->d_bd) (void)hipFree(bt->d_bd);
  if (bt->d_st) (void)hipFree(bt->d_st);
  if (bt->h_bd) (void)hipHostFree(bt->h_bd);
  if (bt->h_st) (void)hipHostFree(bt->h_st);
  if (bt->ev_in) (void)hipEventDestroy(bt->ev_in);
  if (bt->ev_out) (void)hipEventDestroy(bt->ev_out);
  if (bt->exec) (void)hipStreamDestroy(bt->exec);
  delete bt;
}

static epi_status batch_create_impl(int32_t max_slots, int64_t budget, int32_t precision,
                                    int32_t iters_per_step, void* stream, epi_batch** out) {
  if (!out) return fail(EPI_EINVAL, "null argument");
  *out = nullptr;
  if (max_slots < 1 || max_slots > EPI_BATCH_MAX)
    return fail(EPI_EINVAL, "max_slots must be in [1, %d]", EPI_BATCH_MAX);
  if (precision != EPI_PREC_FP32 && precision != EPI_PREC_MIXED)
    return fail(EPI_EINVAL, "unknown precision %d", precision);
  if (iters_per_step < 1) return fail(EPI_EINVAL, "iters_per_step must be >= 1");
  if (budget <= 0) return fail(EPI_EINVAL, "hbm_budget_bytes must be > 0");
  epi_batch* bt = new epi_batch();
  *out = bt;
  bt->max_slots = max_slots;
  bt->budget = budget;
  bt->precision = precision;
  bt->iters_per_step = iters_per_step;
  bt->user = (hipStream_t)stream;
  bt->slots.resize(max_slots);
  int dev = 0;
  BHIPCHK(hipGetDevice(&dev));
  BHIPCHK(hipSetDevice(dev));
  BHIPCHK(hipStreamCreateWithFlags(&bt->exec, hipStreamNonBlocking));
  (void)dct_set_lds_limits();
  BHIPCHK((set_batch_lds<true, 0>(80 * 1024)));
  BHIPCHK((set_batch_lds<true, 1>(80 * 1024)));
  BHIPCHK((set_batch_lds<false, 0>(80 * 1024)));
  BHIPCHK((set_batch_lds<false, 1>(80 * 1024)));
  BHIPCHK(hipEventCreateWithFlags(&bt->ev_in, hipEventDisableTiming));
  BHIPCHK(hipEventCreateWithFlags(&bt->ev_out, hipEventDisableTiming));
  BHIPCHK(hipMalloc(&bt->d_bd, sizeof(BatchDev)));
  BHIPCHK(hipHostMalloc((void**)&bt->h_bd, sizeof(BatchDev), hipHostMallocDefault));
  memset(bt->h_bd, 0, sizeof(BatchDev));
  BHIPCHK(hipMemcpy(bt->d_bd, bt->h_bd, sizeof(BatchDev), hipMemcpyHostToDevice));
  BHIPCHK(hipMalloc(&bt->d_st, sizeof(DevState) * EPI_BATCH_MAX));
  BHIPCHK(hipHostMalloc((void**)&bt->h_st, sizeof(DevState) * EPI_BATCH_MAX, hipHostMallocDefault));
  memset(bt->h_st, 0, sizeof(DevState) * EPI_BATCH_MAX);
  BHIPCHK(hipMemcpy(bt->d_st, bt->h_st, sizeof(DevState) * EPI_BATCH_MAX, hipMemcpyHostToDevice));
  return EPI_OK;
}

EPI_API epi_status epi_batch_create(int32_t max_slots, int64_t hbm_budget_bytes, int32_t precision,
                                    int32_t iters_per_step, void* stream, epi_batch** out) {
  epi_status s = batch_create_impl(max_slots, hbm_budget_bytes, precision, iters_per_step, stream, out);
  if (s != EPI_OK && out && *out) {
    epi_batch_destroy(*out);
    *out = nullptr;
  }
  return s;
}

static void batch_enter(epi_batch* bt) {
  (void)hipEventRecord(bt->ev_in, bt->user);
  (void)hipStreamWaitEvent(bt->exec, bt->ev_in, 0);
}
static void batch_leave(epi_batch* bt) {
  (void)hipEventRecord(bt->ev_out, bt->exec);
  (void)hipStreamWaitEvent(bt->user, bt->ev_out, 0);
}

EPI_API epi_status epi_batch_admit(epi_batch* bt, const epi_grid* grid, const float* d_Iplus,
                                   const float* d_Iminus, float* d_b, float* d_z, float* d_u,
                                   const epi_admm_opts* opts, int32_t* slot_out) {
  if (!bt || !grid || !d_Iplus || !d_Iminus || !d_b || !d_z || !d_u || !opts || !slot_out)
    return fail(EPI_EINVAL, "null argument");
  *slot_out = -1;
  epi_status vs = validate_grid(grid);
  if (vs != EPI_OK) return vs;
  if (!(opts->rho > 0.0) || opts->max_iter < 1 || opts->sqp_iters != 1 || opts->qp_max_iter < 0)
    return fail(EPI_EINVAL, "batched ADMM needs rho > 0, max_iter >= 1, sqp_iters = 1, qp_max_iter >= 0");
  if (opts->with_lagrangian)
    return fail(EPI_EINVAL, "the batched engine does not record the augmented Lagrangian");
  {
    epi_status vo = validate_rho_opts(opts);
    if (vo != EPI_OK) return vo;
  }
  if (grid->image_model != EPI_IMAGE_LINEAR)
    return fail(EPI_ENOTSUP, "the batched engine takes the linear image model only");
  const int64_t fp = epi_batch_footprint(grid, opts->max_iter);
  int sid = -1;
  for (int i = 0; i < bt->max_slots; ++i)
    if (!bt->slots[i].used) {
      sid = i;
      break;
    }
  if (sid < 0) return fail(EPI_EBUSY, "no free slot (%d resident)", bt->max_slots);
  if (bt->used_bytes + fp > bt->budget)
    return fail(EPI_EBUSY, "HBM budget: %lld resident + %lld requested > %lld", (long long)bt->used_bytes,
                (long long)fp, (long long)bt->budget);
  SlotHost& s = bt->slots[sid];
  s = SlotHost();
  s.grid = *grid;
  s.grid.precision = bt->precision;
  s.M = grid->m[0];
  s.m2 = grid->m[1];
  s.m3 = grid->m[2];
  s.L = s.m2 * s.m3;
  s.P = (s.M + 1 + 63) / 64;
  s.n = (long long)(s.M + 1) * s.L;
  s.N = (long long)s.M * s.L;
  s.Ip = d_Iplus;
  s.Im = d_Iminus;
  s.b = d_b;
  s.z = d_z;
  s.u = d_u;
  s.opts = *opts;
  s.footprint = fp;
  s.hist_len = opts->max_iter;
  s.used = true;   // from here on a failure releases the slot
  // a fixed-rho split-bfloat16 volume takes its j-axis pass through per-slice operators (as
  // the single-volume solver does), kept behind t2
  {
    epi_status ws = take_workspace(bt, s, grid, opts);
    if (ws != EPI_OK) {
      batch_free_slot(bt, s, false);   // possibly incomplete: not cached
      return ws;
    }
  }
  auto undo = [&](epi_status st) {
    batch_free_slot(bt, s);
    return st;
  };
  // feasibility of the starting field and the slot's stopping state
  batch_enter(bt);
  DevState* dst = bt->d_st + sid;
  DevState* hst = bt->h_st + sid;
  const LineArgs la = make_line_args(&s.grid, s.Ip, s.Im);
  launch_count_violations(bt->exec, la, d_b, 1.0f + 1e-5f, s.partial);
  FinArgs f{};
  f.kind = FIN_DOT;
  f.partial = s.partial;
  f.nb1 = flat_blocks(s.N);
  launch_finalize(bt->exec, f, dst);
  if (hipGetLastError() != hipSuccess) return undo(fail(EPI_EHIP, "admission check launch"));
  if (hipStreamSynchronize(bt->exec) != hipSuccess) return undo(fail(EPI_EHIP, "sync"));
  DevState tmp;
  if (hipMemcpy(&tmp, dst, sizeof(DevState), hipMemcpyDeviceToHost) != hipSuccess)
    return undo(fail(EPI_EHIP, "state copy"));
  if (tmp.gTd > 0.0) {
    batch_leave(bt);
    return undo(fail(EPI_EINFEASIBLE, "starting field has %.0f cells with |D1 b| > 1", tmp.gTd));
  }
  memset(hst, 0, sizeof(DevState));
  hst->rho = opts->rho;
  hst->eps_abs = opts->eps_abs;
  hst->eps_rel = opts->eps_rel;
  hst->sqrt_n = sqrt((double)s.n);
  hst->v = grid->h[0] * grid->h[1] * grid->h[2];
  hst->admm_max = opts->max_iter;
  hst->qp_max_iter = opts->qp_max_iter;
  init_rho_state(hst, opts);
  if (hipMemcpy(dst, hst, sizeof(DevState), hipMemcpyHostToDevice) != hipSuccess)
    return undo(fail(EPI_EHIP, "state init"));
  batch_leave(bt);
  bt->used_bytes += fp;
  bt->dirty = true;
  *slot_out = sid;
  return EPI_OK;
}

// work tables of the running volumes, uploaded to the device; returns the launch widths
static epi_status batch_rebuild(epi_batch* bt, BatchKey* key) {
  BatchDev* h = bt->h_bd;
  memset(h, 0, sizeof(BatchDev));
  int need[EPI_PMAX + 1] = {0};
  bt->running = 0;
  for (int i = 0; i < bt->max_slots; ++i) {
    SlotHost& s = bt->slots[i];
    if (!s.used || s.finished) continue;
    bt->running += 1;
    BatchSlotDev& d = h->slots[i];
    d.la = make_line_args(&s.grid, s.Ip, s.Im);
    d.b = s.b;
    d.z = s.z;
    d.u = s.u;
    d.w = s.w;
    d.st = bt->d_st + i;
    d.active = 1;
    d.hist = s.hist;
    d.hist_len = s.hist_len;
    const float alpha = (float)s.grid.alpha;
    const bool three = s.m3 > 1;
    d.three_pass = three;
    auto add = [&](RangeTable& T, int items) {
      T.slot[T.n] = i;
      T.first[T.n + 1] = T.first[T.n] + items;
      T.n += 1;
    };
    add(h->bt[s.P], s.L);
    need[s.P] += s.L;
    const int small3 = s.m3 <= 128 ? 0 : 1, small2 = s.m2 <= 128 ? 0 : 1;
    if (three) {
      d.g1 = make_gemm_axis3(s.M, s.m2, s.m3, alpha, s.tab, s.w, s.t1, false, d.st);
      d.g2 = make_gemm_axis2(s.M, s.m2, s.m3, alpha, s.tab, s.t1, s.t2, d.st);
      use_zop(s, d.g2);
      d.g3 = make_gemm_axis3(s.M, s.m2, s.m3, alpha, s.tab, s.t2, s.z, true, d.st);
      d.g3.epi = 1;
      d.g3.b = s.b;
      d.g3.z = s.z;
      d.g3.u = s.u;
      d.g3.partial = s.partial;
      d.last_ntiles = d.g3.nbatch * d.g3.col_tiles;
      d.last_partial = s.partial;
      add(h->dt[0 + small3], d.g1.nbatch * d.g1.col_tiles);
      add(h->dt[2 + small2], d.g2.nbatch * d.g2.col_tiles);
      add(h->dt[6 + small3], d.g3.nbatch * d.g3.col_tiles);
    } else {
      d.g2 = make_gemm_axis2(s.M, s.m2, s.m3, alpha, s.tab, s.w, s.z, d.st);
      use_zop(s, d.g2);
      d.g2.epi = 1;
      d.g2.b = s.b;
      d.g2.z = s.z;
      d.g2.u = s.u;
      d.g2.partial = s.partial;
      d.last_ntiles = d.g2.nbatch * d.g2.col_tiles;
      d.last_partial = s.partial;
      add(h->dt[4 + small2], d.g2.nbatch * d.g2.col_tiles);
    }
  }
  for (int c = 1; c <= EPI_PMAX; ++c) {
    if (need[c] > bt->hard_cap[c]) {
      if (bt->hard[c]) BHIPCHK(hipFree(bt->hard[c]));
      bt->hard[c] = nullptr;
      BHIPCHK(hipMalloc(&bt->hard[c], (size_t)need[c] * sizeof(HardItem)));
      bt->hard_cap[c] = need[c];
    }
    h->hard_list[c] = bt->hard[c];
  }
  BHIPCHK(hipMemcpyAsync(bt->d_bd, h, sizeof(BatchDev), hipMemcpyHostToDevice, bt->exec));
  BatchKey k;
  for (int c = 1; c <= EPI_PMAX; ++c)   // one workgroup per EPI_LINE_WAVES lines
    if (h->bt[c].n) k.bstep[c] = bucket_grid((h->bt[c].first[h->bt[c].n] + EPI_LINE_WAVES - 1) / EPI_LINE_WAVES);
  for (int c = 0; c < 8; ++c)           // one workgroup per 64-column tile
    if (h->dt[c].n) k.dct[c] = bucket_grid(h->dt[c].first[h->dt[c].n]);
  *key = k;
  return EPI_OK;
}

static void batch_iteration(epi_batch* bt, const BatchKey& key) {
  hipStream_t s = bt->exec;
  BatchDev* bd = bt->d_bd;
  for (int P = 1; P <= EPI_PMAX; ++P) {
    const dim3 g(key.bstep[P]), blk(256);
    if (!key.bstep[P]) continue;
    switch (P) {
      case 1: hipLaunchKernelGGL(k_batch_bstep<1>, g, blk, 0, s, bd, P); break;
      case 2: hipLaunchKernelGGL(k_batch_bstep<2>, g, blk, 0, s, bd, P); break;
      case 3: hipLaunchKernelGGL(k_batch_bstep<3>, g, blk, 0, s, bd, P); break;
      case 4: hipLaunchKernelGGL(k_batch_bstep<4>, g, blk, 0, s, bd, P); break;
      case 5: hipLaunchKernelGGL(k_batch_bstep<5>, g, blk, 0, s, bd, P); break;
      case 6: hipLaunchKernelGGL(k_batch_bstep<6>, g, blk, 0, s, bd, P); break;
      case 7: hipLaunchKernelGGL(k_batch_bstep<7>, g, blk, 0, s, bd, P); break;
      default: hipLaunchKernelGGL(k_batch_bstep<8>, g, blk, 0, s, bd, P); break;
    }
  }
  for (int P = 1; P <= EPI_PMAX; ++P) {
    if (!key.bstep[P]) continue;
    switch (P) {
      case 1: hipLaunchKernelGGL(k_batch_hard<1>, dim3(BATCH_HARD_GRID), dim3(64), 0, s, bd, P); break;
      case 2: hipLaunchKernelGGL(k_batch_hard<2>, dim3(BATCH_HARD_GRID), dim3(64), 0, s, bd, P); break;
      case 3: hipLaunchKernelGGL(k_batch_hard<3>, dim3(BATCH_HARD_GRID), dim3(64), 0, s, bd, P); break;
      case 4: hipLaunchKernelGGL(k_batch_hard<4>, dim3(BATCH_HARD_GRID), dim3(64), 0, s, bd, P); break;
      case 5: hipLaunchKernelGGL(k_batch_hard<5>, dim3(BATCH_HARD_GRID), dim3(64), 0, s, bd, P); break;
      case 6: hipLaunchKernelGGL(k_batch_hard<6>, dim3(BATCH_HARD_GRID), dim3(64), 0, s, bd, P); break;
      case 7: hipLaunchKernelGGL(k_batch_hard<7>, dim3(BATCH_HARD_GRID), dim3(64), 0, s, bd, P); break;
      default: hipLaunchKernelGGL(k_batch_hard<8>, dim3(BATCH_HARD_GRID), dim3(64), 0, s, bd, P); break;
    }
  }
  const int prec = bt->precision;
  for (int c = 0; c < 8; ++c) {
    const int g = key.dct[c];
    if (!g) continue;
    const bool small = (c & 1) == 0;
    if (c < 2) launch_batch_dct<false, 0>(s, prec, bd, c, 1, small, g);
    else if (c < 4) launch_batch_dct<true, 0>(s, prec, bd, c, 2, small, g);
    else if (c < 6) launch_batch_dct<true, 1>(s, prec, bd, c, 2, small, g);
    else launch_batch_dct<false, 1>(s, prec, bd, c, 3, small, g);
  }
  hipLaunchKernelGGL(k_batch_finalize, dim3(bt->max_slots), dim3(256), 0, s, bd);
}

EPI_API epi_status epi_batch_step(epi_batch* bt, int32_t* running) {
  if (!bt) return fail(EPI_EINVAL, "null argument");
  batch_enter(bt);
  if (bt->dirty) {
    BatchKey key;
    epi_status s = batch_rebuild(bt, &key);
    if (s != EPI_OK) return s;
    bt->dirty = false;
    // a new capture whenever the launch widths change: a graph replayed with spare width
    // launches the spare workgroups every iteration, and each still reads the work table
    // before it returns (twenty 240x200x110 volumes solved together: 11.8 volumes/s when
    // graphs up to twice the needed width were kept, 15.3 with a capture per change, 17
    // captures for the twenty)
    if (bt->running > 0 && (key != bt->graph_key || !bt->gexec)) {
      if (bt->gexec) BHIPCHK(hipGraphExecDestroy(bt->gexec));
      if (bt->graph) BHIPCHK(hipGraphDestroy(bt->graph));
      bt->gexec = nullptr;
      bt->graph = nullptr;
      BHIPCHK(hipStreamBeginCapture(bt->exec, hipStreamCaptureModeThreadLocal));
      for (int i = 0; i < bt->iters_per_step; ++i) batch_iteration(bt, key);
      hipError_t e1 = hipGetLastError();
      hipError_t e2 = hipStreamEndCapture(bt->exec, &bt->graph);
      if (e1 != hipSuccess || e2 != hipSuccess)
        return fail(EPI_EHIP, "graph capture: %s", hipGetErrorString(e1 != hipSuccess ? e1 : e2));
      BHIPCHK(hipGraphInstantiate(&bt->gexec, bt->graph, nullptr, nullptr, 0));
      bt->graph_key = key;
      bt->captures += 1;
    }
  }
  if (bt->running > 0) {
    BHIPCHK(hipGraphLaunch(bt->gexec, bt->exec));
    BHIPCHK(hipMemcpyAsync(bt->h_st, bt->d_st, sizeof(DevState) * bt->max_slots,
                           hipMemcpyDeviceToHost, bt->exec));
    BHIPCHK(hipStreamSynchronize(bt->exec));
    for (int i = 0; i < bt->max_slots; ++i) {
      SlotHost& s = bt->slots[i];
      if (s.used && !s.finished && bt->h_st[i].admm_done) {
        s.finished = true;
        bt->dirty = true;
        bt->running -= 1;
      }
    }
  }
  batch_leave(bt);
  if (running) *running = bt->running;
  return EPI_OK;
}

EPI_API epi_status epi_batch_poll(epi_batch* bt, int32_t slot, int32_t* finished,
                                  epi_admm_report* rep) {
  if (!bt || !finished) return fail(EPI_EINVAL, "null argument");
  if (slot < 0 || slot >= bt->max_slots || !bt->slots[slot].used)
    return fail(EPI_EINVAL, "slot %d is not in use", slot);
  SlotHost& s = bt->slots[slot];
  *finished = s.finished;
  if (!s.finished || !rep) return EPI_OK;
  const DevState& h = bt->h_st[slot];
  const int iters = h.admm_iter;
  rep->iters = iters;
  rep->converged = h.admm_done == 1 && h.numeric_bad == 0;
  rep->max_active = h.max_active;
  rep->hard_lines = h.hard_total;
  rep->status = h.numeric_bad ? EPI_ENUMERIC : EPI_OK;
  double* outs[EPI_HIST_ROWS - 1] = {rep->r_pri, rep->r_dual, rep->eps_pri, rep->eps_dual, rep->rho};
  for (int k = 0; k < EPI_HIST_ROWS - 1; ++k)
    if (outs[k] && iters > 0)
      BHIPCHK(hipMemcpy(outs[k], s.hist + (size_t)k * s.hist_len,
                        std::min(iters, s.hist_len) * sizeof(double), hipMemcpyDeviceToHost));
  return EPI_OK;
}

EPI_API epi_status epi_batch_stats(const epi_batch* bt, int64_t* admissions,
                                   int64_t* admissions_allocating, int64_t* graph_captures) {
  if (!bt || !admissions || !admissions_allocating || !graph_captures)
    return fail(EPI_EINVAL, "null argument");
  *admissions = bt->admissions;
  *admissions_allocating = bt->admissions_allocating;
  *graph_captures = bt->captures;
  return EPI_OK;
}

EPI_API epi_status epi_batch_release(epi_batch* bt, int32_t slot) {
  if (!bt) return fail(EPI_EINVAL, "null argument");
  if (slot < 0 || slot >= bt->max_slots || !bt->slots[slot].used)
    return fail(EPI_EINVAL, "slot %d is not in use", slot);
  BHIPCHK(hipStreamSynchronize(bt->exec));
  SlotHost& s = bt->slots[slot];   // a running volume may be released (cancelled)
  bt->used_bytes -= s.footprint;
  batch_free_slot(bt, s);
  bt->dirty = true;
  return EPI_OK;
}
