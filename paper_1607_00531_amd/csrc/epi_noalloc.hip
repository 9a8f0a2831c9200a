// Objective evaluation without any device allocation: the variant of epi_objective for
// callers that cannot allocate (code under HIP graph capture, tight serving loops).
//
// The per-workgroup float64 partial sums of the line kernel live in `scratch`, a
// file-scope device array of EPI_NOALLOC_SCRATCH_BYTES that every GPU the library runs on
// holds until the process ends. Its device address is looked up once per device with
// hipGetSymbolAddress (with that device current) and only that address is handed to
// kernels: the array's name is a host-side stand-in in host code. Calls on one GPU share
// the array, so calls that overlap on one GPU (two streams, two threads) race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "epi.h"
#include "epi_common.hpp"
#include "epi_internal.hpp"
#include "epi_launch.hpp"

#define EPI_API extern "C" __attribute__((visibility("default")))

namespace epi {

static __device__ __align__(256) unsigned char scratch[EPI_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {nullptr};

// Device address of `scratch` on the current device (looked up once per device).
epi_status scratch_for_current_device(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(EPI_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(EPI_EINVAL, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(EPI_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return EPI_OK;
}
}  // namespace

}  // namespace epi

using namespace epi;

EPI_API epi_status epi_objective_noalloc(const epi_grid* grid, const float* d_Iplus,
                                         const float* d_Iminus, const float* d_b,
                                         int32_t with_penalty, double* d_terms, float* d_grad,
                                         void* stream) {
  if (!grid || !d_Iplus || !d_Iminus || !d_b || !d_terms) return fail(EPI_EINVAL, "null argument");
  epi_status vs = validate_grid(grid);
  if (vs != EPI_OK) return vs;
  if (grid->image_model != EPI_IMAGE_LINEAR)
    return fail(EPI_ENOTSUP, "the spline image model needs its coefficients from epi_setup");
  const LineArgs a = make_line_args(grid, d_Iplus, d_Iminus);
  const int lb = line_blocks(a);
  const size_t need = (size_t)lb * NQ_EVAL * sizeof(double);
  if (need > (size_t)EPI_NOALLOC_SCRATCH_BYTES)
    return fail(EPI_EINVAL,
                "%d PE lines need %zu bytes of partial sums, more than the %d bytes of the "
                "static scratch (at most %d lines)",
                a.L, need, EPI_NOALLOC_SCRATCH_BYTES,
                (int)(EPI_NOALLOC_SCRATCH_BYTES / (NQ_EVAL * sizeof(double))) * EPI_LINE_WAVES);
  void* sp = nullptr;
  vs = scratch_for_current_device(&sp);
  if (vs != EPI_OK) return vs;
  double* partial = static_cast<double*>(sp);
  hipStream_t s = (hipStream_t)stream;
  const int P = (a.M + 1 + 63) / 64;
  (void)hipGetLastError();
  launch_eval(s, P, d_grad ? 1 : 0, a, d_b, nullptr, 0, with_penalty ? 1 : 0, d_grad, nullptr,
              nullptr, partial, nullptr);
  FinArgs f{};
  f.kind = FIN_TERMS;
  f.partial = partial;
  f.nb1 = lb;
  f.trial = with_penalty ? 1 : 0;
  f.v = grid->h[0] * grid->h[1] * grid->h[2];
  f.alpha = grid->alpha;
  f.beta = grid->beta;
  f.hist = d_terms;
  launch_finalize(s, f, nullptr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(EPI_EHIP, "objective launch: %s", hipGetErrorString(e));
  return EPI_OK;
}
