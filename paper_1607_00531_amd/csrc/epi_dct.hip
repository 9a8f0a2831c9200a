// z-step of ADMM (Section 4.2, eq. dctdiag): z = C^T diag(rho / (rho + alpha Lambda)) C w,
// C = orthonormal DCT-II along the two non-PE axes, as dense matrix products on the
// matrix cores. Three passes over the canonical layout (PE axis contiguous):
//   pass 1: T1 = C3 W                          (axis 3, contraction over k)
//   pass 2: T2 = C2^T S C2 T1  per k-slice     (axis 2 forward, spectral scale, inverse)
//   pass 3: Z  = C3^T T2 (+ u-step epilogue)   (axis 3)
// In 2D (m3 = 1) only pass 2 runs and it carries the epilogue.
//
// Each workgroup owns 64 columns (consecutive faces along the contiguous axis) and all
// rows of the transformed axis: the input tile is read once from HBM into LDS, every
// output row is produced from it, and the small DCT matrix is streamed from L2 as
// pre-packed MFMA fragments.
//   precision 1 (mixed): a = a_hi + a_lo in bfloat16 for both operands; products
//     hi*hi + hi*lo + lo*hi with v_mfma_f32_16x16x32_bf16, float32 accumulation;
//   precision 0 (fp32): v_mfma_f32_16x16x4_f32.
#include <hip/hip_runtime.h>

#include "epi_device.hpp"
#include "epi_common.hpp"
#include "epi_launch.hpp"
#include "epi_dct_body.hpp"

namespace epi {

// Single-volume kernels: one workgroup per (batch entry, 64-column tile).
template <bool FUSED, int EPI, int KSM, int SLOTS>
__global__ __launch_bounds__(64 * EPI_DCT_NW) void k_dct_bf16(GemmArgs g) {
  if (g.done != nullptr && *g.done) return;
  extern __shared__ __attribute__((aligned(16))) unsigned short lds_bf[];
  int batch, c0;
  const int t = dct_tile(g, batch, c0);
  dct_bf16_body<FUSED, EPI, KSM, EPI_DCT_NW>(g, batch, c0, t, lds_bf);
}

template <bool FUSED, int EPI, int KSM, int SLOTS>
__global__ __launch_bounds__(256) void k_dct_f32(GemmArgs g) {
  if (g.done != nullptr && *g.done) return;
  extern __shared__ __attribute__((aligned(16))) float lds_f[];
  int batch, c0;
  const int t = dct_tile(g, batch, c0);
  dct_f32_body<FUSED, EPI, KSM, SLOTS>(g, batch, c0, t, lds_f);
}

template <bool FUSED, int EPI, int KSM, int SLOTS>
static void launch_dct_t(hipStream_t s, int prec, const GemmArgs& g) {
  const dim3 grid(g.nbatch * g.col_tiles);
  const size_t lds = dct_lds_bytes(prec, g);
  if (prec == 1)
    hipLaunchKernelGGL((k_dct_bf16<FUSED, EPI, KSM, SLOTS>), grid, dim3(64 * EPI_DCT_NW), lds, s, g);
  else
    hipLaunchKernelGGL((k_dct_f32<FUSED, EPI, KSM * 8, SLOTS>), grid, dim3(256), lds, s, g);
}

// rows <= 128: 4 contraction steps of 32 and 2 row tiles per wave; rows <= 256: 8 and 4
template <bool FUSED>
static void launch_dct(hipStream_t s, int prec, const GemmArgs& g) {
  const bool small = g.rows <= 128;
  if (g.epi == 1) {
    if (small) launch_dct_t<FUSED, 1, 4, 2>(s, prec, g);
    else launch_dct_t<FUSED, 1, 8, 4>(s, prec, g);
  } else {
    if (small) launch_dct_t<FUSED, 0, 4, 2>(s, prec, g);
    else launch_dct_t<FUSED, 0, 8, 4>(s, prec, g);
  }
}

void launch_dct_axis3(hipStream_t s, int prec, const GemmArgs& g) { launch_dct<false>(s, prec, g); }
void launch_dct_axis2_fused(hipStream_t s, int prec, const GemmArgs& g) {
  launch_dct<true>(s, prec, g);
}

// Kernels need more than 64 KB of dynamic LDS for the largest tiles.
template <bool FUSED, int EPI, int KSM, int SLOTS>
static bool set_lds(int big) {
  bool bad = hipSuccess != hipFuncSetAttribute((const void*)k_dct_bf16<FUSED, EPI, KSM, SLOTS>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, big);
  bad |= hipSuccess != hipFuncSetAttribute((const void*)k_dct_f32<FUSED, EPI, KSM * 8, SLOTS>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, big);
  return bad;
}

int dct_set_lds_limits() {
  const int big = 80 * 1024;   // largest tile: 2 x 64 x 264 bf16 or 256 x 68 float
  bool bad = false;
  bad |= set_lds<false, 0, 8, 4>(big);
  bad |= set_lds<false, 1, 8, 4>(big);
  bad |= set_lds<true, 0, 8, 4>(big);
  bad |= set_lds<true, 1, 8, 4>(big);
  (void)hipGetLastError();
  return bad ? 1 : 0;
}

}  // namespace epi
