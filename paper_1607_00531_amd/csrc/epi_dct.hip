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

template <bool FUSED, int EPI, int KSH, int SLOTS>
__global__ __launch_bounds__(256) void k_dct_f32(GemmArgs g) {
  if (g.done != nullptr && *g.done) return;
  extern __shared__ __attribute__((aligned(16))) float lds_f[];
  int batch, c0;
  const int t = dct_tile(g, batch, c0);
  dct_f32_body<FUSED, EPI, KSH, SLOTS>(g, batch, c0, t, lds_f);
}

template <bool FUSED, int EPI, int KSM, int SLOTS>
static void launch_dct_t(hipStream_t s, int prec, const GemmArgs& g) {
  const dim3 grid(g.nbatch * g.col_tiles);
  const size_t lds = dct_lds_bytes(prec, g);
  if (prec == 1)
    hipLaunchKernelGGL((k_dct_bf16<FUSED, EPI, KSM, SLOTS>), grid, dim3(64 * EPI_DCT_NW), lds, s, g);
  else
    hipLaunchKernelGGL((k_dct_f32<FUSED, EPI, KSM * 4, SLOTS>), grid, dim3(256), lds, s, g);
}

// rows <= 128: 4 contraction steps of 32 (bfloat16; 16 steps of 4 per half in float32)
// and 2 row tiles per wave; rows <= 256: 8 (32) and 4
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

// ------------------------------------------------------------------------------------
// Per-slice operator of the j-axis pass for a fixed rho (split-bfloat16). With the
// even/odd split, the fused pass maps the sums s and differences d of slice k through
// forward, spectral scale and inverse: E = C_e^T S_e C_e s and O = C_o^T S_o C_o d, with
// C_h[r][q] = C[2r+h][q] (q, r < c for h = 0, < f for h = 1) and
// S_h = diag(rho / (rho + alpha (lambda_2(2r+h) + lambda_3(k)))) (eq. dctdiag restricted to
// one slice). M_h = C_h^T S_h C_h is built here in float64 (C in float32 in LDS, products
// and sums in float64) and packed as hi/lo bfloat16 fragments in the layout of the forward
// matrix (row tile rt, contraction step ks), one block of 2 * RT * KS * 64 fragments per
// slice; padding entries stay zero (the buffer is cleared once when allocated).
// ------------------------------------------------------------------------------------
__device__ __forceinline__ unsigned short bf16_rne(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

__device__ __forceinline__ double dct_eig(int k, int m, double h) {
  return (2.0 - 2.0 * cos(M_PI * k / m)) / (h * h);
}

#define ZOP_MAXC 128   // half length limit (transform length <= 256)

// packed position of (row, contraction index q) of half h in one slice's hi block
__device__ __forceinline__ size_t zop_index(int h, int row, int q, int RTh, int KS) {
  const int rt = h * RTh + row / 16, ks = q / 32, l = (row & 15) + 16 * ((q & 31) >> 3);
  return (((size_t)rt * KS + ks) * 64 + l) * 8 + (q & 7);
}
// the same for the float32 fragments (steps of 4): lane (row & 15) + 16 (q & 3)
__device__ __forceinline__ size_t zop_index_f32(int h, int row, int q, int RTh, int KS) {
  const int rt = h * RTh + row / 16, ks = q / 4, l = (row & 15) + 16 * (q & 3);
  return ((size_t)rt * KS + ks) * 64 + l;
}

// One workgroup per (slice, half). Each thread accumulates 4 x 4 blocks of M_h (rows
// 4 bi.., columns 4 bj.., bi <= bj; M_h is symmetric, the mirror is written from the same
// sums) over r, with C_h zero-padded to a multiple of 4 in LDS.
__global__ __launch_bounds__(256) void k_build_zop(int m2, int m3, double h2, double h3,
                                                   double alpha, double rho, int RT, int KS,
                                                   int f32, void* __restrict__ out_raw) {
  extern __shared__ __attribute__((aligned(16))) double zop_lds[];
  double* sc = zop_lds;                                       // [ZOP_MAXC]
  float* Ch = reinterpret_cast<float*>(zop_lds + ZOP_MAXC);   // [cnt][cp]
  const int kb = blockIdx.x, h = blockIdx.y;
  const int ce = (m2 + 1) / 2, fo = m2 / 2, cnt = h ? fo : ce;
  const int cp = (cnt + 3) & ~3, nb = cp / 4;
  const int RTh = RT / 2;
  // spectral index of slice kb along axis 3 (slices are stored in half order)
  const int ce3 = (m3 + 1) / 2;
  const int k3 = kb < ce3 ? 2 * kb : 2 * (kb - ce3) + 1;
  const double lam3 = dct_eig(k3, m3, h3);
  for (int r = threadIdx.x; r < cnt; r += blockDim.x)
    sc[r] = rho / (rho + alpha * (dct_eig(2 * r + h, m2, h2) + lam3));
  for (int e = threadIdx.x; e < cnt * cp; e += blockDim.x) {
    const int r = e / cp, q = e - r * cp, k = 2 * r + h;
    const double nrm = k == 0 ? sqrt(1.0 / m2) : sqrt(2.0 / m2);
    Ch[e] = q < cnt ? (float)(nrm * cos(M_PI * k * (2.0 * q + 1.0) / (2.0 * m2))) : 0.0f;
  }
  __syncthreads();
  const size_t nfr = (size_t)RT * KS * 64 * 8;
  unsigned short* o = reinterpret_cast<unsigned short*>(out_raw) + (size_t)kb * 2 * nfr;
  const size_t nf32 = (size_t)RT * KS * 64;     // float32: one block of RT x KS fragments
  float* of = reinterpret_cast<float*>(out_raw) + (size_t)kb * nf32;
  const int ntask = nb * (nb + 1) / 2;
  for (int t = threadIdx.x; t < ntask; t += blockDim.x) {
    // task t -> (bi, bj) with bi <= bj, row-major over the upper triangle
    int bi = 0, rem = t;
    while (rem >= nb - bi) {
      rem -= nb - bi;
      ++bi;
    }
    const int bj = bi + rem;
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
    for (int r = 0; r < cnt; ++r) {
      const float4 x = *reinterpret_cast<const float4*>(&Ch[r * cp + 4 * bi]);
      const float4 y = *reinterpret_cast<const float4*>(&Ch[r * cp + 4 * bj]);
      const double s = sc[r];
      const double xs[4] = {x.x * s, x.y * s, x.z * s, x.w * s};
      const double yv[4] = {y.x, y.y, y.z, y.w};
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fma(xs[a], yv[b], acc[a][b]);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int row = 4 * bi + a, q = 4 * bj + b;
        if (row >= cnt || q >= cnt) continue;
        if (f32) {
          of[zop_index_f32(h, row, q, RTh, KS)] = (float)acc[a][b];
          if (row != q) of[zop_index_f32(h, q, row, RTh, KS)] = (float)acc[a][b];
          continue;
        }
        const unsigned short hi = bf16_rne((float)acc[a][b]);
        const unsigned short lo =
            bf16_rne((float)(acc[a][b] - (double)__uint_as_float((unsigned)hi << 16)));
        const size_t i1 = zop_index(h, row, q, RTh, KS);
        o[i1] = hi;
        o[nfr + i1] = lo;
        if (row != q) {
          const size_t i2 = zop_index(h, q, row, RTh, KS);
          o[i2] = hi;
          o[nfr + i2] = lo;
        }
      }
  }
}

size_t zop_bytes(int prec, int m2, int m3) {
  const int ce = (m2 + 1) / 2, RTh = (ce + 15) / 16;
  if (ce > ZOP_MAXC) return 0;
  if (prec == 1) return (size_t)m3 * 2 * (2 * RTh) * ((ce + 31) / 32) * 64 * 8 * sizeof(unsigned short);
  return (size_t)m3 * (2 * RTh) * (4 * RTh) * 64 * sizeof(float);
}

int launch_build_zop(hipStream_t s, int prec, int m2, int m3, double h2, double h3, double alpha,
                     double rho, int RT, int KS, void* out) {
  if ((m2 + 1) / 2 > ZOP_MAXC) return 1;
  const int ce = (m2 + 1) / 2, cp = (ce + 3) & ~3;
  const size_t lds = ZOP_MAXC * sizeof(double) + (size_t)ce * cp * sizeof(float);
  hipLaunchKernelGGL(k_build_zop, dim3(m3, 2), dim3(256), lds, s, m2, m3, h2, h3, alpha, rho,
                     RT, KS, prec == 1 ? 0 : 1, out);
  return 0;
}

void launch_dct_axis2_op(hipStream_t s, int prec, const GemmArgs& g) { launch_dct<false>(s, prec, g); }

// Kernels need more than 64 KB of dynamic LDS for the largest tiles.
template <bool FUSED, int EPI, int KSM, int SLOTS>
static bool set_lds(int big) {
  bool bad = hipSuccess != hipFuncSetAttribute((const void*)k_dct_bf16<FUSED, EPI, KSM, SLOTS>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, big);
  bad |= hipSuccess != hipFuncSetAttribute((const void*)k_dct_f32<FUSED, EPI, KSM * 4, SLOTS>,
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
  bad |= hipSuccess != hipFuncSetAttribute((const void*)k_build_zop,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           ZOP_MAXC * sizeof(double) + ZOP_MAXC * ZOP_MAXC * sizeof(float));
  (void)hipGetLastError();
  return bad ? 1 : 0;
}

}  // namespace epi
