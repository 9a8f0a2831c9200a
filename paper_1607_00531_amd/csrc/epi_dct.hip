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

namespace epi {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));
typedef unsigned short us4 __attribute__((ext_vector_type(4)));

#define DCT_NT 64          // columns per workgroup
#define DCT_MAXSLOT 4      // 16-row tiles per wave (rows <= 256)

__device__ __forceinline__ unsigned short f2bf(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) {
  return __uint_as_float(((unsigned)h) << 16);
}
__device__ __forceinline__ void split_bf(float x, unsigned short& hi, unsigned short& lo) {
  hi = f2bf(x);
  lo = f2bf(x - bf2f(hi));
}

// Tile index -> (batch, first column), walking each XCD over a contiguous range.
__device__ __forceinline__ void dct_tile(const GemmArgs& g, int& batch, int& c0) {
  const int ntile = g.nbatch * g.col_tiles;
  const int t = xcd_remap(blockIdx.x, ntile);
  batch = t / g.col_tiles;
  c0 = (t % g.col_tiles) * DCT_NT;
}

// Epilogue of the last pass. EPI 0: store. EPI 1: ADMM u-step and residual sums:
// z_new = value, u_new = u + b - z_new (eq. admmStep3); sums |b - z|^2, |z - z_old|^2,
// |z|^2, |u|^2.
template <int EPI>
__device__ __forceinline__ void dct_store(const GemmArgs& g, size_t idx, float val,
                                          double (&acc)[4]) {
  if (EPI == 0) {
    g.out[idx] = val;
  } else {
    const float zo = g.z[idx];
    const float uo = g.u[idx];
    const float bb = g.b[idx];
    const float r = bb - val;
    const float un = uo + r;
    g.z[idx] = val;
    g.u[idx] = un;
    const float dz = val - zo;
    acc[0] += (double)r * r;
    acc[1] += (double)dz * dz;
    acc[2] += (double)val * val;
    acc[3] += (double)un * un;
  }
}

// ------------------------------------------------------------------------------------
// split-bfloat16 variant
// ------------------------------------------------------------------------------------
template <bool FUSED, int EPI>
__global__ __launch_bounds__(256) void k_dct_bf16(GemmArgs g) {
  if (g.done != nullptr && *g.done) return;
  extern __shared__ __attribute__((aligned(16))) unsigned short lds_bf[];
  const int KP = g.KS * 32 + 8;
  unsigned short* Lhi = lds_bf;
  unsigned short* Llo = lds_bf + DCT_NT * KP;
  int batch, c0;
  dct_tile(g, batch, c0);
  const size_t bofs = (size_t)batch * g.bstride;
  const float* in = g.in + bofs;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

  // fill: thread handles (column, group of 8 consecutive rows)
  const int KG = g.KS * 4;
  for (int pi = threadIdx.x; pi < DCT_NT * KG; pi += 256) {
    const int col = pi % DCT_NT, kg = pi / DCT_NT;
    const bool cok = c0 + col < g.ncol;
    us8 hv, lv;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = kg * 8 + e;
      const float v = (cok && k < g.rows) ? in[(size_t)k * g.ld + c0 + col] : 0.0f;
      unsigned short h, l;
      split_bf(v, h, l);
      hv[e] = h;
      lv[e] = l;
    }
    *reinterpret_cast<us8*>(&Lhi[col * KP + kg * 8]) = hv;
    *reinterpret_cast<us8*>(&Llo[col * KP + kg * 8]) = lv;
  }
  __syncthreads();

  const int nslot = (g.RT - wave + 3) / 4;   // row tiles rt = wave + 4 s
  f4 acc[DCT_MAXSLOT][4];
#pragma unroll
  for (int s = 0; s < DCT_MAXSLOT; ++s)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[s][ct] = f4{0.f, 0.f, 0.f, 0.f};

  const us8* A1h = reinterpret_cast<const us8*>(g.A1);
  const size_t frag_stride = (size_t)g.RT * g.KS * 64;   // hi block, then lo block
  for (int ks = 0; ks < g.KS; ++ks) {
    bf16x8 bh[4], bl[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      const int col = ct * 16 + (lane & 15);
      const int k0 = ks * 32 + (lane >> 4) * 8;
      bh[ct] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const us8*>(&Lhi[col * KP + k0]));
      bl[ct] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const us8*>(&Llo[col * KP + k0]));
    }
#pragma unroll
    for (int s = 0; s < DCT_MAXSLOT; ++s) {
      if (s < nslot) {
        const int rt = wave + 4 * s;
        const size_t fi = ((size_t)rt * g.KS + ks) * 64 + lane;
        const bf16x8 ah = __builtin_bit_cast(bf16x8, A1h[fi]);
        const bf16x8 al = __builtin_bit_cast(bf16x8, A1h[frag_stride + fi]);
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
          acc[s][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[ct], acc[s][ct], 0, 0, 0);
          acc[s][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[ct], acc[s][ct], 0, 0, 0);
          acc[s][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[ct], acc[s][ct], 0, 0, 0);
        }
      }
    }
  }

  if (FUSED) {
    // spectral scale rho / (rho + alpha (lambda_row + lambda_batch)), then the inverse
    const float rho = (float)g.st->rho;
    const float lb = (g.lam_batch != nullptr) ? g.lam_batch[batch] : 0.0f;
    __syncthreads();   // all waves finished reading the input tile
#pragma unroll
    for (int s = 0; s < DCT_MAXSLOT; ++s) {
      if (s < nslot) {
        const int rt = wave + 4 * s;
        const int r0 = rt * 16 + (lane >> 4) * 4;
        float sc[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = r0 + r;
          sc[r] = (row < g.rows) ? rho / (rho + g.alpha * (g.lam_row[row] + lb)) : 0.0f;
        }
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
          const int col = ct * 16 + (lane & 15);
          us4 hv, lv;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            unsigned short h, l;
            split_bf(acc[s][ct][r] * sc[r], h, l);
            hv[r] = h;
            lv[r] = l;
          }
          *reinterpret_cast<us4*>(&Lhi[col * KP + r0]) = hv;
          *reinterpret_cast<us4*>(&Llo[col * KP + r0]) = lv;
          acc[s][ct] = f4{0.f, 0.f, 0.f, 0.f};
        }
      }
    }
    __syncthreads();
    const us8* A2h = reinterpret_cast<const us8*>(g.A2);
    for (int ks = 0; ks < g.KS; ++ks) {
      bf16x8 bh[4], bl[4];
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        const int col = ct * 16 + (lane & 15);
        const int k0 = ks * 32 + (lane >> 4) * 8;
        bh[ct] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const us8*>(&Lhi[col * KP + k0]));
        bl[ct] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const us8*>(&Llo[col * KP + k0]));
      }
#pragma unroll
      for (int s = 0; s < DCT_MAXSLOT; ++s) {
        if (s < nslot) {
          const int rt = wave + 4 * s;
          const size_t fi = ((size_t)rt * g.KS + ks) * 64 + lane;
          const bf16x8 ah = __builtin_bit_cast(bf16x8, A2h[fi]);
          const bf16x8 al = __builtin_bit_cast(bf16x8, A2h[frag_stride + fi]);
#pragma unroll
          for (int ct = 0; ct < 4; ++ct) {
            acc[s][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[ct], acc[s][ct], 0, 0, 0);
            acc[s][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[ct], acc[s][ct], 0, 0, 0);
            acc[s][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[ct], acc[s][ct], 0, 0, 0);
          }
        }
      }
    }
  }

  double red[4] = {0, 0, 0, 0};
#pragma unroll
  for (int s = 0; s < DCT_MAXSLOT; ++s) {
    if (s < nslot) {
      const int rt = wave + 4 * s;
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        const int col = c0 + ct * 16 + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = rt * 16 + (lane >> 4) * 4 + r;
          if (row < g.rows && col < g.ncol)
            dct_store<EPI>(g, bofs + (size_t)row * g.ld + col, acc[s][ct][r], red);
        }
      }
    }
  }
  if (EPI == 1) block_partials<4>(red, g.partial, blockIdx.x);
}

// ------------------------------------------------------------------------------------
// float32 variant (v_mfma_f32_16x16x4_f32), same structure
// ------------------------------------------------------------------------------------
template <bool FUSED, int EPI>
__global__ __launch_bounds__(256) void k_dct_f32(GemmArgs g) {
  if (g.done != nullptr && *g.done) return;
  extern __shared__ __attribute__((aligned(16))) float lds_f[];
  const int LD = DCT_NT + 4;
  const int KP = g.KS * 4;
  int batch, c0;
  dct_tile(g, batch, c0);
  const size_t bofs = (size_t)batch * g.bstride;
  const float* in = g.in + bofs;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int pi = threadIdx.x; pi < DCT_NT * KP; pi += 256) {
    const int col = pi % DCT_NT, k = pi / DCT_NT;
    lds_f[k * LD + col] = (c0 + col < g.ncol && k < g.rows) ? in[(size_t)k * g.ld + c0 + col] : 0.0f;
  }
  __syncthreads();
  const int nslot = (g.RT - wave + 3) / 4;
  f4 acc[DCT_MAXSLOT][4];
#pragma unroll
  for (int s = 0; s < DCT_MAXSLOT; ++s)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[s][ct] = f4{0.f, 0.f, 0.f, 0.f};
  const float* A1 = reinterpret_cast<const float*>(g.A1);
  for (int ks = 0; ks < g.KS; ++ks) {
    float bv[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) bv[ct] = lds_f[(ks * 4 + (lane >> 4)) * LD + ct * 16 + (lane & 15)];
#pragma unroll
    for (int s = 0; s < DCT_MAXSLOT; ++s) {
      if (s < nslot) {
        const int rt = wave + 4 * s;
        const float av = A1[((size_t)rt * g.KS + ks) * 64 + lane];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
          acc[s][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv[ct], acc[s][ct], 0, 0, 0);
      }
    }
  }
  if (FUSED) {
    const float rho = (float)g.st->rho;
    const float lb = (g.lam_batch != nullptr) ? g.lam_batch[batch] : 0.0f;
    __syncthreads();
#pragma unroll
    for (int s = 0; s < DCT_MAXSLOT; ++s) {
      if (s < nslot) {
        const int rt = wave + 4 * s;
        const int r0 = rt * 16 + (lane >> 4) * 4;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = r0 + r;
          const float sc = (row < g.rows) ? rho / (rho + g.alpha * (g.lam_row[row] + lb)) : 0.0f;
#pragma unroll
          for (int ct = 0; ct < 4; ++ct) lds_f[row * LD + ct * 16 + (lane & 15)] = acc[s][ct][r] * sc;
        }
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[s][ct] = f4{0.f, 0.f, 0.f, 0.f};
      }
    }
    __syncthreads();
    const float* A2 = reinterpret_cast<const float*>(g.A2);
    for (int ks = 0; ks < g.KS; ++ks) {
      float bv[4];
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) bv[ct] = lds_f[(ks * 4 + (lane >> 4)) * LD + ct * 16 + (lane & 15)];
#pragma unroll
      for (int s = 0; s < DCT_MAXSLOT; ++s) {
        if (s < nslot) {
          const int rt = wave + 4 * s;
          const float av = A2[((size_t)rt * g.KS + ks) * 64 + lane];
#pragma unroll
          for (int ct = 0; ct < 4; ++ct)
            acc[s][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv[ct], acc[s][ct], 0, 0, 0);
        }
      }
    }
  }
  double red[4] = {0, 0, 0, 0};
#pragma unroll
  for (int s = 0; s < DCT_MAXSLOT; ++s) {
    if (s < nslot) {
      const int rt = wave + 4 * s;
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        const int col = c0 + ct * 16 + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = rt * 16 + (lane >> 4) * 4 + r;
          if (row < g.rows && col < g.ncol)
            dct_store<EPI>(g, bofs + (size_t)row * g.ld + col, acc[s][ct][r], red);
        }
      }
    }
  }
  if (EPI == 1) block_partials<4>(red, g.partial, blockIdx.x);
}

// ------------------------------------------------------------------------------------
static size_t dct_lds_bytes(int prec, const GemmArgs& g) {
  if (prec == 1) return (size_t)2 * DCT_NT * (g.KS * 32 + 8) * sizeof(unsigned short);
  // the fused pass writes back all 16-row tiles, which may exceed the padded contraction
  const int rows = g.KS * 4 > g.RT * 16 ? g.KS * 4 : g.RT * 16;
  return (size_t)rows * (DCT_NT + 4) * sizeof(float);
}

template <bool FUSED>
static void launch_dct(hipStream_t s, int prec, const GemmArgs& g) {
  const dim3 grid(g.nbatch * g.col_tiles), blk(256);
  const size_t lds = dct_lds_bytes(prec, g);
  if (prec == 1) {
    if (g.epi == 1)
      hipLaunchKernelGGL((k_dct_bf16<FUSED, 1>), grid, blk, lds, s, g);
    else
      hipLaunchKernelGGL((k_dct_bf16<FUSED, 0>), grid, blk, lds, s, g);
  } else {
    if (g.epi == 1)
      hipLaunchKernelGGL((k_dct_f32<FUSED, 1>), grid, blk, lds, s, g);
    else
      hipLaunchKernelGGL((k_dct_f32<FUSED, 0>), grid, blk, lds, s, g);
  }
}

void launch_dct_axis3(hipStream_t s, int prec, const GemmArgs& g) { launch_dct<false>(s, prec, g); }
void launch_dct_axis2_fused(hipStream_t s, int prec, const GemmArgs& g) {
  launch_dct<true>(s, prec, g);
}

// Kernels need more than 64 KB of dynamic LDS for the largest tiles.
int dct_set_lds_limits() {
  const int big = 80 * 1024;   // largest tile: 2 x 64 x 264 bf16 or 256 x 68 float
  bool bad = false;
  bad |= hipSuccess != hipFuncSetAttribute((const void*)k_dct_bf16<false, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, big);
  bad |= hipSuccess != hipFuncSetAttribute((const void*)k_dct_bf16<false, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, big);
  bad |= hipSuccess != hipFuncSetAttribute((const void*)k_dct_bf16<true, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, big);
  bad |= hipSuccess != hipFuncSetAttribute((const void*)k_dct_bf16<true, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, big);
  bad |= hipSuccess != hipFuncSetAttribute((const void*)k_dct_f32<false, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, big);
  bad |= hipSuccess != hipFuncSetAttribute((const void*)k_dct_f32<false, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, big);
  bad |= hipSuccess != hipFuncSetAttribute((const void*)k_dct_f32<true, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, big);
  bad |= hipSuccess != hipFuncSetAttribute((const void*)k_dct_f32<true, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, big);
  (void)hipGetLastError();
  return bad ? 1 : 0;
}

}  // namespace epi
