// Device code of the z-step DCT products, shared by the single-volume and the batched
// kernels (see epi_dct.hip for the method).
#pragma once

#include <hip/hip_runtime.h>

#include "epi_device.hpp"
#include "epi_common.hpp"

namespace epi {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));
typedef unsigned short us4 __attribute__((ext_vector_type(4)));

#define DCT_NT 64          // columns per workgroup

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
__device__ __forceinline__ int dct_tile(const GemmArgs& g, int& batch, int& c0) {
  const int ntile = g.nbatch * g.col_tiles;
  const int t = xcd_remap(blockIdx.x, ntile);
  batch = t / g.col_tiles;
  c0 = (t % g.col_tiles) * DCT_NT;
  return t;
}

// Accumulators -> LDS tile [row][col] (float32, row stride DCT_NT + 4), scaled per row.
template <int SLOTS>
__device__ __forceinline__ void acc_to_lds(float* T, const f4 (&acc)[SLOTS][4], int wave,
                                           int lane, int nslot) {
#pragma unroll
  for (int s = 0; s < SLOTS; ++s) {
    if (s < nslot) {
      const int r0 = (wave + 4 * s) * 16 + (lane >> 4) * 4;
#pragma unroll
      for (int ct = 0; ct < 4; ++ct)
#pragma unroll
        for (int r = 0; r < 4; ++r) T[(r0 + r) * (DCT_NT + 4) + ct * 16 + (lane & 15)] = acc[s][ct][r];
    }
  }
}

// Epilogue of the last pass from the LDS tile, one row of 64 consecutive columns per 64
// threads (coalesced). EPI 0: store. EPI 1: ADMM u-step and residual sums:
// z_new = value, u_new = u + b - z_new (eq. admmStep3); sums |b - z|^2, |z - z_old|^2,
// |z|^2, |u|^2, |b|^2 into the partial buffer.
template <int EPI>
__device__ __forceinline__ void tile_epilogue(const GemmArgs& g, const float* T, size_t bofs,
                                              int c0, int pslot) {
  double acc[NQ_ADMM_E] = {0, 0, 0, 0, 0};
  const int col = threadIdx.x & (DCT_NT - 1);
  const bool cok = c0 + col < g.ncol;
  for (int row = threadIdx.x / DCT_NT; row < g.rows; row += 256 / DCT_NT) {
    if (!cok) continue;
    const float val = T[row * (DCT_NT + 4) + col];
    const size_t idx = bofs + (size_t)row * g.ld + c0 + col;
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
      acc[4] += (double)bb * bb;
    }
  }
  if (EPI == 1) block_partials<NQ_ADMM_E>(acc, g.partial, pslot);
}

// ------------------------------------------------------------------------------------
// split-bfloat16 variant. KSM: maximum contraction steps of 32 (rows <= 32 KSM);
// SLOTS: 16-row tiles per wave (rows <= 64 SLOTS).
// ------------------------------------------------------------------------------------
// acc[s][ct] += A(row tile wave + 4 s) * B(LDS tile, column tile ct) over all contraction
// steps. The A fragments of step ks + 1 are loaded while the products of step ks run.
template <int SLOTS>
__device__ __forceinline__ void gemm_bf16(const us8* __restrict__ A, size_t frag_stride, int KS,
                                          int wave, int lane, int nslot,
                                          const unsigned short* Lhi, const unsigned short* Llo,
                                          int KP, f4 (&acc)[SLOTS][4]) {
  us8 nh[SLOTS], nl[SLOTS];
#pragma unroll
  for (int s = 0; s < SLOTS; ++s) {
    if (s < nslot) {
      const size_t fi = ((size_t)(wave + 4 * s) * KS) * 64 + lane;
      nh[s] = A[fi];
      nl[s] = A[frag_stride + fi];
    }
  }
  for (int ks = 0; ks < KS; ++ks) {
    us8 ch[SLOTS], cl[SLOTS];
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      ch[s] = nh[s];
      cl[s] = nl[s];
    }
    if (ks + 1 < KS) {
#pragma unroll
      for (int s = 0; s < SLOTS; ++s) {
        if (s < nslot) {
          const size_t fi = ((size_t)(wave + 4 * s) * KS + ks + 1) * 64 + lane;
          nh[s] = A[fi];
          nl[s] = A[frag_stride + fi];
        }
      }
    }
    bf16x8 bh[4], bl[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      const int col = ct * 16 + (lane & 15);
      const int k0 = ks * 32 + (lane >> 4) * 8;
      bh[ct] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const us8*>(&Lhi[col * KP + k0]));
      bl[ct] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const us8*>(&Llo[col * KP + k0]));
    }
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      if (s < nslot) {
        const bf16x8 ah = __builtin_bit_cast(bf16x8, ch[s]);
        const bf16x8 al = __builtin_bit_cast(bf16x8, cl[s]);
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

// One 64-column tile of one batch entry: fill, product(s), epilogue. pslot = index of this
// tile's partial sums (EPI 1). Every thread of the workgroup must call it.
template <bool FUSED, int EPI, int KSM, int SLOTS>
__device__ __forceinline__ void dct_bf16_body(const GemmArgs& g, int batch, int c0, int pslot,
                                              unsigned short* lds_bf) {
  const int KP = g.KS * 32 + 8;
  unsigned short* Lhi = lds_bf;
  unsigned short* Llo = lds_bf + DCT_NT * KP;
  const size_t bofs = (size_t)batch * g.bstride;
  const float* in = g.in + bofs;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

  // fill: thread handles (column, group of 8 consecutive rows) for KS such pairs; all
  // global loads are issued before the first conversion
  {
    float v[KSM][8];
#pragma unroll
    for (int it = 0; it < KSM; ++it) {
      const int pi = threadIdx.x + 256 * it;
      const int col = pi & (DCT_NT - 1), kg = pi / DCT_NT;
      const bool ok = it < g.KS && c0 + col < g.ncol;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = kg * 8 + e;
        v[it][e] = (ok && k < g.rows) ? in[(size_t)k * g.ld + c0 + col] : 0.0f;
      }
    }
#pragma unroll
    for (int it = 0; it < KSM; ++it) {
      if (it < g.KS) {
        const int pi = threadIdx.x + 256 * it;
        const int col = pi & (DCT_NT - 1), kg = pi / DCT_NT;
        us8 hv, lv;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          unsigned short h, l;
          split_bf(v[it][e], h, l);
          hv[e] = h;
          lv[e] = l;
        }
        *reinterpret_cast<us8*>(&Lhi[col * KP + kg * 8]) = hv;
        *reinterpret_cast<us8*>(&Llo[col * KP + kg * 8]) = lv;
      }
    }
  }
  __syncthreads();

  const int nslot = (g.RT - wave + 3) / 4;   // row tiles rt = wave + 4 s
  f4 acc[SLOTS][4];
#pragma unroll
  for (int s = 0; s < SLOTS; ++s)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[s][ct] = f4{0.f, 0.f, 0.f, 0.f};
  const size_t frag_stride = (size_t)g.RT * g.KS * 64;   // hi block, then lo block
  gemm_bf16<SLOTS>(reinterpret_cast<const us8*>(g.A1), frag_stride, g.KS, wave, lane, nslot,
                   Lhi, Llo, KP, acc);

  if (FUSED) {
    // spectral scale rho / (rho + alpha (lambda_row + lambda_batch)), then the inverse
    const float rho = (float)g.st->rho;
    const float lb = (g.lam_batch != nullptr) ? g.lam_batch[batch] : 0.0f;
    __syncthreads();   // all waves finished reading the input tile
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
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
    gemm_bf16<SLOTS>(reinterpret_cast<const us8*>(g.A2), frag_stride, g.KS, wave, lane, nslot,
                     Lhi, Llo, KP, acc);
  }
  __syncthreads();   // the LDS tile is reused for the output
  float* T = reinterpret_cast<float*>(lds_bf);
  acc_to_lds<SLOTS>(T, acc, wave, lane, nslot);
  __syncthreads();
  tile_epilogue<EPI>(g, T, bofs, c0, pslot);
  __syncthreads();   // LDS free for the next tile
}

// ------------------------------------------------------------------------------------
// float32 variant (v_mfma_f32_16x16x4_f32), same structure; LDS tile [k][col]
// ------------------------------------------------------------------------------------
template <int SLOTS>
__device__ __forceinline__ void gemm_f32(const float* __restrict__ A, int KS, int wave, int lane,
                                         int nslot, const float* L, f4 (&acc)[SLOTS][4]) {
  const int LD = DCT_NT + 4;
  for (int ks = 0; ks < KS; ++ks) {
    float bv[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) bv[ct] = L[(ks * 4 + (lane >> 4)) * LD + ct * 16 + (lane & 15)];
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      if (s < nslot) {
        const float av = A[((size_t)(wave + 4 * s) * KS + ks) * 64 + lane];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
          acc[s][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv[ct], acc[s][ct], 0, 0, 0);
      }
    }
  }
}

template <bool FUSED, int EPI, int KSM, int SLOTS>
__device__ __forceinline__ void dct_f32_body(const GemmArgs& g, int batch, int c0, int pslot,
                                             float* lds_f) {
  const int LD = DCT_NT + 4;
  const int KP = g.KS * 4;
  const size_t bofs = (size_t)batch * g.bstride;
  const float* in = g.in + bofs;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  {
    const int col = threadIdx.x & (DCT_NT - 1);
    const bool cok = c0 + col < g.ncol;
    float v[KSM];   // KSM = maximum contraction steps of 4 rows (rows <= 4 KSM)
#pragma unroll
    for (int q = 0; q < KSM; ++q) {
      const int k = threadIdx.x / DCT_NT + 4 * q;
      v[q] = (cok && k < g.rows) ? in[(size_t)k * g.ld + c0 + col] : 0.0f;
    }
#pragma unroll
    for (int q = 0; q < KSM; ++q) {
      const int k = threadIdx.x / DCT_NT + 4 * q;
      if (k < KP) lds_f[k * LD + col] = v[q];
    }
  }
  __syncthreads();
  const int nslot = (g.RT - wave + 3) / 4;
  f4 acc[SLOTS][4];
#pragma unroll
  for (int s = 0; s < SLOTS; ++s)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[s][ct] = f4{0.f, 0.f, 0.f, 0.f};
  gemm_f32<SLOTS>(reinterpret_cast<const float*>(g.A1), g.KS, wave, lane, nslot, lds_f, acc);
  if (FUSED) {
    const float rho = (float)g.st->rho;
    const float lb = (g.lam_batch != nullptr) ? g.lam_batch[batch] : 0.0f;
    __syncthreads();
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      if (s < nslot) {
        const int r0 = (wave + 4 * s) * 16 + (lane >> 4) * 4;
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
    gemm_f32<SLOTS>(reinterpret_cast<const float*>(g.A2), g.KS, wave, lane, nslot, lds_f, acc);
  }
  __syncthreads();
  acc_to_lds<SLOTS>(lds_f, acc, wave, lane, nslot);
  __syncthreads();
  tile_epilogue<EPI>(g, lds_f, bofs, c0, pslot);
  __syncthreads();
}

// dynamic LDS bytes of one tile
__host__ __device__ inline size_t dct_lds_bytes(int prec, const GemmArgs& g) {
  const size_t out_tile = (size_t)g.RT * 16 * (DCT_NT + 4) * sizeof(float);
  size_t in_tile;
  if (prec == 1) {
    in_tile = (size_t)2 * DCT_NT * (g.KS * 32 + 8) * sizeof(unsigned short);
  } else {
    // the fused pass writes back all 16-row tiles, which may exceed the padded contraction
    const int rows = g.KS * 4 > g.RT * 16 ? g.KS * 4 : g.RT * 16;
    in_tile = (size_t)rows * (DCT_NT + 4) * sizeof(float);
  }
  return in_tile > out_tile ? in_tile : out_tile;
}

// ------------------------------------------------------------------------------------
}  // namespace epi
