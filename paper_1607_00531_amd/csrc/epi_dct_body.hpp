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
typedef float f2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf2v __attribute__((ext_vector_type(2)));
typedef unsigned u2v __attribute__((ext_vector_type(2)));
typedef unsigned u4v __attribute__((ext_vector_type(4)));

#define DCT_NT 64          // columns per workgroup

// padding (bfloat16 elements) of a column of the split-bfloat16 LDS tile
#ifndef EPI_DCT_KPAD
#define EPI_DCT_KPAD 8
#endif

// wavefronts per workgroup of the split-bfloat16 tile kernels (float32 kernels use 4)
#ifndef EPI_DCT_NW
#define EPI_DCT_NW 8
#endif

// Split of two floats into bfloat16 pairs a = a_hi + a_lo (both rounded to nearest even):
// one v_cvt_pk_bf16_f32 per pair for each part. Packed as (first element in the low half).
__device__ __forceinline__ void split_bf2(float a, float b, unsigned& hi, unsigned& lo) {
  const f2v v = {a, b};
  const unsigned h = __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf2v));
  const f2v hf = {__uint_as_float(h << 16), __uint_as_float(h & 0xffff0000u)};
  lo = __builtin_bit_cast(unsigned, __builtin_convertvector(v - hf, bf2v));
  hi = h;
}

// Access at a wave-uniform base plus a 32-bit byte offset: the compiler keeps the base in
// scalar registers and addresses with the offset alone (no per-lane 64-bit arithmetic).
template <typename T>
__device__ __forceinline__ T ld_at(const void* base, unsigned boff) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + boff);
}
template <typename T>
__device__ __forceinline__ void st_at(void* base, unsigned boff, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + boff) = v;
}
__device__ __forceinline__ void st_stream_at(float* base, unsigned boff, float v) {
  store_stream(reinterpret_cast<float*>(reinterpret_cast<char*>(base) + boff), v);
}

// LDS of one workgroup: the input tile (reused for the float32 output tile) and, for the
// split-bfloat16 kernels, the spectral scale of every row tile row (RT * 16 floats).
__host__ __device__ inline size_t dct_tile_bytes(int prec, const GemmArgs& g) {
  const size_t out_tile = (size_t)g.RT * 16 * (DCT_NT + 4) * sizeof(float);
  size_t in_tile;
  if (prec == 1) {
    // hi and lo tiles, both halves of the even/odd split (KS steps of 32 each) + padding
    in_tile = (size_t)2 * DCT_NT * (2 * g.KS * 32 + EPI_DCT_KPAD) * sizeof(unsigned short);
  } else {
    // both halves' contraction blocks (KS steps of 4 each); the output needs RT 16-row tiles
    const int rows = 2 * g.KS * 4 > g.RT * 16 ? 2 * g.KS * 4 : g.RT * 16;
    in_tile = (size_t)rows * (DCT_NT + 4) * sizeof(float);
  }
  const size_t t = in_tile > out_tile ? in_tile : out_tile;
  return (t + 15) & ~(size_t)15;
}
__host__ __device__ inline size_t dct_lds_bytes(int prec, const GemmArgs& g) {
  return dct_tile_bytes(prec, g) + (prec == 1 ? (size_t)g.RT * 16 * sizeof(float) : 0);
}

// Tile index -> (batch, first column), walking each XCD over a contiguous range.
__device__ __forceinline__ int dct_tile(const GemmArgs& g, int& batch, int& c0) {
  const int ntile = g.nbatch * g.col_tiles;
  const int t = xcd_remap(blockIdx.x, ntile);
  batch = t / g.col_tiles;
  c0 = (t % g.col_tiles) * DCT_NT;
  return t;
}

// Output row -> value of the LDS tile [row][col]. OUT_PLAIN: the row itself. With the
// even/odd split (N = transform length, c = ceil(N/2), f = floor(N/2), odd block from tile
// row hrow): OUT_HALF_ORDER: spectral output in half order (rows < c even block, then the
// odd block); OUT_EVEN_ODD: spatial output x_n = E_n + O_n, x_{N-1-n} = E_n - O_n.
enum { OUT_PLAIN = 0, OUT_HALF_ORDER = 1, OUT_EVEN_ODD = 2 };
template <int OUT>
__device__ __forceinline__ float tile_value(const float* T, int row, int col, int N, int hrow) {
  constexpr int LD = DCT_NT + 4;
  if (OUT == OUT_PLAIN) return T[row * LD + col];
  const int ce = (N + 1) / 2, fo = N / 2;
  if (OUT == OUT_HALF_ORDER) return T[(row < ce ? row : hrow + row - ce) * LD + col];
  const int n = row < ce ? row : N - 1 - row;
  const float e = T[n * LD + col];
  const float o = (n < fo) ? T[(hrow + n) * LD + col] : 0.0f;
  return row < ce ? e + o : e - o;
}

// Epilogue of the last pass from the LDS tile, one row of 64 consecutive columns per
// wavefront (coalesced; the row is uniform over the wavefront). EPI 0: store. EPI 1: ADMM
// u-step and residual sums: z_new = value, u_new = u + b - z_new (eq. admmStep3); sums
// |b - z|^2, |z - z_old|^2, |z|^2, |u|^2, |b|^2 into the partial buffer.
template <int EPI, int NW, int OUT>
__device__ __forceinline__ void tile_epilogue(const GemmArgs& g, const float* T, size_t bofs,
                                              int c0, int pslot, int hrow) {
  double acc[NQ_ADMM_E] = {0, 0, 0, 0, 0};
  const int col = threadIdx.x & (DCT_NT - 1);
  const unsigned col4 = (unsigned)col * 4u;
  const bool cok = c0 + col < g.ncol;
  const int r0 = __builtin_amdgcn_readfirstlane(threadIdx.x / DCT_NT);
  constexpr int RS = 64 * NW / DCT_NT;
  if (EPI == 0) {
    float* ob = g.out + bofs + c0;
    for (int row = r0; row < g.rows; row += RS)
      if (cok) st_stream_at(ob + (size_t)row * g.ld, col4, tile_value<OUT>(T, row, col, g.rows, hrow));
  } else {
    // U rows per thread in flight: all their loads are issued before the first store
    // (the stores to z and u could alias the loads as far as the compiler knows)
    constexpr int U = 8;
    const float us = (float)g.st->u_scale;   // pending rescale of u (1 with a fixed rho)
    const float* bb0 = g.b + bofs + c0;
    float* zb0 = g.z + bofs + c0;
    float* ub0 = g.u + bofs + c0;
    for (int rb = r0; rb < g.rows; rb += RS * U) {
      float zo[U], uo[U], bb[U];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int row = rb + RS * q;
        const size_t ro = (size_t)(row < g.rows ? row : 0) * g.ld;
        const bool ok = cok && row < g.rows;
        zo[q] = ok ? ld_at<float>(zb0 + ro, col4) : 0.0f;
        uo[q] = ok ? ld_at<float>(ub0 + ro, col4) * us : 0.0f;
        bb[q] = ok ? ld_at<float>(bb0 + ro, col4) : 0.0f;
      }
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int row = rb + RS * q;
        if (cok && row < g.rows) {
          const size_t ro = (size_t)row * g.ld;
          const float val = tile_value<OUT>(T, row, col, g.rows, hrow);
          const float r = bb[q] - val;
          const float un = uo[q] + r;
          st_at<float>(zb0 + ro, col4, val);
          st_at<float>(ub0 + ro, col4, un);
          const float dz = val - zo[q];
          acc[0] += (double)r * r;
          acc[1] += (double)dz * dz;
          acc[2] += (double)val * val;
          acc[3] += (double)un * un;
          acc[4] += (double)bb[q] * bb[q];
        }
      }
    }
    block_partials<NQ_ADMM_E>(acc, g.partial, pslot);
  }
}

// ------------------------------------------------------------------------------------
// split-bfloat16 variant with the even/odd decomposition of the DCT. With c = ceil(N/2),
// f = floor(N/2) and C[k][N-1-n] = (-1)^k C[k][n]:
//   forward  y_2r   = sum_{q<c} C[2r][q]   s_q,  s_q = x_q + x_{N-1-q} (s_mid = x_mid, N odd)
//            y_2r+1 = sum_{q<f} C[2r+1][q] d_q,  d_q = x_q - x_{N-1-q}
//   inverse  E_n = sum_{r<c} C[2r][n] y_2r,  O_n = sum_{r<f} C[2r+1][n] y_2r+1,
//            x_n = E_n + O_n, x_{N-1-n} = E_n - O_n (x_mid = E_mid, N odd)
// Two half-size products replace one N x N product. Spectral data between the passes is
// kept in half order: even k first (row r <-> k = 2r), then odd k (row c + r <-> 2r + 1).
// The packed matrices hold the even half in row tiles [0, RTh) and the odd half in
// [RTh, 2 RTh), each with KS steps of 32 over its own contraction block; in LDS the even
// block sits at contraction offset 0 and the odd block at KS * 32.
// KSF: maximum steps of 32 of the whole length (N <= 32 KSF), KSM = KSF / 2 those of a
// half; NW wavefronts per workgroup, the first NW / 2 on the even half, the others on the
// odd half, each with up to SLOTS = 4 KSM / NW row tiles.
// ------------------------------------------------------------------------------------
// acc[s][ct] += A(row tile rt0 + rstep s) * B(LDS tile from contraction offset koff, column
// tile ct) over all contraction steps. The A fragments stream from L2 PD steps ahead of the
// products that use them; the step loop is unrolled over its compile-time bound KSM so that
// the fragment ring stays in registers.
template <int SLOTS, int KSM, int PD>
__device__ __forceinline__ void gemm_bf16(const us8* __restrict__ A, size_t frag_stride, int KS,
                                          int rt0, int rstep, int lane, int nslot,
                                          const unsigned short* Lhi, const unsigned short* Llo,
                                          int KP, int koff, f4 (&acc)[SLOTS][4]) {
  // fragment (row tile rt, step ks) of lane l sits at ((rt * KS + ks) * 64 + l) * 16 bytes;
  // rt = rt0 + rstep s is uniform, so only lane * 16 is a per-lane offset
  const us8* Alo = A + frag_stride;
  const unsigned lane16 = (unsigned)lane * 16u;
  us8 fh[KSM][SLOTS], fl[KSM][SLOTS];
#pragma unroll
  for (int ks = 0; ks < PD && ks < KSM; ++ks) {
    if (ks < KS) {
#pragma unroll
      for (int s = 0; s < SLOTS; ++s) {
        if (s < nslot) {
          const size_t fu = ((size_t)(rt0 + rstep * s) * KS + ks) * 64;
          fh[ks][s] = ld_at<us8>(A + fu, lane16);
          fl[ks][s] = ld_at<us8>(Alo + fu, lane16);
        }
      }
    }
  }
#pragma unroll
  for (int ks = 0; ks < KSM; ++ks) {
    if (ks < KS) {
      if (ks + PD < KSM && ks + PD < KS) {
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
          if (s < nslot) {
            const size_t fu = ((size_t)(rt0 + rstep * s) * KS + ks + PD) * 64;
            fh[(ks + PD) % KSM][s] = ld_at<us8>(A + fu, lane16);
            fl[(ks + PD) % KSM][s] = ld_at<us8>(Alo + fu, lane16);
          }
        }
      }
      bf16x8 bh[4], bl[4];
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        const int col = ct * 16 + (lane & 15);
        const int k0 = koff + ks * 32 + (lane >> 4) * 8;
        bh[ct] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const us8*>(&Lhi[col * KP + k0]));
        bl[ct] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const us8*>(&Llo[col * KP + k0]));
      }
#pragma unroll
      for (int s = 0; s < SLOTS; ++s) {
        if (s < nslot) {
          const bf16x8 ah = __builtin_bit_cast(bf16x8, fh[ks][s]);
          const bf16x8 al = __builtin_bit_cast(bf16x8, fl[ks][s]);
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
}

// prefetch depth of the A fragments (contraction steps ahead)
#ifndef EPI_GEMM_PD_SMALL
#define EPI_GEMM_PD_SMALL 4
#endif
#ifndef EPI_GEMM_PD_BIG
#define EPI_GEMM_PD_BIG 2
#endif
template <int KSM>
struct GemmPD {
  static constexpr int value = KSM <= 2 ? EPI_GEMM_PD_SMALL : EPI_GEMM_PD_BIG;
};

// Writes the accumulators (row tiles rt0 + rstep s) to the float32 LDS tile [row][col].
template <int SLOTS>
__device__ __forceinline__ void acc_rows_to_lds(float* T, const f4 (&acc)[SLOTS][4], int rt0,
                                                int rstep, int lane, int nslot) {
#pragma unroll
  for (int s = 0; s < SLOTS; ++s) {
    if (s < nslot) {
      const int r0 = (rt0 + rstep * s) * 16 + (lane >> 4) * 4;
#pragma unroll
      for (int ct = 0; ct < 4; ++ct)
#pragma unroll
        for (int r = 0; r < 4; ++r) T[(r0 + r) * (DCT_NT + 4) + ct * 16 + (lane & 15)] = acc[s][ct][r];
    }
  }
}

// One 64-column tile of one batch entry: fill, product(s), epilogue. pslot = index of this
// tile's partial sums (EPI 1). Every thread of the workgroup (NW wavefronts) must call it.
// FUSED: spatial in, forward, spectral scale, inverse, spatial out; otherwise g.dir = 0
// (spatial in, spectral out in half order), 1 (spectral in half order, spatial out) or 2
// (spatial in and out through one product with the batch entry's own even/odd operator,
// which stands for forward, spectral scale and inverse together).
template <bool FUSED, int EPI, int KSF, int NW>
__device__ __forceinline__ void dct_bf16_body(const GemmArgs& g, int batch, int c0, int pslot,
                                              unsigned short* lds_bf) {
  constexpr int KSM = KSF / 2;                     // KSF: steps of 32 of the whole length
  constexpr int HW = NW / 2;                       // wavefronts per half
  constexpr int SLOTS = (2 * KSM + HW - 1) / HW;   // row tiles per wavefront (RTh <= 2 KSM)
  constexpr int NG = 4 * KSM;                      // 8-row groups per half (maximum)
  constexpr int NIT = (NG + NW - 1) / NW;
  static_assert(64 * KSM <= 64 * NW, "one thread per scale-table row");
  const int N = g.rows, ce = (N + 1) / 2, fo = N / 2;
  const int KPh = g.KS * 32;                       // contraction extent of one half
  const int KP = 2 * KPh + EPI_DCT_KPAD;
  const int RTh = g.RT / 2;
  const bool fwd_in = FUSED || g.dir != 1;
  unsigned short* Lhi = lds_bf;
  unsigned short* Llo = lds_bf + DCT_NT * KP;
  float* SC = reinterpret_cast<float*>(reinterpret_cast<char*>(lds_bf) + dct_tile_bytes(1, g));
  const size_t bofs = (size_t)batch * g.bstride;
  const float* in = g.in + bofs + c0;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

  // fill: thread handles (column = lane, group kg = wave + NW it of 8 contraction positions
  // q of both halves); the positions are uniform over the wavefront; all global loads are
  // issued before the first conversion
  {
    const unsigned lane4 = (unsigned)lane * 4u;
    const bool cok = c0 + lane < g.ncol;
    const int ngroups = 4 * g.KS;
    float va[NIT][8], vb[NIT][8];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int kg = wave + NW * it;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int q = kg * 8 + e;
        const bool live = kg < ngroups && cok;
        // forward: x_q and x_{N-1-q}; inverse: spectral rows q (even) and c + q (odd)
        const int ra = q, rb = fwd_in ? N - 1 - q : ce + q;
        const bool oka = live && q < ce;
        const bool okb = live && q < fo;
        va[it][e] = oka ? ld_at<float>(in + (size_t)ra * g.ld, lane4) : 0.0f;
        vb[it][e] = okb ? ld_at<float>(in + (size_t)(okb ? rb : 0) * g.ld, lane4) : 0.0f;
      }
    }
    if (FUSED) {
      // spectral scale rho / (rho + alpha (lambda_row + lambda_batch)) of each row tile row
      // in half order (0 beyond the half's length), read after the first product
      const int hr = RTh * 16, rows = 2 * hr;
      if ((int)threadIdx.x < rows) {
        const int h = (int)threadIdx.x >= hr, row = (int)threadIdx.x - h * hr;
        const float rho = (float)g.st->rho;
        const float lb = (g.lam_batch != nullptr) ? g.lam_batch[batch] : 0.0f;
        float sc = 0.0f;
        if (row < (h ? fo : ce)) sc = rho * rcp_f(rho + g.alpha * (g.lam_row[h * ce + row] + lb));
        SC[threadIdx.x] = sc;
      }
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int kg = wave + NW * it;
      if (kg < ngroups) {
        const int col = lane;
        u4v hv0, lv0, hv1, lv1;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          float ev[2], od[2];
#pragma unroll
          for (int t = 0; t < 2; ++t) {
            const float a = va[it][2 * e + t], b = vb[it][2 * e + t];
            // forward: the pair sum / difference (b = 0 for q >= f, so s_mid = x_mid)
            ev[t] = fwd_in ? a + b : a;
            od[t] = fwd_in ? a - b : b;
            if (fwd_in && kg * 8 + 2 * e + t >= fo) od[t] = 0.0f;
          }
          unsigned h, l;
          split_bf2(ev[0], ev[1], h, l);
          hv0[e] = h;
          lv0[e] = l;
          split_bf2(od[0], od[1], h, l);
          hv1[e] = h;
          lv1[e] = l;
        }
        *reinterpret_cast<u4v*>(&Lhi[col * KP + kg * 8]) = hv0;
        *reinterpret_cast<u4v*>(&Llo[col * KP + kg * 8]) = lv0;
        *reinterpret_cast<u4v*>(&Lhi[col * KP + KPh + kg * 8]) = hv1;
        *reinterpret_cast<u4v*>(&Llo[col * KP + KPh + kg * 8]) = lv1;
      }
    }
  }
  __syncthreads();

  const int half = wave / HW, lw = wave % HW;
  const int rt0 = half * RTh + lw;                 // row tiles rt0 + HW s of this half
  const int nslot = (RTh - lw + HW - 1) / HW;
  const int koff = half * KPh;
  f4 acc[SLOTS][4];
#pragma unroll
  for (int s = 0; s < SLOTS; ++s)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[s][ct] = f4{0.f, 0.f, 0.f, 0.f};
  const size_t frag_stride = (size_t)g.RT * g.KS * 64;   // hi block, then lo block
  const us8* A1 = reinterpret_cast<const us8*>(g.A1) + (size_t)batch * g.a_bstride;
  gemm_bf16<SLOTS, KSM, GemmPD<KSM>::value>(A1, frag_stride, g.KS, rt0, HW, lane, nslot, Lhi,
                                            Llo, KP, koff, acc);

  if (FUSED) {
    // spectral scale rho / (rho + alpha (lambda_row + lambda_batch)) in half order, then
    // the inverse from the same LDS blocks
    const float* sch = SC + half * RTh * 16;
    __syncthreads();   // all waves finished reading the input tile
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      if (s < nslot) {
        const int r0 = (lw + HW * s) * 16 + (lane >> 4) * 4;   // row within the half
        float sc[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) sc[r] = sch[r0 + r];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
          const int col = ct * 16 + (lane & 15);
          u2v hv, lv;
#pragma unroll
          for (int r = 0; r < 2; ++r) {
            unsigned h, l;
            split_bf2(acc[s][ct][2 * r] * sc[2 * r], acc[s][ct][2 * r + 1] * sc[2 * r + 1], h, l);
            hv[r] = h;
            lv[r] = l;
          }
          *reinterpret_cast<u2v*>(&Lhi[col * KP + koff + r0]) = hv;
          *reinterpret_cast<u2v*>(&Llo[col * KP + koff + r0]) = lv;
          acc[s][ct] = f4{0.f, 0.f, 0.f, 0.f};
        }
      }
    }
    __syncthreads();
    gemm_bf16<SLOTS, KSM, GemmPD<KSM>::value>(reinterpret_cast<const us8*>(g.A2), frag_stride,
                                              g.KS, rt0, HW, lane, nslot, Lhi, Llo, KP, koff, acc);
  }
  __syncthreads();   // the LDS tile is reused for the output
  float* T = reinterpret_cast<float*>(lds_bf);
  acc_rows_to_lds<SLOTS>(T, acc, rt0, HW, lane, nslot);
  __syncthreads();
  if (FUSED || g.dir != 0)
    tile_epilogue<EPI, NW, OUT_EVEN_ODD>(g, T, bofs, c0, pslot, RTh * 16);
  else
    tile_epilogue<EPI, NW, OUT_HALF_ORDER>(g, T, bofs, c0, pslot, RTh * 16);
  __syncthreads();   // LDS free for the next tile
}

// ------------------------------------------------------------------------------------
// float32 variant (v_mfma_f32_16x16x4_f32) with the same even/odd decomposition, spectral
// half order and per-slice operator (dir 2) as the split-bfloat16 one; four wavefronts,
// the first two on the even half, the others on the odd half. Packed matrices: row tiles
// [0, RTh) even, [RTh, 2 RTh) odd, KS = 4 RTh steps of 4 over the half's contraction
// (padded to whole 16-row tiles, so a half's spectral rows fit its contraction block).
// LDS tile [k][col] (row stride DCT_NT + 4): the even block in rows [0, 4 KS), the odd
// block after it; the output reuses it as [row][col].
// ------------------------------------------------------------------------------------
template <int SLOTS>
__device__ __forceinline__ void gemm_f32_half(const float* __restrict__ A, int KS, int rt0,
                                              int rstep, int lane, int nslot, const float* L,
                                              f4 (&acc)[SLOTS][4]) {
  const int LD = DCT_NT + 4;
  for (int ks = 0; ks < KS; ++ks) {
    float bv[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) bv[ct] = L[(ks * 4 + (lane >> 4)) * LD + ct * 16 + (lane & 15)];
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      if (s < nslot) {
        const float av = A[((size_t)(rt0 + rstep * s) * KS + ks) * 64 + lane];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
          acc[s][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv[ct], acc[s][ct], 0, 0, 0);
      }
    }
  }
}

// KSH: maximum steps of 4 of one half (half length <= 4 KSH); SLOTS: row tiles per
// wavefront (RTh <= 2 SLOTS).
template <bool FUSED, int EPI, int KSH, int SLOTS>
__device__ __forceinline__ void dct_f32_body(const GemmArgs& g, int batch, int c0, int pslot,
                                             float* lds_f) {
  constexpr int LD = DCT_NT + 4;
  const int N = g.rows, ce = (N + 1) / 2, fo = N / 2;
  const int KPh = g.KS * 4;                        // contraction rows of one half
  const int RTh = g.RT / 2;
  const bool fwd_in = FUSED || g.dir != 1;
  const size_t bofs = (size_t)batch * g.bstride;
  const float* in = g.in + bofs + c0;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  {
    // fill: thread (column lane, rows q = wave + 4 i of both halves); all loads first
    const unsigned lane4 = (unsigned)lane * 4u;
    const bool cok = c0 + lane < g.ncol;
    float va[KSH], vb[KSH];
#pragma unroll
    for (int it = 0; it < KSH; ++it) {
      const int q = wave + 4 * it;
      // forward: x_q and x_{N-1-q}; inverse: spectral rows q (even) and c + q (odd)
      const bool oka = cok && it < g.KS && q < ce;
      const bool okb = cok && it < g.KS && q < fo;
      const int rb = fwd_in ? N - 1 - q : ce + q;
      va[it] = oka ? ld_at<float>(in + (size_t)q * g.ld, lane4) : 0.0f;
      vb[it] = okb ? ld_at<float>(in + (size_t)(okb ? rb : 0) * g.ld, lane4) : 0.0f;
    }
#pragma unroll
    for (int it = 0; it < KSH; ++it) {
      const int q = wave + 4 * it;
      if (it < g.KS) {
        const float a = va[it], b = vb[it];
        // forward: the pair sum / difference (b = 0 for q >= f, so s_mid = x_mid)
        float ev = fwd_in ? a + b : a;
        float od = fwd_in ? a - b : b;
        if (fwd_in && q >= fo) od = 0.0f;
        lds_f[q * LD + lane] = ev;
        lds_f[(KPh + q) * LD + lane] = od;
      }
    }
  }
  __syncthreads();
  const int half = wave >> 1, lw = wave & 1;
  const int rt0 = half * RTh + lw;                 // row tiles rt0 + 2 s of this half
  const int nslot = (RTh - lw + 1) / 2;
  const float* Lh = lds_f + (size_t)half * KPh * LD;
  f4 acc[SLOTS][4];
#pragma unroll
  for (int s = 0; s < SLOTS; ++s)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[s][ct] = f4{0.f, 0.f, 0.f, 0.f};
  const float* A1 = reinterpret_cast<const float*>(g.A1) + (size_t)batch * g.a_bstride;
  gemm_f32_half<SLOTS>(A1, g.KS, rt0, 2, lane, nslot, Lh, acc);
  if (FUSED) {
    // spectral scale rho / (rho + alpha (lambda_row + lambda_batch)) in half order, written
    // over this half's input block (rows < 16 RTh = KPh), then the inverse from it
    const float rho = (float)g.st->rho;
    const float lb = (g.lam_batch != nullptr) ? g.lam_batch[batch] : 0.0f;
    const int cnt = half ? fo : ce;
    __syncthreads();   // all waves finished reading the input tile
    float* Lw = lds_f + (size_t)half * KPh * LD;
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      if (s < nslot) {
        const int r0 = (lw + 2 * s) * 16 + (lane >> 4) * 4;   // spectral row within the half
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = r0 + r;
          const float sc = (row < cnt) ? rho * rcp_f(rho + g.alpha * (g.lam_row[half * ce + row] + lb)) : 0.0f;
#pragma unroll
          for (int ct = 0; ct < 4; ++ct) Lw[row * LD + ct * 16 + (lane & 15)] = acc[s][ct][r] * sc;
        }
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[s][ct] = f4{0.f, 0.f, 0.f, 0.f};
      }
    }
    __syncthreads();
    gemm_f32_half<SLOTS>(reinterpret_cast<const float*>(g.A2), g.KS, rt0, 2, lane, nslot, Lh,
                         acc);
  }
  __syncthreads();   // the LDS tile is reused for the output
  acc_rows_to_lds<SLOTS>(lds_f, acc, rt0, 2, lane, nslot);
  __syncthreads();
  if (FUSED || g.dir != 0)
    tile_epilogue<EPI, 4, OUT_EVEN_ODD>(g, lds_f, bofs, c0, pslot, RTh * 16);
  else
    tile_epilogue<EPI, 4, OUT_HALF_ORDER>(g, lds_f, bofs, c0, pslot, RTh * 16);
  __syncthreads();
}

// dynamic LDS bytes of one tile

// ------------------------------------------------------------------------------------
}  // namespace epi
