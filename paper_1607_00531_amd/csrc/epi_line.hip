// Line-parallel kernels: one wavefront per PE line, lines staged through LDS.
//
// Section 3: the distance term couples faces only along a PE line (averaging A1 and short
// differences D1 act inside a line), so its residual, gradient and Gauss-Newton Hessian
// (tridiagonal per line) are computed line by line. The cross-line part of the
// regulariser (D2, D3) is added from the neighbouring lines where needed.
#include "epi_device.hpp"
#include "epi_common.hpp"
#include "epi_launch.hpp"
#include "epi_line_body.hpp"

namespace epi {

// ------------------------------------------------------------------------------------
// Objective / gradient / Gauss-Newton pack (eq. D, eq. S, eq. P, eq. dJ, eq. dJGN).
// MODE 0: partial sums only; MODE 1: + gradient; MODE 2: + gradient + line tridiagonal
// of H_D + alpha v D1'D1 + Hess P + gamma I. If d != null the field is b + lam d with
// lam = 2^-trial (line search trial; skipped once the line search has accepted).
// ------------------------------------------------------------------------------------
template <int P, int MODE, int MODEL>
__global__ __launch_bounds__(256) void k_eval(LineArgs a, const float* __restrict__ bsrc,
                                               const float* __restrict__ dsrc, int trial,
                                               int with_pen, float* __restrict__ grad,
                                               float* __restrict__ hdiag,
                                               float* __restrict__ hoff, double* partial,
                                               const DevState* st) {
  if (dsrc != nullptr && st->ls_done) return;
  // per wave: the two image lines, its own field line (read by the neighbouring waves too),
  // the k - 1 and k + 1 lines and, for the workgroup's end waves, the outer j neighbour
  __shared__ float sraw[EPI_LINE_WAVES][LinePad + 6 * LineBuf<P>::SIZE];
  const auto sbuf = [&](int w, int q) { return &sraw[w][LinePad + q * LineBuf<P>::SIZE]; };
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int blk = xcd_remap(blockIdx.x, a.nblk);
  const int line = blk * EPI_LINE_WAVES + wave;
  const bool valid = line < a.L;
  const int lc = valid ? line : 0;
  const int jj = lc % a.m2, kk = lc / a.m2;
  const int NF = a.M + 1;
  const float lam = (dsrc != nullptr) ? ldexpf(1.0f, -trial) : 0.0f;
  const bool j0 = jj > 0, j1 = jj < a.m2 - 1, k0 = kk > 0, k1 = kk < a.m3 - 1;
  const bool jm_lds = j0 && wave > 0, jp_lds = j1 && wave < EPI_LINE_WAVES - 1;
  const int jo = (wave == 0) ? lc - 1 : lc + 1;
  const bool jo_need = (wave == 0) ? j0 : (wave == EPI_LINE_WAVES - 1 ? j1 : false);
  float* sIp = sbuf(wave, 0);
  float* sIm = sbuf(wave, 1);
  float b[P], nb[4][P];   // nb: j - 1, j + 1, k - 1, k + 1 (a missing neighbour: b itself)
  {
    // every global load of the wavefront in one round trip (a second one for d)
    const float* srcs[6] = {a.Ip + (size_t)lc * a.M, a.Im + (size_t)lc * a.M,
                            bsrc + (size_t)lc * NF,
                            bsrc + (size_t)(k0 ? lc - a.m2 : lc) * NF,
                            bsrc + (size_t)(k1 ? lc + a.m2 : lc) * NF,
                            bsrc + (size_t)(jo_need ? jo : lc) * NF};
    const int cnt[6] = {a.M, a.M, NF, NF, NF, NF};
    float v[6][P];
    load_line_n<P, 6>(srcs, cnt, valid, v, lane);
    if (dsrc != nullptr) {
      const float* dsr[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) dsr[q] = dsrc + (srcs[2 + q] - bsrc);
      const int dc[4] = {NF, NF, NF, NF};
      float w[4][P];
      load_line_n<P, 4>(dsr, dc, valid, w, lane);
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int j = 0; j < P; ++j) v[2 + q][j] = fmaf(lam, w[q][j], v[2 + q][j]);
    }
#pragma unroll
    for (int q = 0; q < 6; ++q)
#pragma unroll
      for (int j = 0; j < P; ++j) sbuf(wave, q)[lds_pad(lane + 64 * j)] = v[q][j];
    if (MODEL == 1) {
      pad_spline_line(sIp, a.M, lane);
      pad_spline_line(sIm, a.M, lane);
    }
    __syncthreads();
    const float* own = sbuf(wave, 2);
    const float* jm = jm_lds ? sbuf(wave - 1, 2) : (wave == 0 && j0 ? sbuf(wave, 5) : own);
    const float* jp = jp_lds ? sbuf(wave + 1, 2)
                             : (wave == EPI_LINE_WAVES - 1 && j1 ? sbuf(wave, 5) : own);
    const float* km = k0 ? sbuf(wave, 3) : own;
    const float* kp = k1 ? sbuf(wave, 4) : own;
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const int t = lds_pad(P * lane + j);
      b[j] = own[t];
      nb[0][j] = jm[t];
      nb[1][j] = jp[t];
      nb[2][j] = km[t];
      nb[3][j] = kp[t];
    }
    // the field lines are read by other waves only before this barrier; after it each wave
    // reuses its own buffers 3..5 for the output staging
    __syncthreads();
  }

  // the transverse terms first (the sum for S and the cross-line Laplacian of the
  // gradient), so that the four neighbour lines are dead before the interpolation
  double acc[NQ_EVAL] = {0, 0, 0, 0, 0, 0};
  float lapx[P];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int i = P * lane + j;
    if (valid && i < NF) {
      const float d2 = nb[1][j] - b[j];   // forward difference to j+1 (0 if absent)
      const float d3 = nb[3][j] - b[j];   // forward difference to k+1 (0 if absent)
      acc[2] += (double)d2 * d2 * a.inv_h2sq + (double)d3 * d3 * a.inv_h3sq;
    }
    lapx[j] = ((b[j] - nb[0][j]) + (b[j] - nb[1][j])) * a.inv_h2sq +
              ((b[j] - nb[2][j]) + (b[j] - nb[3][j])) * a.inv_h3sq;
  }

  Cells<P> C;
  eval_cells<P, false, MODEL>(a, b, sIp, sIm, lane, C);

  float phid[P], phidd[P];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int c = P * lane + j;
    phid[j] = 0.0f;
    phidd[j] = 0.0f;
    if (valid && c < a.M) {
      acc[0] += (double)C.r[j] * C.r[j];
      acc[1] += (double)C.g[j] * C.g[j];
      const float x = C.g[j];
      if (fabsf(x) < 1.0f) {
        if (with_pen) {
          float ph, d1, d2;
          phi_terms(x, ph, d1, d2);
          acc[3] += (double)ph;
          phid[j] = d1;
          phidd[j] = d2;
        }
      } else {
        acc[4] += 1.0;
      }
    }
  }

  if (MODE >= 1) {
    float rpJ[P], Jrr[P], gprev[P], phdprev[P];
#pragma unroll
    for (int j = 0; j < P; ++j) Jrr[j] = C.Jr[j] * C.r[j];
    prev_cell<P>(Jrr, rpJ, lane);
    prev_cell<P>(C.g, gprev, lane);
    prev_cell<P>(phid, phdprev, lane);
    const float av = a.alpha * a.v;
    float out[3][P];
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const int i = P * lane + j;
      float gv = a.v * (C.Jl[j] * C.r[j] + rpJ[j]);
      float lap = (gprev[j] - C.g[j]) * a.inv_hp;
      lap += lapx[j];
      gv += av * lap;
      if (with_pen) gv += a.beta * a.v * (phdprev[j] - phid[j]) * a.inv_hp;
      out[0][j] = (i < NF) ? gv : 0.0f;
      if (valid && i < NF) acc[5] += (double)gv * gv;
    }
    if (MODE == 2) {
      float JrPrev[P], phddPrev[P];
      prev_cell<P>(C.Jr, JrPrev, lane);
      prev_cell<P>(phidd, phddPrev, lane);
      const float qa = a.alpha * a.v * a.inv_hp * a.inv_hp;
      const float qb = a.beta * a.v * a.inv_hp * a.inv_hp;
#pragma unroll
      for (int j = 0; j < P; ++j) {
        const int i = P * lane + j;
        const float ncell = (float)((i < a.M) + (i >= 1 && i <= a.M));
        float dgv = a.v * (C.Jl[j] * C.Jl[j] + JrPrev[j] * JrPrev[j]) + qa * ncell + a.gamma;
        float ofv = 0.0f;
        if (i < a.M) ofv = a.v * C.Jl[j] * C.Jr[j] - qa;
        if (with_pen) {
          dgv += qb * (phidd[j] + phddPrev[j]);
          if (i < a.M) ofv -= qb * phidd[j];
        }
        out[1][j] = (i < NF) ? dgv : 1.0f;
        out[2][j] = ofv;
      }
      float* dst[3] = {grad + (size_t)lc * NF, hdiag + (size_t)lc * NF, hoff + (size_t)lc * NF};
      stage_out_n<P, 3>(dst, NF, valid, sbuf(wave, 3), out, lane);
    } else if (grad != nullptr) {
      stage_out<P>(grad + (size_t)lc * NF, NF, valid, sbuf(wave, 3), out[0], lane);
    }
  }
  block_partials<NQ_EVAL>(acc, partial, blockIdx.x);
}

// ------------------------------------------------------------------------------------
// Preconditioner application z = Pinv r for one line held by a wave.
// BLOCK: the line tridiagonal with the transverse coupling replaced by its diagonal
// (eq. Pblock); JACOBI: diagonal of H_JGN; NONE: identity.
// ------------------------------------------------------------------------------------
template <int P>
__device__ __forceinline__ void precond_apply(const LineArgs& a, int precond, const float (&hd)[P],
                                              const float (&ho)[P], float cd, float (&r)[P],
                                              int lane) {
  const int NF = a.M + 1;
  if (precond == 0) {
    float d[P], e[P];
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const int i = P * lane + j;
      d[j] = (i < NF) ? hd[j] + a.alpha * a.v * cd : 1.0f;
      e[j] = (i < NF - 1) ? ho[j] : 0.0f;
      if (i >= NF) r[j] = 0.0f;
    }
    wave_tridiag_solve<P>(d, e, r, lane);
  } else if (precond == 1) {
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const int i = P * lane + j;
      r[j] = (i < NF) ? r[j] / (hd[j] + a.alpha * a.v * cd) : 0.0f;
    }
  }
}

// PCG start: x = 0, r = -grad, z = Pinv r, p = z; partial sums r.z and r.r.
template <int P>
__global__ __launch_bounds__(256) void k_pcg_init(LineArgs a, int precond,
                                                  const float* __restrict__ grad,
                                                  const float* __restrict__ hdiag,
                                                  const float* __restrict__ hoff,
                                                  float* __restrict__ x, float* __restrict__ r,
                                                  float* __restrict__ z, float* __restrict__ p,
                                                  double* partial) {
  __shared__ float sbuf[EPI_LINE_WAVES][4][LineBuf<P>::SIZE];
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int line = blockIdx.x * EPI_LINE_WAVES + wave;
  const bool valid = line < a.L;
  const int lc = valid ? line : 0;
  const int NF = a.M + 1;
  const size_t base = (size_t)lc * NF;
  // all three lines in one memory round trip
  const float* srcs[3] = {grad + base, hdiag + base, hoff + base};
  const int cnt[3] = {NF, NF, NF};
  float v[3][P];
  stage_in_n<P, 3>(srcs, cnt, valid, &sbuf[wave][0][0], v, lane);
  float o[4][P];   // x = 0, r = -grad, z = p = Pinv r
#pragma unroll
  for (int j = 0; j < P; ++j) {
    o[0][j] = 0.0f;
    o[1][j] = -v[0][j];
    o[2][j] = o[1][j];
  }
  precond_apply<P>(a, precond, v[1], v[2], cross_diag(a, lc % a.m2, lc / a.m2), o[2], lane);
  double acc[NQ_PCG] = {0, 0};
#pragma unroll
  for (int j = 0; j < P; ++j) {
    o[3][j] = o[2][j];
    if (valid && P * lane + j < NF) {
      acc[0] += (double)o[1][j] * o[2][j];
      acc[1] += (double)o[1][j] * o[1][j];
    }
  }
  float* dst[4] = {x + base, r + base, z + base, p + base};
  stage_out_n<P, 4>(dst, NF, valid, &sbuf[wave][0][0], o, lane);
  block_partials<NQ_PCG>(acc, partial, blockIdx.x);
}

// PCG update: x += alpha p, r -= alpha q, z = Pinv r; partial sums r.r and r.z. q = H_JGN p
// is formed here again from p (hjgn_apply, as in the matvec, with the same block -> line
// map so that the j neighbours come from the same LDS exchange), instead of being stored by
// the matvec and read back: the p lines of the k and outer j neighbours are L2 hits, so
// the update reads x, r, p and the Hessian blocks from HBM and writes x, r and z.
template <int P>
__global__ __launch_bounds__(256) void k_pcg_update(LineArgs a, int precond,
                                                    const float* __restrict__ hd,
                                                    const float* __restrict__ ho,
                                                    float* __restrict__ x, float* __restrict__ r,
                                                    float* __restrict__ z,
                                                    const float* __restrict__ p, double* partial,
                                                    const DevState* st) {
  if (st->pcg_done) return;
  __shared__ float sp[EPI_LINE_WAVES][64 * P];   // p of the workgroup's lines, face order
  __shared__ float sbuf[EPI_LINE_WAVES][3][LineBuf<P>::SIZE];
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int blk = xcd_remap(blockIdx.x, a.nblk);
  const int line = blk * EPI_LINE_WAVES + wave;
  const bool lv = line < a.L;
  const int lc = lv ? line : 0;
  const int NF = a.M + 1;
  const int jj = lc % a.m2, kk = lc / a.m2;
  const size_t base = (size_t)lc * NF;
  const float al = (float)st->alpha_cg;
  const bool j0 = jj > 0, j1 = jj < a.m2 - 1, k0 = kk > 0, k1 = kk < a.m3 - 1;
  const bool jm_lds = j0 && wave > 0, jp_lds = j1 && wave < EPI_LINE_WAVES - 1;
  const int jo = (wave == 0) ? lc - 1 : lc + 1;
  const bool jo_need = (wave == 0) ? j0 : (wave == EPI_LINE_WAVES - 1 ? j1 : false);
  const int lines[4] = {lc, k0 ? lc - a.m2 : lc, k1 ? lc + a.m2 : lc, jo_need ? jo : lc};
  // every global load first: p of the four lines, x, r and the Hessian blocks of the own
  float pv[4][P], xv[P], rv[P], hdv[P], hov[P];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int i = lane + 64 * j;
    const int ic = (j < P - 1 || i < NF) ? i : NF - 1;   // in bounds; replaced below
#pragma unroll
    for (int t = 0; t < 4; ++t) pv[t][j] = p[(size_t)lines[t] * NF + ic];
    xv[j] = x[base + ic];
    rv[j] = r[base + ic];
    hdv[j] = hd[base + ic];
    hov[j] = ho[base + ic];
  }
  float pc[P];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int i = lane + 64 * j;
    pc[j] = (lv && (j < P - 1 || i < NF)) ? pv[0][j] : 0.0f;
    sp[wave][i] = pc[j];
  }
  __syncthreads();
  float y[P];
  hjgn_apply<P>(a, NF, lane, j0, j1, k0, k1, pc, hdv, hov, pv[1], pv[2], pv[3],
                jm_lds ? sp[wave - 1] : nullptr, jp_lds ? sp[wave + 1] : nullptr, y);
  // x and r in the lane-contiguous layout (coalesced stores); r and the Hessian blocks
  // (zero past the line, as the preconditioner expects) to the lane-blocked layout
  float t3[3][P];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int i = lane + 64 * j;
    const bool ok = lv && (j < P - 1 || i < NF);
    const float xn = fmaf(al, pc[j], xv[j]);
    const float rn = fmaf(-al, y[j], rv[j]);
    if (ok) {
      store_stream(&x[base + i], xn);
      store_stream(&r[base + i], rn);
    }
    t3[0][j] = ok ? rn : 0.0f;
    t3[1][j] = ok ? hdv[j] : 0.0f;
    t3[2][j] = ok ? hov[j] : 0.0f;
  }
  float v[3][P];
  regs_to_blocked_n<P, 3>(t3, &sbuf[wave][0][0], v, lane);
  float zb[P];
#pragma unroll
  for (int j = 0; j < P; ++j) zb[j] = v[0][j];
  precond_apply<P>(a, precond, v[1], v[2], cross_diag(a, jj, kk), zb, lane);
  double acc[NQ_PCG] = {0, 0};
#pragma unroll
  for (int j = 0; j < P; ++j) {
    if (lv && P * lane + j < NF) {
      acc[0] += (double)v[0][j] * v[0][j];
      acc[1] += (double)v[0][j] * zb[j];
    }
  }
  stage_out<P>(z + base, NF, lv, &sbuf[wave][0][0], zb, lane);
  block_partials<NQ_PCG>(acc, partial, blockIdx.x);
}

// z = Pinv r for the line-local preconditioners (BLOCK, JACOBI, NONE) on their own.
template <int P>
__global__ __launch_bounds__(256) void k_precond(LineArgs a, int precond,
                                                 const float* __restrict__ hdiag,
                                                 const float* __restrict__ hoff,
                                                 const float* __restrict__ r,
                                                 float* __restrict__ z) {
  __shared__ float sbuf[EPI_LINE_WAVES][3][LineBuf<P>::SIZE];
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int line = blockIdx.x * EPI_LINE_WAVES + wave;
  const bool valid = line < a.L;
  const int lc = valid ? line : 0;
  const int NF = a.M + 1;
  const size_t base = (size_t)lc * NF;
  const float* srcs[3] = {r + base, hdiag + base, hoff + base};
  const int cnt[3] = {NF, NF, NF};
  float v[3][P];
  stage_in_n<P, 3>(srcs, cnt, valid, &sbuf[wave][0][0], v, lane);
  precond_apply<P>(a, precond, v[1], v[2], cross_diag(a, lc % a.m2, lc / a.m2), v[0], lane);
  stage_out<P>(z + base, NF, valid, &sbuf[wave][0][0], v[0], lane);
}

// ------------------------------------------------------------------------------------
// Symmetric Gauss-Seidel preconditioner (eq. Psgs): z = (U + Dg)^-1 Dg (L + Dg)^-1 r with
// H_JGN = L + Dg + U split in the face order i + (M+1)(j + m2 k). In that order the lower
// neighbours of face (i, j, k) are (i-1, j, k), (i, j-1, k) and (i, j, k-1), so the lines
// of one anti-diagonal j + k = s depend only on the lines of s - 1: each launch takes one
// such level (one wavefront per line), the forward sweep from s = 0 up, the backward sweep
// from the last level down. Along a line the triangular solve is the first-order
// recurrence x_i = a_i x_{i-1} + b_i (x_{i+1} backward), evaluated by a wave-parallel
// scan of affine maps: the same triangular solves as the sequential sweep, summed in a
// different order.
// ------------------------------------------------------------------------------------

// Inclusive scan of the affine maps x -> A x + B over the blocked elements of a line,
// lower indices applied first (BACK: higher indices first); returns x per element for a
// zero value entering the line.
template <int P, bool BACK>
__device__ __forceinline__ void wave_affine_scan(const float (&av)[P], const float (&bv)[P],
                                                 float (&x)[P], int lane) {
  float A = 1.0f, B = 0.0f;
#pragma unroll
  for (int t = 0; t < P; ++t) {
    const int j = BACK ? P - 1 - t : t;
    B = fmaf(av[j], B, bv[j]);
    A *= av[j];
  }
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const float An = BACK ? __shfl_down(A, d, 64) : __shfl_up(A, d, 64);
    const float Bn = BACK ? __shfl_down(B, d, 64) : __shfl_up(B, d, 64);
    const bool has = BACK ? lane + d < 64 : lane >= d;
    if (has) {
      B = fmaf(A, Bn, B);
      A *= An;
    }
  }
  float xin = BACK ? shfl_down0(B, 1, lane) : shfl_up0(B, 1, lane);
#pragma unroll
  for (int t = 0; t < P; ++t) {
    const int j = BACK ? P - 1 - t : t;
    xin = fmaf(av[j], xin, bv[j]);
    x[j] = xin;
  }
}

// One level s of a sweep: lines (j, k) with j + k = s, k from kmin. Forward: z holds the
// forward solution y of the lower levels and receives y on this level. Backward: z holds
// y on this and the lower levels and z on the higher ones; this level's y becomes z.
// gate: skip when the PCG has already stopped (not for the PCG start).
template <int P, bool BACK>
__global__ __launch_bounds__(256) void k_sgs_level(LineArgs a, int level, int kmin, int count,
                                                   const float* __restrict__ hdiag,
                                                   const float* __restrict__ hoff,
                                                   const float* __restrict__ r, float* z,
                                                   const DevState* st, int gate) {
  if (gate && st->pcg_done) return;
  __shared__ float sbuf[EPI_LINE_WAVES][5][LineBuf<P>::SIZE];
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int w = blockIdx.x * EPI_LINE_WAVES + wave;
  const bool valid = w < count;
  const int kk = kmin + (valid ? w : 0), jj = level - kk;
  const int NF = a.M + 1;
  const size_t base = (size_t)(jj + a.m2 * kk) * NF;
  const size_t plane = (size_t)a.m2 * NF;
  const float av = a.alpha * a.v;
  // the two transverse neighbours on the already solved side (own line when absent)
  const bool n2 = BACK ? jj < a.m2 - 1 : jj > 0;
  const bool n3 = BACK ? kk < a.m3 - 1 : kk > 0;
  const float c2 = n2 ? av * a.inv_h2sq : 0.0f, c3 = n3 ? av * a.inv_h3sq : 0.0f;
  const float* own = BACK ? z + base : r + base;
  const float* srcs[5] = {own, hdiag + base, hoff + base,
                          n2 ? (BACK ? z + base + NF : z + base - NF) : own,
                          n3 ? (BACK ? z + base + plane : z + base - plane) : own};
  const int cnt[5] = {NF, NF, NF, NF, NF};
  float v[5][P];
  stage_in_n<P, 5>(srcs, cnt, valid, &sbuf[wave][0][0], v, lane);
  const float dgx = av * cross_diag(a, jj, kk);
  float oprev[P];
  prev_cell<P>(v[2], oprev, lane);
  float ca[P], cb[P], x[P];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int i = P * lane + j;
    const float dg = v[1][j] + dgx;
    const float idg = (i < NF) ? 1.0f / dg : 0.0f;
    const float tr = fmaf(c2, v[3][j], c3 * v[4][j]);
    if (BACK) {
      // Dg_i z_i + o_i z_{i+1} = Dg_i y_i + c2 z(j+1) + c3 z(k+1)
      ca[j] = (i < NF - 1) ? -v[2][j] * idg : 0.0f;
      cb[j] = (i < NF) ? fmaf(tr, idg, v[0][j]) : 0.0f;
    } else {
      // Dg_i y_i + o_{i-1} y_{i-1} = r_i + c2 y(j-1) + c3 y(k-1)
      ca[j] = (i >= 1) ? -oprev[j] * idg : 0.0f;
      cb[j] = (v[0][j] + tr) * idg;
    }
  }
  wave_affine_scan<P, BACK>(ca, cb, x, lane);
  stage_out<P>(z + base, NF, valid, &sbuf[wave][0][0], x, lane);
}

template <int P, int MODEL>
__global__ __launch_bounds__(256) void k_admm_bstep(LineArgs a, float* __restrict__ bvec,
                                                    const float* __restrict__ zvec,
                                                    const float* __restrict__ uvec,
                                                    float* __restrict__ wvec, int* hard_list,
                                                    DevState* st) {
  if (st->admm_done) return;
  __shared__ float sbuf[EPI_LINE_WAVES][LinePad + 5 * LineBuf<P>::SIZE];
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int line = blockIdx.x * EPI_LINE_WAVES + wave;
  const bool valid = line < a.L;
  const bool hard = bstep_line_body<P, MODEL>(a, (float)st->rho, (float)st->u_scale, bvec, zvec, uvec, wvec,
                                       valid ? line : 0, valid, &sbuf[wave][LinePad], lane,
                                       &st->numeric_bad);
  if (valid && hard && lane == 0) {
    const int idx = atomicAdd(&st->hard_count, 1);
    if (idx < a.L) hard_list[idx] = line;   // hard_list holds L entries
  }
}

// Distortion-corrected images (Section 2, the model relation behind eq. D):
// I+(x + A b)(1 + D1 b) and I-(x - A b)(1 - D1 b) at the cell centres of each line, and
// float64 sums of the pair for the SSD and NCC quality measures. outp / outm may be null.
template <int P, int MODEL>
__global__ __launch_bounds__(256) void k_correct(LineArgs a, const float* __restrict__ bsrc,
                                                 float* __restrict__ outp,
                                                 float* __restrict__ outm, double* partial) {
  __shared__ float sraw[EPI_LINE_WAVES][LinePad + 4 * LineBuf<P>::SIZE];
  float* sw = &sraw[threadIdx.x >> 6][LinePad];
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int line = xcd_remap(blockIdx.x, a.nblk) * EPI_LINE_WAVES + wave;
  const bool valid = line < a.L;
  const int lc = valid ? line : 0;
  const int NF = a.M + 1;
  const float* srcs[3] = {a.Ip + (size_t)lc * a.M, a.Im + (size_t)lc * a.M,
                          bsrc + (size_t)lc * NF};
  const int cnt[3] = {a.M, a.M, NF};
  float v[3][P];
  stage_in_n<P, 3>(srcs, cnt, valid, sw, v, lane);
  float* sIp = sw;
  float* sIm = sw + LineBuf<P>::SIZE;
  if (MODEL == 1) {
    pad_spline_line(sIp, a.M, lane);
    pad_spline_line(sIm, a.M, lane);
  }
  const float bnext = shfl_down0(v[2][0], 1, lane);
  float ov[2][P];
  double acc[NQ_QUALITY] = {0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int c = P * lane + j;
    const float bl = v[2][j], br = (j < P - 1) ? v[2][j + 1] : bnext;
    const float aidx = 0.5f * (bl + br) * a.inv_hp;
    const float g = (br - bl) * a.inv_hp;
    float ipv, ipd, imv, imd;
    if (MODEL == 1) {
      interp_spline_lds(sIp, a.M, c, aidx, a.inv_hp, ipv, ipd);
      interp_spline_lds(sIm, a.M, c, -aidx, a.inv_hp, imv, imd);
    } else {
      interp_lds(sIp, a.M, c, aidx, a.inv_hp, ipv, ipd);
      interp_lds(sIm, a.M, c, -aidx, a.inv_hp, imv, imd);
    }
    const bool in = valid && c < a.M;
    const float cp = in ? ipv * (1.0f + g) : 0.0f;
    const float cm = in ? imv * (1.0f - g) : 0.0f;
    ov[0][j] = cp;
    ov[1][j] = cm;
    const double dp = cp, dm = cm;
    acc[0] += dp;
    acc[1] += dm;
    acc[2] += dp * dp;
    acc[3] += dm * dm;
    acc[4] += dp * dm;
    acc[5] += (dp - dm) * (dp - dm);
  }
  const bool store = valid && outp != nullptr && outm != nullptr;
  float* outs[2] = {store ? outp + (size_t)lc * a.M : nullptr,
                    store ? outm + (size_t)lc * a.M : nullptr};
  stage_out_n<P, 2>(outs, a.M, store, sw + 2 * LineBuf<P>::SIZE, ov, lane);
  block_partials<NQ_QUALITY>(acc, partial, blockIdx.x);
}

// Hard lines of the b-step: one wavefront per line (see hard_line_body).
template <int P, int MODEL>
__global__ __launch_bounds__(64) void k_admm_bstep_hard(LineArgs a, float* __restrict__ bvec,
                                                        const float* __restrict__ zvec,
                                                        const float* __restrict__ uvec,
                                                        float* __restrict__ wvec,
                                                        const int* hard_list, DevState* st) {
  if (st->admm_done) return;
  const int nhard = min(st->hard_count, a.L);
  if ((int)blockIdx.x >= nhard) return;
  __shared__ HardLds<P> L;
  for (int h = blockIdx.x; h < nhard; h += gridDim.x)
    hard_line_body<P, MODEL>(a, (float)st->rho, (float)st->u_scale, bvec, zvec, uvec, wvec, hard_list[h], L, threadIdx.x,
                      &st->max_active, st->qp_max_iter);
}

// ------------------------------------------------------------------------------------
// Host-side launchers
// ------------------------------------------------------------------------------------
int line_blocks(const LineArgs& a) { return (a.L + EPI_LINE_WAVES - 1) / EPI_LINE_WAVES; }

void launch_eval(hipStream_t s, int P, int mode, LineArgs a, const float* b, const float* d,
                 int trial, int with_pen, float* grad, float* hdiag, float* hoff,
                 double* partial, const DevState* st) {
  const int nb = line_blocks(a);
  a.nblk = nb;
#define EPI_EVAL_LAUNCH(MD, ML)                                                              \
  EPI_DISPATCH_P(P, hipLaunchKernelGGL((k_eval<PP, MD, ML>), dim3(nb), dim3(256), 0, s, a, b, \
                                       d, trial, with_pen, grad, hdiag, hoff, partial, st))
  if (a.model == 1) {
    if (mode == 0) {
      EPI_EVAL_LAUNCH(0, 1);
    } else if (mode == 1) {
      EPI_EVAL_LAUNCH(1, 1);
    } else {
      EPI_EVAL_LAUNCH(2, 1);
    }
  } else {
    if (mode == 0) {
      EPI_EVAL_LAUNCH(0, 0);
    } else if (mode == 1) {
      EPI_EVAL_LAUNCH(1, 0);
    } else {
      EPI_EVAL_LAUNCH(2, 0);
    }
  }
#undef EPI_EVAL_LAUNCH
}

void launch_pcg_init(hipStream_t s, int P, LineArgs a, int precond, const float* grad,
                     const float* hdiag, const float* hoff, float* x, float* r, float* z,
                     float* p, double* partial) {
  const int nb = line_blocks(a);
  EPI_DISPATCH_P(P, hipLaunchKernelGGL((k_pcg_init<PP>), dim3(nb), dim3(256), 0, s, a, precond,
                                       grad, hdiag, hoff, x, r, z, p, partial));
}

void launch_pcg_update(hipStream_t s, int P, LineArgs a, int precond, const float* hdiag,
                       const float* hoff, float* x, float* r, float* z, const float* p,
                       double* partial, const DevState* st) {
  const int nb = line_blocks(a);
  a.nblk = nb;
  EPI_DISPATCH_P(P, hipLaunchKernelGGL((k_pcg_update<PP>), dim3(nb), dim3(256), 0, s, a,
                                       precond, hdiag, hoff, x, r, z, p, partial, st));
}

void launch_correct(hipStream_t s, int P, LineArgs a, const float* b, float* outp, float* outm,
                    double* partial) {
  const int nb = line_blocks(a);
  a.nblk = nb;
  if (a.model == 1) {
    EPI_DISPATCH_P(P, hipLaunchKernelGGL((k_correct<PP, 1>), dim3(nb), dim3(256), 0, s, a, b,
                                         outp, outm, partial));
  } else {
    EPI_DISPATCH_P(P, hipLaunchKernelGGL((k_correct<PP, 0>), dim3(nb), dim3(256), 0, s, a, b,
                                         outp, outm, partial));
  }
}

void launch_precond(hipStream_t s, int P, LineArgs a, int precond, const float* hdiag,
                    const float* hoff, const float* r, float* z) {
  const int nb = line_blocks(a);
  EPI_DISPATCH_P(P, hipLaunchKernelGGL((k_precond<PP>), dim3(nb), dim3(256), 0, s, a, precond,
                                       hdiag, hoff, r, z));
}

void launch_sgs(hipStream_t s, int P, LineArgs a, const float* hdiag, const float* hoff,
                const float* r, float* z, const DevState* st, int gate) {
  const int levels = a.m2 + a.m3 - 1;
  for (int t = 0; t < 2 * levels; ++t) {
    const bool back = t >= levels;
    const int lev = back ? 2 * levels - 1 - t : t;
    const int kmin = lev - (a.m2 - 1) > 0 ? lev - (a.m2 - 1) : 0;
    const int kmax = lev < a.m3 - 1 ? lev : a.m3 - 1;
    const int count = kmax - kmin + 1;
    const int nb = (count + EPI_LINE_WAVES - 1) / EPI_LINE_WAVES;
    if (back) {
      EPI_DISPATCH_P(P, hipLaunchKernelGGL((k_sgs_level<PP, true>), dim3(nb), dim3(256), 0, s,
                                           a, lev, kmin, count, hdiag, hoff, r, z, st, gate));
    } else {
      EPI_DISPATCH_P(P, hipLaunchKernelGGL((k_sgs_level<PP, false>), dim3(nb), dim3(256), 0, s,
                                           a, lev, kmin, count, hdiag, hoff, r, z, st, gate));
    }
  }
}

void launch_admm_bstep_part(hipStream_t s, int part, int P, LineArgs a, float* b,
                            const float* z, const float* u, float* w, int* hard_list,
                            DevState* st, int hard_blocks) {
  const int nb = line_blocks(a);
  if (part == 0 && a.model == 1) {
    EPI_DISPATCH_P(P, hipLaunchKernelGGL((k_admm_bstep<PP, 1>), dim3(nb), dim3(256), 0, s, a,
                                         b, z, u, w, hard_list, st));
  } else if (part == 0) {
    EPI_DISPATCH_P(P, hipLaunchKernelGGL((k_admm_bstep<PP, 0>), dim3(nb), dim3(256), 0, s, a,
                                         b, z, u, w, hard_list, st));
  } else if (a.model == 1) {
    EPI_DISPATCH_P(P, hipLaunchKernelGGL((k_admm_bstep_hard<PP, 1>), dim3(hard_blocks),
                                         dim3(64), 0, s, a, b, z, u, w, hard_list, st));
  } else {
    EPI_DISPATCH_P(P, hipLaunchKernelGGL((k_admm_bstep_hard<PP, 0>), dim3(hard_blocks),
                                         dim3(64), 0, s, a, b, z, u, w, hard_list, st));
  }
}

void launch_admm_bstep(hipStream_t s, int P, LineArgs a, float* b, const float* z,
                       const float* u, float* w, int* hard_list, DevState* st, int hard_blocks,
                       const std::function<void(int)>& before,
                       const std::function<void()>& after) {
  for (int part = 0; part < 2; ++part) {
    before(part);
    launch_admm_bstep_part(s, part, P, a, b, z, u, w, hard_list, st, hard_blocks);
    after();
  }
}

}  // namespace epi
