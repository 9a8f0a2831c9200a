// Line-parallel kernels: one wavefront per PE line, lines staged through LDS.
//
// Section 3: the distance term couples faces only along a PE line (averaging A1 and short
// differences D1 act inside a line), so its residual, gradient and Gauss-Newton Hessian
// (tridiagonal per line) are computed line by line. The cross-line part of the
// regulariser (D2, D3) is added from the neighbouring lines where needed.
#include "epi_device.hpp"
#include "epi_common.hpp"
#include "epi_launch.hpp"

namespace epi {

// 1D linear interpolation of the cell-centred samples of one line held in LDS at index
// coordinate c + disp (sample c sits at index c); zero outside the M samples; derivative
// with respect to the physical PE coordinate from the segment [k, k+1], k = floor(c + disp)
// (the right-hand segment at a knot). The floor is taken of the displacement alone and
// the integer cell index added afterwards: rounding c + disp in float32 would move small
// displacements (|disp| < ulp(c) / 2) onto the knot and pick the wrong segment.
__device__ __forceinline__ void interp_lds(const float* sT, int M, int c, float disp,
                                           float inv_hp, float& val, float& der) {
  disp = fminf(fmaxf(disp, -(float)(2 * M + 4)), (float)(2 * M + 4));
  const float fl = floorf(disp);
  const int k = c + (int)fl;
  const float f = disp - fl;
  if (k < -1 || k > M - 1) {
    val = 0.0f;
    der = 0.0f;
    return;
  }
  const float t0 = (k >= 0) ? sT[lds_pad(k)] : 0.0f;
  const float t1 = (k + 1 <= M - 1) ? sT[lds_pad(k + 1)] : 0.0f;
  val = fmaf(f, t1 - t0, t0);
  der = (t1 - t0) * inv_hp;
}

// Per-cell quantities of the residual for the cells c = P*lane + j (zero for c >= M):
// g = D1 b, r = I+(x + A b)(1 + g) - I-(x - A b)(1 - g) and the two Jacobian entries
// dr_c/db_c = Jl, dr_c/db_{c+1} = Jr.
template <int P>
struct Cells {
  float g[P], r[P], Jl[P], Jr[P];
};

template <int P>
__device__ __forceinline__ void eval_cells(const LineArgs& a, const float (&b)[P],
                                           const float* sIp, const float* sIm, int lane,
                                           Cells<P>& C) {
  const float bnext = shfl_down0(b[0], 1, lane);
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int c = P * lane + j;
    const float bR = (j < P - 1) ? b[j + 1] : bnext;
    if (c < a.M) {
      const float aidx = 0.5f * (b[j] + bR) * a.inv_hp;
      const float g = (bR - b[j]) * a.inv_hp;
      float ipv, ipd, imv, imd;
      interp_lds(sIp, a.M, c, aidx, a.inv_hp, ipv, ipd);
      interp_lds(sIm, a.M, c, -aidx, a.inv_hp, imv, imd);
      const float gp = 1.0f + g, gm = 1.0f - g;
      C.g[j] = g;
      C.r[j] = ipv * gp - imv * gm;
      const float Sd = ipd * gp + imd * gm, Tv = ipv + imv;
      C.Jl[j] = 0.5f * Sd - Tv * a.inv_hp;
      C.Jr[j] = 0.5f * Sd + Tv * a.inv_hp;
    } else {
      C.g[j] = 0.0f;
      C.r[j] = 0.0f;
      C.Jl[j] = 0.0f;
      C.Jr[j] = 0.0f;
    }
  }
}

// Value of a per-cell array at cell (face index - 1) for each local face j.
template <int P>
__device__ __forceinline__ void prev_cell(const float (&x)[P], float (&out)[P], int lane) {
  const float pl = shfl_up0(x[P - 1], 1, lane);
  out[0] = pl;
#pragma unroll
  for (int j = 1; j < P; ++j) out[j] = x[j - 1];
}

// Number of transverse neighbours divided by h^2 (diagonal of D2'D2 + D3'D3) of line
// (j, k).
__device__ __forceinline__ float cross_diag(const LineArgs& a, int jj, int kk) {
  float s = 0.0f;
  if (a.m2 > 1) s += ((jj > 0) + (jj < a.m2 - 1)) * a.inv_h2sq;
  if (a.m3 > 1) s += ((kk > 0) + (kk < a.m3 - 1)) * a.inv_h3sq;
  return s;
}

// ------------------------------------------------------------------------------------
// Objective / gradient / Gauss-Newton pack (eq. D, eq. S, eq. P, eq. dJ, eq. dJGN).
// MODE 0: partial sums only; MODE 1: + gradient; MODE 2: + gradient + line tridiagonal
// of H_D + alpha v D1'D1 + Hess P + gamma I. If d != null the field is b + lam d with
// lam = 2^-trial (line search trial; skipped once the line search has accepted).
// ------------------------------------------------------------------------------------
template <int P, int MODE>
__global__ __launch_bounds__(256) void k_eval(LineArgs a, const float* __restrict__ bsrc,
                                               const float* __restrict__ dsrc, int trial,
                                               int with_pen, float* __restrict__ grad,
                                               float* __restrict__ hdiag,
                                               float* __restrict__ hoff, double* partial,
                                               const DevState* st) {
  if (dsrc != nullptr && st->ls_done) return;
  __shared__ float sbuf[EPI_LINE_WAVES][7][LineBuf<P>::SIZE];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int blk = xcd_remap(blockIdx.x, a.nblk);
  const int line = blk * EPI_LINE_WAVES + wave;
  const bool valid = line < a.L;
  const int lc = valid ? line : 0;
  const int jj = lc % a.m2, kk = lc / a.m2;
  const int NF = a.M + 1;
  const float lam = (dsrc != nullptr) ? ldexpf(1.0f, -trial) : 0.0f;

  float* sIp = sbuf[wave][0];
  float* sIm = sbuf[wave][1];
  for (int t = lane; t < 64 * P; t += 64) {
    sIp[lds_pad(t)] = (valid && t < a.M) ? a.Ip[(size_t)lc * a.M + t] : 0.0f;
    sIm[lds_pad(t)] = (valid && t < a.M) ? a.Im[(size_t)lc * a.M + t] : 0.0f;
  }
  float b[P], nb[4][P];
  {
    float tmp[P];
    stage_in<P>(bsrc + (size_t)lc * NF, NF, valid, sbuf[wave][2], b, lane);
    if (dsrc != nullptr) {
      stage_in<P>(dsrc + (size_t)lc * NF, NF, valid, sbuf[wave][2], tmp, lane);
#pragma unroll
      for (int j = 0; j < P; ++j) b[j] = fmaf(lam, tmp[j], b[j]);
    }
    // transverse neighbours (j-1, j+1, k-1, k+1); missing ones get a copy of b
    const int nl[4] = {jj > 0 ? lc - 1 : -1, jj < a.m2 - 1 ? lc + 1 : -1,
                       kk > 0 ? lc - a.m2 : -1, kk < a.m3 - 1 ? lc + a.m2 : -1};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const bool ok = valid && nl[q] >= 0;
      stage_in<P>(bsrc + (size_t)(ok ? nl[q] : 0) * NF, NF, ok, sbuf[wave][3 + q], nb[q], lane);
      if (dsrc != nullptr) {
        stage_in<P>(dsrc + (size_t)(ok ? nl[q] : 0) * NF, NF, ok, sbuf[wave][3 + q], tmp, lane);
#pragma unroll
        for (int j = 0; j < P; ++j) nb[q][j] = fmaf(lam, tmp[j], nb[q][j]);
      }
      if (!ok) {
#pragma unroll
        for (int j = 0; j < P; ++j) nb[q][j] = b[j];
      }
    }
  }

  Cells<P> C;
  eval_cells<P>(a, b, sIp, sIm, lane, C);

  double acc[NQ_EVAL] = {0, 0, 0, 0, 0, 0};
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
          acc[3] += (double)phi_f(x);
          phid[j] = dphi_f(x);
          phidd[j] = d2phi_f(x);
        }
      } else {
        acc[4] += 1.0;
      }
    }
    const int i = P * lane + j;
    if (valid && i < NF) {
      const float d2 = nb[1][j] - b[j];   // forward difference to j+1 (0 if absent)
      const float d3 = nb[3][j] - b[j];   // forward difference to k+1 (0 if absent)
      acc[2] += (double)d2 * d2 * a.inv_h2sq + (double)d3 * d3 * a.inv_h3sq;
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
    float gout[P];
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const int i = P * lane + j;
      float gv = a.v * (C.Jl[j] * C.r[j] + rpJ[j]);
      float lap = (gprev[j] - C.g[j]) * a.inv_hp;
      lap += ((b[j] - nb[0][j]) + (b[j] - nb[1][j])) * a.inv_h2sq;
      lap += ((b[j] - nb[2][j]) + (b[j] - nb[3][j])) * a.inv_h3sq;
      gv += av * lap;
      if (with_pen) gv += a.beta * a.v * (phdprev[j] - phid[j]) * a.inv_hp;
      gout[j] = (i < NF) ? gv : 0.0f;
      if (valid && i < NF) acc[5] += (double)gv * gv;
    }
    if (grad != nullptr) stage_out<P>(grad + (size_t)lc * NF, NF, valid, sbuf[wave][2], gout, lane);
  }

  if (MODE == 2) {
    float JrPrev[P], phddPrev[P];
    prev_cell<P>(C.Jr, JrPrev, lane);
    prev_cell<P>(phidd, phddPrev, lane);
    const float qa = a.alpha * a.v * a.inv_hp * a.inv_hp;
    const float qb = a.beta * a.v * a.inv_hp * a.inv_hp;
    float dg[P], of[P];
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
      dg[j] = (i < NF) ? dgv : 1.0f;
      of[j] = ofv;
    }
    stage_out<P>(hdiag + (size_t)lc * NF, NF, valid, sbuf[wave][2], dg, lane);
    stage_out<P>(hoff + (size_t)lc * NF, NF, valid, sbuf[wave][2], of, lane);
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
  __shared__ float sbuf[EPI_LINE_WAVES][LineBuf<P>::SIZE];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int line = blockIdx.x * EPI_LINE_WAVES + wave;
  const bool valid = line < a.L;
  const int lc = valid ? line : 0;
  const int NF = a.M + 1;
  const size_t base = (size_t)lc * NF;
  float rv[P], hd[P], ho[P], zv[P], zero[P];
  stage_in<P>(grad + base, NF, valid, sbuf[wave], rv, lane);
  stage_in<P>(hdiag + base, NF, valid, sbuf[wave], hd, lane);
  stage_in<P>(hoff + base, NF, valid, sbuf[wave], ho, lane);
#pragma unroll
  for (int j = 0; j < P; ++j) {
    rv[j] = -rv[j];
    zv[j] = rv[j];
    zero[j] = 0.0f;
  }
  precond_apply<P>(a, precond, hd, ho, cross_diag(a, lc % a.m2, lc / a.m2), zv, lane);
  double acc[NQ_PCG] = {0, 0};
#pragma unroll
  for (int j = 0; j < P; ++j) {
    if (valid && P * lane + j < NF) {
      acc[0] += (double)rv[j] * zv[j];
      acc[1] += (double)rv[j] * rv[j];
    }
  }
  stage_out<P>(x + base, NF, valid, sbuf[wave], zero, lane);
  stage_out<P>(r + base, NF, valid, sbuf[wave], rv, lane);
  stage_out<P>(z + base, NF, valid, sbuf[wave], zv, lane);
  stage_out<P>(p + base, NF, valid, sbuf[wave], zv, lane);
  block_partials<NQ_PCG>(acc, partial, blockIdx.x);
}

// PCG update: x += alpha p, r -= alpha q, z = Pinv r; partial sums r.r and r.z.
template <int P>
__global__ __launch_bounds__(256) void k_pcg_update(LineArgs a, int precond,
                                                    const float* __restrict__ hdiag,
                                                    const float* __restrict__ hoff,
                                                    float* __restrict__ x, float* __restrict__ r,
                                                    float* __restrict__ z,
                                                    const float* __restrict__ p,
                                                    const float* __restrict__ q, double* partial,
                                                    const DevState* st) {
  if (st->pcg_done) return;
  __shared__ float sbuf[EPI_LINE_WAVES][LineBuf<P>::SIZE];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int line = blockIdx.x * EPI_LINE_WAVES + wave;
  const bool valid = line < a.L;
  const int lc = valid ? line : 0;
  const int NF = a.M + 1;
  const size_t base = (size_t)lc * NF;
  const float al = (float)st->alpha_cg;
  float xv[P], rv[P], pv[P], qv[P], hd[P], ho[P];
  stage_in<P>(x + base, NF, valid, sbuf[wave], xv, lane);
  stage_in<P>(r + base, NF, valid, sbuf[wave], rv, lane);
  stage_in<P>(p + base, NF, valid, sbuf[wave], pv, lane);
  stage_in<P>(q + base, NF, valid, sbuf[wave], qv, lane);
  stage_in<P>(hdiag + base, NF, valid, sbuf[wave], hd, lane);
  stage_in<P>(hoff + base, NF, valid, sbuf[wave], ho, lane);
  float zv[P];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    xv[j] = fmaf(al, pv[j], xv[j]);
    rv[j] = fmaf(-al, qv[j], rv[j]);
    zv[j] = rv[j];
  }
  precond_apply<P>(a, precond, hd, ho, cross_diag(a, lc % a.m2, lc / a.m2), zv, lane);
  double acc[NQ_PCG] = {0, 0};
#pragma unroll
  for (int j = 0; j < P; ++j) {
    if (valid && P * lane + j < NF) {
      acc[0] += (double)rv[j] * rv[j];
      acc[1] += (double)rv[j] * zv[j];
    }
  }
  stage_out<P>(x + base, NF, valid, sbuf[wave], xv, lane);
  stage_out<P>(r + base, NF, valid, sbuf[wave], rv, lane);
  stage_out<P>(z + base, NF, valid, sbuf[wave], zv, lane);
  block_partials<NQ_PCG>(acc, partial, blockIdx.x);
}

// ------------------------------------------------------------------------------------
// ADMM b-step (Section 4.2): per PE line, QP data at b^k
//   c = grad D(b^k) + alpha v D1'D1 b^k + rho v (b^k - z^k + u^k)
//   G = H_D(b^k) + alpha v D1'D1 + rho v I          (SPD tridiagonal)
// and the QP  min 1/2 x'Gx + c'x  s.t.  -1 <= D1 (b^k + x) <= 1.
// ------------------------------------------------------------------------------------
template <int P>
__device__ __forceinline__ void qp_data(const LineArgs& a, float rho, const float (&b)[P],
                                        const float (&z)[P], const float (&u)[P],
                                        const float* sIp, const float* sIm, int lane,
                                        float (&Gd)[P], float (&Go)[P], float (&c)[P],
                                        float (&g)[P]) {
  Cells<P> C;
  eval_cells<P>(a, b, sIp, sIm, lane, C);
  float Jrr[P], rpJ[P], gprev[P], JrPrev[P];
#pragma unroll
  for (int j = 0; j < P; ++j) Jrr[j] = C.Jr[j] * C.r[j];
  prev_cell<P>(Jrr, rpJ, lane);
  prev_cell<P>(C.g, gprev, lane);
  prev_cell<P>(C.Jr, JrPrev, lane);
  const int NF = a.M + 1;
  const float rv = rho * a.v;
  const float qa = a.alpha * a.v * a.inv_hp * a.inv_hp;
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int i = P * lane + j;
    g[j] = C.g[j];
    if (i < NF) {
      c[j] = a.v * (C.Jl[j] * C.r[j] + rpJ[j]) +
             a.alpha * a.v * (gprev[j] - C.g[j]) * a.inv_hp + rv * (b[j] - z[j] + u[j]);
      const float ncell = (float)((i < a.M) + (i >= 1));
      Gd[j] = a.v * (C.Jl[j] * C.Jl[j] + JrPrev[j] * JrPrev[j]) + qa * ncell + rv;
      Go[j] = (i < a.M) ? a.v * C.Jl[j] * C.Jr[j] - qa : 0.0f;
    } else {
      c[j] = 0.0f;
      Gd[j] = 1.0f;
      Go[j] = 0.0f;
    }
  }
}

// Tolerances of the float32 active-set logic (relative to the unit bound on |D1 b|).
#define EPI_TOL_ACTIVE 4e-6f

// Fast path: lines whose starting working set is empty and whose unconstrained step
// -G^{-1} c keeps |D1 b| <= 1 are solved by that single tridiagonal solve (the active-set
// method terminates there). Other lines are appended to hard_list, left untouched, and
// solved by k_admm_bstep_hard. Writes b^{k+1} (in place) and w = b^{k+1} + u^k.
template <int P>
__global__ __launch_bounds__(256) void k_admm_bstep(LineArgs a, float* __restrict__ bvec,
                                                    const float* __restrict__ zvec,
                                                    const float* __restrict__ uvec,
                                                    float* __restrict__ wvec, int* hard_list,
                                                    DevState* st) {
  if (st->admm_done) return;
  __shared__ float sbuf[EPI_LINE_WAVES][5][LineBuf<P>::SIZE];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int line = blockIdx.x * EPI_LINE_WAVES + wave;
  const bool valid = line < a.L;
  const int lc = valid ? line : 0;
  const int NF = a.M + 1;
  const size_t base = (size_t)lc * NF;
  const float* srcs[5] = {a.Ip + (size_t)lc * a.M, a.Im + (size_t)lc * a.M, bvec + base,
                          zvec + base, uvec + base};
  const int cnt[5] = {a.M, a.M, NF, NF, NF};
  float v[5][P];
  stage_in_n<P, 5>(srcs, cnt, valid, &sbuf[wave][0][0], v, lane);
  const float* sIp = sbuf[wave][0];
  const float* sIm = sbuf[wave][1];
  float b[P], z[P], u[P];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    b[j] = v[2][j];
    z[j] = v[3][j];
    u[j] = v[4][j];
  }
  const float rho = (float)st->rho;
  float Gd[P], Go[P], c[P], g[P];
  qp_data<P>(a, rho, b, z, u, sIp, sIm, lane, Gd, Go, c, g);
  float x[P];
  bool hard = false;
#pragma unroll
  for (int j = 0; j < P; ++j) {
    x[j] = -c[j];
    if (P * lane + j < a.M && fabsf(g[j]) >= 1.0f - EPI_TOL_ACTIVE) hard = true;
  }
  wave_tridiag_solve<P>(Gd, Go, x, lane);
  const float xnext = shfl_down0(x[0], 1, lane);
  bool bad = false;
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int cidx = P * lane + j;
    if (cidx < a.M) {
      const float xr = (j < P - 1) ? x[j + 1] : xnext;
      const float gn = g[j] + (xr - x[j]) * a.inv_hp;
      if (!(fabsf(gn) <= 1.0f)) hard = true;   // also catches NaN
    }
    if (cidx < NF && !(fabsf(x[j]) < 3.0e38f)) bad = true;
  }
  hard = __any(hard);
  if (bad && valid && lane == 0) atomicAdd(&st->numeric_bad, 1);
  float bn[P], wn[P];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    bn[j] = b[j] + x[j];
    wn[j] = bn[j] + u[j];
  }
  if (valid && hard && lane == 0) {
    const int idx = atomicAdd(&st->hard_count, 1);
    hard_list[idx] = line;
  }
  const bool wr = valid && !hard;
  float* outs[2] = {bvec + base, wvec + base};
  float ov[2][P];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    ov[0][j] = bn[j];
    ov[1][j] = wn[j];
  }
  stage_out_n<P, 2>(outs, NF, wr, &sbuf[wave][2][0], ov, lane);

}

// Primal active-set method for one line (Section 4.2, eq. qp / eq. schurasqp), run by one
// lane on LDS arrays. The equality-constrained subproblem of a working set W (active
// cells fix D1(x + p) to +-1) is solved in the null space of A_W: faces joined by active
// cells move together, which leaves a tridiagonal system in one unknown per group. This
// gives the same KKT point (p, lambda) as the Schur-complement formulation; the
// multiplier of an active cell is a running sum of G p + G x + c over its group.
//   p = 0 (or a full step was just taken) and lambda >= 0: optimal;
//   some lambda < 0: drop the most negative one (lowest cell on ties);
//   otherwise step to the first blocking constraint and add every blocking constraint.
// st_: 0 free, 1 lower bound active (D1 b = -1), 2 upper bound active (D1 b = +1).
__device__ int active_set_serial(int N, float hp, const float* Gd, const float* Go,
                                 const float* c, const float* g0, float* x, float* p,
                                 float* o, float* q, float* rd, float* ro, float* rr,
                                 int* grp, unsigned char* st_, int max_iter) {
  const int Mc = N - 1;
  const float inv_h = 1.0f / hp;
  for (int i = 0; i < N; ++i) x[i] = 0.0f;
  for (int cc = 0; cc < Mc; ++cc)
    st_[cc] = (g0[cc] <= -1.0f + EPI_TOL_ACTIVE) ? 1 : (g0[cc] >= 1.0f - EPI_TOL_ACTIVE ? 2 : 0);
  int it = 0;
  for (; it < max_iter; ++it) {
    // groups and fixed offsets inside each group
    grp[0] = 0;
    o[0] = 0.0f;
    for (int i = 1; i < N; ++i) {
      const int cc = i - 1;
      if (st_[cc]) {
        grp[i] = grp[i - 1];
        const float target = (st_[cc] == 1) ? -1.0f : 1.0f;
        const float gx = g0[cc] + (x[i] - x[i - 1]) * inv_h;
        o[i] = o[i - 1] + hp * (target - gx);
      } else {
        grp[i] = grp[i - 1] + 1;
        o[i] = 0.0f;
      }
    }
    const int ng = grp[N - 1] + 1;
    for (int t = 0; t < ng; ++t) {
      rd[t] = 0.0f;
      ro[t] = 0.0f;
      rr[t] = 0.0f;
    }
    for (int i = 0; i < N; ++i) {
      float gx = Gd[i] * x[i], go = Gd[i] * o[i];
      if (i > 0) { gx += Go[i - 1] * x[i - 1]; go += Go[i - 1] * o[i - 1]; }
      if (i < N - 1) { gx += Go[i] * x[i + 1]; go += Go[i] * o[i + 1]; }
      q[i] = gx + c[i];
      const int t = grp[i];
      rr[t] -= q[i] + go;
      rd[t] += Gd[i];
      if (i < N - 1) {
        if (grp[i + 1] == t) rd[t] += 2.0f * Go[i];
        else ro[t] = Go[i];
      }
    }
    // Thomas on the group system
    for (int t = 1; t < ng; ++t) {
      const float m = ro[t - 1] / rd[t - 1];
      rd[t] -= m * ro[t - 1];
      rr[t] -= m * rr[t - 1];
    }
    rr[ng - 1] /= rd[ng - 1];
    for (int t = ng - 2; t >= 0; --t) rr[t] = (rr[t] - ro[t] * rr[t + 1]) / rd[t];
    float pmax = 0.0f;
    for (int i = 0; i < N; ++i) {
      p[i] = rr[grp[i]] + o[i];
      pmax = fmaxf(pmax, fabsf(p[i]));
    }
    // multipliers of the active cells
    float lam_min = 0.0f;
    int lam_arg = -1;
    float run = 0.0f;
    for (int i = 0; i < N; ++i) {
      if (i == 0 || st_[i - 1] == 0) run = 0.0f;
      float wv = Gd[i] * p[i] + q[i];
      if (i > 0) wv += Go[i - 1] * p[i - 1];
      if (i < N - 1) wv += Go[i] * p[i + 1];
      run += wv;
      if (i < Mc && st_[i]) {
        const float lam = hp * (st_[i] == 1 ? 1.0f : -1.0f) * (-run);
        if (lam < lam_min) {
          lam_min = lam;
          lam_arg = i;
        }
      }
    }
    if (pmax > 1e-6f * hp) {
      float rmin = 3.0e38f;
      for (int cc = 0; cc < Mc; ++cc) {
        if (st_[cc]) continue;
        const float dp = (p[cc + 1] - p[cc]) * inv_h;
        const float gx = g0[cc] + (x[cc + 1] - x[cc]) * inv_h;
        float ratio = 3.0e38f;
        if (dp < 0.0f) ratio = (-1.0f - gx) / dp;
        else if (dp > 0.0f) ratio = (1.0f - gx) / dp;
        rmin = fminf(rmin, ratio);
      }
      const float sigma = (rmin < 1.0f) ? fmaxf(rmin, 0.0f) : 1.0f;
      for (int i = 0; i < N; ++i) x[i] = fmaf(sigma, p[i], x[i]);
      if (rmin < 1.0f) {
        const float lim = rmin + 1e-6f * fmaxf(1.0f, fabsf(rmin));
        for (int cc = 0; cc < Mc; ++cc) {
          if (st_[cc]) continue;
          const float dp = (p[cc + 1] - p[cc]) * inv_h;
          const float gx0 = g0[cc] + (x[cc + 1] - x[cc]) * inv_h - sigma * dp;
          float ratio = 3.0e38f;
          if (dp < 0.0f) ratio = (-1.0f - gx0) / dp;
          else if (dp > 0.0f) ratio = (1.0f - gx0) / dp;
          if (ratio <= lim) st_[cc] = (dp < 0.0f) ? 1 : 2;
        }
        continue;
      }
    }
    if (lam_arg < 0) break;       // every multiplier >= 0: optimal
    st_[lam_arg] = 0;             // drop the most negative multiplier
  }
  int nact = 0;
  for (int cc = 0; cc < Mc; ++cc) nact += st_[cc] != 0;
  return nact | (it << 16);
}

// Hard lines of the b-step: one wavefront per line, QP data computed wave-parallel, the
// active-set loop by lane 0. Writes b^{k+1} and w for those lines and their |b|^2.
template <int P>
__global__ __launch_bounds__(64) void k_admm_bstep_hard(LineArgs a, float* __restrict__ bvec,
                                                        const float* __restrict__ zvec,
                                                        const float* __restrict__ uvec,
                                                        float* __restrict__ wvec,
                                                        const int* hard_list, DevState* st) {
  if (st->admm_done) return;
  const int nhard = st->hard_count;
  if ((int)blockIdx.x >= nhard) {
    return;
  }
  __shared__ float sIp[LineBuf<P>::SIZE], sIm[LineBuf<P>::SIZE], stg[LineBuf<P>::SIZE];
  __shared__ float Gd[64 * P], Go[64 * P], cv[64 * P], g0[64 * P], x[64 * P], p[64 * P],
      o[64 * P], q[64 * P], rd[64 * P], ro[64 * P], rr[64 * P];
  __shared__ int grp[64 * P];
  __shared__ unsigned char stt[64 * P];
  __shared__ int res_sh;
  const int lane = threadIdx.x;
  const int NF = a.M + 1;
  for (int h = blockIdx.x; h < nhard; h += gridDim.x) {
    const int line = hard_list[h];
    const size_t base = (size_t)line * NF;
    for (int t = lane; t < 64 * P; t += 64) {
      sIp[lds_pad(t)] = (t < a.M) ? a.Ip[(size_t)line * a.M + t] : 0.0f;
      sIm[lds_pad(t)] = (t < a.M) ? a.Im[(size_t)line * a.M + t] : 0.0f;
    }
    float b[P], z[P], u[P];
    stage_in<P>(bvec + base, NF, true, stg, b, lane);
    stage_in<P>(zvec + base, NF, true, stg, z, lane);
    stage_in<P>(uvec + base, NF, true, stg, u, lane);
    float Gdr[P], Gor[P], cr[P], gr[P];
    qp_data<P>(a, (float)st->rho, b, z, u, sIp, sIm, lane, Gdr, Gor, cr, gr);
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const int i = P * lane + j;
      Gd[i] = Gdr[j];
      Go[i] = Gor[j];
      cv[i] = cr[j];
      g0[i] = gr[j];
    }
    __syncthreads();
    if (lane == 0)
      res_sh = active_set_serial(NF, a.hp, Gd, Go, cv, g0, x, p, o, q, rd, ro, rr, grp, stt,
                                 4 * NF);
    __syncthreads();
    float bn[P], wn[P];
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const int i = P * lane + j;
      bn[j] = (i < NF) ? b[j] + x[i] : 0.0f;
      wn[j] = bn[j] + u[j];
    }
    stage_out<P>(bvec + base, NF, true, stg, bn, lane);
    stage_out<P>(wvec + base, NF, true, stg, wn, lane);
    if (lane == 0) atomicMax(&st->max_active, res_sh & 0xffff);
    __syncthreads();
  }
}

// ------------------------------------------------------------------------------------
// Host-side launchers
// ------------------------------------------------------------------------------------
#define EPI_DISPATCH_P(P_, CALL)                       \
  switch (P_) {                                        \
    case 1: { constexpr int PP = 1; CALL; } break;     \
    case 2: { constexpr int PP = 2; CALL; } break;     \
    case 3: { constexpr int PP = 3; CALL; } break;     \
    case 4: { constexpr int PP = 4; CALL; } break;     \
    case 5: { constexpr int PP = 5; CALL; } break;     \
    case 6: { constexpr int PP = 6; CALL; } break;     \
    case 7: { constexpr int PP = 7; CALL; } break;     \
    case 8: { constexpr int PP = 8; CALL; } break;     \
    default: break;                                    \
  }

int line_blocks(const LineArgs& a) { return (a.L + EPI_LINE_WAVES - 1) / EPI_LINE_WAVES; }

void launch_eval(hipStream_t s, int P, int mode, LineArgs a, const float* b, const float* d,
                 int trial, int with_pen, float* grad, float* hdiag, float* hoff,
                 double* partial, const DevState* st) {
  const int nb = line_blocks(a);
  a.nblk = nb;
  if (mode == 0) {
    EPI_DISPATCH_P(P, hipLaunchKernelGGL((k_eval<PP, 0>), dim3(nb), dim3(256), 0, s, a, b, d,
                                         trial, with_pen, grad, hdiag, hoff, partial, st));
  } else if (mode == 1) {
    EPI_DISPATCH_P(P, hipLaunchKernelGGL((k_eval<PP, 1>), dim3(nb), dim3(256), 0, s, a, b, d,
                                         trial, with_pen, grad, hdiag, hoff, partial, st));
  } else {
    EPI_DISPATCH_P(P, hipLaunchKernelGGL((k_eval<PP, 2>), dim3(nb), dim3(256), 0, s, a, b, d,
                                         trial, with_pen, grad, hdiag, hoff, partial, st));
  }
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
                       const float* q, double* partial, const DevState* st) {
  const int nb = line_blocks(a);
  EPI_DISPATCH_P(P, hipLaunchKernelGGL((k_pcg_update<PP>), dim3(nb), dim3(256), 0, s, a,
                                       precond, hdiag, hoff, x, r, z, p, q, partial, st));
}

void launch_admm_bstep(hipStream_t s, int P, LineArgs a, float* b, const float* z,
                       const float* u, float* w, int* hard_list, DevState* st, int hard_blocks,
                       const std::function<void(int)>& before,
                       const std::function<void()>& after) {
  const int nb = line_blocks(a);
  before(0);
  EPI_DISPATCH_P(P, hipLaunchKernelGGL((k_admm_bstep<PP>), dim3(nb), dim3(256), 0, s, a, b, z,
                                       u, w, hard_list, st));
  after();
  before(1);
  EPI_DISPATCH_P(P, hipLaunchKernelGGL((k_admm_bstep_hard<PP>), dim3(hard_blocks), dim3(64), 0,
                                       s, a, b, z, u, w, hard_list, st));
  after();
}

}  // namespace epi
