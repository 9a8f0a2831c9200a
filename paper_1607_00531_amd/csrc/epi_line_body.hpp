// Per-line device code shared by the single-volume and the batched kernels.
//
// Section 3: the distance term couples faces only along a PE line (averaging A1 and short
// differences D1 act inside a line), so its residual, gradient and Gauss-Newton Hessian
// (tridiagonal per line) and the ADMM b-step QP (Section 4.2) are computed line by line.
#pragma once

#include "epi_device.hpp"
#include "epi_common.hpp"

namespace epi {

// 1D linear interpolation of the cell-centred samples of one line held in LDS at index
// coordinate c + disp (sample c sits at index c); zero outside the M samples; derivative
// with respect to the physical PE coordinate from the segment [k, k+1], k = floor(c + disp)
// (the right-hand segment at a knot). The floor is taken of the displacement alone and
// the integer cell index added afterwards: rounding c + disp in float32 would move small
// displacements (|disp| < ulp(c) / 2) onto the knot and pick the wrong segment.
// Branch-free: both samples are read at clamped (always valid) indices and the values
// outside the image are selected to zero afterwards.
__device__ __forceinline__ void interp_lds(const float* sT, int M, int c, float disp,
                                           float inv_hp, float& val, float& der) {
  disp = fminf(fmaxf(disp, -(float)(2 * M + 4)), (float)(2 * M + 4));
  const float fl = floorf(disp);
  const int k = c + (int)fl;
  const float f = disp - fl;
  const int k0 = min(max(k, 0), M - 1), k1 = min(max(k + 1, 0), M - 1);
  float t0 = sT[lds_pad(k0)], t1 = sT[lds_pad(k1)];
  t0 = (k >= 0 && k <= M - 1) ? t0 : 0.0f;
  t1 = (k >= -1 && k <= M - 2) ? t1 : 0.0f;
  val = fmaf(f, t1 - t0, t0);
  der = (t1 - t0) * inv_hp;
}

// The same interpolation from a line whose LDS buffer carries zero samples at the indices
// -2, -1 and M + 1 (and, as staged, at M .. 64 P - 1): the segment index is clamped into
// [-2, M], where both end samples are the zero padding, so no selects are needed.
// sT may be read at lds_pad(-2) = -3 .. lds_pad(M + 1): the caller reserves the 3 floats
// before the buffer (LinePad).
__device__ __forceinline__ void interp_lds_z(const float* sT, int M, int c, float disp,
                                             float inv_hp, float& val, float& der) {
  disp = fminf(fmaxf(disp, -(float)(2 * M + 4)), (float)(2 * M + 4));
  const float fl = floorf(disp);
  const int k = min(max(c + (int)fl, -2), M);
  const float f = disp - fl;
  const float t0 = sT[lds_pad(k)], t1 = sT[lds_pad(k + 1)];
  val = fmaf(f, t1 - t0, t0);
  der = (t1 - t0) * inv_hp;
}

// The cubic B-spline image model (the smoothed spline of the Section 5 comparison): value
// and physical derivative of I(s) = sum_k w_k beta3(s - k) at s = c + disp from the
// coefficients w of one line held in LDS, which must carry zero coefficients at the
// indices -3, -2, -1 and M, M + 1, M + 2 (pad_spline_line). The segment k = floor(disp) + c
// is clamped into [-2, M], so the four taps k - 1 .. k + 2 stay inside the padded buffer;
// outside the support (k < -2 or k > M) the result is zero. The floor is taken of the
// displacement alone, as in interp_lds.
__device__ __forceinline__ void interp_spline_lds(const float* sW, int M, int c, float disp,
                                                  float inv_hp, float& val, float& der) {
  disp = fminf(fmaxf(disp, -(float)(2 * M + 8)), (float)(2 * M + 8));
  const float fl = floorf(disp);
  const int k = c + (int)fl;
  const int kc = min(max(k, -2), M);
  const float f = disp - fl;
  const float g = 1.0f - f;
  const float f2 = f * f, f3 = f2 * f;
  const float w0 = g * g * g * (1.0f / 6.0f);
  const float w1 = 0.5f * f3 - f2 + (2.0f / 3.0f);
  const float w2 = -0.5f * f3 + 0.5f * f2 + 0.5f * f + (1.0f / 6.0f);
  const float w3 = f3 * (1.0f / 6.0f);
  const float d0 = -0.5f * g * g;
  const float d1 = 1.5f * f2 - 2.0f * f;
  const float d2 = -1.5f * f2 + f + 0.5f;
  const float d3 = 0.5f * f2;
  const float c0 = sW[lds_pad(kc - 1)], c1 = sW[lds_pad(kc)], c2 = sW[lds_pad(kc + 1)],
              c3 = sW[lds_pad(kc + 2)];
  const bool in = k == kc;
  const float v = fmaf(w0, c0, fmaf(w1, c1, fmaf(w2, c2, w3 * c3)));
  const float d = fmaf(d0, c0, fmaf(d1, c1, fmaf(d2, c2, d3 * c3)));
  val = in ? v : 0.0f;
  der = in ? d * inv_hp : 0.0f;
}

// Floats reserved in front of a zero-padded line buffer (lds_pad(-3) = -4).
constexpr int LinePad = 4;

// Zero coefficients around one staged spline line: indices -3, -2, -1 (the LinePad floats
// in front of the buffer; for a second buffer they fall on the first one's zero tail) and
// M, M + 1, M + 2 (inside the buffer). One lane writes them; the wavefront's LDS accesses
// are performed in order.
__device__ __forceinline__ void pad_spline_line(float* sW, int M, int lane) {
  if (lane == 0) {
    sW[lds_pad(-3)] = 0.0f;
    sW[lds_pad(-2)] = 0.0f;
    sW[lds_pad(-1)] = 0.0f;
    sW[lds_pad(M)] = 0.0f;
    sW[lds_pad(M + 1)] = 0.0f;
    sW[lds_pad(M + 2)] = 0.0f;
  }
}

// Writes the zero padding of interp_lds_z for one staged line (one lane of the wavefront
// that reads it; LDS accesses of a wavefront are performed in order, so its other lanes see
// the zeros without a barrier).
__device__ __forceinline__ void zero_pad_line(float* sT, int M, int lane) {
  if (lane == 0) {
    sT[lds_pad(-2)] = 0.0f;
    sT[lds_pad(-1)] = 0.0f;
    sT[lds_pad(M + 1)] = 0.0f;
  }
}

// Per-cell quantities of the residual for the cells c = P*lane + j (zero for c >= M):
// g = D1 b, r = I+(x + A b)(1 + g) - I-(x - A b)(1 - g) and the two Jacobian entries
// dr_c/db_c = Jl, dr_c/db_{c+1} = Jr.
template <int P>
struct Cells {
  float g[P], r[P], Jl[P], Jr[P];
};

template <int P, bool PADDED = false, int MODEL = 0>
__device__ __forceinline__ void eval_cells(const LineArgs& a, const float (&b)[P],
                                           const float* sIp, const float* sIm, int lane,
                                           Cells<P>& C) {
  const float bnext = shfl_down0(b[0], 1, lane);
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int c = P * lane + j;
    const float bR = (j < P - 1) ? b[j + 1] : bnext;
    // computed for every slot (interp_lds is safe for any index), zeroed past the line
    const float aidx = 0.5f * (b[j] + bR) * a.inv_hp;
    const float g = (bR - b[j]) * a.inv_hp;
    float ipv, ipd, imv, imd;
    if (MODEL == 1) {
      interp_spline_lds(sIp, a.M, c, aidx, a.inv_hp, ipv, ipd);
      interp_spline_lds(sIm, a.M, c, -aidx, a.inv_hp, imv, imd);
    } else if (PADDED) {
      interp_lds_z(sIp, a.M, c, aidx, a.inv_hp, ipv, ipd);
      interp_lds_z(sIm, a.M, c, -aidx, a.inv_hp, imv, imd);
    } else {
      interp_lds(sIp, a.M, c, aidx, a.inv_hp, ipv, ipd);
      interp_lds(sIm, a.M, c, -aidx, a.inv_hp, imv, imd);
    }
    const float gp = 1.0f + g, gm = 1.0f - g;
    const float Sd = ipd * gp + imd * gm, Tv = ipv + imv;
    const bool in = c < a.M;
    C.g[j] = in ? g : 0.0f;
    C.r[j] = in ? ipv * gp - imv * gm : 0.0f;
    C.Jl[j] = in ? 0.5f * Sd - Tv * a.inv_hp : 0.0f;
    C.Jr[j] = in ? 0.5f * Sd + Tv * a.inv_hp : 0.0f;
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
// ADMM b-step (Section 4.2): per PE line, QP data at b^k
//   c = grad D(b^k) + alpha v D1'D1 b^k + rho v (b^k - z^k + u^k)
//   G = H_D(b^k) + alpha v D1'D1 + rho v I          (SPD tridiagonal)
// and the QP  min 1/2 x'Gx + c'x  s.t.  -1 <= D1 (b^k + x) <= 1.
// ------------------------------------------------------------------------------------
template <int P, bool PADDED = false, int MODEL = 0>
__device__ __forceinline__ void qp_data(const LineArgs& a, float rho, const float (&b)[P],
                                        const float (&z)[P], const float (&u)[P],
                                        const float* sIp, const float* sIm, int lane,
                                        float (&Gd)[P], float (&Go)[P], float (&c)[P],
                                        float (&g)[P], Cells<P>& C) {
  eval_cells<P, PADDED, MODEL>(a, b, sIp, sIm, lane, C);
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
    // slots past the last face get the identity row (c = 0, G = I)
    const bool in = i < NF;
    const float cj = a.v * (C.Jl[j] * C.r[j] + rpJ[j]) +
                     a.alpha * a.v * (gprev[j] - C.g[j]) * a.inv_hp + rv * (b[j] - z[j] + u[j]);
    const float ncell = (float)((i < a.M) + (i >= 1));
    const float gd = a.v * (C.Jl[j] * C.Jl[j] + JrPrev[j] * JrPrev[j]) + qa * ncell + rv;
    c[j] = in ? cj : 0.0f;
    Gd[j] = in ? gd : 1.0f;
    Go[j] = (i < a.M) ? a.v * C.Jl[j] * C.Jr[j] - qa : 0.0f;
  }
}

// G x of the b-step QP in the structured form v J'(J x) + alpha v D1'(D1 x) + rho v x,
// from the per-cell Jacobian entries (C.Jl, C.Jr, zero past the line) and short
// differences of x. For fields that are smooth along the line the diagonal/off-diagonal
// form of G cancels: its diagonal 2 alpha v / h^2 + rho v is rounded to float32 relative
// to alpha v / h^2 (about 1e4 times rho v at 240 faces per line), which perturbs the
// smallest eigenvalues of G, and with them the step, by about 1e-3 relative. Here the
// difference (x_{c+1} - x_c) is formed first, so a constant x gives exactly v J'J x + rho v x.
template <int P>
__device__ __forceinline__ void qp_apply(const LineArgs& a, float rho, const Cells<P>& C,
                                         const float (&x)[P], float (&y)[P], int lane) {
  const float xnext = shfl_down0(x[0], 1, lane);
  float t[P], jx[P];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const float xr = (j < P - 1) ? x[j + 1] : xnext;
    const bool in = P * lane + j < a.M;
    t[j] = in ? (xr - x[j]) * a.inv_hp : 0.0f;       // D1 x (cell)
    jx[j] = C.Jl[j] * x[j] + C.Jr[j] * xr;           // J x (cell; Jl = Jr = 0 past the line)
  }
  float tprev[P], jxprev[P], jrprev[P];
  prev_cell<P>(t, tprev, lane);
  prev_cell<P>(jx, jxprev, lane);
  prev_cell<P>(C.Jr, jrprev, lane);
  const float av = a.alpha * a.v, rv = rho * a.v;
#pragma unroll
  for (int j = 0; j < P; ++j)
    y[j] = a.v * (C.Jl[j] * jx[j] + jrprev[j] * jxprev[j]) + av * (tprev[j] - t[j]) * a.inv_hp +
           rv * x[j];
}

// x = G^{-1} rhs for the b-step QP of one line: the wave-parallel solve with G in
// diagonal/off-diagonal form, then one step of iterative refinement whose residual
// rhs - G x is formed with qp_apply. The first solve is accurate to about kappa(G) eps
// relative to x (1e-3 on the smooth modes of long lines); the refined x to its square.
// Padding slots (faces past the line) have rhs = 0 and the identity row. The Jacobian
// entries and the right-hand side wait in three LDS line buffers of the caller's
// (park[0..2], each thread its own slots) while the matrix is factorised, which keeps the
// factorisation, the largest live set of the b-step, within the register budget of seven
// wavefronts per SIMD.
template <int P>
__device__ __forceinline__ void qp_solve_refined(const LineArgs& a, float rho, const Cells<P>& C,
                                                 const float (&Gd)[P], const float (&Go)[P],
                                                 const float (&rhs)[P], float (&x)[P], int lane,
                                                 float* const (&park)[3]) {
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int t = lds_pad(P * lane + j);
    park[0][t] = C.Jl[j];
    park[1][t] = C.Jr[j];
    park[2][t] = rhs[j];
  }
  // the parked values are read back below, not forwarded in registers
  asm volatile("" ::: "memory");
  WaveTriFactor<P> F;
  wave_tridiag_factor<P>(Gd, Go, F, lane);
  Cells<P> J;
  float b0[P];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int t = lds_pad(P * lane + j);
    x[j] = park[2][t];
  }
  wave_tridiag_apply<P>(F, x, lane);
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int t = lds_pad(P * lane + j);
    J.Jl[j] = park[0][t];
    J.Jr[j] = park[1][t];
    b0[j] = park[2][t];
  }
  float gx[P], res[P];
  qp_apply<P>(a, rho, J, x, gx, lane);
  const int NF = a.M + 1;
#pragma unroll
  for (int j = 0; j < P; ++j) res[j] = (P * lane + j < NF) ? b0[j] - gx[j] : 0.0f;
  wave_tridiag_apply<P>(F, res, lane);
#pragma unroll
  for (int j = 0; j < P; ++j) x[j] += res[j];
}

// Tolerances of the float32 active-set logic (relative to the unit bound on |D1 b|).
#define EPI_TOL_ACTIVE 4e-6f

// Fast path of one line: lines whose starting working set is empty and whose
// unconstrained step -G^{-1} c keeps |D1 b| <= 1 are solved by that single tridiagonal
// solve (the active-set method terminates there); returns true (wave-uniform) for the
// other lines, which are left untouched for the active-set path. Writes b^{k+1} (in
// place) and w = b^{k+1} + u^k. sw: this wave's five LDS line buffers, preceded by LinePad
// floats that receive the zero padding of the first image line. Every wave of the
// workgroup must call it (barriers).
template <int P, int MODEL = 0>
__device__ __forceinline__ bool bstep_line_body(const LineArgs& a, float rho, float us,
                                                float* __restrict__ bvec,
                                                const float* __restrict__ zvec,
                                                const float* __restrict__ uvec,
                                                float* __restrict__ wvec, int lc, bool valid,
                                                float* sw, int lane, int* numeric_bad) {
  const int NF = a.M + 1;
  const size_t base = (size_t)lc * NF;
  const float* srcs[5] = {a.Ip + (size_t)lc * a.M, a.Im + (size_t)lc * a.M, bvec + base,
                          zvec + base, uvec + base};
  const int cnt[5] = {a.M, a.M, NF, NF, NF};
  float v[5][P];
  float* sIp = sw;
  float* sIm = sw + LineBuf<P>::SIZE;
  stage_in_n<P, 5>(srcs, cnt, valid, sw, v, lane);
  if (MODEL == 1) {
    pad_spline_line(sIp, a.M, lane);
    pad_spline_line(sIm, a.M, lane);
  } else {
    zero_pad_line(sIp, a.M, lane);
    zero_pad_line(sIm, a.M, lane);
  }
  float b[P], z[P], u[P];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    b[j] = v[2][j];
    z[j] = v[3][j];
    u[j] = v[4][j] * us;   // pending rescale of the scaled dual (1 with a fixed rho)
  }
  float Gd[P], Go[P], c[P], g[P];
  Cells<P> C;
  qp_data<P, true, MODEL>(a, rho, b, z, u, sIp, sIm, lane, Gd, Go, c, g, C);
  float x[P], mc[P];
  bool hard = false;
#pragma unroll
  for (int j = 0; j < P; ++j) {
    mc[j] = -c[j];
    if (P * lane + j < a.M && fabsf(g[j]) >= 1.0f - EPI_TOL_ACTIVE) hard = true;
  }
  // the image lines and z are no longer needed: their buffers hold the parked values
  float* const park[3] = {sIp, sIm, sw + 3 * LineBuf<P>::SIZE};
  qp_solve_refined<P>(a, rho, C, Gd, Go, mc, x, lane, park);
  // b and u are read again from their staged LDS lines (unchanged since staging) rather
  // than kept in registers across the two solves; g = D1 b is formed as in eval_cells.
  const float* sb = sw + 2 * LineBuf<P>::SIZE;
  const float* su = sw + 4 * LineBuf<P>::SIZE;
  const float xnext = shfl_down0(x[0], 1, lane);
  bool bad = false;
  float ov[2][P];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int cidx = P * lane + j;
    const float bj = sb[lds_pad(cidx)];
    if (cidx < a.M) {
      const float xr = (j < P - 1) ? x[j + 1] : xnext;
      const float gj = (sb[lds_pad(cidx + 1)] - bj) * a.inv_hp;
      const float gn = gj + (xr - x[j]) * a.inv_hp;
      if (!(fabsf(gn) <= 1.0f)) hard = true;   // also catches NaN
    }
    if (cidx < NF && !(fabsf(x[j]) < 3.0e38f)) bad = true;
    ov[0][j] = bj + x[j];
    ov[1][j] = ov[0][j] + su[lds_pad(cidx)] * us;
  }
  hard = __any(hard);
  if (bad && valid && lane == 0) atomicAdd(numeric_bad, 1);
  const bool wr = valid && !hard;
  float* outs[2] = {bvec + base, wvec + base};
  stage_out_n<P, 2>(outs, NF, wr, sw + 2 * LineBuf<P>::SIZE, ov, lane);
  return hard;
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
__device__ inline int active_set_serial(int N, float hp, const float* Gd, const float* Go,
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

// Hard line of the b-step: QP data computed wave-parallel into LDS, the active-set loop by
// lane 0 (active_set_serial), then b^{k+1} and w written back. One wavefront per workgroup.
template <int P>
struct HardLds {
  float simg[LinePad + 2 * LineBuf<P>::SIZE];   // the two image lines after LinePad floats
  float stg[LineBuf<P>::SIZE];
  float Gd[64 * P], Go[64 * P], cv[64 * P], g0[64 * P], x[64 * P], p[64 * P], o[64 * P],
      q[64 * P], rd[64 * P], ro[64 * P], rr[64 * P];
  int grp[64 * P];
  unsigned char stt[64 * P];
  int res;
};

template <int P, int MODEL = 0>
__device__ __forceinline__ void hard_line_body(const LineArgs& a, float rho, float us,
                                               float* __restrict__ bvec,
                                               const float* __restrict__ zvec,
                                               const float* __restrict__ uvec,
                                               float* __restrict__ wvec, int line,
                                               HardLds<P>& L, int lane, int* max_active,
                                               int qp_max) {
  const int NF = a.M + 1;
  const size_t base = (size_t)line * NF;
  float* sIp = L.simg + LinePad;
  float* sIm = sIp + LineBuf<P>::SIZE;
  for (int t = lane; t < 64 * P; t += 64) {
    sIp[lds_pad(t)] = (t < a.M) ? a.Ip[(size_t)line * a.M + t] : 0.0f;
    sIm[lds_pad(t)] = (t < a.M) ? a.Im[(size_t)line * a.M + t] : 0.0f;
  }
  if (MODEL == 1) {
    pad_spline_line(sIp, a.M, lane);
    pad_spline_line(sIm, a.M, lane);
  }
  float b[P], z[P], u[P];
  stage_in<P>(bvec + base, NF, true, L.stg, b, lane);
  stage_in<P>(zvec + base, NF, true, L.stg, z, lane);
  stage_in<P>(uvec + base, NF, true, L.stg, u, lane);
#pragma unroll
  for (int j = 0; j < P; ++j) u[j] *= us;
  float Gdr[P], Gor[P], cr[P], gr[P];
  Cells<P> C;
  qp_data<P, false, MODEL>(a, rho, b, z, u, sIp, sIm, lane, Gdr, Gor, cr, gr, C);
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int i = P * lane + j;
    L.Gd[i] = Gdr[j];
    L.Go[i] = Gor[j];
    L.cv[i] = cr[j];
    L.g0[i] = gr[j];
  }
  __syncthreads();
  if (lane == 0)
    L.res = active_set_serial(NF, a.hp, L.Gd, L.Go, L.cv, L.g0, L.x, L.p, L.o, L.q, L.rd, L.ro,
                              L.rr, L.grp, L.stt, qp_max > 0 ? qp_max : 4 * NF);
  __syncthreads();
  float bn[P], wn[P];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int i = P * lane + j;
    bn[j] = (i < NF) ? b[j] + L.x[i] : 0.0f;
    wn[j] = bn[j] + u[j];
  }
  stage_out<P>(bvec + base, NF, true, L.stg, bn, lane);
  stage_out<P>(wvec + base, NF, true, L.stg, wn, lane);
  if (lane == 0) atomicMax(max_active, L.res & 0xffff);
  __syncthreads();
}

}  // namespace epi
