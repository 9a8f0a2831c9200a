// Device-side building blocks shared by the kernels of the EPI solver library (gfx950).
//
// Wavefronts are 64 lanes. A PE line with M + 1 faces is owned by one wavefront: lane l
// holds the P consecutive faces [P l, P l + P) in registers (P = ceil((M + 1) / 64)), and
// cell c (between faces c and c + 1) lives with face c. Rows beyond the line are padding.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "epi_common.hpp"

namespace epi {

// ------------------------------------------------------------------------------------
// Shuffles and reductions within one wavefront
// ------------------------------------------------------------------------------------
// Neighbour exchange by one lane across the whole wavefront as a DPP move (wave_shr:1 /
// wave_shl:1 of the GFX9 family: a VALU operation, no LDS round trip); the lane without a
// neighbour receives 0. All 64 lanes must be active.
__device__ __forceinline__ float dpp_prev_lane(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                               0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float dpp_next_lane(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                               0x130, 0xf, 0xf, true));
}
// value of v in lane l (wave-uniform)
__device__ __forceinline__ float read_lane(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

__device__ __forceinline__ float shfl_up0(float v, int d, int lane) {
  float t = __shfl_up(v, d, EPI_WAVE);
  return lane >= d ? t : 0.0f;
}
__device__ __forceinline__ float shfl_down0(float v, int d, int lane) {
  float t = __shfl_down(v, d, EPI_WAVE);
  return lane + d < EPI_WAVE ? t : 0.0f;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, EPI_WAVE);
  return v;
}
__device__ __forceinline__ float wave_maxf(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, EPI_WAVE));
  return v;
}
__device__ __forceinline__ int wave_sumi(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, EPI_WAVE);
  return v;
}

// Sum NQ float64 values over the workgroup and store them at partial[blockIdx.x*NQ + q].
// Every thread of the block must call it (it contains a barrier).
template <int NQ>
__device__ __forceinline__ void block_partials(double (&v)[NQ], double* partial, int slot) {
  __shared__ double sh[NQ][16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double s = wave_sum(v[q]);
    if (lane == 0) sh[q][wave] = s;
  }
  __syncthreads();
  if (threadIdx.x < NQ) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += sh[threadIdx.x][w];
    partial[(size_t)slot * NQ + threadIdx.x] = s;
  }
}

// Deterministic sum of partial[b*NQ + q] over b in [0, nb) by one workgroup of NT threads
// (a multiple of 64, at most 1024); returns the sums to every thread via out_sh (fixed
// summation order). Each thread's loads (blocks t, t + NT, ...) are issued before the
// first add; then one shuffle reduction per wavefront and one barrier.
template <int NQ, int NT = 256>
__device__ __forceinline__ void reduce_partials(const double* partial, int nb, double* out_sh) {
  constexpr int NWV = NT / 64;
  __shared__ double red[NQ][NWV];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  double s[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) s[q] = 0.0;
  int b = t;
  for (; b + 3 * NT < nb; b += 4 * NT) {
    double v[4][NQ];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int q = 0; q < NQ; ++q) v[k][q] = partial[(size_t)(b + NT * k) * NQ + q];
#pragma unroll
    for (int q = 0; q < NQ; ++q) s[q] += (v[0][q] + v[1][q]) + (v[2][q] + v[3][q]);
  }
  {
    double v[3][NQ];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        v[k][q] = (b + NT * k < nb) ? partial[(size_t)(b + NT * k) * NQ + q] : 0.0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) s[q] += (v[0][q] + v[1][q]) + v[2][q];
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const double w = wave_sum(s[q]);
    if (lane == 0) red[q][wave] = w;
  }
  __syncthreads();
  if (t < NQ) {
    double a = 0.0;
#pragma unroll
    for (int w = 0; w < NWV; ++w) a += red[t][w];
    out_sh[t] = a;
  }
  __syncthreads();
}

// The float64 stopping test of ADMM (eq. admmStop) at the newest iterates, from the sums
// |b-z|^2, |z_old-z|^2, |z|^2, |u|^2 and |b|^2 of the last z-step pass.
__device__ __forceinline__ void admm_finalize(DevState* st, const double* sums, double* hist,
                                              int hist_len) {
  const double b2 = sums[4];
  const double rho = st->rho;
  const double rpri = sqrt(sums[0]);
  const double rdual = rho * st->v * sqrt(sums[1]);
  const double nb = sqrt(b2), nz = sqrt(sums[2]), nu = sqrt(sums[3]);
  const double epri = st->sqrt_n * st->eps_abs + st->eps_rel * (nb > nz ? nb : nz);
  const double edual = st->sqrt_n * st->eps_abs + st->eps_rel * rho * st->v * nu;
  const int it = st->admm_iter;
  if (it < hist_len) {
    hist[it] = rpri;
    hist[hist_len + it] = rdual;
    hist[2 * hist_len + it] = epri;
    hist[3 * hist_len + it] = edual;
    hist[4 * hist_len + it] = rho;
  }
  st->admm_iter = it + 1;
  st->hard_total += st->hard_count;
  st->hard_count = 0;
  const bool finite = (rpri == rpri) && (rdual == rdual) && rpri < 1e300 && rdual < 1e300;
  if (!finite || st->numeric_bad) {
    st->numeric_bad += 1;
    st->admm_done = 1;
  } else if (rpri <= epri && rdual <= edual) {
    st->admm_done = 1;
  } else if (st->admm_iter >= st->admm_max) {
    st->admm_done = 2;   // iteration cap: later launches of this solve are no-ops
  }
  // Residual balancing for the next iteration: rho * tau when the primal residual exceeds
  // mu times the dual one, rho / tau in the opposite case (mode 2: not below rho_min);
  // the scaled dual u = y / (rho v) is rescaled by rho_old / rho_new.
  st->u_scale = 1.0;
  if (!st->admm_done && st->rho_mode != 0) {
    double rn = rho;
    if (rpri > st->mu * rdual) {
      rn = rho * st->tau;
    } else if (rdual > st->mu * rpri) {
      rn = rho / st->tau;
      if (st->rho_mode == 2 && rn < st->rho_min) rn = rho;
    }
    if (rn != rho) {
      st->u_scale = rho / rn;
      st->rho = rn;
    }
  }
}
// Workgroups are dealt round-robin over the 8 XCDs; remap so that each XCD (and its L2)
// walks one contiguous range of logical block indices.
__device__ __forceinline__ int xcd_remap(int bid, int nblk) {
  const int nx = 8;
  const int q = nblk / nx, r = nblk % nx;
  const int x = bid % nx, k = bid / nx;
  // XCD x owns logical blocks [x*q + min(x,r), ... ) of size q + (x < r)
  const int base = x * q + (x < r ? x : r);
  return base + k;
}

// Stores of streamed results (written once here, read by a later kernel): a relaxed
// system-scope store, which gfx950 performs write-through (global_store ... sc0 sc1), so
// the data does not sit dirty in the XCD's L2 when the next kernel, running on all XCDs,
// reads it. Measured at 240x200x110: b-step and the two unfused DCT passes ~1.3 us faster
// each. Not used where a kernel rewrites lines it has just read (the ADMM epilogue).
#ifndef EPI_WT_STORES
#define EPI_WT_STORES 1
#endif
__device__ __forceinline__ void store_stream(float* p, float v) {
#if EPI_WT_STORES
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
#else
  *p = v;
#endif
}

// ------------------------------------------------------------------------------------
// y = H_JGN p at the faces i = lane + 64 j of one PE line (lane-contiguous layout, eq.
// dJGN): the line's tridiagonal block (diagonal hdv, off-diagonal hov, both along the
// line) plus alpha v (D2'D2 + D3'D3) p, the Neumann Laplacian across lines, with the j -+ 1
// neighbour lines from LDS (spm / spp, face order) or, where those are null, from pjo
// (the outer j neighbour of a workgroup's end wavefront) and the k -+ 1 lines pk0 / pk1.
// j0 / j1 / k0 / k1: the neighbour exists. The matvec and the PCG update both form q with
// this one function, so the q the update subtracts is the q whose p.q the matvec summed.
// ------------------------------------------------------------------------------------
template <int P>
__device__ __forceinline__ void hjgn_apply(const LineArgs& a, int NF, int lane, bool j0, bool j1,
                                           bool k0, bool k1, const float (&pc)[P],
                                           const float (&hdv)[P], const float (&hov)[P],
                                           const float (&pk0)[P], const float (&pk1)[P],
                                           const float (&pjo)[P], const float* spm,
                                           const float* spp, float (&y)[P]) {
  const float av = a.alpha * a.v;
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int i = lane + 64 * j;
    // faces i - 1 and i + 1 (lane shifts; across a 64-face block from the end lane)
    float pp = dpp_prev_lane(pc[j]), ho_p = dpp_prev_lane(hov[j]), pn = dpp_next_lane(pc[j]);
    if (j > 0) {
      const float e0 = read_lane(pc[j - 1], 63), e1 = read_lane(hov[j - 1], 63);
      if (lane == 0) {
        pp = e0;
        ho_p = e1;
      }
    }
    if (j < P - 1) {
      const float e2 = read_lane(pc[j + 1], 0);
      if (lane == 63) pn = e2;
    }
    float yy = hdv[j] * pc[j];
    if (i > 0) yy = fmaf(ho_p, pp, yy);
    if (i < NF - 1) yy = fmaf(hov[j], pn, yy);
    float l2 = 0.0f, l3 = 0.0f;
    if (j0) l2 += pc[j] - (spm ? spm[i] : pjo[j]);
    if (j1) l2 += pc[j] - (spp ? spp[i] : pjo[j]);
    if (k0) l3 += pc[j] - pk0[j];
    if (k1) l3 += pc[j] - pk1[j];
    y[j] = fmaf(av, l2 * a.inv_h2sq + l3 * a.inv_h3sq, yy);
  }
}

// ------------------------------------------------------------------------------------
// LDS staging of one PE line per wavefront (coalesced global access, blocked registers)
// ------------------------------------------------------------------------------------
__device__ __forceinline__ int lds_pad(int t) { return t + (t >> 5); }

template <int P>
struct LineBuf {
  static constexpr int SIZE = 64 * P + 2 * P + 2;
};

// Global -> registers: dst[j] = src[P*lane + j] for P*lane + j < count, else 0.
template <int P>
__device__ __forceinline__ void stage_in(const float* __restrict__ src, int count, bool valid,
                                         float* lds, float (&dst)[P], int lane) {
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int t = lane + 64 * j;
    lds[lds_pad(t)] = (valid && t < count) ? src[t] : 0.0f;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < P; ++j) dst[j] = lds[lds_pad(P * lane + j)];
  __syncthreads();
}

// Global -> registers in the lane-contiguous layout, NA arrays: t[a][j] = src[a][lane + 64 j]
// for indices < count[a], else 0. P = ceil((M + 1) / 64) and count >= M, so only the last
// of the P loads can fall past the end of a line; it reads the line's last element instead
// (in bounds) and the value is replaced by 0, so every load is unconditional and all of
// them are issued back to back. src must point at a valid line also when valid is false.
template <int P, int NA>
__device__ __forceinline__ void load_line_n(const float* const (&src)[NA], const int (&count)[NA],
                                            bool valid, float (&t)[NA][P], int lane) {
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const int i = lane + 64 * j;
      const bool in = j < P - 1 || i < count[a];
      const float x = src[a][in ? i : count[a] - 1];
      t[a][j] = (valid && in) ? x : 0.0f;
    }
}

// Lane-contiguous registers -> LDS (NA consecutive LineBuf<P> buffers, which keep the
// line) -> lane-blocked registers dst[a][j] = line a at P * lane + j.
template <int P, int NA>
__device__ __forceinline__ void regs_to_blocked_n(const float (&t)[NA][P], float* lds,
                                                  float (&dst)[NA][P], int lane) {
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int j = 0; j < P; ++j) lds[a * LineBuf<P>::SIZE + lds_pad(lane + 64 * j)] = t[a][j];
  __syncthreads();
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int j = 0; j < P; ++j) dst[a][j] = lds[a * LineBuf<P>::SIZE + lds_pad(P * lane + j)];
  __syncthreads();
}

// NA arrays at once: every global load is issued before the first LDS write, so one
// memory round trip covers all of them. lds holds NA consecutive LineBuf<P> buffers.
template <int P, int NA>
__device__ __forceinline__ void stage_in_n(const float* const (&src)[NA], const int (&count)[NA],
                                           bool valid, float* lds, float (&dst)[NA][P],
                                           int lane) {
  float t[NA][P];
  load_line_n<P, NA>(src, count, valid, t, lane);
  regs_to_blocked_n<P, NA>(t, lds, dst, lane);
}

// NA arrays out at once (one barrier pair for all of them).
template <int P, int NA>
__device__ __forceinline__ void stage_out_n(float* const (&dst)[NA], int count, bool valid,
                                            float* lds, const float (&v)[NA][P], int lane) {
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int j = 0; j < P; ++j) lds[a * LineBuf<P>::SIZE + lds_pad(P * lane + j)] = v[a][j];
  __syncthreads();
  if (valid) {
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
      for (int j = 0; j < P; ++j) {
        const int t = lane + 64 * j;
        if (j < P - 1 || t < count) store_stream(&dst[a][t], lds[a * LineBuf<P>::SIZE + lds_pad(t)]);
      }
  }
  __syncthreads();
}

// Registers -> global: dst[P*lane + j] = v[j] for indices < count.
template <int P>
__device__ __forceinline__ void stage_out(float* __restrict__ dst, int count, bool valid,
                                          float* lds, const float (&v)[P], int lane) {
#pragma unroll
  for (int j = 0; j < P; ++j) lds[lds_pad(P * lane + j)] = v[j];
  __syncthreads();
  if (valid) {
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const int t = lane + 64 * j;
      if (t < count) store_stream(&dst[t], lds[lds_pad(t)]);
    }
  }
  __syncthreads();
}

// ------------------------------------------------------------------------------------
// Symmetric tridiagonal solve over one wavefront.
//   row i: e[i-1] x[i-1] + d[i] x[i] + e[i] x[i+1] = r[i]
// Lane l holds rows [P l, P l + P) in d[], e[], r[] (e[j] couples local rows j and j+1,
// the last one couples to the next lane). Padding rows must be d = 1, e = 0, r = 0 and
// the last real row must have e = 0. On return r[] holds x.
// Method: each lane eliminates its block downwards (Thomas), then upwards, expressing
// every row through the last unknown of the previous lane and its own last unknown; the
// resulting 64-row tridiagonal system of block-last unknowns is solved by parallel
// cyclic reduction across lanes; the interior rows follow by substitution.
// ------------------------------------------------------------------------------------
// Reciprocal by the hardware approximation (v_rcp_f32, 1 ulp) instead of the IEEE divide
// sequence (about ten instructions): the line solves are bound by instruction issue.
__device__ __forceinline__ float rcp_f(float x) { return __builtin_amdgcn_rcpf(x); }

template <int P>
__device__ __forceinline__ void wave_tridiag_solve(const float (&d)[P], const float (&e)[P],
                                                   float (&r)[P], int lane) {
  float ap[P], cp[P], rp[P];
  const float a0 = shfl_up0(e[P - 1], 1, lane);   // coupling of row P*lane to the row before
  {
    const float inv = rcp_f(d[0]);
    ap[0] = a0 * inv;
    cp[0] = e[0] * inv;
    rp[0] = r[0] * inv;
  }
#pragma unroll
  for (int j = 1; j < P; ++j) {
    const float a = e[j - 1];
    const float inv = rcp_f(d[j] - a * cp[j - 1]);
    ap[j] = -a * ap[j - 1] * inv;
    cp[j] = e[j] * inv;
    rp[j] = (r[j] - a * rp[j - 1]) * inv;
  }
  // x_j = R_j - A_j X_prev - C_j X_own
  float R[P], A[P], C[P];
  R[P - 1] = 0.0f;
  A[P - 1] = 0.0f;
  C[P - 1] = -1.0f;
#pragma unroll
  for (int j = P - 2; j >= 0; --j) {
    R[j] = rp[j] - cp[j] * R[j + 1];
    A[j] = ap[j] - cp[j] * A[j + 1];
    C[j] = -cp[j] * C[j + 1];
  }
  // reduced row of this lane: ap X_{l-1} + X_l + cp x_{first of l+1} = rp (last local row)
  const float Rn = shfl_down0(R[0], 1, lane);
  const float An = shfl_down0(A[0], 1, lane);
  const float Cn = shfl_down0(C[0], 1, lane);
  float ra = (lane == 0) ? 0.0f : ap[P - 1];
  float rb = 1.0f - cp[P - 1] * An;
  float rc = (lane == 63) ? 0.0f : -cp[P - 1] * Cn;
  float rr = rp[P - 1] - cp[P - 1] * Rn;
  // Parallel cyclic reduction. Before the step of distance s, every lane below s has
  // ra = 0 and every lane at or above 64 - s has rc = 0 (true for s = 1 and kept by each
  // step), so a lane without a partner at distance s gets a zero multiplier from its own
  // finite shuffled values: no boundary branches are needed.
#pragma unroll
  for (int s = 1; s < 64; s <<= 1) {
    const float ib = rcp_f(rb);
    const float am = __shfl_up(ra, s, 64), ibm = __shfl_up(ib, s, 64),
                cm = __shfl_up(rc, s, 64), xm = __shfl_up(rr, s, 64);
    const float aq = __shfl_down(ra, s, 64), ibq = __shfl_down(ib, s, 64),
                cq = __shfl_down(rc, s, 64), xq = __shfl_down(rr, s, 64);
    const float al = -ra * ibm, ga = -rc * ibq;
    const float na = al * am, nc = ga * cq;
    const float nb = rb + al * cm + ga * aq;
    const float nr = rr + al * xm + ga * xq;
    ra = na; rb = nb; rc = nc; rr = nr;
  }
  const float X = rr * rcp_f(rb);
  const float Xp = shfl_up0(X, 1, lane);
#pragma unroll
  for (int j = 0; j < P; ++j) r[j] = R[j] - A[j] * Xp - C[j] * X;
}

// The same solve split into a factorisation of the matrix and any number of solves with
// it (the b-step solves twice with one matrix: the step and its refinement). The
// factorisation keeps, per lane, the pivots' reciprocals and the Thomas multipliers of its
// block, the block's coupling coefficients A, C to the neighbouring lanes' last unknowns,
// and the multipliers of the six cyclic-reduction steps; a solve then only sweeps the
// right-hand side through them (twelve shuffles instead of forty-eight).
template <int P>
struct WaveTriFactor {
  float inv[P], cp[P], A[P], e[P];   // C (below) is rebuilt from cp by each solve
  float al[6], ga[6];
  float ibf;
};

template <int P>
__device__ __forceinline__ void wave_tridiag_factor(const float (&d)[P], const float (&e)[P],
                                                    WaveTriFactor<P>& F, int lane) {
  float ap[P];
  const float a0 = shfl_up0(e[P - 1], 1, lane);
  F.inv[0] = rcp_f(d[0]);
  ap[0] = a0 * F.inv[0];
  F.cp[0] = e[0] * F.inv[0];
#pragma unroll
  for (int j = 1; j < P; ++j) {
    const float a = e[j - 1];
    F.inv[j] = rcp_f(d[j] - a * F.cp[j - 1]);
    ap[j] = -a * ap[j - 1] * F.inv[j];
    F.cp[j] = e[j] * F.inv[j];
  }
#pragma unroll
  for (int j = 0; j < P; ++j) F.e[j] = e[j];
  float C[P];
  F.A[P - 1] = 0.0f;
  C[P - 1] = -1.0f;
#pragma unroll
  for (int j = P - 2; j >= 0; --j) {
    F.A[j] = ap[j] - F.cp[j] * F.A[j + 1];
    C[j] = -F.cp[j] * C[j + 1];
  }
  const float An = shfl_down0(F.A[0], 1, lane);
  const float Cn = shfl_down0(C[0], 1, lane);
  const float cpl = F.cp[P - 1];
  float ra = (lane == 0) ? 0.0f : ap[P - 1];
  float rb = 1.0f - cpl * An;
  float rc = (lane == 63) ? 0.0f : -cpl * Cn;
  int q = 0;
#pragma unroll
  for (int s = 1; s < 64; s <<= 1, ++q) {
    const float ib = rcp_f(rb);
    const float am = __shfl_up(ra, s, 64), ibm = __shfl_up(ib, s, 64), cm = __shfl_up(rc, s, 64);
    const float aq = __shfl_down(ra, s, 64), ibq = __shfl_down(ib, s, 64), cq = __shfl_down(rc, s, 64);
    const float al = -ra * ibm, ga = -rc * ibq;
    F.al[q] = al;
    F.ga[q] = ga;
    const float na = al * am, nc = ga * cq;
    rb = rb + al * cm + ga * aq;
    ra = na;
    rc = nc;
  }
  F.ibf = rcp_f(rb);
}

// r <- M^{-1} r with the factorisation F (same arithmetic as wave_tridiag_solve).
template <int P>
__device__ __forceinline__ void wave_tridiag_apply(const WaveTriFactor<P>& F, float (&r)[P],
                                                   int lane) {
  float rp[P];
  rp[0] = r[0] * F.inv[0];
#pragma unroll
  for (int j = 1; j < P; ++j) rp[j] = (r[j] - F.e[j - 1] * rp[j - 1]) * F.inv[j];
  float R[P];
  R[P - 1] = 0.0f;
#pragma unroll
  for (int j = P - 2; j >= 0; --j) R[j] = rp[j] - F.cp[j] * R[j + 1];
  const float Rn = shfl_down0(R[0], 1, lane);
  float rr = rp[P - 1] - F.cp[P - 1] * Rn;
  int q = 0;
#pragma unroll
  for (int s = 1; s < 64; s <<= 1, ++q) {
    const float xm = __shfl_up(rr, s, 64), xq = __shfl_down(rr, s, 64);
    rr = rr + F.al[q] * xm + F.ga[q] * xq;
  }
  const float X = rr * F.ibf;
  const float Xp = shfl_up0(X, 1, lane);
  float C = -1.0f;
#pragma unroll
  for (int j = P - 1; j >= 0; --j) {
    if (j < P - 1) C = -F.cp[j] * C;
    r[j] = R[j] - F.A[j] * Xp - C * X;
  }
}

// ------------------------------------------------------------------------------------
// Penalty phi (eq. P) and its derivatives (eq. dphi), |x| < 1
// ------------------------------------------------------------------------------------
__device__ __forceinline__ float phi_f(float x) {
  const float q = (1.0f - x) * (1.0f + x);
  const float x2 = x * x;
  return x2 * x2 / q;
}
__device__ __forceinline__ float dphi_f(float x) {
  const float q = (1.0f - x) * (1.0f + x);
  const float x2 = x * x;
  return (4.0f - 2.0f * x2) * x2 * x / (q * q);
}
__device__ __forceinline__ float d2phi_f(float x) {
  const float q = (1.0f - x) * (1.0f + x);
  const float x2 = x * x;
  return 2.0f * x2 * (x2 * x2 - 3.0f * x2 + 6.0f) / (q * q * q);
}
// phi, phi' and phi'' together with one hardware reciprocal of q = 1 - x^2 (1 ulp) instead
// of three divisions.
__device__ __forceinline__ void phi_terms(float x, float& ph, float& d1, float& d2) {
  const float q = (1.0f - x) * (1.0f + x);
  const float iq = rcp_f(q);
  const float x2 = x * x;
  const float iq2 = iq * iq;
  ph = x2 * x2 * iq;
  d1 = (4.0f - 2.0f * x2) * x2 * x * iq2;
  d2 = 2.0f * x2 * (x2 * x2 - 3.0f * x2 + 6.0f) * iq2 * iq;
}

}  // namespace epi
