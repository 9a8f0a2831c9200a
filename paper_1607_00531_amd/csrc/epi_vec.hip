// Flat (face-parallel) kernels and the single-block finalisation kernels.
#include <math.h>

#include "epi_device.hpp"
#include "epi_common.hpp"
#include "epi_launch.hpp"

namespace epi {

int flat_blocks(long long n) {
  long long b = (n + 2047) / 2048;
  if (b > 2048) b = 2048;
  if (b < 1) b = 1;
  return (int)b;
}

// Contiguous chunk of a flat index range owned by this workgroup (XCD-aware order).
__device__ __forceinline__ void chunk_of(long long n, long long& lo, long long& hi) {
  const int nb = gridDim.x;
  const int lb = xcd_remap(blockIdx.x, nb);
  const long long per = (n + nb - 1) / nb;
  lo = (long long)lb * per;
  hi = lo + per < n ? lo + per : n;
}

// q = H_JGN p = (line tridiagonal) p + alpha v (D2'D2 + D3'D3) p  (eq. dJGN, Section 3:
// the transverse coupling of the regulariser is a Neumann Laplacian stencil); partial p.q.
// One wavefront per PE line (lane-contiguous faces, 32-bit index arithmetic); the
// neighbours along the line come from lane shifts. The four wavefronts of a workgroup hold
// four consecutive lines and share them through LDS, so the j +- 1 neighbours of the inner
// lines are read there; the other neighbour lines (j +- 1 at the workgroup's ends, k +- 1)
// come from L2. Every global load of a wavefront (its line, the k +- 1 lines and, at the
// workgroup's ends, the outer j neighbour) is issued before the first arithmetic, from
// clamped (always valid) line indices, and missing neighbours are selected away after.
// DIR: the PCG direction update is fused in: p = z + beta p_old is formed on the fly at
// every stencil point (the same value the separate update computes) and written to pnew;
// otherwise p = pold. q itself is not stored: the PCG update forms it again from p (the
// same function, the same values), which saves its round trip through HBM.
template <int P, bool DIR>
__global__ __launch_bounds__(256) void k_matvec(LineArgs a, const float* __restrict__ z,
                                                const float* __restrict__ pold,
                                                float* __restrict__ pnew,
                                                const float* __restrict__ hd,
                                                const float* __restrict__ ho, double* partial,
                                                const DevState* st) {
  if (st->pcg_done) return;
  __shared__ float sp[EPI_LINE_WAVES][64 * P];   // p of the workgroup's lines, face order
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int blk = xcd_remap(blockIdx.x, a.nblk);
  const int line = blk * EPI_LINE_WAVES + wave;
  const float be = DIR ? (float)st->beta_cg : 0.0f;
  double acc[1] = {0.0};
  // the whole wavefront stays active (the neighbour exchanges along the line are lane
  // shifts); invalid lines and faces work on zeros and store nothing
  const bool lv = line < a.L;
  const int lc = lv ? line : 0;
  const int NF = a.M + 1;
  const int jj = lc % a.m2, kk = lc / a.m2;
  const size_t base = (size_t)lc * NF;
  const bool j0 = jj > 0, j1 = jj < a.m2 - 1, k0 = kk > 0, k1 = kk < a.m3 - 1;
  // the j neighbours from LDS when they belong to this workgroup's lines
  const bool jm_lds = j0 && wave > 0, jp_lds = j1 && wave < EPI_LINE_WAVES - 1;
  // lines read from global: 0 own, 1 k - 1, 2 k + 1, 3 the outer j neighbour of an end wave
  const int jo = (wave == 0) ? lc - 1 : lc + 1;
  const bool jo_need = (wave == 0) ? j0 : (wave == EPI_LINE_WAVES - 1 ? j1 : false);
  const int lines[4] = {lc, k0 ? lc - a.m2 : lc, k1 ? lc + a.m2 : lc, jo_need ? jo : lc};
  float pv[4][P], zv[4][P], hdv[P], hov[P];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int i = lane + 64 * j;
    const int ic = (j < P - 1 || i < NF) ? i : NF - 1;   // in bounds; replaced below
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const size_t o = (size_t)lines[t] * NF + ic;
      pv[t][j] = pold[o];
      if (DIR) zv[t][j] = z[o];
    }
    hdv[j] = hd[base + ic];
    hov[j] = ho[base + ic];
  }
  float pc[P], pk0[P], pk1[P], pjo[P];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int i = lane + 64 * j;
    const bool ok = lv && (j < P - 1 || i < NF);
    const auto mk = [&](int t) { return DIR ? fmaf(be, pv[t][j], zv[t][j]) : pv[t][j]; };
    pc[j] = ok ? mk(0) : 0.0f;
    pk0[j] = mk(1);
    pk1[j] = mk(2);
    pjo[j] = mk(3);
    sp[wave][i] = pc[j];
  }
  __syncthreads();
  float y[P];
  hjgn_apply<P>(a, NF, lane, j0, j1, k0, k1, pc, hdv, hov, pk0, pk1, pjo,
                jm_lds ? sp[wave - 1] : nullptr, jp_lds ? sp[wave + 1] : nullptr, y);
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int i = lane + 64 * j;
    if (lv && (j < P - 1 || i < NF)) {
      if (DIR) store_stream(&pnew[base + i], pc[j]);
      acc[0] += (double)pc[j] * y[j];
    }
  }
  block_partials<1>(acc, partial, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_dot(long long n, const float* __restrict__ x,
                                             const float* __restrict__ y, double* partial) {
  long long lo, hi;
  chunk_of(n, lo, hi);
  double acc[1] = {0.0};
  for (long long f = lo + threadIdx.x; f < hi; f += blockDim.x) acc[0] += (double)x[f] * y[f];
  block_partials<1>(acc, partial, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_udot(long long n, const float* __restrict__ u,
                                              const float* __restrict__ b,
                                              const float* __restrict__ z, double* partial) {
  long long lo, hi;
  chunk_of(n, lo, hi);
  double acc[1] = {0.0};
  for (long long f = lo + threadIdx.x; f < hi; f += blockDim.x)
    acc[0] += (double)u[f] * ((double)b[f] - (double)z[f]);
  block_partials<1>(acc, partial, blockIdx.x);
}

// Coefficients of the cubic B-spline image model: per PE line (one lane each, serial) the
// banded SPD system A w = rhs with A = L D L' factored once on the host in float64 (unit
// lower L of half-width 3: Lf[3k + j - 1] = L[k][k - j]; Dinv[k] = 1 / D[k]). rhs = T (the
// interpolating spline, A = B) or B T (the smoothed fit, A = B'B + theta G; B symmetric).
// The forward sweep keeps y in the float64 scratch Y (N entries).
__global__ __launch_bounds__(64) void k_spline_coef(const float* __restrict__ T,
                                                    float* __restrict__ W, double* Y, int M,
                                                    int L, int normal,
                                                    const double* __restrict__ Lf,
                                                    const double* __restrict__ Dinv) {
  const int line = blockIdx.x * blockDim.x + threadIdx.x;
  if (line >= L) return;
  const float* t = T + (size_t)line * M;
  double* y = Y + (size_t)line * M;
  float* w = W + (size_t)line * M;
  double y1 = 0.0, y2 = 0.0, y3 = 0.0;
  for (int k = 0; k < M; ++k) {
    double r = t[k];
    if (normal) {
      r *= 2.0 / 3.0;
      if (k > 0) r += t[k - 1] * (1.0 / 6.0);
      if (k < M - 1) r += t[k + 1] * (1.0 / 6.0);
    }
    const double yk = r - Lf[3 * k] * y1 - Lf[3 * k + 1] * y2 - Lf[3 * k + 2] * y3;
    y[k] = yk;
    y3 = y2;
    y2 = y1;
    y1 = yk;
  }
  double x1 = 0.0, x2 = 0.0, x3 = 0.0;
  for (int k = M - 1; k >= 0; --k) {
    const double a1 = k + 1 < M ? Lf[3 * (k + 1)] : 0.0;
    const double a2 = k + 2 < M ? Lf[3 * (k + 2) + 1] : 0.0;
    const double a3 = k + 3 < M ? Lf[3 * (k + 3) + 2] : 0.0;
    const double xk = y[k] * Dinv[k] - a1 * x1 - a2 * x2 - a3 * x3;
    w[k] = (float)xk;
    x3 = x2;
    x2 = x1;
    x1 = xk;
  }
}

// After a symmetric Gauss-Seidel application: the PCG partial sums with the new z, in the
// order of the line kernel they replace (first = 1: r.z, r.r as at the PCG start, and
// p = z; first = 0: r.r, r.z as in the update). gate: skip once the PCG has stopped.
__global__ __launch_bounds__(256) void k_sgs_finish(long long n, const float* __restrict__ r,
                                                    const float* __restrict__ z,
                                                    float* __restrict__ p, double* partial,
                                                    int first, const DevState* st) {
  if (!first && st->pcg_done) return;
  long long lo, hi;
  chunk_of(n, lo, hi);
  double rz = 0.0, rr = 0.0;
  for (long long f = lo + threadIdx.x; f < hi; f += blockDim.x) {
    const float rv = r[f], zv = z[f];
    rz += (double)rv * zv;
    rr += (double)rv * rv;
    if (first) p[f] = zv;
  }
  double acc[2] = {first ? rz : rr, first ? rr : rz};
  block_partials<2>(acc, partial, blockIdx.x);
}

// b += lam d with the accepted step length (no-op when the line search failed);
// partial sums |lam d|^2 and |b_old|^2 for the stopping tests (eq. stopping1).
__global__ __launch_bounds__(256) void k_gn_step(long long n, float* __restrict__ b,
                                                 const float* __restrict__ d, double* partial,
                                                 const DevState* st) {
  const float lam = (float)st->lam_acc;
  long long lo, hi;
  chunk_of(n, lo, hi);
  double acc[2] = {0.0, 0.0};
  for (long long f = lo + threadIdx.x; f < hi; f += blockDim.x) {
    const float bo = b[f];
    acc[1] += (double)bo * bo;
    if (lam > 0.0f) {
      const float bn = fmaf(lam, d[f], bo);
      const float s = bn - bo;
      acc[0] += (double)s * s;
      b[f] = bn;
    }
  }
  block_partials<2>(acc, partial, blockIdx.x);
}

// Count cells with |D1 b| > thr (feasibility of a starting guess).
__global__ __launch_bounds__(256) void k_count_violations(LineArgs a, const float* __restrict__ b,
                                                          float thr, double* partial) {
  const int NF = a.M + 1;
  const long long n = (long long)a.M * a.L;
  long long lo, hi;
  chunk_of(n, lo, hi);
  double acc[1] = {0.0};
  for (long long c = lo + threadIdx.x; c < hi; c += blockDim.x) {
    const long long line = c / a.M;
    const int ci = (int)(c % a.M);
    const long long f = line * NF + ci;
    const float g = (b[f + 1] - b[f]) * a.inv_hp;
    if (!(fabsf(g) <= thr)) acc[0] += 1.0;
  }
  block_partials<1>(acc, partial, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_count_nonfinite(long long n, const float* __restrict__ x,
                                                         double* partial) {
  long long lo, hi;
  chunk_of(n, lo, hi);
  double acc[1] = {0.0};
  for (long long f = lo + threadIdx.x; f < hi; f += blockDim.x)
    if (!(fabsf(x[f]) < 3.4e38f)) acc[0] += 1.0;
  block_partials<1>(acc, partial, blockIdx.x);
}

// ------------------------------------------------------------------------------------
// Finalisation: deterministic float64 reductions of the partial sums and the scalar
// logic of PCG, the Armijo test and the ADMM stopping test (eq. admmStop).
// ------------------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_finalize(FinArgs f, DevState* st) {
  __shared__ double s[8];
  __shared__ double s2[8];
  __shared__ double s3[8];
  switch (f.kind) {
    case FIN_EVAL: {
      reduce_partials<NQ_EVAL>(f.partial, f.nb1, s);
      if (threadIdx.x == 0) {
        st->evalD = 0.5 * f.v * s[0];
        st->evalS1 = s[1];
        st->evalSx = s[2];
        st->evalP = s[3];
        st->eval_infeasible = (int)s[4];
        st->evalG2 = s[5];
      }
    } break;
    case FIN_PCG_INIT: {
      reduce_partials<2>(f.partial, f.nb1, s);
      if (threadIdx.x == 0) {
        st->rz = s[0];
        st->rhs2 = s[1];
        st->pcg_iters = 0;
        st->pcg_done = !(s[1] > 0.0);
        st->relres = (s[1] > 0.0) ? 1.0 : 0.0;
      }
    } break;
    case FIN_PCG_ALPHA: {
      if (st->pcg_done) return;
      reduce_partials<1>(f.partial, f.nb1, s);
      if (threadIdx.x == 0) {
        st->pq = s[0];
        if (s[0] > 0.0) {
          st->alpha_cg = st->rz / s[0];
        } else {
          st->alpha_cg = 0.0;
          st->pcg_done = 1;
        }
      }
    } break;
    case FIN_PCG_UPDATE: {
      if (st->pcg_done) return;
      reduce_partials<2>(f.partial, f.nb1, s);
      if (threadIdx.x == 0) {
        const double rr = s[0], rzn = s[1];
        st->rr = rr;
        st->pcg_iters += 1;
        st->relres = sqrt(rr / st->rhs2);
        if (rr <= st->eta2 * st->rhs2 || !(rzn == rzn)) {
          st->pcg_done = 1;
        } else {
          st->beta_cg = rzn / st->rz;
          st->rz = rzn;
        }
      }
    } break;
    case FIN_DOT: {
      reduce_partials<1>(f.partial, f.nb1, s);
      if (threadIdx.x == 0) st->gTd = s[0];
    } break;
    case FIN_LS: {
      if (st->ls_done) return;
      reduce_partials<NQ_EVAL>(f.partial, f.nb1, s);
      if (threadIdx.x == 0) {
        const double J = 0.5 * f.v * s[0] + f.alpha * 0.5 * f.v * (s[1] + s[2]) +
                         f.beta * f.v * s[3];
        const double lam = ldexp(1.0, -f.trial);
        st->ls_trials = f.trial + 1;
        if (s[4] == 0.0 && J <= st->J0 + st->c1 * lam * st->gTd) {
          st->ls_done = 1;
          st->lam_acc = lam;
          st->J_acc = J;
        }
      }
    } break;
    case FIN_STEP: {
      reduce_partials<2>(f.partial, f.nb1, s);
      if (threadIdx.x == 0) {
        st->step2 = s[0];
        st->bold2 = s[1];
      }
    } break;
    case FIN_ADMM: {
      if (st->admm_done) return;
      reduce_partials<NQ_ADMM_E>(f.partial, f.nb1, s);
      if (threadIdx.x == 0) admm_finalize(st, s, f.hist, f.hist_len);
    } break;
    case FIN_LS_INIT: {
      if (threadIdx.x == 0) {
        st->J0 = f.value;
        st->ls_done = 0;
        st->ls_trials = 0;
        st->lam_acc = 0.0;
        st->J_acc = f.value;
      }
    } break;
    case FIN_QUALITY: {
      reduce_partials<NQ_QUALITY>(f.partial, f.nb1, s);
      if (threadIdx.x < NQ_QUALITY) st->quality[threadIdx.x] = s[threadIdx.x];
    } break;
    case FIN_LAGRANGIAN: {
      // L_rho = D(b) + (alpha v / 2)|D1 b|^2 + (alpha v / 2)(|D2 z|^2 + |D3 z|^2)
      //       + rho v u'(b - z) + (rho v / 2)|b - z|^2 at the newest iterate (eq. Lp), with
      // the rho of that iteration and u before any rescale of the next one
      const int it = st->admm_iter - 1;
      if (it < 0 || st->lagr_last == st->admm_iter || it >= f.hist_len) return;
      reduce_partials<NQ_EVAL>(f.partial, f.nb1, s);
      reduce_partials<NQ_EVAL>(f.partial2, f.nb2, s2);
      reduce_partials<1>(f.partial3, f.nb3, s3);
      if (threadIdx.x == 0) {
        const double rho = f.hist[4 * f.hist_len + it], rpri = f.hist[it];
        const double L = 0.5 * f.v * s[0] + 0.5 * f.alpha * f.v * s[1] +
                         0.5 * f.alpha * f.v * s2[2] + rho * f.v * s3[0] +
                         0.5 * rho * f.v * rpri * rpri;
        f.hist[5 * f.hist_len + it] = L;
        st->lagr_last = st->admm_iter;
      }
    } break;
    case FIN_TERMS: {
      reduce_partials<NQ_EVAL>(f.partial, f.nb1, s);
      if (threadIdx.x == 0) {
        const double D = 0.5 * f.v * s[0];
        const double S = 0.5 * f.v * (s[1] + s[2]);
        const bool feasible = s[4] == 0.0;
        const double P = f.trial ? (feasible ? f.beta * f.v * s[3] : INFINITY) : 0.0;
        f.hist[0] = D + f.alpha * S + P;
        f.hist[1] = D;
        f.hist[2] = S;
        f.hist[3] = P;
        f.hist[4] = feasible ? 1.0 : 0.0;
      }
    } break;
    case FIN_HARD_RESET: {
      if (threadIdx.x == 0 && !st->admm_done) {
        st->hard_total += st->hard_count;
        st->hard_count = 0;
      }
    } break;
    default:
      break;
  }
}

// ------------------------------------------------------------------------------------
// Launchers
// ------------------------------------------------------------------------------------
void launch_matvec(hipStream_t s, int P, LineArgs a, const float* z, const float* pold,
                   float* pnew, const float* hdiag, const float* hoff, double* partial,
                   const DevState* st) {
  const int nb = line_blocks(a);
  a.nblk = nb;
  if (z != nullptr) {
    EPI_DISPATCH_P(P, hipLaunchKernelGGL((k_matvec<PP, true>), dim3(nb), dim3(256), 0, s, a, z,
                                         pold, pnew, hdiag, hoff, partial, st));
  } else {
    EPI_DISPATCH_P(P, hipLaunchKernelGGL((k_matvec<PP, false>), dim3(nb), dim3(256), 0, s, a,
                                         nullptr, pold, nullptr, hdiag, hoff, partial, st));
  }
}
void launch_dot(hipStream_t s, long long n, const float* x, const float* y, double* partial) {
  hipLaunchKernelGGL(k_dot, dim3(flat_blocks(n)), dim3(256), 0, s, n, x, y, partial);
}
void launch_spline_coef(hipStream_t s, const float* T, float* W, double* Y, int M, int L,
                        int normal, const double* Lf, const double* Dinv) {
  hipLaunchKernelGGL(k_spline_coef, dim3((L + 63) / 64), dim3(64), 0, s, T, W, Y, M, L, normal,
                     Lf, Dinv);
}
void launch_udot(hipStream_t s, long long n, const float* u, const float* b, const float* z,
                 double* partial) {
  hipLaunchKernelGGL(k_udot, dim3(flat_blocks(n)), dim3(256), 0, s, n, u, b, z, partial);
}
void launch_sgs_finish(hipStream_t s, long long n, const float* r, const float* z, float* p,
                       double* partial, int first, const DevState* st) {
  hipLaunchKernelGGL(k_sgs_finish, dim3(flat_blocks(n)), dim3(256), 0, s, n, r, z, p, partial,
                     first, st);
}
void launch_gn_step(hipStream_t s, long long n, float* b, const float* d, double* partial,
                    const DevState* st) {
  hipLaunchKernelGGL(k_gn_step, dim3(flat_blocks(n)), dim3(256), 0, s, n, b, d, partial, st);
}
void launch_count_violations(hipStream_t s, LineArgs a, const float* b, float thr,
                             double* partial) {
  const long long n = (long long)a.M * a.L;
  hipLaunchKernelGGL(k_count_violations, dim3(flat_blocks(n)), dim3(256), 0, s, a, b, thr,
                     partial);
}
void launch_count_nonfinite(hipStream_t s, long long n, const float* x, double* partial) {
  hipLaunchKernelGGL(k_count_nonfinite, dim3(flat_blocks(n)), dim3(256), 0, s, n, x, partial);
}
void launch_finalize(hipStream_t s, const FinArgs& f, DevState* st) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, f, st);
}

}  // namespace epi
