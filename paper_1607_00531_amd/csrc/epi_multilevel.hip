// Multilevel strategy (Section 4.4): coarse-to-fine ADMM with image restriction, field
// prolongation and the restart b0 = z0 = (b_f + z_f) / 2, u0 = 0 of the third strategy.
//
// Transfer operators (the paper defers them to the image-registration literature): an
// axis with an even cell count of at least 4 is halved per level; images are restricted
// by the mean of the fine cells of each coarse cell; the field is prolongated linearly
// along PE on the faces (even fine faces on coarse faces, odd ones at the midpoints) and
// with cell-centred weights 3/4 (nearer) and 1/4 (farther coarse neighbour, clamped at the
// ends) across. Along PE the prolongated field keeps the coarse D1 b values and across it
// is a convex combination of coarse lines, so a feasible coarse field stays feasible.
#include <hip/hip_runtime.h>

#include <string.h>

#include <algorithm>
#include <array>
#include <vector>

#include "epi.h"
#include "epi_common.hpp"
#include "epi_internal.hpp"

#define EPI_API extern "C" __attribute__((visibility("default")))

namespace epi {

static int ml_blocks(long long n) {
  long long b = (n + 255) / 256;
  return (int)std::min<long long>(std::max<long long>(b, 1), 65535LL * 16);
}

// coarse cell (c, j, k) = mean of its fine cells; f* in {1, 2} are the factors per axis
__global__ __launch_bounds__(256) void k_restrict_cells(const float* __restrict__ fine,
                                                        float* __restrict__ coarse, int M,
                                                        int m2, int fM, int f2, int f3,
                                                        int Mc, int m2c, long long nc) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < nc; i += (long long)gridDim.x * 256) {
    const int c = (int)(i % Mc);
    const long long r = i / Mc;
    const int j = (int)(r % m2c), k = (int)(r / m2c);
    float s = 0.0f;
    for (int dk = 0; dk < f3; ++dk)
      for (int dj = 0; dj < f2; ++dj)
        for (int dc = 0; dc < fM; ++dc)
          s += fine[((size_t)(k * f3 + dk) * m2 + (j * f2 + dj)) * M + (c * fM + dc)];
    coarse[i] = s * (1.0f / (float)(fM * f2 * f3));
  }
}

// weights of the cell-centred prolongation along one axis: fine cell jf from coarse cells
__device__ __forceinline__ void cc_weights(int jf, int nc, int f, int& j0, int& j1, float& w0,
                                           float& w1) {
  if (f == 1) {
    j0 = j1 = jf;
    w0 = 1.0f;
    w1 = 0.0f;
    return;
  }
  const int J = jf >> 1;
  j0 = J;
  j1 = (jf & 1) ? min(J + 1, nc - 1) : max(J - 1, 0);
  w0 = 0.75f;
  w1 = 0.25f;
}

// fine face (i, j, k) from the coarse faces (linear along PE, cell-centred across)
__global__ __launch_bounds__(256) void k_prolong_faces(const float* __restrict__ coarse,
                                                       float* __restrict__ fine, int M, int m2,
                                                       int fM, int f2, int f3, int Mc, int m2c,
                                                       int m3c, long long nf) {
  const int NF = M + 1, NFc = Mc + 1;
  for (long long idx = blockIdx.x * 256LL + threadIdx.x; idx < nf;
       idx += (long long)gridDim.x * 256) {
    const int i = (int)(idx % NF);
    const long long r = idx / NF;
    const int j = (int)(r % m2), k = (int)(r / m2);
    int i0, i1;
    float wi0, wi1;
    if (fM == 1) {
      i0 = i1 = i;
      wi0 = 1.0f;
      wi1 = 0.0f;
    } else {
      i0 = i >> 1;
      i1 = (i & 1) ? i0 + 1 : i0;
      wi0 = (i & 1) ? 0.5f : 1.0f;
      wi1 = (i & 1) ? 0.5f : 0.0f;
    }
    int j0, j1, k0, k1;
    float wj0, wj1, wk0, wk1;
    cc_weights(j, m2c, f2, j0, j1, wj0, wj1);
    cc_weights(k, m3c, f3, k0, k1, wk0, wk1);
    auto at = [&](int kk, int jj, int ii) {
      return coarse[((size_t)kk * m2c + jj) * NFc + ii];
    };
    auto line = [&](int kk, int jj) { return wi0 * at(kk, jj, i0) + wi1 * at(kk, jj, i1); };
    const float a = wj0 * line(k0, j0) + wj1 * line(k0, j1);
    const float b = wj0 * line(k1, j0) + wj1 * line(k1, j1);
    fine[idx] = wk0 * a + wk1 * b;
  }
}

__global__ __launch_bounds__(256) void k_average(const float* __restrict__ x,
                                                 const float* __restrict__ y,
                                                 float* __restrict__ out, long long n) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    out[i] = 0.5f * (x[i] + y[i]);
}

// number of cells with |D1 b| > thr (one counter, vector atomics)
__global__ __launch_bounds__(256) void k_violations(const float* __restrict__ b, int M, float inv_hp,
                                                    float thr, long long ncell, int* count) {
  int mine = 0;
  for (long long c = blockIdx.x * 256LL + threadIdx.x; c < ncell;
       c += (long long)gridDim.x * 256) {
    const long long line = c / M;
    const int ci = (int)(c % M);
    const long long f = line * (M + 1) + ci;
    if (!(fabsf((b[f + 1] - b[f]) * inv_hp) <= thr)) ++mine;
  }
  if (mine) atomicAdd(count, mine);
}

}  // namespace epi

using namespace epi;

#define MLCHK(call)                                                                    \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) {                                                            \
      st = fail(e_ == hipErrorOutOfMemory ? EPI_ENOMEM : EPI_EHIP, "%s: %s (%s:%d)",   \
                #call, hipGetErrorString(e_), __FILE__, __LINE__);                     \
      goto done;                                                                       \
    }                                                                                  \
  } while (0)

static bool valid_factors(const int32_t* mf, const int32_t* mc, int f[3]) {
  for (int a = 0; a < 3; ++a) {
    if (mc[a] < 1 || mf[a] < 1) return false;
    if (mf[a] == mc[a]) f[a] = 1;
    else if (mf[a] == 2 * mc[a]) f[a] = 2;
    else return false;
  }
  return true;
}

EPI_API epi_status epi_restrict_cells(const int32_t m_fine[3], const int32_t m_coarse[3],
                                      const float* d_fine, float* d_coarse, void* stream) {
  if (!m_fine || !m_coarse || !d_fine || !d_coarse) return fail(EPI_EINVAL, "null argument");
  int f[3];
  if (!valid_factors(m_fine, m_coarse, f))
    return fail(EPI_EINVAL, "each fine count must equal the coarse count or twice it");
  const long long nc = (long long)m_coarse[0] * m_coarse[1] * m_coarse[2];
  hipLaunchKernelGGL(k_restrict_cells, dim3(ml_blocks(nc)), dim3(256), 0, (hipStream_t)stream,
                     d_fine, d_coarse, m_fine[0], m_fine[1], f[0], f[1], f[2], m_coarse[0],
                     m_coarse[1], nc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(EPI_EHIP, "restriction launch: %s", hipGetErrorString(e));
  return EPI_OK;
}

EPI_API epi_status epi_prolong_faces(const int32_t m_coarse[3], const int32_t m_fine[3],
                                     const float* d_coarse, float* d_fine, void* stream) {
  if (!m_fine || !m_coarse || !d_fine || !d_coarse) return fail(EPI_EINVAL, "null argument");
  int f[3];
  if (!valid_factors(m_fine, m_coarse, f))
    return fail(EPI_EINVAL, "each fine count must equal the coarse count or twice it");
  const long long nf = (long long)(m_fine[0] + 1) * m_fine[1] * m_fine[2];
  hipLaunchKernelGGL(k_prolong_faces, dim3(ml_blocks(nf)), dim3(256), 0, (hipStream_t)stream,
                     d_coarse, d_fine, m_fine[0], m_fine[1], f[0], f[1], f[2], m_coarse[0],
                     m_coarse[1], m_coarse[2], nf);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(EPI_EHIP, "prolongation launch: %s", hipGetErrorString(e));
  return EPI_OK;
}

static int ml_coarse(int m) { return (m % 2 == 0 && m >= 4) ? m / 2 : m; }

namespace {

// Level sizes (coarse to fine) and the restricted image pairs of one multilevel solve.
struct MLHierarchy {
  std::vector<std::array<int, 3>> sizes;
  std::vector<float*> Ip, Im;   // level l images (the finest level borrows the caller's)
  int nl = 0;

  epi_status build(const epi_grid* grid, const float* d_Iplus, const float* d_Iminus,
                   int levels, hipStream_t s) {
    sizes.assign(1, {grid->m[0], grid->m[1], grid->m[2]});
    while ((int)sizes.size() < levels) {
      const auto& l = sizes.back();
      std::array<int, 3> c{ml_coarse(l[0]), ml_coarse(l[1]), l[2] > 1 ? ml_coarse(l[2]) : 1};
      if (c == l) break;
      sizes.push_back(c);
    }
    std::reverse(sizes.begin(), sizes.end());
    nl = (int)sizes.size();
    Ip.assign(nl, nullptr);
    Im.assign(nl, nullptr);
    Ip[nl - 1] = const_cast<float*>(d_Iplus);
    Im[nl - 1] = const_cast<float*>(d_Iminus);
    for (int l = nl - 2; l >= 0; --l) {   // fine to coarse
      hipError_t e = hipMalloc(&Ip[l], ncell(l) * sizeof(float));
      if (e == hipSuccess) e = hipMalloc(&Im[l], ncell(l) * sizeof(float));
      if (e != hipSuccess)
        return fail(e == hipErrorOutOfMemory ? EPI_ENOMEM : EPI_EHIP, "level images: %s",
                    hipGetErrorString(e));
      int32_t mf[3] = {sizes[l + 1][0], sizes[l + 1][1], sizes[l + 1][2]};
      int32_t mc[3] = {sizes[l][0], sizes[l][1], sizes[l][2]};
      epi_status st = epi_restrict_cells(mf, mc, Ip[l + 1], Ip[l], s);
      if (st == EPI_OK) st = epi_restrict_cells(mf, mc, Im[l + 1], Im[l], s);
      if (st != EPI_OK) return st;
    }
    return EPI_OK;
  }
  size_t ncell(int l) const { return (size_t)sizes[l][0] * sizes[l][1] * sizes[l][2]; }
  size_t nface(int l) const { return (size_t)(sizes[l][0] + 1) * sizes[l][1] * sizes[l][2]; }
  // the grid of level l: same domain, h scaled with the cell counts
  epi_grid grid(const epi_grid* fine, int l) const {
    epi_grid g = *fine;
    for (int a = 0; a < 3; ++a) {
      g.m[a] = sizes[l][a];
      if (!(a == 2 && fine->m[2] == 1)) g.h[a] = fine->h[a] * fine->m[a] / sizes[l][a];
    }
    return g;
  }
  epi_status prolong(int l, const float* coarse, float* fine, hipStream_t s) const {
    int32_t mc[3] = {sizes[l - 1][0], sizes[l - 1][1], sizes[l - 1][2]};
    int32_t mf[3] = {sizes[l][0], sizes[l][1], sizes[l][2]};
    return epi_prolong_faces(mc, mf, coarse, fine, s);
  }
  ~MLHierarchy() {
    for (int l = 0; l < nl - 1; ++l) {
      if (Ip[l]) (void)hipFree(Ip[l]);
      if (Im[l]) (void)hipFree(Im[l]);
    }
  }
};

}  // namespace

EPI_API epi_status epi_solve_multilevel_admm(const epi_grid* grid, const float* d_Iplus,
                                             const float* d_Iminus, int32_t levels,
                                             int32_t restart, const epi_admm_opts* opts,
                                             void* stream, float* d_b, epi_ml_report* rep) {
  if (!grid || !d_Iplus || !d_Iminus || !opts || !d_b) return fail(EPI_EINVAL, "null argument");
  if (levels < 1 || levels > EPI_ML_MAX_LEVELS)
    return fail(EPI_EINVAL, "levels must be in [1, %d]", EPI_ML_MAX_LEVELS);
  if (restart < EPI_ML_RESTART_PROLONG_ALL || restart > EPI_ML_RESTART_AVERAGE)
    return fail(EPI_EINVAL, "unknown restart strategy %d", restart);
  epi_status st = validate_grid(grid);
  if (st != EPI_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  MLHierarchy H;
  float *bc = nullptr, *zc = nullptr, *uc = nullptr, *tmp = nullptr, *z = nullptr, *u = nullptr,
        *bl = nullptr;
  int* d_count = nullptr;
  epi_problem* prob = nullptr;
  double rho = opts->rho;
  int nl = 0;
  if (rep) memset(rep, 0, sizeof(*rep));
  if ((st = H.build(grid, d_Iplus, d_Iminus, levels, s)) != EPI_OK) goto done;
  nl = H.nl;
  if (rep) rep->levels = nl;
  MLCHK(hipMalloc(&d_count, sizeof(int)));
  for (int l = 0; l < nl; ++l) {
    const auto& m = H.sizes[l];
    const size_t nf = H.nface(l);
    const epi_grid g = H.grid(grid, l);
    if ((st = epi_setup(&g, H.Ip[l], H.Im[l], s, &prob)) != EPI_OK) goto done;
    bl = (l == nl - 1) ? d_b : nullptr;
    if (!bl) MLCHK(hipMalloc(&bl, nf * sizeof(float)));
    MLCHK(hipMalloc(&z, nf * sizeof(float)));
    MLCHK(hipMalloc(&u, nf * sizeof(float)));
    if (l == 0) {
      MLCHK(hipMemsetAsync(bl, 0, nf * sizeof(float), s));
      MLCHK(hipMemsetAsync(z, 0, nf * sizeof(float), s));
      MLCHK(hipMemsetAsync(u, 0, nf * sizeof(float), s));
    } else if (restart == EPI_ML_RESTART_PROLONG_ALL) {
      // b0 = P b_c, z0 = P z_c, u0 = P u_c
      if ((st = H.prolong(l, bc, bl, s)) != EPI_OK) goto done;
      if ((st = H.prolong(l, zc, z, s)) != EPI_OK) goto done;
      if ((st = H.prolong(l, uc, u, s)) != EPI_OK) goto done;
    } else if (restart == EPI_ML_RESTART_FINE_B) {
      // b0 = z0 = P b_c, u0 = 0
      if ((st = H.prolong(l, bc, bl, s)) != EPI_OK) goto done;
      MLCHK(hipMemcpyAsync(z, bl, nf * sizeof(float), hipMemcpyDeviceToDevice, s));
      MLCHK(hipMemsetAsync(u, 0, nf * sizeof(float), s));
    } else {
      // b0 = z0 = P((b_c + z_c) / 2), u0 = 0; b0 = P b_c if the average violates |D1 b| <= 1
      const size_t ncf = H.nface(l - 1);
      MLCHK(hipMalloc(&tmp, ncf * sizeof(float)));
      hipLaunchKernelGGL(k_average, dim3(ml_blocks((long long)ncf)), dim3(256), 0, s, bc, zc, tmp,
                         (long long)ncf);
      if ((st = H.prolong(l, tmp, z, s)) != EPI_OK) goto done;
      MLCHK(hipMemcpyAsync(bl, z, nf * sizeof(float), hipMemcpyDeviceToDevice, s));
      MLCHK(hipMemsetAsync(u, 0, nf * sizeof(float), s));
      MLCHK(hipMemsetAsync(d_count, 0, sizeof(int), s));
      const long long nce = (long long)m[0] * m[1] * m[2];
      hipLaunchKernelGGL(k_violations, dim3(ml_blocks(nce)), dim3(256), 0, s, bl, m[0],
                         (float)(1.0 / g.h[0]), 1.0f + 1e-5f, nce, d_count);
      int count = 0;
      MLCHK(hipMemcpyAsync(&count, d_count, sizeof(int), hipMemcpyDeviceToHost, s));
      MLCHK(hipStreamSynchronize(s));
      if (count > 0 && (st = H.prolong(l, bc, bl, s)) != EPI_OK) goto done;
      MLCHK(hipFree(tmp));
      tmp = nullptr;
      if (rep) rep->fallback[l] = count > 0;
    }
    if (l > 0) {
      MLCHK(hipStreamSynchronize(s));
      MLCHK(hipFree(bc));
      MLCHK(hipFree(zc));
      MLCHK(hipFree(uc));
      bc = zc = uc = nullptr;
    }
    {
      epi_admm_opts o = *opts;
      o.rho = rho;
      std::vector<double> rh(std::max(o.max_iter, 1));
      epi_admm_report r{};
      r.rho = rh.data();
      st = epi_solve_admm(prob, bl, z, u, &o, &r);
      if (st != EPI_OK) goto done;
      if (r.iters > 0) rho = rh[r.iters - 1];
      if (rep) {
        for (int a = 0; a < 3; ++a) rep->m[l][a] = m[a];
        rep->iters[l] = r.iters;
        rep->converged[l] = r.converged;
        rep->rho_last[l] = rho;
      }
    }
    epi_destroy(prob);
    prob = nullptr;
    if (l < nl - 1) {
      bc = bl;
      zc = z;
      uc = u;
    } else {
      MLCHK(hipStreamSynchronize(s));
      MLCHK(hipFree(z));
      MLCHK(hipFree(u));
    }
    bl = nullptr;
    z = u = nullptr;
  }
  MLCHK(hipStreamSynchronize(s));
done:
  if (prob) epi_destroy(prob);
  if (s) (void)hipStreamSynchronize(s);
  void* rest[] = {bc, zc, uc, tmp, z, u, d_count};
  for (void* p : rest)
    if (p) (void)hipFree(p);
  if (bl && bl != d_b) (void)hipFree(bl);
  return st;
}

EPI_API epi_status epi_solve_multilevel_gnpcg(const epi_grid* grid, const float* d_Iplus,
                                              const float* d_Iminus, int32_t levels,
                                              const epi_gn_opts* opts, void* stream,
                                              float* d_b, epi_ml_report* rep) {
  if (!grid || !d_Iplus || !d_Iminus || !opts || !d_b) return fail(EPI_EINVAL, "null argument");
  if (levels < 1 || levels > EPI_ML_MAX_LEVELS)
    return fail(EPI_EINVAL, "levels must be in [1, %d]", EPI_ML_MAX_LEVELS);
  epi_status st = validate_grid(grid);
  if (st != EPI_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  MLHierarchy H;
  float *bc = nullptr, *bl = nullptr;
  epi_problem* prob = nullptr;
  int nl = 0;
  if (rep) memset(rep, 0, sizeof(*rep));
  if ((st = H.build(grid, d_Iplus, d_Iminus, levels, s)) != EPI_OK) goto done;
  nl = H.nl;
  if (rep) rep->levels = nl;
  for (int l = 0; l < nl; ++l) {
    const size_t nf = H.nface(l);
    const epi_grid g = H.grid(grid, l);
    if ((st = epi_setup(&g, H.Ip[l], H.Im[l], s, &prob)) != EPI_OK) goto done;
    bl = (l == nl - 1) ? d_b : nullptr;
    if (!bl) MLCHK(hipMalloc(&bl, nf * sizeof(float)));
    if (l == 0) {
      MLCHK(hipMemsetAsync(bl, 0, nf * sizeof(float), s));
    } else {
      // b0 = P b_c (feasible when b_c is: prolongation keeps the coarse D1 b values)
      if ((st = H.prolong(l, bc, bl, s)) != EPI_OK) goto done;
      MLCHK(hipStreamSynchronize(s));
      MLCHK(hipFree(bc));
      bc = nullptr;
    }
    {
      const int n1 = std::max(opts->max_iter, 0) + 1;
      std::vector<double> J(n1), gn(n1), rel(n1), stp(n1);
      std::vector<int32_t> pcg(n1);
      epi_gn_report r{};
      r.J = J.data();
      r.grad_norm = gn.data();
      r.pcg_relres = rel.data();
      r.step = stp.data();
      r.pcg_iters = pcg.data();
      st = epi_solve_gnpcg(prob, bl, opts, &r);
      if (st != EPI_OK) goto done;
      if (rep) {
        for (int a = 0; a < 3; ++a) rep->m[l][a] = H.sizes[l][a];
        rep->iters[l] = r.iters;
        rep->converged[l] = r.converged;
        rep->J_last[l] = J[r.iters];
      }
    }
    epi_destroy(prob);
    prob = nullptr;
    if (l < nl - 1) bc = bl;
    bl = nullptr;
  }
  MLCHK(hipStreamSynchronize(s));
done:
  if (prob) epi_destroy(prob);
  if (s) (void)hipStreamSynchronize(s);
  if (bc) (void)hipFree(bc);
  if (bl && bl != d_b) (void)hipFree(bl);
  return st;
}
