// Host-side helpers shared by the single-volume runtime and the batched engine.
#pragma once

#include <hip/hip_runtime.h>

#include "epi.h"
#include "epi_common.hpp"

namespace epi {

// Record the thread-local error message and return s.
epi_status fail(epi_status s, const char* fmt, ...);

// Packed DCT matrices (forward and inverse, axes 2 and 3) and eigenvalue tables.
struct DctTables {
  void *A2f = nullptr, *A2i = nullptr, *A3f = nullptr, *A3i = nullptr;
  int RT2 = 0, KS2 = 0, RT3 = 0, KS3 = 0;
  float *lam2 = nullptr, *lam3 = nullptr;
};
epi_status build_dct_tables(int m2, int m3, double h2, double h3, int precision, DctTables* t);
void free_dct_tables(DctTables* t);

epi_status validate_grid(const epi_grid* grid);
LineArgs make_line_args(const epi_grid* grid, const float* Ip, const float* Im);
GemmArgs make_gemm_axis3(int M, int m2, int m3, float alpha, const DctTables& t,
                         const float* in, float* out, bool inverse, const DevState* st);
GemmArgs make_gemm_axis2(int M, int m2, int m3, float alpha, const DctTables& t,
                         const float* in, float* out, const DevState* st);
int tiles_axis3(int M, int m2);
int tiles_axis2(int M, int m3);

// Rows of the device-side ADMM history: r_pri, r_dual, eps_pri, eps_dual, rho, and the
// augmented Lagrangian (filled only by solves that ask for it).
constexpr int EPI_HIST_ROWS = 6;
epi_status validate_rho_opts(const epi_admm_opts* opts);
void init_rho_state(DevState* h, const epi_admm_opts* opts);

}  // namespace epi
