// Structures shared by the host runtime and the kernels (no HIP types in the public ABI).
#pragma once

#include <stdint.h>

#define EPI_WAVE 64
#define EPI_LINE_WAVES 4            // PE lines (wavefronts) per 256-thread workgroup
#define EPI_PMAX 8                  // faces per lane: M + 1 <= 512

namespace epi {

// Per-problem constants of the line kernels (Section 3 discretisation, canonical layout).
struct LineArgs {
  const float* Ip;   // image with PE direction +v, N cells
  const float* Im;   // image with PE direction -v, N cells
  int M, m2, m3, L;  // cells per PE line, transverse counts, number of lines
  float hp, inv_hp;  // PE voxel edge and its inverse
  float inv_h2sq, inv_h3sq;
  float v;           // cell volume
  float alpha, beta, gamma;
  int nblk;          // workgroups of the launch (for the XCD remap)
  int model;         // image model: 0 linear (Ip, Im are the samples), 1 cubic B-spline
                     // (Ip, Im are the spline coefficients of the two images)
};

// Device-resident scalars of the iterative solvers. Written by the single-block
// finalisation kernels, read by the bulk kernels (so that no host round trip is needed
// inside PCG, the line search or an ADMM iteration).
struct DevState {
  // PCG (Section 4.1)
  double rz, pq, rr, rhs2, alpha_cg, beta_cg, relres, eta2;
  int pcg_done, pcg_iters, pcg_first, pad0;
  // line search on J_GN (Armijo)
  double J0, gTd, lam_acc, J_acc, c1;
  int ls_done, ls_trials, ls_max, pad1;
  // GN bookkeeping of the last evaluation
  double evalD, evalS1, evalSx, evalP, evalG2;
  int eval_infeasible, pad2;
  double step2, bold2;
  // ADMM (Section 4.2)
  double rho, eps_abs, eps_rel, sqrt_n, v;
  int admm_done, admm_iter, admm_max, hard_count;
  int max_active, pad3;
  long long hard_total;
  int numeric_bad, pad4;
  // residual balancing of rho (rho_mode 1, 2): u holds values scaled by u_scale until the
  // next iteration has read it (the rescale rho_old / rho_new of the scaled dual)
  double u_scale, tau, mu, rho_min;
  int rho_mode, pad5;
  // active-set iteration cap of one line's QP (0: 4 (M + 1)); the last iteration whose
  // augmented Lagrangian was recorded (with_lagrangian)
  int qp_max_iter, lagr_last;
  // corrected-image pair: sum a, sum b, sum a^2, sum b^2, sum ab, sum (a - b)^2
  double quality[6];
};

// Number of float64 partial sums written per workgroup by each reduction kernel.
enum : int {
  NQ_EVAL = 6,    // sum r^2, sum g^2, sum cross diffs^2, sum phi, infeasible count, |grad|^2
  NQ_PCG = 2,     // two dot products
  NQ_ADMM_E = 5,  // |b-z|^2, |z-z_old|^2, |z|^2, |u|^2, |b|^2
  NQ_QUALITY = 6  // sums of the corrected-image pair
};

// Arguments of the DCT products of the z-step.
struct GemmArgs {
  const float* in;
  float* out;
  int rows;          // transform length m (= contraction length)
  int ncol;          // columns per batch
  long long ld;      // row stride (elements) of in/out
  long long bstride; // batch stride (elements)
  int nbatch;
  int col_tiles;
  int RT, KS;        // 16-row tiles and contraction steps of the packed matrices
  int dir;           // unfused split-bfloat16 pass: 0 forward, 1 inverse, 2 per-batch
                     // operator (even/odd sums and differences in, even/odd halves out)
  const void* A1;    // packed forward matrix fragments
  long long a_bstride;  // dir 2: 16-byte fragments per batch entry of A1 (hi and lo blocks)
  const void* A2;    // packed inverse matrix fragments (fused pass only)
  const float* lam_row;    // eigenvalues along the transformed axis (fused pass)
  const float* lam_batch;  // eigenvalues along the batch axis (fused pass), may be null
  float alpha;
  const DevState* st;      // rho is read from here
  // epilogue (ADMM u-step and residual sums), epi = 0: plain store
  int epi;
  const float* b;
  float* z;
  float* u;
  double* partial;
  const int* done;
};

// ------------------------------------------------------------------------------------
// Batched (multi-volume) engine: device-side tables read by the persistent kernels
// ------------------------------------------------------------------------------------
#define EPI_BATCH_MAX 128   // resident volumes (slots) per batch

// Work items of one kernel class: the items of slot slot[k] are [first[k], first[k+1]).
struct RangeTable {
  int n, pad;
  int slot[EPI_BATCH_MAX];
  int first[EPI_BATCH_MAX + 1];
};

// One resident volume: its geometry, state arrays (caller-owned, resident), workspace,
// stopping state and the three z-step products (2D: only g2, carrying the epilogue).
struct BatchSlotDev {
  LineArgs la;
  float *b, *z, *u, *w;
  DevState* st;
  GemmArgs g1, g2, g3;
  int three_pass, active;
  double* hist;
  int hist_len;
  int last_ntiles;
  const double* last_partial;
};

struct HardItem {
  int slot, line;
};

// b-step classes by faces per lane P (index P); DCT classes: 0/1 pass 1 (rows <= 128 /
// <= 256), 2/3 pass 2 of 3D volumes, 4/5 pass 2 of 2D volumes (with epilogue), 6/7 pass 3.
struct BatchDev {
  BatchSlotDev slots[EPI_BATCH_MAX];
  RangeTable bt[EPI_PMAX + 1];
  RangeTable dt[8];
  int hard_count[EPI_PMAX + 1];
  HardItem* hard_list[EPI_PMAX + 1];
};

}  // namespace epi
