// Host-side launchers of the kernels (one translation unit per kernel family).
#pragma once

#include <hip/hip_runtime.h>

#include <functional>

#include "epi_common.hpp"

namespace epi {

int line_blocks(const LineArgs& a);

// Launch a line kernel template for the faces-per-lane count P_ (1..8) as PP.
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


// epi_line.hip
void launch_eval(hipStream_t s, int P, int mode, LineArgs a, const float* b, const float* d,
                 int trial, int with_pen, float* grad, float* hdiag, float* hoff,
                 double* partial, const DevState* st);
void launch_pcg_init(hipStream_t s, int P, LineArgs a, int precond, const float* grad,
                     const float* hdiag, const float* hoff, float* x, float* r, float* z,
                     float* p, double* partial);
// x += alpha p, r -= alpha H_JGN p (q formed again from p and its neighbour lines),
// z = Pinv r; partial sums r.r and r.z
void launch_pcg_update(hipStream_t s, int P, LineArgs a, int precond, const float* hdiag,
                       const float* hoff, float* x, float* r, float* z, const float* p,
                       double* partial, const DevState* st);
// z = Pinv r with a line-local preconditioner (BLOCK, JACOBI, NONE)
void launch_precond(hipStream_t s, int P, LineArgs a, int precond, const float* hdiag,
                    const float* hoff, const float* r, float* z);
// symmetric Gauss-Seidel z = P_SGS^-1 r (all levels of both sweeps; z may not alias r)
void launch_sgs(hipStream_t s, int P, LineArgs a, const float* hdiag, const float* hoff,
                const float* r, float* z, const DevState* st, int gate);
// part 0: the fast-path kernel over all lines; part 1: the active-set kernel
void launch_admm_bstep_part(hipStream_t s, int part, int P, LineArgs a, float* b,
                            const float* z, const float* u, float* w, int* hard_list,
                            DevState* st, int hard_blocks);
void launch_admm_bstep(hipStream_t s, int P, LineArgs a, float* b, const float* z,
                       const float* u, float* w, int* hard_list, DevState* st, int hard_blocks,
                       const std::function<void(int)>& before,
                       const std::function<void()>& after);

// epi_vec.hip
int flat_blocks(long long n);
void launch_correct(hipStream_t s, int P, LineArgs a, const float* b, float* outp, float* outm,
                    double* partial);
// partial sums p.q of q = H_JGN p with p = pold (z null) or p = z + beta pold written to
// pnew (fused update); q itself is formed again by the PCG update
void launch_matvec(hipStream_t s, int P, LineArgs a, const float* z, const float* pold,
                   float* pnew, const float* hdiag, const float* hoff, double* partial,
                   const DevState* st);
void launch_dot(hipStream_t s, long long n, const float* x, const float* y, double* partial);
// cubic B-spline coefficients of the N = M L samples T into W (one lane per line; Y: N
// doubles of scratch; Lf, Dinv: the host factorisation of the line system)
void launch_spline_coef(hipStream_t s, const float* T, float* W, double* Y, int M, int L,
                        int normal, const double* Lf, const double* Dinv);
// partial sums of u'(b - z) (the multiplier term of the augmented Lagrangian)
void launch_udot(hipStream_t s, long long n, const float* u, const float* b, const float* z,
                 double* partial);
void launch_sgs_finish(hipStream_t s, long long n, const float* r, const float* z, float* p,
                       double* partial, int first, const DevState* st);
void launch_gn_step(hipStream_t s, long long n, float* b, const float* d, double* partial,
                    const DevState* st);
void launch_count_violations(hipStream_t s, LineArgs a, const float* b, float thr,
                             double* partial);
void launch_count_nonfinite(hipStream_t s, long long n, const float* x, double* partial);

// single-block finalisation kernels
enum FinKind : int {
  FIN_EVAL = 0,        // -> st->eval*
  FIN_PCG_INIT = 1,    // rz, rhs2
  FIN_PCG_ALPHA = 2,   // alpha = rz / pq
  FIN_PCG_UPDATE = 3,  // relres, beta, done
  FIN_DOT = 4,         // gTd
  FIN_LS = 5,          // Armijo test of one trial
  FIN_STEP = 6,        // |lam d|^2, |b_old|^2
  FIN_ADMM = 7,        // residuals, tolerances, stopping flag, history
  FIN_LS_INIT = 8,     // J0 = value; clear the line-search state
  FIN_HARD_RESET = 9,  // fold hard_count into hard_total between SQP linearisations
  FIN_QUALITY = 10,    // -> st->quality (sums of the corrected-image pair)
  FIN_LAGRANGIAN = 11, // augmented Lagrangian of the last ADMM iterate -> history row 5
  FIN_TERMS = 12       // objective terms J, D, S, P, feasible -> hist[0..4] (trial: penalty)
};
struct FinArgs {
  int kind;
  const double* partial;
  int nb1;           // blocks of the first partial range
  int nb2;           // blocks of the second range (ADMM: hard-line kernel)
  const double* partial2;
  int nb3;
  const double* partial3;
  int trial;
  double v, alpha, beta;
  double* hist;      // ADMM history base (EPI_HIST_ROWS arrays of hist_len)
  int hist_len;
  double value;
};
void launch_finalize(hipStream_t s, const FinArgs& f, DevState* st);

// epi_dct.hip
void launch_dct_axis3(hipStream_t s, int prec, const GemmArgs& g);
void launch_dct_axis2_fused(hipStream_t s, int prec, const GemmArgs& g);
// j-axis pass through the per-slice operators (g.dir = 2, g.A1 = operators, g.a_bstride)
void launch_dct_axis2_op(hipStream_t s, int prec, const GemmArgs& g);
// bytes of the per-slice operators in the fragments of precision prec (0: unsupported
// length); builds them for one rho (nonzero: unsupported length)
size_t zop_bytes(int prec, int m2, int m3);
int launch_build_zop(hipStream_t s, int prec, int m2, int m3, double h2, double h3, double alpha,
                     double rho, int RT, int KS, void* out);
int dct_set_lds_limits();

}  // namespace epi
