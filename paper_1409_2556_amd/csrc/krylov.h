// Launchers of the FP64 flexible shifted Arnoldi kernels (krylov.hip).
#pragma once

#include "lt_internal.h"

namespace lt {

// Per-(rhs, shift) Givens least-squares state, pair index p = r * Ks + k, P = R * Ks pairs:
//   Rm[(col*(col+1)/2 + row) * P + p]  complex  upper-triangular factor, packed by column
//   cs[col * P + p]                    real     rotation cosines
//   sn[col * P + p]                    complex  rotation sines
//   g[row * P + p]                     complex  rotated right-hand side beta e_1
//   res[p]                             real     current relative residual
struct LSState {
    double* Rm;
    double* cs;
    double* sn;
    double* g;
    double* res;
    double* eta = nullptr;  // FOM: eta_k of the last step per pair (complex), the residual's coefficient on v_{j+1}
};

// Restarted solves (the FOM variant with an exact preconditioner): the first entry g_0 of
// every pair's least-squares right-hand side (complex per pair; null: beta[r]) and the norm
// the residuals are measured against (per right-hand side; null: beta).
struct LSStart {
    const double* g0 = nullptr;
    const double* bnorm = nullptr;
};

int reduce_blocks(int N, int R);
int launch_scatter_points(hipStream_t st, int R, int N, const int* off, const int* cell, const double* wt,
                          double* b);
int launch_norms(hipStream_t st, int N, int R, size_t vstride, const double* x, double* part, double* out,
                 const int* active);
int launch_scale_into(hipStream_t st, int N, int R, size_t instride, size_t outstride, const double* in,
                      const double* nrm, double* out);
template <typename T>
// cpnx > 0: lo is written in colour-planar order of an nx = cpnx, ny = cpny grid (the order
// of a 3D handle's FP32 V-cycle vectors)
int launch_inner_init(hipStream_t st, int N, int R, size_t qstride, double* v, double* u, size_t ustride,
                      double* rho, T* lo, const int* active, const double* scale = nullptr, int cpnx = 0,
                      int cpny = 0);
// inner_active = active; clear the refinement step counters; count[3] = j; rprev = 1
int launch_iter_begin(hipStream_t st, int R, const int* active, int* inner_active, int* count, int j,
                      double* rprev);
template <typename T>
// cp: e is read and lo written in colour-planar order
int launch_inner_update(hipStream_t st, LevelView<double> L, cdouble tau, int R, const T* e, double* u,
                        size_t ustride, const int* jcol, double* rho, T* lo, double* part, const int* inner_active,
                        int cp = 0, const int* list = nullptr);
// out[r][k] = ||b_r - (K + z_k M) U_r y_rk|| / beta_r for every right-hand side and shift,
// from K applied once to each used basis column (KU: R * max(mmax, 1) * 2N doubles,
// part: R * Ks * reduce_blocks(N, R) doubles).
// blocks per right-hand side of launch_true_residual_cols (its part holds R * Ks * this)
int true_res_blocks(int N, int R);
int launch_true_residual_cols(hipStream_t st, LevelView<double> L, int R, int Ks, int jmax, int mmax,
                              const double* U, size_t ustride, const double* Y, const int* mcols, const double* zs,
                              const double* b, const double* beta, double* KU, double* part, double* out);
// Stopping test after a refinement step; rprev [R] holds each residual norm before the
// step, est[0] receives the largest estimate of steps still needed (0 when none refine).
int launch_inner_finalize(hipStream_t st, int nb, int R, const double* part, const int* active, const double* worst,
                          double relax_tol, double tol, int inner_max, int* inner_active, int* vcycles, int* count,
                          double* rprev, int* est);
// One CGS2 step for column j: unnormalised q_{j+1} in column j + 1 of Q, Hbar column j, and
// scale[r] = 1 / ||q_{j+1}|| (applied by the next launch_inner_init).  partn: R * nb doubles.
int launch_cgs2(hipStream_t st, int N, int R, int j, const double* m, const double* U, size_t ustride, double* Q,
                size_t qstride, double* H, int hstride, size_t hrstride, double* part, int pstride, double* c1,
                double* c2, int cstride, double* scale, double* partn, const int* active);
// fom: the FOM residual (GMRES residual / cosine of the last rotation) decides convergence
// omega: [2][Ks] shift weights, the second row for right-hand sides r >= rinit (the initial head's term)
int launch_ls_update(hipStream_t st, int R, int Ks, int j, cdouble tau, const double* zs, const double* omega,
                     int rinit, double tol, bool fom, const double* H, int hstride, size_t hrstride,
                     const double* beta, const LSState& s, int* active, int* mcols, double* worst, int* conv,
                     const LSStart& start = LSStart());
int launch_gather(hipStream_t st, int R, int N, int np, const int* off, const int* cell, const double* wt,
                  const double* U, size_t ustride, int j, double* G, int jmax, const int* active);
// fom: y solves the square Hessenberg system (FOM) instead of the least-squares problem
int launch_backsolve(hipStream_t st, int R, int Ks, const int* mcols, const LSState& s, double* Y, int jmax,
                     bool fom = false);
// heads of the Rs wells (weights wq), plus the initial head's right-hand side r0 (weights w) on
// every row when r0 >= 0; phi: [max(Rs, 1)][np][ntimes]
int launch_heads(hipStream_t st, int Rs, int r0, int np, int ntimes, int nk, const double* wq, const double* w,
                 const double* G, const double* Y, const int* mcols, int jmax, double* phi, bool accumulate = false);
// Restarts: g0[r][k] = (bnorm[r], 0) for every pair
int launch_fill_g0(hipStream_t st, int R, int Ks, const double* bnorm, double* g0);
// Restarts: for right-hand sides with restart[r]: b[r] = Q[r][:, mcols[r]] (the next basis vector,
// unnormalised) and g0[r][k] = -eta[r][k]
int launch_restart_rhs(hipStream_t st, int R, int N, int Ks, const double* Q, size_t qstride, const int* mcols,
                       const int* restart, const double* eta, double* b, double* g0);
// Y[r][j][k] /= g0[r][k] / bnorm[r] (0 where that is 0), j < mcols[r]: the coefficients of a
// unit right-hand side b / ||b|| per pair, for the true residual of a restarted cycle
int launch_unscale_y(hipStream_t st, int R, int Ks, int jmax, const int* mcols, const double* g0, const double* bnorm,
                     double* Y);
// b[0:N] = m .* phi0 (the real plane of the initial head's right-hand side M phi0)
int launch_mass_rhs(hipStream_t st, int N, const double* m, const double* phi0, double* b);
int launch_form_x(hipStream_t st, int N, int R, int nc, int k0, int Ks, const double* U, size_t ustride,
                  const double* Y, int jmax, const int* mcols, double* X);
template <typename T>
int launch_net_scale(hipStream_t st, LevelView<double> L, cdouble tau, int R, T* d, const double* v, double* part,
                     const int* active);
int launch_net_guard(hipStream_t st, int R, int nb, const double* part, const int* active, int* bad, int* counts);
// mS: the storage part S V of the fine-level mass (L.m less any water-table term)
// P1 handles: the same contraction per cell of `cells` (fields on its interior vertices)
int launch_sens_p1(hipStream_t st, const lt_grid& cells, const double* kappa, const double* S, int ns, int nr,
                   int nk, int t, int ntimes, size_t N, const double* X, const double* zs, const double* wq,
                   double* JK, double* JS);
int launch_sens(hipStream_t st, LevelView<double> L, const double* kappa, const double* mS, int ns, int nr, int nk,
                int t, int ntimes, const double* X, const double* zs, const double* wq, double* JK, double* JS);

}  // namespace lt
