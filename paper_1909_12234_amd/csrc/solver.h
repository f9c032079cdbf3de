// Inexact solves A^{-1}_xi on device-layout FP64 fields.
#pragma once
#include "lqt_internal.h"

namespace lqt {

struct SolveOpts {
    int prec = LQT_F64;
    int restart = 32;
    int maxit = 100000;
    int use_net = 0;
    int max_batch = 0;
    int cgs2 = 0;
    double inner_tol = 0.0;
    int verbose = 0;
    int outer_maxit = 200;
    int graph = 0;
    int sstep = 0;
    double reliable = 0.1;  // 0: the FP64 residual at every restart
    int fallback = 0;       // 1: stalled systems continue down the fallback chain (stall.h)
    int stall_window = 2;   // FP64 residuals without a decrease that count as a stall
    int eig_degree = 128;   // Chebyshev filter degree of the eigensolvers
    double eig_xi = 0.0;    // acceptance tolerance of the coarse eigensolve (0: null_xi)
    int twogrid = 0;        // 1: two-grid right preconditioner (lqt_precond_twogrid) in FGMRES
    int tg_smooth = 4;      // its minimal-residual smoothing steps
    double tg_coarse_tol = 0.1;  // relative residual of its coarse solve
    int tg_coarse_maxit = 32;    // cap on the coarse GMRES steps
};

SolveOpts make_opts(const lqt_solver_opts* u);

// x = A^{-1}_xi b for nrhs fields; returns the number of systems that missed xi.
int solve_fields(lqt_ctx* c, const double2* b, double2* x, int nrhs, double xi, const SolveOpts& o,
                 lqt_solve_stats* stats);

}  // namespace lqt
