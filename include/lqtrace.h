/*
 * lqtrace: deflated Hutchinson estimation of trace(A^{-1}) for the Wilson-Dirac
 * operator on one AMD Instinct MI355X (gfx950).
 *
 * Method: E. Romero, A. Stathopoulos, K. Orginos, "Multigrid deflation for Lattice
 * QCD", arXiv:1909.12234.  Section 1 defines the Hutchinson estimator (Eq. 1), its
 * variance (Eq. 2) and the inexact solve A^{-1}_xi; Section 2.1 the K-weighted oblique
 * projector and its trace identity; Section 2.2 the a-posteriori choice of the deflation
 * rank; Algorithm 1 (orthogonal projector of approximate singular vectors) and
 * Algorithm 2 (oblique projector from the coarse operator of a multigrid prolongator).
 *
 * Operator:  (A psi)(x) = (4+m) psi(x)
 *            - 1/2 sum_mu [ (1-g_mu) U_mu(x) psi(x+mu) + (1+g_mu) U_mu(x-mu)^+ psi(x-mu) ]
 * DeGrand-Rossi gamma matrices, g5 = diag(1,1,-1,-1); periodic boundaries, with an extra
 * -1 on hops across the time boundary when the context is created antiperiodic.
 *
 * Canonical host-visible layouts (x runs fastest, mu = 0..3 <-> x, y, z, t):
 *   links   [t][z][y][x][mu][a][b]          complex128, (re, im) interleaved
 *   spinor  [rhs][t][z][y][x][spin][colour] complex128 (complex64 for LQT_F32 in lqt_apply)
 * i.e. spinor component index i = 12*site + 3*spin + colour, site = x + Lx*(y + Ly*(z + Lz*t)).
 *
 * Conventions for every call:
 *  - Return LQT_OK (0) on success or a negative LQT_E* code; the message is kept in the
 *    context (lqt_last_error).  No C++ exception or abort crosses this boundary.
 *  - Pointers named d_* are device pointers (HBM of the context's device); h_* are host.
 *    Buffers are owned by the caller and never retained after the call returns.
 *  - All device work is ordered on the context's HIP stream.  Calls that return host
 *    values synchronise that stream before returning.
 *  - Calls on one context are not thread-safe; use one context per host thread.
 */
#ifndef LQTRACE_H
#define LQTRACE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lqt_ctx lqt_ctx;
typedef struct lqt_basis lqt_basis;

/* ---- error codes ------------------------------------------------------------------ */
#define LQT_OK 0
#define LQT_EINVAL -1      /* bad argument (null pointer, size, enum)                  */
#define LQT_ENOMEM -2      /* device or host allocation failed                         */
#define LQT_EHIP -3        /* a HIP runtime call failed                                */
#define LQT_ENOTCONV -4    /* a solve did not reach its tolerance; outputs still filled */
#define LQT_ENOTUNITARY -5 /* a gauge link is not special unitary to 1e-10             */
#define LQT_ESTATE -6      /* call out of order (e.g. no gauge field set)              */
#define LQT_ENAN -7        /* a NaN or Inf appeared in an input or a residual          */

/* ---- operators (lqt_apply) ----------------------------------------------------------- */
#define LQT_A 0     /* A                                                                  */
#define LQT_A_DAG 1 /* A^+ (the adjoint: forward and backward spin projectors swap)       */
#define LQT_A_G5 2  /* A g5 : the Hermitian, maximally indefinite operator of Section 3    */
#define LQT_G5_A 3  /* g5 A                                                               */

/* ---- storage precisions ------------------------------------------------------------ */
#define LQT_F64 0
#define LQT_F32 1
#define LQT_F16 2
#define LQT_BF16 3

/* ---- projectors (lqt_trace) ---------------------------------------------------------- */
#define LQT_OBLIQUE_G5 0 /* K = g5 oblique projector of Section 2.1 (Algorithm 2 form)  */
#define LQT_ORTH 1       /* orthogonal projector U U^+ of Algorithm 1                    */

/* Solver options.  Zero-initialised fields take the defaults in brackets. */
typedef struct {
    int inner_prec;  /* storage of links and Krylov vectors in inner cycles [LQT_F64]   */
    int restart;     /* GMRES restart length m, 1..64 [32]                               */
    int maxit;       /* cap on Arnoldi steps per right-hand side [100000]               */
    int use_net;     /* 1: learned preconditioner (lqt_precond_set) inside FGMRES      */
    int max_batch;   /* right-hand sides solved together, 0 = all [0]                    */
    int cgs2;        /* 1: re-orthogonalise each Arnoldi step (CGS2) [0: single CGS]     */
    double inner_tol;/* relative reduction asked of one inner cycle [0: one full cycle]  */
    int verbose;     /* 1: progress lines on stderr from long calls (eigensolver, setup) */
    int outer_maxit; /* cap on eigensolver iterations (lqt_basis_eig / the coarse
                        eigensolve of lqt_basis_prolongator) [200]                       */
    int graph;       /* 1: capture each inner cycle (all m Arnoldi steps, the small
                        Hessenberg updates and the solution update) in a HIP graph once
                        per batch size and replay it; cycles always run all m steps (the
                        steps after a system has converged change nothing), so results
                        are bit-identical to graph = 0 [0]                               */
    int sstep;       /* 1: s-step cycles (restart <= 15 with FP16/BF16 storage, <= 8 with
                        FP32/FP64; no use_net): the cycle's basis is
                        k_{i+1} = (A - theta) k_i / 2 with theta = 4 + m (powers of the
                        hopping term, no Gram-Schmidt between the operator applications),
                        made orthonormal afterwards through one Gram pass and an FP64
                        Cholesky; the same Krylov space and minimisation as GMRES(m) [0]  */
    double reliable; /* s-step cycles on one lattice: the FP64 residual b - A x is formed
                        only when the residual carried in the basis (r - A K beta, with
                        A K = K T from the basis recurrence, written as the next start
                        vector by the solution update's pass) has fallen below `reliable`
                        times the last formed one, meets the tolerance, or is not finite;
                        other cycles start from the carried residual (reliable updates).
                        Values in (0, 1); negative: form it at every restart [0.1]      */
    int fallback;    /* 1: a system whose solve stalls continues from its current x with
                        more robust settings, dropping in turn the network preconditioner,
                        the s-step cycles, 16-bit storage (to FP32) and reduced storage (to
                        FP64 GMRES); maxit applies to each level.  A solve has stalled when
                        stall_window FP64 residuals in a row fail to fall 0.1 % below the
                        smallest before them, when a cycle can take no step (an s-step
                        Gram matrix of rank one: the start vector is an eigenvector of A),
                        or when its residual is not finite (that level restarts from x = 0).
                        0: no fallback; a cycle that takes no step ends its system as failed
                        and other systems run to maxit [0]                                 */
    int stall_window;/* FP64 residuals without a 0.1 % decrease that count as a stall [2]  */
    int eig_degree;  /* degree in H^2 of the Chebyshev filter of the eigensolvers
                        (lqt_basis_eig, the coarse eigensolve of lqt_basis_prolongator) [128] */
    double eig_xi;   /* acceptance tolerance of the coarse eigensolve of
                        lqt_basis_prolongator [0: null_xi]                                */
    int twogrid;     /* 1: the two-grid preconditioner of lqt_precond_twogrid as the right
                        preconditioner of FGMRES (not with use_net, sstep or graph) [0]   */
    int tg_smooth;   /* its minimal-residual smoothing steps on A [4; negative: none]    */
    double tg_coarse_tol; /* relative residual of its coarse GMRES solve [0.1]          */
    int tg_coarse_maxit;  /* cap on the coarse GMRES steps per application [32]         */
} lqt_solver_opts;

/* Per right-hand side solve statistics. */
typedef struct {
    int converged; /* 1 if the FP64 true residual ||b - A x|| <= xi ||b||                  */
    int iters;     /* Arnoldi steps (operator applications inside cycles)               */
    int cycles;    /* restart cycles = FP64 residual recomputations                      */
    double relres; /* final FP64 true relative residual                                  */
    int fallback;  /* fallback level the system finished at (0: the settings asked for;
                      each level drops one of net, s-step, 16-bit, reduced storage)       */
} lqt_solve_stats;

/* Trace estimate, Section 1 and Algorithms 1/2.  All values are FP64. */
typedef struct {
    double trace_re, trace_im; /* t0 + mean_j t_j                                        */
    double t0_re, t0_im;       /* deterministic part (deflated subspace)                 */
    double var_sample;         /* sum_j |t_j - mean|^2 / (s-1): one-probe variance (Eq. 2) */
    double var_mean;           /* var_sample / s: variance of the estimate               */
    double jackknife_err;      /* leave-one-out jackknife standard error of the mean     */
    double var_re_only;        /* one-probe variance of Re t_j alone                     */
    int nsolves;               /* probe solves performed                                  */
    int nfailed;               /* probe solves that missed the tolerance                  */
    long long iters_total;     /* Arnoldi steps summed over the probe solves             */
    double seconds_solve;      /* device time of the probe solves                         */
    double seconds_setup;      /* device time of probe generation and projections         */
    int nfallback;             /* probe solves that finished at a fallback level (opts->fallback) */
} lqt_trace_result;

/* Options of the learned-preconditioner training (lqt_precond_train). */
typedef struct {
    int epochs;        /* passes over the generated pairs [4]                            */
    double lr;         /* Adam learning rate [1e-3]                                      */
    int batch;         /* pairs per optimiser step [4]                                   */
    double pair_xi;    /* 0: errors e are Gaussian; in (0,1): e = A^{-1}_{pair_xi} g, the  */
                       /* solver's output (FP32 inner GMRES) on a Gaussian g [0]          */
    int verbose;       /* 1: one progress line per epoch on stderr [0]                   */
} lqt_train_opts;

/* ---- context ---------------------------------------------------------------------- */

/* Create a context for an Lx x Ly x Lz x Lt lattice (dims[0..3], each >= 2 and even for
 * Lt when t_antiperiodic is used is not required) with bare mass m, bound to hip_stream
 * (a hipStream_t; NULL = the null stream) on the current HIP device.  Operator as in the
 * header comment.  On failure *ctx is NULL and the code is returned. */
int lqt_create(lqt_ctx **ctx, const int dims[4], double mass, int t_antiperiodic,
               void *hip_stream);

/* Create a context for nlat (1..8) lattices solved together (dims[4k..4k+3] = Lx, Ly, Lz, Lt
 * of lattice k, masses[k] its bare mass; all other arguments as lqt_create).  The operator
 * is block diagonal over the lattices and every kernel launch covers all of them (a block
 * of sites never straddles two lattices).  Fields and links in the canonical layout are the
 * lattices' canonical arrays one after the other (per right-hand side for fields).  Probes
 * restrict to each lattice as they would for a context of that lattice alone; a solve stops
 * when every lattice block meets ||b_k - A_k x_k|| <= xi ||b_k||.  lqt_trace_lattices gives
 * one estimate per lattice.  Deflation bases, the prolongator and the network preconditioner
 * need a single-lattice context (LQT_EINVAL).  lqt_set_mass sets every lattice's mass. */
int lqt_create_multi(lqt_ctx **ctx, int nlat, const int *dims, const double *masses,
                     int t_antiperiodic, void *hip_stream);

/* Upload the gauge field (canonical layout, V*4*9 complex128 = 144*V doubles), from host
 * memory (on_device = 0) or device memory (1).  The field is copied into the device
 * layouts of every precision, with the antiperiodic sign folded into the links of the
 * last time slice.  Rejects the field with LQT_ENOTUNITARY when any link has
 * max|U^+U - 1| > 1e-10 or |det U - 1| > 1e-10, and with LQT_ENAN on non-finite values. */
int lqt_set_gauge(lqt_ctx *ctx, const double *links, int on_device);

/* Change the bare mass m of the operator. */
int lqt_set_mass(lqt_ctx *ctx, double mass);

/* out = op(in) for nrhs spinor fields in the canonical layout, device pointers.
 * prec LQT_F64: complex128 in/out, computed in FP64.  LQT_F32: complex64 in/out with FP32
 * links and FP32 arithmetic.  LQT_F16 / LQT_BF16: complex64 in/out, the fields are
 * rounded to 16-bit storage (links and input spinor) and accumulated in FP32.
 * in and out must not overlap. */
int lqt_apply(lqt_ctx *ctx, int op, int prec, const void *d_in, void *d_out, int nrhs);

/* Solve A x_r = b_r for r < nrhs (canonical complex128 device arrays), x0 = 0, until the
 * FP64 true residual ||b - A x|| <= xi ||b|| (the inexact solve A^{-1}_xi of Section 1).
 * Restarted GMRES(m) (FGMRES(m) with use_net) whose inner cycles run in opts->inner_prec
 * storage with FP32 accumulation and whose restarts recompute the residual in FP64
 * (defect correction).  stats (may be NULL) receives nrhs entries.  Returns LQT_ENOTCONV
 * if any system missed the tolerance within opts->maxit steps (x and stats still filled). */
int lqt_solve(lqt_ctx *ctx, const double *d_b, double *d_x, int nrhs, double xi,
              const lqt_solver_opts *opts, lqt_solve_stats *stats);

/* ---- deflation bases ---------------------------------------------------------------- */

/* Algorithm 1, first step: the k eigenpairs of the Hermitian operator H = A g5 with the
 * smallest |lambda| (the largest of H^{-1} = g5 A^{-1}; its eigenvectors are left singular
 * vectors of A).  Chebyshev-filtered subspace iteration on H^2 with a block of 2k vectors
 * (the filter, of degree at most opts->eig_degree in H^2, runs with FP32 links and vectors when
 * xi >= 1e-5, FP64 otherwise, one multi-RHS operator launch per application; at most
 * opts->outer_maxit filtered iterations,
 * default 200), harmonic Rayleigh-Ritz extraction with target 0 and a final Rayleigh-Ritz of
 * H in the span of the k accepted vectors (FP64 Gram matrices and eigenproblems).  A pair
 * (theta, q) is accepted when ||H q - theta q|| <= xi |theta|, which implies the convergence
 * test of the paper's Table 1, ||H^{-1} q - q/theta|| <= xi ||H^{-1}||.  Returns
 * LQT_ENOTCONV (with the basis in *out) if not all k pairs pass.
 * tau: the shift of Algorithm 1, whose eigensolve targets g5 (A + i tau g5)^{-1} =
 * (A g5 + i tau)^{-1}: its eigenvectors are those of A g5 and its largest magnitudes
 * 1/|lambda + i tau| = 1/sqrt(lambda^2 + tau^2) order them as the smallest |lambda|, so the
 * basis and the returned lambda (eigenvalues of A g5) do not depend on tau.  The shift only
 * conditions the inexact inversions of an inverse-based eigensolver; the Chebyshev filter
 * applies H itself and takes no inverse, so tau (any finite value) changes nothing here.
 * *out receives a basis owned by the caller (free with lqt_basis_free); the context
 * must outlive it. */
int lqt_basis_eig(lqt_ctx *ctx, int k, double xi, double tau, const lqt_solver_opts *opts,
                  lqt_basis **out);

/* Algorithm 2, first three steps: the multigrid prolongator W built from nv near-null
 * vectors (approximate solutions of A y = 0 from Gaussian starts y0, Section 2: y = y0 - e
 * with A e = A y0 solved to null_xi or null_maxit Arnoldi steps), blocked on
 * block[0..3]-site aggregates and split by chirality (spins {0,1} and {2,3}), orthonormalised
 * per (aggregate, chirality) by two passes of modified Gram-Schmidt; then the k eigenvectors
 * of the Hermitian coarse operator g5^W W^+ A W with the smallest |lambda| (the eigensolver
 * of lqt_basis_eig in FP64 on the coarse vectors, accepted at opts->eig_xi, default null_xi),
 * rotated so that U^+ g5^W W^+ A W U is diagonal.  The coarse vectors U_c are kept; the
 * fine basis is U = W U_c.  Block extents must divide the lattice; 1 <= nv <= 64; k may be
 * 0 (prolongator only).  Returns LQT_ENOTCONV (with the basis in *out) if the coarse
 * eigenpairs did not all pass. */
int lqt_basis_prolongator(lqt_ctx *ctx, const int block[4], int nv, int k, double null_xi,
                          int null_maxit, const lqt_solver_opts *opts, lqt_basis **out);

/* Algorithm 2 with two multigrid levels (Table 2: the coarse lattice of lqt_basis_prolongator
 * blocked again, Table 3's two-level deflation space).  Level 1 is built as in
 * lqt_basis_prolongator (nv <= 32, so its coarse operator D_c = W^+ A W is the explicit
 * stencil).  Level 2: nv2 near-null vectors of D_c (coarse GMRES on Ae = Ay0 to null_xi or
 * null_maxit steps), blocked on block2 blocks of the coarse lattice and split by chirality
 * (g5^W W2 = W2 g5^{W2}), orthonormalised: W2[A][c][v2][ls * nv + v1] with ls the coarse site
 * inside the level-2 block (x fastest).  The level-2 operator D_cc = W2^+ D_c W2 is a 9-point
 * block stencil (2 nv2 <= 64).  Its k smallest-|lambda| eigenvectors U2 of g5^{W2} D_cc
 * (the coarse eigensolve of lqt_basis_eig, accepted at opts->eig_xi, default null_xi) give
 * the coarse vectors W2 U2 of the level-1 space, which are rotated as in
 * lqt_basis_prolongator: the deflation space is X = W W2 U2.  block2 must divide the coarse
 * lattice; 1 <= nv2 <= 32; 0 <= k <= nc2 / 8 with nc2 = 2 nv2 (coarse sites / level-2 block
 * sites).  Returns LQT_ENOTCONV (with the basis in *out) if the level-2 pairs did not all
 * pass. */
int lqt_basis_prolongator2(lqt_ctx *ctx, const int block[4], int nv, const int block2[4], int nv2,
                           int k, double null_xi, int null_maxit, const lqt_solver_opts *opts,
                           lqt_basis **out);

/* The same from caller-supplied W (as lqt_basis_prolongator_from), W2 (device, the layout
 * above) and k level-2 coarse vectors (device, k x nc2, may be NULL with k = 0). */
int lqt_basis_prolongator2_from(lqt_ctx *ctx, const int block[4], int nv, const double *d_w,
                                const int block2[4], int nv2, const double *d_w2,
                                const double *d_coarse2, int k, lqt_basis **out);

/* D_cc (herm: g5^{W2} D_cc) applied to nrhs level-2 coarse vectors (device, nc2 each). */
int lqt_coarse2_apply(lqt_ctx *ctx, lqt_basis *basis, const double *d_in, double *d_out, int nrhs,
                      int herm);

/* Copy W2 of a two-level basis to d_w2 (may be NULL) and report nc2. */
int lqt_prolongator2_get(const lqt_basis *basis, double *d_w2, long long *nc2);

/* Build a basis from k caller-supplied fine vectors (canonical complex128, device).  The
 * vectors X are used as given for the K = g5 oblique projector (Section 2.1): the library
 * forms M = X^+ g5 A X, diagonalises it and rotates U = X U_hat.  For LQT_ORTH the columns
 * are orthonormalised first. */
int lqt_basis_from_vectors(lqt_ctx *ctx, const double *d_vectors, int k, lqt_basis **out);

/* Largest singular value of A (the conditioning of the solves, Section 1: the solution
 * error of A^{-1}_xi is bounded by kappa(A) xi): square root of the largest Ritz value of
 * 40 Lanczos steps on A A^+ = (A g5)^2, FP64.  Single-lattice contexts. */
int lqt_sigma_max(lqt_ctx *ctx, double *h_sigma);

/* Eigenvalues lambda_i of U^+ g5 A U (ascending |lambda|) and the rank k.  lambda may be
 * NULL to query k; otherwise it must hold 2*k doubles (complex). */
int lqt_basis_eigenvalues(const lqt_basis *basis, double *h_lambda, int *k);

/* Copy the k fine basis vectors U (canonical complex128 layout) to device memory d_out;
 * for a prolongator basis U = W U_c is formed on the fly. */
int lqt_basis_vectors(const lqt_basis *basis, double *d_out);

void lqt_basis_free(lqt_basis *basis);

/* ---- learned preconditioner ------------------------------------------------------- */

/* Set the weights of the 4-layer gauge-equivariant parallel-transport network used as a
 * right preconditioner in FGMRES (features 4 -> 8 -> 8 -> 8 -> 4, i.e. 12 -> 24 -> 24 ->
 * 24 -> 12 complex channels, each feature a colour 3-vector; the 4 input/output features
 * are the 4 spin components of a spinor).  Layer l maps
 *   out_f(x) = sum_{p=0..8} sum_g W_l[p][f][g] (T_p v_g)(x),  T_0 = 1,
 *   T_{1+2mu} v(x) = U_mu(x) v(x+mu),  T_{2+2mu} v(x) = U_mu(x-mu)^+ v(x-mu)
 * (links with the antiperiodic sign), linear, no bias.  Weights concatenated layer by layer,
 * W_l[p][f][g] row-major, as complex FP32 (re, im): 2*9*(32+64+64+32) = 3456 floats
 * (nbytes = 13824); the kernels use them rounded to BF16, with FP32 arithmetic.  Host
 * pointer. */
int lqt_precond_set(lqt_ctx *ctx, const void *h_weights, size_t nbytes);

/* Copy the current weights (complex FP32 in the order above) to the host. */
int lqt_precond_get(lqt_ctx *ctx, void *h_weights, size_t nbytes);

/* Apply the network: out = M(in), canonical complex128 device arrays, nrhs fields. */
int lqt_precond_apply(lqt_ctx *ctx, const double *d_in, double *d_out, int nrhs);

/* Loss and gradient of the network on caller-supplied errors: for the npairs fields e_q
 * (canonical complex128, device) the library forms r_q = A e_q and returns
 *   *h_loss = (1/npairs) sum_q ||M r_q - e_q||^2 / ||e_q||^2
 * and h_grad[2*i], h_grad[2*i+1] = re, im of dL/dconj(W_i) (2 * 1728 doubles, the weight
 * order above; d/dRe W_i = 2 re, d/dIm W_i = 2 im), by back-propagation through the
 * adjoint layers (the adjoint of T_{+mu} is T_{-mu}; weights conjugate-transposed).  Uses
 * the FP32 master weights (not the BF16 copy), FP32 arithmetic and FP64-stored activations. */
int lqt_precond_loss_grad(lqt_ctx *ctx, const double *d_e, int npairs, double *h_loss,
                          double *h_grad);

/* Train the network with Adam (on the real and imaginary parts of every weight) on npairs
 * pairs (r, e) with A e = r: e are drawn on the device from seed, either Gaussian or the
 * solver's own approximate solutions of Gaussian right-hand sides (opts->pair_xi), and kept
 * resident (npairs * 12V complex128; LQT_ENOMEM beyond half the free device memory); r = A e;
 * loss and gradient as in lqt_precond_loss_grad over opts->batch pairs per step, the same
 * pairs every epoch.  Starts from the current weights, else from the identity scaled by
 * |4+m|^{-1/4} per layer (M = 1/(4+m), point Jacobi).  *h_final_loss (may be NULL) receives
 * the mean loss of the last epoch (accumulated over its steps). */
int lqt_precond_train(lqt_ctx *ctx, int npairs, uint64_t seed, const lqt_train_opts *opts,
                      double *h_final_loss);

/* Two-grid preconditioner (Section 2, the two-grid method) from a prolongator basis of this
 * context (lqt_basis_prolongator / _from; its coarse vectors are not used): one application
 * to a residual v, from x = 0, is the coarse grid correction x_c = W D_c^{-1} W^+ v with the
 * explicit coarse operator D_c = W^+ A W (built here if missing), solved by batched FP64
 * GMRES(16) to opts->tg_coarse_tol (at most tg_coarse_maxit steps), followed by
 * opts->tg_smooth minimal-residual steps on A (s = v - A x_c; p = A s, a = p^+ s / p^+ p,
 * x += a s, s -= a p).  solver option twogrid = 1 puts it inside FGMRES as the right
 * preconditioner (the coarse solve and the smoothing depend on v, which flexible GMRES
 * allows).  The basis stays owned by the caller and must outlive its use; basis = NULL
 * clears it (lqt_basis_free of the set basis clears it too).  Single-lattice contexts. */
int lqt_precond_twogrid(lqt_ctx *ctx, lqt_basis *basis);

/* One application of the two-grid preconditioner to nrhs canonical complex128 device
 * fields (the options' tg_* fields), for verification and measurement. */
int lqt_precond_twogrid_apply(lqt_ctx *ctx, const double *d_in, double *d_out, int nrhs,
                              const lqt_solver_opts *opts);

/* ---- trace estimation -------------------------------------------------------------- */

/* Deflated Hutchinson estimate of trace(A^{-1}) (Eq. 1 with the split of Section 2):
 * nprobes real Rademacher probes z_j (entries 1 - 2*bit63(h(seed ^ h(j ^ h(i)))) with h
 * the SplitMix64 output function), y_j = A^{-1}_xi z_j, and
 *   LQT_OBLIQUE_G5: t_j = z_j^T y_j - (z_j^T U) Lambda^{-1} (U^+ g5 z_j),
 *                   t0 = sum_i lambda_i^{-1} u_i^+ g5 u_i                  (Section 2.1)
 *   LQT_ORTH:       y_j = A^{-1}_xi (1 - U U^+) z_j, t_j = z_j^T y_j,
 *                   t0 = sum_i u_i^+ A^{-1}_xi u_i                         (Algorithm 1)
 * The orthogonal projector takes an lqt_basis_eig basis (U its orthonormal eigenvectors) or
 * a prolongator basis with orthonormal coarse vectors (U = W U_c, applied as restriction,
 * coarse products and prolongation; LQT_EINVAL if max |U_c^+ U_c - I| > 1e-10): its
 * variance is the rough lower bound of Section 2.1 for any projector onto the same span.
 * basis = NULL gives the undeflated estimator.  rank_curve (may be NULL) receives
 * (k+1) x 3 doubles: for each rank k' = 0..k the estimate (re), its one-probe variance
 * and the jackknife error, recomputed from the stored k x s products (Section 2.2;
 * oblique projector only, else zeros).  samples (may be NULL) receives the nprobes
 * complex samples t_j (2*nprobes doubles). */
int lqt_trace(lqt_ctx *ctx, const lqt_basis *basis, int projector, int nprobes, uint64_t seed,
              double xi, const lqt_solver_opts *opts, lqt_trace_result *out,
              double *h_rank_curve, double *h_samples);

/* lqt_trace with the partition basis H of Algorithms 1 and 2 (Section 1: spin-colour
 * dilution and hierarchical probing; lqt_trace is hp_vectors = 1, dilute = 0).  Draw j
 * solves the q = hp_vectors * (dilute ? 12 : 1) real vectors
 *   v_{j,m,c} = z_j (.) h_m (.) e_c,   m < hp_vectors, c < 12 (dilute) or e_c = 1,
 * z_j the Rademacher probe of lqt_trace, e_c the indicator of spin-colour component
 * c = 3 spin + colour at every site, and h_m(x) = (-1)^{sum over the set bits beta of m of
 * f_beta(x)} with the nested bit functions of level l = beta / 4 on the coordinate bits
 * x_l = (x >> l) & 1:  f_{4l} = x_l + y_l + z_l + t_l (mod 2), f_{4l+1} = x_l,
 * f_{4l+2} = y_l, f_{4l+3} = z_l.  At the closing colours hp_vectors = 2^{4i} the probing
 * separates every pair of sites that differ modulo 2^i in some direction (hp_vectors = 2:
 * the red-black partition).  The sample of draw j is
 *   t_j = (1/hp_vectors) sum_{m,c} [v^T y_v - (v^T U) Lambda^{-1} (U^+ g5 v)]   (oblique)
 * with y_v = A^{-1}_xi v (the orthogonal projector solves on (1 - U U^+) v instead), an
 * unbiased estimate of the trace of the deflated inverse; t0, the statistics over the
 * nprobes draws and the rank curve are as in lqt_trace.  nsolves and nfailed count the
 * nprobes * q solves.  hp_vectors must be a power of two (at most 2^20), and every
 * extent a multiple of 2^{l+1} for the highest level l in use (LQT_EINVAL otherwise);
 * single-lattice contexts only. */
int lqt_trace_probing(lqt_ctx *ctx, const lqt_basis *basis, int projector, int nprobes,
                      uint64_t seed, double xi, int hp_vectors, int dilute,
                      const lqt_solver_opts *opts, lqt_trace_result *out, double *h_rank_curve,
                      double *h_samples);

/* Result of lqt_trace_tsm. */
typedef struct {
    double trace_re, trace_im;   /* main estimate + mean correction                          */
    double err;                  /* sqrt(var_mean of the main draws + var(d) / ncorr)        */
    double corr_re, corr_im;     /* mean correction: (1/ncorr) sum_j d_j                     */
    double corr_var_sample;      /* one-draw variance of the d_j ((n-1) denominator)         */
    double corr_jackknife_err;   /* jackknife error of the mean correction                   */
    long long nsolves_loose, nsolves_tight, iters_loose, iters_tight;
    int nfailed;                 /* solves of any of the three runs that missed their xi     */
} lqt_tsm_result;

/* Truncated Solver Method (Section 1): the samples of solves stopped at xi_loose are biased
 * by the trace of A^{-1} - A^{-1}_xi_loose, which an independent probe set estimates.  The
 * main run is lqt_trace_probing over nprobes draws of seed at xi_loose (into *main, t0
 * included); the correction draws j < ncorr of seed_corr are solved at xi_loose and at
 * xi_tight, and d_j = t_j(xi_tight) - t_j(xi_loose) (the deflation terms of a draw do not
 * depend on the solves and cancel).  out->trace = main + mean(d); out->err combines the two
 * independent standard errors.  corr_samples (may be NULL): 2*ncorr doubles, the d_j.
 * LQT_EINVAL unless ncorr >= 2, seed_corr != seed and 0 < xi_tight < xi_loose; LQT_ENOTCONV
 * (results filled) when a solve missed its tolerance. */
int lqt_trace_tsm(lqt_ctx *ctx, const lqt_basis *basis, int projector, int nprobes, uint64_t seed,
                  double xi_loose, int ncorr, uint64_t seed_corr, double xi_tight, int hp_vectors,
                  int dilute, const lqt_solver_opts *opts, lqt_trace_result *main,
                  lqt_tsm_result *out, double *h_corr_samples);

/* Undeflated Hutchinson estimates of trace(A_k^{-1}), one per lattice of the context (Eq. 1;
 * the same probes and solves as lqt_trace, the samples split by lattice): res receives nlat
 * results, samples (may be NULL) 2*nlat*nprobes doubles [lattice][probe] (re, im).  nsolves,
 * nfailed and iters_total count the joint solves of all lattices.  Returns LQT_ENOTCONV as
 * lqt_trace. */
int lqt_trace_lattices(lqt_ctx *ctx, int nprobes, uint64_t seed, double xi,
                       const lqt_solver_opts *opts, lqt_trace_result *res, double *h_samples);

/* ---- building blocks (exposed for verification and measurement) ------------------- */

/* Write the real Rademacher probes j0 .. j0+nprobes-1 as canonical complex128 fields. */
int lqt_probes(lqt_ctx *ctx, uint64_t seed, long long j0, int nprobes, double *d_out);

/* Write the partition probe vectors p0 .. p0+nvec-1 of lqt_trace_probing (vector
 * p = j q + m nd + c of draw j, q = hp_vectors nd, nd = 12 with dilution, else 1) as
 * canonical complex128 fields (device).  hp_vectors, dilute and the lattice must be valid as
 * for lqt_trace_probing (LQT_EINVAL otherwise); single-lattice contexts. */
int lqt_partition_probes(lqt_ctx *ctx, uint64_t seed, long long p0, int nvec, int hp_vectors,
                         int dilute, double *d_out);

/* C = X^+ Y for ka fields X and kb fields Y (canonical complex128, device); C is ka x kb
 * complex, row-major, written to host memory.  FP64 MFMA. */
int lqt_gram(lqt_ctx *ctx, const double *d_x, int ka, const double *d_y, int kb, double *h_c);

/* C = X^+ Y as lqt_gram, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the call allocates
 * nothing.  Its workspace (the contraction's chunk partials and the ka x kb result) is a
 * static device array of 32 MiB that each GPU holds from the library's first context on it
 * until the process ends; ka * kb may be at most 1048576 (LQT_EINVAL beyond).  d_x, d_y:
 * canonical complex128 device arrays; h_c: host, ka x kb complex row-major.  Results agree
 * with lqt_gram up to the order of the FP64 sums.  Every call on a GPU shares that GPU's
 * array (it keeps the last call's contents; nothing in it needs clearing), so calls that
 * overlap on one GPU, from several contexts or threads, race and must be serialised by the
 * caller. */
int lqt_gram_noalloc(lqt_ctx *ctx, const double *d_x, int ka, const double *d_y, int kb,
                     double *h_c);

/* C_up = X^+ P_+ Z and C_dn = X^+ P_- Z for the Rademacher probes Z (generated on the
 * fly, j0 .. j0+s-1) where P_+/- keep spins {0,1} / {2,3}: so X^+ Z = C_up + C_dn and
 * X^+ g5 Z = C_up - C_dn.  Outputs ka x s complex row-major on the host.  FP64 MFMA. */
int lqt_project_probes(lqt_ctx *ctx, const double *d_x, int ka, uint64_t seed, long long j0,
                       int s, double *h_cup, double *h_cdn);

/* Y = beta*Y + X C for ka fields X, a ka x kb complex matrix C (row-major, host) and kb
 * output fields Y (device, canonical complex128).  beta is 0 or 1 or -1 (alpha = 1 or
 * -1 via sign).  FP64 MFMA. */
int lqt_combine(lqt_ctx *ctx, const double *d_x, int ka, const double *h_c, int kb, double beta,
                double alpha, double *d_y);

/* Prolongator blocks of a basis built by lqt_basis_prolongator: restrict (c = W^+ y) and
 * prolongate (y = W c) nrhs fields.  Coarse vectors are complex128 with layout
 * [rhs][aggregate][chirality][nv]; fine fields canonical complex128; device pointers. */
int lqt_restrict(lqt_ctx *ctx, const lqt_basis *basis, const double *d_fine, double *d_coarse,
                 int nrhs);
int lqt_prolong(lqt_ctx *ctx, const lqt_basis *basis, const double *d_coarse, double *d_fine,
                int nrhs);
/* Copy W (layout [aggregate][chirality][nv][site_in_block][spin2][colour], complex128,
 * site_in_block with x fastest, spin2 = spin - 2*chirality) to device memory.  Returns the
 * coarse dimension in *nc. */
int lqt_prolongator_get(const lqt_basis *basis, double *d_w, long long *nc);
/* The coarse operator of a prolongator basis as an explicit 9-point stencil of 2nv x 2nv
 * complex blocks (each aggregate couples to itself and to the aggregates one block away in
 * +-mu, because A couples nearest neighbours): out = W^+ A W in (herm = 0) or
 * g5^W W^+ A W in (herm = 1), nrhs coarse vectors [rhs][aggregate][chirality][nv], device
 * pointers.  The stencil (FP64, nagg * 9 * (2nv)^2 complex) is built from W and the links on
 * the first call and kept with the basis; nv <= 32.  lqt_basis_prolongator builds it before
 * the coarse eigensolve. */
int lqt_coarse_apply(lqt_ctx *ctx, lqt_basis *basis, const double *d_in, double *d_out, int nrhs,
                     int herm);

/* Install a prolongator from caller-supplied W in the layout above (device), and optionally
 * k coarse vectors U_bar (device, k x nc, may be NULL when k = 0): the library then forms
 * M = U_bar^+ g5^W W^+ A W U_bar, diagonalises it and keeps U_c = U_bar U_hat (Algorithm 2,
 * third step), giving a basis usable by lqt_trace.  W is used as given (its blocks are
 * expected orthonormal). */
int lqt_basis_prolongator_from(lqt_ctx *ctx, const int block[4], int nv, const double *d_w,
                               const double *d_coarse, int k, lqt_basis **out);

/* Autotuner: time the candidate dslash tilings for (prec, nrhs) now and cache the choice in
 * the context.  Candidates: the vector-ALU kernel (kind 0: right-hand sides per thread 1/2/4,
 * block 64/128/256 threads, block order site-block major or chunks of site blocks swept per
 * right-hand-side group); for FP16/BF16 storage the matrix-core kernel (kind 1: 1 or 2
 * groups of 4 right-hand sides per lane, 16 sites per wave, same blocks and orders); for FP16
 * storage the vector kernel with packed half-precision arithmetic (kind 2: the half spinors
 * rounded to FP16, link products as FP16 dot products accumulated in FP32; tiles as kind 0)
 * and the same arithmetic with each 256-site block's links staged in LDS once and shared by
 * the 8 right-hand-side groups the block loops over (kind 3, 256-thread blocks only), and the
 * streaming kernel whose blocks walk every time slice with the spinors of three slices in
 * registers (kind 4: FP16, one lattice whose time slices hold a multiple of 256 sites, one
 * right-hand side per thread, 256-thread blocks).
 * Block orders: chunks of 16, 64, 256 or 1024 site blocks (1024: the whole of most
 * lattices, right-hand-side groups outermost).  *ms
 * receives the best time and tile[0..3] the chosen (rhs per thread or groups per lane, block,
 * chunk, kind); either may be NULL.  Also tunes the FP64 residual of the solvers' restarts
 * (r = b - A x with its norms; 1 or 2 right-hand sides per thread, block order) for nrhs
 * right-hand sides, used for every batch size until tuned again. */
int lqt_tune(lqt_ctx *ctx, int prec, int nrhs, double *ms, int *tile);

/* Set the dslash tiling used for (prec, nrhs) without timing: tile[0..3] as lqt_tune reports
 * it (kind 1 only for LQT_F16 and LQT_BF16, with 1 or 2 groups per lane; kinds 2, 3 and 4
 * only for LQT_F16, kinds 3 and 4 only with 256-thread blocks, kind 4 with one right-hand
 * side per thread).  LQT_EINVAL for a tiling the kernels do not have. */
int lqt_set_tile(lqt_ctx *ctx, int prec, int nrhs, const int *tile);

/* Kernel timers: HIP event pairs recorded around the library's launches on the context
 * stream, summed per kernel family: 0 Wilson operator of the inner cycles, 1 CGS dot
 * pass, 2 CGS update pass, 3 FP64 residual (defect correction), 4 other Krylov kernels,
 * 5 deflation projections, 6 prolongator restrict/prolong, 7 transport network, 8 graph-
 * captured inner cycles (opts->graph: a whole cycle is one launch).  h_ms, h_calls and
 * h_bytes (each 9 entries, may be NULL) receive the device milliseconds, the
 * launch counts and the algorithmic HBM bytes of the timed launches.  mode 0: read;
 * 1: read, then zero; 2: zero and start timing; 3: stop timing.  Timing is off by default
 * and costs two event records per launch when on. */
int lqt_kernel_times(lqt_ctx *ctx, double *h_ms, long long *h_calls, double *h_bytes, int mode);

const char *lqt_last_error(const lqt_ctx *ctx);
void lqt_destroy(lqt_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* LQTRACE_H */
