/*
 * Plain serial FP64 CPU oracle for the parareal / L1 / spectral-Galerkin
 * solver of the quasilinear Caputo subdiffusion equation
 *     d^alpha_t u = div(D(x,t,u) grad u) + f(x,t,u)   on (0,1)^dim, u = 0 on the boundary.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the CPU-baseline leg of
 * the benchmark may load this library.  The product path (the HIP library) shares
 * no code, header, table or helper with it.
 *
 * Everything is double precision, plain loops, no BLAS, no threads.  Each function
 * states the passage of the paper it follows.  Space is the orthonormal sine basis
 * phi_k(x) = sqrt(2) sin(k pi x) (2D: the tensor product 2 sin(k1 pi x) sin(k2 pi y),
 * index k = (k1-1)*M + (k2-1)), integrated with Gauss-Legendre quadrature on (0,1)
 * (2D: the tensor rule).  The mass matrix is the identity (orthonormal basis).
 *
 * Notation: M modes per direction, Q quadrature points per direction, N fine steps,
 * P parareal slices (the paper's N_t), S = N/P fine steps per slice (the paper's M),
 * dT = T/P, dt = T/N.
 *
 * Parity status: every function here is pinned by the CPU test-suite (closed forms,
 * library routines, invariants and convergence orders), except the values produced
 * with a nonlinear D or a u-dependent f, which have no closed form; those are pinned
 * only through the manufactured-solution convergence test and the invariants.
 */
#ifndef L1PR_ORACLE_H
#define L1PR_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t dim;          /* 1 or 2 */
  int32_t modes;        /* M per direction */
  int32_t quad;         /* Q per direction, Q >= M */
  int32_t steps;        /* N, N % P == 0 */
  int32_t slices;       /* P */
  double  alpha;        /* (0,1] */
  double  T;            /* > 0 */
  int32_t d_sel;        /* diffusion selector; -1 = D identically 0 (oracle-only test hook) */
  double  d_param;      /* constant D for d_sel == 0 */
  int32_t f_sel;        /* source selector */
  int32_t history;      /* 0 hybrid (coarse history in F), 1 full uniform fine L1,
                           2 uniform fine L1 with the history beyond ORACLE_SOE_J0 steps by a
                           sum of exponentials (serial solve only) */
  int32_t source_time;  /* 0 lagged source (the paper), 1 source at the new time level */
  int32_t solver;       /* 0 (or 1): stiffness by Gauss quadrature, dense solve;
                           2: constant D only, stiffness integral taken exactly,
                           D lambda_k on the diagonal (the sine basis diagonalises it) */
} oracle_problem;

/* 0 on success, -1 if the problem is invalid. */
int    oracle_validate(const oracle_problem* p);

/* L1 weight b_x = (x+1)^(1-alpha) - x^(1-alpha), with b_0 = 1 (L1 scheme, Section 2.1). */
double oracle_bweight(double x, double alpha);

/* Sum-of-exponentials form of the L1 weights at distances j >= ORACLE_SOE_J0 (the fast
   history of the paper's outlook, Conclusions (i)): b_j ~ sum_l w_l exp(-lam_l j) for
   ORACLE_SOE_J0 <= j <= N.  From b_j = (1-alpha) int_j^{j+1} s^-alpha ds and
   s^-alpha = (1/Gamma(alpha)) int exp(alpha y - s e^y) dy over the real line, the trapezoid
   rule in y with step ORACLE_SOE_H on the grid y = n h gives
   w = h (1-alpha)/Gamma(alpha) e^{(alpha-1) y} (1 - exp(-e^y)), lam = e^y; the nodes below
   n_lo (lam N negligible) are merged into one node lam = 0 whose weight is their geometric
   sum, and the nodes above n_hi (exp(-lam j) < e^-40 for j >= j0) are dropped.  n_lo keeps
   the merge error below ORACLE_SOE_EPS b_j for every j <= N.  Writes the merged node first,
   then n_lo..n_hi ascending; returns the node count, or -1 if it exceeds max_nodes or alpha
   is not in (0,1). */
#define ORACLE_SOE_J0 16
#define ORACLE_SOE_H 0.3
#define ORACLE_SOE_EPS 1e-13
int32_t oracle_soe_nodes(double alpha, int32_t N, double* lam, double* w, int32_t max_nodes);

/* Gauss-Legendre nodes (ascending) and weights on (0,1); weights sum to 1. */
void   oracle_gauss_legendre01(int32_t Q, double* x, double* w);

/* Diffusion coefficient and source selected by the problem. */
double oracle_D(const oracle_problem* p, double x, double y, double t, double u);
double oracle_f(const oracle_problem* p, double x, double y, double t, double u);

/* Galerkin matrices at coefficient vector c: K (Md x Md, row-major) and the load F
   (Md) with D and f evaluated at (tD, u_c) and (tf, u_c). */
int    oracle_galerkin(const oracle_problem* p, const double* c, double tD, double tf,
                       double* K, double* F);

/* The rows `rows[0..nrows)` of K (Krows [nrows][Md]) and the whole load F, equal to those of
   oracle_galerkin bit for bit (for sampled checks at sizes where the whole K is too slow). */
int    oracle_galerkin_rows(const oracle_problem* p, const double* c, double tD, double tf,
                            int32_t nrows, const int32_t* rows, double* Krows, double* F);

/* One semi-implicit step: solve (I + tau K(c_prev)) c = hist + tau F(c_prev). */
int    oracle_step(const oracle_problem* p, const double* c_prev, double tD, double tf,
                   const double* hist, double tau, double* c_out);

/* Coarse propagator G_n(C_0..C_n) -> out (Md).  C holds n+1 vectors. */
int    oracle_coarse_G(const oracle_problem* p, int32_t n, const double* C, double* out);

/* Fine propagator F_n(C_0..C_n) -> out (Md); traj (S+1 vectors) optional. */
int    oracle_fine_F(const oracle_problem* p, int32_t n, const double* C, double* out,
                     double* traj);

/* Serial solve.  U: P+1 slice ends; traj: N+1 fine states (optional). */
int    oracle_solve_serial(const oracle_problem* p, const double* u0, double* U, double* traj);

/* Parareal (history = 0: hybrid fine propagator; history = 1: full-history fine propagator
   on the previous iterate's fine trajectory, fixed point = the uniform L1 serial solution).
   U: final iterate (P+1 vectors).  U_iters: all iterates
   [max_iter+1][P+1][Md] (optional).  incr: relative increments [max_iter] (optional).
   *iters: number of fine sweeps done.  Returns 0. */
int    oracle_solve_parareal(const oracle_problem* p, const double* u0, double* U,
                             int32_t max_iter, double tol, double* U_iters, double* incr,
                             int32_t* iters);

#ifdef __cplusplus
}
#endif
#endif
