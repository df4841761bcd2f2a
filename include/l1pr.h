/*
 * l1pr — parareal-in-time, L1-in-time, sine-Galerkin-in-space solver for the
 * quasilinear Caputo subdiffusion equation
 *
 *     d^alpha_t u = div( D(x,t,u) grad u ) + f(x,t,u)   on (0,1)^dim,  u = 0 on the boundary,
 *     u(x,0) = u0(x),
 *
 * for MI355X (gfx950).  Method: arXiv 2510.11023, "Parareal in time and spectral in space
 * fast L1 quasilinear subdiffusion solver" (Caballero, Plociniczak, Sadarangani).
 *
 * Space.  Orthonormal sine basis phi_k(x) = sqrt(2) sin(k pi x), k = 1..M (2D: the tensor
 * product 2 sin(k1 pi x) sin(k2 pi y), coefficient index (k1-1)*M + (k2-1)), so the Galerkin
 * mass matrix is the identity.  The stiffness K_kl = sum_q w_q D(x_q,t,u_q) phi_k'(x_q) phi_l'(x_q)
 * and the load F_k = sum_q w_q f(x_q,t,u_q) phi_k(x_q) use Gauss-Legendre quadrature on (0,1)
 * with Q points per direction (the weak form of Section 2.1 with quadrature).
 *
 * Time.  Uniform coarse grid T_n = n T/P (P parareal slices) and fine grid of N = P*S steps.
 *   - coarse propagator G (Section 2.1, semi-implicit sequential L1 scheme, step T/P):
 *       (I + tau_c K(C_n)) C_{n+1} = C_n - sum_{i=1}^{n} b_{n+1-i} (C_i - C_{i-1}) + tau_c F(C_n)
 *   - fine propagator F (Section 2.2, hybrid L1: fine grid in the current slice, coarse grid
 *     for the history), for r = 1..S starting at c_0 = C_n:
 *       (I + tau K(c_{r-1})) c_r = c_{r-1} - sum_{j=1}^{r-1} b_{r-j} (c_j - c_{j-1})
 *                                 - S^-alpha sum_{i=1}^{n} b_{n-i+r/S} (C_i - C_{i-1}) + tau F(c_{r-1})
 *   with b_x = (x+1)^(1-alpha) - x^(1-alpha), b_0 = 1, tau = dt^alpha Gamma(2-alpha),
 *   tau_c = dT^alpha Gamma(2-alpha); D and f lagged to the previous level.
 *   - parareal (Section 2.2 and its flowchart): coarse initial sweep, then per sweep k the
 *     fine propagator on all slices at once and the sequential correction
 *       U^{k+1}_{n+1} = F_n(U^k_0..U^k_n) + (G_n(U^{k+1}_0..U^{k+1}_n) - G_n(U^k_0..U^k_n)).
 *     After k sweeps the first k+1 slice ends equal the serial solution exactly, so at most
 *     P sweeps reproduce it bit for bit.
 *
 * Conventions of every entry point.
 *   - Pointers marked "device" point to device memory of the current HIP device; the caller
 *     owns every buffer (the library allocates nothing and never frees caller memory).
 *   - Vectors of coefficients are float64, contiguous, with Md = M (1D) or M*M (2D)
 *     entries, ordered by mode number.
 *   - Every call is asynchronous and stream-ordered on `stream` (a hipStream_t passed as a
 *     void*; NULL means the default stream), except where a host-side stop test is asked for
 *     (parareal with tol > 0), which synchronises the stream once per sweep.
 *   - Problems are validated on the host before anything is launched; an invalid problem
 *     returns L1PR_EINVAL and touches nothing.
 *   - The first 256 bytes of every workspace hold the call's device status word.  Every solve
 *     clears it when it starts, and its kernels set it when a state or an increment is NaN or
 *     infinite, or when a bounded device wait gives up.  A call that does not synchronise
 *     (serial solves, parareal with tol <= 0, graph-captured calls) cannot return those
 *     conditions itself: l1pr_check(ws, stream) reports them once the call has run.
 *   - No C++ exception crosses this boundary.
 */
#ifndef L1PR_H
#define L1PR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  L1PR_OK = 0,
  L1PR_EINVAL = -1,     /* invalid problem or argument */
  L1PR_ENOMEM = -2,     /* workspace smaller than l1pr_workspace_bytes() */
  L1PR_EHIP = -3,       /* HIP runtime error */
  L1PR_ENOTCONV = -4,   /* parareal stopped at max_iter < P without meeting tol; U holds the last iterate */
  L1PR_ENONFINITE = -5, /* a slice end of a serial solve or a parareal increment was NaN or infinite */
  L1PR_ESOLVE = -6,     /* an iterative step solve (solver = 1) missed its tolerance */
  L1PR_EWAIT = -7       /* a bounded wait inside a kernel gave up: the results of the call are
                           not valid (a device fault, not a property of the problem) */
} l1pr_status;

/* Diffusion selectors D(x,t,u). */
enum { L1PR_D_CONST = 0,      /* d_param (> 0)                 */
       L1PR_D_SIN2 = 1,       /* 1 + sin(u)^2 / 2              */
       L1PR_D_RATIONAL = 2,   /* 1 + 1/(1 + u^2)               */
       L1PR_D_GAUSS = 3,      /* 1 + exp(-u^2) / 2             */
       L1PR_D_LINEAR = 4 };   /* 1 + u (the paper's model problem, Section 4.2) */

/* Source selectors f(x,t,u).  s(x) = sin(pi x) (2D: sin(pi x) sin(pi y)). */
enum { L1PR_F_ZERO = 0,
       L1PR_F_MMS_SIN2 = 1,   /* manufactured: U = (1 + t^alpha) s is exact for D = L1PR_D_SIN2 */
       L1PR_F_LOGISTIC = 2,   /* 0.1 u (1 - u)                 */
       L1PR_F_SIN = 3,        /* sin(u)                        */
       L1PR_F_PAPER = 4,      /* s(x) exp(-t) (Section 4.2)    */
       L1PR_F_MMS_SMOOTH = 5  /* manufactured: U = (1 + t^2) s is exact for constant D = d_param */ };

typedef struct {
  int32_t dim;          /* 1 or 2 */
  int32_t modes;        /* M per direction, >= 1; at most 1024 in 1D and 64 in 2D (M^2
                           coefficients; more than 256 go through the device-memory
                           factorisation); with the diagonal solve (solver = 2) 4096 in 1D
                           (Q <= 8192) and 256 in 2D */
  int32_t quad;         /* Q per direction, >= M */
  int32_t steps;        /* N fine steps, N % P == 0 */
  int32_t slices;       /* P parareal slices (coarse steps) */
  double  alpha;        /* fractional order in (0, 1] (used when no per-instance alpha is given) */
  double  T;            /* final time > 0 */
  int32_t d_sel;        /* L1PR_D_*  */
  double  d_param;      /* constant D for L1PR_D_CONST (> 0); the D of L1PR_F_MMS_SMOOTH */
  int32_t f_sel;        /* L1PR_F_*  */
  int32_t history;      /* 0: hybrid fine propagator (the paper's; parareal's fixed point)
                           1: full uniform L1 over all N steps (serial; parareal with the plain
                              coarse step, whose fine propagators then take the history of
                              earlier slices from the previous iterate's fine trajectories)
                           2: the uniform L1 scheme of 1 with the history terms at distances
                              d >= 16 from sum-of-exponentials weights b_d ~ sum_l w_l e^{-lam_l d}
                              (the fast history of the conclusions' outlook): the trapezoid rule
                              with step 0.3 in log s on b_d = (1-alpha) int_d^{d+1} s^-alpha ds,
                              written as an integral of e^{-s t} t^{alpha-1}; weights within about
                              1e-13 of b_d for 16 <= d <= N, O(log N) nodes (about 100 at
                              N = 4096), carried as per-mode exponential sums, so each step costs
                              O(nodes + 16) per coefficient instead of O(m); serial solve only;
                              not for 1D beyond 256 modes unless solver = 2 */
  int32_t source_time;  /* 0: f lagged to the previous level (the paper)
                           1: f at the new time level (only for u-independent f) */
  int32_t assembly;     /* how the stiffness sum_q w_q D_q phi_k'(x_q) phi_l'(x_q) is formed:
                           0: cosine moments, K_kl = k l pi^2 (m_|k-l| + m_{k+l}) with
                              m_j = sum_q w_q D_q cos(j pi x_q) (product-to-sum identity of the
                              sine basis; the same quadrature sum, 2M+1 moments instead of
                              M^2 dot products), M <= 256; larger M uses 1
                           1: quadrature GEMM dphi^T diag(w D) dphi on FP64 MFMA */
  int32_t tune;         /* variants of the fine and full-history steps (bit 0: 16 x 16
                           split-K tiles for the lagged-state product instead of 32 x 32;
                           bit 1: 16 x 16 split-K tiles for the projections instead of 32 x 32;
                           bit 2: 128-column blocks instead of 256 in the device-memory
                           factorisation of systems with more than 256 coefficients;
                           bit 3: 64 x 64 instead of 128 x 128 tiles in its trailing
                           update); 0 is
                           the default, l1pr_autotune measures the best.  The variants sum in
                           different orders, so runs compared bit for bit must use the same
                           value. */
  int32_t solver;       /* the step's linear system (I + tau K) c = rhs:
                           0: Cholesky factorisation (register-resident for <= 256 coefficients,
                              blocked through device memory beyond);
                           1: preconditioned conjugate gradients, 2D only, Q >= 3M/2 (with
                              fewer points the quadrature stiffness has near-null directions
                              that the preconditioner does not see): K applied as the
                              separable quadrature products (Phi' (x) Phi and Phi (x) Phi' at the
                              Q x Q Gauss points, w w D between them), never formed;
                              preconditioned by the diagonal of I + tau K (from the cosine
                              moments; with constant D the sine basis diagonalises K); started
                              from the lagged state and stopped when ||r|| <= 1e-14 ||rhs||
                              (coarse steps of parareal: 1e-10; they steer the iteration, the
                              fine steps fix its result); at most 200 iterations, else
                              L1PR_ESOLVE.  Each unit iterates on its own data, so parareal
                              stays exact; the host checks convergence every 4 iterations (one
                              stream synchronisation), so such a solve cannot be captured in a
                              graph;
                           2: constant D only (d_sel = L1PR_D_CONST, assembly = 0), 1D or 2D:
                              the stiffness integral taken exactly, D (grad phi_k, grad phi_l) =
                              D lambda_k delta_kl for the orthonormal sine basis (lambda_k =
                              (k pi)^2, or (k1^2 + k2^2) pi^2 in 2D), so a step is the O(M)
                              division c_k = (hist_k + tau F_k) / (1 + tau D lambda_k); the load
                              F stays the quadrature sum.  Equal to solver 0 up to the
                              quadrature error of the stiffness (rounding level at Q = 2M in
                              1D from M of about 64 on, at Q = 3M in 2D for M = 12; smaller M
                              needs a larger ratio); the spectral diagonalisation among the
                              outlook items of the paper's conclusions.  Not for uneven
                              batches. */
} l1pr_problem;

/* Operation codes for l1pr_workspace_bytes. */
enum { L1PR_OP_SERIAL = 0, L1PR_OP_PARAREAL = 1 };

/* Bytes of device workspace that an operation needs for `batch` instances. */
size_t l1pr_workspace_bytes(const l1pr_problem* p, int32_t batch, int32_t op);

/* Returns L1PR_OK if the problem is valid, L1PR_EINVAL otherwise (host only). */
l1pr_status l1pr_validate(const l1pr_problem* p);

/* Serial solve of `batch` independent instances: the fine solution C_{n+1} = F_n(C_0..C_n)
 * (history = 0; the fixed point of parareal, Section 2.2) or the full uniform L1 scheme
 * (history = 1).
 *   alpha : host [batch] per-instance fractional orders, or NULL to use p->alpha for all.
 *   u0    : device [batch][Md]           initial coefficients.
 *   U     : device [batch][P+1][Md]      output slice ends C_0..C_P.
 *   traj  : device [batch][N+1][Md]      output fine trajectory, or NULL.
 *   ws    : device workspace of ws_bytes >= l1pr_workspace_bytes(p, batch, L1PR_OP_SERIAL). */
l1pr_status l1pr_solve_serial(const l1pr_problem* p, int32_t batch, const double* alpha,
                              const double* u0, double* U, double* traj,
                              void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): l1pr_solve_serial with its workspace taken
 * from a device array of L1PR_NOALLOC_SCRATCH_BYTES that the library holds on each device for
 * the life of the process.  The call allocates nothing and frees nothing; arguments, results
 * and errors are those of l1pr_solve_serial, and L1PR_ENOMEM (nothing launched) when
 * l1pr_workspace_bytes(p, batch, L1PR_OP_SERIAL) exceeds L1PR_NOALLOC_SCRATCH_BYTES (for
 * example config 1 fits, and the 1D shape M = 256, Q = 384, N = 4096, P = 64 with up to 200
 * instances).  All calls on one device share that device's array: calls that overlap on
 * one device (several streams or threads) race and must be serialised by the caller.  A host
 * alpha array is copied with a pageable hipMemcpyAsync; pass NULL (p->alpha) to capture the
 * call into a graph. */
#define L1PR_NOALLOC_SCRATCH_BYTES (64u << 20)
l1pr_status l1pr_solve_serial_noalloc(const l1pr_problem* p, int32_t batch, const double* alpha,
                                      const double* u0, double* U, double* traj, void* stream);

/* The two propagators on given slice ends, for every slice at once (Section 2.2):
 *   l1pr_coarse_apply: out[b][n] = G_n(Z_b[0..n])   (one coarse L1 step of size T/P),
 *   l1pr_fine_apply:   out[b][n] = F_n(Z_b[0..n])   (S fine steps with the hybrid history),
 * for n = 0..P-1.  These are the parallel stage of parareal as stand-alone operations (and,
 * applied to a serial solution, the training pairs of the learned coarse propagator).
 *   alpha : host [batch] per-instance orders, or NULL for p->alpha.
 *   Z     : device [batch][P+1][Md];  out : device [batch][P][Md].
 *   ws    : device workspace >= l1pr_workspace_bytes(p, batch, L1PR_OP_PARAREAL). */
l1pr_status l1pr_coarse_apply(const l1pr_problem* p, int32_t batch, const double* alpha,
                              const double* Z, double* out, void* ws, size_t ws_bytes,
                              void* stream);
l1pr_status l1pr_fine_apply(const l1pr_problem* p, int32_t batch, const double* alpha,
                            const double* Z, double* out, void* ws, size_t ws_bytes,
                            void* stream);

/* Coarse propagators of parareal. */
enum { L1PR_COARSE_L1 = 0,       /* the coarse L1 step G of Section 2.1 */
       L1PR_COARSE_LEARNED = 1   /* G plus a learned residual correction (below) */ };

/* Parareal solve of `batch` instances, Section 2.2 and its flowchart.
 * history = 0: the paper's hybrid fine propagator (coarse-grid history of earlier slices);
 * the fixed point is l1pr_solve_serial with history 0.
 * history = 1: full-history fine propagators: slice n's L1 history runs over the whole fine
 * grid, the steps before nS taken from the previous iterate's fine trajectories (before the
 * first sweep, the coarse iterate interpolated linearly over each slice); the fixed point is
 * l1pr_solve_serial with history 1, reached bit for bit after P sweeps (the first k+1 slice
 * ends after k sweeps).  Costs B*P*(2S+1)*Md doubles more workspace and one prefix launch
 * per sweep.  Not with the learned coarse propagator, uneven batches or the batch call.
 *   max_iter : number of fine sweeps allowed, 0 <= max_iter <= P.
 *   tol      : > 0: the stop rule of the flowchart, per instance.  After each sweep the
 *              relative increment ||U^{k+1}_b - U^k_b|| / ||U^{k+1}_b|| (Frobenius over all
 *              P+1 slice ends) is formed; an instance whose increment is <= tol is finished:
 *              later sweeps keep its slice ends and skip its units.  The host synchronises
 *              once per sweep and stops when every instance is finished.
 *              <= 0: exactly min(max_iter, P) sweeps for every instance, no synchronisation
 *              (graph-capturable).
 *   coarse   : L1PR_COARSE_L1 (the coarse L1 step G of Section 2.1) or L1PR_COARSE_LEARNED:
 *              G_L,n = G_n + r with the residual r from the network in `mlp_params` (device,
 *              layout from l1pr_mlp_layout for M = p->modes, 1D, M <= 256, history 0,
 *              256-byte aligned).  The network is a deterministic function of its input, so
 *              parareal keeps its exactness (after k sweeps the first k+1 slice ends equal
 *              the serial solution).  The plain coarse step is the fallback: a unit whose
 *              correction is not finite or larger than ||G_n|| + 1 uses the plain G_n.  The
 *              plain step also judges the learned one per instance: after the first fine
 *              sweep an instance whose learned coarse values are not closer to the fine
 *              results F_n than the plain ones, and later an instance whose increment
 *              shrinks by less than half from one sweep to the next, goes back to the plain
 *              coarse step for good, its stored coarse values replaced by the plain ones (its
 *              iteration is then exactly plain parareal).
 *              ws_bytes must then also cover l1pr_parareal_learned_extra_bytes(p, batch).
 *   iters    : device int32 [batch] or NULL: each instance's status after the call: the
 *              number of sweeps after which it was finished (tol > 0) or that it ran (tol <= 0,
 *              or P sweeps: exact), L1PR_ENOTCONV if tol > 0 was not met within max_iter < P
 *              sweeps, L1PR_ENONFINITE if its increment became NaN or infinite (the instance
 *              is frozen at that sweep).
 *   incr     : device [batch][max_iter] relative increment of each sweep, or NULL.
 *   U_iters  : device [max_iter+1][batch][P+1][Md] every iterate (0 = coarse prediction), or NULL.
 *   U        : device [batch][P+1][Md]   output: each instance's last iterate.
 *   sweeps   : host int32, the number of sweeps run, or NULL.
 * Returns, for tol > 0: L1PR_ENONFINITE if an instance's increment was not finite,
 * L1PR_ENOTCONV if an instance did not meet tol within max_iter < P sweeps, L1PR_EWAIT if a
 * device wait gave up; for tol <= 0 those conditions are left in `iters` and the status word
 * (l1pr_check). */
l1pr_status l1pr_solve_parareal(const l1pr_problem* p, int32_t batch, const double* alpha,
                                const double* u0, double* U, int32_t max_iter, double tol,
                                int32_t coarse, const void* mlp_params, int32_t* iters,
                                double* incr, double* U_iters, int32_t* sweeps,
                                void* ws, size_t ws_bytes, void* stream);

/* Waits for `stream` and reports the device status word of the last call that used the
 * workspace `ws` (device, the call's workspace): L1PR_OK, L1PR_ENONFINITE (a slice end of a
 * serial solve, or a parareal increment, was NaN or infinite), L1PR_EWAIT (a bounded device
 * wait gave up: the results are not valid), or L1PR_EHIP. */
l1pr_status l1pr_check(const void* ws, void* stream);

/* Uneven batches (instances that differ in modes, fine steps per slice and order under one
 * problem).  All arrays are device arrays of `batch` entries; any may be NULL.
 *   modes : instance b's own modes M_b, 1 <= M_b <= p->modes (coefficients k >= M_b are
 *           zero; u0 must be zero there).  Instances with roundup16(M_b) equal to
 *           roundup16(p->modes) reproduce their own runs (modes = M_b, same quad) bit for bit.
 *   spp   : instance b's own fine steps per slice S_b, 1 <= S_b <= p->steps / p->slices; its
 *           fine grid has P S_b steps (dt = T / (P S_b)).
 *   alpha : instance b's order (else p->alpha).
 * Entries outside the ranges are clamped into them.
 * The coarse propagator of l1pr_solve_parareal_uneven:
 *   coarse    : L1PR_COARSE_L1, or L1PR_COARSE_LEARNED with
 *   mlp       : device blob of a network for mlp_modes modes (layout from l1pr_mlp_layout,
 *               256-byte aligned), p->modes <= mlp_modes <= 256: one network serves every
 *               instance; the coefficients an instance does not carry (k >= M_b) enter it as
 *               zeros and only its outputs for k < M_b are used.  Fallback to the plain
 *               coarse step as in l1pr_solve_parareal (per unit and per instance).
 *               ws_bytes must also cover l1pr_parareal_learned_extra_bytes(p, batch). */
typedef struct {
  const int32_t* modes;
  const int32_t* spp;
  const double* alpha;
  int32_t coarse;
  const void* mlp;
  int32_t mlp_modes;
} l1pr_uneven;

/* Serial (hybrid) solve of an uneven batch; the other arguments as in l1pr_solve_serial.
 * Needs a 1D problem with history 0 and roundup16(M) <= 256.  Nothing is copied from the
 * host, so the call can be captured into a HIP graph. */
l1pr_status l1pr_solve_serial_uneven(const l1pr_problem* p, int32_t batch,
                                     const l1pr_uneven* desc, const double* u0, double* U,
                                     void* ws, size_t ws_bytes, void* stream);

/* Parareal over an uneven batch with at most `sweeps` sweeps and no host synchronisation
 * (the whole call can be captured into a HIP graph): the algorithm of l1pr_solve_parareal,
 * with the per-instance stop test on conv_tol: an instance whose increment is <= conv_tol is
 * finished at that sweep (later sweeps keep its slice ends and skip its units); the others
 * run `sweeps` sweeps.  The coarse propagator is desc->coarse (plain or learned).
 *   conv   : device int32 [batch] or NULL: the first sweep k (1-based) whose increment
 *            relative ||U^k - U^(k-1)|| / ||U^k|| is <= conv_tol (the instance's finishing
 *            sweep), -1 if none, L1PR_ENONFINITE if its increment was not finite;
 *   stamps : device int64 [sweeps + 1] or NULL: the device wall clock (constant rate, see
 *            hipDeviceAttributeWallClockRate) at the end of the initial coarse sweep and of
 *            each sweep;
 *   incr   : device [batch][sweeps] or NULL: the increments. */
l1pr_status l1pr_solve_parareal_uneven(const l1pr_problem* p, int32_t batch,
                                       const l1pr_uneven* desc, const double* u0, double* U,
                                       int32_t sweeps, double conv_tol, int32_t* conv,
                                       int64_t* stamps, double* incr, void* ws, size_t ws_bytes,
                                       void* stream);

/* Heterogeneous batch: `count` problems, each with its own parameters and one instance (its
 * own alpha is probs[i].alpha), solved as groups of problems that share launches, one group
 * after another on the stream:
 *  - 1D problems with history 0 and roundup16(modes) <= 256 are grouped by (roundup16(modes),
 *    quad, slices, T, d_sel, d_param, f_sel, source_time, assembly, tune) and run as an uneven
 *    batch (each with its own modes, fine steps per slice steps/slices and order);
 *  - every other problem is grouped with the problems equal to it up to alpha.
 * Each problem's result equals its own l1pr_solve_serial / l1pr_solve_parareal run bit for bit.
 *   op     : L1PR_OP_SERIAL (the serial solutions) or L1PR_OP_PARAREAL (min(sweeps, P_i)
 *            parareal sweeps, no tolerance test, no host synchronisation per sweep)
 *   coarse, mlp_params, mlp_modes : parareal's coarse propagator for every group
 *            (L1PR_COARSE_LEARNED: one network of mlp_modes modes for all problems, each
 *            1D with history 0 and modes <= mlp_modes, zero-padded as in l1pr_uneven;
 *            EINVAL otherwise); ignored for L1PR_OP_SERIAL
 *   u0     : device; problem i's initial coefficients at u0 + u0_off[i] (Md_i values)
 *   U      : device; problem i's slice ends at U + U_off[i] ((P_i + 1) x Md_i values, row-major)
 *   u0_off, U_off : host int64 [count], offsets in doubles
 *   ws     : device workspace, ws_bytes >= l1pr_batch_workspace_bytes(probs, count, op)
 * Returns EINVAL (and launches nothing) if a problem, op or sweeps is invalid (parareal needs
 * history 0 in every problem).  The grouping
 * and the per-instance tables are host work with pageable copies: the call is not meant for
 * graph capture (the uneven entry points above are). */
size_t      l1pr_batch_workspace_bytes(const l1pr_problem* probs, int32_t count, int32_t op);
l1pr_status l1pr_solve_batch(const l1pr_problem* probs, int32_t count, int32_t op, int32_t sweeps,
                             int32_t coarse, const void* mlp_params, int32_t mlp_modes,
                             const double* u0, const int64_t* u0_off, double* U,
                             const int64_t* U_off, void* ws, size_t ws_bytes, void* stream);

/* Rate of the device wall clock that l1pr_solve_parareal_uneven stamps, in kHz (-1 on
 * error); for the current device. */
int64_t     l1pr_wall_clock_khz(void);
/* Writes the device wall clock to t (device int64) when the stream reaches this point. */
l1pr_status l1pr_device_stamp(int64_t* t, void* stream);

/* Measures the variants of a fine step of `batch` instances x P slices (the parareal fine
 * sweep) and writes the fastest as tune bits: the GEMM tiles for systems of at most 256
 * coefficients (bits 0, 1; timed on the fine step and on a step of `batch` units, the serial
 * solve's, the variant with the smaller sum chosen, since serial and parareal must use the
 * same bits), the block width and trailing-update tiles of the blocked factorisation beyond
 * (bits 2, 3); 0 for problems without a choice.
 * Needs a parareal workspace (ws_bytes >= l1pr_workspace_bytes(p, batch, L1PR_OP_PARAREAL));
 * synchronises the stream. */
l1pr_status l1pr_autotune(const l1pr_problem* p, int32_t batch, void* ws, size_t ws_bytes,
                          void* stream, int32_t* tune_out);

size_t l1pr_parareal_learned_extra_bytes(const l1pr_problem* p, int32_t batch);

/* ---- Learned coarse propagator (configuration with a residual MLP) ----------------------
 * Network: inputs x = [G_n coefficients (M) ; alpha ; n/P] (M + 2), normalised per column
 * with the stored mean and standard deviation; three hidden layers of 512 units with SiLU
 * activation z / (1 + exp(-z)); M outputs, the normalised residual F_n - G_n, mapped back with
 * the stored output mean and standard deviation.  Training keeps weights and activations in
 * BF16 with FP32 accumulation (MFMA); inside parareal (and in l1pr_mlp_infer) the same BF16
 * weights are applied in FP64.  Biases and normalisation are FP32.
 *   params : device blob read by inference (normalisation, biases, BF16 weights [out][in] with
 *            the inner dimension padded); offsets and sizes from l1pr_mlp_layout.  Must be
 *            256-byte aligned (EINVAL otherwise): the inference kernel uses 16-byte loads.
 *   state  : device FP32 [3][flat_count]: master parameters, Adam first and second moments;
 *            the flat order is W1 b1 W2 b2 W3 b3 W4 b4 (each W row-major [out][in_padded]).
 * Training data and initial weights are supplied by the caller. */
typedef struct {
  int32_t in, in_padded, hidden, out, out_padded;
  size_t  param_bytes, state_bytes;
  int64_t flat_count;
  size_t  off_in_mean, off_in_std, off_out_mean, off_out_std;   /* FP32 arrays in params */
  size_t  off_w[4], off_b[4];                                   /* in params */
  int64_t flat_w[4], flat_b[4];                                 /* element offsets in state */
} l1pr_mlp_info;

l1pr_status l1pr_mlp_layout(int32_t modes, l1pr_mlp_info* info);
size_t      l1pr_mlp_workspace_bytes(int32_t modes, int32_t n, int32_t train);
/* params weights/biases <- state masters (BF16 rounding to nearest even). */
l1pr_status l1pr_mlp_sync(int32_t modes, const void* state, void* params, void* stream);
/* zero the Adam moments in state */
l1pr_status l1pr_mlp_reset_moments(int32_t modes, void* state, void* stream);
/* normalisation into params: per-column mean and (population) standard deviation of the
 * inputs x [n][M+2] (a column with no spread gets 1; the M coefficient columns' scales are
 * floored at 1e-4 of the largest of them, so that barely varying inputs are not magnified);
 * per-mode mean of the targets t [n][M] and one common output scale, the root mean square of
 * the per-mode standard deviations (a target column with no spread counts as 0) */
l1pr_status l1pr_mlp_stats(int32_t modes, const float* x, const float* t, int64_t n,
                           void* params, void* stream);
/* training pairs from slice ends Z [B][P+1][M] and coarse values G [B][P][M] (device FP64):
 * x [B*P][M+2] = [G_n ; alpha_b ; n/P],  t [B*P][M] = Z_{n+1} - G_n  (device FP32, row b*P+n);
 * alpha is a device array [B]. */
l1pr_status l1pr_mlp_features(int32_t modes, int32_t batch, int32_t slices, const double* alpha,
                              const double* Z, const double* G, float* x, float* t,
                              void* stream);
/* y [n][M] = normalised network output for raw inputs x [n][M+2] (device FP32), evaluated as
 * in training (activations rounded to BF16 between layers). */
l1pr_status l1pr_mlp_forward(int32_t modes, const void* params, const float* x, int32_t n,
                             float* y, void* ws, size_t ws_bytes, void* stream);
/* The same network evaluated as parareal uses it, in FP64: BF16 weights (exact in FP64), FP64
 * activations and sums.  x [n][M+2] raw inputs, y [n][M] normalised output (device FP64).
 * The parareal correction G_L(U^{k+1}) - G_L(U^k) then vanishes as U^{k+1} -> U^k down to
 * FP64 rounding; a shorter activation format would floor it at that format's resolution. */
l1pr_status l1pr_mlp_infer(int32_t modes, const void* params, const double* x, int32_t n,
                           double* y, void* ws, size_t ws_bytes, void* stream);
size_t      l1pr_mlp_infer_workspace_bytes(int32_t modes, int32_t n);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias correction with `step`, 1-based) on the
 * mean squared error of the normalised output over the rows idx[0..n) (device int32, or NULL
 * for rows 0..n-1) of x [*][M+2] and t [*][M]; then params <- masters.  loss (device FP32 [1])
 * and grad_out (device FP32 [flat_count], the gradient before the update) may be NULL. */
l1pr_status l1pr_mlp_train_step(int32_t modes, void* params, void* state, const float* x,
                                const float* t, const int32_t* idx, int32_t n, float lr,
                                int32_t step, float* loss, float* grad_out, void* ws,
                                size_t ws_bytes, void* stream);

/* Kernel-launch profiling (for benchmarks).  After l1pr_profile_start(), every step kernel
 * that the solvers enqueue is bracketed by two HIP events recorded on its stream;
 * l1pr_profile_start_only(names) brackets only the kernels named in the comma-separated
 * list (NULL or "" = all), so that a timed run pays for the events of those launches alone.
 * l1pr_profile_stop() turns recording off, waits for the recorded events, and aggregates
 * the elapsed times by "kernel/mode/units" (kernel = lag | proj | assemble | history | chol |
 * eval | blk_solve | products2d | assemble2d | rhs | prefix | cg_grid | cg_step | cg_finish |
 * mlp | refine, mode = fine | coarse | full, units = systems per launch).  It writes up to max_out
 * entries to `out` (host memory owned by the caller) and returns the number of distinct
 * entries, or -1 on a HIP error.  With launches on several streams at once, a launch's time
 * runs from its stream reaching it to its end, so it includes any wait for CUs held by the
 * other streams.  The events are created on first use and kept by the library for reuse;
 * nothing else is allocated. */
typedef struct {
  char    name[64];
  int64_t launches;
  double  total_ms;
} l1pr_kernel_stat;

void    l1pr_profile_start(void);
void    l1pr_profile_start_only(const char* names);
int32_t l1pr_profile_stop(l1pr_kernel_stat* out, int32_t max_out);

/* Static description of a status code. */
const char* l1pr_status_string(l1pr_status s);

#ifdef __cplusplus
}
#endif
#endif
