/*
 * Plain serial FP64 CPU oracle (test infrastructure only; see oracle.h).
 *
 * Written from the paper "Parareal in time and spectral in space fast L1 quasilinear
 * subdiffusion solver" (arXiv 2510.11023):
 *   - L1 weights and the sequential L1-Galerkin scheme (coarse propagator G):
 *     Section 2.1, the L1 scheme and the semi-implicit sequential scheme.
 *   - Hybrid fine L1 operator and fine propagator F: Section 2.2, the hybrid L1
 *     approximation on the coarse/fine grid and the fine scheme built on it.
 *   - Parareal iteration: Section 2.2, initialisation, iterative correction and the
 *     flowchart of the algorithm.
 * Space: orthonormal sine Galerkin basis with Gauss-Legendre quadrature (the weak form
 * and bilinear form a(w;u,v) of Section 2.1 evaluated with quadrature).
 *
 * Readings where the paper is silent or ambiguous (each repeated in the design notes):
 *   - every L1 history sum is evaluated in difference form, sum b * (y_i - y_{i-1}),
 *     as in the first line of the hybrid L1 formula; this equals the expanded form;
 *   - the coarse history is empty for n = 0 (the expanded fine formula is only valid
 *     for n >= 1);
 *   - D and f are lagged to the previous fine (or coarse) time level and state;
 *   - the parareal update is evaluated as F_old + (G_new - G_old);
 *   - fine time levels are t_m = T*m/N with the global fine index m = n*S + r.
 * Plain loops, no blocking and no reordering beyond these definitions.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_PI 3.14159265358979323846

/* ---------------------------------------------------------------- validation */

static int f_is_u_independent(int f_sel) {
  return f_sel == 0 || f_sel == 1 || f_sel == 4 || f_sel == 5;
}

int oracle_validate(const oracle_problem* p) {
  if (!p) return -1;
  if (p->dim != 1 && p->dim != 2) return -1;
  if (p->modes < 1 || p->quad < p->modes) return -1;
  if (p->steps < 1 || p->slices < 1 || p->steps % p->slices != 0) return -1;
  if (!(p->alpha > 0.0 && p->alpha <= 1.0)) return -1;
  if (!(p->T > 0.0)) return -1;
  if (p->d_sel < -1 || p->d_sel > 4) return -1;
  if (p->d_sel == 0 && !(p->d_param > 0.0)) return -1;
  if (p->f_sel < 0 || p->f_sel > 5) return -1;
  if (p->history < 0 || p->history > 2) return -1;
  if (p->source_time != 0 && p->source_time != 1) return -1;
  if (p->source_time == 1 && !f_is_u_independent(p->f_sel)) return -1;
  if (p->solver < 0 || p->solver > 2) return -1;
  if (p->solver == 2 && p->d_sel != 0) return -1;
  return 0;
}

static int nmodes(const oracle_problem* p) {
  return p->dim == 1 ? p->modes : p->modes * p->modes;
}

/* Fine time level t_m = T*m/N (m is the global fine index). */
static double t_fine(const oracle_problem* p, long m) {
  return (p->T * (double)m) / (double)p->steps;
}

/* ------------------------------------------------------------------- weights */

/* b_x = (x+1)^(1-alpha) - x^(1-alpha) (L1 scheme weights, Section 2.1, evaluated at
   integer x for the uniform scheme and at x = m + r/S for the hybrid operator of
   Section 2.2).  b_0 = 1 for every alpha, including alpha = 1 where pow(0,0) would
   otherwise give 0.  For x > 0 the same quantity is written as
   x^(1-alpha) * (exp((1-alpha) log(1 + 1/x)) - 1), which avoids the cancellation of
   two nearly equal powers at large x. */
double oracle_bweight(double x, double alpha) {
  if (x == 0.0) return 1.0;
  double e = 1.0 - alpha;
  return pow(x, e) * expm1(e * log1p(1.0 / x));
}

/* Sum-of-exponentials weights (see oracle.h): the integral form of b_j, the trapezoid rule
   in y = log(s) on the grid n h, the slow end merged, the fast end dropped. */
int32_t oracle_soe_nodes(double alpha, int32_t N, double* lam, double* w, int32_t max_nodes) {
  if (!(alpha > 0.0 && alpha < 1.0) || N < 1) return -1;
  const double h = ORACLE_SOE_H, g = tgamma(alpha), c = h * (1.0 - alpha) / g;
  /* dropped nodes: exp(-lam j0) <= e^-40 once lam >= 40 / j0 */
  const int n_hi = (int)ceil(log(40.0 / ORACLE_SOE_J0) / h);
  /* merged nodes n < n_lo: sum_n w_n (1 - exp(-lam_n j)) <= j c sum_n e^{(alpha+1) n h}
     <= eps b_j for j <= N, with b_j >= (1-alpha) (j+1)^-alpha */
  const double t = log(ORACLE_SOE_EPS * g * (1.0 - exp(-(alpha + 1.0) * h)) /
                       (h * (double)N * pow((double)N + 1.0, alpha))) / (alpha + 1.0);
  const int n_lo = (int)floor(t / h) + 1;
  const int count = n_hi - n_lo + 2;
  if (count > max_nodes) return -1;
  lam[0] = 0.0;
  w[0] = c * exp(alpha * (double)(n_lo - 1) * h) / (1.0 - exp(-alpha * h));
  for (int n = n_lo; n <= n_hi; n++) {
    const double y = (double)n * h, l = exp(y);
    lam[n - n_lo + 1] = l;
    w[n - n_lo + 1] = c * exp((alpha - 1.0) * y) * (-expm1(-l));
  }
  return count;
}

/* ---------------------------------------------------------------- quadrature */

/* Gauss-Legendre rule mapped from (-1,1) to (0,1): nodes are the roots of the
   Legendre polynomial P_Q found by Newton's method on the three-term recurrence;
   weights 2/((1-z^2) P_Q'(z)^2), halved by the map. */
void oracle_gauss_legendre01(int32_t Q, double* x, double* w) {
  for (int i = 0; i < Q; i++) {
    double z = cos(ORACLE_PI * (i + 0.75) / (Q + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; it++) {
      double p0 = 1.0, p1 = z;
      for (int j = 2; j <= Q; j++) {
        double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      dp = Q * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (fabs(dz) < 1e-15 && it > 2) break;
    }
    /* derivative at the converged root */
    {
      double p0 = 1.0, p1 = z;
      for (int j = 2; j <= Q; j++) {
        double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      dp = Q * (z * p1 - p0) / (z * z - 1.0);
    }
    x[i] = 0.5 * (1.0 - z);
    w[i] = 1.0 / ((1.0 - z * z) * dp * dp);
  }
}

/* ------------------------------------------------------------- coefficients */

double oracle_D(const oracle_problem* p, double x, double y, double t, double u) {
  (void)x; (void)y; (void)t;
  switch (p->d_sel) {
    case -1: return 0.0;                                  /* test hook: no diffusion */
    case 0:  return p->d_param;                           /* constant */
    case 1:  { double s = sin(u); return 1.0 + 0.5 * s * s; }
    case 2:  return 1.0 + 1.0 / (1.0 + u * u);
    case 3:  return 1.0 + 0.5 * exp(-u * u);
    case 4:  return 1.0 + u;                              /* the paper's model problem */
  }
  return 0.0;
}

/* sin(pi x) in 1D, sin(pi x) sin(pi y) in 2D */
static double shape(const oracle_problem* p, double x, double y) {
  double s = sin(ORACLE_PI * x);
  if (p->dim == 2) s *= sin(ORACLE_PI * y);
  return s;
}

double oracle_f(const oracle_problem* p, double x, double y, double t, double u) {
  const double pi = ORACLE_PI;
  double a = p->alpha;
  switch (p->f_sel) {
    case 0: return 0.0;
    case 1: {
      /* Manufactured source for U = (1 + t^alpha) s(x,y) with D(u) = 1 + sin(u)^2/2.
         The Caputo derivative of t^alpha is Gamma(1+alpha), so
         f = Gamma(1+alpha) s - D(U) lap U - D'(U) |grad U|^2. */
      double A = 1.0 + pow(t, a);
      double s = shape(p, x, y);
      double U = A * s;
      double sU = sin(U);
      double DU = 1.0 + 0.5 * sU * sU;
      double dDU = 0.5 * sin(2.0 * U);
      double lap = -(double)p->dim * pi * pi * U;
      double g2;
      if (p->dim == 1) {
        double cx = cos(pi * x);
        g2 = A * A * pi * pi * cx * cx;
      } else {
        double sx = sin(pi * x), cx = cos(pi * x), sy = sin(pi * y), cy = cos(pi * y);
        g2 = A * A * pi * pi * (cx * cx * sy * sy + sx * sx * cy * cy);
      }
      return tgamma(1.0 + a) * s - DU * lap - dDU * g2;
    }
    case 2: return 0.1 * u * (1.0 - u);
    case 3: return sin(u);
    case 4: return shape(p, x, y) * exp(-t);              /* the paper's model problem */
    case 5: {
      /* Smooth manufactured source for U = (1 + t^2) s(x,y) with constant D = d_param:
         the Caputo derivative of t^2 is 2 t^(2-alpha) / Gamma(3-alpha). */
      double s = shape(p, x, y);
      return (2.0 * pow(t, 2.0 - a) / tgamma(3.0 - a) +
              (double)p->dim * p->d_param * pi * pi * (1.0 + t * t)) * s;
    }
  }
  return 0.0;
}

/* ------------------------------------------------------------------- Galerkin */

/* Basis values and gradients at (X,Y) for all Md functions. */
static void basis_at(const oracle_problem* p, double X, double Y, double* val, double* gx,
                     double* gy) {
  const double pi = ORACLE_PI;
  int M = p->modes;
  if (p->dim == 1) {
    for (int k = 0; k < M; k++) {
      double kp = (k + 1) * pi;
      val[k] = sqrt(2.0) * sin(kp * X);
      gx[k] = sqrt(2.0) * kp * cos(kp * X);
      gy[k] = 0.0;
    }
  } else {
    for (int k1 = 0; k1 < M; k1++) {
      for (int k2 = 0; k2 < M; k2++) {
        int k = k1 * M + k2;
        double a1 = (k1 + 1) * pi, a2 = (k2 + 1) * pi;
        val[k] = 2.0 * sin(a1 * X) * sin(a2 * Y);
        gx[k] = 2.0 * a1 * cos(a1 * X) * sin(a2 * Y);
        gy[k] = 2.0 * a2 * sin(a1 * X) * cos(a2 * Y);
      }
    }
  }
}

/* K_kl = sum_q w_q D(x_q, tD, u_q) grad phi_k(x_q) . grad phi_l(x_q)   (bilinear form a)
   F_k  = sum_q w_q f(x_q, tf, u_q) phi_k(x_q)                          (load (f, chi))
   u_q  = sum_k c_k phi_k(x_q). */
int oracle_galerkin(const oracle_problem* p, const double* c, double tD, double tf,
                    double* K, double* F) {
  if (oracle_validate(p)) return -1;
  int Q = p->quad, Md = nmodes(p);
  double* xq = (double*)malloc(sizeof(double) * Q);
  double* wq = (double*)malloc(sizeof(double) * Q);
  double* val = (double*)malloc(sizeof(double) * Md);
  double* gx = (double*)malloc(sizeof(double) * Md);
  double* gy = (double*)malloc(sizeof(double) * Md);
  oracle_gauss_legendre01(Q, xq, wq);
  memset(K, 0, sizeof(double) * (size_t)Md * Md);
  memset(F, 0, sizeof(double) * Md);
  int Q2 = p->dim == 1 ? 1 : Q;
  for (int q1 = 0; q1 < Q; q1++) {
    for (int q2 = 0; q2 < Q2; q2++) {
      double X = xq[q1];
      double Y = p->dim == 1 ? 0.0 : xq[q2];
      double W = p->dim == 1 ? wq[q1] : wq[q1] * wq[q2];
      basis_at(p, X, Y, val, gx, gy);
      double u = 0.0;
      for (int k = 0; k < Md; k++) u += c[k] * val[k];
      double Dq = oracle_D(p, X, Y, tD, u);
      double fq = oracle_f(p, X, Y, tf, u);
      for (int k = 0; k < Md; k++) F[k] += W * fq * val[k];
      for (int k = 0; k < Md; k++) {
        double* Kk = K + (size_t)k * Md;
        double ak = W * Dq * gx[k], bk = W * Dq * gy[k];
        if (p->dim == 1) {
          for (int l = 0; l < Md; l++) Kk[l] += ak * gx[l];
        } else {
          for (int l = 0; l < Md; l++) Kk[l] += ak * gx[l] + bk * gy[l];
        }
      }
    }
  }
  free(xq); free(wq); free(val); free(gx); free(gy);
  return 0;
}

/* Selected rows of the same Galerkin sums: Krows[i][l] = K_{rows[i], l} for the nrows listed
   rows, and the whole load F.  Same quadrature points, same order and the same expressions
   per basis value as oracle_galerkin (the products of the separable factors are formed in
   the order basis_at forms them), so each row equals that row of oracle_galerkin bit for
   bit; the per-direction sines and cosines are evaluated once per point instead of once per
   basis function, which makes single rows affordable at large mode counts. */
int oracle_galerkin_rows(const oracle_problem* p, const double* c, double tD, double tf,
                         int32_t nrows, const int32_t* rows, double* Krows, double* F) {
  if (oracle_validate(p)) return -1;
  const double pi = ORACLE_PI;
  int Q = p->quad, Md = nmodes(p), M = p->modes;
  for (int i = 0; i < nrows; i++)
    if (rows[i] < 0 || rows[i] >= Md) return -1;
  double* xq = (double*)malloc(sizeof(double) * Q);
  double* wq = (double*)malloc(sizeof(double) * Q);
  double* val = (double*)malloc(sizeof(double) * Md);
  double* gx = (double*)malloc(sizeof(double) * Md);
  double* gy = (double*)malloc(sizeof(double) * Md);
  double* sx = (double*)malloc(sizeof(double) * M);
  double* cx = (double*)malloc(sizeof(double) * M);
  double* sy = (double*)malloc(sizeof(double) * M);
  double* cy = (double*)malloc(sizeof(double) * M);
  oracle_gauss_legendre01(Q, xq, wq);
  memset(Krows, 0, sizeof(double) * (size_t)nrows * Md);
  memset(F, 0, sizeof(double) * Md);
  int Q2 = p->dim == 1 ? 1 : Q;
  for (int q1 = 0; q1 < Q; q1++) {
    for (int q2 = 0; q2 < Q2; q2++) {
      double X = xq[q1];
      double Y = p->dim == 1 ? 0.0 : xq[q2];
      double W = p->dim == 1 ? wq[q1] : wq[q1] * wq[q2];
      if (p->dim == 1) {
        basis_at(p, X, Y, val, gx, gy);
      } else {
        for (int k = 0; k < M; k++) {
          double a = (k + 1) * pi;
          sx[k] = sin(a * X); cx[k] = cos(a * X);
          sy[k] = sin(a * Y); cy[k] = cos(a * Y);
        }
        for (int k1 = 0; k1 < M; k1++) {
          for (int k2 = 0; k2 < M; k2++) {
            int k = k1 * M + k2;
            double a1 = (k1 + 1) * pi, a2 = (k2 + 1) * pi;
            val[k] = 2.0 * sx[k1] * sy[k2];
            gx[k] = 2.0 * a1 * cx[k1] * sy[k2];
            gy[k] = 2.0 * a2 * sx[k1] * cy[k2];
          }
        }
      }
      double u = 0.0;
      for (int k = 0; k < Md; k++) u += c[k] * val[k];
      double Dq = oracle_D(p, X, Y, tD, u);
      double fq = oracle_f(p, X, Y, tf, u);
      for (int k = 0; k < Md; k++) F[k] += W * fq * val[k];
      for (int i = 0; i < nrows; i++) {
        int k = rows[i];
        double* Kk = Krows + (size_t)i * Md;
        double ak = W * Dq * gx[k], bk = W * Dq * gy[k];
        if (p->dim == 1) {
          for (int l = 0; l < Md; l++) Kk[l] += ak * gx[l];
        } else {
          for (int l = 0; l < Md; l++) Kk[l] += ak * gx[l] + bk * gy[l];
        }
      }
    }
  }
  free(xq); free(wq); free(val); free(gx); free(gy); free(sx); free(cx); free(sy); free(cy);
  return 0;
}

/* Gaussian elimination with partial pivoting; A (n x n, row-major) is destroyed and
   the solution overwrites b. */
static int solve_dense(int n, double* A, double* b) {
  for (int c = 0; c < n; c++) {
    int piv = c;
    double best = fabs(A[(size_t)c * n + c]);
    for (int r = c + 1; r < n; r++) {
      double v = fabs(A[(size_t)r * n + c]);
      if (v > best) { best = v; piv = r; }
    }
    if (best == 0.0) return -1;
    if (piv != c) {
      for (int j = 0; j < n; j++) {
        double t = A[(size_t)c * n + j];
        A[(size_t)c * n + j] = A[(size_t)piv * n + j];
        A[(size_t)piv * n + j] = t;
      }
      double t = b[c]; b[c] = b[piv]; b[piv] = t;
    }
    for (int r = c + 1; r < n; r++) {
      double m = A[(size_t)r * n + c] / A[(size_t)c * n + c];
      if (m == 0.0) continue;
      for (int j = c; j < n; j++) A[(size_t)r * n + j] -= m * A[(size_t)c * n + j];
      b[r] -= m * b[c];
    }
  }
  for (int r = n - 1; r >= 0; r--) {
    double s = b[r];
    for (int j = r + 1; j < n; j++) s -= A[(size_t)r * n + j] * b[j];
    b[r] = s / A[(size_t)r * n + r];
  }
  return 0;
}

/* Eigenvalue of -Laplace for basis function k (Dirichlet sine basis): (k pi)^2 in 1D,
   (k1^2 + k2^2) pi^2 in 2D for k = (k1-1) M + (k2-1). */
static double sine_eigenvalue(const oracle_problem* p, int k) {
  const double pi = ORACLE_PI;
  if (p->dim == 1) return (double)(k + 1) * (double)(k + 1) * pi * pi;
  double k1 = (double)(k / p->modes + 1), k2 = (double)(k % p->modes + 1);
  return (k1 * k1 + k2 * k2) * pi * pi;
}

/* One semi-implicit L1-Galerkin step (Section 2.1 and Section 2.2): the diffusion
   coefficient and the source are taken at the previous level (c_prev), the gradient
   term at the new level:  (I + tau K) c = hist + tau F.
   solver = 2 (constant D, the spectral diagonalisation named among the paper's outlook
   items in its conclusions): a(phi_k, phi_l) = D (grad phi_k, grad phi_l) = D lambda_k
   delta_kl exactly for the orthonormal sine basis, so c_k = (hist_k + tau F_k) /
   (1 + tau D lambda_k); the load F is still the quadrature sum. */
int oracle_step(const oracle_problem* p, const double* c_prev, double tD, double tf,
                const double* hist, double tau, double* c_out) {
  if (oracle_validate(p)) return -1;
  int Md = nmodes(p);
  double* K = (double*)malloc(sizeof(double) * (size_t)Md * Md);
  double* F = (double*)malloc(sizeof(double) * Md);
  oracle_galerkin(p, c_prev, tD, tf, K, F);
  if (p->solver == 2) {
    for (int k = 0; k < Md; k++)
      c_out[k] = (hist[k] + tau * F[k]) / (1.0 + tau * p->d_param * sine_eigenvalue(p, k));
    free(K); free(F);
    return 0;
  }
  for (int k = 0; k < Md; k++) {
    for (int l = 0; l < Md; l++) K[(size_t)k * Md + l] *= tau;
    K[(size_t)k * Md + k] += 1.0;
    c_out[k] = hist[k] + tau * F[k];
  }
  int rc = solve_dense(Md, K, c_out);
  free(K); free(F);
  return rc;
}

/* ------------------------------------------------------------- propagators */

static double tau_of(const oracle_problem* p, double step) {
  return pow(step, p->alpha) * tgamma(2.0 - p->alpha);
}

/* Coarse propagator G_n (Section 2.1, sequential scheme with step dT = T/P):
   (I + tau_c K(C_n)) C_{n+1} = C_n - sum_{i=1}^{n} b_{n+1-i} (C_i - C_{i-1}) + tau_c F(C_n),
   which is the L1 scheme b_n C_0 + sum (b_{n-i} - b_{n-i+1}) C_i written in difference
   form.  D and f at (T_n, C_n). */
int oracle_coarse_G(const oracle_problem* p, int32_t n, const double* C, double* out) {
  if (oracle_validate(p)) return -1;
  int Md = nmodes(p), S = p->steps / p->slices;
  double tau_c = tau_of(p, p->T / (double)p->slices);
  double* hist = (double*)malloc(sizeof(double) * Md);
  for (int k = 0; k < Md; k++) {
    double acc = 0.0;
    for (int i = 1; i <= n; i++)
      acc += oracle_bweight((double)(n + 1 - i), p->alpha) *
             (C[(size_t)i * Md + k] - C[(size_t)(i - 1) * Md + k]);
    hist[k] = C[(size_t)n * Md + k] - acc;
  }
  double tD = t_fine(p, (long)n * S);
  double tf = p->source_time ? t_fine(p, (long)(n + 1) * S) : tD;
  int rc = oracle_step(p, C + (size_t)n * Md, tD, tf, hist, tau_c, out);
  free(hist);
  return rc;
}

/* Fine propagator F_n (Section 2.2): S steps of size dt = dT/S on [T_n, T_{n+1}]
   starting from c_0 = C_n.  The Caputo derivative at t_{n,r} uses the fine grid on
   [T_n, t_{n,r}] and the coarse grid on [0, T_n]; multiplied by tau = dt^a Gamma(2-a):
     c_r + tau K(c_{r-1}) c_r = c_{r-1} - sum_{j=1}^{r-1} b_{r-j} (c_j - c_{j-1})
                               - S^{-a} sum_{i=1}^{n} b_{n-i+r/S} (C_i - C_{i-1})
                               + tau F(c_{r-1}),
   with D and f at (t_{n,r-1}, c_{r-1}). */
int oracle_fine_F(const oracle_problem* p, int32_t n, const double* C, double* out,
                  double* traj) {
  if (oracle_validate(p)) return -1;
  int Md = nmodes(p), S = p->steps / p->slices;
  double a = p->alpha;
  double tau = tau_of(p, p->T / (double)p->steps);
  double sfac = pow((double)S, -a);
  double* c = (double*)malloc(sizeof(double) * (size_t)(S + 1) * Md);
  double* hist = (double*)malloc(sizeof(double) * Md);
  memcpy(c, C + (size_t)n * Md, sizeof(double) * Md);
  int rc = 0;
  for (int r = 1; r <= S && rc == 0; r++) {
    for (int k = 0; k < Md; k++) {
      double fine = 0.0;
      for (int j = 1; j <= r - 1; j++)
        fine += oracle_bweight((double)(r - j), a) *
                (c[(size_t)j * Md + k] - c[(size_t)(j - 1) * Md + k]);
      double coarse = 0.0;
      for (int i = 1; i <= n; i++) {
        double x = (double)((long)(n - i) * S + r) / (double)S;   /* n - i + r/S */
        coarse += oracle_bweight(x, a) * (C[(size_t)i * Md + k] - C[(size_t)(i - 1) * Md + k]);
      }
      double h = c[(size_t)(r - 1) * Md + k] - fine;
      hist[k] = h - sfac * coarse;
    }
    long m = (long)n * S + r - 1;
    double tD = t_fine(p, m);
    double tf = p->source_time ? t_fine(p, m + 1) : tD;
    rc = oracle_step(p, c + (size_t)(r - 1) * Md, tD, tf, hist, tau, c + (size_t)r * Md);
  }
  if (rc == 0) {
    memcpy(out, c + (size_t)S * Md, sizeof(double) * Md);
    if (traj) memcpy(traj, c, sizeof(double) * (size_t)(S + 1) * Md);
  }
  free(c); free(hist);
  return rc;
}

/* ------------------------------------------------------------------ solvers */

/* Serial solve.  history = 0: C_{n+1} = F_n(C_0..C_n), the fine solution that is the
   fixed point of parareal (Section 2.2).  history = 1: the uniform L1 scheme over all
   N fine steps with full fine history.  history = 2: the same scheme with the history terms
   at distances >= ORACLE_SOE_J0 from the sum-of-exponentials weights (an approximation,
   Conclusions (i); at alpha = 1 the far weights vanish and it is history = 1). */
int oracle_solve_serial(const oracle_problem* p, const double* u0, double* U, double* traj) {
  if (oracle_validate(p)) return -1;
  int Md = nmodes(p), P = p->slices, N = p->steps, S = N / P;
  int rc = 0;
  if (p->history == 0) {
    memcpy(U, u0, sizeof(double) * Md);
    double* tr = (double*)malloc(sizeof(double) * (size_t)(S + 1) * Md);
    if (traj) memcpy(traj, u0, sizeof(double) * Md);
    for (int n = 0; n < P && rc == 0; n++) {
      rc = oracle_fine_F(p, n, U, U + (size_t)(n + 1) * Md, tr);
      if (rc == 0 && traj)
        memcpy(traj + ((size_t)n * S + 1) * Md, tr + Md, sizeof(double) * (size_t)S * Md);
    }
    free(tr);
    return rc;
  }
  double tau = tau_of(p, p->T / (double)N);
  double* c = (double*)malloc(sizeof(double) * (size_t)(N + 1) * Md);
  double* hist = (double*)malloc(sizeof(double) * Md);
  memcpy(c, u0, sizeof(double) * Md);
  /* history = 2: the weights at distances d >= j0 as a sum of exponentials (oracle.h); for
     each mode the exponential sums V_l = sum_{i <= m+1-j0} exp(-lam_l (m+1-i)) (c_i - c_{i-1})
     are carried from step to step, V_l <- exp(-lam_l) V_l + exp(-lam_l j0) (c_i - c_{i-1})
     with i = m+1-j0 the row that has just reached distance j0 */
  const int soe = p->history == 2 && p->alpha < 1.0;
  enum { SOE_MAX = 512 };
  double lam[SOE_MAX], wl[SOE_MAX];
  int L = 0;
  double* V = NULL;
  if (soe) {
    L = oracle_soe_nodes(p->alpha, N, lam, wl, SOE_MAX);
    if (L < 0) rc = -1;
    V = (double*)calloc((size_t)(L > 0 ? L : 1) * Md, sizeof(double));
  }
  const int j0 = ORACLE_SOE_J0;
  for (int m = 0; m < N && rc == 0; m++) {
    for (int k = 0; k < Md; k++) {
      double acc = 0.0;
      if (!soe) {
        for (int i = 1; i <= m; i++)
          acc += oracle_bweight((double)(m + 1 - i), p->alpha) *
                 (c[(size_t)i * Md + k] - c[(size_t)(i - 1) * Md + k]);
      } else {
        const int inew = m + 1 - j0;
        if (inew >= 1) {
          const double d = c[(size_t)inew * Md + k] - c[(size_t)(inew - 1) * Md + k];
          for (int l = 0; l < L; l++)
            V[(size_t)l * Md + k] = exp(-lam[l]) * V[(size_t)l * Md + k] + exp(-lam[l] * j0) * d;
        }
        double far = 0.0;
        for (int l = 0; l < L; l++) far += wl[l] * V[(size_t)l * Md + k];
        double near = 0.0;
        for (int i = (inew + 1 > 1 ? inew + 1 : 1); i <= m; i++)
          near += oracle_bweight((double)(m + 1 - i), p->alpha) *
                  (c[(size_t)i * Md + k] - c[(size_t)(i - 1) * Md + k]);
        acc = far + near;
      }
      hist[k] = c[(size_t)m * Md + k] - acc;
    }
    double tD = t_fine(p, m);
    double tf = p->source_time ? t_fine(p, m + 1) : tD;
    rc = oracle_step(p, c + (size_t)m * Md, tD, tf, hist, tau, c + (size_t)(m + 1) * Md);
  }
  if (rc == 0) {
    for (int n = 0; n <= P; n++)
      memcpy(U + (size_t)n * Md, c + (size_t)n * S * Md, sizeof(double) * Md);
    if (traj) memcpy(traj, c, sizeof(double) * (size_t)(N + 1) * Md);
  }
  free(c); free(hist); free(V);
  return rc;
}

/* Full-history fine propagator (the full-history variant of parareal; not in the paper, whose
   fine step uses the coarse grid for the history before the slice).  S fine steps on
   [T_n, T_{n+1}] from c_0 = C_n with the uniform L1 history over the whole fine grid:
     c_r + tau K(c_{r-1}) c_r = c_{m} - sum_{j=1}^{m} b_{m+1-j} (x_j - x_{j-1}) + tau F(c_{r-1}),
   m = nS + r - 1, where x_j is the current slice's own state for j >= nS (x_{nS} = C_n) and,
   before it, the fine trajectory of the previous parareal iterate: prev [P][S+1][Md] holds,
   for every slice q, the states at its fine levels 0..S, and x_j = prev[q][j - qS] with
   q = (j-1)/S for 1 <= j < nS, x_0 = prev[0][0] (= u0).  Writes the slice's states to
   slot_out [S+1][Md] and its end to out. */
static int fine_F_full(const oracle_problem* p, int n, const double* C, const double* prev,
                       double* out, double* slot_out) {
  int Md = nmodes(p), S = p->steps / p->slices;
  double a = p->alpha;
  double tau = tau_of(p, p->T / (double)p->steps);
  double* c = slot_out;
  double* hist = (double*)malloc(sizeof(double) * Md);
  memcpy(c, C + (size_t)n * Md, sizeof(double) * Md);
  long nS = (long)n * S;
  int rc = 0;
  for (int r = 1; r <= S && rc == 0; r++) {
    long m = nS + r - 1;
    for (int k = 0; k < Md; k++) {
      double acc = 0.0;
      double xprev = (n == 0) ? c[k] : prev[k];
      for (long j = 1; j <= m; j++) {
        double xj;
        if (j >= nS) {
          xj = c[(size_t)(j - nS) * Md + k];
        } else {
          long q = (j - 1) / S;
          xj = prev[((size_t)q * (S + 1) + (size_t)(j - q * S)) * Md + k];
        }
        acc += oracle_bweight((double)(m + 1 - j), a) * (xj - xprev);
        xprev = xj;
      }
      hist[k] = c[(size_t)(r - 1) * Md + k] - acc;
    }
    double tD = t_fine(p, m);
    double tf = p->source_time ? t_fine(p, m + 1) : tD;
    rc = oracle_step(p, c + (size_t)(r - 1) * Md, tD, tf, hist, tau, c + (size_t)r * Md);
  }
  if (rc == 0) memcpy(out, c + (size_t)S * Md, sizeof(double) * Md);
  free(hist);
  return rc;
}

/* Parareal (Section 2.2 and its flowchart); history = 1 runs the full-history variant (fine
   propagator fine_F_full above, fixed point the uniform L1 solution of oracle_solve_serial
   with history = 1).  Initial coarse sweep
   U^0_{n+1} = G_n(U^0_0..U^0_n); then for k = 0, 1, ...:
     parallel stage:   G_old(n) = G_n(U^k_0..U^k_n),  F_old(n) = F_n(U^k_0..U^k_n);
     sequential sweep: G_new(n) = G_n(U^{k+1}_0..U^{k+1}_n),
                       U^{k+1}_{n+1} = F_old(n) + (G_new(n) - G_old(n)),  U^{k+1}_0 = u_0;
   stop after P sweeps (all slice ends then equal the serial solution), after
   max_iter sweeps, or when ||U^{k+1} - U^k|| <= tol ||U^{k+1}|| (tol > 0). */
int oracle_solve_parareal(const oracle_problem* p, const double* u0, double* U,
                          int32_t max_iter, double tol, double* U_iters, double* incr,
                          int32_t* iters) {
  if (oracle_validate(p) || max_iter < 0 || p->history == 2) return -1;
  int Md = nmodes(p), P = p->slices, S = p->steps / p->slices;
  int full = p->history == 1;
  size_t V = (size_t)(P + 1) * Md;
  double* Uk = (double*)malloc(sizeof(double) * V);
  double* Uk1 = (double*)malloc(sizeof(double) * V);
  double* Gold = (double*)malloc(sizeof(double) * (size_t)P * Md);
  double* Fold = (double*)malloc(sizeof(double) * (size_t)P * Md);
  double* Gnew = (double*)malloc(sizeof(double) * Md);
  int rc = 0, done = 0;
  memcpy(Uk, u0, sizeof(double) * Md);
  for (int n = 0; n < P && rc == 0; n++) rc = oracle_coarse_G(p, n, Uk, Uk + (size_t)(n + 1) * Md);
  if (U_iters) memcpy(U_iters, Uk, sizeof(double) * V);
  /* full history: the previous iterate's fine trajectory, slot by slot; before the first
     sweep the linear interpolation of the coarse iterate over each slice */
  size_t slotsz = (size_t)(S + 1) * Md;
  double* prev = full ? (double*)malloc(sizeof(double) * (size_t)P * slotsz) : NULL;
  double* cur = full ? (double*)malloc(sizeof(double) * (size_t)P * slotsz) : NULL;
  if (full)
    for (int q = 0; q < P; q++)
      for (int t = 0; t <= S; t++)
        for (int k = 0; k < Md; k++) {
          double a0 = Uk[(size_t)q * Md + k], a1 = Uk[(size_t)(q + 1) * Md + k];
          prev[(size_t)q * slotsz + (size_t)t * Md + k] = a0 + ((double)t / (double)S) * (a1 - a0);
        }
  for (int k = 0; k < max_iter && rc == 0; k++) {
    for (int n = 0; n < P && rc == 0; n++) {
      rc = oracle_coarse_G(p, n, Uk, Gold + (size_t)n * Md);
      if (rc == 0)
        rc = full ? fine_F_full(p, n, Uk, prev, Fold + (size_t)n * Md, cur + (size_t)n * slotsz)
                  : oracle_fine_F(p, n, Uk, Fold + (size_t)n * Md, NULL);
    }
    if (full) {
      double* t = prev;
      prev = cur;
      cur = t;
    }
    memcpy(Uk1, u0, sizeof(double) * Md);
    for (int n = 0; n < P && rc == 0; n++) {
      rc = oracle_coarse_G(p, n, Uk1, Gnew);
      for (int j = 0; j < Md; j++)
        Uk1[(size_t)(n + 1) * Md + j] =
            Fold[(size_t)n * Md + j] + (Gnew[j] - Gold[(size_t)n * Md + j]);
    }
    double dn = 0.0, un = 0.0;
    for (size_t i = 0; i < V; i++) {
      double d = Uk1[i] - Uk[i];
      dn += d * d;
      un += Uk1[i] * Uk1[i];
    }
    double rel = un > 0.0 ? sqrt(dn) / sqrt(un) : sqrt(dn);
    if (incr) incr[k] = rel;
    memcpy(Uk, Uk1, sizeof(double) * V);
    if (U_iters) memcpy(U_iters + (size_t)(k + 1) * V, Uk, sizeof(double) * V);
    done = k + 1;
    if (done >= P) break;
    if (tol > 0.0 && rel <= tol) break;
  }
  if (rc == 0) memcpy(U, Uk, sizeof(double) * V);
  if (iters) *iters = done;
  free(Uk); free(Uk1); free(Gold); free(Fold); free(Gnew); free(prev); free(cur);
  return rc;
}
