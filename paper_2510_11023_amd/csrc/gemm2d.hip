// Two-dimensional steps (tensor sine basis phi_k1(x) phi_k2(y), coefficients as an M x M
// matrix C with C[k1][k2] = c_{k1 M + k2}).  Everything separable is a batched dense product:
//   U  = Phi C Phi^T                 lagged state at the Q x Q Gauss points  (then D, f)
//   F  = Phi^T G Phi                 load vector, G[q1][q2] = w_q1 w_q2 f
//   m  = Cx^T Dw Cx                  cosine moments m(a, b) = sum_q w w D cos(a pi x) cos(b pi y)
// and the stiffness comes from the moments term by term (product-to-sum identities of the
// sine basis; the same quadrature sum as the bilinear form of the weak problem):
//   K_{(K1 K2),(L1 L2)} = K1 L1 pi^2 [m(d1,d2) - m(d1,s2) + m(s1,d2) - m(s1,s2)]
//                       + K2 L2 pi^2 [m(d1,d2) + m(d1,s2) - m(s1,d2) - m(s1,s2)],
// with 1-based mode numbers, d = |K - L| and s = K + L per direction.
#include "l1pr_internal.h"

namespace l1pr {

typedef double d4 __attribute__((ext_vector_type(4)));

// Element (i, k) of unit u's operand: p[u*su + i*ld + k], or p[u*su + k*ld + i] if trans.
struct BOp {
  const double* p;
  long ld, su;
  int trans;
};

enum { BG_STORE = 0, BG_EVAL2D = 1 };

constexpr int BT = 64, BK = 16;

// C[u] = A[u] B[u] (m x n, inner dimension kd); one 64 x 64 tile per work-group, four waves
// with 2 x 2 FP64 MFMA 16x16x4 tiles each, operands staged through LDS in chunks of 16.
// Each output is a fixed-order sum over its own row and column.  BG_EVAL2D: the product is
// the lagged state u at (x_i, x_j); the epilogue writes d = w_i w_j D and g = w_i w_j f.
__global__ __launch_bounds__(256) void k_bgemm(BOp A, BOp B, double* C, long ldc, long sc, int m,
                                               int n, int kd, int epi, Tables tb, StepArgs a,
                                               double* gout) {
  __shared__ double sA[BT][BK + 1];
  __shared__ double sB[BK][BT + 1];
  const int u = blockIdx.z, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  const int i0 = blockIdx.y * BT, j0 = blockIdx.x * BT;
  const double* Ap = A.p + (long)u * A.su;
  const double* Bp = B.p + (long)u * B.su;
  d4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = d4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < kd; k0 += BK) {
    for (int e = tid; e < BT * BK; e += 256) {
      const int r = e / BK, kk = e % BK;
      const int i = i0 + r, k = k0 + kk;
      double v = 0.0;
      if (i < m && k < kd) v = A.trans ? Ap[(long)k * A.ld + i] : Ap[(long)i * A.ld + k];
      sA[r][kk] = v;
    }
    for (int e = tid; e < BK * BT; e += 256) {
      const int kk = e / BT, c = e % BT;
      const int j = j0 + c, k = k0 + kk;
      sB[kk][c] = (j < n && k < kd) ? Bp[(long)k * B.ld + j] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      const int kq = ks * 4 + (lane >> 4);
      double af[2], bf[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) af[x] = sA[wi * 32 + x * 16 + (lane & 15)][kq];
#pragma unroll
      for (int y = 0; y < 2; ++y) bf[y] = sB[kq][wj * 32 + y * 16 + (lane & 15)];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[x], bf[y], acc[x][y], 0, 0, 0);
    }
    __syncthreads();
  }
  double tD = 0.0, tf = 0.0;
  const double* ins = nullptr;
  if (epi == BG_EVAL2D) {
    const UnitView v = decode_unit(tb, a, u);
    ins = tb.inst + (long)v.b * NSCAL;
    tD = t_level(tb, v.m_prev, v.Nb);
    tf = tb.source_time ? t_level(tb, v.m_src, v.Nb) : tD;
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + wi * 32 + x * 16 + (lane >> 4) + 4 * v;
      if (i >= m) continue;
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        const int j = j0 + wj * 32 + y * 16 + (lane & 15);
        if (j >= n) continue;
        const double val = acc[x][y][v];
        const long o = (long)u * sc + (long)i * ldc + j;
        if (epi == BG_STORE) {
          C[o] = val;
        } else {
          const double w = tb.wq[i] * tb.wq[j], X = tb.xq[i], Y = tb.xq[j];
          C[o] = w * coef_D(tb.d_sel, tb.d_param, val);
          gout[o] = w * coef_f(tb, ins, X, Y, tf, val);
        }
      }
    }
}

hipError_t bgemm(const BOp& A, const BOp& B, double* C, long ldc, long sc, int m, int n, int kd,
                 int units, int epi, const Tables& tb, const StepArgs& a, double* gout,
                 hipStream_t s) {
  dim3 grid((n + BT - 1) / BT, (m + BT - 1) / BT, units);
  k_bgemm<<<grid, 256, 0, s>>>(A, B, C, ldc, sc, m, n, kd, epi, tb, a, gout);
  return hipGetLastError();
}

// Lagged states of the units into a dense [units][Mp] buffer.
__global__ void k_gather_lag(Tables tb, StepArgs a, int units, double* out) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)units * tb.Mp) return;
  const int u = (int)(idx / tb.Mp), k = (int)(idx % tb.Mp);
  const UnitView v = decode_unit(tb, a, u);
  out[idx] = v.y[(long)v.L * tb.Mp + k];
}

// A = I + tau K from the moments, lower 64 x 64 blocks (blocks on the diagonal whole);
// entries outside the instance's modes are identity.  grid (Mp/64 blocks, Mp/64, units).
__global__ __launch_bounds__(256) void k_assemble2d(Tables tb, StepArgs a, const double* mom,
                                                    int Jp, double* A) {
  const int bI = blockIdx.y, bJ = blockIdx.x, u = blockIdx.z;
  if (bJ > bI) return;
  const int Mp = tb.Mp, M1 = tb.M1;
  const UnitView v = decode_unit(tb, a, u);
  const double* ins = tb.inst + (long)v.b * NSCAL;
  const double tau = ins[v.tau_slot];
  const int Mb = (int)ins[IS_MB];
  const double* m = mom + (long)u * Jp * Jp;
  double* Au = A + (long)u * Mp * Mp;
  const double pi2 = kPi * kPi;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int k = bI * 64 + e / 64, l = bJ * 64 + e % 64;
    if (k >= Mp || l >= Mp) continue;
    double val = (k == l) ? 1.0 : 0.0;
    if (k < Mb && l < Mb) {
      const int K1 = k / M1 + 1, K2 = k % M1 + 1, L1 = l / M1 + 1, L2 = l % M1 + 1;
      const int d1 = K1 > L1 ? K1 - L1 : L1 - K1, s1 = K1 + L1;
      const int d2 = K2 > L2 ? K2 - L2 : L2 - K2, s2 = K2 + L2;
      const double mdd = m[(long)d1 * Jp + d2], mds = m[(long)d1 * Jp + s2];
      const double msd = m[(long)s1 * Jp + d2], mss = m[(long)s1 * Jp + s2];
      const double t1 = (double)(K1 * L1) * pi2 * (((mdd - mds) + msd) - mss);
      const double t2 = (double)(K2 * L2) * pi2 * (((mdd + mds) - msd) - mss);
      val += tau * (t1 + t2);
    }
    Au[(long)k * Mp + l] = val;
  }
}

// rhs = hist + tau F for k < Mb, 0 above (the device-memory factorisation reads it whole)
__global__ void k_form_rhs(Tables tb, StepArgs a, int units, const double* F, double* rhs) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)units * tb.Mp) return;
  const int u = (int)(idx / tb.Mp), k = (int)(idx % tb.Mp);
  const UnitView v = decode_unit(tb, a, u);
  const double* ins = tb.inst + (long)v.b * NSCAL;
  rhs[idx] = (k < (int)ins[IS_MB]) ? rhs[idx] + ins[v.tau_slot] * F[idx] : 0.0;
}

// The separable part of a 2D step for `units` units: d, g at the quadrature points, the
// load vector F and the cosine moments.  Scratch: C [units][Mp] (lagged states), T
// [units][Qp * Jp] (intermediate products).
hipError_t launch_step2d_products(const Tables& tb, const StepArgs& a, int units, double* Cbuf,
                                  double* T, double* mom, hipStream_t s, bool moments) {
  const int M1 = tb.M1, M1p = tb.M1p, Q = tb.Q, Qp = tb.Qp, Mp = tb.Mp;
  const int J = 2 * M1 + 1, Jp = 2 * M1p + 1;
  const long sT = (long)Qp * Jp, sQ = (long)Qp * Qp;
  const long n = (long)units * Mp;
  k_gather_lag<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(tb, a, units, Cbuf);
  hipError_t r = hipGetLastError();
  if (r != hipSuccess) return r;
  // T = C Phi^T : [M1][Q]
  r = bgemm(BOp{Cbuf, M1, Mp, 0}, BOp{tb.phiT, Qp, 0, 0}, T, Qp, sT, M1, Q, M1, units, BG_STORE,
            tb, a, nullptr, s);
  if (r != hipSuccess) return r;
  // u = Phi T : [Q][Q] -> d, g
  r = bgemm(BOp{tb.phi, M1p, 0, 0}, BOp{T, Qp, sT, 0}, a.d, Qp, sQ, Q, Q, M1, units, BG_EVAL2D, tb,
            a, a.g, s);
  if (r != hipSuccess) return r;
  // T = G Phi : [Q][M1];  F = Phi^T T : [M1][M1]
  r = bgemm(BOp{a.g, Qp, sQ, 0}, BOp{tb.phi, M1p, 0, 0}, T, M1p, sT, Q, M1, Q, units, BG_STORE, tb,
            a, nullptr, s);
  if (r != hipSuccess) return r;
  r = bgemm(BOp{tb.phiT, Qp, 0, 0}, BOp{T, M1p, sT, 0}, a.F, M1, Mp, M1, M1, Q, units, BG_STORE, tb,
            a, nullptr, s);
  if (r != hipSuccess || !moments) return r;
  // T = Dw Cy : [Q][J];  m = Cx^T T : [J][J]
  r = bgemm(BOp{a.d, Qp, sQ, 0}, BOp{tb.cosq, Jp, 0, 0}, T, Jp, sT, Q, J, Q, units, BG_STORE, tb, a,
            nullptr, s);
  if (r != hipSuccess) return r;
  return bgemm(BOp{tb.cosq, Jp, 0, 1}, BOp{T, Jp, sT, 0}, mom, Jp, (long)Jp * Jp, J, J, Q, units,
               BG_STORE, tb, a, nullptr, s);
}

// First half of K V for every unit (the stiffness without tau, as the quadrature sum of the
// bilinear form, separably): G = [Gx; Gy] = [dphi (V phi^T); phi (V dphi^T)] o (w w D)
// (2Qp x Qp: the x and y derivatives at the Gauss points times w_i w_j D_ij, zero at padding
// nodes).  One work-group per (direction, 64 x 64 tile of G, unit), both products in it:
// T = V B[:, tile columns] (B = phi^T or dphi^T, from the stacked table b12) into LDS, then
// G tile = A[tile rows] T (A = dphi or phi), FP64 MFMA 16x16x4 with 16-wide LDS chunks as in
// k_bgemm.  V holds the M1 x M1 coefficient matrix of each unit at stride Mp (M1 <= 64).  The
// second half, K V = dphi^T Gx phi + phi^T Gy dphi, is in the conjugate-gradient kernels.
__global__ __launch_bounds__(256) void k_stiff2d_grid(Tables tb, StepArgs a, const double* V,
                                                      double* G) {
  __shared__ double sA[BT][BK + 1];
  __shared__ double sB[BK][BT + 1];
  __shared__ double sT[BT][BT + 1];
  const int u = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  const int M1 = tb.M1, M1p = tb.M1p, Q = tb.Q, Qp = tb.Qp, nt = (Qp + BT - 1) / BT;
  const int dir = blockIdx.x / (nt * nt), ib = (blockIdx.x / nt) % nt, jb = blockIdx.x % nt;
  const int i0 = ib * BT, j0 = jb * BT;
  const double* Vu = V + (long)u * tb.Mp;
  const double* Am = dir == 0 ? tb.dphi : tb.phi;
  d4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = d4{0.0, 0.0, 0.0, 0.0};
  // T[k][c] = sum_l V[k][l] B[l][j0 + c]
  for (int l0 = 0; l0 < M1; l0 += BK) {
    for (int e = tid; e < BT * BK; e += 256) {
      const int rr = e / BK, kk = e % BK;
      sA[rr][kk] = (rr < M1 && l0 + kk < M1) ? Vu[rr * M1 + l0 + kk] : 0.0;
    }
    for (int e = tid; e < BK * BT; e += 256) {
      const int kk = e / BT, cc = e % BT;
      sB[kk][cc] = (l0 + kk < M1 && j0 + cc < Qp) ? tb.b12[(long)(l0 + kk) * 2 * Qp + dir * Qp + j0 + cc]
                                                  : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      const int kq = ks * 4 + (lane >> 4);
      double af[2], bf[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) af[x] = sA[wi * 32 + x * 16 + (lane & 15)][kq];
#pragma unroll
      for (int y = 0; y < 2; ++y) bf[y] = sB[kq][wj * 32 + y * 16 + (lane & 15)];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[x], bf[y], acc[x][y], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        sT[wi * 32 + x * 16 + (lane >> 4) + 4 * v][wj * 32 + y * 16 + (lane & 15)] = acc[x][y][v];
        acc[x][y][v] = 0.0;
      }
  __syncthreads();
  // G tile = A[i0 .., :M1] T
  for (int k0 = 0; k0 < M1; k0 += BK) {
    for (int e = tid; e < BT * BK; e += 256) {
      const int rr = e / BK, kk = e % BK;
      sA[rr][kk] = (i0 + rr < Qp && k0 + kk < M1) ? Am[(long)(i0 + rr) * M1p + k0 + kk] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      const int kq = ks * 4 + (lane >> 4);
      double af[2], bf[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) af[x] = sA[wi * 32 + x * 16 + (lane & 15)][kq];
#pragma unroll
      for (int y = 0; y < 2; ++y) bf[y] = sT[k0 + kq][wj * 32 + y * 16 + (lane & 15)];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[x], bf[y], acc[x][y], 0, 0, 0);
    }
    __syncthreads();
  }
  double* Gu = G + ((long)u * 2 + dir) * Qp * Qp;
  const double* dw = a.d + (long)u * Qp * Qp;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + wi * 32 + x * 16 + (lane >> 4) + 4 * v;
      if (i >= Qp) continue;
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        const int j = j0 + wj * 32 + y * 16 + (lane & 15);
        if (j >= Qp) continue;
        Gu[(long)i * Qp + j] = (i < Q && j < Q) ? acc[x][y][v] * dw[(long)i * Qp + j] : 0.0;
      }
    }
}

hipError_t launch_stiff2d_grid(const Tables& tb, const StepArgs& a, int units, const double* V,
                               double* G, hipStream_t s) {
  if (tb.M1 > BT) return hipErrorInvalidValue;
  const int nt = (tb.Qp + BT - 1) / BT;
  k_stiff2d_grid<<<dim3(2 * nt * nt, units), 256, 0, s>>>(tb, a, V, G);
  return hipGetLastError();
}

hipError_t launch_assemble2d(const Tables& tb, const StepArgs& a, int units, const double* mom,
                             hipStream_t s) {
  const int nb = (tb.Mp + 63) / 64;
  dim3 grid(nb, nb, units);
  k_assemble2d<<<grid, 256, 0, s>>>(tb, a, mom, 2 * tb.M1p + 1, a.A);
  return hipGetLastError();
}

// Constant D (solver = 2): the sine basis diagonalises the stiffness, D (grad phi_k, grad phi_l)
// = D lambda_k delta_kl with lambda_k = (k pi)^2 (1D) or (k1^2 + k2^2) pi^2 (2D), so the step is
// c_k = (rhs_k + tau F_k) / (1 + tau D lambda_k), rhs holding the history sums; one thread per
// coefficient, stored through the step's epilogue.
__global__ void k_diag_solve(Tables tb, StepArgs a, Epilogue ep, int units, const double* F,
                             const double* rhs) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)units * tb.Mp) return;
  const int u = (int)(idx / tb.Mp), k = (int)(idx % tb.Mp);
  const UnitView v = decode_unit(tb, a, u);
  const double* ins = tb.inst + (long)v.b * NSCAL;
  double x = 0.0;
  if (k < (int)ins[IS_MB]) {
    const double tau = ins[v.tau_slot];
    double lam;
    if (tb.dim == 1) {
      const double kp = (double)(k + 1) * kPi;
      lam = kp * kp;
    } else {
      const double k1 = (double)(k / tb.M1 + 1), k2 = (double)(k % tb.M1 + 1);
      lam = (k1 * k1 + k2 * k2) * (kPi * kPi);
    }
    x = (rhs[idx] + tau * F[idx]) / (1.0 + tau * (tb.d_param * lam));
  }
  const bool last = (a.mode == MODE_FINE) && (a.r == v.Sb);
  epi_store(a, ep, u, v.slot, last, k, x);
}

hipError_t launch_diag_solve(const Tables& tb, const StepArgs& a, const Epilogue& e, int units,
                             const double* F, hipStream_t s) {
  const long n = (long)units * tb.Mp;
  k_diag_solve<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(tb, a, e, units, F, a.rhs);
  return hipGetLastError();
}

hipError_t launch_form_rhs(const Tables& tb, const StepArgs& a, int units, hipStream_t s) {
  const long n = (long)units * tb.Mp;
  k_form_rhs<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(tb, a, units, a.F, a.rhs);
  return hipGetLastError();
}

}  // namespace l1pr
