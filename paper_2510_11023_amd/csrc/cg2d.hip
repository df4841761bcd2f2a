// Preconditioned conjugate gradients for the 2D step systems (I + tau K) c = rhs.
//
// K is applied separably at the Gauss points (launch_stiff2d_apply), never formed.  The
// preconditioner is the constant-coefficient operator I + tau Dbar pi^2 (k1^2 + k2^2), Dbar
// the quadrature mean of D: with D constant the sine basis diagonalises K (its eigenvalues
// are D pi^2 (k1^2 + k2^2)), so the preconditioned system has its spectrum in
// [min D / Dbar, max D / Dbar] up to quadrature effects, and CG contracts by about
// (sqrt(kappa) - 1) / (sqrt(kappa) + 1) per iteration.  The start is the lagged state (the new
// state differs from it by one time step).
//
// One 256-thread work-group per unit; the unit's vectors live in device memory between the
// stiffness products; dot products are fixed-order sums (per-thread strided sums, then a
// fixed tree), so a unit's iterates depend only on its own data.  Per-unit state in
// cgs[u][8]: rz = r.z, ||rhs||^2, status, Dbar, iteration count.  A unit stops (and is left
// untouched by later launches) once ||r|| <= 1e-14 ||rhs||.
#include "l1pr_internal.h"

namespace l1pr {

constexpr int CG_T = 256;
constexpr int CG_E = 16;  // entries per thread: Mp <= CG_T * CG_E = 4096
constexpr double CG_TOL2 = 1e-28;
enum { CG_RZ = 0, CG_BN = 1, CG_ST = 2, CG_DBAR = 3, CG_IT = 4, CG_NS = 8 };
constexpr double CG_ACTIVE = 0.0, CG_DONE = 1.0, CG_FAIL = 2.0;

__device__ inline double block_sum(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
#pragma unroll
  for (int s = CG_T / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// diagonal of the preconditioner at entry k < M1^2
__device__ inline double cg_pdiag(int k, int M1, double tau, double dbar) {
  const double K1 = (double)(k / M1 + 1), K2 = (double)(k % M1 + 1);
  return 1.0 + tau * dbar * (kPi * kPi) * (K1 * K1 + K2 * K2);
}

__global__ __launch_bounds__(CG_T) void k_cg_init(Tables tb, StepArgs a, const double* x0,
                                                  const double* kx, double* x, double* r,
                                                  double* p, double* cgs) {
  __shared__ double red[CG_T];
  const int u = blockIdx.x, tid = threadIdx.x, Mp = tb.Mp, Qp = tb.Qp, M1 = tb.M1;
  const UnitView v = decode_unit(tb, a, u);
  const double* ins = tb.inst + (long)v.b * NSCAL;
  const double tau = ins[v.tau_slot];
  const int Mb = M1 * M1;
  // Dbar = sum_ij w_i w_j D_ij over the Q x Q Gauss points (the weights of each direction sum
  // to 1; the padded rows and columns of a.d are not written)
  const double* dw = a.d + (long)u * Qp * Qp;
  const int Q = tb.Q;
  double sd = 0.0;
  for (int e = tid; e < Q * Q; e += CG_T) sd += dw[(long)(e / Q) * Qp + e % Q];
  const double dbar = block_sum(sd, red);
  const long o = (long)u * Mp;
  double bn = 0.0;
  for (int k = tid; k < Mp; k += CG_T) {
    const double b = a.rhs[o + k];
    bn += b * b;
  }
  bn = block_sum(bn, red);
  double rz = 0.0, rn = 0.0;
  for (int k = tid; k < Mp; k += CG_T) {
    double xk = 0.0, rk = 0.0, zk = 0.0;
    if (k < Mb && bn > 0.0) {
      xk = x0[o + k];
      rk = a.rhs[o + k] - (xk + tau * kx[o + k]);
      zk = rk / cg_pdiag(k, M1, tau, dbar);
    }
    x[o + k] = xk;
    r[o + k] = rk;
    p[o + k] = zk;
    rz += rk * zk;
    rn += rk * rk;
  }
  rz = block_sum(rz, red);
  rn = block_sum(rn, red);
  if (tid == 0) {
    double* cs = cgs + (long)u * CG_NS;
    cs[CG_RZ] = rz;
    cs[CG_BN] = bn;
    cs[CG_ST] = (bn == 0.0 || rn <= CG_TOL2 * bn) ? CG_DONE : CG_ACTIVE;
    cs[CG_DBAR] = dbar;
    cs[CG_IT] = 0.0;
  }
}

__global__ __launch_bounds__(CG_T) void k_cg_update(Tables tb, StepArgs a, double* x, double* r,
                                                    double* p, const double* kp, double* cgs,
                                                    int cap) {
  __shared__ double red[CG_T];
  const int u = blockIdx.x, tid = threadIdx.x, Mp = tb.Mp, M1 = tb.M1;
  double* cs = cgs + (long)u * CG_NS;
  if (cs[CG_ST] != CG_ACTIVE) return;  // the same for the whole work-group
  const UnitView v = decode_unit(tb, a, u);
  const double tau = tb.inst[(long)v.b * NSCAL + v.tau_slot];
  const double rz = cs[CG_RZ], bn = cs[CG_BN], dbar = cs[CG_DBAR];
  const double it = cs[CG_IT] + 1.0;
  const int Mb = M1 * M1;
  const long o = (long)u * Mp;
  double ap[CG_E];
  double pap = 0.0;
#pragma unroll
  for (int e = 0; e < CG_E; ++e) {
    const int k = tid + e * CG_T;
    ap[e] = 0.0;
    if (k < Mb) {
      const double pk = p[o + k];
      ap[e] = pk + tau * kp[o + k];
      pap += pk * ap[e];
    }
  }
  pap = block_sum(pap, red);
  const double al = rz / pap;
  double rn = 0.0, rz1 = 0.0;
  double zz[CG_E];
#pragma unroll
  for (int e = 0; e < CG_E; ++e) {
    const int k = tid + e * CG_T;
    zz[e] = 0.0;
    if (k < Mb) {
      x[o + k] += al * p[o + k];
      const double rk = r[o + k] - al * ap[e];
      r[o + k] = rk;
      zz[e] = rk / cg_pdiag(k, M1, tau, dbar);
      rn += rk * rk;
      rz1 += rk * zz[e];
    }
  }
  rn = block_sum(rn, red);
  rz1 = block_sum(rz1, red);
  const bool done = rn <= CG_TOL2 * bn;
  if (!done) {
    const double be = rz1 / rz;
#pragma unroll
    for (int e = 0; e < CG_E; ++e) {
      const int k = tid + e * CG_T;
      if (k < Mb) p[o + k] = zz[e] + be * p[o + k];
    }
  }
  if (tid == 0) {
    cs[CG_RZ] = rz1;
    cs[CG_IT] = it;
    cs[CG_ST] = done ? CG_DONE : (it >= (double)cap ? CG_FAIL : CG_ACTIVE);
  }
}

// out[0] = units still iterating, out[1] = units that failed
__global__ __launch_bounds__(CG_T) void k_cg_count(const double* cgs, int units, int32_t* out) {
  __shared__ double red[CG_T];
  double act = 0.0, fail = 0.0;
  for (int u = threadIdx.x; u < units; u += CG_T) {
    const double st = cgs[(long)u * CG_NS + CG_ST];
    act += st == CG_ACTIVE ? 1.0 : 0.0;
    fail += st == CG_FAIL ? 1.0 : 0.0;
  }
  act = block_sum(act, red);
  fail = block_sum(fail, red);
  if (threadIdx.x == 0) {
    out[0] = (int32_t)act;
    out[1] = (int32_t)fail;
  }
}

__global__ void k_cg_finish(Tables tb, StepArgs a, Epilogue ep, int units, const double* x) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)units * tb.Mp) return;
  const int u = (int)(idx / tb.Mp), k = (int)(idx % tb.Mp);
  const UnitView v = decode_unit(tb, a, u);
  const bool last = (a.mode == MODE_FINE) && (a.r == v.Sb);
  epi_store(a, ep, u, v.slot, last, k, x[idx]);
}

hipError_t launch_cg_init(const Tables& tb, const StepArgs& a, int units, const double* x0,
                          const double* kx, double* x, double* r, double* p, double* cgs,
                          hipStream_t s) {
  if (tb.Mp > CG_T * CG_E) return hipErrorInvalidValue;
  k_cg_init<<<units, CG_T, 0, s>>>(tb, a, x0, kx, x, r, p, cgs);
  return hipGetLastError();
}

hipError_t launch_cg_update(const Tables& tb, const StepArgs& a, int units, double* x, double* r,
                            double* p, const double* kp, double* cgs, int cap, hipStream_t s) {
  if (tb.Mp > CG_T * CG_E) return hipErrorInvalidValue;
  k_cg_update<<<units, CG_T, 0, s>>>(tb, a, x, r, p, kp, cgs, cap);
  return hipGetLastError();
}

hipError_t launch_cg_count(const double* cgs, int units, int32_t* out, hipStream_t s) {
  k_cg_count<<<1, CG_T, 0, s>>>(cgs, units, out);
  return hipGetLastError();
}

hipError_t launch_cg_finish(const Tables& tb, const StepArgs& a, const Epilogue& e, int units,
                            const double* x, hipStream_t s) {
  const long n = (long)units * tb.Mp;
  k_cg_finish<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(tb, a, e, units, x);
  return hipGetLastError();
}

}  // namespace l1pr
