// Preconditioned conjugate gradients for the 2D step systems (I + tau K) c = rhs.
//
// K is applied at the Gauss points, never formed: launch_stiff2d_grid forms
// G = [Gx; Gy] = [dphi V phi^T; phi V dphi^T] o (w w D) for the current vector V, and the fused
// step kernel below finishes K V = dphi^T Gx phi + phi^T Gy dphi and updates the iterates.
// The preconditioner is the diagonal of I + tau K (Jacobi), from the cosine moments.  With D
// constant the sine basis diagonalises K, so for the workloads' D (within a factor 1.5 or 2 of
// its mean) the preconditioned spectrum stays within a small interval when the quadrature
// resolves the modes (Q >= 3M/2; below that the quadrature stiffness has near-null directions).
// The start is the lagged state.
//
// One 256-thread work-group per unit; the unit's vectors live in device memory between
// iterations; dot products are fixed-order sums (per-lane sums, then a fixed tree), so a unit's
// iterates depend only on its own data.  Per-unit state in cgs[u][8]: rz = r.z, ||rhs||^2,
// status, iteration count.  A unit stops (and is left untouched by later launches) once
// ||r|| <= tol ||rhs|| (1e-14 for fine and full-history steps, 1e-10 for coarse steps).
#include "l1pr_internal.h"

namespace l1pr {

constexpr int CG_T = 256;
enum { CG_RZ = 0, CG_BN = 1, CG_ST = 2, CG_IT = 3, CG_NS = 8 };
constexpr double CG_ACTIVE = 0.0, CG_DONE = 1.0, CG_FAIL = 2.0;

// Sum over the work-group: a butterfly within each wave (both lanes of a pair add the same
// two values, so every lane ends with the same sum), then the four wave sums in order.
__device__ inline double block_sum(double v, double* red) {
#pragma unroll
  for (int s = 32; s > 0; s >>= 1) v += __shfl_xor(v, s, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int w = 0; w < CG_T / 64; ++w) r += red[w];
  __syncthreads();
  return r;
}

// The second half of the stiffness product, K p = [dphi; phi]^T [Gx phi; Gy dphi], from
// G = [Gx; Gy] (launch_stiff2d_grid; 2Qp x Qp per unit), one work-group per (16-row chunk of G,
// unit): the chunk's rows staged in LDS, H = chunk x table on FP64 MFMA 16x16x4 (the table
// operands loaded one 16-row group ahead, two accumulators), then the chunk's share
// [dphi; phi]_chunk^T H of the M1 x M1 result, written as a partial in the accumulator layout:
// kvp[u][c][tid][16], entry (i, j) (k = i M1 + j) held by one lane.  Spreading a unit over its
// 2Qp/16 chunks keeps single-unit steps off a single CU; the step kernel sums the partials in
// chunk order, so the arithmetic never depends on the number of units in a launch.
constexpr int KV_T = 256;
typedef double d4 __attribute__((ext_vector_type(4)));

// lane entries: (xx, yy, e) -> i = wi 32 + xx 16 + (lane >> 4) + 4 e, j = wj 32 + yy 16 + (lane & 15)
template <int INIT>
__global__ __launch_bounds__(KV_T) void k_cg_part(Tables tb, const double* G, double* kvp,
                                                  const double* cgs) {
  extern __shared__ double sm[];
  const int c = blockIdx.x, u = blockIdx.y, nch = gridDim.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int M1 = tb.M1, M1p = tb.M1p, Qp = tb.Qp;
  if (!INIT && cgs[(long)u * CG_NS + CG_ST] != CG_ACTIVE) return;
  const int ldg = Qp + 1, ldh = 65;
  double* sG = sm;
  double* sH = sG + 16 * ldg;
  const double* Gu = G + (long)u * 2 * Qp * Qp;
  const int wi = wave >> 1, wj = wave & 1;
  const int hcol = wave * 16 + (lane & 15);
  const int q0 = 16 * c;
  for (int e = tid; e < 16 * Qp; e += KV_T) {
    const int rr = e / Qp, q = e % Qp;
    sG[rr * ldg + q] = Gu[(long)(q0 + rr) * Qp + q];
  }
  __syncthreads();
  // H = G[q0 .. q0+15] T with T = phi (rows of Gx) or dphi (rows of Gy); wave w: columns
  // 16w .. 16w+15.  16 rows of T per group (Qp is a multiple of 16).
  const double* Tc = (q0 < Qp ? tb.phi : tb.dphi) + (lane >> 4) * M1p + (hcol < M1 ? hcol : 0);
  const double tmask = hcol < M1 ? 1.0 : 0.0;
  const double* sGr = sG + (lane & 15) * ldg + (lane >> 4);
  d4 h0 = d4{0.0, 0.0, 0.0, 0.0}, h1 = d4{0.0, 0.0, 0.0, 0.0};
  double bv[4], bn[4];
#pragma unroll
  for (int g = 0; g < 4; ++g) bv[g] = Tc[(long)(4 * g) * M1p];
  for (int k0 = 0; k0 < Qp; k0 += 16) {
    const int kn = k0 + 16 < Qp ? k0 + 16 : k0;
#pragma unroll
    for (int g = 0; g < 4; ++g) bn[g] = Tc[(long)(kn + 4 * g) * M1p];
#pragma unroll
    for (int g = 0; g < 4; g += 2) {
      h0 = __builtin_amdgcn_mfma_f64_16x16x4f64(sGr[k0 + 4 * g], bv[g] * tmask, h0, 0, 0, 0);
      h1 = __builtin_amdgcn_mfma_f64_16x16x4f64(sGr[k0 + 4 * g + 4], bv[g + 1] * tmask, h1, 0, 0, 0);
    }
#pragma unroll
    for (int g = 0; g < 4; ++g) bv[g] = bn[g];
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) sH[((lane >> 4) + 4 * v) * ldh + hcol] = h0[v] + h1[v];
  __syncthreads();
  // partial = [dphi; phi][q0 .. q0+15]^T H
  d4 acc[2][2];
#pragma unroll
  for (int xx = 0; xx < 2; ++xx)
#pragma unroll
    for (int yy = 0; yy < 2; ++yy) acc[xx][yy] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k4 = 0; k4 < 16; k4 += 4) {
    const int kk = k4 + (lane >> 4);
    double af[2], bf[2];
#pragma unroll
    for (int xx = 0; xx < 2; ++xx) {
      const int i = wi * 32 + xx * 16 + (lane & 15);
      af[xx] = i < M1 ? tb.s2[(long)(q0 + kk) * M1p + i] : 0.0;
    }
#pragma unroll
    for (int yy = 0; yy < 2; ++yy) bf[yy] = sH[kk * ldh + wj * 32 + yy * 16 + (lane & 15)];
#pragma unroll
    for (int xx = 0; xx < 2; ++xx)
#pragma unroll
      for (int yy = 0; yy < 2; ++yy)
        acc[xx][yy] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[xx], bf[yy], acc[xx][yy], 0, 0, 0);
  }
  double* out = kvp + (((long)u * nch + c) * KV_T + tid) * 16;
#pragma unroll
  for (int xx = 0; xx < 2; ++xx)
#pragma unroll
    for (int yy = 0; yy < 2; ++yy)
#pragma unroll
      for (int e = 0; e < 4; ++e) out[(xx * 2 + yy) * 4 + e] = acc[xx][yy][e];
}

// One conjugate-gradient step (INIT = 0) or the start (INIT = 1) for the unit of each
// work-group, with K p (K x0) = the sum of the unit's nch partials in chunk order.  INIT: the
// Jacobi diagonal d_k = 1 + tau K_kk (from the cosine moments), x = x0, r = rhs - (x0 + tau K x0),
// z = r / d, p = z.  Otherwise the CG update with Ap = p + tau K p.  Dot products are per-lane
// sums followed by the fixed tree.
template <int INIT>
__global__ __launch_bounds__(KV_T) void k_cg_step(Tables tb, StepArgs a, const double* kvp,
                                                  int nch, const double* x0, double* x, double* r,
                                                  double* p, double* pd, double* cgs, int cap,
                                                  double tol2) {
  __shared__ double red[KV_T];
  const int u = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int M1 = tb.M1, M1p = tb.M1p, Mp = tb.Mp;
  double* cs = cgs + (long)u * CG_NS;
  if (!INIT && cs[CG_ST] != CG_ACTIVE) return;  // the same for the whole work-group
  const int wi = wave >> 1, wj = wave & 1;
  d4 acc[2][2];
#pragma unroll
  for (int xx = 0; xx < 2; ++xx)
#pragma unroll
    for (int yy = 0; yy < 2; ++yy) acc[xx][yy] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int c = 0; c < nch; ++c) {
    const double* in = kvp + (((long)u * nch + c) * KV_T + tid) * 16;
#pragma unroll
    for (int xx = 0; xx < 2; ++xx)
#pragma unroll
      for (int yy = 0; yy < 2; ++yy)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[xx][yy][e] += in[(xx * 2 + yy) * 4 + e];
  }

  const UnitView v = decode_unit(tb, a, u);
  const double tau = tb.inst[(long)v.b * NSCAL + v.tau_slot];
  const long o = (long)u * Mp;
  // the lane's entries: (xx, yy, e) -> i = wi 32 + xx 16 + (lane >> 4) + 4e, j = wj 32 + yy 16 + (lane & 15)
  if (INIT) {
    const int Jp = 2 * M1p + 1;
    const double* m = a.mom + (long)u * Jp * Jp;
    const double pi2 = kPi * kPi;
    double bn = 0.0, rz = 0.0, rn = 0.0;
#pragma unroll
    for (int xx = 0; xx < 2; ++xx)
#pragma unroll
      for (int yy = 0; yy < 2; ++yy)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int i = wi * 32 + xx * 16 + (lane >> 4) + 4 * e, j = wj * 32 + yy * 16 + (lane & 15);
          if (i >= M1 || j >= M1) continue;
          const int k = i * M1 + j;
          const int s1 = 2 * (i + 1), s2 = 2 * (j + 1);
          const double m00 = m[0], m0s = m[s2], ms0 = m[(long)s1 * Jp], mss = m[(long)s1 * Jp + s2];
          const double K1 = (double)(i + 1), K2 = (double)(j + 1);
          const double kdiag = K1 * K1 * pi2 * (((m00 - m0s) + ms0) - mss) +
                               K2 * K2 * pi2 * (((m00 + m0s) - ms0) - mss);
          const double dk = 1.0 + tau * kdiag;
          const double b = a.rhs[o + k], xk = x0[o + k];
          const double rk = b - (xk + tau * acc[xx][yy][e]);
          const double zk = rk / dk;
          pd[o + k] = dk;
          x[o + k] = xk;
          r[o + k] = rk;
          p[o + k] = zk;
          bn += b * b;
          rz += rk * zk;
          rn += rk * rk;
        }
    for (int k = M1 * M1 + tid; k < Mp; k += KV_T) {  // padding of the coefficient vector
      x[o + k] = 0.0;
      r[o + k] = 0.0;
      p[o + k] = 0.0;
    }
    bn = block_sum(bn, red);
    rz = block_sum(rz, red);
    rn = block_sum(rn, red);
    if (bn == 0.0) {  // zero right-hand side: the solution is 0
#pragma unroll
      for (int xx = 0; xx < 2; ++xx)
#pragma unroll
        for (int yy = 0; yy < 2; ++yy)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int i = wi * 32 + xx * 16 + (lane >> 4) + 4 * e, j = wj * 32 + yy * 16 + (lane & 15);
            if (i < M1 && j < M1) x[o + i * M1 + j] = 0.0;
          }
    }
    if (tid == 0) {
      cs[CG_RZ] = rz;
      cs[CG_BN] = bn;
      cs[CG_ST] = (bn == 0.0 || rn <= tol2 * bn) ? CG_DONE : CG_ACTIVE;
      cs[CG_IT] = 0.0;
    }
    return;
  }
  const double rz = cs[CG_RZ], bn = cs[CG_BN];
  const double it = cs[CG_IT] + 1.0;
  double ap[2][2][4];
  double pap = 0.0;
#pragma unroll
  for (int xx = 0; xx < 2; ++xx)
#pragma unroll
    for (int yy = 0; yy < 2; ++yy)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = wi * 32 + xx * 16 + (lane >> 4) + 4 * e, j = wj * 32 + yy * 16 + (lane & 15);
        ap[xx][yy][e] = 0.0;
        if (i >= M1 || j >= M1) continue;
        const double pk = p[o + i * M1 + j];
        ap[xx][yy][e] = pk + tau * acc[xx][yy][e];
        pap += pk * ap[xx][yy][e];
      }
  pap = block_sum(pap, red);
  const double al = rz / pap;
  double rn = 0.0, rz1 = 0.0;
#pragma unroll
  for (int xx = 0; xx < 2; ++xx)
#pragma unroll
    for (int yy = 0; yy < 2; ++yy)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = wi * 32 + xx * 16 + (lane >> 4) + 4 * e, j = wj * 32 + yy * 16 + (lane & 15);
        if (i >= M1 || j >= M1) continue;
        const long k = o + i * M1 + j;
        x[k] += al * p[k];
        const double rk = r[k] - al * ap[xx][yy][e];
        r[k] = rk;
        const double zk = rk / pd[k];
        ap[xx][yy][e] = zk;  // z from here on
        rn += rk * rk;
        rz1 += rk * zk;
      }
  rn = block_sum(rn, red);
  rz1 = block_sum(rz1, red);
  const bool done = rn <= tol2 * bn;
  if (!done) {
    const double be = rz1 / rz;
#pragma unroll
    for (int xx = 0; xx < 2; ++xx)
#pragma unroll
      for (int yy = 0; yy < 2; ++yy)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int i = wi * 32 + xx * 16 + (lane >> 4) + 4 * e, j = wj * 32 + yy * 16 + (lane & 15);
          if (i >= M1 || j >= M1) continue;
          const long k = o + i * M1 + j;
          p[k] = ap[xx][yy][e] + be * p[k];
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

hipError_t launch_cg_step(const Tables& tb, const StepArgs& a, int units, const double* G,
                          double* kvp, const double* x0, double* x, double* r, double* p,
                          double* pd, double* cgs, int cap, double tol, bool init, hipStream_t s) {
  const double tol2 = tol * tol;
  if (tb.M1 > 64) return hipErrorInvalidValue;  // the unit's M1 x M1 product is one 64 x 64 tile
  const size_t lds = sizeof(double) * (16 * (tb.Qp + 1) + 16 * 65);
  if (lds > 65536) return hipErrorInvalidValue;  // Qp up to 444
  const int nch = 2 * tb.Qp / 16;
  const dim3 gp(nch, units);
  if (init) {
    k_cg_part<1><<<gp, KV_T, lds, s>>>(tb, G, kvp, cgs);
    k_cg_step<1><<<units, KV_T, 0, s>>>(tb, a, kvp, nch, x0, x, r, p, pd, cgs, cap, tol2);
  } else {
    k_cg_part<0><<<gp, KV_T, lds, s>>>(tb, G, kvp, cgs);
    k_cg_step<0><<<units, KV_T, 0, s>>>(tb, a, kvp, nch, x0, x, r, p, pd, cgs, cap, tol2);
  }
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
