// One semi-implicit L1-Galerkin step for many units at once (1D sine basis).
//
// A "unit" is one system to solve at this step: an (instance, slice) pair of the fine
// sweep, an instance of the coarse sweep, or an instance of the full-history sweep.
// For systems too large for the register-resident kernel (Mp > 256) a step is:
//   k_eval1d     u_q = sum_k phi_k(x_q) c_k at the lagged state, d_q = w_q D(x_q,t,u_q),
//                g_q = w_q f(x_q,t,u_q), the load F = phi^T g, the L1 history sums and the
//                right-hand side rhs = hist + tau F            (Sections 2.1 and 2.2)
//   k_assemble1d A = I + tau dphi^T diag(d) dphi, lower tiles only, FP64 MFMA 16x16x4
// then the blocked factorisation and solve through device memory (chol_blk.hip), whose
// epilogue stores the new state (or applies the parareal correction F_old + (G_new - G_old)).
// This file also holds the small packing, copy and bookkeeping kernels.
// The arithmetic of a unit never depends on the other units of the launch, so a unit's
// result is bit-for-bit the same in a serial sweep and in a parareal sweep.
#include "l1pr_internal.h"

namespace l1pr {

typedef double d4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------------------ eval
__global__ __launch_bounds__(256) void k_eval1d(Tables tb, StepArgs a) {
  extern __shared__ double sm[];
  const int u = blockIdx.x, tid = threadIdx.x;
  const int Mp = tb.Mp, Qp = tb.Qp;
  double* sc = sm;       // lagged state c [Mp]
  double* sg = sm + Mp;  // w_q f_q       [Qp]
  const UnitView v = decode_unit(tb, a, u);
  const double* ins = tb.inst + (long)v.b * NSCAL;
  const double tD = t_level(tb, v.m_prev, v.Nb);
  const double tf = tb.source_time ? t_level(tb, v.m_src, v.Nb) : tD;

  for (int k = tid; k < Mp; k += blockDim.x) sc[k] = v.y[(long)v.L * Mp + k];
  __syncthreads();

  double* dout = a.d + (long)u * Qp;
  for (int q = tid; q < Qp; q += blockDim.x) {
    double uq = 0.0;
    for (int k = 0; k < Mp; ++k) uq += tb.phiT[(long)k * Qp + q] * sc[k];
    const double x = tb.xq[q], w = tb.wq[q];
    dout[q] = w * coef_D(tb.d_sel, tb.d_param, uq);
    sg[q] = w * coef_f(tb, ins, x, 0.0, tf, uq);
  }
  __syncthreads();

  const double tau = ins[v.tau_slot];
  const double* bw = tb.bw + (long)v.b * tb.LB;
  const double* bh = tb.bhyb ? tb.bhyb + (long)v.b * tb.P * tb.S : nullptr;
  for (int k = tid; k < Mp; k += blockDim.x) {
    double F = 0.0;
    for (int q = 0; q < Qp; ++q) F += tb.phi[(long)q * Mp + k] * sg[q];
    if (a.mode == MODE_FINE && a.prev) {
      a.rhs[(long)u * Mp + k] = full_fine_history(tb, a, v, k) + tau * F;
      continue;
    }
    if (a.mode == MODE_FULL) {
      a.rhs[(long)u * Mp + k] = full_serial_history(tb, a, v, k) + tau * F;
      continue;
    }
    // in-sequence L1 history: y_L - sum_{i=1}^{L} b_{L+1-i} (y_i - y_{i-1})
    double acc = 0.0;
    for (int i = 1; i <= v.L; ++i)
      acc = fma(bw[v.L + 1 - i], v.y[(long)i * Mp + k] - v.y[(long)(i - 1) * Mp + k], acc);
    double h = v.y[(long)v.L * Mp + k] - acc;
    if (a.mode == MODE_FINE) {
      // coarse-grid history of the hybrid operator: S^-a sum_{i=1}^{n} b_{n-i+r/S} (C_i - C_{i-1})
      double acc2 = 0.0;
      for (int i = 1; i <= v.nz; ++i)
        acc2 += bh[(long)(v.nz - i) * tb.S + (a.r - 1)] *
                (v.z[(long)i * Mp + k] - v.z[(long)(i - 1) * Mp + k]);
      h = h - ins[IS_SFAC] * acc2;
    }
    a.rhs[(long)u * Mp + k] = h + tau * F;
  }
}

// -------------------------------------------------------------------------- assemble
// Tile (I, J), I >= J, of TB x TB entries of A = I + tau dphi^T diag(d) dphi.  Quadrature
// points stream through LDS in chunks of 16; each wave owns TPW x TPW MFMA 16x16 tiles.
// MFMA f64 16x16x4 operand layout: lane l holds A[l%16][l/16] and B[l/16][l%16]; the
// accumulator holds D[l/16 + 4v][l%16] in element v.
template <int TB>
__global__ __launch_bounds__(256) void k_assemble1d(Tables tb, StepArgs a) {
  constexpr int NW = (TB == 16) ? 1 : 4;
  constexpr int TPW = (TB == 64) ? 2 : 1;
  constexpr int QC = 16;
  __shared__ double sA[QC][TB + 1];
  __shared__ double sB[QC][TB + 1];
  const int t = blockIdx.x, u = blockIdx.y;
  int I = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  while (I * (I + 1) / 2 > t) --I;
  const int J = t - I * (I + 1) / 2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wi = (NW == 4) ? (wave >> 1) : 0, wj = (NW == 4) ? (wave & 1) : 0;
  const int Mp = tb.Mp, Qp = tb.Qp;
  const double* d = a.d + (long)u * Qp;

  d4 acc[TPW][TPW];
#pragma unroll
  for (int ti = 0; ti < TPW; ++ti)
#pragma unroll
    for (int tj = 0; tj < TPW; ++tj) acc[ti][tj] = d4{0.0, 0.0, 0.0, 0.0};

  for (int q0 = 0; q0 < Qp; q0 += QC) {
    for (int e = threadIdx.x; e < QC * TB; e += NW * 64) {
      const int qq = e / TB, c = e % TB;
      const double* row = tb.dphi + (long)(q0 + qq) * Mp;
      sA[qq][c] = row[I * TB + c];
      sB[qq][c] = d[q0 + qq] * row[J * TB + c];
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < QC / 4; ++kk) {
      const int kq = kk * 4 + (lane >> 4);
      double af[TPW], bf[TPW];
#pragma unroll
      for (int ti = 0; ti < TPW; ++ti) af[ti] = sA[kq][wi * 16 * TPW + ti * 16 + (lane & 15)];
#pragma unroll
      for (int tj = 0; tj < TPW; ++tj) bf[tj] = sB[kq][wj * 16 * TPW + tj * 16 + (lane & 15)];
#pragma unroll
      for (int ti = 0; ti < TPW; ++ti)
#pragma unroll
        for (int tj = 0; tj < TPW; ++tj)
          acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[ti], bf[tj], acc[ti][tj], 0, 0, 0);
    }
    __syncthreads();
  }

  const int b = (a.mode == MODE_FINE) ? u / a.nP : u;
  const double tau = tb.inst[(long)b * NSCAL + ((a.mode == MODE_COARSE) ? IS_TAUC : IS_TAU)];
  double* A = a.A + (long)u * Mp * Mp;
#pragma unroll
  for (int ti = 0; ti < TPW; ++ti)
#pragma unroll
    for (int tj = 0; tj < TPW; ++tj)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = I * TB + wi * 16 * TPW + ti * 16 + (lane >> 4) + 4 * e;
        const int col = J * TB + wj * 16 * TPW + tj * 16 + (lane & 15);
        A[(long)row * Mp + col] = tau * acc[ti][tj][e] + (row == col ? 1.0 : 0.0);
      }
}

// ------------------------------------------------------------------------ launchers
hipError_t launch_eval(const Tables& tb, const StepArgs& a, int units, hipStream_t s) {
  const size_t lds = sizeof(double) * (tb.Mp + tb.Qp);
  k_eval1d<<<units, 256, lds, s>>>(tb, a);
  return hipGetLastError();
}

hipError_t launch_assemble(const Tables& tb, const StepArgs& a, int units, hipStream_t s) {
  int TB = (tb.Mp % 64 == 0) ? 64 : ((tb.Mp % 32 == 0) ? 32 : 16);
  const int nt = tb.Mp / TB;
  dim3 grid(nt * (nt + 1) / 2, units);
  if (TB == 64) k_assemble1d<64><<<grid, 256, 0, s>>>(tb, a);
  else if (TB == 32) k_assemble1d<32><<<grid, 256, 0, s>>>(tb, a);
  else k_assemble1d<16><<<grid, 64, 0, s>>>(tb, a);
  return hipGetLastError();
}

// ------------------------------------------------------------------- small kernels
__global__ void k_pack(const double* src, int M, int B, long src_stride, double* dst, int Mp,
                       long dst_stride) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)B * Mp) return;
  const int b = (int)(idx / Mp), k = (int)(idx % Mp);
  dst[b * dst_stride + k] = (k < M) ? src[b * src_stride + k] : 0.0;
}

hipError_t launch_pack(const double* src, int M, int B, long src_stride, double* dst, int Mp,
                       long dst_stride, hipStream_t s) {
  const long n = (long)B * Mp;
  k_pack<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(src, M, B, src_stride, dst, Mp, dst_stride);
  return hipGetLastError();
}

// dst[u][row][k] = src[u][row][k] for row < rows, k < Mp
__global__ void k_copy_rows(const double* src, long sstr, double* dst, long dstr, int rows, int Mp,
                            int units) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long per = (long)rows * Mp;
  if (idx >= per * units) return;
  const long u = idx / per, e = idx % per;
  dst[u * dstr + e] = src[u * sstr + e];
}

hipError_t launch_copy_rows(const double* src, long src_unit_stride, double* dst,
                            long dst_unit_stride, int rows, int Mp, int units, hipStream_t s) {
  const long n = (long)rows * Mp * units;
  if (n == 0) return hipSuccess;
  k_copy_rows<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(src, src_unit_stride, dst,
                                                          dst_unit_stride, rows, Mp, units);
  return hipGetLastError();
}

// traj[b*P + n][0] = Z[b][n] for all b < B, n < P
__global__ void k_fill_slot0(const double* Z, double* traj, int B, int P, int S, int Mp) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)B * P * Mp) return;
  const long slot = idx / Mp;
  const int k = (int)(idx % Mp);
  const long b = slot / P, n = slot % P;
  traj[slot * (long)(S + 1) * Mp + k] = Z[(b * (P + 1) + n) * Mp + k];
}

hipError_t launch_fill_slot0(const Tables& tb, const double* Z, double* traj, int B, int P,
                             hipStream_t s) {
  const long n = (long)B * P * tb.Mp;
  k_fill_slot0<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(Z, traj, B, P, tb.S, tb.Mp);
  return hipGetLastError();
}

// dst[u][row][k<M] = src[u][row][k] (drops the padding)
__global__ void k_unpack(const double* src, int Mp, long sstr, double* dst, int M, long dstr,
                         int rows, int units) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long per = (long)rows * M;
  if (idx >= per * units) return;
  const long u = idx / per, e = idx % per;
  const long row = e / M, k = e % M;
  dst[u * dstr + row * M + k] = src[u * sstr + row * Mp + k];
}

hipError_t launch_unpack(const double* src, int Mp, long src_stride, double* dst, int M,
                         long dst_stride, int rows_per_unit, int units, hipStream_t s) {
  const long n = (long)rows_per_unit * M * units;
  if (n == 0) return hipSuccess;
  k_unpack<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(src, Mp, src_stride, dst, M, dst_stride,
                                                       rows_per_unit, units);
  return hipGetLastError();
}

// dst[u][row][k] = src[u][row][k] for k < M, 0 for M <= k < Mp (adds the padding)
__global__ void k_unpack_pad(const double* src, int M, long sstr, double* dst, int Mp, long dstr,
                             int rows, int units) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long per = (long)rows * Mp;
  if (idx >= per * units) return;
  const long u = idx / per, e = idx % per;
  const long row = e / Mp, k = e % Mp;
  dst[u * dstr + row * Mp + k] = (k < M) ? src[u * sstr + row * M + k] : 0.0;
}

hipError_t launch_unpack_pad(const double* src, int M, long src_stride, double* dst, int Mp,
                             long dst_stride, int rows_per_unit, int units, hipStream_t s) {
  const long n = (long)rows_per_unit * Mp * units;
  if (n == 0) return hipSuccess;
  k_unpack_pad<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(src, M, src_stride, dst, Mp, dst_stride,
                                                           rows_per_unit, units);
  return hipGetLastError();
}

// Relative increment ||Znew_b - Zold_b|| / ||Znew_b|| per instance, fixed-order tree
// reduction (one work-group per instance), then the instance's stop test.
__global__ __launch_bounds__(256) void k_increment(const double* Znew, const double* Zold, int rows,
                                                   int Mp, double* incr_out, int incr_stride, int k,
                                                   double* incr_k, int32_t* done, int32_t* conv,
                                                   double exit_tol, int* flag, int32_t* lg_off,
                                                   double* incr_prev, double* gold,
                                                   const double* gplain, long gper) {
  __shared__ double sd[256], su[256];
  __shared__ int flip;
  const int b = blockIdx.x, tid = threadIdx.x;
  const long per = (long)rows * Mp;
  const double* a = Znew + b * per;
  const double* o = Zold + b * per;
  double dn = 0.0, un = 0.0;
  for (long e = tid; e < per; e += 256) {
    const double d = a[e] - o[e];
    dn += d * d;
    un += a[e] * a[e];
  }
  sd[tid] = dn;
  su[tid] = un;
  if (tid == 0) flip = 0;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) {
      sd[tid] += sd[tid + w];
      su[tid] += su[tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) {
    const bool finished = done && done[b] != 0;
    // a finished instance keeps its slice ends: its increment is 0 from then on
    const double rel = finished ? 0.0 : (su[0] > 0.0 ? sqrt(sd[0]) / sqrt(su[0]) : sqrt(sd[0]));
    if (incr_out) incr_out[(long)b * incr_stride + k] = rel;
    incr_k[b] = rel;
    if (!finished) {
      if (!isfinite(rel)) {
        if (done) done[b] = 1;
        if (conv) conv[b] = L1PR_ENONFINITE;
        if (flag) atomicOr(flag, FLAG_NONFINITE);
      } else if (rel <= exit_tol) {
        if (done) done[b] = 1;
        if (conv) conv[b] = k + 1;
      }
      // learned coarse step: off for good after a sweep that contracted the increment by less
      // than kLearnedMinContraction (the plain coarse step contracts by 0.1-0.3 per sweep on
      // these problems, so a learned step that does worse is not helping)
      if (lg_off) {
        if (k >= 1 && !lg_off[b] && rel > kLearnedMinContraction * incr_prev[b]) {
          lg_off[b] = 1;
          flip = 1;
        }
        incr_prev[b] = rel;
      }
    }
  }
  // an instance back on the plain coarse step gets plain G_old values, so the next correction
  // G_new - G_old compares like with like
  __syncthreads();
  if (flip && gold && gplain)
    for (long e = tid; e < gper; e += 256) gold[b * gper + e] = gplain[b * gper + e];
}

// The learned step's judgement after the first fine sweep: for each unfinished instance still
// on the learned step, the squared distances of the fine results F_old(n) from the learned
// coarse values G_old(n) and from the plain ones Gp(n), summed over its slices in a fixed
// order.  If the learned values are not closer, the instance goes back to the plain coarse
// step for good (lg_off) with G_old replaced by the plain values.  One work-group per instance.
__global__ __launch_bounds__(256) void k_learned_judge(const double* fold, long fold_stride,
                                                       double* gold, const double* gplain, int P,
                                                       int Mp, const int32_t* done,
                                                       int32_t* lg_off) {
  __shared__ double sl[256], sp[256];
  __shared__ int off;
  const int b = blockIdx.x, tid = threadIdx.x;
  if ((done && done[b]) || lg_off[b]) return;  // uniform over the work-group
  const long gper = (long)P * Mp;
  double dl = 0.0, dp = 0.0;
  for (long e = tid; e < gper; e += 256) {
    const int n = (int)(e / Mp), k = (int)(e % Mp);
    const double f = fold[(long)(b * P + n) * fold_stride + k];
    const double a = f - gold[b * gper + e], c = f - gplain[b * gper + e];
    dl += a * a;
    dp += c * c;
  }
  sl[tid] = dl;
  sp[tid] = dp;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) {
      sl[tid] += sl[tid + w];
      sp[tid] += sp[tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) {
    off = !(sl[0] < sp[0]);
    if (off) lg_off[b] = 1;
  }
  __syncthreads();
  if (off)
    for (long e = tid; e < gper; e += 256) gold[b * gper + e] = gplain[b * gper + e];
}

hipError_t launch_learned_judge(const double* fold, long fold_stride, double* gold,
                                const double* gplain, int B, int P, int Mp, const int32_t* done,
                                int32_t* lg_off, hipStream_t s) {
  k_learned_judge<<<B, 256, 0, s>>>(fold, fold_stride, gold, gplain, P, Mp, done, lg_off);
  return hipGetLastError();
}

hipError_t launch_increment(const double* Znew, const double* Zold, int B, int rows, int Mp,
                            double* incr_out, int incr_stride, int k, double* incr_k,
                            int32_t* done, int32_t* conv, double exit_tol, int* flag,
                            hipStream_t s, int32_t* lg_off, double* incr_prev, double* gold,
                            const double* gplain, long gper) {
  k_increment<<<B, 256, 0, s>>>(Znew, Zold, rows, Mp, incr_out, incr_stride, k, incr_k, done,
                                conv, exit_tol, flag, lg_off, incr_prev, gold, gplain, gper);
  return hipGetLastError();
}

// one work-group per instance: the finished ones copy their slice ends
__global__ __launch_bounds__(256) void k_copy_done(const double* Zsrc, double* Zdst,
                                                   const int32_t* done, long per) {
  const int b = blockIdx.x;
  if (!done[b]) return;
  for (long e = threadIdx.x; e < per; e += 256) Zdst[b * per + e] = Zsrc[b * per + e];
}

hipError_t launch_copy_done(const double* Zsrc, double* Zdst, const int32_t* done, int B, long per,
                            hipStream_t s) {
  k_copy_done<<<B, 256, 0, s>>>(Zsrc, Zdst, done, per);
  return hipGetLastError();
}

__global__ void k_finish_status(const int32_t* done, const int32_t* conv, int32_t* out, int B,
                                int sweeps, int notconv) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  out[b] = done[b] ? conv[b] : (notconv ? (int32_t)L1PR_ENOTCONV : sweeps);
}

hipError_t launch_finish_status(const int32_t* done, const int32_t* conv, int32_t* out, int B,
                                int sweeps, bool notconv, hipStream_t s) {
  k_finish_status<<<(B + 255) / 256, 256, 0, s>>>(done, conv, out, B, sweeps, notconv ? 1 : 0);
  return hipGetLastError();
}

__global__ void k_check_finite(const double* x, long n, int* flag) {
  int bad = 0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    bad |= !isfinite(x[i]);
  if (bad) atomicOr(flag, FLAG_NONFINITE);
}

hipError_t launch_check_finite(const double* x, long n, int* flag, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const long blocks = (n + 255) / 256;
  k_check_finite<<<(unsigned)(blocks < 1024 ? blocks : 1024), 256, 0, s>>>(x, n, flag);
  return hipGetLastError();
}

__global__ void k_fill_int(int32_t* x, int n, int32_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

hipError_t launch_fill_int(int32_t* x, int n, int32_t v, hipStream_t s) {
  if (n > 0) k_fill_int<<<(n + 255) / 256, 256, 0, s>>>(x, n, v);
  return hipGetLastError();
}

// the device's constant-rate wall clock, written by one thread (a vector store)
__global__ void k_stamp(int64_t* t) {
  if (threadIdx.x == 0) t[0] = (int64_t)wall_clock64();
}

hipError_t launch_stamp(int64_t* t, hipStream_t s) {
  k_stamp<<<1, 64, 0, s>>>(t);
  return hipGetLastError();
}

}  // namespace l1pr
