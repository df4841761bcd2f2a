// Batched dense contractions and the history sum of one step, over all units of a launch.
//
//   k_lag_gemm1d     U = C Phi^T : u_q = sum_k phi_k(x_q) c_k for every unit (its lagged
//                    state c); then d_q = w_q D(x_q, t, u_q), g_q = w_q f(x_q, t, u_q).
//   k_proj_gemm1d    m = d cosq (cosine moments m_j = sum_q w_q D_q cos(j pi x_q)) and
//                    F = g Phi (load vector F_k = sum_q w_q f_q phi_k(x_q)).
//   k_history1d      hist = y_L - sum_{i=1}^{L} b_{L+1-i} (y_i - y_{i-1})
//                           [- S^-a sum_{i=1}^{n} b_{n-i+r/S} (C_i - C_{i-1})   (fine steps)].
// The GEMMs tile 32 units x 32 columns per work-group (four waves, one MFMA 16x16x4 tile
// each; tile_gemm takes any multiple of 32 in either direction) and stream the shared table
// through LDS in chunks of 32 rows (the next chunk loaded into registers while the current one
// is multiplied), so each table is read once per 32 units instead of once per unit.  (Measured
// at 2048 units of 256 modes and 384 nodes: 64 x 64 tiles leave most CUs with one or two
// waves per SIMD; 32 x 32 tiles take the projections from 55.8 to 38.9 us and the
// lagged-state product from 42 to 23 us, the same sums bit for bit; 32 x 64, 64 x 32 and
// 64-row chunks were slower.)  An output element is a fixed-order sum over
// its own row only, so a unit's values do not depend on the other units of the launch.
#include "l1pr_internal.h"

namespace l1pr {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int GT = 32;   // units and columns per work-group tile
constexpr int GK = 32;   // reduction chunk

// Row pointer of the lagged state of unit u.
__device__ inline const double* lag_row(const Tables& tb, const StepArgs& a, int u) {
  const UnitView v = decode_unit(tb, a, u);
  return v.y + (long)v.L * tb.Mp;
}

// C[u][n] = sum_k Arow(u)[k] * B[k][n] for a TU x TN tile; returns the accumulators.
// A rows come from `rowp(u)` (nullptr rows read as zero), B is [K][ldb] row-major.  The
// reduction runs in chunks of GK rows through LDS; each thread holds its share of the next
// chunk in registers, loaded from global memory while the current chunk's MFMAs run.  Entries
// past K are zeros.  The k-steps of 4 are accumulated in ascending order whatever GK is.
template <int TU, int TN, class RowFn>
__device__ inline void tile_gemm(RowFn rowp, int units, int u0, int n0, int K, const double* B,
                                 int ldb, int ncols, d4 (&acc)[TU / 32][TN / 32],
                                 double (*sA)[GK + 1], double (*sB)[TN + 1]) {
  constexpr int FA = TU / 32, FB = TN / 32;  // MFMA tiles per wave in each direction
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = wave >> 1, wj = wave & 1;
#pragma unroll
  for (int a = 0; a < FA; ++a)
#pragma unroll
    for (int b = 0; b < FB; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  // this thread's entries of a chunk: A rows ar + (256/GK) i at column ak, B rows bk + (256/TN) i at column bc
  constexpr int NA = TU * GK / 256, NB = GK * TN / 256;
  const int ar = tid / GK, ak = tid % GK, bk = tid / TN, bc = tid % TN;
  const double* arow[NA];
#pragma unroll
  for (int i = 0; i < NA; ++i) {
    const int u = u0 + ar + (256 / GK) * i;
    arow[i] = (u < units) ? rowp(u) : nullptr;
  }
  const bool bok = n0 + bc < ncols;
  double ra[NA], rb[NB];
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < NA; ++i) ra[i] = (arow[i] && k0 + ak < K) ? arow[i][k0 + ak] : 0.0;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int kk = k0 + bk + (256 / TN) * i;
      rb[i] = (bok && kk < K) ? B[(long)kk * ldb + n0 + bc] : 0.0;
    }
  };
  load(0);
  for (int k0 = 0; k0 < K; k0 += GK) {
#pragma unroll
    for (int i = 0; i < NA; ++i) sA[ar + (256 / GK) * i][ak] = ra[i];
#pragma unroll
    for (int i = 0; i < NB; ++i) sB[bk + (256 / TN) * i][bc] = rb[i];
    __syncthreads();
    if (k0 + GK < K) load(k0 + GK);
#pragma unroll
    for (int ks = 0; ks < GK / 4; ++ks) {
      const int kq = ks * 4 + (lane >> 4);
      double af[FA], bf[FB];
#pragma unroll
      for (int a = 0; a < FA; ++a) af[a] = sA[wi * (TU / 2) + a * 16 + (lane & 15)][kq];
#pragma unroll
      for (int b = 0; b < FB; ++b) bf[b] = sB[kq][wj * (TN / 2) + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < FA; ++a)
#pragma unroll
        for (int b = 0; b < FB; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
}

// grid: (ceil(Qp / TN), ceil(units / TU))
template <int TU, int TN>
__global__ __launch_bounds__(256) void k_lag_gemm1d(Tables tb, StepArgs a, int units, double* dq,
                                                    double* gq) {
  __shared__ double sA[TU][GK + 1];
  __shared__ double sB[GK][TN + 1];
  const int n0 = blockIdx.x * TN, u0 = blockIdx.y * TU;
  d4 acc[TU / 32][TN / 32];
  tile_gemm<TU, TN>([&](int u) { return lag_row(tb, a, u); }, units, u0, n0, tb.Mp, tb.phiT, tb.Qp,
            tb.Qp, acc, sA, sB);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wi = wave >> 1, wj = wave & 1;
#pragma unroll
  for (int ai = 0; ai < TU / 32; ++ai)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int u = u0 + wi * (TU / 2) + ai * 16 + (lane >> 4) + 4 * e;
      if (u >= units) continue;
      const UnitView v = decode_unit(tb, a, u);
      const double* ins = tb.inst + (long)v.b * NSCAL;
      const double tD = t_level(tb, v.m_prev, v.Nb);
      const double tf = tb.source_time ? t_level(tb, v.m_src, v.Nb) : tD;
#pragma unroll
      for (int bj = 0; bj < TN / 32; ++bj) {
        const int q = n0 + wj * (TN / 2) + bj * 16 + (lane & 15);
        if (q >= tb.Qp) continue;
        const double uq = acc[ai][bj][e];
        const double w = tb.wq[q];
        dq[(long)u * tb.Qp + q] = w * coef_D(tb.d_sel, tb.d_param, uq);
        gq[(long)u * tb.Qp + q] = w * coef_f(tb, ins, tb.xq[q], 0.0, tf, uq);
      }
    }
}

// grid: (ceil(max(Jm, Mp) / TN), ceil(units / TU), 2); z = 0: moments (skipped when m is
// nullptr), z = 1: load vector.
template <int TU, int TN>
__global__ __launch_bounds__(256) void k_proj_gemm1d(Tables tb, int units, const double* dq,
                                                     const double* gq, double* m, int Jm,
                                                     double* F) {
  __shared__ double sA[TU][GK + 1];
  __shared__ double sB[GK][TN + 1];
  const int which = blockIdx.z;
  const int n0 = blockIdx.x * TN, u0 = blockIdx.y * TU;
  const int ncols = which == 0 ? Jm : tb.Mp;
  if (which == 0 && m == nullptr) return;
  if (n0 >= ncols) return;
  const double* Ain = which == 0 ? dq : gq;
  const double* B = which == 0 ? tb.cosq : tb.phi;
  const int ldb = which == 0 ? Jm : tb.Mp;
  double* out = which == 0 ? m : F;
  d4 acc[TU / 32][TN / 32];
  tile_gemm<TU, TN>([&](int u) { return Ain + (long)u * tb.Qp; }, units, u0, n0, tb.Qp, B, ldb,
                    ncols, acc, sA, sB);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wi = wave >> 1, wj = wave & 1;
#pragma unroll
  for (int ai = 0; ai < TU / 32; ++ai)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int u = u0 + wi * (TU / 2) + ai * 16 + (lane >> 4) + 4 * e;
      if (u >= units) continue;
#pragma unroll
      for (int bj = 0; bj < TN / 32; ++bj) {
        const int c = n0 + wj * (TN / 2) + bj * 16 + (lane & 15);
        if (c < ncols) out[(long)u * ncols + c] = acc[ai][bj][e];
      }
    }
}

// Full-history steps (MODE_FULL, and MODE_FINE with the previous trajectories): work-groups
// (unit, block of 256 coefficients), one thread per coefficient, the prefix sum of the earlier
// rows continued row by row (full_fine_history, full_serial_history).  The hybrid steps below
// use k_history_split.
__global__ __launch_bounds__(256) void k_history1d(Tables tb, StepArgs a, double* hist) {
  const int u = blockIdx.x;
  const UnitView v = decode_unit(tb, a, u);
  const double* bw = tb.bw + (long)v.b * tb.LB;
  const int Mp = tb.Mp;
  const bool full_fine = a.mode == MODE_FINE && a.prev;
  for (int k = blockIdx.y * blockDim.x + threadIdx.x; k < Mp; k += blockDim.x * gridDim.y) {
    if (full_fine) {
      hist[(long)u * Mp + k] = full_fine_history(tb, a, v, k);
      continue;
    }
    if (a.mode == MODE_FULL) {
      hist[(long)u * Mp + k] = full_serial_history(tb, a, v, k);
      continue;
    }
    const double* y = v.y + k;
    double acc = 0.0;
    double prev = y[0];
    int i = 1;
    for (; i + 3 <= v.L; i += 4) {
      const double y1 = y[(long)i * Mp], y2 = y[(long)(i + 1) * Mp];
      const double y3 = y[(long)(i + 2) * Mp], y4 = y[(long)(i + 3) * Mp];
      acc = fma(bw[v.L + 1 - i], y1 - prev, acc);
      acc = fma(bw[v.L - i], y2 - y1, acc);
      acc = fma(bw[v.L - 1 - i], y3 - y2, acc);
      acc = fma(bw[v.L - 2 - i], y4 - y3, acc);
      prev = y4;
    }
    for (; i <= v.L; ++i) {
      const double yi = y[(long)i * Mp];
      acc = fma(bw[v.L + 1 - i], yi - prev, acc);
      prev = yi;
    }
    double h = y[(long)v.L * Mp] - acc;
    if (a.mode == MODE_FINE) {
      const double* bh = tb.bhyb + (long)v.b * tb.P * tb.S + (a.r - 1);
      const double* z = v.z + k;
      double acc2 = 0.0;
      double zp = z[0];
      int c = 1;
      for (; c + 3 <= v.nz; c += 4) {
        const double z1 = z[(long)c * Mp], z2 = z[(long)(c + 1) * Mp];
        const double z3 = z[(long)(c + 2) * Mp], z4 = z[(long)(c + 3) * Mp];
        acc2 += bh[(long)(v.nz - c) * tb.S] * (z1 - zp);
        acc2 += bh[(long)(v.nz - c - 1) * tb.S] * (z2 - z1);
        acc2 += bh[(long)(v.nz - c - 2) * tb.S] * (z3 - z2);
        acc2 += bh[(long)(v.nz - c - 3) * tb.S] * (z4 - z3);
        zp = z4;
      }
      for (; c <= v.nz; ++c) {
        const double zc = z[(long)c * Mp];
        acc2 += bh[(long)(v.nz - c) * tb.S] * (zc - zp);
        zp = zc;
      }
      h = h - tb.inst[(long)v.b * NSCAL + IS_SFAC] * acc2;
    }
    hist[(long)u * Mp + k] = h;
  }
}

// ------------------------------------------------------------------ skinny variants
// For launches with few units (the coarse steps: one unit per instance) the 32 x 32 tiles
// leave most of the chip idle and expose every load's latency.  These variants give each
// work-group one 16 x 16 output tile and cut the reduction into 32-wide chunks: lane group q
// of wave w owns chunk 4 (w + 4 i) + q, loads all of it before its first MFMA, and the four
// waves' partial tiles are added in LDS in wave order.  Each output is still a fixed-order
// sum over its own row, independent of the other units of the launch.
constexpr int ST = 16;

template <class RowFn>
__device__ inline double skinny_tile(RowFn rowp, int units, int u0, int n0, int K, const double* B,
                                     int ldb, int ncols, double (*red)[ST][ST + 1]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r = lane & 15, q = lane >> 4;
  const double* ap = (u0 + r < units) ? rowp(u0 + r) : nullptr;
  const int col = n0 + r;
  const bool bc = col < ncols;
  const int nchunk = (K + 31) / 32;
  d4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int blk = w; 4 * blk < nchunk; blk += 4) {
    const int k0 = (4 * blk + q) * 32;
    double xa[32], xb[32];
#pragma unroll
    for (int t = 0; t < 32; ++t) {
      const int k = k0 + t;
      xa[t] = (ap != nullptr && k < K) ? ap[k] : 0.0;
      xb[t] = (bc && k < K) ? B[(long)k * ldb + col] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < 32; ++t) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[t], xb[t], acc, 0, 0, 0);
  }
  // accumulator element v of lane (r, q) is tile entry [q + 4v][r]
#pragma unroll
  for (int v = 0; v < 4; ++v) red[w][q + 4 * v][r] = acc[v];
  __syncthreads();
  const int ro = threadIdx.x >> 4, co = threadIdx.x & 15;
  return red[0][ro][co] + red[1][ro][co] + red[2][ro][co] + red[3][ro][co];
}

// grid: (ceil(Qp / 16), ceil(units / 16))
__global__ __launch_bounds__(256) void k_lag_skinny1d(Tables tb, StepArgs a, int units, double* dq,
                                                      double* gq) {
  __shared__ double red[4][ST][ST + 1];
  const int n0 = blockIdx.x * ST, u0 = blockIdx.y * ST;
  const double uq = skinny_tile([&](int u) { return lag_row(tb, a, u); }, units, u0, n0, tb.Mp,
                                tb.phiT, tb.Qp, tb.Qp, red);
  const int u = u0 + (threadIdx.x >> 4), q = n0 + (threadIdx.x & 15);
  if (u >= units || q >= tb.Qp) return;
  const UnitView v = decode_unit(tb, a, u);
  const double* ins = tb.inst + (long)v.b * NSCAL;
  const double tD = t_level(tb, v.m_prev, v.Nb);
  const double tf = tb.source_time ? t_level(tb, v.m_src, v.Nb) : tD;
  const double w = tb.wq[q];
  dq[(long)u * tb.Qp + q] = w * coef_D(tb.d_sel, tb.d_param, uq);
  gq[(long)u * tb.Qp + q] = w * coef_f(tb, ins, tb.xq[q], 0.0, tf, uq);
}

// grid: (ceil(max(Jm, Mp) / 16), ceil(units / 16), 2); z as in k_proj_gemm1d
__global__ __launch_bounds__(256) void k_proj_skinny1d(Tables tb, int units, const double* dq,
                                                       const double* gq, double* m, int Jm,
                                                       double* F) {
  __shared__ double red[4][ST][ST + 1];
  const int which = blockIdx.z;
  const int n0 = blockIdx.x * ST, u0 = blockIdx.y * ST;
  const int ncols = which == 0 ? Jm : tb.Mp;
  if (which == 0 && m == nullptr) return;   // uniform per work-group
  if (n0 >= ncols) return;
  const double* Ain = which == 0 ? dq : gq;
  const double* B = which == 0 ? tb.cosq : tb.phi;
  double* out = which == 0 ? m : F;
  const double x = skinny_tile([&](int u) { return Ain + (long)u * tb.Qp; }, units, u0, n0, tb.Qp,
                               B, ncols, ncols, red);
  const int u = u0 + (threadIdx.x >> 4), c = n0 + (threadIdx.x & 15);
  if (u < units && c < ncols) out[(long)u * ncols + c] = x;
}

hipError_t launch_lag_gemm(const Tables& tb, const StepArgs& a, int units, double* dq, double* gq,
                           bool skinny, hipStream_t s) {
  if (skinny) {
    dim3 grid((tb.Qp + ST - 1) / ST, (units + ST - 1) / ST);
    k_lag_skinny1d<<<grid, 256, 0, s>>>(tb, a, units, dq, gq);
  } else {
    dim3 grid((tb.Qp + GT - 1) / GT, (units + GT - 1) / GT);
    k_lag_gemm1d<GT, GT><<<grid, 256, 0, s>>>(tb, a, units, dq, gq);
  }
  return hipGetLastError();
}

hipError_t launch_proj_gemm(const Tables& tb, int units, const double* dq, const double* gq,
                            double* m, double* F, bool skinny, hipStream_t s) {
  const int Jm = 2 * tb.Mp + 1;
  const int nc = Jm > tb.Mp ? Jm : tb.Mp;
  if (skinny) {
    dim3 grid((nc + ST - 1) / ST, (units + ST - 1) / ST, 2);
    k_proj_skinny1d<<<grid, 256, 0, s>>>(tb, units, dq, gq, m, Jm, F);
  } else {
    dim3 grid((nc + GT - 1) / GT, (units + GT - 1) / GT, 2);
    k_proj_gemm1d<GT, GT><<<grid, 256, 0, s>>>(tb, units, dq, gq, m, Jm, F);
  }
  return hipGetLastError();
}

// Hybrid fine steps and coarse steps: h = y_L - sum_{i=1}^{L} b_{L+1-i} (y_i - y_{i-1}), and for
// fine steps also - S^-a sum_{c=1}^{n} b_{n-c+r/S} (z_c - z_{c-1}) over the slice ends.  One
// work-group per (unit, block of 128 coefficients); its four waves take the same coefficients
// (two adjacent ones per lane, so every row read is a coalesced 1 KiB segment of 16-byte
// loads) and split the rows of each sum into four contiguous chunks fixed by the row count
// alone (never by the launch), each an ascending fma chain with eight rows in flight; the
// chunk partials meet in LDS and are added as (0 + 1) + (2 + 3).  A serial solve and a
// parareal sweep therefore sum in the same order, bit for bit.  (Measured on the config-2
// fine sweep against one coefficient per lane: 3.8 -> 4.3 TB/s; eight or sixteen chunks, or
// four coefficients per lane, were slower.)
constexpr int HL = 64;       // lanes per wave, two coefficients each
constexpr int HB = 2 * HL;   // coefficients per work-group
constexpr int HW = 4;        // waves (row chunks) per work-group
static_assert(HW == 4, "the chunk partials are added as (0 + 1) + (2 + 3)");

typedef double h2 __attribute__((ext_vector_type(2)));

// sum_{i=i0}^{i1} w(i) (x_i - x_{i-1}) for this lane's two coefficients, rows at x + i stride
template <class WFn>
__device__ inline h2 chunk_sum(const double* x, long stride, int i0, int i1, WFn w) {
  h2 p = {0.0, 0.0};
  if (i0 > i1) return p;
  h2 prev = *reinterpret_cast<const h2*>(x + (long)(i0 - 1) * stride);
  int i = i0;
  for (; i + 7 <= i1; i += 8) {
    h2 r[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) r[q] = *reinterpret_cast<const h2*>(x + (long)(i + q) * stride);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double wq = w(i + q);
      p.x = fma(wq, r[q].x - prev.x, p.x);
      p.y = fma(wq, r[q].y - prev.y, p.y);
      prev = r[q];
    }
  }
  for (; i <= i1; ++i) {
    const h2 xi = *reinterpret_cast<const h2*>(x + (long)i * stride);
    const double wq = w(i);
    p.x = fma(wq, xi.x - prev.x, p.x);
    p.y = fma(wq, xi.y - prev.y, p.y);
    prev = xi;
  }
  return p;
}

__global__ __launch_bounds__(HL * HW) void k_history_split(Tables tb, StepArgs a, double* hist) {
  __shared__ h2 red[2][HW][HL];
  // work-groups reach the 8 XCDs round robin by linear id (x fastest): with the unit count a
  // multiple of 8, XCD x % 8 takes the contiguous eighth x % 8 of the units, so the units of an
  // instance, which share its slice ends, read them into one XCD's L2
  const int nu = gridDim.x;
  const int u = (nu & 7) ? blockIdx.x : (blockIdx.x & 7) * (nu >> 3) + (blockIdx.x >> 3);
  const int lane = threadIdx.x & (HL - 1);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / HL);
  const UnitView v = decode_unit(tb, a, u);
  // Mp is a multiple of 16, so a lane's pair is either wholly inside or wholly past it; lanes
  // past it read coefficients 0 and 1 (in range) and store nothing
  const int Mp = tb.Mp, k = blockIdx.y * HB + 2 * lane;
  const bool in = k < Mp;
  const int kk = in ? k : 0;
  const double* bw = tb.bw + (long)v.b * tb.LB;
  {  // trajectory (or slice-end) part: rows 1..L in HW chunks
    const int L = v.L, len = (L + HW - 1) / HW;
    const int i0 = 1 + wave * len, i1 = min(L, (wave + 1) * len);
    red[0][wave][lane] = chunk_sum(v.y + kk, Mp, i0, i1, [&](int i) { return bw[L + 1 - i]; });
  }
  const bool fine = a.mode == MODE_FINE;
  if (fine) {  // coarse-grid history of the hybrid fine step: slice ends 1..n in HW chunks
    const int nz = v.nz, len = (nz + HW - 1) / HW;
    const int c0 = 1 + wave * len, c1 = min(nz, (wave + 1) * len);
    const double* bh = tb.bhyb + (long)v.b * tb.P * tb.S + (a.r - 1);
    const long S = tb.S;
    red[1][wave][lane] = chunk_sum(v.z + kk, Mp, c0, c1, [&](int c) { return bh[(long)(nz - c) * S]; });
  }
  __syncthreads();
  if (wave != 0 || !in) return;
  const h2 acc = (red[0][0][lane] + red[0][1][lane]) + (red[0][2][lane] + red[0][3][lane]);
  h2 h = *reinterpret_cast<const h2*>(v.y + (long)v.L * Mp + k) - acc;
  if (fine) {
    const h2 acc2 = (red[1][0][lane] + red[1][1][lane]) + (red[1][2][lane] + red[1][3][lane]);
    const double sf = tb.inst[(long)v.b * NSCAL + IS_SFAC];
    h.x = h.x - sf * acc2.x;
    h.y = h.y - sf * acc2.y;
  }
  *reinterpret_cast<h2*>(hist + (long)u * Mp + k) = h;
}

// Full uniform L1 step m with the far history as sums of exponentials (history = 2; the fast
// history of the paper's conclusions): the L1 weights at distances d >= j0 are replaced by
// sum_l w_l e^{-lam_l d}, so the far part of the sum is sum_l w_l V_l with
// V_l = sum_{i <= m+1-j0} e^{-lam_l (m+1-i)} (y_i - y_{i-1}), carried from step to step:
// V_l <- e^{-lam_l} V_l + e^{-lam_l j0} (y_i - y_{i-1}) for the row i = m+1-j0 that has just
// reached distance j0.  The near part (d < j0) uses the exact weights.  One work-group per
// (instance, 128 coefficients), two adjacent coefficients per lane (16-byte loads); its 16
// waves split the nodes into 16 contiguous ranges (fixed by the node count; with few nodes
// the last ranges are empty) and wave 0 also forms the near part; the wave partials of the
// far sum are added pairwise in a fixed tree.  Only B * Mp / 128 work-groups exist (64 at 32
// instances of 256 modes), so the node split across 16 waves is what keeps enough loads in
// flight.  The state goes to HBM between steps (B * soeL * Mp doubles).
constexpr int SL = 64;  // lanes per wave, two coefficients each
constexpr int SW = 16;  // waves (node ranges) per work-group
static_assert(SW == 16, "the wave partials are added pairwise in a fixed tree");

__global__ __launch_bounds__(SL * SW) void k_history_soe(Tables tb, StepArgs a, double* hist) {
  __shared__ h2 red[SW][SL];
  const int u = blockIdx.x, lane = threadIdx.x & (SL - 1);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / SL);
  const int Mp = tb.Mp, k = blockIdx.y * (2 * SL) + 2 * lane;
  const bool in = k < Mp;
  const int kk = in ? k : 0;  // lanes past Mp work on coefficients 0, 1 and store nothing
  const UnitView v = decode_unit(tb, a, u);
  const int m = a.m, L = tb.soeL;
  const double* y = v.y + kk;
  const double* tab = tb.soe + (long)v.b * L * 3;
  double* V = a.soeV + (long)v.b * L * Mp + kk;
  const int inew = m + 1 - kSoeJ0;
  h2 d = {0.0, 0.0};
  if (inew >= 1)
    d = *reinterpret_cast<const h2*>(y + (long)inew * Mp) - *reinterpret_cast<const h2*>(y + (long)(inew - 1) * Mp);
  const int len = (L + SW - 1) / SW, l0 = wave * len, l1 = min(L, l0 + len);
  h2 far = {0.0, 0.0};
  int l = l0;
  for (; l + 7 < l1; l += 8) {
    h2 s[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) s[q] = *reinterpret_cast<const h2*>(V + (long)(l + q) * Mp);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double* t = tab + (l + q) * 3;
      if (inew >= 1) {
        s[q].x = t[1] * s[q].x + t[2] * d.x;
        s[q].y = t[1] * s[q].y + t[2] * d.y;
        if (in) *reinterpret_cast<h2*>(V + (long)(l + q) * Mp) = s[q];
      }
      far.x = fma(t[0], s[q].x, far.x);
      far.y = fma(t[0], s[q].y, far.y);
    }
  }
  for (; l < l1; ++l) {
    const double* t = tab + l * 3;
    h2 sl = *reinterpret_cast<const h2*>(V + (long)l * Mp);
    if (inew >= 1) {
      sl.x = t[1] * sl.x + t[2] * d.x;
      sl.y = t[1] * sl.y + t[2] * d.y;
      if (in) *reinterpret_cast<h2*>(V + (long)l * Mp) = sl;
    }
    far.x = fma(t[0], sl.x, far.x);
    far.y = fma(t[0], sl.y, far.y);
  }
  red[wave][lane] = far;
  __syncthreads();
  if (wave != 0 || !in) return;
  h2 p8[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) p8[q] = red[2 * q][lane] + red[2 * q + 1][lane];
  const h2 farsum = ((p8[0] + p8[1]) + (p8[2] + p8[3])) + ((p8[4] + p8[5]) + (p8[6] + p8[7]));
  const double* bw = tb.bw + (long)v.b * tb.LB;
  h2 near = {0.0, 0.0};
  for (int i = inew + 1 > 1 ? inew + 1 : 1; i <= m; ++i) {
    const h2 di = *reinterpret_cast<const h2*>(y + (long)i * Mp) - *reinterpret_cast<const h2*>(y + (long)(i - 1) * Mp);
    near.x = fma(bw[m + 1 - i], di.x, near.x);
    near.y = fma(bw[m + 1 - i], di.y, near.y);
  }
  const h2 ym = *reinterpret_cast<const h2*>(y + (long)m * Mp);
  *reinterpret_cast<h2*>(hist + (long)u * Mp + k) = ym - (farsum + near);
}

hipError_t launch_history(const Tables& tb, const StepArgs& a, int units, double* hist,
                          hipStream_t s) {
  if (a.mode == MODE_FULL && tb.soe) {
    if (tb.Mp % 2 != 0) return hipErrorInvalidValue;
    k_history_soe<<<dim3(units, (tb.Mp + 2 * SL - 1) / (2 * SL)), SL * SW, 0, s>>>(tb, a, hist);
    return hipGetLastError();
  }
  const bool full = a.mode == MODE_FULL || (a.mode == MODE_FINE && a.prev);
  if (full) {
    const int threads = tb.Mp < 256 ? roundup(tb.Mp, 64) : 256;
    k_history1d<<<dim3(units, (tb.Mp + threads - 1) / threads), threads, 0, s>>>(tb, a, hist);
  } else {
    const int nblk = (tb.Mp + HB - 1) / HB;
    if (nblk > 65535 || tb.Mp % 2 != 0) return hipErrorInvalidValue;
    k_history_split<<<dim3(units, nblk), HL * HW, 0, s>>>(tb, a, hist);
  }
  return hipGetLastError();
}

}  // namespace l1pr
