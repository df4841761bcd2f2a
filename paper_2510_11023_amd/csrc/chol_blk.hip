// Blocked Cholesky factorisation and solve of one step's system per unit, through device
// memory, for systems too large for one work-group's registers (padded size Mp > 256; the
// 2D tensor basis at 64 x 64 modes gives Mp = 4096).  A = I + tau K is symmetric positive
// definite (Section 2.1: the stiffness is positive semidefinite for D > 0, the mass matrix
// is the identity in the orthonormal sine basis), so no pivoting is needed.
//
// Right-looking by blocks of nb columns (nb <= 256, a multiple of 16), rows and columns of
// the block j at r0 = j nb:
//   k_blk_diag   (step1d_reg.hip) factors A_jj in registers, forward-substitutes the
//                right-hand side block (y_j over b_j), and replaces A_jj by X_j = L_jj^-1;
//   k_blk_panel  L_ij = A_ij X_j^T for the rows below (a GEMM with the triangular X_j, staged
//                through LDS; tiles of X_j above its diagonal are skipped), and b_i -= L_ij y_j;
//   k_blk_trail  A_ik -= L_ij L_kj^T on the lower 128 x 128 tiles of the trailing matrix
//                (FP64 MFMA 16x16x4, eight waves of 64 x 32, operands staged through LDS, the
//                next chunk prefetched into registers while the current one is multiplied).
// Back substitution L^T x = y, last block first:
//   k_blk_bs_part  q_ij = L_ij^T x_i for every block i > j (one 1024-thread work-group per block)
//   k_blk_bs_diag  x_j = X_j^T (y_j - sum_{i > j} q_ij), the sum in ascending i, then the
//                  step's epilogue for the block's entries.
// 1D steps add one step of iterative refinement (k_blk_resid1d, k_blk_fs, the back
// substitution again; see there).
// Every output is a fixed-order sum that depends only on its own unit's data, so a unit's
// result does not depend on the number of units in the launch (a serial solve and a parareal
// fine sweep agree bit for bit).
#include "l1pr_internal.h"

namespace l1pr {

typedef double d4 __attribute__((ext_vector_type(4)));

// LDS row stride of the staged 16-column chunks: an MFMA operand read takes 16 rows x 4
// columns (lane l: row l%16, column l/16); with 18 doubles per row the 32 lanes of each half
// of a 64-bit read fall on 64 distinct banks (17 would put two lanes on some banks).
constexpr int TKP = 18;

__device__ inline bool unit_idle(const Tables& tb, const StepArgs& a, int u) {
  if (a.mode != MODE_FINE) return false;
  const int b = u / a.nP;
  return a.r > (int)tb.inst[(long)b * NSCAL + IS_SB];
}

// ---------------------------------------------------------------------------- panel
// One work-group per 64 rows R0 .. R0+63 of the panel below block j (w = nb columns):
// L[R][c] = sum_k A[R][r0 + k] X[c][k], X lower triangular, so column tile T (16 wide) takes
// the k chunks kc <= T.  Wave v owns the column tiles {v, 7-v, 8+v, 15-v} (equal work: the
// chunk counts add up to 34 for every wave) for all four 16-row tiles; the A chunk (64 x 16)
// and the X chunk (rows 16 kc .. w-1) are staged in LDS.  MFMA operands: A lane l =
// A[R0 + 16 x + l%16][k0 + l/16], B lane l = X[16 T + l%16][k0 + l/16]; the result tile holds
// L[R0 + 16 x + l/16 + 4v][16 T + l%16].  Then b_R -= sum_c L[R][c] y[c] (lane partials, the
// 16 lanes of a row, then the four waves in order), and L is stored over A: the work-group's
// reads of its rows all precede the last barrier of the loop.
__device__ inline int panel_tile(int v, int y) {
  return y == 0 ? v : (y == 1 ? 7 - v : (y == 2 ? 8 + v : 15 - v));
}

__global__ __launch_bounds__(256) void k_blk_panel(Tables tb, StepArgs a, double* A, double* rhs,
                                                   int r0, int w) {
  __shared__ double sA[64][TKP];
  __shared__ double sX[256][TKP];
  __shared__ double sred[4][64];
  const int u = blockIdx.y, tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  if (unit_idle(tb, a, u)) return;
  const int Mp = tb.Mp, nt = w / 16;
  const int R0 = r0 + w + blockIdx.x * 64;
  const int lr = lane >> 4, lc = lane & 15;
  double* Au = A + (long)u * Mp * Mp;
  const double* X = Au + (long)r0 * Mp + r0;
  d4 acc[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = d4{0.0, 0.0, 0.0, 0.0};
  // chunk kc: A rows R0 + (e >> 4), X rows 16 kc + (e >> 4), column 16 kc + (e & 15) for the
  // thread's e = tid + 256 q; the next chunk is loaded into registers during the MFMAs
  double na[4], nx[16];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q, r = e >> 4, k = e & 15;
      na[q] = (R0 + r < Mp) ? Au[(long)(R0 + r) * Mp + r0 + k0 + k] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = tid + 256 * q;
      if (e < (w - k0) * 16) nx[q] = X[(long)(k0 + (e >> 4)) * Mp + k0 + (e & 15)];
    }
  };
  load(0);
  for (int kc = 0; kc < nt; ++kc) {
    const int k0 = kc * 16;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      sA[e >> 4][e & 15] = na[q];
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = tid + 256 * q;
      if (e < (w - k0) * 16) sX[k0 + (e >> 4)][e & 15] = nx[q];
    }
    __syncthreads();
    if (kc + 1 < nt) load(k0 + 16);
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int kq = ks * 4 + lr;
      double af[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) af[x] = sA[x * 16 + lc][kq];
#pragma unroll
      for (int y = 0; y < 4; ++y) {
        const int T = panel_tile(wv, y);
        if (T >= nt || T < kc) continue;  // wave-uniform
        const double bf = sX[T * 16 + lc][kq];
#pragma unroll
        for (int x = 0; x < 4; ++x)
          acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[x], bf, acc[x][y], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // b_R -= sum_c L[R][c] y[c]
  const double* yv = rhs + (long)u * Mp + r0;
  double p[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int v = 0; v < 4; ++v) p[x][v] = 0.0;
#pragma unroll
  for (int y = 0; y < 4; ++y) {
    const int T = panel_tile(wv, y);
    if (T >= nt) continue;
    const double yc = yv[T * 16 + lc];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int v = 0; v < 4; ++v) p[x][v] = fma(acc[x][y][v], yc, p[x][v]);
  }
#pragma unroll
  for (int off = 8; off >= 1; off >>= 1)
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int v = 0; v < 4; ++v) p[x][v] += __shfl_xor(p[x][v], off, 16);
  if (lc == 0) {
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int v = 0; v < 4; ++v) sred[wv][x * 16 + lr + 4 * v] = p[x][v];
  }
  __syncthreads();
  if (tid < 64 && R0 + tid < Mp)
    rhs[(long)u * Mp + R0 + tid] -= (sred[0][tid] + sred[1][tid]) + (sred[2][tid] + sred[3][tid]);
#pragma unroll
  for (int y = 0; y < 4; ++y) {
    const int T = panel_tile(wv, y);
    if (T >= nt) continue;
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      if (R0 + x * 16 >= Mp) continue;  // the panel height is a multiple of 16
#pragma unroll
      for (int v = 0; v < 4; ++v)
        Au[(long)(R0 + x * 16 + lr + 4 * v) * Mp + r0 + T * 16 + lc] = acc[x][y][v];
    }
  }
}

// ---------------------------------------------------------------------------- trailing
// Lower 128 x 128 tiles (I >= K) of the trailing matrix, rows and columns from rs = r0 + w.
// Eight waves as 2 x 4, each a 64 x 32 part (4 x 2 MFMA tiles); each tile starts from A_IK
// and takes -L_I L_K^T in chunks of 16 panel columns staged in LDS, the next chunk loaded into
// registers during the MFMAs.  Loads are branch-free (a row past Mp is clamped to row Mp - 1
// and its value replaced by 0; the padded size is a multiple of 16); rows past Mp are not
// written.  The linear work-group index is remapped so that the work-groups the dispatcher
// sends to one XCD (every 8th) take a contiguous run of (unit, tile) pairs, row by row: they
// share panel rows in that XCD's L2.
constexpr int TB = 128, TK = 16, TT = 512, NXCD = 8;
static_assert(TKP >= TK, "chunk rows hold TK columns");

__device__ inline int xcd_remap(int id, int total) {
  const int q = total / NXCD, rem = total % NXCD, x = id % NXCD, k = id / NXCD;
  return x < rem ? x * (q + 1) + k : rem * (q + 1) + (x - rem) * q + k;
}

__global__ __launch_bounds__(TT, 4) void k_blk_trail(Tables tb, StepArgs a, double* A, int r0, int w,
                                                  int ntile) {
  __shared__ double sI[TB][TKP];
  __shared__ double sK[TB][TKP];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lin = xcd_remap(blockIdx.x, gridDim.x);
  const int u = lin / ntile, t = lin % ntile;
  if (unit_idle(tb, a, u)) return;
  const int Mp = tb.Mp, rs = r0 + w;
  // tile (I, K) from the triangular index t = I (I + 1) / 2 + K
  int I = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  while (I * (I + 1) / 2 > t) --I;
  const int K = t - I * (I + 1) / 2;
  const int i0 = rs + I * TB, k0r = rs + K * TB;
  const int wi = wave >> 2, wj = wave & 3, lr = lane >> 4, lc = lane & 15;
  double* Au = A + (long)u * Mp * Mp;
  // (the accumulators are filled 8 loads at a time: a scheduling fence between the groups
  // keeps the register peak, and so the occupancy, at that of the main loop)
  d4 acc[4][2];
#pragma unroll
  for (int x = 0; x < 4; ++x) {
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + wi * 64 + x * 16 + lr + 4 * v, j = k0r + wj * 32 + y * 16 + lc;
        const double c = Au[(long)min(i, Mp - 1) * Mp + min(j, Mp - 1)];
        acc[x][y][v] = (i < Mp && j < Mp) ? c : 0.0;
      }
    __builtin_amdgcn_sched_barrier(0);
  }
  // chunk loads: thread tid takes rows (tid >> 4) + 32 q (q < 4), column tid & 15 of each operand
  const int lrow = tid >> 4, lcol = tid & 15;
  const double* pc = Au + r0 + lcol;
  double nI[4], nK[4];
  auto load = [&](int kb) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ri = i0 + lrow + 32 * q, rk = k0r + lrow + 32 * q;
      const double vi = pc[(long)min(ri, Mp - 1) * Mp + kb];
      const double vk = pc[(long)min(rk, Mp - 1) * Mp + kb];
      nI[q] = ri < Mp ? vi : 0.0;
      nK[q] = rk < Mp ? vk : 0.0;
    }
  };
  load(0);
  for (int kb = 0; kb < w; kb += TK) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      sI[lrow + 32 * q][lcol] = nI[q];
      sK[lrow + 32 * q][lcol] = nK[q];
    }
    __syncthreads();
    if (kb + TK < w) load(kb + TK);
#pragma unroll
    for (int ks = 0; ks < TK / 4; ++ks) {
      const int kq = ks * 4 + lr;
      double af[4], bf[2];
#pragma unroll
      for (int x = 0; x < 4; ++x) af[x] = -sI[wi * 64 + x * 16 + lc][kq];
#pragma unroll
      for (int y = 0; y < 2; ++y) bf[y] = sK[wj * 32 + y * 16 + lc][kq];
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[x], bf[y], acc[x][y], 0, 0, 0);
    }
    __syncthreads();
  }
  const bool whole = i0 + TB <= Mp && k0r + TB <= Mp;  // uniform
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + wi * 64 + x * 16 + lr + 4 * v, j = k0r + wj * 32 + y * 16 + lc;
        if (whole || (i < Mp && j < Mp)) Au[(long)i * Mp + j] = acc[x][y][v];
      }
}

// The 64 x 64 variant (tune bit TUNE_TRAIL64): four waves of 32 x 32 (2 x 2 MFMA tiles), the
// same chunking, remap and branch-free loads.
constexpr int TB64 = 64;

__global__ __launch_bounds__(256) void k_blk_trail64(Tables tb, StepArgs a, double* A, int r0, int w,
                                                     int ntile) {
  __shared__ double sI[TB64][TKP];
  __shared__ double sK[TB64][TKP];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lin = xcd_remap(blockIdx.x, gridDim.x);
  const int u = lin / ntile, t = lin % ntile;
  if (unit_idle(tb, a, u)) return;
  const int Mp = tb.Mp, rs = r0 + w;
  int I = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  while (I * (I + 1) / 2 > t) --I;
  const int K = t - I * (I + 1) / 2;
  const int i0 = rs + I * TB64, k0r = rs + K * TB64;
  const int wi = wave >> 1, wj = wave & 1, lr = lane >> 4, lc = lane & 15;
  double* Au = A + (long)u * Mp * Mp;
  d4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + wi * 32 + x * 16 + lr + 4 * v, j = k0r + wj * 32 + y * 16 + lc;
        const double c = Au[(long)min(i, Mp - 1) * Mp + min(j, Mp - 1)];
        acc[x][y][v] = (i < Mp && j < Mp) ? c : 0.0;
      }
  // chunk loads: thread tid takes rows (tid >> 4) + 16 q (q < 4), column tid & 15
  const int lrow = tid >> 4, lcol = tid & 15;
  const double* pc = Au + r0 + lcol;
  double nI[4], nK[4];
  auto load = [&](int kb) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ri = i0 + lrow + 16 * q, rk = k0r + lrow + 16 * q;
      const double vi = pc[(long)min(ri, Mp - 1) * Mp + kb];
      const double vk = pc[(long)min(rk, Mp - 1) * Mp + kb];
      nI[q] = ri < Mp ? vi : 0.0;
      nK[q] = rk < Mp ? vk : 0.0;
    }
  };
  load(0);
  for (int kb = 0; kb < w; kb += TK) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      sI[lrow + 16 * q][lcol] = nI[q];
      sK[lrow + 16 * q][lcol] = nK[q];
    }
    __syncthreads();
    if (kb + TK < w) load(kb + TK);
#pragma unroll
    for (int ks = 0; ks < TK / 4; ++ks) {
      const int kq = ks * 4 + lr;
      double af[2], bf[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) af[x] = -sI[wi * 32 + x * 16 + lc][kq];
#pragma unroll
      for (int y = 0; y < 2; ++y) bf[y] = sK[wj * 32 + y * 16 + lc][kq];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[x], bf[y], acc[x][y], 0, 0, 0);
    }
    __syncthreads();
  }
  const bool whole = i0 + TB64 <= Mp && k0r + TB64 <= Mp;  // uniform
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + wi * 32 + x * 16 + lr + 4 * v, j = k0r + wj * 32 + y * 16 + lc;
        if (whole || (i < Mp && j < Mp)) Au[(long)i * Mp + j] = acc[x][y][v];
      }
}

// ---------------------------------------------------------------------------- back substitution
// q[u][i][c] = sum_r L[ri + r][r0 + c] x[ri + r] over the rows of block i (ri = i nb, width
// wi), one work-group of 1024 threads per block i > j: thread (g, c) sums the rows r = g mod 4
// (coalesced rows of L), then the four partial sums are added in the order (0 + 1) + (2 + 3).
__global__ __launch_bounds__(1024) void k_blk_bs_part(Tables tb, StepArgs a, const double* A,
                                                      const double* rhs, double* q, int j, int nb,
                                                      int nblk) {
  __shared__ double red[4][256];
  const int u = blockIdx.y, c = threadIdx.x & 255, g = threadIdx.x >> 8;
  if (unit_idle(tb, a, u)) return;
  const int Mp = tb.Mp, i = j + 1 + blockIdx.x;
  const int r0 = j * nb, ri = i * nb, wi = (Mp - ri) < nb ? (Mp - ri) : nb;
  const int wj = (Mp - r0) < nb ? (Mp - r0) : nb;
  double sum = 0.0;
  if (c < wj) {
    const double* L = A + (long)u * Mp * Mp + (long)ri * Mp + r0 + c;
    const double* x = rhs + (long)u * Mp + ri;
#pragma unroll 4
    for (int r = g; r < wi; r += 4) sum = fma(L[(long)r * Mp], x[r], sum);
  }
  red[g][c] = sum;
  __syncthreads();
  if (g == 0 && c < wj) q[((long)u * nblk + i) * nb + c] = (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
}

// x_j = X_j^T z_j with z_j = y_j - sum_{i > j} q_ij (ascending i); X_j[r][c] is read for r
// at or below the diagonal tile of c (the tiles above it are stale), thread (g, c) taking the
// rows r = g mod 4 and the partial sums added as (0 + 1) + (2 + 3).  Then the epilogue.
__global__ __launch_bounds__(1024) void k_blk_bs_diag(Tables tb, StepArgs a, Epilogue ep,
                                                      const double* A, double* rhs, const double* q,
                                                      int j, int nb, int nblk, const double* xadd) {
  __shared__ double z[256];
  __shared__ double red[4][256];
  const int u = blockIdx.x, c = threadIdx.x & 255, g = threadIdx.x >> 8;
  if (unit_idle(tb, a, u)) return;
  const int Mp = tb.Mp, r0 = j * nb, wj = (Mp - r0) < nb ? (Mp - r0) : nb;
  double* yu = rhs + (long)u * Mp + r0;
  if (g == 0 && c < wj) {
    double zc = yu[c];
    for (int i = j + 1; i < nblk; ++i) zc -= q[((long)u * nblk + i) * nb + c];
    z[c] = zc;
  }
  __syncthreads();
  double sum = 0.0;
  if (c < wj) {
    const double* X = A + (long)u * Mp * Mp + (long)r0 * Mp + r0 + c;
#pragma unroll 4
    for (int r = (c & ~15) + g; r < wj; r += 4) sum = fma(X[(long)r * Mp], z[r], sum);
  }
  red[g][c] = sum;
  __syncthreads();
  if (g != 0 || c >= wj) return;
  const double x = (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
  yu[c] = x;
  if (ep.kind == EPI_NONE) return;
  // refinement: the correction is added to the first solution
  const double xo = xadd ? xadd[(long)u * Mp + r0 + c] + x : x;
  const UnitView v = decode_unit(tb, a, u);
  const bool last = (a.mode == MODE_FINE) && (a.r == v.Sb);
  epi_store(a, ep, u, v.slot, last, r0 + c, xo);
}

// ---------------------------------------------------------------------------- refinement
// The panels and the back substitution apply each diagonal block through its explicit
// inverse X_j = L_jj^-1, whose rounding error grows with the block's condition number (at
// nb = 256 and cond(A) of 1e5 to 1e6 the solve error is a few 1e-11 relative, per step).  One
// step of fixed-precision iterative refinement removes that: the residual of the computed x
// is formed in FP64 with the step's own operator, r = rhs0 - x - tau dphi^T (d o (dphi x)),
// the correction e solves L L^T e = r with the stored factor, and x + e is stored.  The
// solve only has to reduce the error by a constant factor for the refined x to reach the
// accuracy of the residual (a backward-stable solve's).  Every sum has a fixed order over the
// unit's own data, so serial and parareal runs still agree bit for bit.

// wave-wide sum, read from lane 0 (xor butterfly: lane 0's order is fixed)
__device__ inline double wave_sum0(double p) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) p += __shfl_xor(p, off);
  return p;
}

// One 256-thread work-group per unit; LDS holds x [Mp] and the weighted gradient [Qp].
__global__ __launch_bounds__(256) void k_blk_resid1d(Tables tb, StepArgs a, const double* rhs0,
                                                     double* rhs, double* xs) {
  extern __shared__ double sm[];
  const int u = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (unit_idle(tb, a, u)) return;
  const int Mp = tb.Mp, Qp = tb.Qp;
  double* sx = sm;
  double* sw = sm + Mp;
  double* ru = rhs + (long)u * Mp;
  for (int k = tid; k < Mp; k += 256) {
    const double x = ru[k];
    sx[k] = x;
    xs[(long)u * Mp + k] = x;
  }
  __syncthreads();
  // sw_q = d_q sum_k dphi[q][k] x_k (one wave per node, lanes along the row)
  const double* d = a.d + (long)u * Qp;
  for (int q = wave; q < Qp; q += 4) {
    const double* row = tb.dphi + (long)q * Mp;
    double p = 0.0;
    for (int k = lane; k < Mp; k += 64) p = fma(row[k], sx[k], p);
    p = wave_sum0(p);
    if (lane == 0) sw[q] = d[q] * p;
  }
  __syncthreads();
  const int b = (a.mode == MODE_FINE) ? u / a.nP : u;
  const double tau = tb.inst[(long)b * NSCAL + ((a.mode == MODE_COARSE) ? IS_TAUC : IS_TAU)];
  for (int k = tid; k < Mp; k += 256) {
    double s = 0.0;
    for (int q = 0; q < Qp; ++q) s = fma(tb.dphi[(long)q * Mp + k], sw[q], s);
    ru[k] = (rhs0[(long)u * Mp + k] - sx[k]) - tau * s;
  }
}

// Forward substitution L y = r with the stored factor, one 1024-thread work-group per unit
// (Mp <= 1024), block by block: z_j = r_j - sum_{t < r0} L[r0 + c][t] y_t, then y_j = X_j z_j
// (row c of X_j read up to the end of its diagonal 16 x 16 tile; the tiles above are stale).
// One wave per row, lanes along it.
constexpr int kFsMax = 1024;

__global__ __launch_bounds__(1024) void k_blk_fs(Tables tb, StepArgs a, const double* A,
                                                 double* rhs, int nb) {
  __shared__ double sy[kFsMax];
  __shared__ double sz[256];
  const int u = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (unit_idle(tb, a, u)) return;
  const int Mp = tb.Mp;
  const double* Au = A + (long)u * Mp * Mp;
  double* ru = rhs + (long)u * Mp;
  for (int k = tid; k < Mp; k += 1024) sy[k] = ru[k];
  __syncthreads();
  for (int r0 = 0; r0 < Mp; r0 += nb) {
    const int w = (Mp - r0) < nb ? (Mp - r0) : nb;
    for (int c = wave; c < w; c += 16) {
      const double* row = Au + (long)(r0 + c) * Mp;
      double p = 0.0;
      for (int t = lane; t < r0; t += 64) p = fma(row[t], sy[t], p);
      p = wave_sum0(p);
      if (lane == 0) sz[c] = sy[r0 + c] - p;
    }
    __syncthreads();
    for (int c = wave; c < w; c += 16) {
      const double* row = Au + (long)(r0 + c) * Mp + r0;
      const int tend = (c | 15) + 1;
      double p = 0.0;
      for (int t = lane; t < tend; t += 64) p = fma(row[t], sz[t], p);
      p = wave_sum0(p);
      if (lane == 0) sy[r0 + c] = p;
    }
    __syncthreads();
  }
  for (int k = tid; k < Mp; k += 1024) ru[k] = sy[k];
}

// L^T x = y by blocks, last first; the epilogue stores x (plus xadd when set)
static hipError_t blk_back_subst(const Tables& tb, const StepArgs& a, const Epilogue& e, int units,
                                 double* q, const double* xadd, hipStream_t s) {
  const int Mp = tb.Mp, nb = tb.nb, nblk = (Mp + nb - 1) / nb;
  for (int j = nblk - 1; j >= 0; --j) {
    if (j < nblk - 1) {
      k_blk_bs_part<<<dim3(nblk - 1 - j, units), 1024, 0, s>>>(tb, a, a.A, a.rhs, q, j, nb, nblk);
      hipError_t r = hipGetLastError();
      if (r != hipSuccess) return r;
    }
    k_blk_bs_diag<<<units, 1024, 0, s>>>(tb, a, e, a.A, a.rhs, q, j, nb, nblk, xadd);
    hipError_t r = hipGetLastError();
    if (r != hipSuccess) return r;
  }
  return hipSuccess;
}

hipError_t launch_blk_solve(const Tables& tb, const StepArgs& a, const Epilogue& e, int units,
                            double* q, hipStream_t s) {
  const int Mp = tb.Mp, nb = tb.nb, nblk = (Mp + nb - 1) / nb;
  if (nb < 16 || nb > 256 || nb % 16 != 0 || Mp % 16 != 0) return hipErrorInvalidValue;
  for (int j = 0; j < nblk; ++j) {
    const int r0 = j * nb, w = (Mp - r0) < nb ? (Mp - r0) : nb;
    hipError_t r = launch_blk_diag(tb, a, units, a.A, a.rhs, r0, w, s);
    if (r != hipSuccess) return r;
    const int below = Mp - r0 - w;
    if (below == 0) break;
    k_blk_panel<<<dim3((below + 63) / 64, units), 256, 0, s>>>(tb, a, a.A, a.rhs, r0, w);
    if ((r = hipGetLastError()) != hipSuccess) return r;
    const bool t64 = (tb.tune & TUNE_TRAIL64) != 0;
    const int tbw = t64 ? TB64 : TB, tt = (below + tbw - 1) / tbw, ntile = tt * (tt + 1) / 2;
    const long nwg = (long)ntile * units;
    if (nwg > 0x7fffffffL) return hipErrorInvalidValue;
    if (t64) k_blk_trail64<<<(unsigned)nwg, 256, 0, s>>>(tb, a, a.A, r0, w, ntile);
    else k_blk_trail<<<(unsigned)nwg, TT, 0, s>>>(tb, a, a.A, r0, w, ntile);
    if ((r = hipGetLastError()) != hipSuccess) return r;
  }
  return blk_back_subst(tb, a, e, units, q, nullptr, s);
}

hipError_t launch_blk_refine1d(const Tables& tb, const StepArgs& a, const Epilogue& e, int units,
                               double* q, const double* rhs0, double* xs, hipStream_t s) {
  const int Mp = tb.Mp, nb = tb.nb;
  if (tb.dim != 1 || Mp > kFsMax || nb < 16 || nb > 256 || nb % 16 != 0 || Mp % 16 != 0 ||
      (size_t)(tb.Mp + tb.Qp) * sizeof(double) > 64 * 1024)
    return hipErrorInvalidValue;
  const size_t lds = sizeof(double) * (tb.Mp + tb.Qp);
  k_blk_resid1d<<<units, 256, lds, s>>>(tb, a, rhs0, a.rhs, xs);
  hipError_t r = hipGetLastError();
  if (r != hipSuccess) return r;
  k_blk_fs<<<units, 1024, 0, s>>>(tb, a, a.A, a.rhs, nb);
  if ((r = hipGetLastError()) != hipSuccess) return r;
  return blk_back_subst(tb, a, e, units, q, xs, s);
}

}  // namespace l1pr
