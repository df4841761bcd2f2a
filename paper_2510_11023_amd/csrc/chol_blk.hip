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
//   k_blk_panel  L_ij = A_ij X_j^T for the rows below (a GEMM with the triangular X_j; tiles
//                of X_j above its diagonal are skipped), and b_i -= L_ij y_j;
//   k_blk_trail  A_ik -= L_ij L_kj^T on the lower 64 x 64 tiles of the trailing matrix
//                (FP64 MFMA 16x16x4, operands staged through LDS, the next chunk prefetched
//                into registers while the current one is multiplied).
// Back substitution L^T x = y, last block first:
//   k_blk_bs_part  q_ij = L_ij^T x_i for every block i > j (one work-group per block)
//   k_blk_bs_diag  x_j = X_j^T (y_j - sum_{i > j} q_ij), the sum in ascending i, then the
//                  step's epilogue for the block's entries.
// Every output is a fixed-order sum that depends only on its own unit's data, so a unit's
// result does not depend on the number of units in the launch (a serial solve and a parareal
// fine sweep agree bit for bit).
#include "l1pr_internal.h"

namespace l1pr {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ inline bool unit_idle(const Tables& tb, const StepArgs& a, int u) {
  if (a.mode != MODE_FINE) return false;
  const int b = u / a.nP;
  return a.r > (int)tb.inst[(long)b * NSCAL + IS_SB];
}

// ---------------------------------------------------------------------------- panel
// One wave per 16 rows R0 .. R0+15 of the panel below block j (w = nb columns): 16 output
// tiles in registers, L_T[r][c] = sum_k A[R0 + r][r0 + k] X[16 T + c][k] over the k chunks
// kc <= T (X is lower triangular).  MFMA operands: A lane l = A[R0 + l%16][k0 + l/16],
// B lane l = X[16 T + l%16][k0 + l/16]; the result tile holds L[R0 + l/16 + 4v][16 T + l%16].
// Reads of a wave's rows all precede its stores, and no other wave touches those rows.
__global__ __launch_bounds__(256) void k_blk_panel(Tables tb, StepArgs a, double* A, double* rhs,
                                                   int r0, int w) {
  const int u = blockIdx.y, lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int Mp = tb.Mp, nt = w / 16;
  const int R0 = r0 + w + blockIdx.x * 64 + wave * 16;
  if (R0 >= Mp || unit_idle(tb, a, u)) return;
  const int lr = lane >> 4, lc = lane & 15;
  double* Au = A + (long)u * Mp * Mp;
  const double* arow = Au + (long)(R0 + lc) * Mp + r0 + lr;     // A[R0 + lc][r0 + lr + k0]
  const double* X = Au + (long)r0 * Mp + r0;                     // X_j, row stride Mp
  d4 acc[16];
#pragma unroll
  for (int T = 0; T < 16; ++T) acc[T] = d4{0.0, 0.0, 0.0, 0.0};
  for (int kc = 0; kc < nt; ++kc) {
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int k0 = kc * 16 + ks * 4;
      const double av = arow[k0];
#pragma unroll
      for (int T = 0; T < 16; ++T) {
        if (T < kc || T >= nt) continue;  // wave-uniform
        const double bv = X[(long)(T * 16 + lc) * Mp + k0 + lr];
        acc[T] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[T], 0, 0, 0);
      }
    }
  }
  // b_R -= sum_c L[R][c] y[c]: lane partials over the tiles, then over the 16 lanes of a row
  const double* y = rhs + (long)u * Mp + r0;
  double p[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int T = 0; T < 16; ++T) {
    if (T >= nt) continue;
    const double yc = y[T * 16 + lc];
#pragma unroll
    for (int v = 0; v < 4; ++v) p[v] = fma(acc[T][v], yc, p[v]);
  }
#pragma unroll
  for (int off = 8; off >= 1; off >>= 1)
#pragma unroll
    for (int v = 0; v < 4; ++v) p[v] += __shfl_xor(p[v], off, 16);
  // all reads of these rows are done (their values are in registers); store L over A
#pragma unroll
  for (int T = 0; T < 16; ++T) {
    if (T >= nt) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) Au[(long)(R0 + lr + 4 * v) * Mp + r0 + T * 16 + lc] = acc[T][v];
  }
  if (lc == 0) {
    double* bR = rhs + (long)u * Mp + R0 + lr;
#pragma unroll
    for (int v = 0; v < 4; ++v) bR[4 * v] -= p[v];
  }
}

// ---------------------------------------------------------------------------- trailing
// Lower 64 x 64 tiles (I >= K) of the trailing matrix, rows and columns from rs = r0 + w;
// blockIdx.x enumerates them row by row (t = I (I + 1) / 2 + K).  Four waves, 2 x 2 MFMA
// tiles each; the tile starts from A_IK and takes -L_I L_K^T in chunks of 16 columns of the
// panel.  Rows past Mp (a partial last tile) are neither read nor written.
constexpr int TB = 64, TK = 16;

__global__ __launch_bounds__(256) void k_blk_trail(Tables tb, StepArgs a, double* A, int r0, int w) {
  __shared__ double sI[TB][TK + 1];
  __shared__ double sK[TB][TK + 1];
  const int u = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (unit_idle(tb, a, u)) return;
  const int Mp = tb.Mp, rs = r0 + w;
  // tile (I, K) from the triangular index
  const int t = blockIdx.x;
  int I = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  while (I * (I + 1) / 2 > t) --I;
  const int K = t - I * (I + 1) / 2;
  const int i0 = rs + I * TB, k0r = rs + K * TB;
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
        acc[x][y][v] = (i < Mp && j < Mp) ? Au[(long)i * Mp + j] : 0.0;
      }
  // chunk loads: thread tid takes (row tid / 4 + 0 / 64 ..., 4 columns); four rows per thread
  const int lrow = tid >> 2, lcol = (tid & 3) * 4;
  double nI[4], nK[4];
  auto load = [&](int kb) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = r0 + kb + lcol + q;
      nI[q] = (i0 + lrow < Mp) ? Au[(long)(i0 + lrow) * Mp + c] : 0.0;
      nK[q] = (k0r + lrow < Mp) ? Au[(long)(k0r + lrow) * Mp + c] : 0.0;
    }
  };
  load(0);
  for (int kb = 0; kb < w; kb += TK) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      sI[lrow][lcol + q] = nI[q];
      sK[lrow][lcol + q] = nK[q];
    }
    __syncthreads();
    if (kb + TK < w) load(kb + TK);
#pragma unroll
    for (int ks = 0; ks < TK / 4; ++ks) {
      const int kq = ks * 4 + lr;
      double af[2], bf[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) af[x] = sI[wi * 32 + x * 16 + lc][kq];
#pragma unroll
      for (int y = 0; y < 2; ++y) bf[y] = sK[wj * 32 + y * 16 + lc][kq];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(-af[x], bf[y], acc[x][y], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + wi * 32 + x * 16 + lr + 4 * v, j = k0r + wj * 32 + y * 16 + lc;
        if (i < Mp && j < Mp) Au[(long)i * Mp + j] = acc[x][y][v];
      }
}

// ---------------------------------------------------------------------------- back substitution
// q[u][i][c] = sum_r L[ri + r][r0 + c] x[ri + r] over the rows of block i (ri = i nb, width
// wi), one work-group per block i > j, thread c per column (coalesced rows of L).
__global__ __launch_bounds__(256) void k_blk_bs_part(Tables tb, StepArgs a, const double* A,
                                                     const double* rhs, double* q, int j, int nb,
                                                     int nblk) {
  const int u = blockIdx.y, c = threadIdx.x;
  if (unit_idle(tb, a, u)) return;
  const int Mp = tb.Mp, i = j + 1 + blockIdx.x;
  const int r0 = j * nb, ri = i * nb, wi = (Mp - ri) < nb ? (Mp - ri) : nb;
  const int wj = (Mp - r0) < nb ? (Mp - r0) : nb;
  if (c >= wj) return;
  const double* L = A + (long)u * Mp * Mp + (long)ri * Mp + r0 + c;
  const double* x = rhs + (long)u * Mp + ri;
  double s = 0.0;
  for (int r = 0; r < wi; ++r) s = fma(L[(long)r * Mp], x[r], s);
  q[((long)u * nblk + i) * nb + c] = s;
}

// x_j = X_j^T z_j with z_j = y_j - sum_{i > j} q_ij; X_j[r][c] is read for r at or below the
// diagonal tile of c (the tiles above it are stale).  Then the epilogue for the block.
__global__ __launch_bounds__(256) void k_blk_bs_diag(Tables tb, StepArgs a, Epilogue ep,
                                                     const double* A, double* rhs, const double* q,
                                                     int j, int nb, int nblk) {
  __shared__ double z[256];
  const int u = blockIdx.x, c = threadIdx.x;
  if (unit_idle(tb, a, u)) return;
  const int Mp = tb.Mp, r0 = j * nb, wj = (Mp - r0) < nb ? (Mp - r0) : nb;
  double* yu = rhs + (long)u * Mp + r0;
  if (c < wj) {
    double zc = yu[c];
    for (int i = j + 1; i < nblk; ++i) zc -= q[((long)u * nblk + i) * nb + c];
    z[c] = zc;
  }
  __syncthreads();
  if (c >= wj) return;
  const double* X = A + (long)u * Mp * Mp + (long)r0 * Mp + r0 + c;
  double x = 0.0;
  for (int r = c & ~15; r < wj; ++r) x = fma(X[(long)r * Mp], z[r], x);
  yu[c] = x;
  const UnitView v = decode_unit(tb, a, u);
  const bool last = (a.mode == MODE_FINE) && (a.r == v.Sb);
  epi_store(a, ep, u, v.slot, last, r0 + c, x);
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
    const int tt = (below + TB - 1) / TB;
    k_blk_trail<<<dim3(tt * (tt + 1) / 2, units), 256, 0, s>>>(tb, a, a.A, r0, w);
    if ((r = hipGetLastError()) != hipSuccess) return r;
  }
  for (int j = nblk - 1; j >= 0; --j) {
    if (j < nblk - 1) {
      k_blk_bs_part<<<dim3(nblk - 1 - j, units), 256, 0, s>>>(tb, a, a.A, a.rhs, q, j, nb, nblk);
      hipError_t r = hipGetLastError();
      if (r != hipSuccess) return r;
    }
    k_blk_bs_diag<<<units, 256, 0, s>>>(tb, a, e, a.A, a.rhs, q, j, nb, nblk);
    hipError_t r = hipGetLastError();
    if (r != hipSuccess) return r;
  }
  return hipSuccess;
}

}  // namespace l1pr
