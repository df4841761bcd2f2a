// Factorisation and solve of one step's system per unit, in a single 512-thread
// work-group with the matrix held in registers (1D sine basis, M padded to Mp <= 256).
//
// The lower triangle of A = I + tau K is split into 16x16 tiles (at most 136); wave w keeps
// the tile-rows w and nt-1-w in its registers as FP64 MFMA accumulators (at most 17 tiles,
// 136 registers, per wave).  Two ways to fill the tiles:
//   SRC_MOMENTS  from the cosine moments m_j = sum_q w_q D_q cos(j pi x_q): in the sine basis
//                phi_k' phi_l' = k l pi^2 [cos((k-l) pi x) + cos((k+l) pi x)], so the
//                quadrature stiffness is K_kl = k l pi^2 (m_|k-l| + m_{k+l}) term by term
//                (Toeplitz-plus-Hankel form; 2M+1 moments instead of M^2 dot products);
//   SRC_LOAD     from the stiffness tiles that k_assemble1d (quadrature GEMM) wrote.
// The right-hand side is hist + tau F (history sums and load vector from the batched
// kernels).  Then a right-looking Cholesky by 16-column blocks without leaving the chip:
//   - wave 0 factors the diagonal tile (one row per lane, values broadcast with readlane,
//     pivots from a reciprocal square root refined by two Newton steps), forms
//     W = L_jj^-T by column substitution and y_j = W^T b_j;
//   - panel tiles become L_Ij = A_Ij W (MFMA), staged in LDS;
//   - the owners of trailing tiles subtract L_Ij L_Kj^T (MFMA), and b_I -= L_Ij y_j.
// Back substitution L^T x = y uses the L tiles still in registers and W_j kept in the
// diagonal tiles.  All reductions have a fixed order, so a unit's result does not depend on
// the launch it is part of.
#include "l1pr_internal.h"

namespace l1pr {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int RW = 8;           // waves per work-group
constexpr int RT = RW * 64;     // threads per work-group
constexpr int RNS = 17;         // tile slots per wave: 136 / 8
constexpr int RMAXMP = 256;

enum { SRC_MOMENTS = 0, SRC_LOAD = 1 };

__device__ inline double bcast(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Tile ownership: wave w owns the whole tile-rows w and nt-1-w of the lower triangle
// (w + 1 + nt - w = nt + 1 <= 17 tiles), so slot s maps to (I, K) with scalar arithmetic.
__device__ inline void slot_tile(int s, int wave, int nt, int& I, int& K) {
  const int ra = wave, rb = nt - 1 - wave;
  I = -1;
  K = -1;
  if (ra > rb) return;
  if (s <= ra) {
    I = ra;
    K = s;
  } else if (ra < rb && s <= ra + 1 + rb) {
    I = rb;
    K = s - ra - 1;
  }
}

// Slot coordinates for use inside the block loop.  The empty asm marks them as redefined on
// every use, so the compiler does not hoist per-slot addresses out of the loop and keep
// them live next to the 136 accumulator registers.
__device__ inline void slot_tile_here(int s, int wave, int nt, int& I, int& K) {
  slot_tile(s, wave, nt, I, K);
  I = __builtin_amdgcn_readfirstlane(I);
  K = __builtin_amdgcn_readfirstlane(K);
  asm volatile("" : "+s"(I), "+s"(K));
}

// owner wave and slot of the diagonal tile (j, j)
__device__ inline void diag_owner(int j, int nt, int& w, int& s) {
  w = j < nt - 1 - j ? j : nt - 1 - j;
  s = (w == j) ? j : w + 1 + j;
}

#define SLOT_FENCE() __builtin_amdgcn_sched_barrier(0)

struct RegLds {
  int sb, sD, sW, sI, ct, big;  // offsets in doubles; `big` holds the moments, then the panel
  int total;
};

__host__ __device__ inline RegLds reg_lds(int Mp) {
  RegLds L;
  L.sb = 0;
  L.sD = Mp;
  L.sW = L.sD + 16 * 17;
  L.sI = L.sW + 16 * 17;
  L.ct = L.sI + 16;
  L.big = L.ct + 16 * 16;
  const int Jm = 2 * Mp + 1;
  L.total = L.big + (Jm > Mp * 17 ? Jm : Mp * 17);
  return L;
}

// 1/sqrt(x) to full double precision: hardware estimate plus two Newton steps
__device__ inline double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  y = y * fma(-hx * y, y, 1.5);
  y = y * fma(-hx * y, y, 1.5);
  return y;
}

template <int SRC>
__global__ __launch_bounds__(RT) void k_chol_reg(Tables tb, StepArgs a, Epilogue ep,
                                                 const double* mom, const double* F,
                                                 const double* hist) {
  extern __shared__ double lds[];
  const int u = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
  // wave index as a scalar: tile ownership and every per-slot branch stay on the scalar unit
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int Mp = tb.Mp, M = tb.M, nt = Mp / 16;
  const RegLds LO = reg_lds(Mp);
  double* sb = lds + LO.sb;
  double* sD = lds + LO.sD;
  double* sW = lds + LO.sW;
  double* sI = lds + LO.sI;
  double* ct = lds + LO.ct;
  double* sP = lds + LO.big;
  d4 acc[RNS];
  const int lr = lane >> 4, lc = lane & 15;

  const int b = (a.mode == MODE_FINE) ? u / a.nP : u;
  const double tau = tb.inst[(long)b * NSCAL + ((a.mode == MODE_COARSE) ? IS_TAUC : IS_TAU)];
  for (int k = tid; k < Mp; k += RT)
    sb[k] = hist[(long)u * Mp + k] + tau * F[(long)u * Mp + k];

  if (SRC == SRC_MOMENTS) {
    const int Jm = 2 * Mp + 1;
    double* sm = sP;
    for (int j = tid; j < Jm; j += RT) sm[j] = mom[(long)u * Jm + j];
    __syncthreads();
    const double pi2 = kPi * kPi;
#pragma unroll
    for (int s = 0; s < RNS; ++s) {
      int tI, tK;
      slot_tile(s, wave, nt, tI, tK);
      if (tI < 0) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int k = tI * 16 + lr + 4 * e, l = tK * 16 + lc;
        double val = (k == l) ? 1.0 : 0.0;
        if (k < M && l < M) {
          const int dkl = k > l ? k - l : l - k;
          const double Kkl = ((double)(k + 1) * (double)(l + 1)) * pi2 * (sm[dkl] + sm[k + l + 2]);
          val += tau * Kkl;
        }
        acc[s][e] = val;
      }
    }
    __syncthreads();  // the moments share LDS with the panel
  } else {
    const double* A = a.A + (long)u * Mp * Mp;
#pragma unroll
    for (int s = 0; s < RNS; ++s) {
      int tI, tK;
      slot_tile(s, wave, nt, tI, tK);
      if (tI < 0) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e)
        acc[s][e] = A[(long)(tI * 16 + lr + 4 * e) * Mp + tK * 16 + lc];
    }
    __syncthreads();
  }

  // ------------------------------------------------------------ factorisation
  for (int j = 0; j < nt; ++j) {
    const int j0 = 16 * j;
    int wd, sdg;
    diag_owner(j, nt, wd, sdg);
    // stage the diagonal tile and the panel tiles (I, j), I > j
    if (wave == wd) {
#pragma unroll
      for (int s = 0; s < RNS; ++s)
        if (s == sdg)
#pragma unroll
          for (int e = 0; e < 4; ++e) sD[(lr + 4 * e) * 17 + lc] = acc[s][e];
    }
#pragma unroll
    for (int s = 0; s < RNS; ++s) {
      int tI, tK;
      slot_tile_here(s, wave, nt, tI, tK);
      if (tK == j && tI > j)
#pragma unroll
        for (int e = 0; e < 4; ++e) sP[(tI * 16 + lr + 4 * e) * 17 + lc] = acc[s][e];
    }
    __syncthreads();
    if (wave == 0) {
      // Lane r holds row r of the diagonal block; columns are factored left to right.
      // Branch-free: every lane scales its entry of column c (the entries above the diagonal
      // are zero, so the same product is right for every row), every lane publishes it
      // through LDS (lanes r and r + 16k hold identical rows and write identical values), and
      // every lane applies the rank-one update; entries above the diagonal collect values
      // that are never read and are masked when the factor is written out.
      const int r = lane & 15;
      double* col = ct;  // exchange space (the back substitution reuses it)
      double v[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) v[c] = (c <= r) ? sD[r * 17 + c] : 0.0;
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        col[r] = v[c];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const double inv = rsqrt_nr(col[c]);
        v[c] = v[c] * inv;
        sI[c] = inv;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        col[r] = v[c];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        double lsc[16];
#pragma unroll
        for (int s2 = c + 1; s2 < 16; ++s2) lsc[s2] = col[s2];
#pragma unroll
        for (int s2 = c + 1; s2 < 16; ++s2) v[s2] = fma(-v[c], lsc[s2], v[s2]);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
#pragma unroll
      for (int c = 0; c < 16; ++c) sD[r * 17 + c] = (c <= r) ? v[c] : 0.0;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // Column c of X = L^-1 (lane c), right-looking: once x_p is known it is removed from
      // every later row, so the dependency chain is 16 steps deep.  W = X^T = L^-T.
      {
        const int c = lane & 15;
        double sx[16];
#pragma unroll
        for (int rr = 0; rr < 16; ++rr) sx[rr] = (rr == c) ? 1.0 : 0.0;
#pragma unroll
        for (int p2 = 0; p2 < 16; ++p2) {
          sx[p2] = sx[p2] * sI[p2];
#pragma unroll
          for (int rr = p2 + 1; rr < 16; ++rr) sx[rr] -= sD[rr * 17 + p2] * sx[p2];
        }
#pragma unroll
        for (int rr = 0; rr < 16; ++rr) sW[c * 17 + rr] = sx[rr];
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // y_j = L_jj^-1 b_j = W^T b_j
      double y = 0.0;
#pragma unroll
      for (int c = 0; c < 16; ++c) y += sW[c * 17 + r] * sb[j0 + c];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      sb[j0 + r] = y;
    }
    __syncthreads();
    if (wave == wd) {
      // keep W_j in the diagonal tile for the back substitution
#pragma unroll
      for (int s = 0; s < RNS; ++s)
        if (s == sdg)
#pragma unroll
          for (int e = 0; e < 4; ++e) acc[s][e] = sW[(lr + 4 * e) * 17 + lc];
    }
    // L_Ij = A_Ij W; each wave reads and rewrites only the rows of its own panel tiles
#pragma unroll
    for (int s = 0; s < RNS; ++s) {
      int tI, tK;
      slot_tile_here(s, wave, nt, tI, tK);
      if (tK == j && tI > j) {
        d4 l = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const double aop = sP[(tI * 16 + lc) * 17 + 4 * kk + lr];
          const double bop = sW[(4 * kk + lr) * 17 + lc];
          l = __builtin_amdgcn_mfma_f64_16x16x4f64(aop, bop, l, 0, 0, 0);
        }
        acc[s] = l;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int e = 0; e < 4; ++e) sP[(tI * 16 + lr + 4 * e) * 17 + lc] = l[e];
      }
      SLOT_FENCE();
    }
    __syncthreads();
    // right-hand side below the block, and the trailing tiles
    for (int i = j0 + 16 + tid; i < Mp; i += RT) {
      double bi = sb[i];
#pragma unroll
      for (int c = 0; c < 16; ++c) bi -= sP[i * 17 + c] * sb[j0 + c];
      sb[i] = bi;
    }
#pragma unroll
    for (int s = 0; s < RNS; ++s) {
      int tI, tK;
      slot_tile_here(s, wave, nt, tI, tK);
      if (tK > j) {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const double aop = -sP[(tI * 16 + lc) * 17 + 4 * kk + lr];
          const double bop = sP[(tK * 16 + lc) * 17 + 4 * kk + lr];
          acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(aop, bop, acc[s], 0, 0, 0);
        }
      }
      SLOT_FENCE();
    }
    __syncthreads();
  }

  // ------------------------------------------------------- back substitution
  // L^T x = y, last block first.  Tile-row j (W_j on the diagonal and L_jK, K < j) belongs to
  // one wave, which forms x_j = W_j y_j in registers and removes L_jK^T x_j from every y_K.
  for (int j = nt - 1; j >= 0; --j) {
    const int j0 = 16 * j;
    int wd, sdg;
    diag_owner(j, nt, wd, sdg);
    if (wave == wd) {
      const double sv = sb[j0 + lc];
      // x_j = W_j y_j: lane holds W[lr + 4e][lc]; sum over the 16 columns
      double xr[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < RNS; ++s) {
        if (s == sdg) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            double p = acc[s][e] * sv;
            p += __shfl_xor(p, 1);
            p += __shfl_xor(p, 2);
            p += __shfl_xor(p, 4);
            p += __shfl_xor(p, 8);
            xr[e] = p;
          }
        }
      }
      // y_K -= L_jK^T x_j: lane holds L_jK[lr + 4e][lc] and x_j[lr + 4e]
#pragma unroll
      for (int s = 0; s < RNS; ++s) {
        int tI, tK;
        slot_tile_here(s, wave, nt, tI, tK);
        if (tI == j && tK < j) {
          double p = 0.0;
#pragma unroll
          for (int e = 0; e < 4; ++e) p += acc[s][e] * xr[e];
          p += __shfl_xor(p, 16);
          p += __shfl_xor(p, 32);
          if (lane < 16) sb[tK * 16 + lc] -= p;
        }
        SLOT_FENCE();
      }
      if (lc == 0)
#pragma unroll
        for (int e = 0; e < 4; ++e) sb[j0 + lr + 4 * e] = xr[e];
    }
    __syncthreads();
  }

  // --------------------------------------------------------------- epilogue
  long slot = u;
  if (a.mode == MODE_FINE) {
    const int b = u / a.nP, n = a.n_lo + u % a.nP;
    slot = (long)b * a.trajP + (n - a.trajN0);
  }
  for (int k = tid; k < Mp; k += RT) {
    const double x = sb[k];
    if (ep.kind == EPI_CORRECT) {
      const double go = ep.gold[(long)u * ep.gold_stride + k];
      ep.out[(long)u * ep.out_stride + k] = ep.fold[(long)u * ep.fold_stride + k] + (x - go);
      ep.gold[(long)u * ep.gold_stride + k] = x;
    } else {
      ep.out[slot * ep.out_stride + k] = x;
      if (ep.kind == EPI_STORE2) ep.gold[(long)u * ep.gold_stride + k] = x;
    }
  }
}

bool reg_path_ok(int Mp, int Qp) {
  (void)Qp;
  return Mp <= RMAXMP && reg_lds(Mp).total * sizeof(double) <= 64 * 1024;
}

hipError_t launch_chol_reg(const Tables& tb, const StepArgs& a, const Epilogue& e, int units,
                           const double* mom, const double* F, const double* hist,
                           hipStream_t s) {
  const size_t lds = sizeof(double) * reg_lds(tb.Mp).total;
  if (mom) k_chol_reg<SRC_MOMENTS><<<units, RT, lds, s>>>(tb, a, e, mom, F, hist);
  else k_chol_reg<SRC_LOAD><<<units, RT, lds, s>>>(tb, a, e, mom, F, hist);
  return hipGetLastError();
}

}  // namespace l1pr
