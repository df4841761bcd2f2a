// Factorisation and solve of one step's system per unit, in a single 512-thread
// work-group with the matrix held in registers (1D sine basis, M padded to Mp <= 256).
//
// The lower triangle of A = I + tau K is split into 16x16 tiles (at most 136); wave w keeps
// the tile-rows w and nt-1-w in its registers as FP64 MFMA accumulators (at most 17 tiles,
// 136 registers, per wave).  A tile is stored transposed: slot (I, K) holds A_IK^T in the
// accumulator layout (lane l, element v <-> row l/16 + 4v, column l%16).  That layout is
// the B-operand layout of MFMA 16x16x4 (k-chunk v): the panel product takes its register
// tile straight as B operand, and a published panel tile serves as A or B operand lane for
// lane (linear, conflict-free LDS reads):
//   panel     L_Ij^T = W_j^T A_Ij^T                (W_j = L_jj^-T from LDS, A_Ij^T registers)
//   trailing  A_IK^T -= L_Kj L_Ij^T                 (both published panel tiles)
// Two ways to fill the tiles:
//   SRC_MOMENTS  from the cosine moments m_j = sum_q w_q D_q cos(j pi x_q): in the sine basis
//                phi_k' phi_l' = k l pi^2 [cos((k-l) pi x) + cos((k+l) pi x)], so the
//                quadrature stiffness is K_kl = k l pi^2 (m_|k-l| + m_{k+l}) term by term
//                (Toeplitz-plus-Hankel form; 2M+1 moments instead of M^2 dot products);
//   SRC_LOAD     from the stiffness tiles that k_assemble1d (quadrature GEMM) wrote.
// The right-hand side is hist + tau F (history sums and load vector from the batched
// kernels).  Right-looking Cholesky by 16-column blocks, with look-ahead: while the other
// waves apply block j to the right-hand side, the owner of diagonal tile j+1 updates that
// tile and turns it into W_{j+1} = L^-T directly (column elimination on [A ; I] in the
// accumulator layout); then every wave updates its trailing tiles.  Forward substitution
// runs alongside (y_j = W_j^T b_j, then b_I -= L_Ij y_j).  Before the back substitution
// L^T x = y every wave transposes its tiles back (L_IK, and L_jj^-1 on the diagonal); the back
// substitution then runs as a pipeline across waves (see there).  All reductions have a
// fixed order, so a unit's result does not depend on the launch it is part of.
#include "l1pr_internal.h"

namespace l1pr {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int RW = 8;           // waves per work-group
constexpr int RT = RW * 64;     // threads per work-group
constexpr int RNS = 17;         // tile slots per wave: 136 / 8
constexpr int RMAXMP = 256;

enum { SRC_MOMENTS = 0, SRC_LOAD = 1 };

// Value of lane P of the caller's 16-lane row (DPP row broadcast), for a double.
template <int P>
__device__ inline double rowbc(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x150 + P, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x150 + P, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// Tile ownership: wave w owns the whole tile-rows ra = w and rb = nt-1-w of the lower
// triangle (w + 1 + nt - w = nt + 1 <= 17 tiles).  Its diagonal tiles come first, in slots 0
// (ra, ra) and 1 (rb, rb), so the code that picks a wave's diagonal tile chooses between two
// slots; then row ra's tiles (ra, K) in slots nd + K and row rb's (rb, K) in slots nd + ra + K
// (nd = number of diagonal slots), all with scalar arithmetic.
__device__ inline void slot_tile(int s, int wave, int nt, int& I, int& K) {
  const int ra = wave, rb = nt - 1 - wave;
  I = -1;
  K = -1;
  if (ra > rb) return;
  const int nd = (ra < rb) ? 2 : 1;
  if (s == 0) {
    I = ra;
    K = ra;
  } else if (s < nd) {
    I = rb;
    K = rb;
  } else if (s < nd + ra) {
    I = ra;
    K = s - nd;
  } else if (ra < rb && s < nd + ra + rb) {
    I = rb;
    K = s - nd - ra;
  }
}

// owner wave and slot (0 or 1) of the diagonal tile (j, j)
__device__ inline void diag_owner(int j, int nt, int& w, int& s) {
  w = j < nt - 1 - j ? j : nt - 1 - j;
  s = (w == j) ? 0 : 1;
}

#define SLOT_FENCE() __builtin_amdgcn_sched_barrier(0)

struct RegLds {
  int sb;     // right-hand side, then y, then x            [Mp]
  int sWA;    // W_j in A-operand order: [v][lane]           [4][64]
  int prog;   // back-substitution turn counters per tile-row (16 ints)
  int big;    // the moments (fill), the published panel [nt][4][64], then per-wave
              // transposition scratch [8][16 x 17]
  int total;
};

__host__ __device__ inline RegLds reg_lds(int Mp) {
  RegLds L;
  L.sb = 0;
  L.sWA = Mp;
  L.prog = L.sWA + 256;
  L.big = L.prog + 8;
  const int Jm = 2 * Mp + 1;
  const int panel = (Mp / 16) * 256;
  const int scratch = RW * 16 * 17;
  int big = Jm > panel ? Jm : panel;
  big = big > scratch ? big : scratch;
  L.total = L.big + big;
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

// 1/x to full double precision: the hardware estimate (relative error about 2^-23) and one
// third-order step, y0 (1 + e + e^2) with e = 1 - x y0 (error about e^3): three dependent
// operations after the estimate.
__device__ inline double rcp_nr(double x) {
  const double y = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, y, 1.0);
  return fma(y, fma(e, e, e), y);
}

#define WAVE_FENCE()                                     \
  do {                                                   \
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront"); \
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront"); \
  } while (0)

// Cross-row exchanges with the gfx950 row swaps (VALU, no LDS): for one register,
// permlane16_swap gives the row pairs (r0, r0, r2, r2) and (r1, r1, r3, r3), and
// permlane32_swap gives (r0, r1, r0, r1) and (r2, r3, r2, r3), where r_g is the value a lane
// at the same position of 16-lane row g holds.
__device__ inline void swap16(double v, double& even, double& odd) {
  const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(v), __double2loint(v), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(v), __double2hiint(v), false, false);
  even = __hiloint2double(hi[0], lo[0]);
  odd = __hiloint2double(hi[1], lo[1]);
}
__device__ inline void swap32(double v, double& low, double& high) {
  const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(v), __double2loint(v), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(v), __double2hiint(v), false, false);
  low = __hiloint2double(hi[0], lo[0]);
  high = __hiloint2double(hi[1], lo[1]);
}

// Value of lane `src` (any lane) for every lane, for a double (LDS crossbar, no memory).
__device__ inline double lane_read(double v, int src) {
  const int lo = __builtin_amdgcn_ds_bpermute(src << 2, __double2loint(v));
  const int hi = __builtin_amdgcn_ds_bpermute(src << 2, __double2hiint(v));
  return __hiloint2double(hi, lo);
}

// (r0 + r1) + (r2 + r3) over the four 16-lane rows, in every lane.
__device__ inline double rowgroup_sum(double v) {
  double e, o, l, h;
  swap16(v, e, o);
  swap32(e + o, l, h);
  return l + h;
}

// Value of lane `src` as a wave-uniform double.
__device__ inline double lane_uniform(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

// W = L^-T for the Cholesky factor L of one symmetric positive definite 16x16 tile, inside
// one wave, both in the accumulator layout (lane l, element v <-> row l/16 + 4v, column
// l%16).  Column elimination on the stacked pair [A ; I]: step p subtracts
// (a_pc / a_pp) x column p from every column c > p, so A E_0 ... E_15 = Lt is lower
// triangular with column p equal to the trailing column at step p, and I E_0 ... E_15
// S = A^-1 L = L^-T with S = diag(1 / sqrt(a_pp)) (a_pp: the pivot at step p).  Each lane owns four entries of each half:
// the pivot comes from one lane (readlane), the pivot row from the lanes of its row group
// (bpermute, whose latency overlaps the reciprocal), the pivot column from lane p of the
// caller's 16-lane row (DPP broadcast).
// Work that is zero by structure is skipped: at step p the pivot column of the A half is only
// needed in rows >= p (rows above feed nothing that is read again), and the pivot column of
// the I half is zero below row p.  The A half goes first, alone: its steps are the pivot chain,
// and leaving the I half out of them halves the instructions each step issues.  The I half
// then replays the 16 column operations with the kept multipliers; the pivots (the column
// scales) are read off the eliminated A half at the end.
struct DiagFactor {
  double a[4], w[4], mm[16], sc;  // mm: multipliers of each step; sc: the pivot of this lane's column

  __device__ __attribute__((always_inline)) void init(const d4& t, int lane) {
    const int lr = lane >> 4, lc = lane & 15;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      a[v] = t[v];
      w[v] = (lr + 4 * v == lc) ? 1.0 : 0.0;
    }
    sc = 1.0;
  }

  // step P on the A half only (the pivot chain); the multipliers are kept for the I half
  template <int P>
  __device__ __attribute__((always_inline)) void step(int lane) {
    const int lc = lane & 15;
    const double piv = lane_uniform(a[P / 4], (P % 4) * 16 + P);
    const double rowp = lane_read(a[P / 4], (P % 4) * 16 + lc);
    const double m = (lc > P) ? rowp * rcp_nr(piv) : 0.0;
    mm[P] = m;
#pragma unroll
    for (int v = P / 4; v < 4; ++v) a[v] = fma(-rowbc<P>(a[v]), m, a[v]);
  }
  // step P on the I half: the same column operation with the kept multipliers (it reads only
  // the I half, so it can follow all of the A steps; each entry sees the same operations in
  // the same order)
  template <int P>
  __device__ __attribute__((always_inline)) void stepw() {
#pragma unroll
    for (int v = 0; v <= P / 4; ++v) w[v] = fma(-rowbc<P>(w[v]), mm[P], w[v]);
  }
  // the pivot of this lane's column c: entry (c, c), which no step after c changes
  __device__ __attribute__((always_inline)) void pivots(int lane) {
    const int lc = lane & 15;
    const int src = (lc & 3) * 16 + lc;
    const double p0 = lane_read(a[0], src), p1 = lane_read(a[1], src);
    const double p2 = lane_read(a[2], src), p3 = lane_read(a[3], src);
    const int q = lc >> 2;
    sc = q == 0 ? p0 : (q == 1 ? p1 : (q == 2 ? p2 : p3));
  }

  // W in the accumulator layout; also published in A-operand order,
  // sWA[v][lane] = W[4v + lane/16][lane%16]
  __device__ __attribute__((always_inline)) d4 finish(int lane, double* sWA) {
    sc = rsqrt_nr(sc);
    d4 out;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      out[v] = w[v] * sc;
      sWA[v * 64 + lane] = out[v];
    }
    WAVE_FENCE();
    return out;
  }
};

#define L1PR_DIAG_STEPS(DF, BETWEEN)                                                    \
  DF.step<0>(lane); BETWEEN(0) DF.step<1>(lane); BETWEEN(1) DF.step<2>(lane); BETWEEN(2)    \
  DF.step<3>(lane); BETWEEN(3) DF.step<4>(lane); BETWEEN(4) DF.step<5>(lane); BETWEEN(5)    \
  DF.step<6>(lane); BETWEEN(6) DF.step<7>(lane); BETWEEN(7) DF.step<8>(lane); BETWEEN(8)    \
  DF.step<9>(lane); BETWEEN(9) DF.step<10>(lane); BETWEEN(10) DF.step<11>(lane);           \
  BETWEEN(11) DF.step<12>(lane); BETWEEN(12) DF.step<13>(lane); BETWEEN(13)                \
  DF.step<14>(lane); BETWEEN(14) DF.step<15>(lane); BETWEEN(15)                            \
  DF.pivots(lane);                                                                         \
  DF.stepw<0>(); DF.stepw<1>(); DF.stepw<2>(); DF.stepw<3>(); DF.stepw<4>(); DF.stepw<5>();  \
  DF.stepw<6>(); DF.stepw<7>(); DF.stepw<8>(); DF.stepw<9>(); DF.stepw<10>(); DF.stepw<11>(); \
  DF.stepw<12>(); DF.stepw<13>(); DF.stepw<14>(); DF.stepw<15>();

// Right-looking Cholesky of the nt x nt tile lower triangle that the waves hold in `acc`
// (transposed tiles, slot ownership as in slot_tile), with the forward substitution of the
// right-hand side sb[0, Mp) alongside; ends with every slot back in the accumulator layout of
// the untransposed tile: L_IK off the diagonal, L_jj^-1 on it, and y = L^-1 b in sb.
__device__ __attribute__((always_inline)) inline void factor_tiles(d4 (&acc)[RNS], double* sb,
                                                                   double* sWA, double* sP,
                                                                   int nt, int Mp, int wave,
                                                                   int tid) {
  const int lane = tid & 63, lr = lane >> 4, lc = lane & 15;
  // ------------------------------------------------------------ factorisation
  {
    int wd, sdg;
    diag_owner(0, nt, wd, sdg);
    if (wave == wd) {  // wave 0 keeps (0, 0) in slot 0
      DiagFactor df;
      df.init(acc[0], lane);
#define L1PR_NOTHING(P)
      L1PR_DIAG_STEPS(df, L1PR_NOTHING)
#undef L1PR_NOTHING
      acc[0] = df.finish(lane, sWA);
    }
  }
  __syncthreads();
  for (int j = 0; j < nt; ++j) {
    const int j0 = 16 * j;
    // ---- panel: L_Ij^T = W_j^T A_Ij^T for the tiles (I, j), I > j, of this wave
#pragma unroll
    for (int s = 0; s < RNS; ++s) {
      int tI, tK;
      slot_tile(s, wave, nt, tI, tK);
      if (tK == j && tI > j) {
        d4 t = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int v = 0; v < 4; ++v)
          t = __builtin_amdgcn_mfma_f64_16x16x4f64(sWA[v * 64 + lane], acc[s][v], t, 0, 0, 0);
        acc[s] = t;
#pragma unroll
        for (int v = 0; v < 4; ++v) sP[(tI * 4 + v) * 64 + lane] = t[v];
      }
      SLOT_FENCE();
    }
    // ---- forward substitution for the block: y_j = W_j^T b_j
    {
      int wd, sdg;
      diag_owner(j, nt, wd, sdg);
      if (wave == wd) {
        double pr = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) pr += sWA[v * 64 + lane] * sb[j0 + 4 * v + lr];
        pr = rowgroup_sum(pr);
        WAVE_FENCE();
        if (lane < 16) sb[j0 + lc] = pr;
      }
    }
    __syncthreads();
    // ---- look-ahead: the owner of diagonal tile j+1 updates it and turns it into W_{j+1}
    // while the other waves apply block j to the right-hand side; then every wave updates
    // its trailing tiles, A_IK^T -= L_Kj L_Ij^T for K > j.
    const int j1 = j + 1;
    int wd1 = -1, sd1 = -1;
    if (j1 < nt) diag_owner(j1, nt, wd1, sd1);
    if (wave == wd1) {
      d4 t = (sd1 == 0) ? acc[0] : acc[1];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double px = sP[(j1 * 4 + v) * 64 + lane];
        t = __builtin_amdgcn_mfma_f64_16x16x4f64(-px, px, t, 0, 0, 0);
      }
      DiagFactor df;
      df.init(t, lane);
#define L1PR_NOTHING(P)
      L1PR_DIAG_STEPS(df, L1PR_NOTHING)
#undef L1PR_NOTHING
      t = df.finish(lane, sWA);
      if (sd1 == 0)
        acc[0] = t;
      else
        acc[1] = t;
    } else {
      // right-hand side below the block: b_i -= L_ij y_j
      const int nthr = (wd1 >= 0) ? RT - 64 : RT;
      const int tt = (wd1 >= 0 && wave > wd1) ? tid - 64 : tid;
      for (int i = j0 + 16 + tt; i < Mp; i += nthr) {
        const int I = i >> 4, r = i & 15;
        double bi = sb[i];
#pragma unroll
        for (int c = 0; c < 16; ++c) bi -= sP[(I * 4 + (c >> 2)) * 64 + (c & 3) * 16 + r] * sb[j0 + c];
        sb[i] = bi;
      }
    }
#define L1PR_TRAIL(S)                                                                          \
  {                                                                                            \
    int tI, tK;                                                                                \
    slot_tile((S), wave, nt, tI, tK);                                                     \
    if (tK > j && !(tI == j1 && tK == j1)) {                                                   \
      _Pragma("unroll") for (int v = 0; v < 4; ++v) acc[(S)] =                                 \
          __builtin_amdgcn_mfma_f64_16x16x4f64(-sP[(tK * 4 + v) * 64 + lane],                  \
                                               sP[(tI * 4 + v) * 64 + lane], acc[(S)], 0, 0, 0); \
    }                                                                                          \
    SLOT_FENCE();                                                                              \
  }
#pragma unroll
    for (int s = 0; s < RNS; ++s) L1PR_TRAIL(s)
    __syncthreads();
#undef L1PR_TRAIL
  }

  // ---- every slot back to the accumulator layout of the untransposed tile: L_IK off the
  // diagonal, X_j = W_j^T = L_jj^-1 on it; per-wave scratch in the panel space
  {
    double* scr = sP + wave * (16 * 17);
#pragma unroll
    for (int s = 0; s < RNS; ++s) {
      int tI, tK;
      slot_tile(s, wave, nt, tI, tK);
      if (tI >= 0) {
#pragma unroll
        for (int v = 0; v < 4; ++v) scr[(lr + 4 * v) * 17 + lc] = acc[s][v];
        WAVE_FENCE();
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[s][v] = scr[lc * 17 + lr + 4 * v];
        WAVE_FENCE();
      }
      SLOT_FENCE();
    }
  }
  __syncthreads();
}

template <int SRC>
__global__ __launch_bounds__(RT) void k_chol_reg(Tables tb, StepArgs a, Epilogue ep,
                                                 const double* mom, const double* F,
                                                 const double* hist) {
  extern __shared__ double lds[];
  const int u = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
  // wave index as a scalar: tile ownership and every per-slot branch stay on the scalar unit
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int Mp = tb.Mp, nt = Mp / 16;
  const RegLds LO = reg_lds(Mp);
  double* sb = lds + LO.sb;
  double* sWA = lds + LO.sWA;
  double* sP = lds + LO.big;
  d4 acc[RNS];
  const int lr = lane >> 4, lc = lane & 15;

  const int b = (a.mode == MODE_FINE) ? u / a.nP : u;
  const double* ins = tb.inst + (long)b * NSCAL;
  // every global read of the set-up is issued before any of them is needed
  const double ins_sb = ins[IS_SB], ins_mb = ins[IS_MB];
  const double tau = ins[(a.mode == MODE_COARSE) ? IS_TAUC : IS_TAU];
  const int fin = a.done ? a.done[b] : 0;
  const int Jm = 2 * Mp + 1;
  double hv = 0.0, fv = 0.0, m0 = 0.0, m1 = 0.0;
  if (tid < Mp) {
    hv = hist[(long)u * Mp + tid];
    fv = F[(long)u * Mp + tid];
  }
  if (SRC == SRC_MOMENTS) {
    if (tid < Jm) m0 = mom[(long)u * Jm + tid];
    if (tid + RT < Jm) m1 = mom[(long)u * Jm + tid + RT];
  }
  // past the instance's last fine step of the slice (uneven batches): nothing to do
  if (a.mode == MODE_FINE && a.r > (int)ins_sb) return;
  // a finished parareal instance keeps its slice ends: nothing to factor or store
  if (fin) return;
  // the instance's own modes: entries k >= Mb are identity rows with zero right-hand side
  const int Mb = (int)ins_mb;
  if (tid < Mp) sb[tid] = (tid < Mb) ? hv + tau * fv : 0.0;

  // slot (I, K) element v of lane l holds A[16 I + l%16][16 K + l/16 + 4v]
  if (SRC == SRC_MOMENTS) {
    double* sm = sP;
    if (tid < Jm) sm[tid] = m0;
    if (tid + RT < Jm) sm[tid + RT] = m1;
    __syncthreads();
    const double pi2 = kPi * kPi;
    const double tpi2 = tau * pi2;
#pragma unroll
    for (int s = 0; s < RNS; ++s) {
      int tI, tK;
      slot_tile(s, wave, nt, tI, tK);
      if (tI < 0) continue;
      if (tI > tK && 16 * tI + 16 <= Mb) {
        // strictly below the diagonal with every row inside the instance's modes: k > l, so
        // the entries e read m_{k-l} at k - l0 - 4e and m_{k+l+2} at k + l0 + 2 + 4e
        const int k = tI * 16 + lc, l0 = tK * 16 + lr;
        const double ck = tpi2 * (double)(k + 1);
        const double* pd = sm + (k - l0 - 12);
        const double* ps = sm + (k + l0 + 2);
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[s][e] = ck * (double)(l0 + 1 + 4 * e) * (pd[12 - 4 * e] + ps[4 * e]);
        continue;
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int k = tI * 16 + lc, l = tK * 16 + lr + 4 * e;
        double val = (k == l) ? 1.0 : 0.0;
        if (k < Mb && l < Mb) {
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
      for (int e = 0; e < 4; ++e) {
        const int k = tI * 16 + lc, l = tK * 16 + lr + 4 * e;
        acc[s][e] = (k < Mb && l < Mb) ? A[(long)k * Mp + l] : ((k == l) ? 1.0 : 0.0);
      }
    }
  }

  factor_tiles(acc, sb, sWA, sP, nt, Mp, wave, tid);
  int* tok = reinterpret_cast<int*>(lds + LO.prog);
  if (tid < 16) tok[tid] = 0;
  __syncthreads();

  // ------------------------------------------------------- back substitution
  // L^T x = y by tile-rows, last first: z_j = y_j - sum_{I > j} L_Ij^T x_I, x_j = X_j^T z_j.
  // z lives in sb in place of y.  The owner of tile-row j waits until every row I > j has
  // subtracted its part from z_j (tok[j] == nt-1-j), forms x_j (stored over z_j), then
  // subtracts L_jK^T x_j from z_K for K = j-1, j-2, ..., 0.  Each of those subtractions first
  // waits for its turn on block K (tok[K] == nt-1-j), so the parts reach z_K in a fixed order
  // (rows from the last down) whatever the timing.  A row only waits on higher rows, and each
  // wave takes its higher row first, so every wait ends.  The spins are bounded all the same:
  // a wait that gives up sets FLAG_WAIT in the call's status word (the unit's result is then
  // invalid and the call reports L1PR_EWAIT), and the kernel still runs to its end.
  {
    const int ra = wave, rb = nt - 1 - wave;
#define L1PR_WAIT_TOKEN(K, WANT)                                                              \
  if (lane == 0) {                                                                             \
    int it = 0;                                                                                \
    for (; it < tb.spin; ++it) {                                                               \
      if (__hip_atomic_load(&tok[(K)], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) >= (WANT)) \
        break;                                                                                 \
      __builtin_amdgcn_s_sleep(1);                                                             \
    }                                                                                          \
    if (it >= tb.spin && tb.flag) atomicOr(tb.flag, FLAG_WAIT);                                \
  }                                                                                            \
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
      const int j = pass == 0 ? rb : ra;
      if (ra > rb || (pass == 1 && ra == rb)) continue;  // wave-uniform
      const int j0 = 16 * j;
      int wd, sdg;
      diag_owner(j, nt, wd, sdg);
      L1PR_WAIT_TOKEN(j, nt - 1 - j)
      double z[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) z[v] = sb[j0 + lr + 4 * v];
      const d4 X = (sdg == 0) ? acc[0] : acc[1];
      double pr = 0.0;
#pragma unroll
      for (int v = 0; v < 4; ++v) pr += X[v] * z[v];
      pr = rowgroup_sum(pr);
      WAVE_FENCE();
      if (lane < 16) sb[j0 + lc] = pr;  // x_j over z_j
      WAVE_FENCE();
      double xv[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) xv[v] = sb[j0 + lr + 4 * v];
      // nearest block first.  Slots of row ra are s = nd + K, of row rb (when rb > ra)
      // s = nd + ra + K, so the slot range of row j is known without decoding every slot.
      const int nd = (ra < rb) ? 2 : 1;
      const int s_lo = (pass == 0 && ra < rb) ? nd + ra : nd;  // slot of (j, 0)
#pragma unroll
      for (int s = RNS - 1; s >= 0; --s) {
        if (s >= s_lo && s < s_lo + j) {
          const int tK = s - s_lo;
          double q = 0.0;
#pragma unroll
          for (int v = 0; v < 4; ++v) q += acc[s][v] * xv[v];
          q = rowgroup_sum(q);
          L1PR_WAIT_TOKEN(tK, nt - 1 - j)
          if (lane < 16) sb[tK * 16 + lc] -= q;
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
          if (lane == 0) __hip_atomic_store(&tok[tK], nt - j, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        SLOT_FENCE();
      }
    }
#undef L1PR_WAIT_TOKEN
  }
  __syncthreads();

  // --------------------------------------------------------------- epilogue
  const UnitView v = decode_unit(tb, a, u);
  const bool last = (a.mode == MODE_FINE) && (a.r == v.Sb);
  for (int k = tid; k < Mp; k += RT) epi_store(a, ep, u, v.slot, last, k, sb[k]);
}

// Diagonal block of the blocked factorisation through device memory: the w x w block at
// (r0, r0) of unit u's matrix A (row stride Mp; w <= 256, a multiple of 16), already updated
// by the panels to its left, is factored in registers as above, with the forward substitution
// of the right-hand side block rhs[r0, r0 + w) (y over b).  The block is then replaced by the
// full inverse X = L^-1 (lower triangle; within the diagonal 16 x 16 tiles the upper part is
// exact zeros, the tiles above them keep stale values and are never read).  X is formed by
// tile columns: X_cc = L_cc^-1 from the factorisation and, going down the column,
//   X_Ic = -X_II sum_{J=c}^{I-1} L_IJ X_Jc,
// wave w taking the columns w and nt-1-w (nt+1 tiles, the row ownership mirrored), one
// tile-row I at a time with row I of L staged in LDS after every wave has stored its tiles.
__device__ inline void col_slot(int s, int wave, int nt, int& I, int& c) {
  const int ca = wave, cb = nt - 1 - wave;
  I = -1;
  c = -1;
  if (ca > cb) return;
  if (s < nt - ca) {
    c = ca;
    I = ca + s;
  } else if (ca < cb && s < nt - ca + wave + 1) {
    c = cb;
    I = cb + (s - (nt - ca));
  }
}

__global__ __launch_bounds__(RT) void k_blk_diag(Tables tb, StepArgs a, double* A, double* rhs,
                                                 int r0, int w) {
  extern __shared__ double lds[];
  const int u = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int Mp = tb.Mp, nt = w / 16;
  const RegLds LO = reg_lds(w);
  double* sb = lds + LO.sb;
  double* sWA = lds + LO.sWA;
  double* sP = lds + LO.big;
  d4 acc[RNS];
  const int lr = lane >> 4, lc = lane & 15;
  const int b = (a.mode == MODE_FINE) ? u / a.nP : u;
  if (a.mode == MODE_FINE && a.r > (int)tb.inst[(long)b * NSCAL + IS_SB]) return;

  double* blk = A + (long)u * Mp * Mp + (long)r0 * Mp + r0;
  double* bu = rhs + (long)u * Mp + r0;
  for (int k = tid; k < w; k += RT) sb[k] = bu[k];
#pragma unroll
  for (int s = 0; s < RNS; ++s) {
    int tI, tK;
    slot_tile(s, wave, nt, tI, tK);
    if (tI < 0) continue;
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[s][e] = blk[(long)(tI * 16 + lc) * Mp + tK * 16 + lr + 4 * e];
  }

  factor_tiles(acc, sb, sWA, sP, nt, w, wave, tid);
  for (int k = tid; k < w; k += RT) bu[k] = sb[k];

  // L_IK and X_II = L_II^-1 back into the block (row-major 16-lane segments)
#pragma unroll
  for (int s = 0; s < RNS; ++s) {
    int tI, tK;
    slot_tile(s, wave, nt, tI, tK);
    if (tI < 0) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = lr + 4 * v;
      const double x = (tI == tK && r < lc) ? 0.0 : acc[s][v];
      blk[(long)(tI * 16 + r) * Mp + tK * 16 + lc] = x;
    }
  }
  __syncthreads();

  // tile columns of X, one tile-row of L at a time: at step I the work-group copies row I of
  // the stored block (L_IJ for J < I, X_II) into LDS in A-operand order
  // (sR[(J * 4 + v) * 64 + l] = T_J[l%16][4v + l/16]), then each wave extends its columns c < I
  // by X_Ic = -X_II sum_{J=c}^{I-1} L_IJ X_Jc; B operands are the wave's own X_Jc tiles.
  double* sR = sP;
#pragma unroll
  for (int s = 0; s < RNS; ++s) {
    int I, c;
    col_slot(s, wave, nt, I, c);
    if (I != c || I < 0) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[s][v] = blk[(long)(c * 16 + lr + 4 * v) * Mp + c * 16 + lc];
  }
  for (int I = 1; I < nt; ++I) {
    for (int e = tid; e < (I + 1) * 256; e += RT) {
      const int J = e >> 8, r = (e >> 4) & 15, cc = e & 15;
      sR[(J * 4 + (cc >> 2)) * 64 + r + 16 * (cc & 3)] = blk[(long)(I * 16 + r) * Mp + J * 16 + cc];
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < RNS; ++s) {
      int Is, c;
      col_slot(s, wave, nt, Is, c);
      if (Is != I || c >= I) continue;  // wave-uniform
      d4 t = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s2 = 0; s2 < s; ++s2) {
        int J, c2;
        col_slot(s2, wave, nt, J, c2);
        if (c2 != c) continue;  // J runs over c .. I-1: the earlier slots of the same column
#pragma unroll
        for (int v = 0; v < 4; ++v)
          t = __builtin_amdgcn_mfma_f64_16x16x4f64(sR[(J * 4 + v) * 64 + lane], acc[s2][v], t, 0, 0, 0);
      }
      d4 x = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int v = 0; v < 4; ++v)
        x = __builtin_amdgcn_mfma_f64_16x16x4f64(-sR[(I * 4 + v) * 64 + lane], t[v], x, 0, 0, 0);
      acc[s] = x;
    }
    __syncthreads();
  }
#pragma unroll
  for (int s = 0; s < RNS; ++s) {
    int I, c;
    col_slot(s, wave, nt, I, c);
    if (I < 0 || I == c) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) blk[(long)(I * 16 + lr + 4 * v) * Mp + c * 16 + lc] = acc[s][v];
  }
}

hipError_t launch_blk_diag(const Tables& tb, const StepArgs& a, int units, double* A, double* rhs,
                           int r0, int w, hipStream_t s) {
  if (w < 16 || w > RMAXMP || w % 16 != 0) return hipErrorInvalidValue;
  const size_t lds = sizeof(double) * reg_lds(w).total;
  k_blk_diag<<<units, RT, lds, s>>>(tb, a, A, rhs, r0, w);
  return hipGetLastError();
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
