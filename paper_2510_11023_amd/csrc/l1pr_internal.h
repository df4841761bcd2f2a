// Internal definitions shared by the HIP sources of libl1pr (not part of the C-ABI).
//
// Data layout in device memory (all float64 unless stated):
//   - coefficient vectors are padded from M to Mp = roundup(M, 16) entries (the padded
//     basis functions are identically zero, so padded entries stay exactly 0);
//   - quadrature is padded from Q to Qp = roundup(Q, 16) nodes with zero weight;
//   - phi [Qp][Mp]  = sqrt2 sin(k pi x_q),  phiT [Mp][Qp] its transpose,
//     dphi[Qp][Mp]  = sqrt2 k pi cos(k pi x_q);
//   - per-instance tables: scalars inst[b][NSCAL], L1 weights bw[b][LB] = b_j,
//     hybrid weights bhyb[b][m*S + r-1] = b_{m + r/S};
//   - slice ends Z[b][P+1][Mp]; fine trajectories traj[slot][S+1][Mp];
//   - per-unit step buffers d[u][Qp] (w_q D), rhs[u][Mp], A[u][Mp][Mp] (row-major, the
//     lower triangle is what the factorisation reads).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "l1pr.h"

namespace l1pr {

constexpr double kPi = 3.14159265358979323846;

// per-instance scalar slots; IS_MB and IS_SB hold the instance's own number of modes and of
// fine steps per slice (integers stored exactly as doubles; equal to M and S unless the batch
// is uneven)
enum { IS_ALPHA = 0, IS_TAU, IS_TAUC, IS_SFAC, IS_G1A, IS_G3A, IS_MB, IS_SB, NSCAL = 8 };

// tuning bits (l1pr_problem.tune): GEMM variant of the lagged-state product and of the
// projections in fine and full-history steps
enum { TUNE_LAG_SKINNY = 1, TUNE_PROJ_SKINNY = 2, TUNE_NB128 = 4, TUNE_TRAIL64 = 8 };

// kinds of step
enum { MODE_FINE = 0, MODE_COARSE = 1, MODE_FULL = 2 };

// epilogue kinds of the solve kernel
// EPI_NONE: the solve leaves its result in the right-hand-side buffer and stores nothing else
// (the first solve of an iteratively refined step)
enum { EPI_STORE = 0, EPI_STORE2 = 1, EPI_CORRECT = 2, EPI_NONE = 3 };

// bits of the call's device status word (the first bytes of every workspace)
enum { FLAG_NONFINITE = 1, FLAG_WAIT = 2 };

struct Tables {
  // M, Mp: coefficients per instance (M^2 in 2D) and their padded count; M1, M1p: modes per
  // direction (the basis tables' width); Q, Qp: Gauss points per direction
  int dim, M, Q, Mp, Qp, M1, M1p, N, P, S, B, LB;  // S, N: the largest steps per slice and steps
  int d_sel, f_sel, source_time, tune;
  int nb;  // column block of the device-memory factorisation (Mp > 256)
  double d_param, T;
  const double* xq;
  const double* wq;
  const double* phi;
  const double* phiT;
  const double* dphi;
  const double* inst;
  const double* bw;
  const double* bhyb;
  const double* cosq;  // [Qp][2 Mp + 1] = cos(j pi x_q) (zero for padding nodes)
  const double* b12;   // 2D: [M1p][2 Qp] = [phi^T | dphi^T]
  const double* s2;    // 2D: [2 Qp][M1p] = [dphi; phi]
  int* flag;           // the call's device status word (FLAG_* bits, set with atomicOr)
  // history = 2 (sum-of-exponentials far history): per instance and node, (w, e^-lam,
  // e^-lam j0) [B][soeL][3]; nullptr otherwise
  const double* soe;
  int soeL;
  int spin;            // polls of a bounded device wait before it gives up (sets FLAG_WAIT)
};

// What one step-launch computes for each of its units.
struct StepArgs {
  int mode;
  int r;        // MODE_FINE: fine step 1..S
  int n;        // MODE_COARSE: slice
  int nP, n_lo; // MODE_FINE: unit u -> instance u / nP, slice n_lo + u % nP
  int m;        // MODE_FULL: the step computes c_{m+1}
  double* traj; // MODE_FINE: slots [B*trajP][S+1][Mp]; MODE_FULL: [B][N+1][Mp]
  int trajP, trajN0;
  const double* Z;  // slice-end sequence [B][P+1][Mp]
  double* d;        // [units][Qp]   w_q D_q   (2D: [units][Qp][Qp])
  double* rhs;      // [units][Mp]   right-hand side (history sums on the batched path)
  double* A;        // [units][Mp][Mp]
  double* g;        // [units][Qp]   w_q f_q
  double* mom;      // [units][2 Mp + 1] cosine moments (2D: [units][Jp][Jp], Jp = 2 M1p + 1)
  double* F;        // [units][Mp]   load vector
  double* C2;       // 2D: [units][Mp] lagged states
  double* T2;       // 2D: [units][Qp Jp] intermediate products
  // full-history fine steps (MODE_FINE with prev set): the previous iterate's fine
  // trajectories, slots [B*P][S+1][Mp] as traj, and the prefix sums over earlier slices,
  // hp[B*P][S][Mp] (row r-1 of slot b*P + n for step r); both nullptr otherwise.
  // Full-history serial steps (MODE_FULL) with hp set: hp[B][hw][Mp] holds, for the block of
  // hw steps containing m, the sums over j < (m / hw) hw (row m mod hw).
  const double* prev;
  const double* hp;
  int hw;
  // parareal: instances that have met their stop test (nonzero) keep their slice ends; their
  // units skip the factorisation and store nothing (nullptr: no instance is finished)
  const int32_t* done;
  // history = 2: the exponential sums V [B][soeL][Mp] carried from step to step
  double* soeV;
};

// near window of the sum-of-exponentials history: distances below it use the exact weights
constexpr int kSoeJ0 = 16;

// instance of unit u in a step launch
__host__ __device__ inline int unit_instance(const StepArgs& a, int u) {
  return a.mode == MODE_FINE ? u / a.nP : u;
}

__device__ inline bool unit_done(const StepArgs& a, int u) {
  return a.done != nullptr && a.done[unit_instance(a, u)] != 0;
}

struct Epilogue {
  int kind;
  double* out;
  long out_stride;   // doubles between consecutive units
  double* gold;
  long gold_stride;
  const double* fold;
  long fold_stride;
};

__host__ __device__ inline int roundup(int x, int m) { return (x + m - 1) / m * m; }

// L1 weight b_x = (x+1)^(1-a) - x^(1-a), b_0 = 1; written as x^(1-a) (exp((1-a) log(1+1/x)) - 1)
// so that large x loses no digits to cancellation.
__device__ inline double l1_weight(double x, double a) {
  if (x == 0.0) return 1.0;
  const double e = 1.0 - a;
  return pow(x, e) * expm1(e * log1p(1.0 / x));
}

// Diffusion coefficient by selector.
__device__ inline double coef_D(int sel, double dparam, double u) {
  switch (sel) {
    case L1PR_D_CONST: return dparam;
    case L1PR_D_SIN2: { const double s = sin(u); return 1.0 + 0.5 * s * s; }
    case L1PR_D_RATIONAL: return 1.0 + 1.0 / (1.0 + u * u);
    case L1PR_D_GAUSS: return 1.0 + 0.5 * exp(-u * u);
    case L1PR_D_LINEAR: return 1.0 + u;
  }
  return 0.0;
}

// Source by selector at (x, y, t) with state u (y unused in 1D).
__device__ inline double coef_f(const Tables& tb, const double* inst, double x, double y,
                                double t, double u) {
  const double a = inst[IS_ALPHA];
  switch (tb.f_sel) {
    case L1PR_F_ZERO: return 0.0;
    case L1PR_F_MMS_SIN2: {
      // U = (1 + t^a) s,  f = Gamma(1+a) s - D(U) lap U - D'(U) |grad U|^2, D = 1 + sin^2/2
      const double At = 1.0 + pow(t, a);
      const double sx = sin(kPi * x), cx = cos(kPi * x);
      double s, grad2;
      if (tb.dim == 1) {
        s = sx;
        grad2 = At * At * kPi * kPi * cx * cx;
      } else {
        const double sy = sin(kPi * y), cy = cos(kPi * y);
        s = sx * sy;
        grad2 = At * At * kPi * kPi * (cx * cx * sy * sy + sx * sx * cy * cy);
      }
      const double U = At * s;
      const double sU = sin(U);
      const double DU = 1.0 + 0.5 * sU * sU;
      return inst[IS_G1A] * s + DU * (tb.dim * kPi * kPi * U) - 0.5 * sin(2.0 * U) * grad2;
    }
    case L1PR_F_LOGISTIC: return 0.1 * u * (1.0 - u);
    case L1PR_F_SIN: return sin(u);
    case L1PR_F_PAPER: {
      double s = sin(kPi * x);
      if (tb.dim == 2) s *= sin(kPi * y);
      return s * exp(-t);
    }
    case L1PR_F_MMS_SMOOTH: {
      double s = sin(kPi * x);
      if (tb.dim == 2) s *= sin(kPi * y);
      return (2.0 * pow(t, 2.0 - a) / inst[IS_G3A] + tb.dim * tb.d_param * kPi * kPi * (1.0 + t * t)) * s;
    }
  }
  return 0.0;
}

// fine time level t_m = T m / N (N: the instance's number of fine steps)
__device__ inline double t_level(const Tables& tb, long m, double N) { return (tb.T * (double)m) / N; }

// Where a unit's data lives and which time level / step size it uses.
struct UnitView {
  int b, n;
  const double* y;   // sequence whose last entry is the lagged state
  int L;             // index of that last entry
  const double* z;   // coarse sequence for the hybrid history (MODE_FINE) or nullptr
  int nz;
  long m_prev;       // fine index of the lagged time level
  long m_src;        // fine index of the new time level (source_time = 1)
  int tau_slot;      // IS_TAU or IS_TAUC
  long slot;         // trajectory slot (MODE_FINE)
  int Sb;            // the instance's fine steps per slice
  double Nb;         // the instance's fine steps, P Sb
};

__device__ inline UnitView decode_unit(const Tables& tb, const StepArgs& a, int u) {
  UnitView v;
  const long vecP = (long)(tb.P + 1) * tb.Mp;
  if (a.mode == MODE_FINE) {
    v.b = u / a.nP;
    v.Sb = (int)tb.inst[(long)v.b * NSCAL + IS_SB];
    v.Nb = (double)tb.P * (double)v.Sb;
    v.n = a.n_lo + u % a.nP;
    v.slot = (long)v.b * a.trajP + (v.n - a.trajN0);
    v.y = a.traj + v.slot * (long)(tb.S + 1) * tb.Mp;
    v.L = a.r - 1;
    v.z = a.Z + v.b * vecP;
    v.nz = v.n;
    v.m_prev = (long)v.n * v.Sb + a.r - 1;
    v.m_src = v.m_prev + 1;
    v.tau_slot = IS_TAU;
  } else {
    // coarse steps (one unit per instance, on the slice-end sequence) and full-history
    // steps (one unit per instance, on the whole fine trajectory) differ only in these
    // selects; one branch keeps the mode test from splitting into a switch
    const bool coarse = a.mode == MODE_COARSE;
    v.b = u;
    v.Sb = coarse ? (int)tb.inst[(long)v.b * NSCAL + IS_SB] : tb.S;
    v.Nb = coarse ? (double)tb.P * (double)v.Sb : (double)tb.N;
    v.n = coarse ? a.n : 0;
    v.slot = u;
    v.y = coarse ? a.Z + v.b * vecP : a.traj + (long)v.b * (tb.N + 1) * tb.Mp;
    v.L = coarse ? a.n : a.m;
    v.z = nullptr;
    v.nz = 0;
    v.m_prev = coarse ? (long)a.n * v.Sb : (long)a.m;
    v.m_src = coarse ? (long)(a.n + 1) * v.Sb : (long)a.m + 1;
    v.tau_slot = coarse ? IS_TAUC : IS_TAU;
  }
  return v;
}

// Full-history fine step r of slice n (Section 2.2 with the history taken over the whole
// fine grid): y_m - sum_{j=1}^{m} b_{m+1-j} (x_j - x_{j-1}), m = nS + r - 1, where x_j for
// j < nS are the previous iterate's fine states (row t = j - qS of slot q = (j-1)/S, x_0 =
// slot 0 row 0) and x_j for j >= nS the slice's own states, row j - nS.  The terms j < nS
// come first in the ascending sum and are known before the sweep, so their partial sum is
// read from hp; the loop continues it with the same fma sequence as the full-history serial
// step, which makes the result bit-for-bit that step's when the states agree.
__device__ inline double full_fine_history(const Tables& tb, const StepArgs& a,
                                           const UnitView& v, int k) {
  const int S = tb.S, Mp = tb.Mp;
  const long nS = (long)v.n * S, m = nS + a.r - 1;
  const double* bw = tb.bw + (long)v.b * tb.LB;
  const double* y = v.y + k;
  double acc, xp;
  int i = 0;
  if (v.n == 0) {
    acc = 0.0;
    xp = y[0];
    i = 1;
  } else {
    acc = a.hp[(v.slot * S + (a.r - 1)) * (long)Mp + k];
    const long j = nS - 1, q = j > 0 ? (j - 1) / S : 0, t = j - q * S;
    xp = a.prev[((v.slot - v.n + q) * (S + 1) + t) * (long)Mp + k];
  }
  for (; i < a.r; ++i) {
    const double x = y[(long)i * Mp];
    acc = fma(bw[m + 1 - (nS + i)], x - xp, acc);
    xp = x;
  }
  return y[(long)(a.r - 1) * Mp] - acc;
}

// Full-history serial step m (MODE_FULL): y_m - sum_{j=1}^{m} b_{m+1-j} (y_j - y_{j-1}) over
// the instance's trajectory.  With hp set, the terms j < nW (W = hw, n = m / W) were summed
// before the block's first step and the loop continues the chain from j = nW; either way the
// fma sequence is the ascending one.
__device__ inline double full_serial_history(const Tables& tb, const StepArgs& a,
                                             const UnitView& v, int k) {
  const int Mp = tb.Mp;
  const long m = a.m;
  const double* bw = tb.bw + (long)v.b * tb.LB;
  const double* y = v.y + k;
  double acc = 0.0, xp = y[0];
  long j = 1;
  if (a.hp) {
    const long nW = m / a.hw * a.hw;
    if (nW > 0) {
      acc = a.hp[((long)v.b * a.hw + (m - nW)) * Mp + k];
      xp = y[(nW - 1) * Mp];
      j = nW;
    }
  }
  for (; j + 3 <= m; j += 4) {
    const double x1 = y[j * Mp], x2 = y[(j + 1) * Mp], x3 = y[(j + 2) * Mp], x4 = y[(j + 3) * Mp];
    acc = fma(bw[m + 1 - j], x1 - xp, acc);
    acc = fma(bw[m - j], x2 - x1, acc);
    acc = fma(bw[m - 1 - j], x3 - x2, acc);
    acc = fma(bw[m - 2 - j], x4 - x3, acc);
    xp = x4;
  }
  for (; j <= m; ++j) {
    const double x = y[j * Mp];
    acc = fma(bw[m + 1 - j], x - xp, acc);
    xp = x;
  }
  return y[m * Mp] - acc;
}

// Where the new value x of entry k of unit u goes.  Fine steps: the trajectory row `out` at
// every step of the unit and, at the instance's last step of the slice (r == Sb), the slice
// end `gold` as well when it is set (both indexed by the unit's trajectory slot, so a launch
// may cover a subset of the slices).  Other steps: by kind (STORE, STORE2 = also gold,
// CORRECT = the parareal update F_old + (x - G_old), then G_old = x).
__device__ inline void epi_store(const StepArgs& a, const Epilogue& ep, int u, long slot,
                                 bool last_fine, int k, double x) {
  if (ep.kind == EPI_NONE || unit_done(a, u)) return;
  if (ep.kind == EPI_CORRECT) {
    const double go = ep.gold[(long)u * ep.gold_stride + k];
    ep.out[(long)u * ep.out_stride + k] = ep.fold[(long)u * ep.fold_stride + k] + (x - go);
    ep.gold[(long)u * ep.gold_stride + k] = x;
    return;
  }
  ep.out[slot * ep.out_stride + k] = x;
  const bool g = (a.mode == MODE_FINE) ? last_fine : (ep.kind == EPI_STORE2);
  const long gi = (a.mode == MODE_FINE) ? slot : (long)u;  // fine steps: by trajectory slot
  if (g && ep.gold) ep.gold[gi * ep.gold_stride + k] = x;
}

// ---- launchers (implemented in the .hip files) ----
hipError_t launch_tables(const Tables& tb, double* xq, double* wq, double* phi, double* phiT,
                         double* dphi, double* inst, double* bw, double* bhyb, double* cosq,
                         const double* alpha_dev, const int32_t* Mb, const int32_t* Sb,
                         hipStream_t s, double* b12 = nullptr, double* s2 = nullptr);
// 2D steps (gemm2d.hip)
hipError_t launch_step2d_products(const Tables& tb, const StepArgs& a, int units, double* Cbuf,
                                  double* T, double* mom, hipStream_t s, bool moments = true);
hipError_t launch_stiff2d_grid(const Tables& tb, const StepArgs& a, int units, const double* V,
                               double* G, hipStream_t s);
// preconditioned conjugate gradients for the 2D step systems (cg2d.hip): the start (init) or
// one iteration, after the second half of the stiffness product from G (per-chunk partials in
// kvp [units][2Qp/16][256][16]); cgs [units][8], pd [units][Mp] the Jacobi diagonal
hipError_t launch_cg_step(const Tables& tb, const StepArgs& a, int units, const double* G,
                          double* kvp, const double* x0, double* x, double* r, double* p,
                          double* pd, double* cgs, int cap, double tol, bool init, hipStream_t s);
// constant-D diagonal step solve (gemm2d.hip): rhs holds the history sums, F the load vector
hipError_t launch_diag_solve(const Tables& tb, const StepArgs& a, const Epilogue& e, int units,
                             const double* F, hipStream_t s);
hipError_t launch_cg_count(const double* cgs, int units, int32_t* out, hipStream_t s);
hipError_t launch_cg_finish(const Tables& tb, const StepArgs& a, const Epilogue& e, int units,
                            const double* x, hipStream_t s);
hipError_t launch_assemble2d(const Tables& tb, const StepArgs& a, int units, const double* mom,
                             hipStream_t s);
hipError_t launch_form_rhs(const Tables& tb, const StepArgs& a, int units, hipStream_t s);
hipError_t launch_fill(double* x, long n, double v, hipStream_t s);
hipError_t launch_identity(double* A, int units, int n, hipStream_t s);
// full-history parareal (histfull.hip)
hipError_t launch_interp_slots(const Tables& tb, const double* Z, double* prev, hipStream_t s);
// Prefix sums of full-history L1 sums, for every step r = 1..S of slices n_hi - n_cnt + 1 ..
// n_hi (all >= 1): hp[(b hpP + n - hp_n0) S + r - 1][k] = sum_{j=1}^{nS-1} b_{nS+r-j}
// (x_j - x_{j-1}), ascending j, where instance b's states x_j (j = qS + t, t = 1..S) are row
// q slot_rows + t of x + b inst_stride, and x_0 its row 0.
struct PrefixArgs {
  const double* x;
  long inst_stride;
  int slot_rows, S, n_hi, n_cnt;
  double* hp;
  int hpP, hp_n0;
  bool narrow;  // 8 steps per wave (few slices per launch) instead of 32
};
hipError_t launch_hist_prefix(const Tables& tb, const PrefixArgs& pa, hipStream_t s);
hipError_t launch_eval(const Tables& tb, const StepArgs& a, int units, hipStream_t s);
hipError_t launch_assemble(const Tables& tb, const StepArgs& a, int units, hipStream_t s);
// blocked factorisation and solve through device memory (chol_blk.hip): A and rhs of the
// step arguments are overwritten; q is scratch of units * ceil(Mp / nb) * nb doubles
hipError_t launch_blk_solve(const Tables& tb, const StepArgs& a, const Epilogue& e, int units,
                            double* q, hipStream_t s);
hipError_t launch_blk_diag(const Tables& tb, const StepArgs& a, int units, double* A, double* rhs,
                           int r0, int w, hipStream_t s);
// One step of iterative refinement after launch_blk_solve (1D, epilogue EPI_NONE, so the
// solution x is in a.rhs): xs = x, r = rhs0 - (I + tau dphi^T diag(d) dphi) x with the step's
// own d, then L L^T e = r with the stored factor, and the epilogue e stores x + e.
hipError_t launch_blk_refine1d(const Tables& tb, const StepArgs& a, const Epilogue& e, int units,
                               double* q, const double* rhs0, double* xs, hipStream_t s);
bool reg_path_ok(int Mp, int Qp);
// skinny: 16 x 16 tiles with a split reduction (few units) instead of 32 x 32 tiles.  Both
// give every output as a fixed-order sum over its own row, but the two orders differ, so
// every step whose result must match another run bit for bit (the fine steps of a serial
// solve and of a parareal sweep) has to use the same variant.
hipError_t launch_lag_gemm(const Tables& tb, const StepArgs& a, int units, double* dq, double* gq,
                           bool skinny, hipStream_t s);
hipError_t launch_proj_gemm(const Tables& tb, int units, const double* dq, const double* gq,
                            double* m, double* F, bool skinny, hipStream_t s);
hipError_t launch_history(const Tables& tb, const StepArgs& a, int units, double* hist,
                          hipStream_t s);
hipError_t launch_chol_reg(const Tables& tb, const StepArgs& a, const Epilogue& e, int units,
                           const double* mom, const double* F, const double* hist,
                           hipStream_t s);
hipError_t launch_pack(const double* src, int M, int B, long src_stride, double* dst, int Mp,
                       long dst_stride, hipStream_t s);
hipError_t launch_copy_rows(const double* src, long src_unit_stride, double* dst,
                            long dst_unit_stride, int rows, int Mp, int units, hipStream_t s);
hipError_t launch_fill_slot0(const Tables& tb, const double* Z, double* traj, int B, int P,
                             hipStream_t s);
hipError_t launch_unpack(const double* src, int Mp, long src_stride, double* dst, int M,
                         long dst_stride, int rows_per_unit, int units, hipStream_t s);
hipError_t launch_unpack_pad(const double* src, int M, long src_stride, double* dst, int Mp,
                             long dst_stride, int rows_per_unit, int units, hipStream_t s);
// Per-instance relative increment ||Znew_b - Zold_b|| / ||Znew_b|| of sweep k (0-based), and
// the per-instance stop test: an unfinished instance whose increment is <= exit_tol is marked
// done (done[b] = 1, conv[b] = k + 1); a non-finite increment marks it done with
// conv[b] = L1PR_ENONFINITE and sets FLAG_NONFINITE.  Finished instances keep their record.
// With lg_off set (learned coarse step), an unfinished instance whose increment exceeds
// kLearnedMinContraction times its previous sweep's (incr_prev) gets lg_off[b] = 1: the learned
// correction is off for it from then on, and its G_old rows (gold, gper doubles per instance)
// are replaced by the plain coarse values stored in gplain.
constexpr double kLearnedMinContraction = 0.5;
hipError_t launch_increment(const double* Znew, const double* Zold, int B, int rows, int Mp,
                            double* incr_out, int incr_stride, int k, double* incr_k,
                            int32_t* done, int32_t* conv, double exit_tol, int* flag,
                            hipStream_t s, int32_t* lg_off = nullptr, double* incr_prev = nullptr,
                            double* gold = nullptr, const double* gplain = nullptr, long gper = 0);
// After the first fine sweep of a learned parareal run: each unfinished instance on the learned
// coarse step whose learned G_old(n) are not closer to the fine results F_old(n) (row
// (b P + n) of fold, fold_stride apart) than the plain values gplain goes back to the plain
// step (lg_off) with G_old replaced by the plain values.
hipError_t launch_learned_judge(const double* fold, long fold_stride, double* gold,
                                const double* gplain, int B, int P, int Mp, const int32_t* done,
                                int32_t* lg_off, hipStream_t s);
// Zdst[b] = Zsrc[b] (rows x Mp) for the finished instances
hipError_t launch_copy_done(const double* Zsrc, double* Zdst, const int32_t* done, int B, long per,
                            hipStream_t s);
// per-instance status after `sweeps` sweeps: finished instances keep conv[b]; the others get
// `sweeps` if notconv is false, else L1PR_ENOTCONV
hipError_t launch_finish_status(const int32_t* done, const int32_t* conv, int32_t* out, int B,
                                int sweeps, bool notconv, hipStream_t s);
// sets FLAG_NONFINITE if any of x[0..n) is NaN or infinite
hipError_t launch_check_finite(const double* x, long n, int* flag, hipStream_t s);
hipError_t launch_fill_int(int32_t* x, int n, int32_t v, hipStream_t s);
hipError_t launch_stamp(int64_t* t, hipStream_t s);

}  // namespace l1pr
