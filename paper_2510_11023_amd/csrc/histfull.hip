// Full-history parareal: the fine propagator of slice n takes its L1 history over the whole
// fine grid, from the previous iterate's fine trajectories for the steps before nS (the fixed
// point is the uniform full-history L1 solution; Section 2.2's propagators with the history
// of Section 2.1 left untruncated).
//
// The sum for step r of slice n is, in ascending j,
//   sum_{j=1}^{nS-1} b_{nS+r-j} (x_j - x_{j-1})   (earlier slices, previous iterate)
// + sum_{j=nS}^{nS+r-1} ...                        (the slice's own states, step by step).
// The first part depends only on data fixed before the sweep, so one launch per sweep
// computes it for every (slice, step) and stores it in hp; each fine step then continues the
// same fma chain over its own rows (full_fine_history).  The chain's order is that of the
// full-history serial step, so a slice whose inputs equal the serial states reproduces them
// bit for bit, and parareal's exactness after k sweeps holds bitwise.
//
// The full-history serial solve uses the same kernel on its own trajectory, block by block:
// before the first step of block n (W steps), the sums over j < nW for all W steps of the
// block; each step then continues over at most W rows instead of all m.
//
// Prefix kernel: one wave per (instance, 64 coefficients, slice n, chunk of RC steps r).
// Lane = coefficient; it holds RC accumulators (one per step r) and streams the rows x_j of
// the instance's previous trajectory once, JB rows per block.  The weights b_{nS+r-j} of a
// block are wave-uniform and span RC + JB - 1 consecutive table entries, loaded as scalars;
// every x_j then feeds RC fmas.  Waves are issued longest first (slice P-1 down to 1): the
// work per wave grows with n, and this order leaves no long wave for the end of the launch
// (11% faster than grouping the waves of one instance per XCD).  Work-group ids go round
// robin over the 8 XCDs, so when B * blocks * chunks is a multiple of 8 the waves of one
// (instance, block, chunk) for every n land on the same XCD and share its L2.
#include "l1pr_internal.h"

namespace l1pr {

constexpr int HP_RC = 32;  // steps per wave
constexpr int HP_JB = 8;   // rows per block
static_assert(HP_RC % 8 == 0, "steps are taken eight at a time");

// prev[b*P + q][t][k] = Z_q + (t/S) (Z_{q+1} - Z_q): the linear interpolation of the coarse
// iterate over each slice, the history before the first fine sweep.
__global__ void k_interp_slots(const double* Z, double* prev, int B, int P, int S, int Mp) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long per = (long)(S + 1) * Mp;
  if (idx >= (long)B * P * per) return;
  const long slot = idx / per, e = idx % per;
  const int t = (int)(e / Mp), k = (int)(e % Mp);
  const long b = slot / P, q = slot % P;
  const double a0 = Z[(b * (P + 1) + q) * Mp + k], a1 = Z[(b * (P + 1) + q + 1) * Mp + k];
  prev[idx] = t == 0 ? a0 : a0 + ((double)t / (double)S) * (a1 - a0);
}

template <int RC, int JB>
__global__ __launch_bounds__(64) void k_hist_prefix(Tables tb, PrefixArgs pa, int nrc, int nkb) {
  const int S = pa.S, Mp = tb.Mp;
  // slices n_hi down to n_hi - n_cnt + 1 (the longest sums first), then (instance, block,
  // chunk)
  const int lin = blockIdx.x;
  const int per_n = tb.B * nkb * nrc;
  const int n = pa.n_hi - lin / per_n, w = lin % per_n;
  const int b = w / (nkb * nrc), kb = (w / nrc) % nkb, rc = w % nrc;
  const int k = kb * 64 + (int)threadIdx.x;
  const int kc = k < Mp ? k : Mp - 1;  // lanes past Mp load a valid row entry, store nothing
  const int r0 = rc * RC + 1;
  const long nS = (long)n * S;
  const double* bw = tb.bw + (long)b * tb.LB + nS + r0;  // bw[j'] = b_{nS + r0 + j'}
  const double* x = pa.x + (long)b * pa.inst_stride + kc;

  double acc[RC];
#pragma unroll
  for (int i = 0; i < RC; ++i) acc[i] = 0.0;
  double xp = x[0];  // x_0
  // j = qS + t for slots q = 0..n-1, rows t = 1..S (the last slot stops at t = S-1)
  for (int q = 0; q < n; ++q) {
    const int tend = q == n - 1 ? S - 1 : S;
    const double* row = x + (long)q * pa.slot_rows * Mp;
    const long jq = (long)q * S;
    int t = 1;
    for (; t + JB - 1 <= tend; t += JB) {
      double xv[JB];
#pragma unroll
      for (int jj = 0; jj < JB; ++jj) xv[jj] = row[(long)(t + jj) * Mp];
      double d[JB];
#pragma unroll
      for (int jj = 0; jj < JB; ++jj) {
        d[jj] = xv[jj] - xp;
        xp = xv[jj];
      }
      // weights b_{nS + r - j} for r = r0 + ri, j = jq + t + jj: entry ri - jj - jq - t of bw;
      // eight steps at a time, so that the window (8 + JB - 1 scalars) stays in SGPRs
      const double* wb = bw - jq - t - (JB - 1);
#pragma unroll
      for (int rs = 0; rs < RC; rs += 8) {
        double wv[8 + JB - 1];
#pragma unroll
        for (int i = 0; i < 8 + JB - 1; ++i) wv[i] = wb[rs + i];
#pragma unroll
        for (int jj = 0; jj < JB; ++jj)
#pragma unroll
          for (int ri = 0; ri < 8; ++ri)
            acc[rs + ri] = fma(wv[ri - jj + JB - 1], d[jj], acc[rs + ri]);
      }
    }
    for (; t <= tend; ++t) {
      const double xj = row[(long)t * Mp];
      const double d = xj - xp;
      xp = xj;
      const double* wb = bw - jq - t;
#pragma unroll
      for (int rs = 0; rs < RC; rs += 8) {
        double wv[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) wv[i] = wb[rs + i];
#pragma unroll
        for (int ri = 0; ri < 8; ++ri) acc[rs + ri] = fma(wv[ri], d, acc[rs + ri]);
      }
    }
  }
  if (k < Mp) {
    double* out = pa.hp + ((long)(b * pa.hpP + n - pa.hp_n0) * S + (r0 - 1)) * Mp + k;
#pragma unroll
    for (int ri = 0; ri < RC; ++ri)
      if (r0 + ri <= S) out[(long)ri * Mp] = acc[ri];
  }
}

hipError_t launch_interp_slots(const Tables& tb, const double* Z, double* prev, hipStream_t s) {
  const long n = (long)tb.B * tb.P * (tb.S + 1) * tb.Mp;
  k_interp_slots<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(Z, prev, tb.B, tb.P, tb.S, tb.Mp);
  return hipGetLastError();
}

// A chunk's last steps r may pass S: their (never stored) weights are read from the padding
// of the weight table, which must reach index n_hi S + S + RC - 2.
hipError_t launch_hist_prefix(const Tables& tb, const PrefixArgs& pa, hipStream_t s) {
  if (pa.n_cnt < 1) return hipSuccess;
  const int RC = pa.narrow ? 8 : HP_RC;
  if (pa.n_hi - pa.n_cnt + 1 < 1 || (long)pa.n_hi * pa.S + pa.S + RC - 1 > tb.LB)
    return hipErrorInvalidValue;
  const int nrc = (pa.S + RC - 1) / RC, nkb = (tb.Mp + 63) / 64;
  const long waves = (long)tb.B * nkb * pa.n_cnt * nrc;
  if (waves > 0x7fffffffL) return hipErrorInvalidValue;
  if (pa.narrow)
    k_hist_prefix<8, HP_JB><<<(unsigned)waves, 64, 0, s>>>(tb, pa, nrc, nkb);
  else
    k_hist_prefix<HP_RC, HP_JB><<<(unsigned)waves, 64, 0, s>>>(tb, pa, nrc, nkb);
  return hipGetLastError();
}

}  // namespace l1pr
