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
// Prefix kernel: one wave per (instance, 64 coefficients, slice n, chunk of RC steps r).
// Lane = coefficient; it holds RC accumulators (one per step r) and streams the rows x_j of
// the instance's previous trajectory once, JB rows per block.  The weights b_{nS+r-j} of a
// block are wave-uniform and span RC + JB - 1 consecutive table entries, loaded as scalars;
// every x_j then feeds RC fmas.  Waves of one (instance, coefficient block) read the same
// rows at about the same pace; the work-group ids are remapped so that they run on one XCD
// and share its L2, with the largest slices first.
#include "l1pr_internal.h"

namespace l1pr {

namespace {

constexpr int NXCD = 8;
constexpr int HP_RC = 32;  // steps per wave
constexpr int HP_JB = 4;   // rows per block
static_assert(HP_RC % 8 == 0, "steps are taken eight at a time");

__device__ inline int xcd_remap_hp(int id, int total) {
  const int q = total / NXCD, rem = total % NXCD, x = id % NXCD, k = id / NXCD;
  return x < rem ? x * (q + 1) + k : rem * (q + 1) + (x - rem) * q + k;
}

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
__global__ __launch_bounds__(64) void k_hist_prefix(Tables tb, const double* prev, double* hp,
                                                    int nrc, int nkb) {
  const int S = tb.S, P = tb.P, Mp = tb.Mp;
  const int lin = xcd_remap_hp(blockIdx.x, gridDim.x);
  const int per_group = (P - 1) * nrc;
  const int grp = lin / per_group, w = lin % per_group;
  const int b = grp / nkb, kb = grp % nkb;
  const int n = P - 1 - w / nrc, rc = w % nrc;  // slices 1..P-1, largest first
  const int k = kb * 64 + (int)threadIdx.x;
  const int kc = k < Mp ? k : Mp - 1;  // lanes past Mp load a valid row entry, store nothing
  const int r0 = rc * RC + 1;
  const long nS = (long)n * S;
  const double* bw = tb.bw + (long)b * tb.LB + nS + r0;  // bw[j'] = b_{nS + r0 + j'}
  const double* x = prev + (long)b * P * (S + 1) * Mp + kc;

  double acc[RC];
#pragma unroll
  for (int i = 0; i < RC; ++i) acc[i] = 0.0;
  double xp = x[0];  // x_0
  // j = qS + t for slots q = 0..n-1, rows t = 1..S (the last slot stops at t = S-1)
  for (int q = 0; q < n; ++q) {
    const int tend = q == n - 1 ? S - 1 : S;
    const double* row = x + (long)q * (S + 1) * Mp;
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
    double* out = hp + ((long)(b * P + n) * S + (r0 - 1)) * Mp + k;
#pragma unroll
    for (int ri = 0; ri < RC; ++ri)
      if (r0 + ri <= S) out[(long)ri * Mp] = acc[ri];
  }
}

}  // namespace

hipError_t launch_interp_slots(const Tables& tb, const double* Z, double* prev, hipStream_t s) {
  const long n = (long)tb.B * tb.P * (tb.S + 1) * tb.Mp;
  k_interp_slots<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(Z, prev, tb.B, tb.P, tb.S, tb.Mp);
  return hipGetLastError();
}

// Needs the weight table padded to LB >= N + HP_RC - 1 entries per instance: a chunk's last
// steps r may pass S, and their (never stored) weights are read from the padding.
hipError_t launch_hist_prefix(const Tables& tb, const double* prev, double* hp, hipStream_t s) {
  if (tb.P < 2) return hipSuccess;
  if (tb.LB < tb.N + HP_RC - 1) return hipErrorInvalidValue;
  const int nrc = (tb.S + HP_RC - 1) / HP_RC, nkb = (tb.Mp + 63) / 64;
  const long waves = (long)tb.B * nkb * (tb.P - 1) * nrc;
  if (waves > 0x7fffffffL) return hipErrorInvalidValue;
  k_hist_prefix<HP_RC, HP_JB><<<(unsigned)waves, 64, 0, s>>>(tb, prev, hp, nrc, nkb);
  return hipGetLastError();
}

}  // namespace l1pr
