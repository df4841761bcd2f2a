// Host orchestration and the C-ABI of libl1pr.
//
// serial (hybrid):  for n = 0..P-1, r = 1..S: one step over the B instances (units = B).
// serial (full):    for m = 0..N-1: one full-history step over the B instances.
// parareal:         coarse initial sweep (P steps, units = B); then per sweep the fine
//                   propagator of all B*P (instance, slice) units in lockstep (S steps,
//                   units = B*P) followed by the sequential correction sweep (P steps,
//                   units = B) and the increment reduction (Section 2.2, flowchart).
//                   Full history: the fine sweep also reads the previous iterate's fine
//                   trajectories (one prefix launch forms their share of every history sum).
// Everything is enqueued on the caller's stream; nothing is allocated.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "l1pr_internal.h"
#include "l1pr_mlp.h"

namespace l1pr {

namespace {

constexpr int kMaxModes1D = 1024;  // the 1D evaluation kernel stages Mp + Qp doubles in LDS
constexpr int kMaxModes2D = 64;
constexpr int kMaxModes2DDiag = 256;  // the diagonal solve forms no system matrix
constexpr int kMaxModes1DDiag = 4096;  // ... and in 1D runs the GEMM products at any size
constexpr int kSerialBlock = 64;  // steps per prefix launch of the full-history serial solve
constexpr int kCgCap = 200;       // conjugate-gradient iterations per step solve, at most
constexpr int kCgCheck = 4;       // iterations between the host's convergence checks
// relative residual at which a step solve stops: the fine (and full-history) steps define
// the solution; a coarse step only steers parareal's convergence, its fixed point being that
// of the fine propagator, and it is deterministic at any tolerance, so exactness holds
constexpr double kCgTolFine = 1e-14, kCgTolCoarse = 1e-10;

struct Layout {
  size_t total = 0;
  size_t flags = 0;  // the call's device status word: offset 0 of every workspace (l1pr_check)
  size_t done = 0, conv = 0;  // parareal: per-instance finished flags and stop records [B]
  size_t lgoff = 0, incrp = 0;  // parareal: learned step switched off [B], previous increment [B]
  size_t xq, wq, phi, phiT, dphi, cosq, inst, bw, bhyb, alpha, Z0, Z1, Gold, traj, d, rhs, A, incrk;
  size_t g, mom, F, C2, T2, q;
  size_t rhs0 = 0, xs = 0;  // 1D blocked solve: right-hand side and first solution (refinement)
  size_t soe = 0, soeV = 0;  // history = 2: node tables [B][soeL][3], exponential sums [B][soeL][Mp]
  bool hasA = false;        // A [units][Mp][Mp] is part of the workspace
  size_t prev = 0, hp = 0;  // full-history parareal: previous trajectories, prefix sums
  size_t b12 = 0, s2 = 0;    // 2D: stacked basis tables of the separable stiffness products
  // conjugate-gradient solves (solver = 1): x, r, p, Jacobi diagonal [units][Mp];
  // G [units][2][Qp][Qp]; partial products [units][2Qp/16][4096]; per-unit scalars [units][8];
  // two counters
  size_t cgx = 0, cgr = 0, cgp = 0, cgpd = 0, cgG = 0, cgkv = 0, cgs = 0, cgcnt = 0;
};

size_t take(size_t& cur, size_t bytes) {
  const size_t off = cur;
  cur += (bytes + 255) / 256 * 256;
  return off;
}

bool valid(const l1pr_problem* p) {
  if (!p) return false;
  if (p->dim != 1 && p->dim != 2) return false;
  if (p->modes < 1 || p->quad < p->modes) return false;
  if (p->dim == 1 && p->solver == 2 && (p->modes > kMaxModes1DDiag || p->quad > 2 * kMaxModes1DDiag))
    return false;
  if (p->dim == 1 && p->solver != 2 &&
      (p->modes > kMaxModes1D || roundup(p->modes, 16) + roundup(p->quad, 16) > 8192))
    return false;
  if (p->dim == 2 && p->modes > (p->solver == 2 ? kMaxModes2DDiag : kMaxModes2D)) return false;
  if (p->dim == 2 && p->assembly != 0) return false;  // 2D forms the stiffness from moments
  if (p->steps < 1 || p->slices < 1 || p->steps % p->slices != 0) return false;
  if (!(p->alpha > 0.0 && p->alpha <= 1.0)) return false;
  if (!(p->T > 0.0) || !std::isfinite(p->T)) return false;
  if (p->d_sel < L1PR_D_CONST || p->d_sel > L1PR_D_LINEAR) return false;
  if (p->d_sel == L1PR_D_CONST && !(p->d_param > 0.0)) return false;
  if (p->f_sel < L1PR_F_ZERO || p->f_sel > L1PR_F_MMS_SMOOTH) return false;
  if (p->history < 0 || p->history > 2) return false;
  // the sum-of-exponentials history runs in the history kernel, which the 1D device-memory
  // factorisation path (history inside its evaluation kernel) does not use
  if (p->history == 2 && p->dim == 1 && p->solver != 2 && roundup(p->modes, 16) > 256) return false;
  if (p->source_time != 0 && p->source_time != 1) return false;
  if (p->source_time == 1 && (p->f_sel == L1PR_F_LOGISTIC || p->f_sel == L1PR_F_SIN)) return false;
  if (p->assembly != 0 && p->assembly != 1) return false;
  if (p->tune < 0 || p->tune > (TUNE_LAG_SKINNY | TUNE_PROJ_SKINNY | TUNE_NB128 | TUNE_TRAIL64))
    return false;
  if (p->solver < 0 || p->solver > 2) return false;
  if (p->solver == 1 && p->dim != 2) return false;  // the iterative solve is the 2D one
  // the diagonal solve needs the sine basis to diagonalise the stiffness: constant D, whose
  // stiffness it takes exactly (assembly does not apply)
  if (p->solver == 2 && (p->d_sel != L1PR_D_CONST || p->assembly != 0)) return false;
  // with fewer Gauss points the quadrature stiffness aliases into near-null directions that
  // the constant-coefficient preconditioner does not see
  if (p->solver == 1 && 2 * p->quad < 3 * p->modes) return false;
  return true;
}

// ---- sum-of-exponentials weights of the far L1 history (history = 2) ----------------------
// From b_j = (1-a) int_j^{j+1} s^-a ds and s^-a = (1/Gamma(a)) int_R exp(a y - s e^y) dy, the
// trapezoid rule in y on the grid y_n = n h gives b_j ~ sum_n w_n exp(-e^{y_n} j) with
// w_n = h (1-a)/Gamma(a) e^{(a-1) y_n} (1 - exp(-e^{y_n})).  Nodes with e^{y_n} >= 40 / j0 are
// dropped (their terms are below e^-40 at j >= j0); the nodes below n_lo, whose decay over N
// steps is below the tolerance, are merged into one node of rate 0 with their geometric sum
// as weight.  With h = 0.3 the weights match b_j to about 1e-13 for j0 <= j <= N.
constexpr double kSoeH = 0.3, kSoeEps = 1e-13;

int soe_n_hi() { return (int)std::ceil(std::log(40.0 / kSoeJ0) / kSoeH); }

int soe_n_lo(double a, int N) {
  const double num = kSoeEps * std::tgamma(a) * (1.0 - std::exp(-(a + 1.0) * kSoeH));
  const double den = kSoeH * (double)N * std::pow((double)N + 1.0, a);
  return (int)std::floor(std::log(num / den) / (a + 1.0) / kSoeH) + 1;
}

// nodes (rate, weight) for order a < 1, the merged rate-0 node first
void soe_nodes(double a, int N, std::vector<double>& rate, std::vector<double>& w) {
  const int lo = soe_n_lo(a, N), hi = soe_n_hi();
  const double c = kSoeH * (1.0 - a) / std::tgamma(a);
  rate.assign(1, 0.0);
  w.assign(1, c * std::exp(a * (double)(lo - 1) * kSoeH) / (1.0 - std::exp(-a * kSoeH)));
  for (int n = lo; n <= hi; ++n) {
    const double y = (double)n * kSoeH, lam = std::exp(y);
    rate.push_back(lam);
    w.push_back(c * std::exp((a - 1.0) * y) * (-std::expm1(-lam)));
  }
}

// nodes per instance for any order: the largest count over a fine grid of orders, plus two
int soe_max_nodes(int N) {
  int mx = 0;
  for (int i = 1; i < 1000; ++i) mx = std::max(mx, soe_n_hi() - soe_n_lo(i / 1000.0, N) + 2);
  return mx + 2;
}

void make_layout(const l1pr_problem* p, int B, int op, Layout& L, Tables& tb) {
  tb.dim = p->dim;
  tb.M1 = p->modes;
  tb.M1p = roundup(p->modes, 16);
  tb.M = p->dim == 1 ? p->modes : p->modes * p->modes;
  tb.Q = p->quad;
  tb.Mp = roundup(tb.M, 16);
  tb.Qp = roundup(p->quad, 16);
  tb.N = p->steps;
  tb.P = p->slices;
  tb.S = p->steps / p->slices;
  tb.B = B;
  // full history: b_0..b_N, plus entries read (never used) by the prefix kernel's last
  // block and step chunk
  tb.LB = p->history >= 1 ? p->steps + 1 + kSerialBlock + 64 : std::max(tb.S, tb.P) + 1;
  tb.soe = nullptr;
  tb.soeL = 0;
  tb.d_sel = p->d_sel;
  tb.f_sel = p->f_sel;
  tb.source_time = p->source_time;
  tb.tune = p->tune;
  tb.nb = (p->tune & TUNE_NB128) ? 128 : 256;
  tb.d_param = p->d_param;
  tb.T = p->T;
  const size_t D = sizeof(double);
  const size_t Mp = tb.Mp, Qp = tb.Qp, P = tb.P, S = tb.S, N = tb.N, M1p = tb.M1p;
  const size_t Jp = 2 * M1p + 1;
  const bool two = p->dim == 2;
  size_t cur = 0;
  L.flags = take(cur, 256);
  L.xq = take(cur, D * Qp);
  L.wq = take(cur, D * Qp);
  L.phi = take(cur, D * Qp * M1p);
  L.phiT = take(cur, D * Qp * M1p);
  // the 1D diagonal solve (solver 2) needs neither the derivative table nor the cosine table
  // (no stiffness is formed): at 4096 modes and 8192 points that saves 0.8 GB
  const bool diag1d = p->dim == 1 && p->solver == 2;
  L.dphi = diag1d ? 0 : take(cur, D * Qp * M1p);
  L.cosq = diag1d ? 0 : take(cur, D * Qp * Jp);
  L.inst = take(cur, D * B * NSCAL);
  L.bw = take(cur, D * B * tb.LB);
  L.bhyb = take(cur, D * B * P * S);
  L.alpha = take(cur, D * B);
  L.Z0 = take(cur, D * B * (P + 1) * Mp);
  const bool para = (op == L1PR_OP_PARAREAL);
  L.Z1 = para ? take(cur, D * B * (P + 1) * Mp) : 0;
  L.Gold = para ? take(cur, D * B * P * Mp) : 0;
  size_t units;
  if (para) {
    units = (size_t)B * P;
    L.traj = take(cur, D * units * (S + 1) * Mp);
    if (p->history == 1) {
      L.prev = take(cur, D * units * (S + 1) * Mp);
      L.hp = take(cur, D * units * S * Mp);
    }
  } else {
    units = B;
    L.traj = take(cur, D * B * ((p->history >= 1 ? N : S) + 1) * Mp);
    if (p->history == 1) L.hp = take(cur, D * B * kSerialBlock * Mp);
    if (p->history == 2) {
      tb.soeL = soe_max_nodes(p->steps);
      L.soe = take(cur, D * B * tb.soeL * 3);
      L.soeV = take(cur, D * B * tb.soeL * Mp);
    }
  }
  const size_t nq = two ? Qp * Qp : Qp;  // quadrature points per unit
  L.d = take(cur, D * units * nq);
  L.rhs = take(cur, D * units * Mp);
  const bool pcg = p->solver == 1, diag = p->solver == 2;
  // the system matrix goes through device memory only for the quadrature-GEMM assembly and
  // the blocked factorisation; with the cosine moments the factor kernel builds it in registers
  const bool in_regs = !two && !pcg && !diag && p->assembly == 0 && reg_path_ok(tb.Mp, tb.Qp);
  L.hasA = !(pcg || diag || in_regs);
  L.A = L.hasA ? take(cur, D * units * Mp * Mp) : 0;
  L.g = take(cur, D * units * nq);
  L.mom = diag ? 0 : take(cur, D * units * (two ? Jp * Jp : 2 * Mp + 1));
  L.F = take(cur, D * units * Mp);
  L.C2 = two ? take(cur, D * units * Mp) : 0;
  L.T2 = two ? take(cur, D * units * Qp * Jp) : 0;
  // back-substitution partial sums of the device-memory factorisation
  const size_t nblk = (Mp + tb.nb - 1) / tb.nb;
  const bool blocked = !(pcg || diag || reg_path_ok(tb.Mp, tb.Qp));
  L.q = blocked ? take(cur, D * units * nblk * tb.nb) : 0;
  if (blocked && !two) {
    L.rhs0 = take(cur, D * units * Mp);
    L.xs = take(cur, D * units * Mp);
  }
  if (two) {
    L.b12 = take(cur, D * M1p * 2 * Qp);
    L.s2 = take(cur, D * 2 * Qp * M1p);
  }
  if (pcg) {
    L.cgx = take(cur, D * units * Mp);
    L.cgr = take(cur, D * units * Mp);
    L.cgp = take(cur, D * units * Mp);
    L.cgpd = take(cur, D * units * Mp);
    L.cgG = take(cur, D * units * 2 * Qp * Qp);
    L.cgkv = take(cur, D * units * (2 * Qp / 16) * 4096);
    L.cgs = take(cur, D * units * 8);
    L.cgcnt = take(cur, 2 * sizeof(int32_t));
  }
  L.incrk = take(cur, D * B);
  if (para) {
    L.done = take(cur, sizeof(int32_t) * B);
    L.conv = take(cur, sizeof(int32_t) * B);
    L.lgoff = take(cur, sizeof(int32_t) * B);
    L.incrp = take(cur, D * B);
  }
  L.total = cur;
}

struct Ctx {
  Tables tb;
  Layout L;
  bool reg;      // register-resident step kernel (Mp <= 256)
  bool moments;  // stiffness from cosine moments, inside that kernel
  bool full;     // parareal with full-history fine propagators
  bool pcg;      // 2D step systems by preconditioned conjugate gradients
  bool diag;     // constant D: the diagonal solve in the sine basis
  const int32_t* done = nullptr;  // parareal: finished instances (skip their units)
  const int32_t* lg_off = nullptr;  // parareal, learned step: instances that went back to plain G
  char* ws;
  hipStream_t s;
  double* ptr(size_t off) const { return reinterpret_cast<double*>(ws + off); }
};

#define L1PR_TRY(expr)                          \
  do {                                          \
    if ((expr) != hipSuccess) return L1PR_EHIP; \
  } while (0)

// Per-instance inputs of an uneven batch (device arrays; any may be null).
struct Uneven {
  const double* alpha = nullptr;
  const int32_t* modes = nullptr;
  const int32_t* spp = nullptr;
};

// Set while l1pr_solve_batch runs its groups: the groups share one status word, cleared once
// by the batch call, so each group's setup leaves it as it is.
thread_local bool t_keep_flag = false;

l1pr_status setup(const l1pr_problem* p, int B, int op, const double* alpha, void* ws,
                  size_t ws_bytes, void* stream, Ctx& c, const Uneven& un = Uneven()) {
  if (!valid(p) || B < 1 || !ws) return L1PR_EINVAL;
  std::vector<double> al(B, p->alpha);
  if (alpha) {
    for (int b = 0; b < B; ++b) {
      if (!(alpha[b] > 0.0 && alpha[b] <= 1.0)) return L1PR_EINVAL;
      al[b] = alpha[b];
    }
  }
  make_layout(p, B, op, c.L, c.tb);
  if (ws_bytes < c.L.total) return L1PR_ENOMEM;
  c.ws = static_cast<char*>(ws);
  c.s = static_cast<hipStream_t>(stream);
  Tables& tb = c.tb;
  tb.xq = c.ptr(c.L.xq);
  tb.wq = c.ptr(c.L.wq);
  tb.phi = c.ptr(c.L.phi);
  tb.phiT = c.ptr(c.L.phiT);
  tb.dphi = c.L.dphi ? c.ptr(c.L.dphi) : nullptr;
  tb.inst = c.ptr(c.L.inst);
  tb.bw = c.ptr(c.L.bw);
  tb.bhyb = c.ptr(c.L.bhyb);
  tb.cosq = c.L.cosq ? c.ptr(c.L.cosq) : nullptr;
  tb.b12 = c.L.b12 ? c.ptr(c.L.b12) : nullptr;
  tb.s2 = c.L.s2 ? c.ptr(c.L.s2) : nullptr;
  tb.flag = reinterpret_cast<int*>(c.ws + c.L.flags);
  // bounded device waits poll up to 2^18 times; L1PR_TEST_SPIN_LIMIT lowers the bound so that
  // tests can exercise the give-up path (the kernels still run to their end)
  tb.spin = 1 << 18;
  if (const char* e = std::getenv("L1PR_TEST_SPIN_LIMIT")) tb.spin = std::max(0, std::atoi(e));
  if (!t_keep_flag) L1PR_TRY(launch_fill_int(tb.flag, 1, 0, c.s));
  c.pcg = p->solver == 1;
  c.diag = p->solver == 2;
  c.reg = reg_path_ok(tb.Mp, tb.Qp);
  c.moments = c.reg && p->assembly == 0 && p->dim == 1 && !c.diag;
  c.full = op == L1PR_OP_PARAREAL && p->history == 1;
  const double* alpha_dev = c.ptr(c.L.alpha);
  if (un.alpha)  // device array of the caller (nothing is copied, so the call can be captured)
    alpha_dev = un.alpha;
  else if (alpha)  // pageable source: the copy is staged before the call returns
    L1PR_TRY(hipMemcpyAsync(c.ptr(c.L.alpha), al.data(), sizeof(double) * B, hipMemcpyHostToDevice, c.s));
  else
    L1PR_TRY(launch_fill(c.ptr(c.L.alpha), B, p->alpha, c.s));
  L1PR_TRY(launch_tables(tb, c.ptr(c.L.xq), c.ptr(c.L.wq), c.ptr(c.L.phi), c.ptr(c.L.phiT),
                         c.L.dphi ? c.ptr(c.L.dphi) : nullptr, c.ptr(c.L.inst), c.ptr(c.L.bw),
                         c.ptr(c.L.bhyb), c.L.cosq ? c.ptr(c.L.cosq) : nullptr, alpha_dev,
                         un.modes, un.spp, c.s,
                         c.L.b12 ? c.ptr(c.L.b12) : nullptr, c.L.s2 ? c.ptr(c.L.s2) : nullptr));
  if (c.L.soe) {
    // per instance and node: (w, e^-lam, e^-lam j0); nodes past an instance's own count, and
    // every node at order 1 (where the far weights vanish), are zero
    const int Ls = tb.soeL;
    std::vector<double> tab((size_t)B * Ls * 3, 0.0), rate, w;
    for (int b = 0; b < B; ++b) {
      if (!(al[b] < 1.0)) continue;
      soe_nodes(al[b], p->steps, rate, w);
      if ((int)rate.size() > Ls) return L1PR_EINVAL;
      for (size_t l = 0; l < rate.size(); ++l) {
        double* t = &tab[((size_t)b * Ls + l) * 3];
        t[0] = w[l];
        t[1] = std::exp(-rate[l]);
        t[2] = std::exp(-rate[l] * kSoeJ0);
      }
    }
    // pageable source: the copy is staged before hipMemcpyAsync returns
    L1PR_TRY(hipMemcpyAsync(c.ptr(c.L.soe), tab.data(), sizeof(double) * tab.size(),
                            hipMemcpyHostToDevice, c.s));
    tb.soe = c.ptr(c.L.soe);
  }
  return L1PR_OK;
}

// Optional per-launch timing with HIP events recorded on the launch stream around each
// step kernel (l1pr_profile_start / l1pr_profile_stop).  Events come from a pool that
// persists across calls, so steady-state timing creates no events.
struct Profiler {
  std::mutex mu;
  bool on = false;
  std::vector<std::string> only;  // kernels to bracket (empty: all)
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  struct Rec { std::string name; size_t ev; };
  std::vector<Rec> recs;
  hipEvent_t next() {
    if (used == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
};
Profiler& prof() {
  static Profiler p;
  return p;
}

const char* mode_name(int mode) {
  return mode == MODE_FINE ? "fine" : (mode == MODE_COARSE ? "coarse" : "full");
}

template <class F>
hipError_t timed(const char* kernel, const StepArgs& a, int units, hipStream_t s, F&& launch) {
  Profiler& p = prof();
  if (!p.on) return launch();
  std::lock_guard<std::mutex> g(p.mu);
  if (!p.only.empty() && std::find(p.only.begin(), p.only.end(), kernel) == p.only.end())
    return launch();
  const size_t i0 = p.used;
  hipEvent_t e0 = p.next(), e1 = p.next();
  if (!e0 || !e1) return hipErrorOutOfMemory;
  hipError_t r = hipEventRecord(e0, s);
  if (r == hipSuccess) r = launch();
  if (r == hipSuccess) r = hipEventRecord(e1, s);
  char name[64];
  std::snprintf(name, sizeof(name), "%s/%s/%d", kernel, mode_name(a.mode), units);
  p.recs.push_back({name, i0});
  return r;
}

// One step for `units` units.
// Mp <= 256: batched MFMA GEMMs for the lagged state on the quadrature grid (then D and f)
//   and for the moments and load vector, a streaming kernel for the history sums, then the
//   register-resident factorisation and solve (stiffness from the moments, or from the
//   quadrature-GEMM assembly kernel when assembly = 1).
// Mp > 256: evaluation (1D) or the separable products (2D), the assembly, and the blocked
//   factorisation through device memory.
l1pr_status run_step(const Ctx& c, const StepArgs& a, const Epilogue& e, int units) {
  if (c.diag) {
    // constant D: the load vector at the lagged state (separable products in 2D, the two
    // GEMMs in 1D at any size), the history sums, then the diagonal solve
    if (c.tb.dim == 2) {
      L1PR_TRY(timed("products2d", a, units, c.s, [&] {
        return launch_step2d_products(c.tb, a, units, a.C2, a.T2, a.mom, c.s, false);
      }));
    } else {
      const bool coarse = a.mode == MODE_COARSE;
      const bool sk_lag = coarse || (c.tb.tune & TUNE_LAG_SKINNY);
      const bool sk_proj = coarse || (c.tb.tune & TUNE_PROJ_SKINNY);
      L1PR_TRY(timed("lag", a, units, c.s, [&] { return launch_lag_gemm(c.tb, a, units, a.d, a.g, sk_lag, c.s); }));
      L1PR_TRY(timed("proj", a, units, c.s, [&] {
        return launch_proj_gemm(c.tb, units, a.d, a.g, nullptr, a.F, sk_proj, c.s);
      }));
    }
    L1PR_TRY(timed("history", a, units, c.s, [&] { return launch_history(c.tb, a, units, a.rhs, c.s); }));
    L1PR_TRY(timed("diag", a, units, c.s, [&] { return launch_diag_solve(c.tb, a, e, units, a.F, c.s); }));
    return L1PR_OK;
  }
  if (c.tb.dim == 2 && c.pcg) {
    // separable products (lagged state, D, f, load vector, cosine moments for the Jacobi
    // diagonal), the history sums and the right-hand side, then conjugate gradients from the
    // lagged state with K applied separably; the host looks at the units' status every 4
    // iterations
    L1PR_TRY(timed("products2d", a, units, c.s, [&] {
      return launch_step2d_products(c.tb, a, units, a.C2, a.T2, a.mom, c.s);
    }));
    L1PR_TRY(timed("history", a, units, c.s, [&] { return launch_history(c.tb, a, units, a.rhs, c.s); }));
    L1PR_TRY(timed("rhs", a, units, c.s, [&] { return launch_form_rhs(c.tb, a, units, c.s); }));
    double* x = c.ptr(c.L.cgx);
    double* r = c.ptr(c.L.cgr);
    double* p = c.ptr(c.L.cgp);
    double* pd = c.ptr(c.L.cgpd);
    double* G = c.ptr(c.L.cgG);
    double* kv = c.ptr(c.L.cgkv);
    double* cgs = c.ptr(c.L.cgs);
    int32_t* cnt = reinterpret_cast<int32_t*>(c.ws + c.L.cgcnt);
    const double cg_tol = a.mode == MODE_COARSE ? kCgTolCoarse : kCgTolFine;
    auto grid = [&](const double* v) {
      return timed("cg_grid", a, units, c.s, [&] {
        return launch_stiff2d_grid(c.tb, a, units, v, G, c.s);
      });
    };
    L1PR_TRY(grid(a.C2));
    L1PR_TRY(timed("cg_step", a, units, c.s, [&] {
      return launch_cg_step(c.tb, a, units, G, kv, a.C2, x, r, p, pd, cgs, kCgCap, cg_tol, true, c.s);
    }));
    bool done = false;
    for (int it = 0; it < kCgCap && !done; it += kCgCheck) {
      for (int j = 0; j < kCgCheck; ++j) {
        L1PR_TRY(grid(p));
        L1PR_TRY(timed("cg_step", a, units, c.s, [&] {
          return launch_cg_step(c.tb, a, units, G, kv, nullptr, x, r, p, pd, cgs, kCgCap, cg_tol, false,
                                c.s);
        }));
      }
      int32_t h[2] = {0, 0};
      L1PR_TRY(launch_cg_count(cgs, units, cnt, c.s));
      L1PR_TRY(hipMemcpyAsync(h, cnt, sizeof(h), hipMemcpyDeviceToHost, c.s));
      L1PR_TRY(hipStreamSynchronize(c.s));
      if (h[1] > 0) return L1PR_ESOLVE;
      done = h[0] == 0;
    }
    if (!done) return L1PR_ESOLVE;
    L1PR_TRY(timed("cg_finish", a, units, c.s, [&] { return launch_cg_finish(c.tb, a, e, units, x, c.s); }));
    return L1PR_OK;
  }
  if (c.tb.dim == 2) {
    // separable products (lagged state at the Gauss points, D, f, load vector, cosine
    // moments), the system from the moments, the history sums, then the factorisation
    L1PR_TRY(timed("products2d", a, units, c.s, [&] {
      return launch_step2d_products(c.tb, a, units, a.C2, a.T2, a.mom, c.s);
    }));
    L1PR_TRY(timed("assemble2d", a, units, c.s, [&] { return launch_assemble2d(c.tb, a, units, a.mom, c.s); }));
    L1PR_TRY(timed("history", a, units, c.s, [&] { return launch_history(c.tb, a, units, a.rhs, c.s); }));
    if (c.reg) {
      L1PR_TRY(timed("chol", a, units, c.s, [&] {
        return launch_chol_reg(c.tb, a, e, units, nullptr, a.F, a.rhs, c.s);
      }));
    } else {
      L1PR_TRY(timed("rhs", a, units, c.s, [&] { return launch_form_rhs(c.tb, a, units, c.s); }));
      L1PR_TRY(timed("blk_solve", a, units, c.s, [&] {
        return launch_blk_solve(c.tb, a, e, units, c.ptr(c.L.q), c.s);
      }));
    }
    return L1PR_OK;
  }
  if (c.reg) {
    // GEMM variants.  Coarse steps (one unit per instance) take the skinny tiles for both
    // products.  Fine and full-history steps take the variants in the problem's tuning bits
    // (default: 32 x 32 tiles for both products), never a choice made from
    // the unit count, so a serial solve and a parareal fine sweep do the same arithmetic.
    const bool coarse = a.mode == MODE_COARSE;
    const bool sk_lag = coarse || (c.tb.tune & TUNE_LAG_SKINNY);
    const bool sk_proj = coarse || (c.tb.tune & TUNE_PROJ_SKINNY);
    L1PR_TRY(timed("lag", a, units, c.s, [&] { return launch_lag_gemm(c.tb, a, units, a.d, a.g, sk_lag, c.s); }));
    L1PR_TRY(timed("proj", a, units, c.s, [&] {
      return launch_proj_gemm(c.tb, units, a.d, a.g, c.moments ? a.mom : nullptr, a.F, sk_proj, c.s);
    }));
    if (!c.moments)
      L1PR_TRY(timed("assemble", a, units, c.s, [&] { return launch_assemble(c.tb, a, units, c.s); }));
    L1PR_TRY(timed("history", a, units, c.s, [&] { return launch_history(c.tb, a, units, a.rhs, c.s); }));
    L1PR_TRY(timed("chol", a, units, c.s, [&] {
      return launch_chol_reg(c.tb, a, e, units, c.moments ? a.mom : nullptr, a.F, a.rhs, c.s);
    }));
    return L1PR_OK;
  }
  // 1D beyond the register path: evaluation and history, quadrature-GEMM assembly, the blocked
  // factorisation and solve (result left in rhs), then one step of iterative refinement with
  // the step's own operator, whose epilogue stores the refined state
  L1PR_TRY(timed("eval", a, units, c.s, [&] { return launch_eval(c.tb, a, units, c.s); }));
  L1PR_TRY(timed("assemble", a, units, c.s, [&] { return launch_assemble(c.tb, a, units, c.s); }));
  double* rhs0 = c.ptr(c.L.rhs0);
  L1PR_TRY(launch_copy_rows(a.rhs, c.tb.Mp, rhs0, c.tb.Mp, 1, c.tb.Mp, units, c.s));
  Epilogue none{};
  none.kind = EPI_NONE;
  L1PR_TRY(timed("blk_solve", a, units, c.s, [&] {
    return launch_blk_solve(c.tb, a, none, units, c.ptr(c.L.q), c.s);
  }));
  L1PR_TRY(timed("refine", a, units, c.s, [&] {
    return launch_blk_refine1d(c.tb, a, e, units, c.ptr(c.L.q), rhs0, c.ptr(c.L.xs), c.s);
  }));
  return L1PR_OK;
}

StepArgs base_args(const Ctx& c) {
  StepArgs a;
  std::memset(&a, 0, sizeof(a));
  a.d = c.ptr(c.L.d);
  a.rhs = c.ptr(c.L.rhs);
  a.A = c.L.hasA ? c.ptr(c.L.A) : nullptr;
  a.g = c.ptr(c.L.g);
  a.mom = c.L.mom ? c.ptr(c.L.mom) : nullptr;
  a.F = c.ptr(c.L.F);
  a.C2 = c.L.C2 ? c.ptr(c.L.C2) : nullptr;
  a.T2 = c.L.T2 ? c.ptr(c.L.T2) : nullptr;
  a.done = c.done;
  a.soeV = c.L.soeV ? c.ptr(c.L.soeV) : nullptr;
  return a;
}

l1pr_status serial_hybrid(const Ctx& c, const double* u0, double* U, double* traj_out) {
  const Tables& tb = c.tb;
  const int B = tb.B, P = tb.P, S = tb.S, Mp = tb.Mp, M = tb.M;
  const long vecP = (long)(P + 1) * Mp, slotS = (long)(S + 1) * Mp;
  double* Z = c.ptr(c.L.Z0);
  double* traj = c.ptr(c.L.traj);
  L1PR_TRY(launch_pack(u0, M, B, M, Z, Mp, vecP, c.s));
  if (traj_out) L1PR_TRY(launch_unpack(Z, Mp, vecP, traj_out, M, (long)(tb.N + 1) * M, 1, B, c.s));
  for (int n = 0; n < P; ++n) {
    L1PR_TRY(launch_copy_rows(Z + (long)n * Mp, vecP, traj, slotS, 1, Mp, B, c.s));
    for (int r = 1; r <= S; ++r) {
      StepArgs a = base_args(c);
      a.mode = MODE_FINE;
      a.r = r;
      a.nP = 1;
      a.n_lo = n;
      a.traj = traj;
      a.trajP = 1;
      a.trajN0 = n;
      a.Z = Z;
      Epilogue e{};  // the slice end is written at the instance's last step of the slice
      e.kind = EPI_STORE2;
      e.out = traj + (long)r * Mp;
      e.out_stride = slotS;
      e.gold = Z + (long)(n + 1) * Mp;
      e.gold_stride = vecP;
      l1pr_status st = run_step(c, a, e, B);
      if (st != L1PR_OK) return st;
    }
    if (traj_out)
      L1PR_TRY(launch_unpack(traj + Mp, Mp, slotS, traj_out + ((long)n * S + 1) * M, M,
                             (long)(tb.N + 1) * M, S, B, c.s));
  }
  L1PR_TRY(launch_unpack(Z, Mp, vecP, U, M, (long)(P + 1) * M, P + 1, B, c.s));
  L1PR_TRY(launch_check_finite(U, (long)B * (P + 1) * M, tb.flag, c.s));
  return L1PR_OK;
}

l1pr_status serial_full(const Ctx& c, const double* u0, double* U, double* traj_out) {
  const Tables& tb = c.tb;
  const int B = tb.B, P = tb.P, S = tb.S, N = tb.N, Mp = tb.Mp, M = tb.M;
  const long trajN = (long)(N + 1) * Mp;
  double* traj = c.ptr(c.L.traj);
  // history = 1: exact sums, by prefix blocks; history = 2: the far part by exponential sums
  const bool soe = tb.soe != nullptr;
  double* hp = soe ? nullptr : c.ptr(c.L.hp);
  L1PR_TRY(launch_pack(u0, M, B, M, traj, Mp, trajN, c.s));
  if (soe) L1PR_TRY(launch_fill(c.ptr(c.L.soeV), (long)B * tb.soeL * Mp, 0.0, c.s));
  for (int m = 0; m < N; ++m) {
    StepArgs a = base_args(c);
    a.mode = MODE_FULL;
    a.m = m;
    a.traj = traj;
    a.hp = hp;
    a.hw = kSerialBlock;
    if (!soe && m > 0 && m % kSerialBlock == 0) {
      // block n = m / W: the sums over j < nW for its W steps
      PrefixArgs pa{};
      pa.x = traj;
      pa.inst_stride = trajN;
      pa.slot_rows = kSerialBlock;
      pa.S = kSerialBlock;
      pa.n_hi = m / kSerialBlock;
      pa.n_cnt = 1;
      pa.hp = hp;
      pa.hpP = 1;
      pa.hp_n0 = pa.n_hi;
      pa.narrow = true;
      L1PR_TRY(timed("prefix", a, B, c.s, [&] { return launch_hist_prefix(tb, pa, c.s); }));
    }
    Epilogue e{};
    e.kind = EPI_STORE;
    e.out = traj + (long)(m + 1) * Mp;
    e.out_stride = trajN;
    l1pr_status st = run_step(c, a, e, B);
    if (st != L1PR_OK) return st;
  }
  for (int n = 0; n <= P; ++n)
    L1PR_TRY(launch_unpack(traj + (long)n * S * Mp, Mp, trajN, U + (long)n * M, M,
                           (long)(P + 1) * M, 1, B, c.s));
  if (traj_out) L1PR_TRY(launch_unpack(traj, Mp, trajN, traj_out, M, (long)(N + 1) * M, N + 1, B, c.s));
  L1PR_TRY(launch_check_finite(U, (long)B * (P + 1) * M, tb.flag, c.s));
  return L1PR_OK;
}

// Learned coarse propagator: network parameters and scratch (plain G values, network
// activations) carved after the solver's own workspace.
struct Learned {
  const void* params = nullptr;
  MlpLayout L{};
  double* G = nullptr;   // [B][Mp]: the plain coarse values of the current step
  double* Gp = nullptr;  // [B][P][Mp]: the plain coarse value behind each stored G_old(n)
  void* ws = nullptr;
};

// Scratch of the learned coarse step: the plain G values of the current step and of every
// stored G_old(n), and the inference activations of a network of up to kMlpMaxModes modes (a
// network may cover more modes than the batch).
size_t learned_extra_bytes(const Tables& tb) {
  const MlpLayout L = mlp_layout(kMlpMaxModes);
  return (sizeof(double) * (size_t)tb.B * tb.Mp + 255) / 256 * 256 +
         (sizeof(double) * (size_t)tb.B * tb.P * tb.Mp + 255) / 256 * 256 +
         mlp_infer_ws_bytes(L, tb.B);
}

// The learned coarse step of a parareal call: network `params` for `mnet` >= M modes (1D,
// history 0), scratch after the solver's workspace.
l1pr_status make_learned(const Ctx& c, const void* params, int mnet, size_t ws_bytes, Learned& lg) {
  if (!params || ((uintptr_t)params & 255) || c.tb.dim != 1 || c.full || mnet < c.tb.M ||
      mnet > kMlpMaxModes)
    return L1PR_EINVAL;
  if (ws_bytes < c.L.total + learned_extra_bytes(c.tb)) return L1PR_ENOMEM;
  lg.params = params;
  lg.L = mlp_layout(mnet);
  size_t off = c.L.total;
  lg.G = c.ptr(off);
  off += (sizeof(double) * (size_t)c.tb.B * c.tb.Mp + 255) / 256 * 256;
  lg.Gp = c.ptr(off);
  off += (sizeof(double) * (size_t)c.tb.B * c.tb.P * c.tb.Mp + 255) / 256 * 256;
  lg.ws = c.ws + off;
  return L1PR_OK;
}

// One coarse step G_n over all instances; `e` decides what is stored.  With a learned
// propagator, the plain step goes to a scratch vector and the network adds its correction
// before the epilogue.
l1pr_status coarse_step(const Ctx& c, double* Z, int n, const Epilogue& e, const Learned* lg) {
  StepArgs a = base_args(c);
  a.mode = MODE_COARSE;
  a.n = n;
  a.Z = Z;
  if (!lg) return run_step(c, a, e, c.tb.B);
  Epilogue tmp{};
  tmp.kind = EPI_STORE;
  tmp.out = lg->G;
  tmp.out_stride = c.tb.Mp;
  l1pr_status st = run_step(c, a, tmp, c.tb.B);
  if (st != L1PR_OK) return st;
  // where G_old(n) is stored, its plain value goes to Gp(n): the fallback to the plain coarse
  // step can then restore a plain G_old exactly
  const bool keeps_gold = e.kind == EPI_STORE2 || e.kind == EPI_CORRECT;
  double* gp = (keeps_gold && lg->Gp) ? lg->Gp + (long)n * c.tb.Mp : nullptr;
  L1PR_TRY(timed("mlp", a, c.tb.B, c.s, [&] {
    return mlp_coarse_apply(lg->L, lg->params, lg->G, c.tb.Mp, c.tb.inst, c.tb.B, c.tb.M, c.tb.Mp,
                            n, c.tb.P, e, lg->ws, c.s, c.done, c.lg_off, gp,
                            (long)c.tb.P * c.tb.Mp);
  }));
  return L1PR_OK;
}

// All B*P fine propagators at once on the slice ends Z: traj[b*P + n][r] = c_{n,r}.  With
// prev set (full history), the history of slice n also runs over the earlier slices' states
// in prev (the previous iterate's trajectories); their part of each sum is formed first, for
// every (slice, step), into hp.
// Slices below n_lo are not launched: their trajectory slots keep the previous sweep's values.
l1pr_status fine_sweep(const Ctx& c, const double* Z, double* traj, const double* prev,
                       int n_lo = 0) {
  const Tables& tb = c.tb;
  const int B = tb.B, P = tb.P, S = tb.S, Mp = tb.Mp;
  const long slotS = (long)(S + 1) * Mp;
  double* hp = prev ? c.ptr(c.L.hp) : nullptr;
  if (prev) {
    StepArgs a = base_args(c);
    a.mode = MODE_FINE;
    PrefixArgs pa{};
    pa.x = prev;
    pa.inst_stride = (long)P * slotS;
    pa.slot_rows = S + 1;
    pa.S = S;
    pa.n_hi = P - 1;
    pa.n_cnt = P - 1;
    pa.hp = hp;
    pa.hpP = P;
    pa.hp_n0 = 0;
    pa.narrow = false;
    L1PR_TRY(timed("prefix", a, B * P, c.s, [&] { return launch_hist_prefix(tb, pa, c.s); }));
  }
  L1PR_TRY(launch_fill_slot0(tb, Z, traj, B, P, c.s));
  const int nP = P - n_lo;
  for (int r = 1; r <= S; ++r) {
    StepArgs a = base_args(c);
    a.mode = MODE_FINE;
    a.r = r;
    a.nP = nP;
    a.n_lo = n_lo;
    a.traj = traj;
    a.trajP = P;
    a.trajN0 = 0;
    a.Z = Z;
    a.prev = prev;
    a.hp = hp;
    Epilogue e{};  // row r, and row S at the instance's last step of the slice
    e.kind = EPI_STORE;
    e.out = traj + (long)r * Mp;
    e.out_stride = slotS;
    e.gold = traj + (long)S * Mp;
    e.gold_stride = slotS;
    l1pr_status st = run_step(c, a, e, B * nP);
    if (st != L1PR_OK) return st;
  }
  return L1PR_OK;
}

// Uneven batches' convergence record: conv[b] = the first sweep whose increment is <=
// conv_tol (-1 if none; the instance is finished from then on); stamps[k] = device wall clock
// at the end of sweep k (k = 0: initial coarse sweep).  Both optional; neither needs the host,
// so the whole loop can be graph-captured.
struct Track {
  bool uneven = false;  // the stop test is conv_tol (no host synchronisation)
  int32_t* conv = nullptr;
  double conv_tol = -1.0;
  int64_t* stamps = nullptr;
};

// Parareal (Section 2.2 and its flowchart) with a per-instance stop: an instance whose
// increment meets the stop test (tol > 0, or the uneven batch's conv_tol) is finished; later
// sweeps keep its slice ends, and its units skip the factorisation and store nothing.  The
// status of each instance goes to status_out (device [B], may be null); the number of sweeps
// run to *sweeps_out.
l1pr_status parareal(const Ctx& c0, const double* u0, double* U, int max_iter, double tol,
                     double* U_iters, double* incr, int* sweeps_out, int32_t* status_out,
                     const Learned* lg, const Track& tr = Track()) {
  Ctx c = c0;
  const Tables& tb = c.tb;
  const int B = tb.B, P = tb.P, S = tb.S, Mp = tb.Mp, M = tb.M;
  const long vecP = (long)(P + 1) * Mp, slotS = (long)(S + 1) * Mp;
  double* Zk = c.ptr(c.L.Z0);
  double* Zk1 = c.ptr(c.L.Z1);
  double* Gold = c.ptr(c.L.Gold);
  double* traj = c.ptr(c.L.traj);
  // full history: the previous iterate's fine trajectories (swapped with traj every sweep)
  double* prev = c.full ? c.ptr(c.L.prev) : nullptr;
  double* incrk = c.ptr(c.L.incrk);
  int32_t* done = reinterpret_cast<int32_t*>(c.ws + c.L.done);
  int32_t* conv = tr.conv ? tr.conv : reinterpret_cast<int32_t*>(c.ws + c.L.conv);
  const double exit_tol = tr.uneven ? tr.conv_tol : (tol > 0.0 ? tol : -1.0);
  const long iterStride = (long)B * (P + 1) * M;

  L1PR_TRY(launch_fill_int(done, B, 0, c.s));
  L1PR_TRY(launch_fill_int(conv, B, -1, c.s));
  // learned coarse step: an instance goes back to the plain coarse step for good when, after
  // the first fine sweep, its learned coarse values are not closer to the fine results than the
  // plain ones, or when a later sweep shrinks its increment by less than half; its stored
  // G_old then become the plain values, so from the next sweep on its iteration is exactly
  // plain parareal (the first k+1 slice ends after k sweeps stay the serial ones whatever the
  // coarse step is)
  int32_t* lgoff = lg ? reinterpret_cast<int32_t*>(c.ws + c.L.lgoff) : nullptr;
  if (lgoff) L1PR_TRY(launch_fill_int(lgoff, B, 0, c.s));
  c.lg_off = lgoff;
  // coarse initial sweep: U^0_{n+1} = G_n(U^0_0..U^0_n), G_old(n) = the same value
  L1PR_TRY(launch_pack(u0, M, B, M, Zk, Mp, vecP, c.s));
  for (int n = 0; n < P; ++n) {
    Epilogue e{};
    e.kind = EPI_STORE2;
    e.out = Zk + (long)(n + 1) * Mp;
    e.out_stride = vecP;
    e.gold = Gold + (long)n * Mp;
    e.gold_stride = (long)P * Mp;
    l1pr_status st = coarse_step(c, Zk, n, e, lg);
    if (st != L1PR_OK) return st;
  }
  if (U_iters) L1PR_TRY(launch_unpack(Zk, Mp, vecP, U_iters, M, (long)(P + 1) * M, P + 1, B, c.s));
  if (tr.stamps) L1PR_TRY(launch_stamp(tr.stamps, c.s));
  // before the first sweep the history of earlier slices is the interpolated coarse iterate
  if (prev) L1PR_TRY(launch_interp_slots(tb, Zk, prev, c.s));

  // from here on the steps skip the units of finished instances
  c.done = done;
  int sweeps = 0;
  bool met = false;
  int hflag = 0;
  std::vector<double> h_incr(B);
  for (int k = 0; k < max_iter; ++k) {
    // parallel stage: F_old(n) = F_n(U^k_0..U^k_n) for all (b, n).  After k sweeps the slice
    // ends U^k_0..U^k_k equal those of the previous iterate bit for bit (they are the serial
    // solution), so for n < k the inputs of F_n are unchanged and its slot still holds F_n
    // from an earlier sweep: those units are not launched.  (Full history: the fine
    // propagators also read the previous trajectories, which swap every sweep; no skip.)
    const int n_lo = prev ? 0 : std::min(k, P - 1);
    l1pr_status stf = fine_sweep(c, Zk, traj, prev, n_lo);
    if (stf != L1PR_OK) return stf;
    // learned coarse step, first sweep: the plain step judges it against the fine results
    if (lg && k == 0)
      L1PR_TRY(launch_learned_judge(traj + (long)S * Mp, slotS, Gold, lg->Gp, B, P, Mp, done,
                                    lgoff, c.s));
    // sequential sweep: U^{k+1}_{n+1} = F_old(n) + (G_n(U^{k+1}_0..U^{k+1}_n) - G_old(n)).
    // For n <= k the inputs of G_n are the converged slice ends, the same as when G_old(n) was
    // formed, so the bracket is exactly zero: those rows are F_old(n), copied, and G_old(n)
    // stays.  Finished instances then take back their slice ends whole.
    L1PR_TRY(launch_pack(u0, M, B, M, Zk1, Mp, vecP, c.s));
    const int n_conv = std::min(k + 1, P);
    for (int n = 0; n < n_conv; ++n)
      L1PR_TRY(launch_copy_rows(traj + ((long)n * (S + 1) + S) * Mp, (long)P * slotS,
                                Zk1 + (long)(n + 1) * Mp, vecP, 1, Mp, B, c.s));
    L1PR_TRY(launch_copy_done(Zk, Zk1, done, B, vecP, c.s));
    for (int n = n_conv; n < P; ++n) {
      Epilogue e{};
      e.kind = EPI_CORRECT;
      e.out = Zk1 + (long)(n + 1) * Mp;
      e.out_stride = vecP;
      e.gold = Gold + (long)n * Mp;
      e.gold_stride = (long)P * Mp;
      e.fold = traj + ((long)n * (S + 1) + S) * Mp;
      e.fold_stride = (long)P * slotS;
      l1pr_status st = coarse_step(c, Zk1, n, e, lg);
      if (st != L1PR_OK) return st;
    }
    L1PR_TRY(launch_increment(Zk1, Zk, B, P + 1, Mp, incr, max_iter, k, incrk, done, conv,
                              exit_tol, tb.flag, c.s, lgoff, c.ptr(c.L.incrp), Gold,
                              lg ? lg->Gp : nullptr, (long)P * Mp));
    if (tr.stamps) L1PR_TRY(launch_stamp(tr.stamps + k + 1, c.s));
    if (U_iters)
      L1PR_TRY(launch_unpack(Zk1, Mp, vecP, U_iters + (long)(k + 1) * iterStride, M,
                             (long)(P + 1) * M, P + 1, B, c.s));
    std::swap(Zk, Zk1);
    if (prev) std::swap(traj, prev);
    sweeps = k + 1;
    if (sweeps >= P) {
      met = true;
      break;
    }
    if (tol > 0.0) {
      // host stop test: every instance finished (a finished instance's increment reads 0)
      L1PR_TRY(hipMemcpyAsync(h_incr.data(), incrk, sizeof(double) * B, hipMemcpyDeviceToHost, c.s));
      L1PR_TRY(hipMemcpyAsync(&hflag, tb.flag, sizeof(int), hipMemcpyDeviceToHost, c.s));
      L1PR_TRY(hipStreamSynchronize(c.s));
      if (hflag & FLAG_WAIT) break;
      double mx = 0.0;
      for (double v : h_incr) mx = std::max(mx, v);
      if (mx <= tol) {
        met = true;
        break;
      }
    }
  }
  L1PR_TRY(launch_unpack(Zk, Mp, vecP, U, M, (long)(P + 1) * M, P + 1, B, c.s));
  if (status_out)
    L1PR_TRY(launch_finish_status(done, conv, status_out, B, sweeps, tol > 0.0 && !met, c.s));
  if (sweeps_out) *sweeps_out = sweeps;
  if (tol > 0.0) {
    // the host synchronised every sweep: report the device status word now
    L1PR_TRY(hipMemcpyAsync(&hflag, tb.flag, sizeof(int), hipMemcpyDeviceToHost, c.s));
    L1PR_TRY(hipStreamSynchronize(c.s));
    if (hflag & FLAG_WAIT) return L1PR_EWAIT;
    if (hflag & FLAG_NONFINITE) return L1PR_ENONFINITE;
    if (!met) return L1PR_ENOTCONV;
  }
  return L1PR_OK;
}

// l1pr_solve_parareal with a network of mnet >= M modes (0: M)
l1pr_status solve_parareal_net(const l1pr_problem* p, int32_t batch, const double* alpha,
                               const double* u0, double* U, int32_t max_iter, double tol,
                               int32_t coarse, const void* mlp_params, int32_t mnet, int32_t* iters,
                               double* incr, double* U_iters, int32_t* sweeps, void* ws,
                               size_t ws_bytes, void* stream) {
  if (!u0 || !U || !p || p->history == 2) return L1PR_EINVAL;  // history 2: serial only
  if (max_iter < 0 || max_iter > p->slices || std::isnan(tol)) return L1PR_EINVAL;
  if (coarse != L1PR_COARSE_L1 && coarse != L1PR_COARSE_LEARNED) return L1PR_EINVAL;
  const bool learned = coarse == L1PR_COARSE_LEARNED;
  if (learned && (!mlp_params || p->dim != 1 || p->modes > kMlpMaxModes || p->history != 0))
    return L1PR_EINVAL;
  Ctx c;
  l1pr_status st = setup(p, batch, L1PR_OP_PARAREAL, alpha, ws, ws_bytes, stream, c);
  if (st != L1PR_OK) return st;
  Learned lg;
  if (learned) {
    st = make_learned(c, mlp_params, mnet > 0 ? mnet : c.tb.M, ws_bytes, lg);
    if (st != L1PR_OK) return st;
  }
  int it = 0;
  st = parareal(c, u0, U, max_iter, tol, U_iters, incr, &it, iters, learned ? &lg : nullptr);
  if (sweeps) *sweeps = it;
  return st;
}
}  // namespace
}  // namespace l1pr

using namespace l1pr;

extern "C" {

l1pr_status l1pr_validate(const l1pr_problem* p) { return valid(p) ? L1PR_OK : L1PR_EINVAL; }

size_t l1pr_workspace_bytes(const l1pr_problem* p, int32_t batch, int32_t op) {
  if (!valid(p) || batch < 1 || (op != L1PR_OP_SERIAL && op != L1PR_OP_PARAREAL)) return 0;
  Layout L;
  Tables tb;
  make_layout(p, batch, op, L, tb);
  return L.total;
}

l1pr_status l1pr_solve_serial(const l1pr_problem* p, int32_t batch, const double* alpha,
                              const double* u0, double* U, double* traj, void* ws,
                              size_t ws_bytes, void* stream) {
  try {
    if (!u0 || !U) return L1PR_EINVAL;
    Ctx c;
    l1pr_status st = setup(p, batch, L1PR_OP_SERIAL, alpha, ws, ws_bytes, stream, c);
    if (st != L1PR_OK) return st;
    return p->history >= 1 ? serial_full(c, u0, U, traj) : serial_hybrid(c, u0, U, traj);
  } catch (...) {
    return L1PR_EHIP;
  }
}

l1pr_status l1pr_solve_parareal(const l1pr_problem* p, int32_t batch, const double* alpha,
                                const double* u0, double* U, int32_t max_iter, double tol,
                                int32_t coarse, const void* mlp_params, int32_t* iters,
                                double* incr, double* U_iters, int32_t* sweeps, void* ws,
                                size_t ws_bytes, void* stream) {
  try {
    return solve_parareal_net(p, batch, alpha, u0, U, max_iter, tol, coarse, mlp_params, 0, iters,
                              incr, U_iters, sweeps, ws, ws_bytes, stream);
  } catch (...) {
    return L1PR_EHIP;
  }
}

l1pr_status l1pr_solve_serial_uneven(const l1pr_problem* p, int32_t batch,
                                     const l1pr_uneven* desc, const double* u0, double* U,
                                     void* ws, size_t ws_bytes, void* stream) {
  try {
    if (!p || !desc || !u0 || !U || p->history != 0 || p->dim != 1 || p->solver != 0)
      return L1PR_EINVAL;
    Uneven un;
    un.alpha = desc->alpha;
    un.modes = desc->modes;
    un.spp = desc->spp;
    Ctx c;
    l1pr_status st = setup(p, batch, L1PR_OP_SERIAL, nullptr, ws, ws_bytes, stream, c, un);
    if (st != L1PR_OK) return st;
    if (!c.reg) return L1PR_EINVAL;
    return serial_hybrid(c, u0, U, nullptr);
  } catch (...) {
    return L1PR_EHIP;
  }
}

l1pr_status l1pr_solve_parareal_uneven(const l1pr_problem* p, int32_t batch,
                                       const l1pr_uneven* desc, const double* u0, double* U,
                                       int32_t sweeps, double conv_tol, int32_t* conv,
                                       int64_t* stamps, double* incr, void* ws, size_t ws_bytes,
                                       void* stream) {
  try {
    if (!p || !desc || !u0 || !U || p->history != 0 || p->dim != 1 || p->solver != 0)
      return L1PR_EINVAL;
    if (sweeps < 0 || sweeps > p->slices || !(conv_tol >= 0.0)) return L1PR_EINVAL;
    Uneven un;
    un.alpha = desc->alpha;
    un.modes = desc->modes;
    un.spp = desc->spp;
    Ctx c;
    l1pr_status st = setup(p, batch, L1PR_OP_PARAREAL, nullptr, ws, ws_bytes, stream, c, un);
    if (st != L1PR_OK) return st;
    if (!c.reg) return L1PR_EINVAL;
    if (desc->coarse != L1PR_COARSE_L1 && desc->coarse != L1PR_COARSE_LEARNED) return L1PR_EINVAL;
    Learned lg;
    if (desc->coarse == L1PR_COARSE_LEARNED) {
      st = make_learned(c, desc->mlp, desc->mlp_modes, ws_bytes, lg);
      if (st != L1PR_OK) return st;
    }
    Track tr;
    tr.uneven = true;
    tr.conv = conv;
    tr.conv_tol = conv_tol;
    tr.stamps = stamps;
    int it = 0;
    return parareal(c, u0, U, sweeps, 0.0, nullptr, incr, &it, nullptr,
                    desc->coarse == L1PR_COARSE_LEARNED ? &lg : nullptr, tr);
  } catch (...) {
    return L1PR_EHIP;
  }
}

l1pr_status l1pr_autotune(const l1pr_problem* p, int32_t batch, void* ws, size_t ws_bytes,
                          void* stream, int32_t* tune_out) {
  try {
    if (!p || !tune_out) return L1PR_EINVAL;
    l1pr_problem q = *p;
    q.tune = 0;
    Ctx c;
    l1pr_status st = setup(&q, batch, L1PR_OP_PARAREAL, nullptr, ws, ws_bytes, stream, c);
    if (st != L1PR_OK) return st;
    const Tables& tb = c.tb;
    if (c.pcg) {  // no factorisation: nothing to choose
      *tune_out = 0;
      return L1PR_OK;
    }
    if (!c.reg && !c.diag) {
      // blocked factorisation: block width (256 / 128) and trailing tiles (128 / 64), timed on
      // a fine step's systems (B P units, set to the identity before each factorisation; the
      // kernels' work does not depend on the values)
      hipEvent_t e0, e1;
      L1PR_TRY(hipEventCreate(&e0));
      L1PR_TRY(hipEventCreate(&e1));
      const int units = tb.B * tb.P;
      float best = 1e30f;
      int32_t best_t = 0;
      for (int32_t t : {0, (int32_t)TUNE_NB128, (int32_t)TUNE_TRAIL64, (int32_t)(TUNE_NB128 | TUNE_TRAIL64)}) {
        c.tb.tune = t;
        c.tb.nb = (t & TUNE_NB128) ? 128 : 256;  // the layout's scratch covers both widths
        StepArgs a = base_args(c);
        a.mode = MODE_FINE;
        a.r = 1;
        a.nP = tb.P;
        a.traj = c.ptr(c.L.traj);
        a.trajP = tb.P;
        a.Z = c.ptr(c.L.Z0);
        Epilogue e{};
        e.kind = EPI_STORE;
        e.out = c.ptr(c.L.traj) + tb.Mp;  // row 1 of every slot
        e.out_stride = (long)(tb.S + 1) * tb.Mp;
        float total = 0.f;
        for (int rep = 0; rep < 3; ++rep) {
          L1PR_TRY(launch_identity(a.A, units, tb.Mp, c.s));
          L1PR_TRY(launch_fill(a.rhs, (long)units * tb.Mp, 0.0, c.s));
          L1PR_TRY(hipEventRecord(e0, c.s));
          L1PR_TRY(launch_blk_solve(c.tb, a, e, units, c.ptr(c.L.q), c.s));
          L1PR_TRY(hipEventRecord(e1, c.s));
          L1PR_TRY(hipEventSynchronize(e1));
          float ms = 0.f;
          L1PR_TRY(hipEventElapsedTime(&ms, e0, e1));
          if (rep > 0) total += ms;  // the first run warms up
        }
        if (total < best) {
          best = total;
          best_t = t;
        }
      }
      hipEventDestroy(e0);
      hipEventDestroy(e1);
      *tune_out = best_t;
      return L1PR_OK;
    }
    if (q.history != 0 || q.dim != 1) {  // no variants to choose between
      *tune_out = 0;
      return L1PR_OK;
    }
    const long vecP = (long)(tb.P + 1) * tb.Mp;
    double* Z = c.ptr(c.L.Z0);
    L1PR_TRY(launch_fill(Z, (long)tb.B * vecP, 0.0, c.s));
    L1PR_TRY(launch_fill_slot0(tb, Z, c.ptr(c.L.traj), tb.B, tb.P, c.s));
    hipEvent_t e0, e1;
    L1PR_TRY(hipEventCreate(&e0));
    L1PR_TRY(hipEventCreate(&e1));
    float best = 1e30f;
    int32_t best_t = 0;
    for (int32_t t = 0; t <= (TUNE_LAG_SKINNY | TUNE_PROJ_SKINNY); ++t) {
      c.tb.tune = t;
      StepArgs a = base_args(c);
      a.mode = MODE_FINE;
      a.r = 1;
      a.nP = tb.P;
      a.traj = c.ptr(c.L.traj);
      a.trajP = tb.P;
      a.Z = Z;
      Epilogue e{};
      e.kind = EPI_STORE;
      e.out = c.ptr(c.L.traj) + tb.Mp;  // row 1 of every slot
      e.out_stride = (long)(tb.S + 1) * tb.Mp;
      // the lagged-state product and the projections are what the bits change; time them
      // over a few launches after one warm-up, on a fine step (B P units, parareal) and on a
      // step of B units (the serial solve, which the same bits govern), and take the variant
      // with the smaller sum of the two
      const bool sk_lag = (t & TUNE_LAG_SKINNY) != 0, sk_proj = (t & TUNE_PROJ_SKINNY) != 0;
      float sum = 0.f;
      for (int units : {tb.B * tb.P, tb.B}) {
        float ms = 0.f;
        for (int rep = 0; rep < 4; ++rep) {
          if (rep == 1) L1PR_TRY(hipEventRecord(e0, c.s));
          L1PR_TRY(launch_lag_gemm(c.tb, a, units, a.d, a.g, sk_lag, c.s));
          L1PR_TRY(launch_proj_gemm(c.tb, units, a.d, a.g, c.moments ? a.mom : nullptr, a.F,
                                    sk_proj, c.s));
        }
        L1PR_TRY(hipEventRecord(e1, c.s));
        L1PR_TRY(hipEventSynchronize(e1));
        L1PR_TRY(hipEventElapsedTime(&ms, e0, e1));
        sum += ms;
      }
      (void)e;
      if (sum < best) {
        best = sum;
        best_t = t;
      }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    *tune_out = best_t;
    return L1PR_OK;
  } catch (...) {
    return L1PR_EHIP;
  }
}

size_t l1pr_parareal_learned_extra_bytes(const l1pr_problem* p, int32_t batch) {
  if (!valid(p) || batch < 1 || p->modes > kMlpMaxModes) return 0;
  Layout L;
  Tables tb;
  make_layout(p, batch, L1PR_OP_PARAREAL, L, tb);
  return learned_extra_bytes(tb);
}

l1pr_status l1pr_coarse_apply(const l1pr_problem* p, int32_t batch, const double* alpha,
                              const double* Z, double* out, void* ws, size_t ws_bytes,
                              void* stream) {
  try {
    if (!Z || !out) return L1PR_EINVAL;
    Ctx c;
    l1pr_status st = setup(p, batch, L1PR_OP_PARAREAL, alpha, ws, ws_bytes, stream, c);
    if (st != L1PR_OK) return st;
    if (p->history != 0) return L1PR_EINVAL;
    const Tables& tb = c.tb;
    const int B = tb.B, P = tb.P, Mp = tb.Mp, M = tb.M;
    const long vecP = (long)(P + 1) * Mp;
    double* Zp = c.ptr(c.L.Z0);
    double* Gout = c.ptr(c.L.Gold);
    L1PR_TRY(launch_unpack_pad(Z, M, (long)(P + 1) * M, Zp, Mp, vecP, P + 1, B, c.s));
    for (int n = 0; n < P; ++n) {
      Epilogue e{};
      e.kind = EPI_STORE;
      e.out = Gout + (long)n * Mp;
      e.out_stride = (long)P * Mp;
      st = coarse_step(c, Zp, n, e, nullptr);
      if (st != L1PR_OK) return st;
    }
    L1PR_TRY(launch_unpack(Gout, Mp, (long)P * Mp, out, M, (long)P * M, P, B, c.s));
    return L1PR_OK;
  } catch (...) {
    return L1PR_EHIP;
  }
}

l1pr_status l1pr_fine_apply(const l1pr_problem* p, int32_t batch, const double* alpha,
                            const double* Z, double* out, void* ws, size_t ws_bytes,
                            void* stream) {
  try {
    if (!Z || !out) return L1PR_EINVAL;
    Ctx c;
    l1pr_status st = setup(p, batch, L1PR_OP_PARAREAL, alpha, ws, ws_bytes, stream, c);
    if (st != L1PR_OK) return st;
    if (p->history != 0) return L1PR_EINVAL;
    const Tables& tb = c.tb;
    const int B = tb.B, P = tb.P, S = tb.S, Mp = tb.Mp, M = tb.M;
    const long vecP = (long)(P + 1) * Mp;
    double* Zp = c.ptr(c.L.Z0);
    L1PR_TRY(launch_unpack_pad(Z, M, (long)(P + 1) * M, Zp, Mp, vecP, P + 1, B, c.s));
    st = fine_sweep(c, Zp, c.ptr(c.L.traj), nullptr);
    if (st != L1PR_OK) return st;
    // slot b*P + n, row S  ->  out[b][n]
    L1PR_TRY(launch_unpack(c.ptr(c.L.traj) + (long)S * Mp, Mp, (long)(S + 1) * Mp, out, M, M, 1,
                           B * P, c.s));
    return L1PR_OK;
  } catch (...) {
    return L1PR_EHIP;
  }
}

void l1pr_profile_start_only(const char* names) {
  Profiler& p = prof();
  std::lock_guard<std::mutex> g(p.mu);
  p.on = true;
  p.used = 0;
  p.recs.clear();
  p.only.clear();
  for (const char* c = names; c && *c;) {
    const char* e = std::strchr(c, ',');
    const size_t n = e ? (size_t)(e - c) : std::strlen(c);
    if (n) p.only.emplace_back(c, n);
    c = e ? e + 1 : c + n;
  }
}

void l1pr_profile_start(void) { l1pr_profile_start_only(nullptr); }

int32_t l1pr_profile_stop(l1pr_kernel_stat* out, int32_t max_out) {
  Profiler& p = prof();
  std::lock_guard<std::mutex> g(p.mu);
  p.on = false;
  std::map<std::string, std::pair<int64_t, double>> agg;
  for (const auto& r : p.recs) {
    if (hipEventSynchronize(p.pool[r.ev + 1]) != hipSuccess) return -1;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.pool[r.ev], p.pool[r.ev + 1]) != hipSuccess) return -1;
    auto& a = agg[r.name];
    a.first += 1;
    a.second += ms;
  }
  p.recs.clear();
  p.used = 0;
  int32_t n = 0;
  for (const auto& kv : agg) {
    if (out && n < max_out) {
      std::memset(&out[n], 0, sizeof(l1pr_kernel_stat));
      std::snprintf(out[n].name, sizeof(out[n].name), "%s", kv.first.c_str());
      out[n].launches = kv.second.first;
      out[n].total_ms = kv.second.second;
    }
    ++n;
  }
  return n;
}

l1pr_status l1pr_device_stamp(int64_t* t, void* stream) {
  if (!t) return L1PR_EINVAL;
  return launch_stamp(t, static_cast<hipStream_t>(stream)) == hipSuccess ? L1PR_OK : L1PR_EHIP;
}

int64_t l1pr_wall_clock_khz(void) {
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) return -1;
  return khz;
}

l1pr_status l1pr_check(const void* ws, void* stream) {
  if (!ws) return L1PR_EINVAL;
  int f = 0;
  if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess) return L1PR_EHIP;
  if (hipMemcpy(&f, ws, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return L1PR_EHIP;
  if (f & FLAG_WAIT) return L1PR_EWAIT;
  if (f & FLAG_NONFINITE) return L1PR_ENONFINITE;
  return L1PR_OK;
}

const char* l1pr_status_string(l1pr_status s) {
  switch (s) {
    case L1PR_OK: return "ok";
    case L1PR_EINVAL: return "invalid problem or argument";
    case L1PR_ENOMEM: return "workspace too small";
    case L1PR_EHIP: return "HIP runtime error";
    case L1PR_ENOTCONV: return "parareal did not meet the tolerance within max_iter sweeps";
    case L1PR_ENONFINITE: return "non-finite state or parareal increment";
    case L1PR_ESOLVE: return "iterative step solve missed its tolerance";
    case L1PR_EWAIT: return "a bounded device wait gave up; the results of the call are not valid";
  }
  return "unknown status";
}

}  // extern "C"

namespace {

// One group of a heterogeneous batch: the problem it runs as, its members, and whether it
// runs as an uneven batch.
struct BatchGroup {
  l1pr_problem p;
  bool uneven;
  std::vector<int> members;
};

int batch_md(const l1pr_problem& p) { return p.dim == 1 ? p.modes : p.modes * p.modes; }

bool uneven_capable(const l1pr_problem& p) {
  return p.dim == 1 && p.history == 0 && p.solver == 0 && roundup(p.modes, 16) <= 256;
}

// Groups in order of first appearance; members in input order.
std::vector<BatchGroup> batch_groups(const l1pr_problem* probs, int count) {
  std::vector<BatchGroup> g;
  for (int i = 0; i < count; ++i) {
    const l1pr_problem& q = probs[i];
    const bool un = uneven_capable(q);
    int found = -1;
    for (size_t k = 0; k < g.size() && found < 0; ++k) {
      const l1pr_problem& r = probs[g[k].members[0]];
      if (g[k].uneven != un) continue;
      bool same = q.dim == r.dim && q.quad == r.quad && q.slices == r.slices && q.T == r.T &&
                  q.d_sel == r.d_sel && q.d_param == r.d_param && q.f_sel == r.f_sel &&
                  q.history == r.history && q.source_time == r.source_time &&
                  q.assembly == r.assembly && q.tune == r.tune && q.solver == r.solver;
      if (un) same = same && roundup(q.modes, 16) == roundup(r.modes, 16);
      else same = same && q.modes == r.modes && q.steps == r.steps;
      if (same) found = (int)k;
    }
    if (found < 0) {
      BatchGroup ng;
      ng.p = q;
      ng.uneven = un;
      g.push_back(ng);
      found = (int)g.size() - 1;
    }
    BatchGroup& G = g[found];
    G.members.push_back(i);
    if (un) {  // the group runs at its largest modes and steps per slice
      G.p.modes = std::max(G.p.modes, q.modes);
      G.p.steps = std::max(G.p.steps / G.p.slices, q.steps / q.slices) * G.p.slices;
    }
  }
  return g;
}

size_t al256(size_t b) { return (b + 255) / 256 * 256; }

// Workspace of one group: its solver workspace, then the packed inputs and outputs, then the
// uneven per-instance arrays.
struct GroupWs {
  size_t solver, u0p, Up, modes, spp, alpha, total;
};

GroupWs group_ws(const BatchGroup& G, int op) {
  const int B = (int)G.members.size(), Md = batch_md(G.p);
  GroupWs w;
  w.solver = al256(l1pr_workspace_bytes(&G.p, B, op) +
                   (op == L1PR_OP_PARAREAL ? l1pr_parareal_learned_extra_bytes(&G.p, B) : 0));
  w.u0p = w.solver;
  w.Up = w.u0p + al256(sizeof(double) * (size_t)B * Md);
  w.modes = w.Up + al256(sizeof(double) * (size_t)B * (G.p.slices + 1) * Md);
  w.spp = w.modes + al256(sizeof(int32_t) * (size_t)B);
  w.alpha = w.spp + al256(sizeof(int32_t) * (size_t)B);
  w.total = w.alpha + al256(sizeof(double) * (size_t)B);
  return w;
}

}  // namespace

extern "C" {

size_t l1pr_batch_workspace_bytes(const l1pr_problem* probs, int32_t count, int32_t op) {
  if (!probs || count < 0 || (op != L1PR_OP_SERIAL && op != L1PR_OP_PARAREAL)) return 0;
  for (int i = 0; i < count; ++i)
    if (!valid(&probs[i]) || (op == L1PR_OP_PARAREAL && probs[i].history != 0)) return 0;
  size_t mx = 256;
  for (const BatchGroup& G : batch_groups(probs, count)) mx = std::max(mx, group_ws(G, op).total);
  return mx;
}

l1pr_status l1pr_solve_batch(const l1pr_problem* probs, int32_t count, int32_t op, int32_t sweeps,
                             int32_t coarse, const void* mlp_params, int32_t mlp_modes,
                             const double* u0, const int64_t* u0_off, double* U,
                             const int64_t* U_off, void* ws, size_t ws_bytes, void* stream) {
  try {
    if (!probs || count < 0 || (op != L1PR_OP_SERIAL && op != L1PR_OP_PARAREAL) || sweeps < 0)
      return L1PR_EINVAL;
    const bool learned = op == L1PR_OP_PARAREAL && coarse == L1PR_COARSE_LEARNED;
    if (op == L1PR_OP_PARAREAL && coarse != L1PR_COARSE_L1 && !learned) return L1PR_EINVAL;
    if (learned) {
      if (!mlp_params || mlp_modes < 1 || mlp_modes > kMlpMaxModes) return L1PR_EINVAL;
      for (int i = 0; i < count; ++i)
        if (probs[i].dim != 1 || probs[i].modes > mlp_modes) return L1PR_EINVAL;
    }
    if (count == 0) return L1PR_OK;
    if (!u0 || !u0_off || !U || !U_off || !ws) return L1PR_EINVAL;
    for (int i = 0; i < count; ++i)
      if (!valid(&probs[i]) || u0_off[i] < 0 || U_off[i] < 0 ||
          (op == L1PR_OP_PARAREAL && probs[i].history != 0))
        return L1PR_EINVAL;
    const std::vector<BatchGroup> groups = batch_groups(probs, count);
    for (const BatchGroup& G : groups)
      if (group_ws(G, op).total > ws_bytes) return L1PR_ENOMEM;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* base = static_cast<char*>(ws);
    // one status word for the whole call (offset 0, as in every group's workspace)
    L1PR_TRY(launch_fill_int(reinterpret_cast<int*>(base), 1, 0, s));
    struct KeepFlag {
      KeepFlag() { t_keep_flag = true; }
      ~KeepFlag() { t_keep_flag = false; }
    } keep;
    for (const BatchGroup& G : groups) {
      const int B = (int)G.members.size(), Md = batch_md(G.p), P = G.p.slices;
      const GroupWs w = group_ws(G, op);
      double* u0p = reinterpret_cast<double*>(base + w.u0p);
      double* Up = reinterpret_cast<double*>(base + w.Up);
      // gather the initial coefficients, zero above each member's own modes
      L1PR_TRY(launch_fill(u0p, (long)B * Md, 0.0, s));
      std::vector<int32_t> modes(B), spp(B);
      std::vector<double> alpha(B);
      for (int b = 0; b < B; ++b) {
        const l1pr_problem& q = probs[G.members[b]];
        modes[b] = q.modes;
        spp[b] = q.steps / q.slices;
        alpha[b] = q.alpha;
        L1PR_TRY(hipMemcpyAsync(u0p + (long)b * Md, u0 + u0_off[G.members[b]],
                                sizeof(double) * batch_md(q), hipMemcpyDeviceToDevice, s));
      }
      const int k = std::min(sweeps, P);
      l1pr_status st;
      if (G.uneven) {
        int32_t* dm = reinterpret_cast<int32_t*>(base + w.modes);
        int32_t* ds = reinterpret_cast<int32_t*>(base + w.spp);
        double* da = reinterpret_cast<double*>(base + w.alpha);
        // pageable sources: each copy is staged before hipMemcpyAsync returns
        L1PR_TRY(hipMemcpyAsync(dm, modes.data(), sizeof(int32_t) * B, hipMemcpyHostToDevice, s));
        L1PR_TRY(hipMemcpyAsync(ds, spp.data(), sizeof(int32_t) * B, hipMemcpyHostToDevice, s));
        L1PR_TRY(hipMemcpyAsync(da, alpha.data(), sizeof(double) * B, hipMemcpyHostToDevice, s));
        l1pr_uneven desc{dm, ds, da, learned ? L1PR_COARSE_LEARNED : L1PR_COARSE_L1,
                         learned ? mlp_params : nullptr, learned ? mlp_modes : 0};
        st = (op == L1PR_OP_SERIAL)
                 ? l1pr_solve_serial_uneven(&G.p, B, &desc, u0p, Up, base, w.solver, stream)
                 : l1pr_solve_parareal_uneven(&G.p, B, &desc, u0p, Up, k, 0.0, nullptr, nullptr,
                                              nullptr, base, w.solver, stream);
      } else {
        st = (op == L1PR_OP_SERIAL)
                 ? l1pr_solve_serial(&G.p, B, alpha.data(), u0p, Up, nullptr, base, w.solver, stream)
                 : solve_parareal_net(&G.p, B, alpha.data(), u0p, Up, k, 0.0,
                                      learned ? L1PR_COARSE_LEARNED : L1PR_COARSE_L1,
                                      learned ? mlp_params : nullptr, learned ? mlp_modes : 0,
                                      nullptr, nullptr, nullptr, nullptr, base, w.solver, stream);
      }
      if (st != L1PR_OK) return st;
      // scatter each member's slice ends (its own Md columns of every row)
      for (int b = 0; b < B; ++b) {
        const l1pr_problem& q = probs[G.members[b]];
        const size_t mdq = (size_t)batch_md(q);
        L1PR_TRY(hipMemcpy2DAsync(U + U_off[G.members[b]], sizeof(double) * mdq,
                                  Up + (long)b * (P + 1) * Md, sizeof(double) * Md,
                                  sizeof(double) * mdq, P + 1, hipMemcpyDeviceToDevice, s));
      }
    }
    return L1PR_OK;
  } catch (...) {
    return L1PR_EHIP;
  }
}

}  // extern "C"
