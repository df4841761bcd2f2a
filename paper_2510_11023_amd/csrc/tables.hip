// Tables of the method, computed on the device once per call:
//   - Gauss-Legendre nodes and weights on (0,1) (padded with zero-weight nodes);
//   - sine basis values and derivatives at the nodes, phi, phiT and dphi;
//   - per instance: alpha, tau = dt^a Gamma(2-a), tau_c = dT^a Gamma(2-a), S^-a,
//     Gamma(1+a), Gamma(3-a), the L1 weights b_j (L1 scheme, Section 2.1) and the hybrid
//     weights b_{m+r/S} of the fine operator (Section 2.2).
#include "l1pr_internal.h"

namespace l1pr {

// One thread per node.  The i-th root of the Legendre polynomial P_Q (descending in i on
// (-1,1)) is refined by Newton steps on the three-term recurrence, starting from the
// classical cosine estimate; the node maps to x = (1 - z)/2 so nodes ascend on (0,1).
__global__ void k_gauss_legendre(int Q, int Qp, double* xq, double* wq) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Qp) return;
  if (i >= Q) {  // padding node: weight 0
    xq[i] = 0.5;
    wq[i] = 0.0;
    return;
  }
  double z = cos(kPi * (4.0 * i + 3.0) / (4.0 * Q + 2.0));
  double deriv = 1.0;
  for (int it = 0; it < 12; ++it) {
    // P_0 = 1, P_1 = z, (j) P_j = (2j-1) z P_{j-1} - (j-1) P_{j-2}
    double pm = 1.0, pc = z;
    for (int j = 2; j <= Q; ++j) {
      const double pn = ((2 * j - 1) * z * pc - (j - 1) * pm) / j;
      pm = pc;
      pc = pn;
    }
    deriv = Q * (pm - z * pc) / (1.0 - z * z);
    z -= pc / deriv;
  }
  double pm = 1.0, pc = z;
  for (int j = 2; j <= Q; ++j) {
    const double pn = ((2 * j - 1) * z * pc - (j - 1) * pm) / j;
    pm = pc;
    pc = pn;
  }
  deriv = Q * (pm - z * pc) / (1.0 - z * z);
  xq[i] = 0.5 * (1.0 - z);
  wq[i] = 1.0 / ((1.0 - z * z) * deriv * deriv);
}

// phi[q][k] = sqrt2 sin((k+1) pi x_q), dphi[q][k] = sqrt2 (k+1) pi cos((k+1) pi x_q) (when
// dphi is set), zero outside k < M, q < Q.  When b12 is set (2D), also the stacked tables of the
// separable stiffness products: b12 [Mp][2 Qp] = [phi^T | dphi^T], s2 [2 Qp][Mp] = [dphi; phi].
__global__ void k_basis(int M, int Q, int Mp, int Qp, const double* xq, double* phi,
                        double* phiT, double* dphi, double* b12, double* s2) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)Qp * Mp) return;
  const int q = (int)(idx / Mp), k = (int)(idx % Mp);
  double v = 0.0, dv = 0.0;
  if (k < M && q < Q) {
    const double kp = (k + 1) * kPi;
    const double arg = kp * xq[q];
    v = sqrt(2.0) * sin(arg);
    dv = sqrt(2.0) * kp * cos(arg);
  }
  phi[(long)q * Mp + k] = v;
  phiT[(long)k * Qp + q] = v;
  if (dphi) dphi[(long)q * Mp + k] = dv;
  if (b12) {
    b12[(long)k * 2 * Qp + q] = v;
    b12[(long)k * 2 * Qp + Qp + q] = dv;
    s2[(long)q * Mp + k] = dv;
    s2[(long)(Qp + q) * Mp + k] = v;
  }
}

// cosq[q][j] = cos(j pi x_q), j = 0..Jp-1 (cosine moments of the stiffness)
__global__ void k_cosq(int Q, int Qp, int Jp, const double* xq, double* cosq) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)Qp * Jp) return;
  const int q = (int)(idx / Jp), j = (int)(idx % Jp);
  cosq[idx] = (q < Q) ? cos((j * kPi) * xq[q]) : 0.0;
}

// Per-instance scalars.  Mb, Sb (nullable): the instance's own modes and fine steps per
// slice in an uneven batch (entries outside 1..M, 1..S are clamped); its number of fine
// steps is P Sb.
__global__ void k_inst_scalars(int B, int M, int P, int S, double T, const double* alpha,
                               const int32_t* Mb, const int32_t* Sb, double* inst) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const double a = alpha[b];
  const int m = Mb ? min(max(Mb[b], 1), M) : M;
  const int sb = Sb ? min(max(Sb[b], 1), S) : S;
  const double g2 = tgamma(2.0 - a);
  double* o = inst + (long)b * NSCAL;
  o[IS_ALPHA] = a;
  o[IS_TAU] = pow(T / (double)((long)P * sb), a) * g2;
  o[IS_TAUC] = pow(T / (double)P, a) * g2;
  o[IS_SFAC] = pow((double)sb, -a);
  o[IS_G1A] = tgamma(1.0 + a);
  o[IS_G3A] = tgamma(3.0 - a);
  o[IS_MB] = (double)m;
  o[IS_SB] = (double)sb;
}

// bw[b][j] = b_j for j < LB
__global__ void k_weights(int B, int LB, const double* alpha, double* bw) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)B * LB) return;
  const int b = (int)(idx / LB), j = (int)(idx % LB);
  bw[idx] = l1_weight((double)j, alpha[b]);
}

// bhyb[b][m*S + r-1] = b_{m + r/Sb}, m < P, 1 <= r <= Sb (the instance's own steps per
// slice, from inst), with m + r/Sb formed as (m Sb + r)/Sb; entries r > Sb are unused (0).
__global__ void k_hybrid_weights(int B, int P, int S, const double* alpha, const double* inst,
                                 double* bhyb) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long per = (long)P * S;
  if (idx >= (long)B * per) return;
  const int b = (int)(idx / per);
  const long rem = idx % per;
  const int m = (int)(rem / S), r = (int)(rem % S) + 1;
  const int sb = (int)inst[(long)b * NSCAL + IS_SB];
  if (r > sb) {
    bhyb[idx] = 0.0;
    return;
  }
  const double x = (double)((long)m * sb + r) / (double)sb;
  bhyb[idx] = l1_weight(x, alpha[b]);
}

__global__ void k_fill(double* x, long n, double v) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

// A[u] = I for `units` matrices of order n (grid-stride)
__global__ void k_identity(double* A, long total, int n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
    const long e = i % ((long)n * n);
    A[i] = (e / n == e % n) ? 1.0 : 0.0;
  }
}

hipError_t launch_identity(double* A, int units, int n, hipStream_t s) {
  const long total = (long)units * n * n;
  if (total > 0) k_identity<<<4096, 256, 0, s>>>(A, total, n);
  return hipGetLastError();
}

hipError_t launch_fill(double* x, long n, double v, hipStream_t s) {
  if (n > 0) k_fill<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(x, n, v);
  return hipGetLastError();
}

hipError_t launch_tables(const Tables& tb, double* xq, double* wq, double* phi, double* phiT,
                         double* dphi, double* inst, double* bw, double* bhyb, double* cosq,
                         const double* alpha_dev, const int32_t* Mb, const int32_t* Sb,
                         hipStream_t s, double* b12, double* s2) {
  const int T = 256;
  k_gauss_legendre<<<(tb.Qp + T - 1) / T, T, 0, s>>>(tb.Q, tb.Qp, xq, wq);
  // basis tables per direction: M1 modes padded to M1p (M1 = M in 1D)
  const long nb = (long)tb.Qp * tb.M1p;
  k_basis<<<(unsigned)((nb + T - 1) / T), T, 0, s>>>(tb.M1, tb.Q, tb.M1p, tb.Qp, xq, phi, phiT, dphi,
                                                    b12, s2);
  if (cosq) {
    const long nc = (long)tb.Qp * (2 * tb.M1p + 1);
    k_cosq<<<(unsigned)((nc + T - 1) / T), T, 0, s>>>(tb.Q, tb.Qp, 2 * tb.M1p + 1, xq, cosq);
  }
  k_inst_scalars<<<(tb.B + T - 1) / T, T, 0, s>>>(tb.B, tb.M, tb.P, tb.S, tb.T, alpha_dev, Mb, Sb, inst);
  const long nw = (long)tb.B * tb.LB;
  k_weights<<<(unsigned)((nw + T - 1) / T), T, 0, s>>>(tb.B, tb.LB, alpha_dev, bw);
  const long nh = (long)tb.B * tb.P * tb.S;
  if (bhyb && nh > 0)
    k_hybrid_weights<<<(unsigned)((nh + T - 1) / T), T, 0, s>>>(tb.B, tb.P, tb.S, alpha_dev, inst, bhyb);
  return hipGetLastError();
}

}  // namespace l1pr
