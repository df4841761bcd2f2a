// Learned coarse propagator: a residual MLP that corrects the coarse L1 step,
//   G_L,n = G_L1,n + MLP([G_L1,n(C_0..C_n) ; alpha ; n/P]),
// with BF16 weights and activations and FP32 accumulation (MFMA bf16 16x16x16), trained on
// fine trajectories of the solver itself (targets F_n - G_L1,n on serial solutions).
//
// Network: IN = M + 2 inputs (normalised), three hidden layers of 512 with SiLU
// (z / (1 + exp(-z))), OUT = M outputs (normalised residual).  Parameters:
//   params (device, read by inference): per-column normalisation (FP32), biases (FP32),
//           weights (BF16, row-major [out][in], inner dimension padded);
//   state  (device, training only): FP32 master copy of every parameter, Adam moments.
// Every GEMM is a fixed-order reduction, so the network is a deterministic function of its
// input; the parareal correction stays exact.
#include <hip/hip_runtime.h>

#include "l1pr_internal.h"
#include "l1pr_mlp.h"

namespace l1pr {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned short bf16;

__device__ inline bf16 to_bf16(float x) {
  // round to nearest even
  unsigned int u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return (bf16)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (bf16)(u >> 16);
}
__device__ inline float from_bf16(bf16 h) { return __uint_as_float(((unsigned int)h) << 16); }
__device__ inline float silu(float z) { return z / (1.0f + expf(-z)); }
__device__ inline float silu_grad(float z) {
  const float s = 1.0f / (1.0f + expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// ------------------------------------------------------------------ tiled bf16 GEMM
// C[M][N] = sum_k A(i,k) B(k,j):  A(i,k) = AT ? A[k*lda+i] : A[i*lda+k],
//                                   B(k,j) = BT ? B[j*ldb+k] : B[k*ldb+j].
// 64x64 tile per 256-thread work-group (2x2 waves of 2x2 MFMA tiles), K in chunks of 32.
// The operands' leading dimensions and their 16-byte vectors are aligned by the layout
// (multiples of 32 elements, 256-byte aligned arrays).
enum { GE_STORE = 0, GE_BIAS_ACT = 1, GE_BIAS = 2, GE_DACT = 3 };

struct GemmEpi {
  int kind;
  float* c32;          // GE_STORE: C; GE_BIAS_ACT: pre-activation; GE_BIAS: output
  int ldc;
  const float* bias;   // GE_BIAS_ACT, GE_BIAS
  bf16* h;             // GE_BIAS_ACT: activation; GE_DACT: activation gradient (bf16)
  int ldh;
  const float* zsave;  // GE_DACT: saved pre-activation
  int ldz;
};

constexpr int MB = 64, MK = 32;

// With a split reduction (gridDim.z > 1) work-group z sums k in [z kz, (z+1) kz) and stores its
// partial tile (GE_STORE) at ep.c32 + z M ldc; k_sum_partials adds the parts in z order.
// Staging: per 32-wide k chunk each thread moves one 16-byte vector of A and one of B (8
// values along the operand's contiguous dimension) into LDS, A as [i][k] and B as [j][k], so
// each MFMA operand (4 consecutive k) is one 8-byte LDS read; the next chunk's vectors are
// loaded into registers while the current chunk is multiplied.
union V8 {
  uint4 v;
  bf16 h[8];
};

template <bool AT, bool BT>
__global__ __launch_bounds__(256) void k_gemm_bf16(const bf16* A, int lda, const bf16* B, int ldb,
                                                   int M, int N, int K, int kz, GemmEpi ep) {
  __shared__ __align__(16) bf16 sA[MB][MK + 8];
  __shared__ __align__(16) bf16 sB[MB][MK + 8];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  const int i0 = blockIdx.y * MB, j0 = blockIdx.x * MB;
  const int kb0 = blockIdx.z * kz, kb1 = min(K, kb0 + kz);
  if (gridDim.z > 1) ep.c32 += (long)blockIdx.z * M * ep.ldc;
  // this thread's vectors: along k (row ar / column bc) or along i / j (k row ak / bk)
  const int ar = AT ? (tid & 7) * 8 : tid >> 2, ak = AT ? tid >> 3 : (tid & 3) * 8;
  const int bc = BT ? tid >> 2 : (tid & 7) * 8, bk = BT ? (tid & 3) * 8 : tid >> 3;
  V8 va, vb;
  auto load = [&](int k0) {
    if (!AT) {
      const int i = i0 + ar, k = k0 + ak;
      if (i < M && k + 8 <= kb1) va.v = *(const uint4*)(A + (long)i * lda + k);
      else
        for (int e = 0; e < 8; ++e) va.h[e] = (i < M && k + e < kb1) ? A[(long)i * lda + k + e] : (bf16)0;
    } else {
      const int i = i0 + ar, k = k0 + ak;
      if (k < kb1 && i + 8 <= M) va.v = *(const uint4*)(A + (long)k * lda + i);
      else
        for (int e = 0; e < 8; ++e) va.h[e] = (k < kb1 && i + e < M) ? A[(long)k * lda + i + e] : (bf16)0;
    }
    if (BT) {
      const int j = j0 + bc, k = k0 + bk;
      if (j < N && k + 8 <= kb1) vb.v = *(const uint4*)(B + (long)j * ldb + k);
      else
        for (int e = 0; e < 8; ++e) vb.h[e] = (j < N && k + e < kb1) ? B[(long)j * ldb + k + e] : (bf16)0;
    } else {
      const int j = j0 + bc, k = k0 + bk;
      if (k < kb1 && j + 8 <= N) vb.v = *(const uint4*)(B + (long)k * ldb + j);
      else
        for (int e = 0; e < 8; ++e) vb.h[e] = (k < kb1 && j + e < N) ? B[(long)k * ldb + j + e] : (bf16)0;
    }
  };
  f4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
  if (kb0 < kb1) load(kb0);
  for (int k0 = kb0; k0 < kb1; k0 += MK) {
    if (!AT) {
      *(uint4*)&sA[ar][ak] = va.v;
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) sA[ar + e][ak] = va.h[e];
    }
    if (BT) {
      *(uint4*)&sB[bc][bk] = vb.v;
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) sB[bc + e][bk] = vb.h[e];
    }
    __syncthreads();
    if (k0 + MK < kb1) load(k0 + MK);
#pragma unroll
    for (int ks = 0; ks < MK / 16; ++ks) {
      const int kb = ks * 16 + 4 * (lane >> 4);
      s4 af[2], bfr[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) af[a] = *(const s4*)&sA[wi * 32 + a * 16 + (lane & 15)][kb];
#pragma unroll
      for (int b = 0; b < 2; ++b) bfr[b] = *(const s4*)&sB[wj * 32 + b * 16 + (lane & 15)][kb];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[a], bfr[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + wi * 32 + a * 16 + MFMA_BF16_ROW(lane, v);
        const int j = j0 + wj * 32 + b * 16 + (lane & 15);
        if (i >= M || j >= N) continue;
        const float x = acc[a][b][v];
        switch (ep.kind) {
          case GE_STORE: ep.c32[(long)i * ep.ldc + j] = x; break;
          case GE_BIAS_ACT: {
            const float z = x + ep.bias[j];
            ep.c32[(long)i * ep.ldc + j] = z;
            ep.h[(long)i * ep.ldh + j] = to_bf16(silu(z));
            break;
          }
          case GE_BIAS: ep.c32[(long)i * ep.ldc + j] = x + ep.bias[j]; break;
          case GE_DACT:
            ep.h[(long)i * ep.ldh + j] = to_bf16(x * silu_grad(ep.zsave[(long)i * ep.ldz + j]));
            break;
        }
      }
}

hipError_t gemm_bf16(bool at, bool bt, const bf16* A, int lda, const bf16* B, int ldb, int M, int N,
                     int K, const GemmEpi& ep, hipStream_t s, int splits = 1) {
  const int kz = ((K + splits - 1) / splits + MK - 1) / MK * MK;
  dim3 grid((N + MB - 1) / MB, (M + MB - 1) / MB, splits);
  if (!at && !bt) k_gemm_bf16<false, false><<<grid, 256, 0, s>>>(A, lda, B, ldb, M, N, K, kz, ep);
  else if (!at && bt) k_gemm_bf16<false, true><<<grid, 256, 0, s>>>(A, lda, B, ldb, M, N, K, kz, ep);
  else if (at && !bt) k_gemm_bf16<true, false><<<grid, 256, 0, s>>>(A, lda, B, ldb, M, N, K, kz, ep);
  else k_gemm_bf16<true, true><<<grid, 256, 0, s>>>(A, lda, B, ldb, M, N, K, kz, ep);
  return hipGetLastError();
}

// C[i][j] = sum_z P[z][i][j] in z order (the parts of a split reduction)
__global__ void k_sum_partials(const float* P, int parts, long mn, float* C) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= mn) return;
  float t = 0.f;
  for (int z = 0; z < parts; ++z) t += P[z * mn + e];
  C[e] = t;
}

// weight gradient dW[M][N] = A^T B over the batch (K = n rows), split KSPLIT ways over the
// batch so that a few 64 x 64 output tiles still fill the machine
constexpr int KSPLIT = 8;
hipError_t gemm_wgrad(const bf16* A, int lda, const bf16* B, int ldb, int M, int N, int K, float* dW,
                      float* part, hipStream_t s) {
  GemmEpi e{};
  e.kind = GE_STORE;
  e.c32 = part;
  e.ldc = N;
  hipError_t r = gemm_bf16(true, false, A, lda, B, ldb, M, N, K, e, s, KSPLIT);
  if (r != hipSuccess) return r;
  const long mn = (long)M * N;
  k_sum_partials<<<(unsigned)((mn + 255) / 256), 256, 0, s>>>(part, KSPLIT, mn, dW);
  return hipGetLastError();
}

// ------------------------------------------------------------ FP64 inference GEMM
// Y[M][N] = act(X[M][K] W[N][K]^T + b) in FP64: BF16 weights (exact in FP64), FP64
// activations, FP64 sums.  Parareal evaluates the network in this form: its correction
// G_L(U^{k+1}) - G_L(U^k) must shrink with U^{k+1} - U^k down to the solver's tolerance, and
// any rounding of the input or the activations to a shorter format puts a floor under it at
// that format's resolution.
//
// A coarse step carries one row per instance, so the product is skinny (M of tens, K and N
// of hundreds) and latency-bound.  One 16x16 output tile per work-group (FP64 MFMA 16x16x4);
// K is cut into 32-wide chunks, each lane group q of each wave owns one chunk of a 128-wide
// block and loads it with wide loads before the first MFMA, so every load is in flight at
// once; the four waves take interleaved blocks and their partial tiles are added in LDS in
// wave order (a fixed order: the network stays a deterministic function of its input).
// K must be a multiple of 32 (the layout pads every inner dimension to that).
typedef double d4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_gemm_f64_skinny(const double* X, int ldx, const bf16* Wt,
                                                         int ldw, const float* bias, int M, int N,
                                                         int K, int act, double* Y, int ldy) {
  __shared__ double red[4][16][17];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r = lane & 15, q = lane >> 4;
  const int i0 = blockIdx.y * 16, j0 = blockIdx.x * 16;
  const bool xrow = i0 + r < M, wrow = j0 + r < N;
  const double* xp = X + (long)(xrow ? i0 + r : 0) * ldx;
  const bf16* wp = Wt + (long)(wrow ? j0 + r : 0) * ldw;
  const int nchunk = K / 32;
  d4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int blk = w; 4 * blk < nchunk; blk += 4) {
    const int c = 4 * blk + q;
    double xa[32];
    unsigned int wr[16];
    if (c < nchunk && xrow) {
      const double2* px = (const double2*)(xp + c * 32);
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        const double2 v = px[t];
        xa[2 * t] = v.x;
        xa[2 * t + 1] = v.y;
      }
    } else {
#pragma unroll
      for (int t = 0; t < 32; ++t) xa[t] = 0.0;
    }
    if (c < nchunk && wrow) {
      const uint4* pw = (const uint4*)(wp + c * 32);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const uint4 v = pw[t];
        wr[4 * t] = v.x;
        wr[4 * t + 1] = v.y;
        wr[4 * t + 2] = v.z;
        wr[4 * t + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int t = 0; t < 16; ++t) wr[t] = 0u;
    }
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      // element 2t is the low half of word t (little-endian BF16 pairs)
      const double w0 = (double)__uint_as_float(wr[t] << 16);
      const double w1 = (double)__uint_as_float(wr[t] & 0xffff0000u);
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[2 * t], w0, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[2 * t + 1], w1, acc, 0, 0, 0);
    }
  }
  // accumulator element v of lane (r, q) is D[q + 4v][r]
#pragma unroll
  for (int v = 0; v < 4; ++v) red[w][q + 4 * v][r] = acc[v];
  __syncthreads();
  const int ro = threadIdx.x >> 4, co = threadIdx.x & 15;
  const int i = i0 + ro, j = j0 + co;
  if (i < M && j < N) {
    const double z = red[0][ro][co] + red[1][ro][co] + red[2][ro][co] + red[3][ro][co] + (double)bias[j];
    Y[(long)i * ldy + j] = act ? z / (1.0 + exp(-z)) : z;
  }
}

// ---------------------------------------------------------------- layout helpers
MlpLayout mlp_layout(int modes) {
  MlpLayout L{};
  L.in = modes + 2;
  L.out = modes;
  L.hidden = kMlpHidden;
  L.inp = roundup(L.in, MK);
  L.outp = roundup(L.out, 64);
  size_t cur = 0;
  auto take = [&](size_t bytes) {
    const size_t o = cur;
    cur += (bytes + 255) / 256 * 256;
    return o;
  };
  L.in_mean = take(4 * L.inp);
  L.in_std = take(4 * L.inp);
  L.out_mean = take(4 * L.outp);
  L.out_std = take(4 * L.outp);
  L.b[0] = take(4 * L.hidden);
  L.b[1] = take(4 * L.hidden);
  L.b[2] = take(4 * L.hidden);
  L.b[3] = take(4 * L.outp);
  L.w[0] = take(2 * (size_t)L.hidden * L.inp);
  L.w[1] = take(2 * (size_t)L.hidden * L.hidden);
  L.w[2] = take(2 * (size_t)L.hidden * L.hidden);
  L.w[3] = take(2 * (size_t)L.outp * L.hidden);
  L.param_bytes = cur;
  // flat FP32 vector [W1 b1 W2 b2 W3 b3 W4 b4] for masters, gradients and Adam moments
  size_t f = 0;
  L.fw[0] = f; f += (size_t)L.hidden * L.inp;
  L.fb[0] = f; f += L.hidden;
  L.fw[1] = f; f += (size_t)L.hidden * L.hidden;
  L.fb[1] = f; f += L.hidden;
  L.fw[2] = f; f += (size_t)L.hidden * L.hidden;
  L.fb[2] = f; f += L.hidden;
  L.fw[3] = f; f += (size_t)L.outp * L.hidden;
  L.fb[3] = f; f += L.outp;
  L.nflat = f;
  L.state_bytes = 4 * 3 * f;  // masters, m, v
  return L;
}

// ------------------------------------------------------------ elementwise kernels
// X0[i][c] = bf16((x[row(i)][c] - mean[c]) / std[c]) (0 in the padding); rows gathered
// through idx when given.  Tn likewise for targets (FP32).
__global__ void k_gather_norm(const float* x, int ldx, int ncols, const int* idx, int n,
                              const float* mean, const float* sd, bf16* X0, int ldo) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * ldo) return;
  const int i = (int)(e / ldo), c = (int)(e % ldo);
  const long row = idx ? idx[i] : i;
  float v = 0.f;
  if (c < ncols) v = (x[row * ldx + c] - mean[c]) / sd[c];
  X0[e] = to_bf16(v);
}

__global__ void k_gather_norm_f32(const float* x, int ldx, int ncols, const int* idx, int n,
                                  const float* mean, const float* sd, float* out, int ldo) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * ldo) return;
  const int i = (int)(e / ldo), c = (int)(e % ldo);
  const long row = idx ? idx[i] : i;
  out[e] = (c < ncols) ? (x[row * ldx + c] - mean[c]) / sd[c] : 0.f;
}

// dO = 2 (O - Tn) / (n * out) in bf16 and the per-row squared error (for the loss)
__global__ void k_out_grad(const float* O, const float* Tn, int n, int outp, int out, bf16* dO,
                           float* rowloss) {
  const int i = blockIdx.x;
  __shared__ float red[256];
  float acc = 0.f;
  for (int c = threadIdx.x; c < outp; c += blockDim.x) {
    const long e = (long)i * outp + c;
    float g = 0.f;
    if (c < out) {
      const float d = O[e] - Tn[e];
      acc += d * d;
      g = 2.f * d / ((float)n * (float)out);
    }
    dO[e] = to_bf16(g);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) rowloss[i] = red[0];
}

// out[c] = sum_i g[i][c] (bias gradients).  A work-group takes 16 columns; its 16 row groups
// sum the rows i = r, r + 16, ... of each column, and the 16 partials are added in row-group
// order (a fixed order).
__global__ __launch_bounds__(256) void k_colsum_bf16(const bf16* g, int n, int ld, int ncols,
                                                     float* out) {
  __shared__ float red[16][17];
  const int r = threadIdx.x >> 4, cl = threadIdx.x & 15;
  const int c = blockIdx.x * 16 + cl;
  float s = 0.f;
  if (c < ncols)
    for (int i = r; i < n; i += 16) s += from_bf16(g[(long)i * ld + c]);
  red[r][cl] = s;
  __syncthreads();
  if (r == 0 && c < ncols) {
    float t = 0.f;
#pragma unroll
    for (int q = 0; q < 16; ++q) t += red[q][cl];
    out[c] = t;
  }
}

// loss = sum rowloss / (n * out)
__global__ void k_loss(const float* rowloss, int n, int out, float* loss) {
  __shared__ float red[256];
  float s = 0.f;
  for (int i = threadIdx.x; i < n; i += 256) s += rowloss[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = red[0] / ((float)n * (float)out);
}

// Adam on the flat FP32 vector; bias-corrected with step t (1-based)
__global__ void k_adam(float* w, float* m, float* v, const float* g, long n, float lr, int t) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float mm = b1 * m[e] + (1.f - b1) * g[e];
  const float vv = b2 * v[e] + (1.f - b2) * g[e] * g[e];
  m[e] = mm;
  v[e] = vv;
  const float mh = mm / (1.f - powf(b1, (float)t));
  const float vh = vv / (1.f - powf(b2, (float)t));
  w[e] -= lr * mh / (sqrtf(vh) + eps);
}

__global__ void k_cast_bf16(const float* w, long n, bf16* out) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) out[e] = to_bf16(w[e]);
}

__global__ void k_copy_f32(const float* a, long n, float* b) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) b[e] = a[e];
}

__global__ void k_zero_f32(float* a, long n) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) a[e] = 0.f;
}

// Column mean and standard deviation (population) over n rows, one work-group per column,
// fixed-order tree reduction; a column with zero spread gets std = 1.
__global__ void k_colstats(const float* x, int ld, int n, float* mean, float* sd) {
  const int c = blockIdx.x;
  __shared__ double r1[256], r2[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += x[(long)i * ld + c];
  r1[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) r1[threadIdx.x] += r1[threadIdx.x + w];
    __syncthreads();
  }
  const double mu = r1[0] / n;
  double q = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    const double d = x[(long)i * ld + c] - mu;
    q += d * d;
  }
  r2[threadIdx.x] = q;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) r2[threadIdx.x] += r2[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double var = r2[0] / n;
    mean[c] = (float)mu;
    sd[c] = var > 0.0 ? (float)sqrt(var) : 0.0f;  // 0: no spread (set by k_floor_scale)
  }
}

// Input scales: a column with no spread gets 1; the coefficient columns (c < ncoef) are
// floored at frac times the largest coefficient scale, so that inputs that barely vary (modes
// the training states hardly excite) are not magnified into the network: their variation
// between parareal iterates would otherwise move its output far more than the state moves.
__global__ void k_floor_scale(float* sd, int ncoef, int ncols, float frac) {
  __shared__ float red[256];
  float mx = 0.f;
  for (int c = threadIdx.x; c < ncoef; c += 256) mx = fmaxf(mx, sd[c]);
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  const float lo = frac * red[0];
  for (int c = threadIdx.x; c < ncols; c += 256) {
    const float v = sd[c];
    sd[c] = v == 0.f ? 1.f : (c < ncoef ? fmaxf(v, lo) : v);
  }
}

// sd[c] <- sqrt(mean_c sd[c]^2) for every c (fixed-order reduction)
__global__ void k_common_scale(float* sd, int n) {
  __shared__ double red[256];
  double q = 0.0;
  for (int c = threadIdx.x; c < n; c += 256) q += (double)sd[c] * (double)sd[c];
  red[threadIdx.x] = q;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const float v = (float)sqrt(red[0] / n);
  __syncthreads();
  for (int c = threadIdx.x; c < n; c += 256) sd[c] = v > 0.f ? v : 1.f;
}

// Training samples from slice ends Z [B][P+1][Mz] (stride Mz) and coarse values
// G [B][P][Mz]: x = [G_n ; alpha_b ; n/P], t = Z_{n+1} - G_n.
__global__ void k_features(const double* Z, const double* G, const double* alpha, int B, int P,
                           int M, int Mz, float* x, float* t) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int in = M + 2;
  if (e >= (long)B * P * in) return;
  const long s = e / in;
  const int c = (int)(e % in);
  const int b = (int)(s / P), n = (int)(s % P);
  const double* g = G + ((long)b * P + n) * Mz;
  float v;
  if (c < M) v = (float)g[c];
  else if (c == M) v = (float)alpha[b];
  else v = (float)((double)n / (double)P);
  x[s * in + c] = v;
  if (c < M) t[s * M + c] = (float)(Z[((long)b * (P + 1) + n + 1) * Mz + c] - g[c]);
}

// Inference input: x = normalise([G_L1 ; alpha_b ; n/P]) in FP64 for B rows.  The network
// has Mn >= M mode inputs: coefficients of modes the batch does not carry (k >= M) enter as
// zeros, as do the modes above an uneven instance's own count (its G is exactly zero there).
__global__ void k_infer_input(const double* G, long gstride, const double* inst, int B, int M,
                              int Mn, int n, int P, const float* mean, const float* sd, double* X0,
                              int ldo) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)B * ldo) return;
  const int b = (int)(e / ldo), c = (int)(e % ldo);
  double v = 0.0;
  if (c < M) v = G[b * gstride + c];
  else if (c == Mn) v = inst[(long)b * NSCAL + IS_ALPHA];
  else if (c == Mn + 1) v = (double)n / (double)P;
  X0[e] = c < Mn + 2 ? (v - (double)mean[c]) / (double)sd[c] : 0.0;
}

__global__ void k_norm_f64(const double* x, int ldx, int ncols, int n, const float* mean,
                           const float* sd, double* X0, int ldo) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * ldo) return;
  const int i = (int)(e / ldo), c = (int)(e % ldo);
  X0[e] = (c < ncols) ? (x[(long)i * ldx + c] - (double)mean[c]) / (double)sd[c] : 0.0;
}

// G_L = G_L1 + (O * out_std + out_mean) on the unit's own modes (k < M_b, the instance's
// count; the network's outputs for other modes are not used); falls back to G_L1 for a unit
// whose correction is not finite or larger than ||G_L1|| + 1, or whose instance is marked in
// lg_off.  Then the step epilogue; with gp set, the plain value G_L1 is also stored there.
// One work-group per unit.
__global__ __launch_bounds__(256) void k_infer_apply(const double* G, long gstride, const double* O,
                                                     int outp, int M, int Mp, const float* om,
                                                     const float* osd, Epilogue ep,
                                                     const int32_t* done, const double* inst,
                                                     const int32_t* lg_off, double* gp,
                                                     long gpstride) {
  const int u = blockIdx.x;
  if (done && done[u]) return;  // a finished parareal instance keeps its slice ends
  {
    const int mb = (int)inst[(long)u * NSCAL + IS_MB];
    M = mb < M ? mb : M;
  }
  __shared__ double rc[256], rg[256];
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  double sc = 0.0, sg = 0.0;
  for (int k = threadIdx.x; k < M; k += blockDim.x) {
    const double c = O[(long)u * outp + k] * (double)osd[k] + (double)om[k];
    if (!isfinite(c)) atomicOr(&bad, 1);
    sc += c * c;
    const double g = G[u * gstride + k];
    sg += g * g;
  }
  rc[threadIdx.x] = sc;
  rg[threadIdx.x] = sg;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      rc[threadIdx.x] += rc[threadIdx.x + w];
      rg[threadIdx.x] += rg[threadIdx.x + w];
    }
    __syncthreads();
  }
  const bool use = (bad == 0) && isfinite(rc[0]) && sqrt(rc[0]) <= sqrt(rg[0]) + 1.0 &&
                   !(lg_off && lg_off[u]);
  for (int k = threadIdx.x; k < Mp; k += blockDim.x) {
    double x = G[u * gstride + k];
    if (gp) gp[(long)u * gpstride + k] = x;
    if (use && k < M) x = x + (O[(long)u * outp + k] * (double)osd[k] + (double)om[k]);
    if (ep.kind == EPI_CORRECT) {
      const double go = ep.gold[(long)u * ep.gold_stride + k];
      ep.out[(long)u * ep.out_stride + k] = ep.fold[(long)u * ep.fold_stride + k] + (x - go);
      ep.gold[(long)u * ep.gold_stride + k] = x;
    } else {
      ep.out[(long)u * ep.out_stride + k] = x;
      if (ep.kind == EPI_STORE2) ep.gold[(long)u * ep.gold_stride + k] = x;
    }
  }
}

static inline unsigned nblk(long n) { return (unsigned)((n + 255) / 256); }

// workspace for a batch of n rows (train: activations of every layer, gradients)
size_t mlp_ws_bytes(const MlpLayout& L, int n, bool train) {
  size_t b = 0;
  auto add = [&](size_t x) { b += (x + 255) / 256 * 256; };
  add(2 * (size_t)n * L.inp);                       // X0
  for (int l = 0; l < 3; ++l) { add(4 * (size_t)n * L.hidden); add(2 * (size_t)n * L.hidden); }  // Z, H
  add(4 * (size_t)n * L.outp);                      // O
  if (train) {
    add(4 * (size_t)n * L.outp);                    // Tn
    add(2 * (size_t)n * L.outp);                    // dO
    add(2 * (size_t)n * L.hidden);                  // dZ (ping)
    add(2 * (size_t)n * L.hidden);                  // dZ (pong)
    add(4 * L.nflat);                               // gradients
    add(4 * (size_t)n);                             // row losses
    add(4 * (size_t)KSPLIT * L.hidden * (L.hidden > L.inp ? L.hidden : L.inp));  // wgrad parts
  }
  return b;
}

struct MlpWs {
  bf16* X0;
  float* Z[3];
  bf16* H[3];
  float* O;
  float* Tn;
  bf16* dO;
  bf16* dZa;
  bf16* dZb;
  float* grad;
  float* rowloss;
  float* part;
};

MlpWs carve(const MlpLayout& L, int n, bool train, void* ws) {
  char* p = (char*)ws;
  size_t b = 0;
  auto take = [&](size_t x) {
    char* q = p + b;
    b += (x + 255) / 256 * 256;
    return q;
  };
  MlpWs W{};
  W.X0 = (bf16*)take(2 * (size_t)n * L.inp);
  for (int l = 0; l < 3; ++l) {
    W.Z[l] = (float*)take(4 * (size_t)n * L.hidden);
    W.H[l] = (bf16*)take(2 * (size_t)n * L.hidden);
  }
  W.O = (float*)take(4 * (size_t)n * L.outp);
  if (train) {
    W.Tn = (float*)take(4 * (size_t)n * L.outp);
    W.dO = (bf16*)take(2 * (size_t)n * L.outp);
    W.dZa = (bf16*)take(2 * (size_t)n * L.hidden);
    W.dZb = (bf16*)take(2 * (size_t)n * L.hidden);
    W.grad = (float*)take(4 * L.nflat);
    W.rowloss = (float*)take(4 * (size_t)n);
    W.part = (float*)take(4 * (size_t)KSPLIT * L.hidden * (L.hidden > L.inp ? L.hidden : L.inp));
  }
  return W;
}

// FP64 forward from Xf [n][inp] through two ping-pong buffers to O [n][outp]
hipError_t mlp_forward_f64(const MlpLayout& L, const char* params, int n, double* Xf, double* Ha,
                           double* Hb, double* O, hipStream_t s) {
  const double* in = Xf;
  int kin = L.inp;
  double* outs[3] = {Ha, Hb, Ha};
  for (int l = 0; l < 3; ++l) {
    dim3 grid(L.hidden / 16, (n + 15) / 16);
    k_gemm_f64_skinny<<<grid, 256, 0, s>>>(in, kin, (const bf16*)(params + L.w[l]), kin,
                                           (const float*)(params + L.b[l]), n, L.hidden, kin, 1,
                                           outs[l], L.hidden);
    in = outs[l];
    kin = L.hidden;
  }
  dim3 grid(L.outp / 16, (n + 15) / 16);
  k_gemm_f64_skinny<<<grid, 256, 0, s>>>(in, L.hidden, (const bf16*)(params + L.w[3]), L.hidden,
                                         (const float*)(params + L.b[3]), n, L.outp, L.hidden, 0, O,
                                         L.outp);
  return hipGetLastError();
}

// Inference buffers (FP64): input, two hidden, output.
struct InferWs {
  double *X, *Ha, *Hb, *O;
};
static size_t r256(size_t x) { return (x + 255) / 256 * 256; }
size_t mlp_infer_ws_bytes(const MlpLayout& L, int n) {
  return r256(8 * (size_t)n * L.inp) + 2 * r256(8 * (size_t)n * L.hidden) +
         r256(8 * (size_t)n * L.outp);
}
static InferWs carve_infer(const MlpLayout& L, int n, void* ws) {
  char* w = (char*)ws;
  InferWs W;
  W.X = (double*)w;
  W.Ha = (double*)(w + r256(8 * (size_t)n * L.inp));
  W.Hb = (double*)((char*)W.Ha + r256(8 * (size_t)n * L.hidden));
  W.O = (double*)((char*)W.Hb + r256(8 * (size_t)n * L.hidden));
  return W;
}

// forward from X0 (already in the workspace) to O
hipError_t mlp_forward_ws(const MlpLayout& L, const char* params, int n, MlpWs& W, hipStream_t s) {
  const bf16* in = W.X0;
  int ldin = L.inp, kin = L.inp;
  for (int l = 0; l < 3; ++l) {
    GemmEpi e{};
    e.kind = GE_BIAS_ACT;
    e.c32 = W.Z[l];
    e.ldc = L.hidden;
    e.bias = (const float*)(params + L.b[l]);
    e.h = W.H[l];
    e.ldh = L.hidden;
    hipError_t r = gemm_bf16(false, true, in, ldin, (const bf16*)(params + L.w[l]), kin, n,
                             L.hidden, kin, e, s);
    if (r != hipSuccess) return r;
    in = W.H[l];
    ldin = L.hidden;
    kin = L.hidden;
  }
  GemmEpi e{};
  e.kind = GE_BIAS;
  e.c32 = W.O;
  e.ldc = L.outp;
  e.bias = (const float*)(params + L.b[3]);
  return gemm_bf16(false, true, in, ldin, (const bf16*)(params + L.w[3]), L.hidden, n, L.outp,
                   L.hidden, e, s);
}

// learned correction and epilogue for B units whose plain coarse values are in G
hipError_t mlp_coarse_apply(const MlpLayout& L, const void* params, const double* G, long gstride,
                            const double* inst, int B, int M, int Mp, int n, int P,
                            const Epilogue& ep, void* ws, hipStream_t s, const int32_t* done,
                            const int32_t* lg_off, double* gp, long gpstride) {
  if (M > L.out) return hipErrorInvalidValue;  // the network covers at least the batch's modes
  const char* pp = (const char*)params;
  const InferWs W = carve_infer(L, B, ws);
  k_infer_input<<<nblk((long)B * L.inp), 256, 0, s>>>(G, gstride, inst, B, M, L.out, n, P,
                                                       (const float*)(pp + L.in_mean),
                                                       (const float*)(pp + L.in_std), W.X, L.inp);
  hipError_t r = mlp_forward_f64(L, pp, B, W.X, W.Ha, W.Hb, W.O, s);
  if (r != hipSuccess) return r;
  k_infer_apply<<<B, 256, 0, s>>>(G, gstride, W.O, L.outp, M, Mp, (const float*)(pp + L.out_mean),
                                  (const float*)(pp + L.out_std), ep, done, inst, lg_off, gp,
                                  gpstride);
  return hipGetLastError();
}

}  // namespace l1pr

using namespace l1pr;

extern "C" {

l1pr_status l1pr_mlp_layout(int32_t modes, l1pr_mlp_info* info) {
  if (modes < 1 || modes > kMlpMaxModes || !info) return L1PR_EINVAL;
  const MlpLayout L = mlp_layout(modes);
  info->in = L.in;
  info->in_padded = L.inp;
  info->hidden = L.hidden;
  info->out = L.out;
  info->out_padded = L.outp;
  info->param_bytes = L.param_bytes;
  info->state_bytes = L.state_bytes;
  info->flat_count = (int64_t)L.nflat;
  info->off_in_mean = L.in_mean;
  info->off_in_std = L.in_std;
  info->off_out_mean = L.out_mean;
  info->off_out_std = L.out_std;
  for (int l = 0; l < 4; ++l) {
    info->off_w[l] = L.w[l];
    info->off_b[l] = L.b[l];
    info->flat_w[l] = (int64_t)L.fw[l];
    info->flat_b[l] = (int64_t)L.fb[l];
  }
  return L1PR_OK;
}

size_t l1pr_mlp_workspace_bytes(int32_t modes, int32_t n, int32_t train) {
  if (modes < 1 || modes > kMlpMaxModes || n < 1) return 0;
  return mlp_ws_bytes(mlp_layout(modes), n, train != 0);
}

l1pr_status l1pr_mlp_sync(int32_t modes, const void* state, void* params, void* stream) {
  if (modes < 1 || modes > kMlpMaxModes || !state || !params) return L1PR_EINVAL;
  const MlpLayout L = mlp_layout(modes);
  hipStream_t s = (hipStream_t)stream;
  const float* w = (const float*)state;
  char* p = (char*)params;
  const long nw[4] = {(long)L.hidden * L.inp, (long)L.hidden * L.hidden, (long)L.hidden * L.hidden,
                      (long)L.outp * L.hidden};
  const long nb[4] = {L.hidden, L.hidden, L.hidden, L.outp};
  for (int l = 0; l < 4; ++l) {
    k_cast_bf16<<<nblk(nw[l]), 256, 0, s>>>(w + L.fw[l], nw[l], (bf16*)(p + L.w[l]));
    k_copy_f32<<<nblk(nb[l]), 256, 0, s>>>(w + L.fb[l], nb[l], (float*)(p + L.b[l]));
  }
  return hipGetLastError() == hipSuccess ? L1PR_OK : L1PR_EHIP;
}

l1pr_status l1pr_mlp_reset_moments(int32_t modes, void* state, void* stream) {
  if (modes < 1 || modes > kMlpMaxModes || !state) return L1PR_EINVAL;
  const MlpLayout L = mlp_layout(modes);
  float* f = (float*)state;
  k_zero_f32<<<nblk(2 * (long)L.nflat), 256, 0, (hipStream_t)stream>>>(f + L.nflat, 2 * (long)L.nflat);
  return hipGetLastError() == hipSuccess ? L1PR_OK : L1PR_EHIP;
}

l1pr_status l1pr_mlp_stats(int32_t modes, const float* x, const float* t, int64_t n, void* params,
                           void* stream) {
  if (modes < 1 || modes > kMlpMaxModes || !x || !t || n < 1 || !params) return L1PR_EINVAL;
  const MlpLayout L = mlp_layout(modes);
  char* p = (char*)params;
  hipStream_t s = (hipStream_t)stream;
  k_colstats<<<L.in, 256, 0, s>>>(x, L.in, (int)n, (float*)(p + L.in_mean), (float*)(p + L.in_std));
  k_floor_scale<<<1, 256, 0, s>>>((float*)(p + L.in_std), modes, L.in, 1e-4f);
  k_colstats<<<L.out, 256, 0, s>>>(t, L.out, (int)n, (float*)(p + L.out_mean), (float*)(p + L.out_std));
  // one output scale for every mode: the root mean square of the per-mode deviations, so the
  // loss weighs each mode by its absolute contribution to the error of the state
  k_common_scale<<<1, 256, 0, s>>>((float*)(p + L.out_std), L.out);
  return hipGetLastError() == hipSuccess ? L1PR_OK : L1PR_EHIP;
}

l1pr_status l1pr_mlp_forward(int32_t modes, const void* params, const float* x, int32_t n,
                             float* y, void* ws, size_t ws_bytes, void* stream) {
  if (modes < 1 || modes > kMlpMaxModes || !params || ((uintptr_t)params & 255) || !x || !y ||
      n < 1 || !ws)
    return L1PR_EINVAL;
  const MlpLayout L = mlp_layout(modes);
  if (ws_bytes < mlp_ws_bytes(L, n, false)) return L1PR_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  const char* p = (const char*)params;
  MlpWs W = carve(L, n, false, ws);
  k_gather_norm<<<nblk((long)n * L.inp), 256, 0, s>>>(x, L.in, L.in, nullptr, n,
                                                      (const float*)(p + L.in_mean),
                                                      (const float*)(p + L.in_std), W.X0, L.inp);
  if (mlp_forward_ws(L, p, n, W, s) != hipSuccess) return L1PR_EHIP;
  // y = O (normalised output), first `out` columns
  GemmEpi e{};  // unused
  (void)e;
  hipError_t r = hipMemcpy2DAsync(y, sizeof(float) * L.out, W.O, sizeof(float) * L.outp,
                                  sizeof(float) * L.out, n, hipMemcpyDeviceToDevice, s);
  return r == hipSuccess ? L1PR_OK : L1PR_EHIP;
}

l1pr_status l1pr_mlp_infer(int32_t modes, const void* params, const double* x, int32_t n, double* y,
                           void* ws, size_t ws_bytes, void* stream) {
  if (modes < 1 || modes > kMlpMaxModes || !params || ((uintptr_t)params & 255) || !x || !y ||
      n < 1 || !ws)
    return L1PR_EINVAL;
  const MlpLayout L = mlp_layout(modes);
  if (ws_bytes < mlp_infer_ws_bytes(L, n)) return L1PR_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  const char* p = (const char*)params;
  const InferWs W = carve_infer(L, n, ws);
  k_norm_f64<<<nblk((long)n * L.inp), 256, 0, s>>>(x, L.in, L.in, n, (const float*)(p + L.in_mean),
                                                   (const float*)(p + L.in_std), W.X, L.inp);
  if (mlp_forward_f64(L, p, n, W.X, W.Ha, W.Hb, W.O, s) != hipSuccess) return L1PR_EHIP;
  hipError_t r = hipMemcpy2DAsync(y, sizeof(double) * L.out, W.O, sizeof(double) * L.outp,
                                  sizeof(double) * L.out, n, hipMemcpyDeviceToDevice, s);
  return r == hipSuccess ? L1PR_OK : L1PR_EHIP;
}

size_t l1pr_mlp_infer_workspace_bytes(int32_t modes, int32_t n) {
  if (modes < 1 || modes > kMlpMaxModes || n < 1) return 0;
  return mlp_infer_ws_bytes(mlp_layout(modes), n);
}

l1pr_status l1pr_mlp_train_step(int32_t modes, void* params, void* state, const float* x,
                                const float* t, const int32_t* idx, int32_t n, float lr,
                                int32_t step, float* loss, float* grad_out, void* ws,
                                size_t ws_bytes, void* stream) {
  if (modes < 1 || modes > kMlpMaxModes || !params || !state || !x || !t || n < 1 || !ws ||
      step < 1 || !(lr >= 0.f))
    return L1PR_EINVAL;
  const MlpLayout L = mlp_layout(modes);
  if (ws_bytes < mlp_ws_bytes(L, n, true)) return L1PR_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  char* p = (char*)params;
  MlpWs W = carve(L, n, true, ws);
  k_gather_norm<<<nblk((long)n * L.inp), 256, 0, s>>>(x, L.in, L.in, idx, n,
                                                      (const float*)(p + L.in_mean),
                                                      (const float*)(p + L.in_std), W.X0, L.inp);
  k_gather_norm_f32<<<nblk((long)n * L.outp), 256, 0, s>>>(t, L.out, L.out, idx, n,
                                                           (const float*)(p + L.out_mean),
                                                           (const float*)(p + L.out_std), W.Tn,
                                                           L.outp);
  if (mlp_forward_ws(L, p, n, W, s) != hipSuccess) return L1PR_EHIP;
  k_out_grad<<<n, 256, 0, s>>>(W.O, W.Tn, n, L.outp, L.out, W.dO, W.rowloss);
  if (loss) k_loss<<<1, 256, 0, s>>>(W.rowloss, n, L.out, loss);
  // layer 4: dW4 = dO^T H3, db4 = colsum dO, dZ3 = (dO W4) * silu'(Z3)
  {
    if (gemm_wgrad(W.dO, L.outp, W.H[2], L.hidden, L.outp, L.hidden, n, W.grad + L.fw[3], W.part,
                   s) != hipSuccess)
      return L1PR_EHIP;
    k_colsum_bf16<<<(L.outp + 15) / 16, 256, 0, s>>>(W.dO, n, L.outp, L.outp, W.grad + L.fb[3]);
    GemmEpi d{};
    d.kind = GE_DACT;
    d.h = W.dZa;
    d.ldh = L.hidden;
    d.zsave = W.Z[2];
    d.ldz = L.hidden;
    if (gemm_bf16(false, false, W.dO, L.outp, (const bf16*)(p + L.w[3]), L.hidden, n, L.hidden,
                  L.outp, d, s) != hipSuccess)
      return L1PR_EHIP;
  }
  // hidden layers 3, 2, 1
  bf16* dz = W.dZa;
  bf16* dzn = W.dZb;
  for (int l = 2; l >= 0; --l) {
    const bf16* hin = (l == 0) ? W.X0 : W.H[l - 1];
    const int kin = (l == 0) ? L.inp : L.hidden;
    if (gemm_wgrad(dz, L.hidden, hin, kin, L.hidden, kin, n, W.grad + L.fw[l], W.part, s) !=
        hipSuccess)
      return L1PR_EHIP;
    k_colsum_bf16<<<(L.hidden + 15) / 16, 256, 0, s>>>(dz, n, L.hidden, L.hidden, W.grad + L.fb[l]);
    if (l > 0) {
      GemmEpi d{};
      d.kind = GE_DACT;
      d.h = dzn;
      d.ldh = L.hidden;
      d.zsave = W.Z[l - 1];
      d.ldz = L.hidden;
      if (gemm_bf16(false, false, dz, L.hidden, (const bf16*)(p + L.w[l]), L.hidden, n, L.hidden,
                    L.hidden, d, s) != hipSuccess)
        return L1PR_EHIP;
      bf16* tmp = dz;
      dz = dzn;
      dzn = tmp;
    }
  }
  if (grad_out)
    k_copy_f32<<<nblk((long)L.nflat), 256, 0, s>>>(W.grad, (long)L.nflat, grad_out);
  float* w = (float*)state;
  k_adam<<<nblk((long)L.nflat), 256, 0, s>>>(w, w + L.nflat, w + 2 * L.nflat, W.grad, (long)L.nflat,
                                             lr, step);
  return l1pr_mlp_sync(modes, state, params, stream);
}

l1pr_status l1pr_mlp_features(int32_t modes, int32_t batch, int32_t slices, const double* alpha,
                              const double* Z, const double* G, float* x, float* t,
                              void* stream) {
  if (modes < 1 || batch < 1 || slices < 1 || !alpha || !Z || !G || !x || !t) return L1PR_EINVAL;
  const long total = (long)batch * slices * (modes + 2);
  k_features<<<nblk(total), 256, 0, (hipStream_t)stream>>>(Z, G, alpha, batch, slices, modes, modes,
                                                           x, t);
  return hipGetLastError() == hipSuccess ? L1PR_OK : L1PR_EHIP;
}

}  // extern "C"
