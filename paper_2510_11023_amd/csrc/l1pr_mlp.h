// Internal layout of the learned coarse propagator's parameters (see mlp.hip).
#pragma once
#include <stddef.h>
#include <stdint.h>

#include "l1pr.h"

namespace l1pr {

constexpr int kMlpHidden = 512;
constexpr int kMlpMaxModes = 256;

// FP32 accumulator of MFMA f32_16x16x16_bf16: lane l, element v holds row 4 (l / 16) + v,
// column l % 16.
#define MFMA_BF16_ROW(lane, v) (4 * ((lane) >> 4) + (v))

struct MlpLayout {
  int in, out, hidden, inp, outp;
  size_t in_mean, in_std, out_mean, out_std;  // byte offsets in params (FP32 arrays)
  size_t b[4];                                // byte offsets of the FP32 biases
  size_t w[4];                                // byte offsets of the BF16 weights [out][in]
  size_t param_bytes;
  size_t fw[4], fb[4];                        // element offsets in the flat FP32 vector
  size_t nflat;
  size_t state_bytes;                         // masters, first and second moments
};

MlpLayout mlp_layout(int modes);
size_t mlp_ws_bytes(const MlpLayout& L, int n, bool train);
size_t mlp_infer_ws_bytes(const MlpLayout& L, int n);
struct Epilogue;
hipError_t mlp_coarse_apply(const MlpLayout& L, const void* params, const double* G, long gstride,
                            const double* inst, int B, int M, int Mp, int n, int P,
                            const Epilogue& ep, void* ws, hipStream_t s,
                            const int32_t* done = nullptr, const int32_t* lg_off = nullptr,
                            double* gp = nullptr, long gpstride = 0);

}  // namespace l1pr
