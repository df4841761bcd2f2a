// Serial solve without any allocation, for callers that cannot allocate device memory (code
// under HIP graph capture, serving loops, harnesses that forbid hipMalloc).
//
// The workspace of l1pr_solve_serial is taken from a file-scope device array of
// L1PR_NOALLOC_SCRATCH_BYTES instead of a caller buffer.  Each device holds its own copy of
// the array for the life of the process.  Host code never uses the array's name as an
// address: at a device's first call its address is looked up once with
// hipGetSymbolAddress (with that device current) and kept per device.
//
// Every call on one device shares that device's array, so calls that overlap on one device
// (two streams, two threads) race.  Nothing in it has to start at zero: the serial solve
// writes every workspace entry it reads (its tables, the packed initial state, the per-step
// buffers) before reading it, exactly as it does with an uninitialised caller workspace.
#include <hip/hip_runtime.h>

#include <mutex>

#include "l1pr.h"

namespace {

__device__ __align__(256) unsigned char scratch[L1PR_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;

// Device address of `scratch` on the current device, looked up once per device.
void* scratch_address() {
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    addr[dev] = p;
  }
  return addr[dev];
}

}  // namespace

extern "C" l1pr_status l1pr_solve_serial_noalloc(const l1pr_problem* p, int32_t batch,
                                                 const double* alpha, const double* u0,
                                                 double* U, double* traj, void* stream) {
  try {
    if (!p || !u0 || !U || batch < 1) return L1PR_EINVAL;
    const size_t need = l1pr_workspace_bytes(p, batch, L1PR_OP_SERIAL);
    if (need == 0) return L1PR_EINVAL;
    if (need > (size_t)L1PR_NOALLOC_SCRATCH_BYTES) return L1PR_ENOMEM;
    void* ws = scratch_address();
    if (!ws) return L1PR_EHIP;
    return l1pr_solve_serial(p, batch, alpha, u0, U, traj, ws, (size_t)L1PR_NOALLOC_SCRATCH_BYTES,
                             stream);
  } catch (...) {
    return L1PR_EHIP;
  }
}
