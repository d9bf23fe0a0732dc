// Error bounds without any device allocation, for callers that cannot call
// hipMalloc. The residual kernel's block partials and sums live in `scratch`,
// a fixed array in the library's code object: every device the library runs
// on holds its own copy until the process ends. Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the
// symbol); it looks up each device's address once, with that device current,
// and uses that address everywhere.

#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "bounds.hpp"
#include "condest.h"
#include "internal.hpp"
#include "kernels.hpp"

using namespace condest;

namespace {

// three sets of block partials (r.r, x.x, b.b) of at most kMaxParts blocks,
// then the three sums
constexpr int kScratchDoubles = 4 * kMaxParts;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Address of `scratch` on the current device, looked up on the first call
// on that device.
int scratch_on_current_device(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(COND_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(COND_EINVAL, "device index beyond 64");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(COND_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return COND_OK;
}

}  // namespace

extern "C" int cond_error_bounds_noalloc(int32_t n, int64_t nnz, const int64_t* rowptr,
                                         const int32_t* col, const double* val,
                                         const double* x_hat, const double* b, double kappa,
                                         double norm_a, void* stream, cond_bounds_t* out) {
  if (!rowptr || !col || !val || !x_hat || !b || !out) return fail(COND_EINVAL, "null argument");
  if (n < 1 || nnz < 0) return fail(COND_EINVAL, "n must be >= 1 and nnz >= 0");
  if (!(kappa >= 1.0) || !std::isfinite(kappa) || !(norm_a > 0.0) || !std::isfinite(norm_a))
    return fail(COND_EINVAL, "kappa must be >= 1 and norm_a > 0, both finite");
  const int grid = grid_for(n);
  if (grid > kMaxParts)  // grid_for caps the grid; the scratch holds one slot per block
    return fail(COND_EINVAL, "launch needs more partial slots than the scratch holds");
  double* scr = nullptr;
  int st = scratch_on_current_device(&scr);
  if (st) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  launch_residual(n, rowptr, 1, col, val, x_hat, b, scr, scr + 3 * kMaxParts, grid, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(COND_EHIP, std::string("residual launch: ") + hipGetErrorString(e));
  double sums[3];
  e = hipMemcpyAsync(sums, scr + 3 * kMaxParts, sizeof(sums), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(COND_EHIP, std::string("residual sums: ") + hipGetErrorString(e));
  if ((st = fill_bounds(sums, kappa, norm_a, out))) return fail(st, "zero or non-finite norm");
  return COND_OK;
}
