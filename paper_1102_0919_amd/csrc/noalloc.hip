// The Gram product of slamg_op_gram for callers that cannot allocate device memory: its
// per-workgroup partial sums live in a fixed device array instead of a hipMalloc'd buffer.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/slamg_ops.h"
#include "common.h"

using namespace slamg;

namespace {

// Partial sums of the reduction (one 16 x 16 slot per workgroup, GRAM_MAX_GRID workgroups at
// most).  Every GPU holds its own copy until the process ends.  In host code this name is not a
// device address: kernels get the address from hipGetSymbolAddress (scratch_ptr below).
constexpr size_t SCRATCH_DOUBLES = PARTIAL_DOUBLES;
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
double* g_ptr[MAX_DEVICES] = {};

// The current device's scratch address, looked up once per device with that device current.
hipError_t scratch_ptr(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" size_t slamg_op_gram_noalloc_scratch_bytes(void) { return SCRATCH_DOUBLES * sizeof(double); }

extern "C" slamg_status slamg_op_gram_noalloc(int32_t rows, int32_t w, const double* d_x, const double* d_y,
                                              double* d_g, void* stream) {
  if (rows < 0 || w < 1 || w > 16 || !d_x || !d_y || !d_g) return SLAMG_E_INVALID;
  // one 256-double slot per workgroup of the reduction
  const size_t need = (size_t)gram_grid(rows) * 256;
  if (need > SCRATCH_DOUBLES) return SLAMG_E_BUDGET;
  double* part = nullptr;
  if (scratch_ptr(&part) != hipSuccess) {
    (void)hipGetLastError();
    return SLAMG_E_DEVICE;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  launch_gram(rows, w, d_x, d_y, part, d_g, s);
  if (hipGetLastError() != hipSuccess) return SLAMG_E_DEVICE;
  return SLAMG_OK;
}
