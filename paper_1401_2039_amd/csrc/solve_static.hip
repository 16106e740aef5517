// qiral_solve_static: qiral_solve for callers that cannot allocate device
// memory.  Its workspace is a fixed array in the library's device data, one
// copy per GPU, held from the library's load until the process ends.
#include <hip/hip_runtime.h>
#include <mutex>

#include "qiral_int.h"

using namespace qiral;

namespace {

// The workspace of every qiral_solve_static call on a GPU.  In host code this
// name stands for the array and is not a device address: kernels and copies
// get the address hipGetSymbolAddress returns for the current device.
__device__ __align__(256) unsigned char scratch[QIRAL_STATIC_WORKSPACE_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void *g_scratch[MAX_DEVICES] = {};

// The device address of `scratch` on the current device (looked up once per device).
qiral_status scratch_address(int dev, void **out) {
  if (dev < 0 || dev >= MAX_DEVICES) {
    set_error("qiral_solve_static: device index beyond 63");
    return QIRAL_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p || ((uintptr_t)p & 255) != 0) {
      set_error("qiral_solve_static: the static workspace is not 256-byte aligned");
      return QIRAL_ERR_HIP;
    }
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return QIRAL_OK;
}

}  // namespace

extern "C" qiral_status qiral_solve_static(qiral_lattice *lat, double *x_canon, const double *b_canon, int32_t nrhs,
                                           const qiral_solve_params *params, qiral_solve_info *info,
                                           qiral_stream_t stream) {
  qiral_status st = check_solve_args(lat, x_canon, b_canon, nrhs, params, info);
  if (st != QIRAL_OK) return st;
  if ((st = check_solve_links(lat, params)) != QIRAL_OK) return st;
  if (params->use_graph) {
    set_error("qiral_solve_static runs without a HIP graph (instantiating one allocates)");
    return QIRAL_ERR_UNSUPPORTED;
  }
  const size_t need = qiral_solve_workspace_bytes(lat, params, nrhs);
  if (need == 0 || need > QIRAL_STATIC_WORKSPACE_BYTES) {
    set_error("qiral_solve_static: the solve needs more workspace than the static 32 MiB "
              "(qiral_solve_workspace_bytes); use qiral_solve with a caller workspace");
    return QIRAL_ERR_WORKSPACE;
  }
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != lat->device) {
    set_error("qiral_solve_static: the current device is not the lattice's");
    return QIRAL_ERR_INVALID_ARG;
  }
  void *ws = nullptr;
  if ((st = scratch_address(dev, &ws)) != QIRAL_OK) return st;
  return solve_in(lat, x_canon, b_canon, nrhs, params, ws, QIRAL_STATIC_WORKSPACE_BYTES, info, (hipStream_t)stream);
}
