// hard_hydro_step_noalloc: hard_hydro_step with the workspace taken from a
// file-scope device array instead of a caller buffer, for callers that
// cannot allocate device memory.
//
// The array `scratch` below exists once per GPU that loads the library and
// lives until the process ends.  In host code its name only stands for the
// symbol; the device address of each GPU's copy comes from
// hipGetSymbolAddress, taken once per device with that device current, and
// only that address is ever handed to kernels.  The control block at the
// start of the array is cleared by a fill kernel at every call (no memset
// node, so the call stays capturable); calls that overlap on one GPU share
// the array and race.

#include <mutex>

#include "../../include/hard.h"
#include "api_internal.hpp"
#include "hydro_device.hpp"
#include "launch.hpp"

namespace hard {

static __device__ __align__(256) unsigned char scratch[HARD_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of scratch per device (null: not taken yet)

// Device address of the current device's scratch array.
hard_status_t scratch_of_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hard_hydro_step_noalloc: hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices)
    return fail(HARD_ERR_UNSUPPORTED, "hard_hydro_step_noalloc: device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hard_hydro_step_noalloc: hipGetSymbolAddress");
    if (!p || (reinterpret_cast<uintptr_t>(p) & 255u))
      return fail(HARD_ERR_HIP, "hard_hydro_step_noalloc: scratch address %p is not 256-byte aligned", p);
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return HARD_OK;
}

__global__ void flags_out_kernel(const Control* ctl, uint32_t* flags) {
  if (threadIdx.x == 0) *flags = ctl->flags;
}

}  // namespace
}  // namespace hard

using namespace hard;

extern "C" hard_status_t hard_hydro_step_noalloc(const hard_grid_t* g, void* U, const double* dt_dev,
                                                 double cfl, double* next_dt_dev,
                                                 uint32_t* flags_dev, void* stream) {
  Grid G;
  hard_status_t st = check_grid(g, &G);
  if (st) return st;
  if (flags_dev && (st = check_ptr(flags_dev, 4, "flags_dev"))) return st;
  const size_t need = layout_of(G).total;
  if (need > (size_t)HARD_NOALLOC_SCRATCH_BYTES)
    return fail(HARD_ERR_WORKSPACE,
                "hard_hydro_step_noalloc: the grid needs %zu bytes of workspace, the static "
                "scratch holds %zu; use hard_hydro_step with a caller workspace",
                need, (size_t)HARD_NOALLOC_SCRATCH_BYTES);
  void* work = nullptr;
  if ((st = scratch_of_current_device(&work))) return st;
  hipStream_t s = (hipStream_t)stream;
  Control* ctl = static_cast<Control*>(work);
  hipError_t e = launch_control_clear(ctl, s);
  if (e != hipSuccess) return hip_fail(e, "hard_hydro_step_noalloc clear");
  if ((st = hard_hydro_step(g, U, dt_dev, cfl, next_dt_dev, work, (size_t)HARD_NOALLOC_SCRATCH_BYTES,
                            stream)))
    return st;
  if (flags_dev) {
    hipLaunchKernelGGL(flags_out_kernel, dim3(1), dim3(64), 0, s, ctl, flags_dev);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "hard_hydro_step_noalloc flags");
  }
  return ok();
}
