// sg_step_noalloc: sine-Gordon steps whose work arrays live in a fixed,
// file-scope device array instead of the plan's workspace, so that the call
// allocates nothing (for callers under HIP graph capture, in tight serving
// loops, or in harnesses that forbid allocation).
//
// The array is device memory of this library's code object: each GPU the
// library runs on holds its own copy (kScratchBytes) until the process ends,
// at an address obtained once per device with hipGetSymbolAddress.  In host
// code the array's name is not a device address; only that address is ever
// passed to kernels.  Every call on a GPU shares that GPU's copy, so calls
// that overlap on one GPU (on different streams, or from several threads)
// race; calls ordered on one stream do not.  No word of it needs to start at
// zero: a call writes each element of U and S (entry row pass) and of W
// (column pass) before it reads it, so the previous call's contents never
// leak into a result.
#include <hip/hip_runtime.h>

#include <mutex>

#include "launch.hpp"
#include "pst.h"
#include "runtime.hpp"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on device dev (the current device), looked up
// on the first call there.
pst_status scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return pst::fail(PST_ERR_UNSUPPORTED, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev[dev] == nullptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) return pst::hip_check(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                                               "hipGetSymbolAddress(scratch)");
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return PST_OK;
}

}  // namespace

extern "C" pst_status sg_step_noalloc(pst_plan pl, void* u_prev, void* u_curr, const pst_sg_params* p,
                                      int nsteps) {
  pst_status st = pst::sg_params_check(pl, p, "sg_step_noalloc");
  if (st == PST_OK) st = pst::check_field(u_prev, "u_prev");
  if (st == PST_OK) st = pst::check_field(u_curr, "u_curr");
  if (st != PST_OK) return st;
  if (u_prev == u_curr) return pst::fail(PST_ERR_INVALID, "sg_step_noalloc: u_prev and u_curr must differ");
  if (nsteps < 0) return pst::fail(PST_ERR_INVALID, "nsteps must be >= 0");
  const size_t need = pst::sg_work_bytes(pl);
  if (need > kScratchBytes)
    return pst::fail(PST_ERR_INVALID,
                     "sg_step_noalloc: %d field(s) of %d x %d need %zu bytes of scratch; the maximum is %zu",
                     pl->batch, pl->nx, pl->ny, need, kScratchBytes);
  int dev = -1;
  st = pst::hip_check(hipGetDevice(&dev), "hipGetDevice");
  if (st != PST_OK) return st;
  if (dev != pl->device)
    return pst::fail(PST_ERR_INVALID, "sg_step_noalloc: the plan's device (%d) must be current, not %d", pl->device,
                     dev);
  void* base = nullptr;
  if ((st = scratch_address(dev, &base)) != PST_OK) return st;
  const size_t fb = (size_t)pl->nx * pl->ny * pl->rsize;
  return pst::sg_run_in(pl, pst::sg_work_at(pl, base), pst::contiguous(u_prev, fb), pst::contiguous(u_curr, fb), p,
                        nsteps, nullptr, false);
}
