// The preconditioner apply for callers that cannot allocate device memory
// (spand_apply_noalloc): the apply's scratch is a fixed array in the library's
// device image instead of the handle's allocated workspace.
//
// In host code `scratch` names a host-side stand-in of the device array, not a
// device address; only the per-device address obtained from hipGetSymbolAddress is
// ever handed to a kernel or a copy.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "context.h"

namespace spand {
size_t apply_scratch_doubles(const spand_ctx* h, int32_t nrhs);
}

namespace {

// 8 Mi doubles (64 MiB) on every GPU the library runs on, held until the process ends.
constexpr size_t NOALLOC_SCRATCH_DOUBLES = size_t(8) << 20;
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
double* g_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on the current device, looked up once per device.
hipError_t scratch_ptr(int dev, double** out) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" spand_status spand_apply_noalloc(spand_t h, int32_t nrhs, const double* r, double* z) {
  if (!h) return SPAND_E_INVALID;
  if (!h->factored) return spand::set_err(h, SPAND_E_STATE, "apply called before a successful factor");
  if (nrhs < 1 || !r || !z || r == z) return spand::set_err(h, SPAND_E_INVALID, "bad apply arguments");
  const size_t need = spand::apply_scratch_doubles(h, nrhs);
  if (need > NOALLOC_SCRATCH_DOUBLES)
    return spand::set_err(h, SPAND_E_INVALID,
                          "spand_apply_noalloc needs " + std::to_string(need) + " doubles of scratch; its fixed buffer holds " +
                              std::to_string(NOALLOC_SCRATCH_DOUBLES) + " (use spand_apply or fewer right-hand sides)");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= MAX_DEVICES)
    return spand::set_err(h, SPAND_E_HIP, "no usable HIP device for the fixed scratch");
  double* ptr = nullptr;
  if ((e = scratch_ptr(dev, &ptr)) != hipSuccess)
    return spand::set_err(h, SPAND_E_HIP, std::string("hipGetSymbolAddress of the fixed scratch: ") + hipGetErrorString(e));
  // the apply only launches kernels; every scratch entry is written before it is read
  return spand::apply_precond(h, nrhs, r, z, ptr, h->stream);
}
