// The adjoint for callers that cannot allocate device memory: its scratch
// (the per-cell and per-particle accumulators of the recompute mode) lives in
// a device array of the library's own, one per GPU, held until the process
// ends.
#include <mutex>

#include "trevr_internal.h"

namespace trevr {

constexpr size_t kScratchBytes = (size_t)64 << 20;  // 64 MiB per GPU
constexpr int kMaxDevices = 64;

// The array.  In host code its name stands for the host-side shadow, not a
// device address: the device address comes from hipGetSymbolAddress, per
// device, and only that pointer is handed to kernels.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices] = {};

// Looks up this device's copy of the array (once per device; `device` must be
// the current device).  Called by trevr_tree_create and, should that not have
// run on this device, by the entry point's first call there.
int noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices)
    return fail(TREVR_E_CAPACITY, "device index beyond the no-allocation scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return TREVR_OK;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
  if (!p) return fail(TREVR_E_HIP, "hipGetSymbolAddress(scratch) gave NULL");
  g_scratch_ptr[device] = p;
  return TREVR_OK;
}

}  // namespace trevr

extern "C" int trevr_compute_flux_adjoint_noalloc(trevr_tree *tree, double theta_open,
                                                  double tau_ref, const int32_t *sinks,
                                                  int64_t n_sinks, const void *grad_flux,
                                                  void *grad_rho, void *grad_kappa,
                                                  void *grad_lum, hipStream_t stream) {
  if (!tree) return trevr::fail(TREVR_E_ARG, "tree is NULL");
  if (!tree->built) return trevr::fail(TREVR_E_STATE, "tree holds no built tree");
  size_t need = 0;
  int rc = trevr::adjoint_scratch_size_impl(tree, TREVR_ADJ_RECOMPUTE, n_sinks, &need);
  if (rc != TREVR_OK) return rc;
  if (need > trevr::kScratchBytes)
    return trevr::fail(TREVR_E_CAPACITY,
                       "the tree needs " + std::to_string(need) + " bytes of adjoint scratch, "
                       "more than the 64 MiB the no-allocation adjoint holds");
  int dev = -1;
  TREVR_HIP(hipGetDevice(&dev));
  if (dev != tree->device)
    return trevr::fail(TREVR_E_ARG, "the tree's device is not the current device");
  void *p = nullptr;
  {
    std::lock_guard<std::mutex> lock(trevr::g_scratch_mu);
    p = trevr::g_scratch_ptr[dev];
  }
  if (!p) {
    rc = trevr::noalloc_setup(dev);
    if (rc != TREVR_OK) return rc;
    std::lock_guard<std::mutex> lock(trevr::g_scratch_mu);
    p = trevr::g_scratch_ptr[dev];
  }
  return trevr_compute_flux_adjoint(tree, theta_open, tau_ref, sinks, n_sinks, grad_flux,
                                    grad_rho, grad_kappa, grad_lum, TREVR_ADJ_RECOMPUTE, p,
                                    trevr::kScratchBytes, stream);
}
