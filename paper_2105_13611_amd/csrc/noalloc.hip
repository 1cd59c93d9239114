// Allocation-free ODF reduction (C ABI: odf_reduce_noalloc in include/odf.h).
//
// The same kernels as odf_stage_reduce: floor, per-bin bitonic sort, sub-bin
// means (Sec. 2.3).  Bins whose padded size exceeds the LDS capacity sort in
// a global slab; here that slab is a file-scope static device array instead
// of the plan's workspace, so the call allocates nothing and waits for
// nothing.  Each GPU the library runs on holds its own copy of the array
// until the process ends.  Host code never passes the array's name to a
// kernel (on the host it is only a stand-in for the symbol): the device
// address is resolved once per device with hipGetSymbolAddress, at plan
// time, and kept.
#include <mutex>

#include "plan.h"

namespace odf {

namespace {

__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

// Device address of this device's scratch array (resolved on first use
// with `dev` current), or nullptr with the error set.
void* noalloc_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device %d out of range for the static scratch", dev);
    return nullptr;
  }
  std::lock_guard<std::mutex> guard(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      set_error("hipGetSymbolAddress of the static scratch failed on device %d: %s", dev,
                hipGetErrorString(e));
      return nullptr;
    }
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

}  // namespace odf

using namespace odf;

extern "C" {

int64_t odf_noalloc_scratch_need(const odf_plan_t* p, int32_t n_points) {
  if (!p || n_points < 0) return -1;
  const int64_t key = p->opts.precision == ODF_PREC_MIXED ? 4 : 8;
  return p->gscr_elems * key * (int64_t)n_points;
}

odf_status odf_reduce_noalloc(odf_plan_t* p, const void* kappa_dev, int32_t n_points, void* out_dev,
                              void* stream) {
  g_last_error_clear();
  if (!p) { set_error("plan is NULL"); return ODF_E_INVALID; }
  if (n_points < 0 || n_points > 65535) { set_error("n_points must be in [0, 65535]"); return ODF_E_INVALID; }
  if (n_points == 0) return ODF_OK;
  if (!kappa_dev || !out_dev) { set_error("reduce_noalloc: NULL buffer"); return ODF_E_INVALID; }
  if (p->opts.output != ODF_OUT_TABLE) {
    set_error("reduce_noalloc: the plan writes fine-grid opacity, not an ODF table");
    return ODF_E_INVALID;
  }
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) { set_error("hipGetDevice failed: %s", hipGetErrorString(e)); return ODF_E_DEVICE; }
  if (dev != p->device) {
    set_error("reduce_noalloc: device %d is current, the plan lives on device %d", dev, p->device);
    return ODF_E_INVALID;
  }
  const int64_t need = odf_noalloc_scratch_need(p, n_points);
  if (need > kNoAllocScratchBytes) {
    set_error("reduce_noalloc: %d grids need %lld bytes of sort scratch for bins beyond LDS, "
              "the static scratch holds %lld", n_points, (long long)need, (long long)kNoAllocScratchBytes);
    return ODF_E_NOMEM;
  }
  void* scr = noalloc_scratch(dev);   // resolved at plan time on this device
  if (!scr) return ODF_E_DEVICE;
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : static_cast<hipStream_t>(p->opts.stream);
  e = launch_odf(s, p->params, kappa_dev, p->N, n_points, out_dev, p->odf_classes, scr, p->d_goff,
                 p->gscr_elems);
  if (e != hipSuccess) { set_error("reduce_noalloc launch failed: %s", hipGetErrorString(e)); return ODF_E_DEVICE; }
  return ODF_OK;
}

}  // extern "C"
