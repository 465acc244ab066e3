// hdcg_coarse_solve_noalloc: the persistent coarse CG with its work memory
// in one static device array instead of handle buffers, for callers that
// cannot allocate device memory.  r, the two search-direction buffers, A p,
// the per-workgroup partial sums and the grid-barrier state are carved from
// `scratch`.  Each device the library runs on holds its own copy of the
// array until the process ends; its device address is looked up once per
// device (hipGetSymbolAddress) and kept, and only that address is passed to
// kernels or copies: in host code the array's name is a host-side stand-in,
// not a device address.
#include <mutex>
#include <string>

#include "hdcg_impl.h"

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
constexpr int kMaxRhs = 16;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::once_flag g_once[kMaxDevices];
void* g_ptr[kMaxDevices] = {};

// The device address of this device's `scratch` (nullptr on failure); the
// lookup runs once per device, with that device current.
void* scratch_address(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::call_once(g_once[dev], [dev] {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess) g_ptr[dev] = p;
  });
  return g_ptr[dev];
}

}  // namespace

using namespace hdk;

extern "C" {

int hdcg_coarse_solve_noalloc(hdcg_t h, void* x, const void* b, int prec, int nrhs, double tol, int maxiter,
                              int* iters, void* stream) {
  if (!h || !x || !b || !(tol > 0) || maxiter < 1)
    return fail(DWF_ERR_ARG, "bad arguments to hdcg_coarse_solve_noalloc");
  if (prec != DWF_C64 && prec != DWF_BF16 && prec != DWF_F16)
    return fail(DWF_ERR_ARG, "hdcg_coarse_solve_noalloc: prec must be DWF_C64, DWF_BF16 or DWF_F16");
  if (nrhs < 1 || nrhs > kMaxRhs) return fail(DWF_ERR_ARG, "hdcg_coarse_solve_noalloc: nrhs must be in 1..16");
  if (h->ng > 0 && h->prm.ldop_defl != 0)
    return fail(DWF_ERR_STATE, "hdcg_coarse_solve_noalloc: the deflated coarse solve is not covered (ldop_defl = 0)");
  if ((prec == DWF_BF16 && !h->mf_have_bf16) || (prec == DWF_F16 && !h->mf_have_f16))
    return fail(DWF_ERR_STATE, "hdcg_coarse_solve_noalloc: the 16-bit coarse storage is not built");
  const size_t need = coarse_cg_work_bytes(h, prec, nrhs);
  if (need == 0)
    return fail(DWF_ERR_ARG, "hdcg_coarse_solve_noalloc: shape not covered by the persistent solve (nvec <= 64)");
  if (need > kScratchBytes)
    return fail(DWF_ERR_ARG, "hdcg_coarse_solve_noalloc: needs " + std::to_string(need) +
                                 " bytes of work memory, above the static limit of " + std::to_string(kScratchBytes));
  int dev = 0;
  HDCG_HIP(hipGetDevice(&dev));
  void* base = scratch_address(dev);
  if (!base) return fail(DWF_ERR_HIP, "hipGetSymbolAddress of the coarse-solve scratch array failed");
  int it = 0;
  HDCG_TRY(coarse_cg_persistent_in(h, base, prec, static_cast<c64*>(x), static_cast<const c64*>(b), nrhs, tol, maxiter,
                                   &it, static_cast<hipStream_t>(stream)));
  if (iters) *iters = it;
  return it >= maxiter ? DWF_NOT_CONVERGED : DWF_OK;
}

}  // extern "C"
