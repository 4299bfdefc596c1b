// pw_energy_noalloc: the discrete wave energy of pw_energy for callers that
// cannot allocate device memory (code under HIP graph capture, serving
// loops).  The per-workgroup partial sums of the reduction live in a
// file-scope device array of fixed size instead of a context buffer; the
// kernels are those of pw_energy (energy_pair), so both calls give the same
// bits for the same input.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "pw_internal.h"

// Partial sums of one call: 4 doubles per workgroup of the energy kernel
// (32 KiB).  Each GPU the library runs on holds its own copy until the
// process ends; all calls on one GPU share it.
static __device__ __align__(256) double scratch[pw::kEnergyPartials];

namespace pw {
namespace {

// Largest grid accepted (the energy kernel derives per-axis indices in int).
constexpr long long kMaxPoints = 2147483647LL;

// Device address of this GPU's copy of `scratch`, looked up once per device
// with that device current.  In host code the array's name is only a
// stand-in, never a device address, so kernels receive this pointer.
double* scratch_ptr() {
  static std::mutex mu;
  static std::vector<double*> ptrs;
  int dev = -1;
  PW_HIP(hipGetDevice(&dev));
  if (dev < 0) fail(PW_EHIP, "no current device");
  std::lock_guard<std::mutex> lock(mu);
  if ((size_t)dev >= ptrs.size()) ptrs.resize((size_t)dev + 1, nullptr);
  if (!ptrs[(size_t)dev]) {
    void* ptr = nullptr;
    PW_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) fail(PW_EHIP, "hipGetSymbolAddress gave a null address for the scratch array");
    ptrs[(size_t)dev] = (double*)ptr;
  }
  return ptrs[(size_t)dev];
}

void energy_noalloc(const pw_problem* desc, const double* c, const void* u, const void* p,
                    const void* u_ref, const void* p_ref, double* out, void* stream) {
  if (!desc) fail(PW_EINVAL, "null problem description");
  if (desc->dim < 1 || desc->dim > 3) fail(PW_EINVAL, "dim must be 1, 2 or 3");
  Grid g;
  g.dim = desc->dim;
  long long npts = 1;
  for (int a = 0; a < 3; ++a) {
    const int n = desc->n_fine[a];
    if (a < g.dim && n < 1) fail(PW_EINVAL, "n_fine must be positive");
    if (a >= g.dim && n != 1) fail(PW_EINVAL, "unused axes must have n_fine = 1");
    g.n[a] = n;
    npts *= n;
    if (npts > kMaxPoints)
      fail(PW_EINVAL, "grid larger than pw_energy_noalloc supports (2^31 - 1 points)");
  }
  g.dx = 1.0 / desc->n_fine[0];
  const int order = desc->grad_order == 0 ? 4 : desc->grad_order;
  if (order != 2 && order != 4 && order != 6 && order != 8)
    fail(PW_EINVAL, "grad_order must be 2, 4, 6, 8 or 0 (spectral)");
  if (desc->state_dtype != PW_F32 && desc->state_dtype != PW_F64)
    fail(PW_EINVAL, "bad state dtype");
  if (!c || !u || !p || !out || (u_ref && !p_ref)) fail(PW_EINVAL, "null pointer argument");
  hipStream_t st = (hipStream_t)stream;
  // every partial slot is rewritten by its workgroup in each call: nothing
  // in the scratch has to be cleared between calls
  double* part = scratch_ptr();
  if (desc->state_dtype == PW_F64)
    energy_pair<double>(g, (const double*)u, (const double*)p, (const double*)u_ref,
                        (const double*)p_ref, c, order, part, out, st);
  else
    energy_pair<float>(g, (const float*)u, (const float*)p, (const float*)u_ref,
                       (const float*)p_ref, c, order, part, out, st);
}

}  // namespace
}  // namespace pw

extern "C" pw_status pw_energy_noalloc(const pw_problem* desc, const double* c, const void* u,
                                       const void* p, const void* u_ref, const void* p_ref,
                                       double* out, void* stream) {
  try {
    pw::energy_noalloc(desc, c, u, p, u_ref, p_ref, out, stream);
    return PW_OK;
  } catch (const pw::Error& e) {
    pw::set_last_error(e.msg);
    return e.status;
  } catch (const std::exception& e) {
    pw::set_last_error(e.what());
    return PW_EINVAL;
  }
}
