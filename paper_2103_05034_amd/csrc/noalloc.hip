// dwf_dot_noalloc: the inner products of dwf_dot without a handle and without
// any device allocation.  The per-workgroup partial sums go to a file-scope
// device array instead of a handle's workspace; its address on each device is
// looked up once (hipGetSymbolAddress, with that device current) and kept, and
// only that address ever reaches a kernel or a copy.
#include <mutex>

#include "dwf_internal.hpp"
#include "kernels.hpp"

namespace {

// partial sums of up to DWF_DOT_NOALLOC_MAX_RHS right-hand sides: RED_BLOCKS
// (re, im) pairs per rhs, 1 MiB in all; every block of a call writes its own
// pair, so nothing needs clearing between calls
constexpr size_t kScratchDoubles = (size_t)DWF_DOT_NOALLOC_MAX_RHS * dwf::RED_BLOCKS * 2;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device (looked up on the first
// call on that device)
int scratch_on_current_device(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return dwf::fail(DWF_EHIP, "dwf_dot_noalloc: hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return dwf::fail(DWF_EINVAL, "dwf_dot_noalloc: device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      return dwf::fail(DWF_EHIP, "dwf_dot_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
    g_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_ptr[dev];
  return DWF_OK;
}

}  // namespace

extern "C" int dwf_dot_noalloc(const int dims[4], int Ls, int prec, const void* a, const void* b, int nrhs,
                               double* result, void* stream) {
  if (!dims || !a || !b || !result) return dwf::fail(DWF_EINVAL, "dwf_dot_noalloc: null pointer");
  std::string why;
  if (!dwf::plan::valid_dims(dims, Ls, prec, 1, 0, &why)) return dwf::fail(DWF_EINVAL, "dwf_dot_noalloc: %s", why.c_str());
  if (nrhs < 1 || nrhs > DWF_DOT_NOALLOC_MAX_RHS)
    return dwf::fail(DWF_EINVAL, "dwf_dot_noalloc: nrhs %d outside [1, %d] (the size of its fixed scratch array)",
                     nrhs, DWF_DOT_NOALLOC_MAX_RHS);
  const long long V4 = (long long)dims[0] * dims[1] * dims[2] * dims[3];  // below 2^32 after the check
  double* partials = nullptr;
  if (int rc = scratch_on_current_device(&partials)) return rc;
  // a host-side description of the lattice and the stream: no workspace is carved
  dwf_context c{};
  c.g = {dims[0], dims[1], dims[2], dims[3], Ls, V4, V4 / 2};
  c.prec = prec;
  c.stream = reinterpret_cast<hipStream_t>(stream);
  HIP_TRY(dwf::blas_dot_to(&c, prec, reinterpret_cast<const char*>(a), reinterpret_cast<const char*>(b), nrhs,
                           partials, result));
  return DWF_OK;
}
