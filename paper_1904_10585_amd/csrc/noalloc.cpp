// pf_extract_noalloc: one extraction that allocates no device memory.  Its
// workspace lives in `scratch`, a fixed array of the library's code object:
// every GPU the library runs on holds its own copy (kScratchBytes) from the
// moment the library is loaded on that device until the process ends.
//
// In host code `scratch` is only a host-side stand-in for the symbol: its
// device address comes from hipGetSymbolAddress, taken once per device with
// that device current, and only that address is passed to kernels.
#include "pf_internal.h"

#include <algorithm>
#include <functional>
#include <mutex>
#include <string>

namespace pfx {
pf_status run_guarded(const std::function<void()>& f);

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;   // 64 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up on the first
// call on the device, with the device current).
void* scratch_on(int dev) {
  if (dev < 0 || dev >= kMaxDevices) fail(PF_ERR_DEVICE, "device ordinal beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      fail(PF_ERR_DEVICE, std::string("hipGetSymbolAddress of the scratch array failed: ") + hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

// Clears the first `bytes` of the workspace (a multiple of 256) with plain
// vector stores; a kernel rather than a memset so that the call can be
// captured into a graph.
__global__ __launch_bounds__(256) void zero_kernel(uint4* p, size_t n16) {
  const size_t stride = (size_t)gridDim.x * 256;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += stride) p[i] = make_uint4(0, 0, 0, 0);
}

}  // namespace
}  // namespace pfx

using namespace pfx;

extern "C" {

size_t pf_extract_noalloc_max_bytes(void) { return kScratchBytes; }

pf_status pf_extract_noalloc(const pf_desc* desc, const pf_mat* X_filter, const pf_mat* X_rr, void* U_inout,
                             int64_t ldu, double* theta_out, pf_info* info_out, void* stream) {
  return run_guarded([&] {
    if (!desc) fail(PF_ERR_ARG, "desc is NULL");
    plan_validate(*desc, X_filter, X_rr);
    if (desc->op != PF_OP_SYM) fail(PF_ERR_UNSUPPORTED, "pf_extract_noalloc serves PF_OP_SYM only");
    if (!U_inout) fail(PF_ERR_ARG, "U_inout is NULL");
    if (ldu < desc->n) fail(PF_ERR_ARG, "ldu is smaller than n");
    if (!theta_out) fail(PF_ERR_ARG, "theta_out is NULL");
    const size_t need = plan_bytes(*desc);
    if (need > kScratchBytes)
      fail(PF_ERR_ARG, "pf_extract_noalloc: this shape needs a workspace of " + std::to_string(need) +
                           " bytes, more than the fixed " + std::to_string(kScratchBytes) + " bytes");
    int dev = 0;
    PFX_HIP(hipGetDevice(&dev));
    void* base = scratch_on(dev);
    hipStream_t st = static_cast<hipStream_t>(stream);
    // the previous call left its own contents: padding rows and columns of
    // every block must read as zero
    const size_t n16 = need / 16;
    const unsigned blocks = (unsigned)std::min<size_t>((n16 + 255) / 256, 2048);
    hipLaunchKernelGGL(zero_kernel, dim3(blocks), dim3(256), 0, st, static_cast<uint4*>(base), n16);
    PFX_HIP(hipGetLastError());
    enqueue_extraction_in(*desc, base, *X_filter, *X_rr, U_inout, ldu, theta_out, info_out, st);
  });
}

}  // extern "C"
