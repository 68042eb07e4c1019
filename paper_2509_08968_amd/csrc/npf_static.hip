// npf_run on a workspace the library holds itself, for callers that cannot allocate device
// memory: a file-scope device array per GPU, addressed through hipGetSymbolAddress.
#include <map>
#include <mutex>
#include <string>

#include "npf_internal.h"

namespace npf {

namespace {

constexpr int64_t kScratchBytes = int64_t(256) << 20;   // NPF_STATIC_WORKSPACE_BYTES

// The workspace of npf_run_static.  Its name is a host-side stand-in: host code uses only
// the device address taken below, never the array itself.
__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
std::map<int, char *> g_addr;   // device -> address of that device's copy of scratch

// Address of the current device's scratch, taken once per device with that device current.
int scratch_address(char **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(NPF_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_addr.find(dev);
    if (it != g_addr.end()) {
        *out = it->second;
        return NPF_OK;
    }
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(NPF_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                      hipGetErrorString(e != hipSuccess ? e : hipErrorUnknown));
    g_addr[dev] = static_cast<char *>(p);
    *out = static_cast<char *>(p);
    return NPF_OK;
}

}  // namespace

}  // namespace npf

using namespace npf;

extern "C" int npf_run_static(npf_plan_t plan, const npf_tensor *A, const void *U, const void *V,
                              const void *lambda, void *P_out, void *npf_out, void *stream)
{
    if (!plan) return fail(NPF_E_INVALID, "null plan");
    if (plan->lay.total > kScratchBytes)
        return fail(NPF_E_UNSUPPORTED, "the plan's workspace (" + std::to_string(plan->lay.total) +
                                           " bytes) exceeds the static workspace of " +
                                           std::to_string(kScratchBytes) +
                                           " bytes; use npf_run with a workspace");
    if (plan->prof.on)
        return fail(NPF_E_INVALID, "npf_run_static does not record kernel times (profiling is on)");
    char *ws = nullptr;
    const int rc = scratch_address(&ws);
    if (rc) return rc;
    return run_eager_checked(plan, A, U, V, lambda, ws, kScratchBytes, P_out, npf_out,
                             static_cast<hipStream_t>(stream));
}
