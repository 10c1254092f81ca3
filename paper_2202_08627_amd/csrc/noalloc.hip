// Cost and gradient without a caller workspace: the evaluation's scratch buffers (trial-point
// transpose, projections and adjoint seeds, cost partials, the split adjoint's partial planes)
// live in one file-scope device array per GPU instead. For callers that cannot allocate
// device memory (code under graph capture, tight serving loops).
//
// The array's host-side name is only a stand-in for the symbol: its device address is looked
// up once per device with hipGetSymbolAddress and cached, and only that address is handed to
// the kernels. Every call on one GPU shares the array, so calls that overlap on one GPU race;
// the evaluation writes every scratch word it reads, so nothing needs clearing between calls.
#include <hip/hip_runtime.h>

#include <mutex>

#include "eitomo.h"

namespace {

constexpr size_t kScratchBytes = (size_t)EIT_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this GPU's scratch array (looked up once per device).
int scratch_for_current_device(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return EIT_ERR_DEVICE;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return EIT_ERR_DEVICE;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return EIT_OK;
}

}  // namespace

namespace eit {
int report_failure(int code, const char* msg);   // api.cpp: sets eit_last_error
}

extern "C" int eit_cost_and_grad_noalloc(const eit_plan* plan, const float* x, const float* s_exp,
                                         double lam_mu, double lam_delta, double* cost_dev,
                                         float* grad, void* stream) {
    if (!plan) return eit::report_failure(EIT_ERR_INVALID_ARG, "plan is NULL");
    const size_t need = eit_workspace_bytes(plan, EIT_OP_COST_GRAD, 0);
    if (need == 0) return eit::report_failure(EIT_ERR_INVALID_ARG, "invalid plan");
    if (need > kScratchBytes)
        return eit::report_failure(EIT_ERR_NOMEM,
                                   "problem needs more scratch than the static limit "
                                   "EIT_NOALLOC_SCRATCH_BYTES; use eit_cost_and_grad with a workspace");
    void* ws = nullptr;
    if (scratch_for_current_device(&ws) != EIT_OK)
        return eit::report_failure(EIT_ERR_DEVICE, "hipGetSymbolAddress of the scratch array failed");
    return eit_cost_and_grad(plan, x, s_exp, lam_mu, lam_delta, cost_dev, grad, ws, kScratchBytes,
                             stream);
}
