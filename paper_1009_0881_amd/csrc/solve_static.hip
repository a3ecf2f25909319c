// nmf_solve_static: the multilevel solve of nmf_solve for callers that cannot
// allocate device memory.  The workspace is a fixed-size array in device
// global memory that the library holds on every GPU it runs on (module
// memory, loaded with the code object, kept until the process ends), instead
// of a caller-allocated buffer; the kernels are those of nmf_solve.
#include <mutex>

#include "exec.h"

namespace nmf {

namespace {

// The workspace of nmf_solve_static.  In host code this name is a host-side
// stand-in, not a device address: the address of each device's copy comes
// from hipGetSymbolAddress (static_workspace below), and only that address is
// handed to kernels.
static __device__ __align__(256) char scratch[NMF_STATIC_WORKSPACE_BYTES];

constexpr int kMaxDevices = 64;

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};   // per device: address of that device's scratch

// Address of the current device's copy of `scratch`, looked up once per device
// (with that device current).
nmf_status static_workspace(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(nullptr, NMF_E_DEVICE, std::string("hipGetDevice: ") +
                                                                 hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(nullptr, NMF_E_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(nullptr, NMF_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                                   hipGetErrorString(e));
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return NMF_OK;
}

}  // namespace

}  // namespace nmf

extern "C" nmf_status nmf_solve_static(nmf_plan_t plan, const float *dM, float *dV, float *dW,
                                       int32_t iters, void *stream, nmf_result *hOut) {
    using namespace nmf;
    if (!plan || !dM || !dV || !dW) return fail(plan, NMF_E_ARG, "null plan or buffer");
    if (iters < 0) return fail(plan, NMF_E_ARG, "iters must be >= 0");
    if (plan->p.ws.total > (size_t)NMF_STATIC_WORKSPACE_BYTES)
        return fail(plan, NMF_E_NOMEM,
                    "plan needs " + std::to_string(plan->p.ws.total) +
                        " workspace bytes; nmf_solve_static holds " +
                        std::to_string((size_t)NMF_STATIC_WORKSPACE_BYTES));
    void *ws = nullptr;
    nmf_status st = static_workspace(&ws);
    if (st != NMF_OK) return st;
    return solve_on(plan, dM, dV, dW, iters, ws, static_cast<hipStream_t>(stream), hOut, false,
                    false);
}
