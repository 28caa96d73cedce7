// Allocation-free filter application (flp_filter_apply_noalloc in
// include/flp.h): the Clenshaw recurrence of flp_filter_apply on CSR storage
// with its three ring buffers (and, in FP32, the FP32 copy of the input
// block) in a fixed device array instead of the thread's workspace, for
// callers that may not allocate device memory.
#include <hip/hip_runtime.h>

#include <climits>
#include <mutex>
#include <new>

#include "flp_host.h"

namespace flp {
namespace {

// Room for the ring of three n x r FP64 blocks, or three n x r FP32 blocks
// plus the FP32 copy of V, at n * r <= kNoAllocMaxElems.
constexpr int64_t kNoAllocMaxElems = int64_t(1) << 20;
constexpr size_t kScratchBytes = 3 * sizeof(double) * (size_t)kNoAllocMaxElems;  // 24 MiB

// Every GPU the library runs on holds its own copy until the process ends.
// Host code reaches a device's copy only through the address
// hipGetSymbolAddress returned for it (scratch_ptr), never through the name.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device, looked up once per
// device with that device current.
int scratch_ptr(void **out) {
    int dev = 0;
    CK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(FLP_E_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        CK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(FLP_E_DEVICE, "hipGetSymbolAddress returned NULL for the scratch array");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return FLP_OK;
}

}  // namespace
}  // namespace flp

using namespace flp;

extern "C" int flp_filter_apply_noalloc(const flp_filter *p, const flp_csr *A, const double *V, int64_t ldv,
                                        double *W, int64_t ldw, int32_t r, int32_t prec, void *stream) {
    if (!p) return fail(FLP_E_ARG, "filter is NULL");
    CKR(check_csr(A));
    if (r < 1 || r > 32) return fail(FLP_E_ARG, "r must be in [1, 32]");
    if (!V || !W) return fail(FLP_E_ARG, "V and W must be non-NULL");
    if (ldv < r || ldw < r || ldv > INT32_MAX || ldw > INT32_MAX)
        return fail(FLP_E_ARG, "leading dimensions must be in [r, 2^31)");
    const double *vend = V + (size_t)(A->n - 1) * ldv + r;
    const double *wend = W + (size_t)(A->n - 1) * ldw + r;
    if (V < wend && W < vend) return fail(FLP_E_ARG, "W must not overlap V");
    if (prec != FLP_PREC_FP64 && prec != FLP_PREC_FP32_FILTER) return fail(FLP_E_ARG, "bad precision");
    const bool fp32 = prec == FLP_PREC_FP32_FILTER;
    if (fp32 && A->nnz > 0 && !A->val32)
        return fail(FLP_E_ARG, "FP32 filter without allocation needs the caller's FP32 values (A->val32)");
    const int64_t elems = (int64_t)A->n * r;
    if (elems > kNoAllocMaxElems)
        return fail(FLP_E_NOMEM, "n * r exceeds the allocation-free limit of 1048576 elements");
    try {
        hipStream_t s = (hipStream_t)stream;
        void *base = nullptr;
        CKR(scratch_ptr(&base));
        const size_t es = fp32 ? sizeof(float) : sizeof(double);
        char *c = (char *)base;
        void *U[3] = {c, c + es * elems, c + 2 * es * elems};
        const void *vin = V;
        int ldin = (int)ldv;
        if (fp32) {  // FP32 copy of V behind the ring (4 blocks of 4 bytes fit in 3 of 8)
            float *v32 = (float *)(c + 3 * es * elems);
            CK(launch_copy_block(A->n, r, 1.0, V, ldv, DMat{nullptr, 0, 0, 0}, 0, v32, r, s));
            vin = v32;
            ldin = r;
        }
        // the default launch shape over all r columns at once (every shape
        // gives the same bits); no tuning, which would time and allocate
        const auto plan = clenshaw_plan(p, r, vin, ldin, W, (int)ldw, U[0], U[1], U[2], fp32);
        for (const auto &st : plan) CKR(launch_plan_step(A, A->val32, r, st, fp32, s, StepShape{}, false));
        return FLP_OK;
    } catch (const std::bad_alloc &) {
        return fail(FLP_E_NOMEM, "host allocation failed");
    }
}
