// Deterministic apply whose element-value buffer is a library-owned device
// array instead of caller memory: for callers that cannot allocate device
// memory (code under stream capture, serving loops, harnesses that forbid
// allocation).  The array is a file-scope __device__ object, so each GPU the
// library runs on holds one copy, at its own address, until the process ends;
// its address is looked up once per device with hipGetSymbolAddress and that
// address (never the symbol itself) is what host code hands to the kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "mfhex.h"
#include "op.h"

namespace {
constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per device
}

static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices];  // device address of `scratch` per device, null until looked up

// Device address of this device's copy of the array (the device must be current).
int scratch_address(mfhex_op op, int dev, void **out)
{
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void *ptr = nullptr;
        const int c = mfhex::check_hip(op, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress");
        if (c) return c;
        if (!ptr) return mfhex::set_error(op, MFHEX_ERR_HIP, "hipGetSymbolAddress returned a null address");
        g_ptr[dev] = ptr;
    }
    *out = g_ptr[dev];
    return MFHEX_OK;
}

}  // namespace

extern "C" size_t mfhex_apply_static_max_bytes(void) { return kScratchBytes; }

extern "C" int mfhex_apply_static(mfhex_op op, int prec, const void *x_dev, void *y_dev, void *stream)
{
    using namespace mfhex;
    if (!op) return fail_global(MFHEX_ERR_ARG, "null handle");
    if (prec != MFHEX_F64 && prec != MFHEX_F32) return set_error(op, MFHEX_ERR_ARG, "prec must be F64 or F32");
    // element values of one right-hand side: [E][P^3][ncomp]
    const size_t need = (size_t)op->E * op->P * op->P * op->P * op->d.ncomp * (prec == MFHEX_F32 ? 4 : 8);
    if (need > kScratchBytes)
        return set_error(op, MFHEX_ERR_ARG,
                         "mfhex_apply_static: the element values need " + std::to_string(need) +
                             " bytes, above the library's static buffer of " + std::to_string(kScratchBytes) +
                             " bytes; use mfhex_apply on an operator created with MFHEX_FLAG_DETERMINISTIC");
    int dev = -1;
    int c = check_hip(op, hipGetDevice(&dev), "hipGetDevice");
    if (c) return c;
    if (dev != op->device)
        return set_error(op, MFHEX_ERR_STATE, "mfhex_apply_static: the operator's device must be current");
    if (dev < 0 || dev >= kMaxDevices) return set_error(op, MFHEX_ERR_UNSUPPORTED, "device index out of range");
    void *ebuf = nullptr;
    c = scratch_address(op, dev, &ebuf);
    if (c) return c;
    // Every element value the assembly reads is written by the apply first (masked nodes are
    // neither stored nor read), so the buffer needs no clearing.
    return apply_impl(op, prec, 1, x_dev, y_dev, static_cast<hipStream_t>(stream), true, -1, 0, ebuf);
}
