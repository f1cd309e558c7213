// noalloc.hip -- hlb_cp_mm_noalloc: hlb_cp_mm with its workspace in a static device array, for
// callers that cannot allocate device memory.
//
// The array below is a device-side object: in host code its name stands for a host-side
// symbol, not a device address.  Its device address is looked up once per device (with that
// device current) with hipGetSymbolAddress and kept; only that address is ever handed to
// kernels.  The planner then carves the call's workspace from it (a ScratchScope), so the
// kernels are exactly hlb_cp_mm's, taking their buffers as arguments.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/hlb.h"
#include "host.hpp"

namespace {

constexpr size_t kScratchBytes = (size_t)HLB_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];  // device address of `scratch` per device, once looked up

// The device address of `scratch` on the current device (looked up on first use there).
hlb_status scratch_address(void **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return HLB_EDEVICE;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return HLB_EDEVICE;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return HLB_OK;
}

}  // namespace

extern "C" hlb_status hlb_cp_mm_noalloc(int64_t m, int64_t k, int64_t nA, int64_t nB, const int64_t *P,
                                        int64_t ldp, int64_t p_absmax, const uint64_t *A, const uint64_t *B,
                                        const uint64_t *primes, int L, uint64_t *PA, uint64_t *PB, int form,
                                        void *stream) {
    if (p_absmax < 1) return HLB_EINVAL;  // a measured bound would need a device allocation
    hlb_status st = hlb::device_ready(nullptr);
    if (st != HLB_OK) return st;
    void *base = nullptr;
    if ((st = scratch_address(&base)) != HLB_OK) return st;
    hlb::ScratchScope scope(base, kScratchBytes);
    return hlb::cp_mm_entry(m, k, nA, nB, P, ldp, p_absmax, A, B, primes, L, PA, PB, form, (hipStream_t)stream);
}
