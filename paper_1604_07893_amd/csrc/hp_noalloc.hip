// hp_solve_noalloc: hp_solve with its workspace in a fixed array of the
// library's device code object instead of caller memory, for callers that
// cannot allocate device memory (code under stream capture, tight serving
// loops, harnesses that forbid hipMalloc).
//
// The array below is a host-side stand-in in host code: its device address
// comes from hipGetSymbolAddress, taken once per device with that device
// current (hp_create, or the entry point's first call on a device if that
// failed), and only that address is ever handed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "hp_host.h"

namespace {

static __device__ __align__(256) unsigned char scratch[HP_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};  // device address of `scratch` on each device

}  // namespace

namespace hp {

int noalloc_init(int device) {
    if (device < 0 || device >= kMaxDevices) return HP_EINVAL;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_scratch[device]) return HP_OK;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != device) return HP_EHIP;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return HP_EHIP;
    if (reinterpret_cast<uintptr_t>(ptr) % kAlign) return HP_EHIP;
    g_scratch[device] = ptr;
    return HP_OK;
}

}  // namespace hp

extern "C" int hp_solve_noalloc(hp_handle* h, const hp_params* p, const double* A, int64_t m,
                                int64_t n, int64_t lda, const double* X0, int64_t ldx0, double* X,
                                int64_t ldx, void* stream, hp_result* out) {
    if (!h || !p) return HP_EINVAL;
    size_t need = 0;
    const int rc = hp_workspace_bytes(p, m, n, &need);
    if (rc != HP_OK) return rc;
    if (need > (size_t)HP_NOALLOC_SCRATCH_BYTES) return HP_EWORKSPACE;
    if (h->device < 0 || h->device >= kMaxDevices) return HP_EINVAL;
    void* ws = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        ws = g_scratch[h->device];
    }
    if (!ws) {
        if (hipSetDevice(h->device) != hipSuccess) return HP_EHIP;
        if (hp::noalloc_init(h->device) != HP_OK) return HP_EHIP;
        std::lock_guard<std::mutex> lock(g_mu);
        ws = g_scratch[h->device];
    }
    // the solve allocates nothing (no graph capture: with device_stop its
    // loops are launched one by one); it clears the split-K counters with a
    // fill kernel and writes every other scratch value before reading it, so
    // the previous call's contents do not matter
    return hp::solve_entry(h, p, A, m, n, lda, X0, ldx0, X, ldx, ws,
                           (size_t)HP_NOALLOC_SCRATCH_BYTES, stream, out, false);
}
