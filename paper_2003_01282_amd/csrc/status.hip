// Device status word: numeric problems that only the device sees (a
// non-finite Lanczos coefficient, a tridiagonal eigensolve that reached its
// sweep cap) are ORed into one word per device, which slaq_device_status
// reports and clears.  The word is a file-scope __device__ variable; host code
// uses the address hipGetSymbolAddress returns for the current device (each
// device holds its own copy) and passes it to the kernels.
#include <mutex>

#include "common.hpp"

namespace slaq {

__device__ unsigned int g_device_status;

constexpr int kMaxDevices = 64;

unsigned* device_status_word() {
    static std::mutex mu;
    static unsigned* addr[kMaxDevices] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(g_device_status)) != hipSuccess) return nullptr;
        addr[dev] = (unsigned*)p;
    }
    return addr[dev];
}

}  // namespace slaq

using namespace slaq;

extern "C" {

slaq_status slaq_device_status(unsigned* bits, int clear, void* stream) {
    clear_error();
    unsigned* w = device_status_word();
    SLAQ_REQUIRE(w, SLAQ_ERR_HIP, "device status word unavailable on the current device");
    hipStream_t st = (hipStream_t)stream;
    unsigned v = 0;
    SLAQ_HIP(hipMemcpyAsync(&v, w, sizeof(v), hipMemcpyDeviceToHost, st));
    SLAQ_HIP(hipStreamSynchronize(st));
    if (clear && v) {
        const unsigned zero = 0;
        SLAQ_HIP(hipMemcpyAsync(w, &zero, sizeof(zero), hipMemcpyHostToDevice, st));
        SLAQ_HIP(hipStreamSynchronize(st));
    }
    if (bits) *bits = v;
    SLAQ_REQUIRE(v == 0, SLAQ_ERR_NUMERIC, "device status 0x%x (1 non-finite coefficient, 2 eigensolve sweep cap)",
                 v);
    return SLAQ_OK;
}

}  // extern "C"
