// qaoa_gradient_noalloc: the expectation and adjoint gradient of
// qaoa_gradient with no device allocation, for callers that cannot allocate
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// it).  The adjoint vector, the per-workgroup partial sums and the summed
// slots live in `scratch`, a fixed device array that each GPU the library
// runs on holds until the process ends.  Its device address is looked up
// once per device (hipGetSymbolAddress, with that device current) and only
// that address is handed to kernels and copies: in host code the array's
// name is a host-side stand-in, not a device address.
#include "qaoa.h"
#include "qaoa_internal.h"

#include <mutex>

namespace {

// 16 MiB of adjoint vector (complex128 n <= 20, complex64 n <= 21) plus the
// partial sums of up to 32 layers.
constexpr size_t kScratchBytes = ((size_t)16 << 20) + ((size_t)256 << 10);

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices];  // device address of `scratch` per device, once looked up

// Device address of `scratch` on the current device `dev`.
qaoa_status scratch_address(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxDevices) {
        qk::set_error_message("device index outside the no-allocation gradient's table");
        return QAOA_ERR_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            qk::set_error_message(std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
            return QAOA_ERR_DEVICE;
        }
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return QAOA_OK;
}

}  // namespace

extern "C" qaoa_status qaoa_gradient_noalloc(qaoa_handle h, int32_t p, const double *gamma,
                                             const double *beta, double *E, double *dgamma,
                                             double *dbeta, int32_t out_is_device)
{
    qaoa_status st = qk::noalloc_check(h, p, gamma, beta, dgamma, dbeta, kScratchBytes);
    if (st != QAOA_OK) return st;
    const int dev = qk::handle_device(h);
    int old = -1;
    hipError_t e = hipGetDevice(&old);
    if (e == hipSuccess && old != dev) e = hipSetDevice(dev);
    if (e != hipSuccess) {
        qk::set_error_message(std::string("selecting the handle's device failed: ") + hipGetErrorString(e));
        return QAOA_ERR_DEVICE;
    }
    void *ptr = nullptr;
    st = scratch_address(dev, &ptr);
    if (st == QAOA_OK) st = qk::gradient_on_scratch(h, p, gamma, beta, E, dgamma, dbeta, out_is_device, ptr);
    if (old >= 0 && old != dev) (void)hipSetDevice(old);
    return st;
}
