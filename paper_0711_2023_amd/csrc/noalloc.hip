// tucker_fit_static: the fit of a given Tucker model (tucker_fit) with its
// scratch space in a static device array of this file instead of a caller
// workspace, for callers that cannot allocate device memory (code under
// stream capture, tight serving loops).
//
// The array is a file-scope __device__ object: every device the library runs
// on holds its own copy, at its own address, from the load of the code
// object until the process ends. Host code never passes the array's name to
// a kernel (on the host that name is only a stand-in for the symbol): the
// first call on a device looks the device address up with
// hipGetSymbolAddress, with that device current, and keeps it per device.
// Every call on one device shares that device's copy and leaves its contents
// behind; the fit clears or overwrites everything it reads before reading
// it, exactly as with a caller's uninitialised workspace. Calls that overlap
// on one device (several host threads, or several streams) race on the array.
#include "../../include/tucker.h"
#include "common.h"

#include <mutex>

namespace tk {

static_assert(TK_STATIC_SCRATCH_BYTES % 256 == 0, "static scratch size must be a multiple of 256");

static __device__ __align__(256) char scratch[TK_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`.
int scratch_of_current_device(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_hip_error(e, "hipGetDevice");
        return TK_ERR_DEVICE;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        set_hip_error(hipErrorInvalidDevice, "tucker_fit_static: device ordinal beyond 63");
        return TK_ERR_DEVICE;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) {
            set_hip_error(e, "hipGetSymbolAddress(scratch)");
            return TK_ERR_DEVICE;
        }
        if (!p) {
            set_hip_error(hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch) gave a null address");
            return TK_ERR_DEVICE;
        }
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return TK_OK;
}
}  // namespace

}  // namespace tk

extern "C" int tucker_fit_static(const tk_coo *X, const int32_t *core_dims, const double *core,
                                 const double *const *factors, double *fit, void *stream) {
    size_t need = 0;
    int st = tucker_workspace_bytes(TK_ALGO_FIT, X, core_dims, nullptr, &need);
    if (st) return st;
    if (!core || !factors || !factors[0] || !factors[1] || !factors[2] || !fit) return TK_ERR_ARG;
    if (need > (size_t)TK_STATIC_SCRATCH_BYTES) return TK_ERR_SIZE;
    void *ws = nullptr;
    if ((st = tk::scratch_of_current_device(&ws))) return st;
    return tucker_fit(X, core_dims, core, factors, fit, ws, (size_t)TK_STATIC_SCRATCH_BYTES, stream);
}
