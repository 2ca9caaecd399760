// The fixed workspace of the allocation-free CG entry point
// (stag_cg_solve_noalloc): a file-scope device array of kScratchBytes, of
// which every GPU the library runs on holds its own copy until the process
// ends.  Its device address is looked up once per device at stag_create,
// with that device current, and only that address is handed to kernels and
// copies (the array's name in host code is a host-side stand-in, not a device
// address).  The host-side mirror of the solve's state records is a fixed
// host buffer per device.  Calls on one device are serialised by a per-device
// lock, and each call re-initialises everything its kernels read before
// writing it (states, search directions, residuals and partial sums are all
// written by the solve's own initialisation kernel and steps), so nothing
// has to be cleared between calls.
#include <mutex>

#include "runtime.hpp"

namespace stag {

// 128 MiB: an FP64 solve of one right-hand side needs about 480 bytes per
// checkerboard site (a 24^4 lattice, 331 776 sites: 80 MB); FP32 and FP16
// solves less.
constexpr size_t kScratchBytes = (size_t)128 << 20;
constexpr int kMaxDevices = 64;
constexpr size_t kHostBytes = 4096;  // host mirror of one solve's state records

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
void *g_scratch_ptr[kMaxDevices];
hipError_t g_setup_rc[kMaxDevices];
std::once_flag g_once[kMaxDevices];
std::mutex g_lock[kMaxDevices];
alignas(256) unsigned char g_host[kMaxDevices][kHostBytes];
}  // namespace

int noalloc_setup(int device)
{
    if (device < 0 || device >= kMaxDevices)
        return set_error(STAG_EINVAL, "device %d: the fixed workspace supports devices 0..%d", device,
                         kMaxDevices - 1);
    std::call_once(g_once[device], [device] {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
        g_setup_rc[device] = e;
        g_scratch_ptr[device] = e == hipSuccess ? ptr : nullptr;
    });
    if (g_setup_rc[device] != hipSuccess)
        return set_error(STAG_EHIP, "fixed workspace on device %d: hipGetSymbolAddress failed: %s", device,
                         hipGetErrorString(g_setup_rc[device]));
    return STAG_OK;
}

void *noalloc_scratch(int device, size_t *bytes)
{
    if (device < 0 || device >= kMaxDevices)
        return nullptr;
    if (bytes)
        *bytes = kScratchBytes;
    return g_scratch_ptr[device];
}

void *noalloc_host(int device, size_t *bytes)
{
    if (device < 0 || device >= kMaxDevices)
        return nullptr;
    if (bytes)
        *bytes = kHostBytes;
    return g_host[device];
}

std::mutex &noalloc_lock(int device) { return g_lock[device < 0 || device >= kMaxDevices ? 0 : device]; }

}  // namespace stag
