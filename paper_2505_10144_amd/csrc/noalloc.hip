// The radix sort of (key, value) pairs with its workspace in a fixed device
// array instead of caller memory, for callers that cannot allocate device
// memory (code under HIP graph capture, serving loops, harnesses that forbid
// hipMalloc).  The kernels are those of vrs_sort_pairs; only where the
// workspace lives differs.
//
// The array is a file-scope __device__ variable: every GPU the library runs
// on holds its own copy (sort_ws_layout_bytes(VRS_SORT_NOALLOC_MAX_PAIRS),
// about 30 MiB) from module load until the process ends.  Its host-side name
// is not a device address, so the device address is taken once per device
// with hipGetSymbolAddress (with that device current) and only that address
// is handed to kernels.
#include <mutex>

#include "vrs_internal.h"

namespace vrs {
int launch_sort_pairs(uint64_t* keys, uint32_t* vals, const uint32_t* n_dev, size_t capacity, int key_bits,
                      void* ws, int* err, hipStream_t s);
}

namespace {

constexpr size_t kScratchBytes = vrs::sort_ws_layout_bytes(VRS_SORT_NOALLOC_MAX_PAIRS);

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of the current device's scratch array, looked up on the
// first call on that device.  Returns VRS_OK and sets *out, or an error.
int scratch_for_current_device(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return VRS_ERR_HIP;
    if (dev < 0 || dev >= kMaxDevices) return VRS_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return VRS_ERR_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return VRS_OK;
}

}  // namespace

extern "C" {

int vrs_sort_pairs_noalloc(uint64_t* keys, uint32_t* vals, const uint32_t* n_dev, size_t capacity,
                           int32_t key_bits, int32_t* status_dev, vrs_stream_t stream) {
    if (key_bits < 0 || key_bits > 64 || !n_dev) return VRS_ERR_INVALID_ARG;
    if (capacity > VRS_SORT_NOALLOC_MAX_PAIRS) return VRS_ERR_SCRATCH;
    if (capacity > 0 && (!keys || !vals || (reinterpret_cast<uintptr_t>(keys) & 7u))) return VRS_ERR_INVALID_ARG;
    if (capacity == 0) return VRS_OK;
    void* ws = nullptr;
    const int rc = scratch_for_current_device(&ws);
    if (rc != VRS_OK) return rc;
    return vrs::launch_sort_pairs(keys, vals, n_dev, capacity, key_bits, ws, status_dev,
                                  reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"
