// Device memory of the no-allocation sort (ls_sort_noalloc): one static
// array per device, placed by the loader together with the library's code
// object, so a sort that works out of it calls no allocator.
//
// In host code the array's name only stands in for the symbol; its device
// address is looked up once per device (noalloc_setup, from ls_create with
// that device current) and only that address is handed to kernels and copies.
#include "lsort_internal.h"

#include <algorithm>
#include <mutex>

namespace lsort {

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

constexpr int kNoAllocDevices = 64;

std::mutex g_mu;
void* g_ptr[kNoAllocDevices] = {};

}  // namespace

hipError_t noalloc_setup(int device, void** out, size_t* bytes)
{
    *out = nullptr;
    *bytes = 0;
    if (device < 0 || device >= kNoAllocDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        if (!p)
            return hipErrorInvalidSymbol;
        g_ptr[device] = p;
    }
    *out = g_ptr[device];
    *bytes = kNoAllocBytes;
    return hipSuccess;
}

// Clear `words` 8-byte words at p (a fill kernel rather than a memset node,
// so the call stays plain kernel launches).
__global__ __launch_bounds__(256) void k_zero_words(uint64_t* p, uint64_t words)
{
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < words; i += (uint64_t)gridDim.x * 256)
        p[i] = 0;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t st)
{
    const uint64_t words = bytes / 8;
    if (!words)
        return hipSuccess;
    const uint64_t grid = std::min<uint64_t>((words + 255) / 256, 1024);
    k_zero_words<<<(uint32_t)grid, 256, 0, st>>>((uint64_t*)p, words);
    return hipGetLastError();
}

}  // namespace lsort
