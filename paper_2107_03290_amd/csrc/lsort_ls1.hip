// LearnedSort 1.0's spill bucket on the GPU, as an ablation against the
// fragment partition (Sec. 2, Fig. 1, Sec. 3).  One partition of the whole
// array into fixed-capacity buckets (k_scatter_ls1 in lsort_partition.hip):
// the keys a bucket cannot hold go to a spill area.  The buckets are then
// sorted (by the library's own pipeline, as segments), the spill area by a
// general-purpose sort, and the two sorted sequences are merged.  LS1 sorted
// its spill bucket with std::sort and merged it last; here rocPRIM's radix
// sort and merge take those two roles, so the ablation prices the spill
// bucket's extra passes over its keys, not a slower comparison sort.
#include "lsort_internal.h"
#include "lsort_device.h"

#include <rocprim/device/device_merge.hpp>
#include <rocprim/device/device_radix_sort.hpp>

#pragma clang fp contract(off)

namespace lsort {

size_t ls1_scatter_lds_bytes(uint32_t fanout, uint32_t leaves)
{
    return scatter_lds_bytes(kLs1Tile, fanout) + ls1_model_lds_bytes(leaves) + (size_t)fanout * 24;
}

// Keys of entry e = (bucket b, chunk c) past the bucket's capacity: the
// entry's keys take the bucket ranks [r0, r0 + cnt), r0 its position in the
// bucket's count-ordered layout.
__global__ __launch_bounds__(256) void k_ls1_spill_counts(const uint64_t* pos, const uint32_t* cnt,
                                                          uint64_t entries, uint32_t nchunks, uint64_t cap,
                                                          uint32_t* spilled)
{
    const uint64_t e = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= entries)
        return;
    const uint64_t r0 = pos[e] - pos[e / nchunks * nchunks];
    const uint64_t c = cnt[e];
    const uint64_t fit = cap > r0 ? min(cap - r0, c) : 0;
    spilled[e] = (uint32_t)(c - fit);
}

hipError_t launch_ls1_spill_counts(const uint64_t* d_pos, const uint32_t* d_cnt, uint64_t entries,
                                   uint32_t nchunks, uint64_t cap, uint32_t* d_spilled, hipStream_t st)
{
    if (!entries)
        return hipSuccess;
    k_ls1_spill_counts<<<(uint32_t)((entries + 255) / 256), 256, 0, st>>>(d_pos, d_cnt, entries, nchunks, cap,
                                                                          d_spilled);
    return hipGetLastError();
}

// out[b] = first position of bucket b in the count-ordered layout (b < f),
// out[f] = n, out[f + 1] = keys in the spill area.
__global__ __launch_bounds__(256) void k_ls1_buckets(const uint64_t* pos, const uint64_t* spoff,
                                                     const uint32_t* spilled, uint32_t fanout, uint32_t nchunks,
                                                     uint64_t n, uint64_t* out)
{
    const uint32_t b = blockIdx.x * 256 + threadIdx.x;
    if (b < fanout)
        out[b] = pos[(uint64_t)b * nchunks];
    if (b == fanout) {
        const uint64_t last = (uint64_t)fanout * nchunks - 1;
        out[fanout] = n;
        out[fanout + 1] = spoff[last] + spilled[last];
    }
}

hipError_t launch_ls1_buckets(const uint64_t* d_pos, const uint64_t* d_spoff, const uint32_t* d_spilled,
                              uint32_t fanout, uint32_t nchunks, uint64_t n, uint64_t* d_out, hipStream_t st)
{
    k_ls1_buckets<<<(fanout + 1 + 255) / 256, 256, 0, st>>>(d_pos, d_spoff, d_spilled, fanout, nchunks, n, d_out);
    return hipGetLastError();
}

// The sorted buckets, one workgroup each, packed into one run of order words:
// bucket b's fill[b + 1] - fill[b] keys from slot b cap go to out + fill[b].
__global__ __launch_bounds__(256) void k_ls1_compact(const uint64_t* slots, const uint64_t* fill, uint64_t cap,
                                                     uint32_t dtype, uint64_t* out)
{
    const uint32_t b = blockIdx.x;
    const uint64_t lo = fill[b], m = fill[b + 1] - lo;
    const gptr<const uint64_t> src = as_global(slots + (uint64_t)b * cap);
    const gptr<uint64_t> dst = as_global(out + lo);
    for (uint64_t i = threadIdx.x; i < m; i += 256)
        dst[i] = to_ord(src[i], dtype);
}

hipError_t launch_ls1_compact(const uint64_t* d_slots, const uint64_t* d_fill, uint64_t cap, uint32_t fanout,
                              uint32_t dtype, uint64_t* d_out, hipStream_t st)
{
    if (!fanout)
        return hipSuccess;
    k_ls1_compact<<<fanout, 256, 0, st>>>(d_slots, d_fill, cap, dtype, d_out);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_from_ord(const uint64_t* ord, uint64_t n, uint32_t dtype, uint64_t* out)
{
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n)
        out[i] = from_ord(ord[i], dtype);
}

hipError_t launch_from_ord(const uint64_t* d_ord, uint64_t n, uint32_t dtype, uint64_t* d_out, hipStream_t st)
{
    if (!n)
        return hipSuccess;
    k_from_ord<<<(uint32_t)((n + 255) / 256), 256, 0, st>>>(d_ord, n, dtype, d_out);
    return hipGetLastError();
}

// The spill area's order words, sorted (a null temp returns its size).
hipError_t ls1_radix_sort(void* d_temp, size_t* temp_bytes, const uint64_t* d_in, uint64_t* d_out, uint64_t n,
                          hipStream_t st)
{
    return rocprim::radix_sort_keys(d_temp, *temp_bytes, d_in, d_out, (size_t)n, 0u, 64u, st);
}

// Merge of two sorted runs of order words (a null temp returns its size).
hipError_t ls1_merge(void* d_temp, size_t* temp_bytes, const uint64_t* d_a, uint64_t na, const uint64_t* d_b,
                     uint64_t nb, uint64_t* d_out, hipStream_t st)
{
    return rocprim::merge(d_temp, *temp_bytes, d_a, d_b, d_out, (size_t)na, (size_t)nb, rocprim::less<uint64_t>(),
                          st);
}

}  // namespace lsort
