// Measurement aid: the device's random-probe rate for the expansion's two
// probe patterns (a word of the visited bitmap, an entry of the level array),
// which bounds the scan once the column reads are streamed.
#include "../../include/bfs_test.h"
#include "bfs_internal.h"

#include <hip/hip_runtime.h>

namespace s3bfs {
namespace {

constexpr int kProbeU = 4;  // independent probes in flight per lane

__global__ void __launch_bounds__(kBlock) k_probe(const int32_t* __restrict__ idx, int64_t count,
                                                  const uint32_t* __restrict__ table, int64_t words, int shift,
                                                  int32_t* sink) {
    uint32_t acc = 0;
    const int64_t stride = (int64_t)gridDim.x * kBlock * kProbeU;
    for (int64_t base = (int64_t)blockIdx.x * kBlock * kProbeU + threadIdx.x; base < count; base += stride) {
        int32_t v[kProbeU];
#pragma unroll
        for (int u = 0; u < kProbeU; ++u) {
            const int64_t i = base + (int64_t)u * kBlock;
            v[u] = i < count ? __builtin_nontemporal_load(idx + i) : -1;
        }
#pragma unroll
        for (int u = 0; u < kProbeU; ++u) {
            const int64_t w = v[u] >= 0 ? ((int64_t)v[u] >> shift) : -1;
            if (w >= 0 && w < words) acc += (table[w] >> (v[u] & 31)) & 1u;
        }
    }
    // one lane per wave adds its wave's sum, so the probes cannot be dropped
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if ((threadIdx.x & 63) == 0 && acc == 0xdeadbeefu) atomicAdd(sink, 1);
}

}  // namespace
}  // namespace s3bfs

extern "C" bfs_status_t bfs_probe_rate_kernel(const int32_t* idx, int64_t count, const uint32_t* table,
                                              int64_t table_words, int32_t shift, int32_t* sink, void* stream) {
    if (!idx || !table || !sink || count < 0 || table_words < 1 || shift < 0 || shift > 5) return BFS_EINVAL;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return BFS_EHIP;
    const int64_t per_block = (int64_t)s3bfs::kBlock * s3bfs::kProbeU;
    int64_t grid = (count + per_block - 1) / per_block;
    grid = grid < 1 ? 1 : (grid > 8LL * cus ? 8LL * cus : grid);
    hipLaunchKernelGGL(s3bfs::k_probe, dim3((unsigned)grid), dim3(s3bfs::kBlock), 0,
                       reinterpret_cast<hipStream_t>(stream), idx, count, table, table_words, shift, sink);
    return hipGetLastError() == hipSuccess ? BFS_OK : BFS_EHIP;
}
