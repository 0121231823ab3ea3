// Graph set-up for BFS_SORT_ROWS: each row of a CSR sorted ascending into a
// separate array, by a device segmented radix sort (hipCUB).  The min-id parent
// rule and the pulled parents read rows in sorted order.
#include "bfs_internal.h"

#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

namespace s3bfs {

hipError_t sort_rows_device(const int32_t* offsets, const int32_t* cols_in, int32_t* cols_out, int32_t n, int64_t m,
                            hipStream_t s) {
    if (m <= 0 || n <= 0) return hipSuccess;
    size_t bytes = 0;
    hipError_t e = hipcub::DeviceSegmentedSort::SortKeys(nullptr, bytes, cols_in, cols_out, (int)m, n, offsets,
                                                         offsets + 1, s);
    if (e != hipSuccess) return e;
    void* tmp = nullptr;
    e = hipMalloc(&tmp, bytes > 0 ? bytes : 1);
    if (e != hipSuccess) return e;
    e = hipcub::DeviceSegmentedSort::SortKeys(tmp, bytes, cols_in, cols_out, (int)m, n, offsets, offsets + 1, s);
    const hipError_t e2 = hipStreamSynchronize(s);
    (void)hipFree(tmp);
    return e != hipSuccess ? e : e2;
}

}  // namespace s3bfs
