// Batched device-to-device staging for the serving loop: every array of every
// request packed into one launch is gathered (and the launch's outputs
// scattered back) by one kernel over a table of copy descriptors, instead of
// one copy call per array per request.
#include "pinmpc_internal.h"

namespace pinmpc {

namespace {

// Work item g belongs to descriptor d with D[d].row0 <= g < D[d + 1].row0.
__device__ inline int find_desc(const CopyDesc* D, int nd, uint64_t g) {
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (D[mid].row0 <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ void __launch_bounds__(256) copy_batch_kernel(const CopyDesc* D, int nd,
                                                         uint64_t rows_total) {
  for (uint64_t g = blockIdx.x; g < rows_total; g += gridDim.x) {
    const CopyDesc d = D[find_desc(D, nd, g)];
    const uint64_t row = g - d.row0;
    char* dst = (char*)d.dst + row * d.dst_pitch;
    const char* src = d.src ? (const char*)d.src + row * d.src_pitch : nullptr;
    switch (d.op) {
      case COPY_WORDS:
        for (uint32_t i = threadIdx.x; i < d.row_bytes / 4; i += blockDim.x)
          ((uint32_t*)dst)[i] = ((const uint32_t*)src)[i];
        break;
      case COPY_BYTES:
        for (uint32_t i = threadIdx.x; i < d.row_bytes; i += blockDim.x) dst[i] = src[i];
        break;
      case COPY_FILL:   // int32 pattern a + b i
        for (uint32_t i = threadIdx.x; i < d.row_bytes / 4; i += blockDim.x)
          ((int32_t*)dst)[i] = d.a + d.b * (int32_t)i;
        break;
      case COPY_HALF:   // 0.5 x float source
        for (uint32_t i = threadIdx.x; i < d.row_bytes / 4; i += blockDim.x)
          ((float*)dst)[i] = 0.5f * ((const float*)src)[i];
        break;
    }
  }
}

}  // namespace

hipError_t launch_copy_batch(const CopyDesc* table, int nd, uint64_t rows_total, hipStream_t st) {
  if (nd == 0 || rows_total == 0) return hipSuccess;
  const unsigned grid = (unsigned)(rows_total < 8192 ? rows_total : 8192);
  hipLaunchKernelGGL(copy_batch_kernel, dim3(grid), dim3(256), 0, st, table, nd, rows_total);
  return hipGetLastError();
}

}  // namespace pinmpc
