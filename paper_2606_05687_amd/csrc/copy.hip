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

// Copy n units of T from s to d with four loads in flight per thread (a
// block-strided loop with one load per thread waits on every load in turn).
template <class T>
__device__ inline void copy_units(T* __restrict__ d, const T* __restrict__ s, uint32_t n) {
  constexpr uint32_t B = 256;
  uint32_t i = threadIdx.x;
  for (; i + 3 * B < n; i += 4 * B) {
    const T v0 = s[i], v1 = s[i + B], v2 = s[i + 2 * B], v3 = s[i + 3 * B];
    d[i] = v0;
    d[i + B] = v1;
    d[i + 2 * B] = v2;
    d[i + 3 * B] = v3;
  }
  for (; i < n; i += B) d[i] = s[i];
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
        // 16-byte units when both ends and the length allow it
        if ((((uintptr_t)dst | (uintptr_t)src | d.row_bytes) & 15) == 0)
          copy_units((uint4*)dst, (const uint4*)src, d.row_bytes / 16);
        else
          copy_units((uint32_t*)dst, (const uint32_t*)src, d.row_bytes / 4);
        break;
      case COPY_BYTES:
        copy_units((uint8_t*)dst, (const uint8_t*)src, d.row_bytes);
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
