// Streaming kernels that measure the HBM rate this chip sustains for plain
// reads, plain writes and a copy: the ceiling that the appearance kernels'
// algorithmic bytes are compared against beside the 8 TB/s specification.
//
// Every lane moves 16 bytes per access (global_load/store_dwordx4); a thread
// handles U consecutive block-strided 16-byte elements per pass (U loads in
// flight before the first use), and the grid strides over the buffer. The
// read kernel folds every word it loads into an XOR and stores it only if it
// equals a value no buffer of interest produces, so the loads cannot be
// removed; the write kernel stores a value derived from the index. With `NT`
// the accesses are nontemporal (the cache policy of streaming data).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/nasg.h"

namespace nasg {

constexpr int kStreamBlock = 256;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <int MODE, int U, bool NT>
__global__ __launch_bounds__(kStreamBlock) void hbm_stream_kernel(const u32x4* __restrict__ src,
                                                                 u32x4* __restrict__ dst,
                                                                 int64_t n16) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kStreamBlock * U;
  int64_t i = static_cast<int64_t>(blockIdx.x) * kStreamBlock * U + threadIdx.x;
  uint32_t acc = 0;
  auto load = [&](int64_t k) -> u32x4 {
    if constexpr (NT) return __builtin_nontemporal_load(src + k);
    return src[k];
  };
  auto store = [&](int64_t k, u32x4 v) {
    if constexpr (NT) {
      __builtin_nontemporal_store(v, dst + k);
    } else {
      dst[k] = v;
    }
  };
  // full groups of U elements
  for (; i + static_cast<int64_t>(U - 1) * kStreamBlock < n16; i += stride) {
    u32x4 v[U];
    if constexpr (MODE != NASG_STREAM_WRITE) {
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = load(i + u * kStreamBlock);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t k = i + u * kStreamBlock;
      if constexpr (MODE == NASG_STREAM_READ) {
        acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
      } else if constexpr (MODE == NASG_STREAM_COPY) {
        store(k, v[u]);
      } else {
        const uint32_t s = static_cast<uint32_t>(k);
        store(k, u32x4{s, s + 1u, s + 2u, s + 3u});
      }
    }
  }
  // the one partial group this thread may still own (the next starts beyond n16)
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t k = i + u * kStreamBlock;
    if (k < n16) {
      if constexpr (MODE == NASG_STREAM_READ) {
        const u32x4 v = load(k);
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
      } else if constexpr (MODE == NASG_STREAM_COPY) {
        store(k, load(k));
      } else {
        const uint32_t s = static_cast<uint32_t>(k);
        store(k, u32x4{s, s + 1u, s + 2u, s + 3u});
      }
    }
  }
  if constexpr (MODE == NASG_STREAM_READ) {
    if (acc == 0x9e3779b9u) dst[0] = u32x4{acc, acc, acc, acc};
  }
}

template <int MODE, bool NT>
static hipError_t launch_mode(const u32x4* src, u32x4* dst, int64_t n16, int grid, int unroll,
                              hipStream_t s) {
  switch (unroll) {
    case 1: hipLaunchKernelGGL((hbm_stream_kernel<MODE, 1, NT>), dim3(grid), dim3(kStreamBlock), 0, s, src, dst, n16); break;
    case 2: hipLaunchKernelGGL((hbm_stream_kernel<MODE, 2, NT>), dim3(grid), dim3(kStreamBlock), 0, s, src, dst, n16); break;
    case 4: hipLaunchKernelGGL((hbm_stream_kernel<MODE, 4, NT>), dim3(grid), dim3(kStreamBlock), 0, s, src, dst, n16); break;
    default: hipLaunchKernelGGL((hbm_stream_kernel<MODE, 8, NT>), dim3(grid), dim3(kStreamBlock), 0, s, src, dst, n16); break;
  }
  return hipGetLastError();
}

template <int MODE>
static hipError_t launch_nt(const u32x4* src, u32x4* dst, int64_t n16, int grid, int unroll,
                            bool nt, hipStream_t s) {
  return nt ? launch_mode<MODE, true>(src, dst, n16, grid, unroll, s)
            : launch_mode<MODE, false>(src, dst, n16, grid, unroll, s);
}

}  // namespace nasg

extern "C" int nasg_hbm_stream(int32_t mode, const void* src, void* dst, int64_t bytes,
                               int32_t blocks, int32_t unroll, int32_t nontemporal,
                               void* stream) {
  if (mode != NASG_STREAM_READ && mode != NASG_STREAM_WRITE && mode != NASG_STREAM_COPY)
    return NASG_ERR_MODE;
  if (bytes < 0 || (bytes & 15) != 0 || blocks < 1 || blocks > (1 << 20) ||
      (unroll != 1 && unroll != 2 && unroll != 4 && unroll != 8) ||
      (nontemporal != 0 && nontemporal != 1))
    return NASG_ERR_SHAPE;
  if (bytes == 0) return NASG_OK;
  if (dst == nullptr || (mode != NASG_STREAM_WRITE && src == nullptr)) return NASG_ERR_NULL;
  if ((reinterpret_cast<uintptr_t>(src) & 15) != 0 || (reinterpret_cast<uintptr_t>(dst) & 15) != 0)
    return NASG_ERR_ALIGN;
  const auto* s = static_cast<const nasg::u32x4*>(src);
  auto* d = static_cast<nasg::u32x4*>(dst);
  const int64_t n16 = bytes / 16;
  const bool nt = nontemporal != 0;
  const hipStream_t hs = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (mode == NASG_STREAM_READ) {
    e = nasg::launch_nt<NASG_STREAM_READ>(s, d, n16, blocks, unroll, nt, hs);
  } else if (mode == NASG_STREAM_WRITE) {
    e = nasg::launch_nt<NASG_STREAM_WRITE>(s, d, n16, blocks, unroll, nt, hs);
  } else {
    e = nasg::launch_nt<NASG_STREAM_COPY>(s, d, n16, blocks, unroll, nt, hs);
  }
  return e == hipSuccess ? NASG_OK : NASG_ERR_LAUNCH;
}
