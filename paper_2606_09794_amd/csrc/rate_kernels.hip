// Camera-spacing statistic of the training set-up (Section 4, implementation
// details): for every camera centre the mean distance to its k nearest other
// centres, and the average of that over the cameras. The appearance learning
// rates are scaled by powers of this statistic against a reference scene's.
//
// One thread per camera. A block stages 256 centres at a time in LDS (three
// FP64 planes, so a wave reads consecutive words) and every thread scans the
// staged tile, keeping the KMAX smallest squared distances in registers as a
// sorted list: a candidate below the largest kept one is merged in by a chain
// of min/max pairs over fixed register slots (no dynamically indexed array,
// so nothing goes to scratch). Squaring is monotonic, so the kept set is that
// of the distances; the square roots are taken once, for the k kept values.
// KMAX is the smallest power of two >= k; the sum runs over the first k
// slots. The average over cameras is a second launch: one block, each thread
// summing a fixed strided slice, then a fixed tree in LDS, so the result is
// the same bit for bit on every run.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "../../include/nasg.h"

namespace nasg {

constexpr int kKnnBlock = 256;

template <int KMAX>
__global__ __launch_bounds__(kKnnBlock) void camera_knn_kernel(const double* __restrict__ centres,
                                                              int32_t n, int32_t k,
                                                              double* __restrict__ per_camera) {
  __shared__ double sx[kKnnBlock], sy[kKnnBlock], sz[kKnnBlock];
  const int32_t i = static_cast<int32_t>(blockIdx.x) * kKnnBlock + static_cast<int32_t>(threadIdx.x);
  double px = 0.0, py = 0.0, pz = 0.0;
  if (i < n) {
    px = centres[3 * i + 0];
    py = centres[3 * i + 1];
    pz = centres[3 * i + 2];
  }
  double best[KMAX];
#pragma unroll
  for (int m = 0; m < KMAX; ++m) best[m] = INFINITY;

  for (int32_t base = 0; base < n; base += kKnnBlock) {
    const int32_t j = base + static_cast<int32_t>(threadIdx.x);
    if (j < n) {
      sx[threadIdx.x] = centres[3 * j + 0];
      sy[threadIdx.x] = centres[3 * j + 1];
      sz[threadIdx.x] = centres[3 * j + 2];
    }
    __syncthreads();
    const int32_t len = min(kKnnBlock, n - base);
    for (int32_t t = 0; t < len; ++t) {
      if (base + t == i) continue;
      const double dx = sx[t] - px, dy = sy[t] - py, dz = sz[t] - pz;
      double x = fma(dx, dx, fma(dy, dy, dz * dz));
      if (x < best[KMAX - 1]) {
#pragma unroll
        for (int m = 0; m < KMAX; ++m) {
          const double lo = fmin(best[m], x);
          x = fmax(best[m], x);
          best[m] = lo;
        }
      }
    }
    __syncthreads();
  }
  if (i < n) {
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < KMAX; ++m)
      if (m < k) s += sqrt(best[m]);
    per_camera[i] = s / static_cast<double>(k);
  }
}

__global__ __launch_bounds__(kKnnBlock) void camera_mean_kernel(const double* __restrict__ per_camera,
                                                               int32_t n, double* __restrict__ mean) {
  __shared__ double part[kKnnBlock];
  double s = 0.0;
  for (int32_t i = static_cast<int32_t>(threadIdx.x); i < n; i += kKnnBlock) s += per_camera[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = kKnnBlock / 2; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) mean[0] = part[0] / static_cast<double>(n);
}

template <int KMAX>
static hipError_t launch_knn(const double* c, int32_t n, int32_t k, double* per, hipStream_t s) {
  const int grid = (n + kKnnBlock - 1) / kKnnBlock;
  hipLaunchKernelGGL((camera_knn_kernel<KMAX>), dim3(grid), dim3(kKnnBlock), 0, s, c, n, k, per);
  return hipGetLastError();
}

}  // namespace nasg

extern "C" int nasg_camera_knn(const double* centres, int32_t n_cams, int32_t k,
                               double* per_camera, double* mean, void* stream) {
  if (k < 1 || k > NASG_KNN_MAX_K || n_cams <= k || n_cams > NASG_KNN_MAX_CAMERAS)
    return NASG_ERR_SHAPE;
  if (centres == nullptr || per_camera == nullptr || mean == nullptr) return NASG_ERR_NULL;
  if ((reinterpret_cast<uintptr_t>(centres) & 7) != 0 ||
      (reinterpret_cast<uintptr_t>(per_camera) & 7) != 0 ||
      (reinterpret_cast<uintptr_t>(mean) & 7) != 0)
    return NASG_ERR_ALIGN;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (k <= 1) {
    e = nasg::launch_knn<1>(centres, n_cams, k, per_camera, s);
  } else if (k <= 2) {
    e = nasg::launch_knn<2>(centres, n_cams, k, per_camera, s);
  } else if (k <= 4) {
    e = nasg::launch_knn<4>(centres, n_cams, k, per_camera, s);
  } else if (k <= 8) {
    e = nasg::launch_knn<8>(centres, n_cams, k, per_camera, s);
  } else if (k <= 16) {
    e = nasg::launch_knn<16>(centres, n_cams, k, per_camera, s);
  } else {
    e = nasg::launch_knn<32>(centres, n_cams, k, per_camera, s);
  }
  if (e != hipSuccess) return NASG_ERR_LAUNCH;
  hipLaunchKernelGGL(nasg::camera_mean_kernel, dim3(1), dim3(nasg::kKnnBlock), 0, s,
                     per_camera, n_cams, mean);
  return hipGetLastError() == hipSuccess ? NASG_OK : NASG_ERR_LAUNCH;
}
