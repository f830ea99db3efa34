// Host/device contract of the compositing kernels (raster_kernels.hip):
// launch arguments and the per-primitive projection record kept in the
// caller's workspace between the forward and the backward call.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nasg {

constexpr int kTile = 16;              // tile edge in pixels (one 256-thread block)
constexpr int kMaxTileCapacity = 4096; // entries per tile list (sorted in 32 KiB of LDS)

struct ProjRec {
  double u, v;        // pixel-space mean
  double a, b, c;     // inverse projected covariance: q = a dx^2 + 2 b dx dy + c dy^2
  double z;           // camera depth of the mean (sort key)
  float ex, ey;       // half-extents of the q <= 9 ellipse, rounded outward
  int16_t tx0, tx1;   // inclusive tile range touched (empty when tx0 > tx1)
  int16_t ty0, ty1;
};
static_assert(sizeof(ProjRec) == 64, "projection record is one 64-byte line");

struct RasterArgs {
  const float* means;   // [N][3]
  const float* scales;  // [N][3]
  const float* rots;    // [N][4]
  const float* opac;    // [N]
  const float* colors;  // [N][3]
  int64_t n;
  double cam_rot[9];
  double cam_t[3];
  double fx, fy, cx, cy;
  int32_t width, height;
  int32_t tiles_x, tiles_y;
  int32_t cap;
  // workspace views
  int32_t* overflow;
  int32_t* cursor;   // [tiles]
  uint64_t* lists;   // [tiles][cap] keys: float32 depth bits << 32 | primitive index
  ProjRec* proj;     // [N]
  double* pix_state; // [H][W][2] forward's final transmittance t and exponent E (T = t 2^E)
  double* grad_acc;  // [N][4] backward accumulators (dL/dc, dL/dsigma)
  // forward output / backward inputs and outputs
  float* image_out;         // [H][W][3]
  const float* grad_image;  // [H][W][3]
  float* grad_colors;       // [N][3] or null
  float* grad_opac;         // [N] or null
};

hipError_t launch_raster(const RasterArgs& a, bool bwd, hipStream_t s);

}  // namespace nasg
