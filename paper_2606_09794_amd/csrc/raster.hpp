// Host/device contract of the compositing kernels (raster_kernels.hip):
// launch arguments and the per-primitive projection record kept in the
// caller's workspace between the forward and the backward call.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nasg {

constexpr int kTile = 16;              // tile edge in pixels (one 256-thread block)
constexpr int kMaxTileCapacity = 4096; // entries per tile list (sorted in 32 KiB of LDS)
constexpr int kAccStride = 10;         // FP64 accumulators per primitive: dL/dc (3),
                                       // dL/dsigma, dL/d(u, v, a, b, c), one spare

// What the render kernels read of a primitive, in one 64-byte record (so a
// tile's staging gathers one line per entry): pixel-space mean, conic with
// q = a dx^2 + b2 dx dy + c dy^2 (b2 = twice the off-diagonal), colour,
// opacity and the q <= 9 ellipse's half-extents rounded outward.
struct RenderRec {
  double u, v;
  double a, b2, c;
  float c0, c1, c2, sigma;
  float ex, ey;
};
static_assert(sizeof(RenderRec) == 64, "render record is one 64-byte line");

// What binning and sorting read: the camera depth of the mean (sort key) and
// the inclusive tile range touched (empty when tx0 > tx1).
struct BinRec {
  double z;
  int16_t tx0, tx1, ty0, ty1;
};
static_assert(sizeof(BinRec) == 16, "bin record is 16 bytes");

// Written into the workspace header by the forward; the backward checks it
// before reading any tile list, so a workspace without a forward of the same
// sizes is never indexed with stale entries.
struct RasterStamp {
  uint32_t magic;
  int32_t cap, tiles_x, tiles_y;
  int64_t n;
};
constexpr uint32_t kStampMagic = 0x4e534731u;

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
  int32_t* overflow;    // header byte 0: a tile list overflowed (forward)
  int32_t* stale;       // header byte 4: the backward found no matching forward
  RasterStamp* stamp;   // header byte 16
  int32_t* cursor;   // [tiles]
  uint64_t* lists;   // [tiles][cap] keys: float32 depth bits << 32 | primitive index
  RenderRec* rec;    // [N]
  BinRec* bins;      // [N]
  double* pix_state; // [H][W][2] forward's final transmittance t and exponent E (T = t 2^E)
  double* grad_acc;  // [N][kAccStride] backward accumulators
  // forward output / backward inputs and outputs
  float* image_out;         // [H][W][3]
  const float* grad_image;  // [H][W][3]
  float* grad_colors;       // [N][3] or null
  float* grad_opac;         // [N] or null
  float* grad_means;        // [N][3] or null
  float* grad_scales;       // [N][3] or null
  float* grad_rots;         // [N][4] or null
};

hipError_t launch_raster(const RasterArgs& a, bool bwd, hipStream_t s);

// One-thread copy of a device int32 (the overflow flag out of a workspace).
hipError_t launch_copy_flag(const int32_t* src, int32_t* dst, hipStream_t s);

}  // namespace nasg
