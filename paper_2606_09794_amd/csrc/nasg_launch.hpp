// Kernel argument blocks and launchers shared by the kernels and the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nasg {

struct NasgArgs {
  const void* quat;
  const void* shape;
  const void* rgbw;
  const float* c0;
  const float* means;
  const float* cams;
  const float* dirs;
  const float* grad_rgb;
  float* rgb;
  float* g_quat;
  float* g_shape;
  float* g_rgbw;
  float* g_c0;
  float* g_geom;
  int64_t n;
  int32_t k;
  int32_t v;
  int32_t norm;
  int32_t accumulate;
  int32_t param;       // 0: quaternion + (lam, a, k, zeta); 1: the paper's raw values
  int32_t family;      // lobe family (kFam*)
};

constexpr int kParamQuat = 0;
constexpr int kParamAngles = 1;

// lobe families (the values of nasg_family)
constexpr int kFamNasgabor = 0;
constexpr int kFamNasg = 1;
constexpr int kFamSg = 2;
constexpr int kFamSb = 3;
constexpr int kFamSc = 4;
constexpr int kFamAsg = 5;

// The lane mappings compiled for the families other than NASGabor, by view
// count: (1, 1) for V = 1, (2, 2) up to 4, (4, 2) up to 8, (8, 2) above.
inline void family_mapping(int v, int& lanes, int& vpl) {
  if (v <= 1) { lanes = 1; vpl = 1; }
  else if (v <= 4) { lanes = 2; vpl = 2; }
  else if (v <= 8) { lanes = 4; vpl = 2; }
  else { lanes = 8; vpl = 2; }
}

struct ShArgs {
  const float* sh;
  const float* means;
  const float* cams;
  const float* dirs;
  const float* grad_rgb;
  float* rgb;
  float* g_sh;
  float* g_geom;
  int64_t n;
  int32_t v;
  int32_t accumulate;
};

// (lanes per primitive, views per lane) pairs compiled into the library.
#define NASG_FOR_EACH_CONFIG(X) \
  X(1, 1)                       \
  X(1, 2)                       \
  X(1, 4)                       \
  X(2, 1)                       \
  X(2, 2)                       \
  X(2, 4)                       \
  X(4, 1)                       \
  X(4, 2)                       \
  X(4, 4)                       \
  X(8, 1)                       \
  X(8, 2)                       \
  X(16, 1)

// (lanes per primitive, views per lane) pairs compiled with the views
// broadcast to every lane of the group (lanes own lobes, per-view sums reduced
// over the group): the mappings for few views.
#define NASG_FOR_EACH_BCAST_CONFIG(X) \
  X(4, 1)                             \
  X(8, 1)                             \
  X(16, 1)                            \
  X(8, 2)                             \
  X(8, 4)

// Persistent multi-scene launch: device-side plan layout (in the caller's
// workspace): BatchHeader | BatchScene[n_scenes] | BatchItem[n_items].
struct BatchHeader {
  uint64_t token;
  int32_t n_items;
  int32_t n_scenes;
  uint32_t counter;   // work-queue head, reset by every run
  int32_t pad[11];
};
static_assert(sizeof(BatchHeader) == 64, "batch header layout");

struct BatchScene {
  NasgArgs args;
  int32_t variant;     // lane mapping (lanes, views per lane): 0 = (1, 1), 1 = (1, 2),
                       // 2 = (1, 4), 3 = (4, 2), 4 = (4, 4); 5..9: the same for the
                       // paper's raw values
  int32_t tile_iters;
};

struct BatchItem {
  int32_t scene;
  int32_t pad;
  int64_t start;       // first primitive of the tile
};

constexpr int kBatchVariants = 5;   // lane mappings per parametrisation
constexpr int kBatchLanes[2 * kBatchVariants] = {1, 1, 1, 4, 4, 1, 1, 1, 4, 4};
constexpr int kBatchViewsPerLane[2 * kBatchVariants] = {1, 2, 4, 2, 4, 1, 2, 4, 2, 4};

hipError_t launch_batched(const BatchHeader* hdr, const BatchScene* scenes, const BatchItem* items,
                          uint32_t* counter, uint64_t token, int grid, bool raw, hipStream_t s);

// SG, SB, SC and ASG lobes (csrc/family_kernels.hip), lane mapping by view count.
hipError_t launch_family(const NasgArgs& a, bool bwd, bool bf16, int block, hipStream_t s);

hipError_t launch_nasg(const NasgArgs& a, int lanes, int vpl, bool bcast, bool bwd, bool bf16,
                       int block, hipStream_t s);
hipError_t launch_sh(const ShArgs& a, int lanes, int vpl, bool bwd, int block, hipStream_t s);

}  // namespace nasg
