// C ABI of libnasg: host-side argument validation, launch-configuration
// choice (built-in heuristic or a caller-supplied tuning table) and dispatch
// to the HIP kernels. No allocation, synchronisation or host<->device copy
// happens here, so every evaluation call can be captured into a hipGraph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/nasg.h"
#include "nasg_launch.hpp"
#include "raster.hpp"

namespace {

using nasg::NasgArgs;
using nasg::ShArgs;

bool aligned(const void* p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

struct Key {
  int32_t kernel, k, v, dtype;
  bool operator<(const Key& o) const {
    return std::tie(kernel, k, v, dtype) < std::tie(o.kernel, o.k, o.v, o.dtype);
  }
};

std::map<Key, nasg_tuning>& tuning_table() {
  static std::map<Key, nasg_tuning> t;
  return t;
}

bool supported(int lanes, int vpl, int bcast) {
  if (bcast == 1) {
#define NASG_OK_BC(P_, V_) \
    if (lanes == P_ && vpl == V_) return true;
    NASG_FOR_EACH_BCAST_CONFIG(NASG_OK_BC)
#undef NASG_OK_BC
    return false;
  }
  if (bcast != 0) return false;
#define NASG_OK_CASE(P_, V_) \
  if (lanes == P_ && vpl == V_) return true;
  NASG_FOR_EACH_CONFIG(NASG_OK_CASE)
#undef NASG_OK_CASE
  return false;
}

bool block_ok(int b) { return b == 64 || b == 128 || b == 256; }

// Built-in choice when no tuning entry exists (the tuner's picks at K = 8 on
// MI355X): one lane per primitive up to four views (no slot transfers, and
// no more view slots than views), then four lanes with two or four views
// each, so that a lane evaluates several independent lobe-views per step
// within the registers of two waves per SIMD.
nasg_tuning heuristic(int32_t v) {
  if (v <= 1) return {1, 1, 256, 0};
  if (v <= 2) return {1, 2, 256, 0};
  if (v <= 4) return {1, 4, 256, 0};
  if (v <= 8) return {4, 2, 128, 0};
  return {4, 4, 128, 0};
}

nasg_tuning choose(int32_t kernel, int32_t k, int32_t v, int32_t dtype) {
  const auto& tab = tuning_table();
  auto it = tab.find(Key{kernel, kernel >= 2 ? 0 : k, v, kernel >= 2 ? 0 : dtype});
  if (it != tab.end()) return it->second;
  return heuristic(v);
}

int check_views(const nasg_views* vw, int64_t n) {
  if (vw == nullptr) return NASG_ERR_NULL;
  if (vw->v < 1 || vw->v > NASG_MAX_VIEWS) return NASG_ERR_SHAPE;
  if (n == 0) return NASG_OK;
  if (vw->dirs != nullptr) {
    if (vw->v != 1) return NASG_ERR_SHAPE;
    if (!aligned(vw->dirs, 4)) return NASG_ERR_ALIGN;
  } else {
    if (vw->means == nullptr || vw->cams == nullptr) return NASG_ERR_NULL;
    if (!aligned(vw->means, 4) || !aligned(vw->cams, 4)) return NASG_ERR_ALIGN;
  }
  return NASG_OK;
}

int check_params(const nasg_params* p) {
  if (p == nullptr) return NASG_ERR_NULL;
  if (p->n < 0 || p->k < 1 || p->k > NASG_MAX_LOBES) return NASG_ERR_SHAPE;
  if (p->dtype != NASG_F32 && p->dtype != NASG_BF16) return NASG_ERR_DTYPE;
  if (p->param != NASG_PARAM_QUAT && p->param != NASG_PARAM_ANGLES) return NASG_ERR_MODE;
  if (p->family < NASG_FAMILY_NASGABOR || p->family > NASG_FAMILY_ASG) return NASG_ERR_MODE;
  if (p->param == NASG_PARAM_ANGLES && p->family > NASG_FAMILY_NASG) return NASG_ERR_MODE;
  if (p->n == 0) return NASG_OK;  // nothing is read: pointers may be NULL
  if (p->quat == nullptr || p->shape == nullptr || p->rgbw == nullptr || p->c0 == nullptr)
    return NASG_ERR_NULL;
  const uintptr_t a4 = p->dtype == NASG_F32 ? 16 : 8;
  const uintptr_t a1 = p->dtype == NASG_F32 ? 4 : 2;
  if (!aligned(p->quat, a4) || !aligned(p->shape, a4) || !aligned(p->rgbw, a1) ||
      !aligned(p->c0, 4))
    return NASG_ERR_ALIGN;
  return NASG_OK;
}

NasgArgs make_args(const nasg_params* p, const nasg_views* vw) {
  NasgArgs a{};
  a.quat = p->quat;
  a.shape = p->shape;
  a.rgbw = p->rgbw;
  a.c0 = p->c0;
  a.means = vw->dirs ? nullptr : vw->means;
  a.cams = vw->dirs ? nullptr : vw->cams;
  a.dirs = vw->dirs;
  a.n = p->n;
  a.k = p->k;
  a.v = vw->v;
  a.param = p->param;
  a.family = p->family;
  return a;
}

int check_grad_ptrs(const float* grad_rgb, const nasg_grads* g, const float* rgb) {
  if (grad_rgb == nullptr || g == nullptr) return NASG_ERR_NULL;
  if (!aligned(grad_rgb, 4) || (rgb && !aligned(rgb, 4)) || (g->quat && !aligned(g->quat, 16)) ||
      (g->shape && !aligned(g->shape, 16)) || (g->rgbw && !aligned(g->rgbw, 4)) ||
      (g->c0 && !aligned(g->c0, 4)) || (g->geom && !aligned(g->geom, 4)))
    return NASG_ERR_ALIGN;
  return NASG_OK;
}

// ---- persistent batches
// A scene's lane mapping in the persistent batch: the tuning table's choice
// for its (K, V) when the batch kernel carries that mapping, else the
// smallest view chunk that holds its views ((1, 1), (1, 2), (1, 4), (4, 2),
// (4, 4) for V = 1, 2, 3..4, 5..8, more); plus kBatchVariants for the paper's
// raw values.
int batch_variant(int32_t k, int32_t v, int32_t param) {
  int var = v <= 1 ? 0 : v <= 2 ? 1 : v <= 4 ? 2 : v <= 8 ? 3 : 4;
  const auto& tab = tuning_table();
  const auto it = tab.find(Key{1, k, v, NASG_F32});   // kernel 1: the NASG backward
  if (it != tab.end() && it->second.bcast == 0) {
    for (int c = 0; c < nasg::kBatchVariants; ++c)
      if (nasg::kBatchLanes[c] == it->second.lanes &&
          nasg::kBatchViewsPerLane[c] == it->second.views_per_lane)
        var = c;
  }
  return var + (param == NASG_PARAM_ANGLES ? nasg::kBatchVariants : 0);
}

struct BatchLayout {
  size_t items_off;
  size_t total;
  int64_t n_items;
};

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

BatchLayout batch_layout(const nasg_scene* sc, int32_t n, int32_t tile_iters) {
  BatchLayout L{};
  L.items_off = align_up(sizeof(nasg::BatchHeader) + sizeof(nasg::BatchScene) * n, 64);
  for (int32_t s = 0; s < n; ++s) {
    const int64_t tile = static_cast<int64_t>(tile_iters) * (256 / nasg::kBatchLanes[batch_variant(sc[s].p.k, sc[s].views.v, sc[s].p.param)]);
    L.n_items += (sc[s].p.n + tile - 1) / tile;
  }
  L.total = L.items_off + sizeof(nasg::BatchItem) * static_cast<size_t>(L.n_items);
  return L;
}

nasg_batch_tuning batch_defaults(const nasg_batch_tuning* t) {
  return t ? *t : nasg_batch_tuning{4, 2};
}

// ---- compositing
struct RasterLayout {
  int32_t tiles_x, tiles_y;
  size_t cursor_off, lists_off, rec_off, bins_off, image_off, acc_off, total;
};

bool raster_layout(int64_t n, const nasg_camera* cam, int32_t cap, RasterLayout* L) {
  if (cam == nullptr || n < 0 || n > INT32_MAX || cap < 1 || cap > NASG_MAX_TILE_CAPACITY ||
      cam->width < 1 || cam->height < 1 || cam->width > NASG_MAX_IMAGE_SIDE ||
      cam->height > NASG_MAX_IMAGE_SIDE)
    return false;
  L->tiles_x = (cam->width + nasg::kTile - 1) / nasg::kTile;
  L->tiles_y = (cam->height + nasg::kTile - 1) / nasg::kTile;
  const size_t tiles = static_cast<size_t>(L->tiles_x) * L->tiles_y;
  L->cursor_off = 256;
  L->lists_off = align_up(L->cursor_off + 4 * tiles, 256);
  L->rec_off = align_up(L->lists_off + 8 * tiles * static_cast<size_t>(cap), 256);
  L->bins_off = align_up(L->rec_off + sizeof(nasg::RenderRec) * static_cast<size_t>(n), 256);
  L->image_off = align_up(L->bins_off + sizeof(nasg::BinRec) * static_cast<size_t>(n), 256);
  L->acc_off = align_up(L->image_off + 2 * sizeof(double) * static_cast<size_t>(cam->width) *
                                           static_cast<size_t>(cam->height),
                        256);
  L->total = L->acc_off + nasg::kAccStride * sizeof(double) * static_cast<size_t>(n);
  return true;
}

int raster_args(const nasg_gaussians* g, const nasg_camera* cam, int32_t cap, const void* ws,
                size_t ws_bytes, nasg::RasterArgs* a) {
  if (g == nullptr || cam == nullptr) return NASG_ERR_NULL;
  RasterLayout L{};
  if (!raster_layout(g->n, cam, cap, &L)) return NASG_ERR_SHAPE;
  if (ws == nullptr) return NASG_ERR_NULL;
  if (ws_bytes < L.total) return NASG_ERR_WORKSPACE;
  if (!aligned(ws, 256)) return NASG_ERR_ALIGN;
  if (g->n > 0) {
    if (!g->means || !g->scales || !g->rots || !g->opac || !g->colors) return NASG_ERR_NULL;
    if (!aligned(g->means, 4) || !aligned(g->scales, 4) || !aligned(g->rots, 4) ||
        !aligned(g->opac, 4) || !aligned(g->colors, 4))
      return NASG_ERR_ALIGN;
  }
  *a = nasg::RasterArgs{};
  a->means = g->means;
  a->scales = g->scales;
  a->rots = g->rots;
  a->opac = g->opac;
  a->colors = g->colors;
  a->n = g->n;
  for (int i = 0; i < 9; ++i) a->cam_rot[i] = cam->rot[i];
  for (int i = 0; i < 3; ++i) a->cam_t[i] = cam->t[i];
  a->fx = cam->fx;
  a->fy = cam->fy;
  a->cx = cam->cx;
  a->cy = cam->cy;
  a->width = cam->width;
  a->height = cam->height;
  a->tiles_x = L.tiles_x;
  a->tiles_y = L.tiles_y;
  a->cap = cap;
  unsigned char* base = static_cast<unsigned char*>(const_cast<void*>(ws));
  a->overflow = reinterpret_cast<int32_t*>(base);
  a->stale = reinterpret_cast<int32_t*>(base + 4);
  a->stamp = reinterpret_cast<nasg::RasterStamp*>(base + 16);
  a->cursor = reinterpret_cast<int32_t*>(base + L.cursor_off);
  a->lists = reinterpret_cast<uint64_t*>(base + L.lists_off);
  a->rec = reinterpret_cast<nasg::RenderRec*>(base + L.rec_off);
  a->bins = reinterpret_cast<nasg::BinRec*>(base + L.bins_off);
  a->pix_state = reinterpret_cast<double*>(base + L.image_off);
  a->grad_acc = reinterpret_cast<double*>(base + L.acc_off);
  return NASG_OK;
}

}  // namespace

// ---- compositing forward without allocation
// The workspace of nasg_raster_fwd_noalloc: a file-scope device array, one per
// GPU the library runs on, held until the process ends. In host code its name
// is only a stand-in; the device address comes from hipGetSymbolAddress, taken
// once per device with that device current.
static __device__ __align__(256) unsigned char scratch[NASG_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxScratchDevices = 64;

struct ScratchSlot {
  std::once_flag once;
  void* ptr = nullptr;
  hipError_t err = hipSuccess;
};

ScratchSlot& scratch_slot(int dev) {
  static ScratchSlot slots[kMaxScratchDevices];
  return slots[dev];
}

// Device address of this GPU's scratch array (the current device's).
void* device_scratch() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxScratchDevices) return nullptr;
  ScratchSlot& sl = scratch_slot(dev);
  std::call_once(sl.once, [&sl] {
    void* p = nullptr;
    sl.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    sl.ptr = sl.err == hipSuccess ? p : nullptr;
  });
  return sl.ptr;
}

}  // namespace

extern "C" {

const char* nasg_status_string(int status) {
  switch (status) {
    case NASG_OK: return "ok";
    case NASG_ERR_NULL: return "required pointer is NULL";
    case NASG_ERR_SHAPE: return "invalid size (n, k or v)";
    case NASG_ERR_ALIGN: return "pointer misaligned for its layout";
    case NASG_ERR_DTYPE: return "unknown storage dtype";
    case NASG_ERR_MODE: return "unknown normaliser or gradient mode";
    case NASG_ERR_LAUNCH: return "kernel launch failed";
    case NASG_ERR_WORKSPACE: return "workspace missing, too small or stale";
    default: return "unknown status";
  }
}

int nasg_set_tuning(int32_t kernel, int32_t k, int32_t v, int32_t dtype, const nasg_tuning* t) {
  if (kernel < 0 || kernel > 3) return NASG_ERR_MODE;
  if (t == nullptr) return NASG_ERR_NULL;
  const Key key{kernel, kernel >= 2 ? 0 : k, v, kernel >= 2 ? 0 : dtype};
  if (t->lanes == 0) {
    tuning_table().erase(key);
    return NASG_OK;
  }
  if (!supported(t->lanes, t->views_per_lane, t->bcast) || !block_ok(t->block) ||
      (kernel >= 2 && t->bcast != 0))
    return NASG_ERR_SHAPE;
  tuning_table()[key] = *t;
  return NASG_OK;
}

int nasg_get_tuning(int32_t kernel, int32_t k, int32_t v, int32_t dtype, nasg_tuning* t) {
  if (kernel < 0 || kernel > 3) return NASG_ERR_MODE;
  if (t == nullptr) return NASG_ERR_NULL;
  *t = choose(kernel, k, v, dtype);
  return NASG_OK;
}

int nasg_eval_fwd(const nasg_params* p, const nasg_views* views, float* rgb, int32_t norm,
                  void* stream) {
  int st = check_params(p);
  if (st != NASG_OK) return st;
  if ((st = check_views(views, p->n)) != NASG_OK) return st;
  if (norm != NASG_NORM_EXACT && norm != NASG_NORM_APPROX) return NASG_ERR_MODE;
  if (p->n == 0) return NASG_OK;
  if (rgb == nullptr) return NASG_ERR_NULL;
  if (!aligned(rgb, 4)) return NASG_ERR_ALIGN;
  NasgArgs a = make_args(p, views);
  a.rgb = rgb;
  a.norm = norm;
  const nasg_tuning t = choose(0, p->k, views->v, p->dtype);
  const hipError_t e = nasg::launch_nasg(a, t.lanes, t.views_per_lane, t.bcast != 0, false,
                                         p->dtype == NASG_BF16, t.block,
                                         static_cast<hipStream_t>(stream));
  return e == hipSuccess ? NASG_OK : NASG_ERR_LAUNCH;
}

int nasg_eval_bwd(const nasg_params* p, const nasg_views* views, const float* grad_rgb,
                  const nasg_grads* g, float* rgb, int32_t norm, int32_t grad_mode,
                  void* stream) {
  int st = check_params(p);
  if (st != NASG_OK) return st;
  if ((st = check_views(views, p->n)) != NASG_OK) return st;
  if (norm != NASG_NORM_EXACT && norm != NASG_NORM_APPROX) return NASG_ERR_MODE;
  if (grad_mode != NASG_GRAD_OVERWRITE && grad_mode != NASG_GRAD_ACCUMULATE) return NASG_ERR_MODE;
  if (g == nullptr) return NASG_ERR_NULL;
  if (p->n == 0) return NASG_OK;
  if ((st = check_grad_ptrs(grad_rgb, g, rgb)) != NASG_OK) return st;
  NasgArgs a = make_args(p, views);
  a.grad_rgb = grad_rgb;
  a.rgb = rgb;
  a.g_quat = g->quat;
  a.g_shape = g->shape;
  a.g_rgbw = g->rgbw;
  a.g_c0 = g->c0;
  a.g_geom = g->geom;
  a.norm = norm;
  a.accumulate = grad_mode == NASG_GRAD_ACCUMULATE;
  const nasg_tuning t = choose(1, p->k, views->v, p->dtype);
  const hipError_t e = nasg::launch_nasg(a, t.lanes, t.views_per_lane, t.bcast != 0, true,
                                         p->dtype == NASG_BF16, t.block,
                                         static_cast<hipStream_t>(stream));
  return e == hipSuccess ? NASG_OK : NASG_ERR_LAUNCH;
}

int sh3_eval_fwd(const float* sh, int64_t n, const nasg_views* views, float* rgb, void* stream) {
  if (n < 0) return NASG_ERR_SHAPE;
  int st = check_views(views, n);
  if (st != NASG_OK) return st;
  if (n == 0) return NASG_OK;
  if (sh == nullptr || rgb == nullptr) return NASG_ERR_NULL;
  if (!aligned(sh, 4) || !aligned(rgb, 4)) return NASG_ERR_ALIGN;
  if (n == 0) return NASG_OK;
  ShArgs a{};
  a.sh = sh;
  a.means = views->dirs ? nullptr : views->means;
  a.cams = views->dirs ? nullptr : views->cams;
  a.dirs = views->dirs;
  a.rgb = rgb;
  a.n = n;
  a.v = views->v;
  const nasg_tuning t = choose(2, 0, views->v, 0);
  const hipError_t e = nasg::launch_sh(a, t.lanes, t.views_per_lane, false, t.block,
                                       static_cast<hipStream_t>(stream));
  return e == hipSuccess ? NASG_OK : NASG_ERR_LAUNCH;
}

int sh3_eval_bwd(const float* sh, int64_t n, const nasg_views* views, const float* grad_rgb,
                 float* grad_sh, float* grad_geom, float* rgb, int32_t grad_mode, void* stream) {
  if (n < 0) return NASG_ERR_SHAPE;
  int st = check_views(views, n);
  if (st != NASG_OK) return st;
  if (grad_mode != NASG_GRAD_OVERWRITE && grad_mode != NASG_GRAD_ACCUMULATE) return NASG_ERR_MODE;
  if (n == 0) return NASG_OK;
  if (sh == nullptr || grad_rgb == nullptr) return NASG_ERR_NULL;
  if (!aligned(sh, 4) || !aligned(grad_rgb, 4) || (grad_sh && !aligned(grad_sh, 4)) ||
      (grad_geom && !aligned(grad_geom, 4)) || (rgb && !aligned(rgb, 4)))
    return NASG_ERR_ALIGN;
  if (n == 0) return NASG_OK;
  ShArgs a{};
  a.sh = sh;
  a.means = views->dirs ? nullptr : views->means;
  a.cams = views->dirs ? nullptr : views->cams;
  a.dirs = views->dirs;
  a.grad_rgb = grad_rgb;
  a.rgb = rgb;
  a.g_sh = grad_sh;
  a.g_geom = grad_geom;
  a.n = n;
  a.v = views->v;
  a.accumulate = grad_mode == NASG_GRAD_ACCUMULATE;
  const nasg_tuning t = choose(3, 0, views->v, 0);
  const hipError_t e = nasg::launch_sh(a, t.lanes, t.views_per_lane, true, t.block,
                                       static_cast<hipStream_t>(stream));
  return e == hipSuccess ? NASG_OK : NASG_ERR_LAUNCH;
}

size_t nasg_batched_workspace_bytes(const nasg_scene* scenes, int32_t n_scenes,
                                    const nasg_batch_tuning* t) {
  if (n_scenes < 0 || (n_scenes > 0 && scenes == nullptr)) return 0;
  const nasg_batch_tuning tt = batch_defaults(t);
  if (tt.tile_iters < 1 || tt.tile_iters > 64) return 0;
  for (int32_t s = 0; s < n_scenes; ++s)
    if (scenes[s].p.n < 0 || scenes[s].views.v < 1) return 0;
  return batch_layout(scenes, n_scenes, tt.tile_iters).total;
}

int nasg_batched_plan(const nasg_scene* scenes, int32_t n_scenes, int32_t norm,
                      const nasg_batch_tuning* t, void* workspace, size_t ws_bytes,
                      nasg_batch* out, void* stream) {
  if (out == nullptr || (n_scenes > 0 && scenes == nullptr)) return NASG_ERR_NULL;
  if (n_scenes < 0) return NASG_ERR_SHAPE;
  if (norm != NASG_NORM_EXACT && norm != NASG_NORM_APPROX) return NASG_ERR_MODE;
  const nasg_batch_tuning tt = batch_defaults(t);
  if (tt.tile_iters < 1 || tt.tile_iters > 64 || tt.blocks_per_cu < 1 || tt.blocks_per_cu > 8)
    return NASG_ERR_SHAPE;
  for (int32_t s = 0; s < n_scenes; ++s) {
    const nasg_scene& sc = scenes[s];
    int st = check_params(&sc.p);
    if (st != NASG_OK) return st;
    if (sc.p.dtype != NASG_F32) return NASG_ERR_DTYPE;
    if (sc.p.family != NASG_FAMILY_NASGABOR) return NASG_ERR_MODE;
    if ((st = check_views(&sc.views, sc.p.n)) != NASG_OK) return st;
    if (sc.p.n > 0 && (st = check_grad_ptrs(sc.grad_rgb, &sc.g, sc.rgb)) != NASG_OK) return st;
  }
  const BatchLayout L = batch_layout(scenes, n_scenes, tt.tile_iters);
  if (L.n_items > INT32_MAX) return NASG_ERR_SHAPE;
  if (workspace == nullptr) return NASG_ERR_WORKSPACE;
  if (!aligned(workspace, 64) || ws_bytes < L.total) return NASG_ERR_WORKSPACE;

  static std::atomic<uint64_t> serial{0};
  const uint64_t token =
      (static_cast<uint64_t>(std::chrono::steady_clock::now().time_since_epoch().count()) << 16) ^
      (++serial);

  std::vector<unsigned char> host(L.total, 0);
  auto* hdr = reinterpret_cast<nasg::BatchHeader*>(host.data());
  hdr->token = token;
  hdr->n_items = static_cast<int32_t>(L.n_items);
  hdr->n_scenes = n_scenes;
  hdr->counter = 0;
  auto* bs = reinterpret_cast<nasg::BatchScene*>(host.data() + sizeof(nasg::BatchHeader));
  struct Tile {
    double cost;
    nasg::BatchItem item;
  };
  std::vector<Tile> tiles;
  tiles.reserve(static_cast<size_t>(L.n_items));
  for (int32_t s = 0; s < n_scenes; ++s) {
    const nasg_scene& sc = scenes[s];
    NasgArgs a = make_args(&sc.p, &sc.views);
    a.grad_rgb = sc.grad_rgb;
    a.rgb = sc.rgb;
    a.g_quat = sc.g.quat;
    a.g_shape = sc.g.shape;
    a.g_rgbw = sc.g.rgbw;
    a.g_c0 = sc.g.c0;
    a.g_geom = sc.g.geom;
    a.norm = norm;
    a.accumulate = 0;
    bs[s].args = a;
    bs[s].variant = batch_variant(sc.p.k, sc.views.v, sc.p.param);
    bs[s].tile_iters = tt.tile_iters;
    const int64_t tile = static_cast<int64_t>(tt.tile_iters) * (256 / nasg::kBatchLanes[bs[s].variant]);
    for (int64_t st0 = 0; st0 < sc.p.n; st0 += tile) {
      const int64_t cnt = std::min(tile, sc.p.n - st0);
      tiles.push_back({static_cast<double>(cnt) * sc.p.k * std::max(1, sc.views.v),
                       nasg::BatchItem{s, 0, st0}});
    }
  }
  // the layout counted the tiles with the same lane mappings (a tuning change
  // between the two counts, from another thread, would show here)
  if (static_cast<int64_t>(tiles.size()) != L.n_items) return NASG_ERR_SHAPE;
  std::stable_sort(tiles.begin(), tiles.end(),
                   [](const Tile& x, const Tile& y) { return x.cost > y.cost; });
  auto* items = reinterpret_cast<nasg::BatchItem*>(host.data() + L.items_off);
  for (size_t k = 0; k < tiles.size(); ++k) items[k] = tiles[k].item;

  hipStream_t hs = static_cast<hipStream_t>(stream);
  if (hipMemcpyAsync(workspace, host.data(), L.total, hipMemcpyHostToDevice, hs) != hipSuccess)
    return NASG_ERR_LAUNCH;
  if (hipStreamSynchronize(hs) != hipSuccess) return NASG_ERR_LAUNCH;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return NASG_ERR_LAUNCH;
  out->workspace = workspace;
  out->bytes = L.total;
  out->n_items = static_cast<int32_t>(L.n_items);
  out->n_scenes = n_scenes;
  out->grid = std::max(1, cus * tt.blocks_per_cu);
  out->norm = norm;
  out->token = token;
  out->raw = 0;
  for (int32_t s = 0; s < n_scenes; ++s)
    if (bs[s].variant >= nasg::kBatchVariants) out->raw = 1;
  out->pad = 0;
  return NASG_OK;
}

int nasg_batched_run(const nasg_batch* b, void* stream) {
  if (b == nullptr || b->workspace == nullptr) return NASG_ERR_NULL;
  if (b->n_scenes < 0 || b->n_items < 0 || b->grid < 1 || (b->raw != 0 && b->raw != 1))
    return NASG_ERR_WORKSPACE;
  if (b->n_items == 0) return NASG_OK;
  auto* base = static_cast<unsigned char*>(b->workspace);
  auto* hdr = reinterpret_cast<nasg::BatchHeader*>(base);
  auto* scenes = reinterpret_cast<const nasg::BatchScene*>(base + sizeof(nasg::BatchHeader));
  const size_t items_off =
      align_up(sizeof(nasg::BatchHeader) + sizeof(nasg::BatchScene) * b->n_scenes, 64);
  auto* items = reinterpret_cast<const nasg::BatchItem*>(base + items_off);
  const hipError_t e = nasg::launch_batched(hdr, scenes, items, &hdr->counter, b->token, b->grid,
                                            b->raw != 0, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? NASG_OK : NASG_ERR_LAUNCH;
}

size_t nasg_raster_workspace_bytes(int64_t n, const nasg_camera* cam, int32_t tile_capacity) {
  RasterLayout L{};
  return raster_layout(n, cam, tile_capacity, &L) ? L.total : 0;
}

int nasg_raster_fwd(const nasg_gaussians* g, const nasg_camera* cam, int32_t tile_capacity,
                    void* workspace, size_t ws_bytes, float* image, void* stream) {
  nasg::RasterArgs a{};
  const int st = raster_args(g, cam, tile_capacity, workspace, ws_bytes, &a);
  if (st != NASG_OK) return st;
  if (image == nullptr) return NASG_ERR_NULL;
  if (!aligned(image, 4)) return NASG_ERR_ALIGN;
  a.image_out = image;
  return nasg::launch_raster(a, false, static_cast<hipStream_t>(stream)) == hipSuccess
             ? NASG_OK
             : NASG_ERR_LAUNCH;
}

int nasg_raster_fwd_noalloc(const nasg_gaussians* g, const nasg_camera* cam,
                            int32_t tile_capacity, float* image, int32_t* overflow,
                            void* stream) {
  if (g == nullptr || cam == nullptr) return NASG_ERR_NULL;
  RasterLayout L{};
  if (!raster_layout(g->n, cam, tile_capacity, &L)) return NASG_ERR_SHAPE;
  if (L.total > static_cast<size_t>(NASG_NOALLOC_SCRATCH_BYTES)) return NASG_ERR_WORKSPACE;
  if (image == nullptr) return NASG_ERR_NULL;
  if (!aligned(image, 4) || (overflow && !aligned(overflow, 4))) return NASG_ERR_ALIGN;
  // every argument is validated before the runtime is touched: the first
  // raster_args only checks and lays out (at a stand-in aligned address)
  nasg::RasterArgs a{};
  int st = raster_args(g, cam, tile_capacity, reinterpret_cast<const void*>(uintptr_t{256}),
                       NASG_NOALLOC_SCRATCH_BYTES, &a);
  if (st != NASG_OK) return st;
  void* ws = device_scratch();
  if (ws == nullptr) return NASG_ERR_LAUNCH;
  st = raster_args(g, cam, tile_capacity, ws, NASG_NOALLOC_SCRATCH_BYTES, &a);
  if (st != NASG_OK) return st;
  a.image_out = image;
  const hipStream_t hs = static_cast<hipStream_t>(stream);
  if (nasg::launch_raster(a, false, hs) != hipSuccess) return NASG_ERR_LAUNCH;
  if (overflow != nullptr && nasg::launch_copy_flag(a.overflow, overflow, hs) != hipSuccess)
    return NASG_ERR_LAUNCH;
  return NASG_OK;
}

int nasg_raster_bwd(const nasg_gaussians* g, const nasg_camera* cam, int32_t tile_capacity,
                    void* workspace, size_t ws_bytes, const float* grad_image,
                    float* grad_colors, float* grad_opac, float* grad_means,
                    float* grad_scales, float* grad_rots, void* stream) {
  nasg::RasterArgs a{};
  const int st = raster_args(g, cam, tile_capacity, workspace, ws_bytes, &a);
  if (st != NASG_OK) return st;
  if (grad_image == nullptr) return NASG_ERR_NULL;
  if (!aligned(grad_image, 4) || (grad_colors && !aligned(grad_colors, 4)) ||
      (grad_opac && !aligned(grad_opac, 4)) || (grad_means && !aligned(grad_means, 4)) ||
      (grad_scales && !aligned(grad_scales, 4)) || (grad_rots && !aligned(grad_rots, 4)))
    return NASG_ERR_ALIGN;
  a.grad_image = grad_image;
  a.grad_colors = grad_colors;
  a.grad_opac = grad_opac;
  a.grad_means = grad_means;
  a.grad_scales = grad_scales;
  a.grad_rots = grad_rots;
  return nasg::launch_raster(a, true, static_cast<hipStream_t>(stream)) == hipSuccess
             ? NASG_OK
             : NASG_ERR_LAUNCH;
}

}  // extern "C"
