// Compositing of the primitives' colours into an image for one camera
// (Section 3.1: C = sum_i T_i alpha_i c_i, alpha_i = sigma_i rho_i,
// T_i = prod_{j<i} (1 - alpha_j)), with the gradients of a loss on the image
// with respect to the per-primitive colours and opacities, which is what the
// appearance backward consumes.
//
// The primitives are 3D Gaussians (mean, per-axis scale, quaternion
// rotation); rho on a pixel's ray is the Gaussian projected onto the image
// plane (the local affine approximation of the perspective map at the mean),
// evaluated at the pixel centre. A primitive reaches a pixel only inside its
// 3-sigma ellipse and only in front of the near plane Z = 0.2; alpha is
// clamped at 0.99; the background is black.
//
// Pipeline (all on the caller's stream, nothing allocated, no host sync):
//   project : per primitive, FP64 pixel mean, inverse 2D covariance, depth and
//             the 16 x 16-pixel tiles its ellipse's bounding box touches;
//   bin     : each primitive appends itself to the lists of those tiles
//             (an atomic cursor per tile, fixed capacity per tile; entries
//             beyond it are dropped and flagged);
//   sort    : per tile, the list is sorted by (depth, primitive index) with
//             a bitonic network on 64-bit keys held in registers and LDS,
//             which fixes the compositing order;
//   render  : one block per tile, each lane one or more pixels of one column
//             (they share the entry's dx terms), front to back over the list
//             in chunks staged through LDS; an entry's q <= 9 box decides per
//             row band whether a wavefront looks at it at all. The support
//             test and the quadratic form are FP64 (so both sides of a
//             parity check take the same support decisions), rho = exp(-q/2)
//             is FP32, and the transmittance (with an explicit power-of-two
//             exponent) and the colour sum are FP64: with no early
//             termination a pixel may composite thousands of layers;
//   backward: back to front over the same list, with dC/dc_i = alpha_i T_i
//             and dC/dalpha_i = T_i (c_i - R_{i+1}), R the colour seen from
//             the next layer on in units of its transmittance, built by a
//             convex-combination recursion (no cancellation at any depth),
//             and T_i recovered from the forward's final transmittance. Per
//             primitive, a lane sums its pixels' terms, the wavefront
//             sums over lanes in registers, and one lane adds the sums to
//             FP64 per-primitive accumulators with one atomic per value; a
//             last kernel rounds the accumulators to the float32 outputs.
#include <hip/hip_runtime.h>

#include "../../include/nasg.h"
#include "nasg_device.hpp"
#include "raster.hpp"

namespace nasg {

constexpr double kNear = 0.2;
constexpr float kClamp = 0.99f;
constexpr double kSupport = 9.0;

__global__ void raster_zero(int32_t* cursor, int64_t n_tiles, int32_t* overflow) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < n_tiles) cursor[t] = 0;
  if (t == 0) *overflow = 0;
}

__global__ void raster_zero_acc(double* acc, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) {
    acc[4 * i + 0] = 0.0;
    acc[4 * i + 1] = 0.0;
    acc[4 * i + 2] = 0.0;
    acc[4 * i + 3] = 0.0;
  }
}

__global__ void raster_finish_grads(const double* acc, float* gc, float* go, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) {
    if (gc != nullptr) {
      gc[3 * i + 0] = static_cast<float>(acc[4 * i + 0]);
      gc[3 * i + 1] = static_cast<float>(acc[4 * i + 1]);
      gc[3 * i + 2] = static_cast<float>(acc[4 * i + 2]);
    }
    if (go != nullptr) go[i] = static_cast<float>(acc[4 * i + 3]);
  }
}

__global__ void raster_project(RasterArgs a) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  ProjRec rec{};
  rec.tx0 = 1;  // empty tile range unless the ellipse lands on the image
  rec.tx1 = 0;
  rec.ty0 = 1;
  rec.ty1 = 0;
  const double mx = a.means[3 * i], my = a.means[3 * i + 1], mz = a.means[3 * i + 2];
  const double* R = a.cam_rot;
  const double X = R[0] * mx + R[1] * my + R[2] * mz + a.cam_t[0];
  const double Y = R[3] * mx + R[4] * my + R[5] * mz + a.cam_t[1];
  const double Z = R[6] * mx + R[7] * my + R[8] * mz + a.cam_t[2];
  rec.z = Z;
  if (Z > kNear) {
    const double iz = 1.0 / Z;
    rec.u = a.fx * X * iz + a.cx;
    rec.v = a.fy * Y * iz + a.cy;
    // world rotation of the normalised quaternion
    double qw = a.rots[4 * i], qx = a.rots[4 * i + 1], qy = a.rots[4 * i + 2], qz = a.rots[4 * i + 3];
    const double qn = 1.0 / sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    qw *= qn;
    qx *= qn;
    qy *= qn;
    qz *= qn;
    const double Rw[9] = {1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy),
                          2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx),
                          2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)};
    const double s[3] = {a.scales[3 * i], a.scales[3 * i + 1], a.scales[3 * i + 2]};
    // M = J R_cw R_w S (2 x 3), projected covariance Sigma_2 = M M^T
    const double J0[3] = {a.fx * iz, 0.0, -a.fx * X * iz * iz};
    const double J1[3] = {0.0, a.fy * iz, -a.fy * Y * iz * iz};
    double A0[3], A1[3];
    for (int c = 0; c < 3; ++c) {
      A0[c] = J0[0] * R[c] + J0[1] * R[3 + c] + J0[2] * R[6 + c];
      A1[c] = J1[0] * R[c] + J1[1] * R[3 + c] + J1[2] * R[6 + c];
    }
    double m0[3], m1[3];
    for (int c = 0; c < 3; ++c) {
      m0[c] = (A0[0] * Rw[c] + A0[1] * Rw[3 + c] + A0[2] * Rw[6 + c]) * s[c];
      m1[c] = (A1[0] * Rw[c] + A1[1] * Rw[3 + c] + A1[2] * Rw[6 + c]) * s[c];
    }
    const double sxx = m0[0] * m0[0] + m0[1] * m0[1] + m0[2] * m0[2];
    const double sxy = m0[0] * m1[0] + m0[1] * m1[1] + m0[2] * m1[2];
    const double syy = m1[0] * m1[0] + m1[1] * m1[1] + m1[2] * m1[2];
    const double det = sxx * syy - sxy * sxy;
    if (det > 0.0) {
      const double id = 1.0 / det;
      rec.a = syy * id;
      rec.b = -sxy * id;
      rec.c = sxx * id;
      // q <= 9 implies |dx| <= 3 sqrt(sxx) and |dy| <= 3 sqrt(syy). The
      // float half-extents are rounded outward (relative 1e-5 plus 1e-2
      // pixel, far above the rounding of the inverse), and binning adds a
      // pixel more; pixel px has its centre at px + 1/2
      const double ex = 3.0 * sqrt(sxx), ey = 3.0 * sqrt(syy);
      rec.ex = static_cast<float>(ex * (1.0 + 1e-5) + 1e-2);
      rec.ey = static_cast<float>(ey * (1.0 + 1e-5) + 1e-2);
      const double px0 = fmax(rec.u - ex - 1.5, 0.0), px1 = fmin(rec.u + ex + 0.5, a.width - 1.0);
      const double py0 = fmax(rec.v - ey - 1.5, 0.0), py1 = fmin(rec.v + ey + 0.5, a.height - 1.0);
      if (px0 <= px1 && py0 <= py1) {
        rec.tx0 = static_cast<int16_t>(static_cast<int32_t>(px0) / kTile);
        rec.tx1 = static_cast<int16_t>(static_cast<int32_t>(px1) / kTile);
        rec.ty0 = static_cast<int16_t>(static_cast<int32_t>(py0) / kTile);
        rec.ty1 = static_cast<int16_t>(static_cast<int32_t>(py1) / kTile);
      }
    }
  }
  a.proj[i] = rec;
}

__global__ void raster_bin(RasterArgs a) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const ProjRec r = a.proj[i];
  for (int ty = r.ty0; ty <= r.ty1; ++ty) {
    for (int tx = r.tx0; tx <= r.tx1; ++tx) {
      const int64_t tile = static_cast<int64_t>(ty) * a.tiles_x + tx;
      const int32_t pos = atomicAdd(a.cursor + tile, 1);
      if (pos < a.cap) {
        a.lists[tile * a.cap + pos] = static_cast<int32_t>(i);
      } else {
        atomicMax(a.overflow, 1);
      }
    }
  }
}

// Per-tile depth sort. Key = (float32 of the FP64 depth, primitive index):
// rounding to float is monotone, so sorting the 64-bit keys orders the list
// by depth except inside runs of equal float depth, which a final pass puts
// in (FP64 depth, index) order; padding keys (all ones) sort last. Bitonic
// network over 256 EPT keys, EPT consecutive keys per thread in registers:
// strides below EPT are exchanged in registers, larger ones through LDS.
template <int EPT>
__device__ void bitonic_keys(uint64_t (&v)[EPT], uint64_t* lds) {
  constexpr int M = 256 * EPT;
  const int t = static_cast<int>(threadIdx.x);
  for (int k = 2; k <= M; k <<= 1) {
    for (int j = k >> 1; j >= EPT; j >>= 1) {
      __syncthreads();
#pragma unroll
      for (int r = 0; r < EPT; ++r) lds[t * EPT + r] = v[r];
      __syncthreads();
#pragma unroll
      for (int r = 0; r < EPT; ++r) {
        const int e = t * EPT + r, pe = e ^ j;
        const uint64_t o = lds[pe];
        const bool keep_min = ((e & k) == 0) == (e < pe);
        v[r] = keep_min ? (o < v[r] ? o : v[r]) : (o > v[r] ? o : v[r]);
      }
    }
#pragma unroll
    for (int jj = EPT / 2; jj >= 1; jj >>= 1) {
      if (jj < k) {
#pragma unroll
        for (int r = 0; r < EPT; ++r) {
          const int p = r ^ jj;
          if (p > r) {
            const bool up = ((t * EPT + r) & k) == 0;
            const uint64_t a = v[r], b = v[p];
            const uint64_t lo = a < b ? a : b, hi = a < b ? b : a;
            v[r] = up ? lo : hi;
            v[p] = up ? hi : lo;
          }
        }
      }
    }
  }
}

template <int EPT>
__device__ void sort_tile(const RasterArgs& a, int32_t* list, int cnt, uint64_t* lds) {
  const int t = static_cast<int>(threadIdx.x);
  uint64_t v[EPT];
#pragma unroll
  for (int r = 0; r < EPT; ++r) {
    const int e = t * EPT + r;
    if (e < cnt) {
      const int32_t idx = list[e];
      const float zf = __double2float_rn(a.proj[idx].z);  // z > 0.2: the bits are monotone
      v[r] = (static_cast<uint64_t>(__float_as_uint(zf)) << 32) | static_cast<uint32_t>(idx);
    } else {
      v[r] = ~0ull;
    }
  }
  bitonic_keys<EPT>(v, lds);
  __syncthreads();
#pragma unroll
  for (int r = 0; r < EPT; ++r) lds[t * EPT + r] = v[r];
  __syncthreads();
  // runs of equal float depth (already in index order): a stable insertion
  // sort by FP64 depth, done by the thread that owns the run's first entry
  for (int e = t; e < cnt; e += 256) {
    const uint32_t hi = static_cast<uint32_t>(lds[e] >> 32);
    const bool start = e == 0 || static_cast<uint32_t>(lds[e - 1] >> 32) != hi;
    if (!start || e + 1 >= cnt || static_cast<uint32_t>(lds[e + 1] >> 32) != hi) continue;
    int end = e + 1;
    while (end < cnt && static_cast<uint32_t>(lds[end] >> 32) == hi) ++end;
    for (int i = e + 1; i < end; ++i) {
      const uint64_t key = lds[i];
      const double z = a.proj[static_cast<uint32_t>(key)].z;
      int p = i - 1;
      while (p >= e && a.proj[static_cast<uint32_t>(lds[p])].z > z) {
        lds[p + 1] = lds[p];
        --p;
      }
      lds[p + 1] = key;
    }
  }
  __syncthreads();
  for (int e = t; e < cnt; e += 256) list[e] = static_cast<int32_t>(static_cast<uint32_t>(lds[e]));
}

__global__ __launch_bounds__(256) void raster_sort(RasterArgs a) {
  __shared__ uint64_t lds[256 * 16];
  const int64_t tile = blockIdx.x;
  const int cnt = min(a.cursor[tile], a.cap);
  if (cnt <= 1) return;
  int32_t* list = a.lists + tile * a.cap;
  if (cnt <= 256) {
    sort_tile<1>(a, list, cnt, lds);
  } else if (cnt <= 512) {
    sort_tile<2>(a, list, cnt, lds);
  } else if (cnt <= 1024) {
    sort_tile<4>(a, list, cnt, lds);
  } else if (cnt <= 2048) {
    sort_tile<8>(a, list, cnt, lds);
  } else {
    sort_tile<16>(a, list, cnt, lds);
  }
}

struct StageEntry {
  double u, v, a, b, c;
  float bx0, bx1, by0, by1;  // the entry's q <= 9 box in pixel coordinates (outward)
  float sigma, c0, c1, c2;
  int32_t idx;
  int32_t pad;
};

// Sum over the 64 lanes of a wavefront (every lane active): DPP row sums;
// row_bcast:15 adds row 0's sum into row 1 and row 2's into row 3;
// row_bcast:31 adds lane 31 (rows 0 + 1) into rows 2 and 3; lane 63 then
// holds the total, read out as a uniform value.
__device__ inline float wave_sum(float x) {
  x = group_sum<16>(x);
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x142, 0xA, 0xF, false));
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x143, 0xC, 0xF, false));
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

// Transmittance as t * 2^E (E a multiple of kRenorm, t kept away from the
// bottom of the double range), so a pixel behind thousands of layers keeps
// its exact value for the backward's recovery by division.
constexpr int kRenorm = 600;

__device__ inline void stage_entry(const RasterArgs& a, const int32_t* list, int e,
                                   StageEntry* slot) {
  const int32_t idx = list[e];
  const ProjRec r = a.proj[idx];
  StageEntry s;
  s.u = r.u;
  s.v = r.v;
  s.a = r.a;
  s.b = r.b;
  s.c = r.c;
  s.bx0 = static_cast<float>(r.u) - r.ex;
  s.bx1 = static_cast<float>(r.u) + r.ex;
  s.by0 = static_cast<float>(r.v) - r.ey;
  s.by1 = static_cast<float>(r.v) + r.ey;
  s.sigma = a.opac[idx];
  s.c0 = a.colors[3 * idx];
  s.c1 = a.colors[3 * idx + 1];
  s.c2 = a.colors[3 * idx + 2];
  s.idx = idx;
  s.pad = 0;
  *slot = s;
}

// Thread layout of the render kernels: a block of 256 / RPL threads per
// 16 x 16 tile; lane l of wavefront w owns column l & 15 and the RPL rows
// 4 RPL w + (l >> 4) + 4 j, j < RPL, so an entry's dx terms are shared by a
// lane's RPL pixels, and a wavefront skips a row band j (rows 4 RPL w + 4 j
// .. + 3) whose pixel-centre rows the entry's box misses.
// Rows per lane, measured on MI355X at 3 M primitives and 1920 x 1080: the
// forward is fastest at one pixel per thread (occupancy hides the LDS and
// FP64 latencies), the backward at two (the per-entry wavefront sums are
// shared by two pixels per lane while four would cost occupancy).
constexpr int kFwdRows = 1;
constexpr int kBwdRows = 2;

template <int RPL>
struct TileMap {
  int px, py0;               // the lane's column and first row
  float tx0, tx1;            // the tile's pixel-centre column range
  float ty0;                 // pixel-centre row of the wavefront's first band
  bool in_x;
  int height;
};

template <int RPL>
__device__ inline TileMap<RPL> tile_map(const RasterArgs& a, int64_t tile) {
  TileMap<RPL> m;
  const int tx = static_cast<int>(tile % a.tiles_x), ty = static_cast<int>(tile / a.tiles_x);
  const int lane = static_cast<int>(threadIdx.x) & 63, wave = static_cast<int>(threadIdx.x) >> 6;
  const int row0 = ty * kTile + 4 * RPL * wave;
  m.px = tx * kTile + (lane & 15);
  m.py0 = row0 + (lane >> 4);
  m.tx0 = tx * kTile + 0.5f;
  m.tx1 = tx * kTile + 15.5f;
  m.ty0 = row0 + 0.5f;
  m.in_x = m.px < a.width;
  m.height = a.height;
  return m;
}

template <int RPL>
__device__ inline bool band_misses(const StageEntry& s, const TileMap<RPL>& m, int j) {
  const float y0 = m.ty0 + 4.0f * j;
  return s.by1 < y0 || s.by0 > y0 + 3.0f;
}

template <int RPL>
__global__ __launch_bounds__(256 / RPL) void raster_render_fwd(RasterArgs a) {
  constexpr int kBlock = 256 / RPL;
  __shared__ StageEntry stage[kBlock];
  const int64_t tile = blockIdx.x;
  const TileMap<RPL> m = tile_map<RPL>(a, tile);
  const double cxp = m.px + 0.5;
  const int cnt = min(a.cursor[tile], a.cap);
  const int32_t* list = a.lists + tile * a.cap;

  double C[RPL][3], t[RPL], pw[RPL];
  int E[RPL];
  bool in[RPL];
#pragma unroll
  for (int j = 0; j < RPL; ++j) {
    C[j][0] = C[j][1] = C[j][2] = 0.0;
    t[j] = 1.0;  // T = t * pw, pw = 2^E
    pw[j] = 1.0;
    E[j] = 0;
    in[j] = m.in_x && m.py0 + 4 * j < m.height;
  }
  for (int base = 0; base < cnt; base += kBlock) {
    __syncthreads();
    const int e = base + static_cast<int>(threadIdx.x);
    if (e < cnt) stage_entry(a, list, e, &stage[threadIdx.x]);
    __syncthreads();
    const int lim = min(kBlock, cnt - base);
    for (int k = 0; k < lim; ++k) {
      const StageEntry& s = stage[k];
      if (s.bx1 < m.tx0 || s.bx0 > m.tx1) continue;  // uniform
      const double dx = cxp - s.u;
      const double A = s.a * dx * dx, B = 2.0 * s.b * dx;
#pragma unroll
      for (int j = 0; j < RPL; ++j) {
        if (band_misses(s, m, j)) continue;  // uniform
        const double dy = (m.py0 + 4 * j + 0.5) - s.v;
        const double q = fma(dy, fma(s.c, dy, B), A);
        if (in[j] && q <= kSupport) {
          const float rho = __expf(static_cast<float>(-0.5 * q));
          const float al = fminf(s.sigma * rho, kClamp);
          const double w = static_cast<double>(al) * t[j] * pw[j];
          C[j][0] = fma(w, static_cast<double>(s.c0), C[j][0]);
          C[j][1] = fma(w, static_cast<double>(s.c1), C[j][1]);
          C[j][2] = fma(w, static_cast<double>(s.c2), C[j][2]);
          t[j] *= 1.0 - static_cast<double>(al);
          if (t[j] < 0x1p-600) {
            t[j] *= 0x1p600;
            E[j] -= kRenorm;
            pw[j] = ldexp(1.0, E[j]);
          }
        }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < RPL; ++j) {
    if (!in[j]) continue;
    const int64_t pix = static_cast<int64_t>(m.py0 + 4 * j) * a.width + m.px;
    a.image_out[3 * pix] = static_cast<float>(C[j][0]);
    a.image_out[3 * pix + 1] = static_cast<float>(C[j][1]);
    a.image_out[3 * pix + 2] = static_cast<float>(C[j][2]);
    a.pix_state[2 * pix] = t[j];
    a.pix_state[2 * pix + 1] = static_cast<double>(E[j]);
  }
}

// Back to front over the same sorted list. With R_k the colour seen from
// layer k onwards in units of T_k (R_k = alpha_k c_k + (1 - alpha_k) R_{k+1},
// R = 0 behind the last layer), the colour behind i is S_i = T_i (1 -
// alpha_i) R_{i+1}, so dC/dalpha_i = T_i (c_i - R_{i+1}): no difference of
// large sums, whatever the depth. T_i is recovered from the forward's final
// transmittance, T_i = T_{i+1} / (1 - alpha_i).
template <int RPL>
__global__ __launch_bounds__(256 / RPL) void raster_render_bwd(RasterArgs a) {
  constexpr int kBlock = 256 / RPL;
  __shared__ StageEntry stage[kBlock];
  const int64_t tile = blockIdx.x;
  const TileMap<RPL> m = tile_map<RPL>(a, tile);
  const double cxp = m.px + 0.5;
  const int cnt = min(a.cursor[tile], a.cap);
  const int32_t* list = a.lists + tile * a.cap;

  double t[RPL], pw[RPL], R[RPL][3];
  float g[RPL][3];
  int E[RPL];
  bool in[RPL];
#pragma unroll
  for (int j = 0; j < RPL; ++j) {
    in[j] = m.in_x && m.py0 + 4 * j < m.height;
    R[j][0] = R[j][1] = R[j][2] = 0.0;
    t[j] = 1.0;
    pw[j] = 1.0;
    E[j] = 0;
    g[j][0] = g[j][1] = g[j][2] = 0.f;
    if (in[j]) {
      const int64_t pix = static_cast<int64_t>(m.py0 + 4 * j) * a.width + m.px;
      t[j] = a.pix_state[2 * pix];
      E[j] = static_cast<int>(a.pix_state[2 * pix + 1]);
      pw[j] = ldexp(1.0, E[j]);
      g[j][0] = a.grad_image[3 * pix];
      g[j][1] = a.grad_image[3 * pix + 1];
      g[j][2] = a.grad_image[3 * pix + 2];
    }
  }
  for (int end = cnt; end > 0; end -= kBlock) {
    const int base = max(0, end - kBlock);
    __syncthreads();
    const int e = base + static_cast<int>(threadIdx.x);
    if (e < end) stage_entry(a, list, e, &stage[threadIdx.x]);
    __syncthreads();
    for (int k = end - base - 1; k >= 0; --k) {
      const StageEntry& s = stage[k];
      if (s.bx1 < m.tx0 || s.bx0 > m.tx1) continue;  // uniform
      const double dx = cxp - s.u;
      const double A = s.a * dx * dx, B = 2.0 * s.b * dx;
      const double c0 = s.c0, c1 = s.c1, c2 = s.c2;
      float gc0 = 0.f, gc1 = 0.f, gc2 = 0.f, gop = 0.f;
      bool any = false;
#pragma unroll
      for (int j = 0; j < RPL; ++j) {
        if (band_misses(s, m, j)) continue;  // uniform
        const double dy = (m.py0 + 4 * j + 0.5) - s.v;
        const double q = fma(dy, fma(s.c, dy, B), A);
        if (in[j] && q <= kSupport) {
          any = true;
          const float rho = __expf(static_cast<float>(-0.5 * q));
          const float raw = s.sigma * rho;
          const float al = fminf(raw, kClamp);
          const double ald = static_cast<double>(al);
          const double om = 1.0 - ald;
          t[j] *= rcp64(om);  // now T_i = t * pw
          if (t[j] > 0x1p300 && E[j] < 0) {
            t[j] *= 0x1p-600;
            E[j] += kRenorm;
            pw[j] = ldexp(1.0, E[j]);
          }
          const double T = t[j] * pw[j];
          const double w = ald * T;
          gc0 += static_cast<float>(w * g[j][0]);
          gc1 += static_cast<float>(w * g[j][1]);
          gc2 += static_cast<float>(w * g[j][2]);
          if (raw < kClamp) {
            const double da = g[j][0] * (c0 - R[j][0]) + g[j][1] * (c1 - R[j][1]) +
                              g[j][2] * (c2 - R[j][2]);
            gop += static_cast<float>(da * T * rho);
          }
          R[j][0] = fma(om, R[j][0], ald * c0);
          R[j][1] = fma(om, R[j][1], ald * c1);
          R[j][2] = fma(om, R[j][2], ald * c2);
        }
      }
      if (__ballot(any) != 0) {  // uniform: every lane reads the same staged entry
        gc0 = wave_sum(gc0);
        gc1 = wave_sum(gc1);
        gc2 = wave_sum(gc2);
        gop = wave_sum(gop);
        if ((threadIdx.x & 63) == 0) {
          double* acc = a.grad_acc + 4 * static_cast<int64_t>(s.idx);
          unsafeAtomicAdd(acc + 0, static_cast<double>(gc0));
          unsafeAtomicAdd(acc + 1, static_cast<double>(gc1));
          unsafeAtomicAdd(acc + 2, static_cast<double>(gc2));
          unsafeAtomicAdd(acc + 3, static_cast<double>(gop));
        }
      }
    }
  }
}

hipError_t launch_raster(const RasterArgs& a, bool bwd, hipStream_t s) {
  const int64_t n_tiles = static_cast<int64_t>(a.tiles_x) * a.tiles_y;
  const unsigned gt = static_cast<unsigned>((n_tiles + 255) / 256);
  const unsigned gn = static_cast<unsigned>((a.n + 255) / 256);
  if (!bwd) {
    hipLaunchKernelGGL(raster_zero, dim3(gt), dim3(256), 0, s, a.cursor, n_tiles, a.overflow);
    if (a.n > 0) {
      hipLaunchKernelGGL(raster_project, dim3(gn), dim3(256), 0, s, a);
      hipLaunchKernelGGL(raster_bin, dim3(gn), dim3(256), 0, s, a);
    }
    hipLaunchKernelGGL(raster_sort, dim3(static_cast<unsigned>(n_tiles)), dim3(256), 0, s, a);
    hipLaunchKernelGGL(raster_render_fwd<kFwdRows>, dim3(static_cast<unsigned>(n_tiles)),
                       dim3(256 / kFwdRows), 0, s, a);
  } else {
    if (a.n == 0) return hipGetLastError();
    hipLaunchKernelGGL(raster_zero_acc, dim3(gn), dim3(256), 0, s, a.grad_acc, a.n);
    hipLaunchKernelGGL(raster_render_bwd<kBwdRows>, dim3(static_cast<unsigned>(n_tiles)),
                       dim3(256 / kBwdRows), 0, s, a);
    hipLaunchKernelGGL(raster_finish_grads, dim3(gn), dim3(256), 0, s, a.grad_acc, a.grad_colors,
                       a.grad_opac, a.n);
  }
  return hipGetLastError();
}

}  // namespace nasg
