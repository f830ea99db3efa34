// Compositing of the primitives' colours into an image for one camera
// (Section 3.1: C = sum_i T_i alpha_i c_i, alpha_i = sigma_i rho_i,
// T_i = prod_{j<i} (1 - alpha_j)), with the gradients of a loss on the image
// with respect to the per-primitive colours (what the appearance backward
// consumes), opacities and, on request, the geometry (mean, scales,
// quaternion) through rho.
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
//             the 16 x 16-pixel tiles its ellipse's bounding box touches, kept
//             with the colour and opacity in a 64-byte render record;
//   bin     : each primitive's 64-bit depth key (float depth bits, index)
//             goes to the lists of those tiles (a cursor per tile, fixed
//             capacity per tile; entries beyond it are dropped and flagged);
//             blocks count their entries per tile in LDS and take one device
//             atomic per touched tile;
//   sort    : per tile, the list is sorted by (depth, primitive index), which
//             fixes the compositing order: a bucket sort on the depth bits in
//             LDS, or a bitonic network on the 64-bit keys for small tiles
//             and for tiles whose depths crowd into few buckets;
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
//             totals them over its lanes by halving exchanges, and the lanes
//             holding the totals add them to FP64 per-primitive accumulators
//             with one atomic instruction. With
//             geometry gradients the same pass also sums dL/d(u, v, a, b, c)
//             (dL/dq = -sigma rho / 2 times the pixel's dL/dalpha);
//   finish  : per primitive, the accumulators rounded to the float32
//             outputs and, with geometry gradients, the FP64 chain from
//             dL/d(u, v, a, b, c) through the projection to the mean, scales
//             and quaternion.
#include <hip/hip_runtime.h>

#include "../../include/nasg.h"
#include "nasg_device.hpp"
#include "raster.hpp"

namespace nasg {

constexpr double kNear = 0.2;
constexpr float kClamp = 0.99f;
constexpr double kSupport = 9.0;
constexpr int kBinParts = 8;  // most tile classes of the binning pass
constexpr int kBinLdsTiles = 8192;      // class tiles one LDS-counting block holds
constexpr int kBinPrimsPerThread = 32;  // primitives per thread of an LDS-counting block

__global__ void raster_begin(RasterArgs a) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < static_cast<int64_t>(a.tiles_x) * a.tiles_y) a.cursor[t] = 0;
  if (t == 0) {
    *a.overflow = 0;
    RasterStamp st;
    st.magic = kStampMagic;
    st.cap = a.cap;
    st.tiles_x = a.tiles_x;
    st.tiles_y = a.tiles_y;
    st.n = a.n;
    *a.stamp = st;
  }
}

__global__ void raster_zero_acc(double* acc, int64_t n, int32_t* stale) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i == 0) *stale = 0;
  if (i < n) {
#pragma unroll
    for (int k = 0; k < kAccStride; ++k) acc[kAccStride * i + k] = 0.0;
  }
}

// Gradients of the loss with respect to a primitive's mean, scales and
// quaternion from its sums g2 = (dL/du, dL/dv, dL/da, dL/db, dL/dc) over the
// image (b the conic's off-diagonal entry), in FP64, by the chain through the
// projection: K = Sigma_2^{-1} with dL/dSigma_2 = -K dL/dK K, Sigma_2 = M M^T
// (dL/dM = 2 dL/dSigma_2 M), M = J R_cw R(q/|q|) S, and u, v and J functions
// of the camera-space mean.
__device__ void geometry_chain(const RasterArgs& a, int64_t i, const double* g2, float* gm,
                               float* gs, float* gr) {
  double out_m[3] = {0.0, 0.0, 0.0}, out_s[3] = {0.0, 0.0, 0.0}, out_q[4] = {0.0, 0.0, 0.0, 0.0};
  const double* R = a.cam_rot;
  const double mx = a.means[3 * i], my = a.means[3 * i + 1], mz = a.means[3 * i + 2];
  const double X = R[0] * mx + R[1] * my + R[2] * mz + a.cam_t[0];
  const double Y = R[3] * mx + R[4] * my + R[5] * mz + a.cam_t[1];
  const double Z = R[6] * mx + R[7] * my + R[8] * mz + a.cam_t[2];
  const bool any = g2[0] != 0.0 || g2[1] != 0.0 || g2[2] != 0.0 || g2[3] != 0.0 || g2[4] != 0.0;
  if (any && Z > kNear) {
    const double iz = 1.0 / Z, iz2 = iz * iz;
    double qw = a.rots[4 * i], qx = a.rots[4 * i + 1], qy = a.rots[4 * i + 2], qz = a.rots[4 * i + 3];
    const double qn = 1.0 / sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    qw *= qn;
    qx *= qn;
    qy *= qn;
    qz *= qn;
    const double Rw[3][3] = {{1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy)},
                             {2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx)},
                             {2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)}};
    const double sc[3] = {a.scales[3 * i], a.scales[3 * i + 1], a.scales[3 * i + 2]};
    double A[3][3];  // R_cw R_w S
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c)
        A[r][c] = (R[3 * r] * Rw[0][c] + R[3 * r + 1] * Rw[1][c] + R[3 * r + 2] * Rw[2][c]) * sc[c];
    const double J[2][3] = {{a.fx * iz, 0.0, -a.fx * X * iz2}, {0.0, a.fy * iz, -a.fy * Y * iz2}};
    double M[2][3];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 3; ++c) M[r][c] = J[r][0] * A[0][c] + J[r][1] * A[1][c] + J[r][2] * A[2][c];
    const double sxx = M[0][0] * M[0][0] + M[0][1] * M[0][1] + M[0][2] * M[0][2];
    const double sxy = M[0][0] * M[1][0] + M[0][1] * M[1][1] + M[0][2] * M[1][2];
    const double syy = M[1][0] * M[1][0] + M[1][1] * M[1][1] + M[1][2] * M[1][2];
    const double id = 1.0 / (sxx * syy - sxy * sxy);
    const double K[2][2] = {{syy * id, -sxy * id}, {-sxy * id, sxx * id}};
    const double gK[2][2] = {{g2[2], 0.5 * g2[3]}, {0.5 * g2[3], g2[4]}};
    double T1[2][2], gS[2][2];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 2; ++c) T1[r][c] = K[r][0] * gK[0][c] + K[r][1] * gK[1][c];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 2; ++c) gS[r][c] = -(T1[r][0] * K[0][c] + T1[r][1] * K[1][c]);
    double gM[2][3];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 3; ++c) gM[r][c] = 2.0 * (gS[r][0] * M[0][c] + gS[r][1] * M[1][c]);
    double gJ[2][3];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 3; ++c) gJ[r][c] = gM[r][0] * A[c][0] + gM[r][1] * A[c][1] + gM[r][2] * A[c][2];
    double gA[3][3];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) gA[r][c] = J[0][r] * gM[0][c] + J[1][r] * gM[1][c];
    double gRw[3][3];
    for (int k = 0; k < 3; ++k) {
      for (int c = 0; c < 3; ++c) {
        const double grs = R[k] * gA[0][c] + R[3 + k] * gA[1][c] + R[6 + k] * gA[2][c];  // (R_cw^T gA)
        out_s[c] += grs * Rw[k][c];
        gRw[k][c] = grs * sc[c];
      }
    }
    // d R(u) / d(w, x, y, z) contracted with gRw, then the unit-norm projection
    const double gw = 2.0 * (-gRw[0][1] * qz + gRw[0][2] * qy + gRw[1][0] * qz - gRw[1][2] * qx -
                             gRw[2][0] * qy + gRw[2][1] * qx);
    const double gx = 2.0 * (gRw[0][1] * qy + gRw[0][2] * qz + gRw[1][0] * qy - 2.0 * gRw[1][1] * qx -
                             gRw[1][2] * qw + gRw[2][0] * qz + gRw[2][1] * qw - 2.0 * gRw[2][2] * qx);
    const double gy = 2.0 * (-2.0 * gRw[0][0] * qy + gRw[0][1] * qx + gRw[0][2] * qw + gRw[1][0] * qx +
                             gRw[1][2] * qz - gRw[2][0] * qw + gRw[2][1] * qz - 2.0 * gRw[2][2] * qy);
    const double gz = 2.0 * (-2.0 * gRw[0][0] * qz - gRw[0][1] * qw + gRw[0][2] * qx + gRw[1][0] * qw -
                             2.0 * gRw[1][1] * qz + gRw[1][2] * qy + gRw[2][0] * qx + gRw[2][1] * qy);
    const double dot = gw * qw + gx * qx + gy * qy + gz * qz;
    out_q[0] = (gw - qw * dot) * qn;
    out_q[1] = (gx - qx * dot) * qn;
    out_q[2] = (gy - qy * dot) * qn;
    out_q[3] = (gz - qz * dot) * qn;
    // camera-space mean through (u, v) and J
    const double gX = g2[0] * a.fx * iz - gJ[0][2] * a.fx * iz2;
    const double gY = g2[1] * a.fy * iz - gJ[1][2] * a.fy * iz2;
    const double gZ = -g2[0] * a.fx * X * iz2 - g2[1] * a.fy * Y * iz2 - gJ[0][0] * a.fx * iz2 +
                      gJ[0][2] * 2.0 * a.fx * X * iz2 * iz - gJ[1][1] * a.fy * iz2 +
                      gJ[1][2] * 2.0 * a.fy * Y * iz2 * iz;
    for (int k = 0; k < 3; ++k) out_m[k] = gX * R[k] + gY * R[3 + k] + gZ * R[6 + k];
  }
  if (gm != nullptr)
    for (int k = 0; k < 3; ++k) gm[3 * i + k] = static_cast<float>(out_m[k]);
  if (gs != nullptr)
    for (int k = 0; k < 3; ++k) gs[3 * i + k] = static_cast<float>(out_s[k]);
  if (gr != nullptr)
    for (int k = 0; k < 4; ++k) gr[4 * i + k] = static_cast<float>(out_q[k]);
}

template <bool GEOM>
__global__ void raster_finish_grads(RasterArgs a) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const double* acc = a.grad_acc + kAccStride * i;
  if (a.grad_colors != nullptr) {
    a.grad_colors[3 * i + 0] = static_cast<float>(acc[0]);
    a.grad_colors[3 * i + 1] = static_cast<float>(acc[1]);
    a.grad_colors[3 * i + 2] = static_cast<float>(acc[2]);
  }
  if (a.grad_opac != nullptr) a.grad_opac[i] = static_cast<float>(acc[3]);
  if constexpr (GEOM) geometry_chain(a, i, acc + 4, a.grad_means, a.grad_scales, a.grad_rots);
}

__global__ void raster_project(RasterArgs a) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  RenderRec rec{};
  BinRec bin{};
  bin.tx0 = 1;  // empty tile range unless the ellipse lands on the image
  bin.tx1 = 0;
  bin.ty0 = 1;
  bin.ty1 = 0;
  const double mx = a.means[3 * i], my = a.means[3 * i + 1], mz = a.means[3 * i + 2];
  const double* R = a.cam_rot;
  const double X = R[0] * mx + R[1] * my + R[2] * mz + a.cam_t[0];
  const double Y = R[3] * mx + R[4] * my + R[5] * mz + a.cam_t[1];
  const double Z = R[6] * mx + R[7] * my + R[8] * mz + a.cam_t[2];
  bin.z = Z;
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
      rec.b2 = -2.0 * sxy * id;
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
        bin.tx0 = static_cast<int16_t>(static_cast<int32_t>(px0) / kTile);
        bin.tx1 = static_cast<int16_t>(static_cast<int32_t>(px1) / kTile);
        bin.ty0 = static_cast<int16_t>(static_cast<int32_t>(py0) / kTile);
        bin.ty1 = static_cast<int16_t>(static_cast<int32_t>(py1) / kTile);
      }
    }
  }
  rec.c0 = a.colors[3 * i];
  rec.c1 = a.colors[3 * i + 1];
  rec.c2 = a.colors[3 * i + 2];
  rec.sigma = a.opac[i];
  a.rec[i] = rec;
  a.bins[i] = bin;
}

// Sort key of a list entry: the float32 of its FP64 depth (z > 0.2, so the
// float's bits order like the depths) above its primitive index.
__device__ inline uint64_t depth_key(double z, int64_t i) {
  return (static_cast<uint64_t>(__float_as_uint(__double2float_rn(z))) << 32) |
         static_cast<uint32_t>(i);
}

// Tile binning. A primitive's depth key goes to the list of every tile its
// box touches; the order of appends does not matter (the per-tile sort orders
// each list by its keys). The tiles are split into `parts` classes by tile
// index mod parts (a power of two): block b serves class b mod parts for the
// primitives of chunk b / parts.

// Calls f(tile) for each tile of box r in class `part` of `parts`: in each
// row, the box's columns whose tile index is part mod parts.
template <class F>
__device__ inline void for_class_tiles(const BinRec& r, int64_t tiles_x, int part, int parts,
                                       F&& f) {
  for (int y = r.ty0; y <= r.ty1; ++y) {
    const int64_t row = static_cast<int64_t>(y) * tiles_x;
    for (int tx = r.tx0 + static_cast<int>((part - (row + r.tx0)) & (parts - 1)); tx <= r.tx1;
         tx += parts)
      f(row + tx);
  }
}

// Images whose tiles fit kBinLdsTiles per class in at most kBinParts classes
// (parts = the smallest power of two that does it). A block first counts its
// chunk's entries per class tile in LDS, then reserves each touched tile's
// range in its list with one device atomic on the tile's cursor, then places
// the keys in those ranges with LDS atomics: one device atomic per (block,
// tile) instead of one per entry.
__global__ __launch_bounds__(256) void raster_bin_lds(RasterArgs a, int pshift) {
  __shared__ int cnt[kBinLdsTiles];
  const int parts = 1 << pshift;
  const int part = static_cast<int>(blockIdx.x & (parts - 1));
  const int64_t first = static_cast<int64_t>(blockIdx.x >> pshift) * (256 * kBinPrimsPerThread);
  const int64_t last = min(first + 256 * kBinPrimsPerThread, a.n);
  const int64_t n_tiles = static_cast<int64_t>(a.tiles_x) * a.tiles_y;
  const int n_local = static_cast<int>((n_tiles - part + parts - 1) >> pshift);
  for (int m = threadIdx.x; m < n_local; m += 256) cnt[m] = 0;
  __syncthreads();
  for (int64_t i = first + threadIdx.x; i < last; i += 256) {
    const BinRec r = a.bins[i];
    for_class_tiles(r, a.tiles_x, part, parts, [&](int64_t t) { atomicAdd(&cnt[t >> pshift], 1); });
  }
  __syncthreads();
  for (int m = threadIdx.x; m < n_local; m += 256) {
    const int c = cnt[m];
    if (c > 0) cnt[m] = atomicAdd(a.cursor + (static_cast<int64_t>(m) << pshift) + part, c);
  }
  __syncthreads();
  for (int64_t i = first + threadIdx.x; i < last; i += 256) {
    const BinRec r = a.bins[i];
    const uint64_t key = depth_key(r.z, i);
    for_class_tiles(r, a.tiles_x, part, parts, [&](int64_t t) {
      const int pos = atomicAdd(&cnt[t >> pshift], 1);
      if (pos < a.cap) {
        a.lists[t * a.cap + pos] = key;
      } else {
        atomicMax(a.overflow, 1);
      }
    });
  }
}

// Larger images: one device atomic per entry on the tile's cursor, those of
// up to eight tiles issued before their results are used, so their latencies
// overlap. The tiles are split into kBinParts classes as above (each XCD of
// the chip, which takes every eighth workgroup, then appends to its own
// lists); slot (row y, j) of a box is column first(y) + kBinParts * j, where
// first(y) is the box's first column in this class.
__global__ void raster_bin(RasterArgs a) {
  const int part = static_cast<int>(blockIdx.x & (kBinParts - 1));
  const int64_t i = static_cast<int64_t>(blockIdx.x / kBinParts) * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const BinRec r = a.bins[i];
  const int w = r.tx1 - r.tx0 + 1, h = r.ty1 - r.ty0 + 1;
  if (w <= 0 || h <= 0) return;
  const int cw = (w + kBinParts - 1) / kBinParts;
  const int slots = cw * h;
  const uint64_t key = depth_key(r.z, i);
  for (int k0 = 0; k0 < slots; k0 += 8) {
    int64_t tl[8];
    int32_t pos[8];
    bool use[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = k0 + u;
      tl[u] = 0;
      pos[u] = 0;
      use[u] = false;
      if (k < slots) {
        const int y = r.ty0 + k / cw;
        const int64_t row = static_cast<int64_t>(y) * a.tiles_x;
        const int lead = static_cast<int>((part - (row + r.tx0)) & (kBinParts - 1));
        const int tx = r.tx0 + lead + kBinParts * (k % cw);
        if (tx <= r.tx1) {
          use[u] = true;
          tl[u] = row + tx;
          pos[u] = atomicAdd(a.cursor + tl[u], 1);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (use[u]) {
        if (pos[u] < a.cap) {
          a.lists[tl[u] * a.cap + pos[u]] = key;
        } else {
          atomicMax(a.overflow, 1);
        }
      }
    }
  }
}

// Per-tile depth sort. Key = (float32 of the FP64 depth, primitive index):
// rounding to float is monotone, so sorting the 64-bit keys orders the list
// by depth except inside runs of equal float depth, which a final pass puts
// in (FP64 depth, index) order; padding keys (all ones) sort last. Bitonic
// network over 256 EPT keys, EPT consecutive keys per thread in registers:
// strides below EPT are exchanged in registers, strides whose partner is in
// the same wavefront by lane shuffles, the rest through LDS.
template <int EPT>
__device__ void bitonic_keys(uint64_t (&v)[EPT], uint64_t* lds) {
  constexpr int M = 256 * EPT;
  const int t = static_cast<int>(threadIdx.x);
  for (int k = 2; k <= M; k <<= 1) {
    for (int j = k >> 1; j >= EPT; j >>= 1) {
      const int tj = j / EPT;  // partner thread t ^ tj holds the partner keys
      if (tj >= 64) {          // another wavefront: through LDS
        __syncthreads();
#pragma unroll
        for (int r = 0; r < EPT; ++r) lds[t * EPT + r] = v[r];
        __syncthreads();
      }
#pragma unroll
      for (int r = 0; r < EPT; ++r) {
        const int e = t * EPT + r, pe = e ^ j;
        const uint64_t o = tj >= 64 ? lds[pe] : __shfl_xor(v[r], tj, 64);
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

// Runs of equal float depth (in index order on entry): a stable insertion
// sort by FP64 depth, done by the thread that owns the run's first entry;
// then the sorted keys go back to the tile's list.
__device__ void order_runs_and_store(const RasterArgs& a, uint64_t* list, int cnt,
                                     uint64_t* lds) {
  const int t = static_cast<int>(threadIdx.x);
  for (int e = t; e < cnt; e += 256) {
    const uint32_t hi = static_cast<uint32_t>(lds[e] >> 32);
    const bool start = e == 0 || static_cast<uint32_t>(lds[e - 1] >> 32) != hi;
    if (!start || e + 1 >= cnt || static_cast<uint32_t>(lds[e + 1] >> 32) != hi) continue;
    int end = e + 1;
    while (end < cnt && static_cast<uint32_t>(lds[end] >> 32) == hi) ++end;
    for (int i = e + 1; i < end; ++i) {
      const uint64_t key = lds[i];
      const double z = a.bins[static_cast<uint32_t>(key)].z;
      int p = i - 1;
      while (p >= e && a.bins[static_cast<uint32_t>(lds[p])].z > z) {
        lds[p + 1] = lds[p];
        --p;
      }
      lds[p + 1] = key;
    }
  }
  __syncthreads();
  for (int e = t; e < cnt; e += 256) list[e] = lds[e];
}

template <int EPT>
__device__ void sort_tile(const RasterArgs& a, uint64_t* list, int cnt, uint64_t* lds) {
  const int t = static_cast<int>(threadIdx.x);
  // coalesced load through LDS into the blocked register layout
  for (int e = t; e < 256 * EPT; e += 256) lds[e] = e < cnt ? list[e] : ~0ull;
  __syncthreads();
  uint64_t v[EPT];
#pragma unroll
  for (int r = 0; r < EPT; ++r) v[r] = lds[t * EPT + r];
  bitonic_keys<EPT>(v, lds);
  __syncthreads();
#pragma unroll
  for (int r = 0; r < EPT; ++r) lds[t * EPT + r] = v[r];
  __syncthreads();
  order_runs_and_store(a, list, cnt, lds);
}

// Bucket sort of one tile's keys (257 .. 4096 of them) on the float depth
// bits, which order like the depths: bucket (bits - min) >> shift, with the
// shift that fits the tile's span of bits into kSortBuckets buckets, is
// monotone in the key, so sorting each bucket by the full key (depth bits,
// then index) sorts the list. An LDS histogram, a block scan of it and a
// scatter place the keys; the owner of 16 consecutive buckets then sorts
// each of them by insertion. Returns false, having changed nothing, when a
// bucket holds more than kSortBucketRun keys: the bitonic network takes
// that tile instead.
constexpr int kSortBuckets = 4096;
constexpr int kSortBucketRun = 32;

__device__ bool bucket_sort_tile(const RasterArgs& a, uint64_t* list, int cnt, uint64_t* out,
                                 int* bucket, uint32_t* red) {
  constexpr int BPT = kSortBuckets / 256;  // buckets owned by each thread
  const int t = static_cast<int>(threadIdx.x), lane = t & 63, wave = t >> 6;
  // the keys' high words (float depth bits) are read from the list where
  // only they are needed, which keeps the keys out of registers
  const uint32_t* hw = reinterpret_cast<const uint32_t*>(list) + 1;
  uint32_t lo = 0xffffffffu, hi = 0u;
  for (int e = t; e < cnt; e += 256) {
    const uint32_t h = hw[2 * e];
    lo = min(lo, h);
    hi = max(hi, h);
  }
  for (int k = t; k < kSortBuckets; k += 256) bucket[k] = 0;
  for (int o = 32; o >= 1; o >>= 1) {
    lo = min(lo, static_cast<uint32_t>(__shfl_xor(static_cast<int>(lo), o, 64)));
    hi = max(hi, static_cast<uint32_t>(__shfl_xor(static_cast<int>(hi), o, 64)));
  }
  if (lane == 0) {
    red[wave] = lo;
    red[4 + wave] = hi;
  }
  __syncthreads();
  lo = min(min(red[0], red[1]), min(red[2], red[3]));
  hi = max(max(red[4], red[5]), max(red[6], red[7]));
  const uint32_t span = hi - lo;
  const int shift = span == 0 ? 0 : max(0, 32 - __clz(static_cast<int>(span)) - 12);
  for (int e = t; e < cnt; e += 256) atomicAdd(&bucket[(hw[2 * e] - lo) >> shift], 1);
  __syncthreads();
  int c[BPT];
  int sum = 0, cmax = 0;
#pragma unroll
  for (int k = 0; k < BPT; ++k) {
    c[k] = bucket[BPT * t + k];
    sum += c[k];
    cmax = max(cmax, c[k]);
  }
  if (__syncthreads_or(cmax > kSortBucketRun)) return false;
  // exclusive scan of the per-thread bucket totals over the block
  int incl = sum;
  for (int o = 1; o < 64; o <<= 1) {
    const int v = __shfl_up(incl, o, 64);
    if (lane >= o) incl += v;
  }
  if (lane == 63) red[wave] = static_cast<uint32_t>(incl);
  __syncthreads();
  int run = incl - sum;
  for (int w = 0; w < wave; ++w) run += static_cast<int>(red[w]);
#pragma unroll
  for (int k = 0; k < BPT; ++k) {
    bucket[BPT * t + k] = run;
    run += c[k];
  }
  __syncthreads();
  for (int e = t; e < cnt; e += 256) {
    const uint64_t key = list[e];
    out[atomicAdd(&bucket[(static_cast<uint32_t>(key >> 32) - lo) >> shift], 1)] = key;
  }
  __syncthreads();
  // bucket b now ends at bucket[b] and starts where bucket b - 1 ends
  for (int k = 0; k < BPT; ++k) {
    const int b = BPT * t + k;
    const int s0 = b == 0 ? 0 : bucket[b - 1], s1 = bucket[b];
    for (int i = s0 + 1; i < s1; ++i) {
      const uint64_t v = out[i];
      int p = i - 1;
      while (p >= s0 && out[p] > v) {
        out[p + 1] = out[p];
        --p;
      }
      out[p + 1] = v;
    }
  }
  __syncthreads();
  order_runs_and_store(a, list, cnt, out);
  return true;
}

__global__ __launch_bounds__(256) void raster_sort(RasterArgs a) {
  __shared__ uint64_t lds[256 * 16];
  __shared__ int bucket[kSortBuckets];
  __shared__ uint32_t red[8];
  const int64_t tile = blockIdx.x;
  const int cnt = min(a.cursor[tile], a.cap);
  if (cnt <= 1) return;
  uint64_t* list = a.lists + tile * a.cap;
  if (cnt <= 256) {
    sort_tile<1>(a, list, cnt, lds);
  } else if (!bucket_sort_tile(a, list, cnt, lds, bucket, red)) {
    // left to raster_sort_network, which this mark (the tile's count, bit
    // inverted) tells to take the tile and restore the count; every thread
    // read the cursor before the barrier inside the bucket sort
    if (threadIdx.x == 0) a.cursor[tile] = ~a.cursor[tile];
  }
}

// The tiles the bucket sort left: the bitonic network, whose registers would
// otherwise cap the occupancy of every tile's sort.
__global__ __launch_bounds__(256) void raster_sort_network(RasterArgs a) {
  __shared__ uint64_t lds[256 * 16];
  const int64_t tile = blockIdx.x;
  const int c = a.cursor[tile];
  if (c >= 0) return;
  const int cnt = min(~c, a.cap);
  uint64_t* list = a.lists + tile * a.cap;
  if (cnt <= 512) {
    sort_tile<2>(a, list, cnt, lds);
  } else if (cnt <= 1024) {
    sort_tile<4>(a, list, cnt, lds);
  } else if (cnt <= 2048) {
    sort_tile<8>(a, list, cnt, lds);
  } else {
    sort_tile<16>(a, list, cnt, lds);
  }
  __syncthreads();  // every thread has read the mark
  if (threadIdx.x == 0) a.cursor[tile] = ~c;
}

struct StageEntry {
  double u, v, a, b2, c;  // pixel-space mean and conic, b2 = 2 b
  double c0, c1, c2;      // colour
  float sigma;
  uint32_t mask;          // row bands (rows 4 b .. 4 b + 3 of the tile) the q <= 9 box meets
  int32_t idx;
  int32_t pad;
};

// Totals of several per-lane values over the 64 lanes of a wavefront (every
// lane active) by halving exchanges: at each step a lane keeps half of the
// values it holds, adds its partner's partial sums of that half and passes
// the other half on, so the totals end up spread over the lanes instead of
// being reduced one value at a time. Partners: lane ^ 32 and lane ^ 16 (the
// permlane swaps), lane ^ 1 and lane ^ 2 (quad DPP); lane bits 2 and 3 are
// then summed with row rotations by 8 and 4.
__device__ inline float swap32_sum(float x, float y) {
  // lanes 0-31: x[l] + x[l + 32]; lanes 32-63: y[l - 32] + y[l]
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false,
                                                  false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ inline float swap16_sum(float x, float y) {
  // rows 0 and 2 (lane bit 4 clear): x[l] + x[l ^ 16]; rows 1 and 3: y[l ^ 16] + y[l]
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false,
                                                  false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

constexpr int kQuadXor1 = 0xB1;  // quad_perm [1, 0, 3, 2]
constexpr int kQuadXor2 = 0x4E;  // quad_perm [2, 3, 0, 1]
constexpr int kRowRor8 = 0x128;
constexpr int kRowRor4 = 0x124;

// Nine values: lane l ends with the total of value lane_slot9(l); lanes 0, 1,
// 2, 16, 17, 32, 33, 48, 49 hold the nine totals once each.
__device__ inline float lane_sums9(const float (&x)[9], int lane) {
  const float a0 = swap32_sum(x[0], x[1]), a1 = swap32_sum(x[2], x[3]);
  const float a2 = swap32_sum(x[4], x[5]), a3 = swap32_sum(x[6], x[7]);
  const float a4 = swap32_sum(x[8], x[8]);
  const float b0 = swap16_sum(a0, a1), b1 = swap16_sum(a2, a3), b2 = swap16_sum(a4, a4);
  const bool o1 = (lane & 1) != 0, o2 = (lane & 2) != 0;
  const float c0 = (o1 ? b1 : b0) + dpp_f<kQuadXor1>(o1 ? b0 : b1);
  const float c1 = b2 + dpp_f<kQuadXor1>(b2);
  float d = (o2 ? c1 : c0) + dpp_f<kQuadXor2>(o2 ? c0 : c1);
  d += dpp_f<kRowRor8>(d);
  d += dpp_f<kRowRor4>(d);
  return d;
}
__device__ inline bool lane_writes9(int lane) { return (lane & 0xE) == 0 || lane == 2; }
__device__ inline int lane_slot9(int lane) {
  return lane == 2 ? 8 : 4 * (lane & 1) + 2 * ((lane >> 4) & 1) + ((lane >> 5) & 1);
}

// Four values: lanes 0, 16, 32, 48 hold the totals of values 0, 2, 1, 3.
__device__ inline float lane_sums4(const float (&x)[4]) {
  float b = swap16_sum(swap32_sum(x[0], x[1]), swap32_sum(x[2], x[3]));
  b += dpp_f<kQuadXor1>(b);
  b += dpp_f<kQuadXor2>(b);
  b += dpp_f<kRowRor8>(b);
  b += dpp_f<kRowRor4>(b);
  return b;
}
__device__ inline bool lane_writes4(int lane) { return (lane & 0xF) == 0; }
__device__ inline int lane_slot4(int lane) { return 2 * ((lane >> 4) & 1) + ((lane >> 5) & 1); }

// Transmittance as t * 2^E (E a multiple of kRenorm). t is renormalised every
// kRenormEvery entries of a wavefront's list and at the end of each chunk, so
// at most kRenormEvery layers (each multiplying t by at least 0.01 going
// forward, or dividing it by at least 0.01 going back) pass between checks:
// t stays within [2^-500 1e-64, 1] in the forward and below 2^300 1e64 in the
// backward, normal doubles, and a pixel behind thousands of layers keeps an
// exact transmittance for the backward's recovery by division.
constexpr int kRenorm = 500;
constexpr int kRenormEvery = 32;
// rho = exp(-q/2) = 2^(q * (-log2(e) / 2)); the constant is exact in float
// (half of the float log2 e), so this is the float exponential of -q/2
constexpr float kNegHalfLog2e = -0.72134752044448170368f;

// Minimum over the rectangle [x0, x1] x [y0, y1] of the positive definite
// q = a dx^2 + b2 dx dy + c dy^2 (dx = x - u, dy = y - v): zero if (u, v) is
// inside; otherwise on the boundary, where each edge is a 1D quadratic
// minimised at its vertex clamped to the edge.
__device__ inline double quad_min_rect(double a, double b2, double c, double u, double v,
                                       double x0, double x1, double y0, double y1) {
  if (u >= x0 && u <= x1 && v >= y0 && v <= y1) return 0.0;
  const double hb = 0.5 * b2, ia = rcp64(a), ic = rcp64(c);
  double best = INFINITY;
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const double dx = (side ? x1 : x0) - u;  // vertical edge
    const double dy = fmin(fmax(-hb * dx * ic, y0 - v), y1 - v);
    best = fmin(best, a * dx * dx + b2 * dx * dy + c * dy * dy);
    const double ey = (side ? y1 : y0) - v;  // horizontal edge
    const double ex = fmin(fmax(-hb * ey * ia, x0 - u), x1 - u);
    best = fmin(best, a * ex * ex + b2 * ex * ey + c * ey * ey);
  }
  return best;
}

// EXACT adds the exact band test to the box test; it pays in the backward,
// whose per-entry work is large, not in the forward, where its staging cost
// outweighs the entries it removes (measured).
template <bool EXACT>
__device__ inline void stage_entry(const RasterArgs& a, const uint64_t* list, int e, double x0,
                                   double y0, StageEntry* slot) {
  const int32_t idx = static_cast<int32_t>(static_cast<uint32_t>(list[e]));
  const RenderRec r = a.rec[idx];
  StageEntry s;
  s.u = r.u;
  s.v = r.v;
  s.a = r.a;
  s.b2 = r.b2;
  s.c = r.c;
  s.c0 = r.c0;
  s.c1 = r.c1;
  s.c2 = r.c2;
  s.sigma = r.sigma;
  s.idx = idx;
  s.pad = 0;
  // a band's bit is set when the ellipse q <= 9 can reach one of its pixel
  // centres: the box test and, with EXACT, the minimum of q over the band's
  // rectangle of pixel centres (with a relative margin far above rounding)
  uint32_t mask = 0;
  if (r.u + r.ex >= x0 + 0.5 && r.u - r.ex <= x0 + 15.5) {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const double ylo = y0 + 4 * b + 0.5, yhi = ylo + 3.0;
      if (r.v + r.ey >= ylo && r.v - r.ey <= yhi &&
          (!EXACT || quad_min_rect(r.a, r.b2, r.c, r.u, r.v, x0 + 0.5, x0 + 15.5, ylo, yhi) <=
                         kSupport * (1.0 + 1e-9)))
        mask |= 1u << b;
    }
  }
  s.mask = mask;
  *slot = s;
}

// Each wavefront lists, in order, the staged entries whose band mask meets
// `bits`; returns the list length (uniform).
__device__ inline int wave_compact(const StageEntry* stage, int lim, uint32_t bits,
                                   int16_t* wl) {
  const int lane = static_cast<int>(threadIdx.x) & 63;
  int n = 0;
  for (int g = 0; g < lim; g += 64) {
    const int k = g + lane;
    const bool want = k < lim && (stage[k].mask & bits) != 0;
    const uint64_t bal = __ballot(want);
    const int below = __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(bal >> 32),
                                                 __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(bal), 0));
    if (want) wl[n + below] = static_cast<int16_t>(k);
    n += __popcll(bal);
  }
  return n;
}

// Thread layout of the render kernels: a block of 256 / RPL threads per
// 16 x 16 tile; lane l of wavefront w owns column l & 15 and the RPL rows
// 4 RPL w + (l >> 4) + 4 j, j < RPL (row band RPL w + j), so an entry's dx
// terms are shared by a lane's RPL pixels.
// Rows per lane, measured on MI355X at 3 M primitives and 1920 x 1080: the
// forward is fastest at one pixel per thread (occupancy hides the LDS and
// FP64 latencies), the backward at four (one wavefront per tile: the four
// per-entry wavefront sums and atomics are shared by four pixels per lane).
constexpr int kFwdRows = 1;
constexpr int kBwdRows = 4;

template <int RPL>
struct TileMap {
  int px, py0;     // the lane's column and first row
  int wave;
  double x0, y0;   // the tile's corner
  bool in_x;
  int height;
};

template <int RPL>
__device__ inline TileMap<RPL> tile_map(const RasterArgs& a, int64_t tile) {
  TileMap<RPL> m;
  const int tx = static_cast<int>(tile % a.tiles_x), ty = static_cast<int>(tile / a.tiles_x);
  const int lane = static_cast<int>(threadIdx.x) & 63;
  m.wave = static_cast<int>(threadIdx.x) >> 6;
  m.px = tx * kTile + (lane & 15);
  m.py0 = ty * kTile + 4 * RPL * m.wave + (lane >> 4);
  m.x0 = tx * kTile;
  m.y0 = ty * kTile;
  m.in_x = m.px < a.width;
  m.height = a.height;
  return m;
}

template <int RPL>
__global__ __launch_bounds__(256 / RPL) void raster_render_fwd(RasterArgs a) {
  constexpr int kBlock = 256 / RPL;
  __shared__ StageEntry stage[kBlock];
  __shared__ int16_t wlist[kBlock / 64][kBlock];
  const int64_t tile = blockIdx.x;
  const TileMap<RPL> m = tile_map<RPL>(a, tile);
  const double cxp = m.px + 0.5;
  const int cnt = __builtin_amdgcn_readfirstlane(min(a.cursor[tile], a.cap));
  const uint64_t* list = a.lists + tile * a.cap;
  const uint32_t bits = ((1u << RPL) - 1u) << (RPL * m.wave);
  int16_t* wl = wlist[m.wave];

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
  auto renorm = [&]() {
#pragma unroll
    for (int j = 0; j < RPL; ++j) {
      if (t[j] < 0x1p-500) {
        t[j] *= 0x1p500;
        E[j] -= kRenorm;
        pw[j] = ldexp(1.0, E[j]);
      }
    }
  };
  for (int base = 0; base < cnt; base += kBlock) {
    __syncthreads();
    const int e = base + static_cast<int>(threadIdx.x);
    if (e < cnt) stage_entry<false>(a, list, e, m.x0, m.y0, &stage[threadIdx.x]);
    __syncthreads();
    const int nl = wave_compact(stage, min(kBlock, cnt - base), bits, wl);
    __syncthreads();
    for (int i = 0; i < nl; ++i) {
      const StageEntry& s = stage[wl[i]];
      const double dx = cxp - s.u;
      const double A = s.a * dx * dx, B = s.b2 * dx;
#pragma unroll
      for (int j = 0; j < RPL; ++j) {
        if (RPL > 1 && ((s.mask >> (RPL * m.wave + j)) & 1u) == 0) continue;  // uniform
        const double dy = (m.py0 + 4 * j + 0.5) - s.v;
        const double q = fma(dy, fma(s.c, dy, B), A);
        if (in[j] && q <= kSupport) {
          const float rho = __builtin_amdgcn_exp2f(static_cast<float>(q) * kNegHalfLog2e);
          const float al = fminf(s.sigma * rho, kClamp);
          const double ald = static_cast<double>(al);
          const double w = ald * t[j] * pw[j];
          C[j][0] = fma(w, s.c0, C[j][0]);
          C[j][1] = fma(w, s.c1, C[j][1]);
          C[j][2] = fma(w, s.c2, C[j][2]);
          t[j] *= 1.0 - ald;
        }
      }
      if ((i & (kRenormEvery - 1)) == kRenormEvery - 1) renorm();
    }
    renorm();
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
template <int RPL, bool GEOM>
__global__ __launch_bounds__(256 / RPL) void raster_render_bwd(RasterArgs a) {
  constexpr int kBlock = 256 / RPL;
  __shared__ StageEntry stage[kBlock];
  __shared__ int16_t wlist[kBlock / 64][kBlock];
  {
    const RasterStamp st = *a.stamp;  // same for every thread: a uniform exit
    if (st.magic != kStampMagic || st.cap != a.cap || st.tiles_x != a.tiles_x ||
        st.tiles_y != a.tiles_y || st.n != a.n) {
      if (blockIdx.x == 0 && threadIdx.x == 0) *a.stale = 1;
      return;
    }
  }
  const int64_t tile = blockIdx.x;
  const TileMap<RPL> m = tile_map<RPL>(a, tile);
  const double cxp = m.px + 0.5;
  const int cnt = __builtin_amdgcn_readfirstlane(min(a.cursor[tile], a.cap));
  const uint64_t* list = a.lists + tile * a.cap;
  const uint32_t bits = ((1u << RPL) - 1u) << (RPL * m.wave);
  int16_t* wl = wlist[m.wave];

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
  auto renorm = [&]() {
#pragma unroll
    for (int j = 0; j < RPL; ++j) {
      if (t[j] > 0x1p300 && E[j] < 0) {
        t[j] *= 0x1p-500;
        E[j] += kRenorm;
        pw[j] = ldexp(1.0, E[j]);
      }
    }
  };
  const int lane = static_cast<int>(threadIdx.x & 63);
  const bool writer = GEOM ? lane_writes9(lane) : lane_writes4(lane);
  const int slot = GEOM ? lane_slot9(lane) : lane_slot4(lane);
  for (int end = cnt; end > 0; end -= kBlock) {
    const int base = max(0, end - kBlock);
    __syncthreads();
    const int e = base + static_cast<int>(threadIdx.x);
    if (e < end) stage_entry<true>(a, list, e, m.x0, m.y0, &stage[threadIdx.x]);
    __syncthreads();
    const int nl = wave_compact(stage, end - base, bits, wl);
    __syncthreads();
    for (int i = nl - 1; i >= 0; --i) {
      const StageEntry& s = stage[wl[i]];
      const double dx = cxp - s.u;
      const double A = s.a * dx * dx, B = s.b2 * dx;
      double gc0 = 0.0, gc1 = 0.0, gc2 = 0.0;
      float gop = 0.f;
      // geometry: a lane's pixels share dx, so it sums dL/dq, dL/dq dy and
      // dL/dq dy^2 over them and forms dL/d(u, v, a, b, c) once per entry
      double q0 = 0.0, q1 = 0.0, q2 = 0.0;
      const double nhs = -0.5 * static_cast<double>(s.sigma);  // dalpha/dq = -sigma rho / 2
#pragma unroll
      for (int j = 0; j < RPL; ++j) {
        if (RPL > 1 && ((s.mask >> (RPL * m.wave + j)) & 1u) == 0) continue;  // uniform
        const double dy = (m.py0 + 4 * j + 0.5) - s.v;
        const double q = fma(dy, fma(s.c, dy, B), A);
        if (in[j] && q <= kSupport) {
          const float rho = __builtin_amdgcn_exp2f(static_cast<float>(q) * kNegHalfLog2e);
          const float raw = s.sigma * rho;
          const float al = fminf(raw, kClamp);
          const double ald = static_cast<double>(al);
          const double om = 1.0 - ald;
          t[j] *= rcp64(om);  // now T_i = t * pw
          const double T = t[j] * pw[j];
          const double w = ald * T;
          gc0 = fma(w, g[j][0], gc0);
          gc1 = fma(w, g[j][1], gc1);
          gc2 = fma(w, g[j][2], gc2);
          // c - R_{i+1} serves both dC/dalpha and R_i = R_{i+1} + alpha (c - R_{i+1})
          const double d0 = s.c0 - R[j][0], d1 = s.c1 - R[j][1], d2 = s.c2 - R[j][2];
          if (raw < kClamp) {
            const double da = fma(g[j][0], d0, fma(g[j][1], d1, g[j][2] * d2));
            const double gs = da * (T * rho);  // dL/dsigma of this pixel
            gop += static_cast<float>(gs);
            if constexpr (GEOM) {
              const double dq = nhs * gs;  // dL/dq of this pixel
              const double dqy = dq * dy;
              q0 += dq;
              q1 += dqy;
              q2 = fma(dqy, dy, q2);
            }
          }
          R[j][0] = fma(ald, d0, R[j][0]);
          R[j][1] = fma(ald, d1, R[j][1]);
          R[j][2] = fma(ald, d2, R[j][2]);
        }
      }
      // the entry's totals over the wavefront, one per writing lane
      float tot;
      if constexpr (GEOM) {
        // q = a dx^2 + b2 dx dy + c dy^2, dx = px - u, dy = py - v
        const double dq0 = dx * q0;
        const float v[9] = {static_cast<float>(gc0), static_cast<float>(gc1),
                            static_cast<float>(gc2), gop,
                            static_cast<float>(-(2.0 * s.a * dq0 + s.b2 * q1)),  // dL/du
                            static_cast<float>(-(s.b2 * dq0 + 2.0 * s.c * q1)),  // dL/dv
                            static_cast<float>(dx * dq0),                        // dL/da
                            static_cast<float>(2.0 * dx * q1),                   // dL/db
                            static_cast<float>(q2)};                             // dL/dc
        tot = lane_sums9(v, lane);
      } else {
        const float v[4] = {static_cast<float>(gc0), static_cast<float>(gc1),
                            static_cast<float>(gc2), gop};
        tot = lane_sums4(v);
      }
      if (writer && tot != 0.f)
        unsafeAtomicAdd(a.grad_acc + kAccStride * static_cast<int64_t>(s.idx) + slot,
                        static_cast<double>(tot));
      if ((i & (kRenormEvery - 1)) == 0) renorm();
    }
    renorm();
  }
}

__global__ void raster_copy_flag(const int32_t* src, int32_t* dst) { *dst = *src; }

hipError_t launch_copy_flag(const int32_t* src, int32_t* dst, hipStream_t s) {
  hipLaunchKernelGGL(raster_copy_flag, dim3(1), dim3(1), 0, s, src, dst);
  return hipGetLastError();
}

hipError_t launch_raster(const RasterArgs& a, bool bwd, hipStream_t s) {
  const int64_t n_tiles = static_cast<int64_t>(a.tiles_x) * a.tiles_y;
  const unsigned gt = static_cast<unsigned>((n_tiles + 255) / 256);
  const unsigned gn = static_cast<unsigned>((a.n + 255) / 256);
  if (!bwd) {
    hipLaunchKernelGGL(raster_begin, dim3(gt), dim3(256), 0, s, a);
    if (a.n > 0) {
      hipLaunchKernelGGL(raster_project, dim3(gn), dim3(256), 0, s, a);
      int pshift = 0;  // 2^pshift tile classes, the fewest that fit the LDS counters
      while ((1 << pshift) < kBinParts && ((n_tiles - 1) >> pshift) + 1 > kBinLdsTiles) ++pshift;
      if (((n_tiles - 1) >> pshift) + 1 <= kBinLdsTiles) {
        const int64_t chunk = 256 * kBinPrimsPerThread;
        const unsigned gc = static_cast<unsigned>((a.n + chunk - 1) / chunk);
        hipLaunchKernelGGL(raster_bin_lds, dim3(gc << pshift), dim3(256), 0, s, a, pshift);
      } else {
        hipLaunchKernelGGL(raster_bin, dim3(gn * kBinParts), dim3(256), 0, s, a);
      }
    }
    hipLaunchKernelGGL(raster_sort, dim3(static_cast<unsigned>(n_tiles)), dim3(256), 0, s, a);
    hipLaunchKernelGGL(raster_sort_network, dim3(static_cast<unsigned>(n_tiles)), dim3(256), 0, s,
                       a);
    hipLaunchKernelGGL(raster_render_fwd<kFwdRows>, dim3(static_cast<unsigned>(n_tiles)),
                       dim3(256 / kFwdRows), 0, s, a);
  } else {
    if (a.n == 0) return hipGetLastError();
    const bool geom = a.grad_means != nullptr || a.grad_scales != nullptr || a.grad_rots != nullptr;
    hipLaunchKernelGGL(raster_zero_acc, dim3(gn), dim3(256), 0, s, a.grad_acc, a.n, a.stale);
    if (geom) {
      hipLaunchKernelGGL((raster_render_bwd<kBwdRows, true>), dim3(static_cast<unsigned>(n_tiles)),
                         dim3(256 / kBwdRows), 0, s, a);
      hipLaunchKernelGGL(raster_finish_grads<true>, dim3(gn), dim3(256), 0, s, a);
    } else {
      hipLaunchKernelGGL((raster_render_bwd<kBwdRows, false>), dim3(static_cast<unsigned>(n_tiles)),
                         dim3(256 / kBwdRows), 0, s, a);
      hipLaunchKernelGGL(raster_finish_grads<false>, dim3(gn), dim3(256), 0, s, a);
    }
  }
  return hipGetLastError();
}

}  // namespace nasg
